"""Writes c3_energy_fixture.npz with the FP64 oracle only: the 2D TFIM 10x10
workload (h = 3, zig-zag 2D GRU + GLU, d_h = 64 Xavier weights from seed 0
grown to 128 by the oracle's grow_hidden with noise 1e-3 and seed 2, then
rounded to float32 as the library stores them), 2048 configurations sampled
by the oracle from the Philox uniforms of seed 1, counter 0, and their local
energies.  The GPU test feeds the same configurations to the library and
compares the mean energy per site.

    python tests/golden/make_c3_energy_fixture.py   (minutes on a few cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2507_18700_amd import synth  # noqa: E402

NS = 2048


def c3_params():
    """float32 parameters of the workload, grown by the oracle."""
    spec0 = synth.ModelSpec(dims=2, Lx=10, Ly=10, d_h=64, glu=True)
    m0 = O.model(dims=2, Lx=10, Ly=10, d_h=64, glu=True)
    p0 = synth.xavier_params(spec0, 0).astype(np.float64)
    return O.grow_hidden(m0, p0, 128, 2, 1e-3).astype(np.float32)


def main():
    om = O.model(dims=2, Lx=10, Ly=10, d_h=128, glu=True)
    p = c3_params().astype(np.float64)
    uni = O.philox_uniforms(1, 0, NS, 100)
    cfg, _, _ = O.sample(om, p, uni)
    e = O.local_energy(om, p, O.ham(O.TFIM, J=1.0, h=3.0), cfg)
    np.savez_compressed(os.path.join(HERE, "c3_energy_fixture.npz"), configs_packed=np.packbits(cfg, axis=1),
                        eloc_real=e.real, eloc_imag=e.imag)
    print("mean E/N %.10f over %d samples" % (e.real.mean() / 100, NS))


if __name__ == "__main__":
    main()
