"""The precision bar of the BF16 path on the 2D TFIM 10x10 workload (d_h =
128, h = 3): on 2048 configurations that the FP64 oracle sampled from the
workload's Philox stream (fixture tests/golden/c3_energy_fixture.npz, written
by make_c3_energy_fixture.py from the oracle alone), the library's local
energies match the oracle's: the mean energy per site within 1e-4 (BF16) and
1e-6 (FP32), every E_loc within 1e-2 (BF16) and 1e-5 (FP32) relative to
max(|E_ref|, N).  The BF16 per-sample error is about 1e-3 per site (the
rounding of the contraction operands), so 2048 samples resolve the mean to
about 2e-5."""
import importlib.util
import os

import numpy as np
import pytest

from tests.gpu_util import rel_l2, torch_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "c3_energy_fixture.npz")


def _fixture_module():
    spec = importlib.util.spec_from_file_location("make_c3", os.path.join(HERE, "golden", "make_c3_energy_fixture.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("bf16", [True, False], ids=["bf16", "fp32"])
def test_c3_energy_per_site(bf16):
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    fx = np.load(FIXTURE)
    N = 100
    cfg = np.unpackbits(fx["configs_packed"], axis=1)[:, :N].astype(np.uint8)
    ref = fx["eloc_real"] + 1j * fx["eloc_imag"]
    p = _fixture_module().c3_params()
    m = V.model(dims=2, Lx=10, Ly=10, d_h=128, glu=True, precision=V.VMC_BF16 if bf16 else V.VMC_FP32)
    e = V.local_energy(m, torch.from_numpy(p).cuda(), V.ham(V.VMC_TFIM, J=1.0, h=3.0), torch.from_numpy(cfg).cuda())
    torch.cuda.synchronize()
    e = e.cpu().numpy()
    eg = e[:, 0] + 1j * e[:, 1]
    err = (eg.real - ref.real) / N
    mean_err = abs(err.mean())
    print("energy per site: oracle %.8f, error of the mean %.2e, per-sample rms %.2e, max %.2e"
          % (ref.real.mean() / N, mean_err, np.sqrt(np.mean(err ** 2)), np.abs(err).max()))
    assert mean_err <= (1e-4 if bf16 else 1e-6)
    tol = 1e-2 if bf16 else 1e-5
    assert rel_l2(eg, ref) < tol
    assert np.max(np.abs(eg - ref) / np.maximum(np.abs(ref), N)) < tol
