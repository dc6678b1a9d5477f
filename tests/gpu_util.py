"""Shared helpers of the GPU parity tests: seeded inputs for both sides, the
library and oracle descriptors of one model, and the tolerance measures."""
import numpy as np
import pytest

from paper_2507_18700_amd import synth


def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def lib_and_oracle(dims, Lx, Ly, d_h, cplx, glu, bf16=False):
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    spec = synth.ModelSpec(dims=dims, Lx=Lx, Ly=Ly if dims == 2 else 1, d_h=d_h, is_complex=cplx, glu=glu)
    gm = V.model(dims=dims, Lx=Lx, Ly=Ly, d_h=d_h, is_complex=cplx, glu=glu,
                 precision=V.VMC_BF16 if bf16 else V.VMC_FP32)
    om = O.model(dims=dims, Lx=Lx, Ly=Ly, d_h=d_h, is_complex=cplx, glu=glu, bf16=bf16)
    return spec, gm, om


def rel_max(got, ref):
    """max_s |got - ref| / |ref| (log psi measure)."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)))


def rel_l2(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def order_sites(Lx, Ly):
    res = []
    for n in range(Lx * Ly):
        j, k = divmod(n, Lx)
        res.append(j * Lx + (k if j % 2 == 0 else Lx - 1 - k))
    return np.array(res)


def check_samples(O, om, params64, cfg_gpu, uni, Lx, Ly, delta):
    """Every sampling decision of the GPU agrees with the oracle's conditional
    along the GPU's own configuration, except within delta of a tie; returns
    (number of near-tie samples, mask of samples with no near tie)."""
    _, _, lpc, _ = O.logpsi(om, params64, cfg_gpu, conditionals=True)
    sites = order_sites(Lx, Ly)
    p0 = np.exp(lpc[:, :, 0])
    sig = cfg_gpu[:, sites]
    want = (uni >= p0).astype(np.uint8)
    near = np.abs(uni - p0) < delta
    bad = (sig != want) & ~near
    assert not bad.any(), "sampling decisions differ away from ties: %d" % int(bad.sum())
    clean = ~near.any(axis=1)
    return int((~clean).sum()), clean
