"""Parity at the full sizes of the workloads (the bench configuration and the
other configurations of the path), in the launch configuration that bench.py
times (one vmc_step per batch), on sampled outputs that the FP64 oracle can
compute one by one:

  * the sampling decisions and log psi of sampled rows against the oracle
    (FP32 against the FP64 model; BF16 against the oracle's bfloat16-operand
    emulation, with the tie band widened accordingly);
  * the local energy of sampled rows against the oracle (full re-evaluation of
    every connected configuration); at 16x16 with d_h = 256 two rows against
    the oracle and, in addition, against the teacher-forced log psi of every
    connected configuration of the sampled rows (a second GPU code path);
  * the gradient restricted to the sampled rows (weights nonzero only there)
    against the oracle's gradient of those rows with the same local energies.
"""
import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import check_samples, lib_and_oracle, rel_l2, rel_max, torch_gpu

pytestmark = pytest.mark.gpu

# name, dims, Lx, Ly, d_h (start -> full), complex, glu, hamiltonian, h, Ns, bf16
FULL = [
    ("1d_heis_N50_dh64_fp32", 1, 50, 1, 32, 64, True, False, "heis", 0.0, 10000, False),
    ("2d_tfim_10x10_dh128_fp32", 2, 10, 10, 64, 128, False, True, "tfim", 3.0, 10000, False),
    ("2d_tfim_10x10_dh128_bf16", 2, 10, 10, 64, 128, False, True, "tfim", 3.0, 10000, True),
    ("2d_heis_16x16_dh256_bf16", 2, 16, 16, 256, 256, True, True, "heis", 0.0, 4096, True),
]
PICK = [0, 1, 2, 3, 1234, 4095]  # sampled rows


def _setup(case):
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    name, dims, Lx, Ly, dh0, dh, cplx, glu, kind, hx, ns, bf16 = case
    spec, gm, om_emul = lib_and_oracle(dims, Lx, Ly, dh, cplx, glu, bf16)
    _, _, om = lib_and_oracle(dims, Lx, Ly, dh, cplx, glu, False)
    spec0 = synth.ModelSpec(dims=dims, Lx=Lx, Ly=Ly if dims == 2 else 1, d_h=dh0, is_complex=cplx, glu=glu)
    p0 = torch.from_numpy(synth.xavier_params(spec0, 0, bias_scale=0.1)).cuda()
    if dh0 != dh:
        m0 = V.model(dims=dims, Lx=Lx, Ly=Ly, d_h=dh0, is_complex=cplx, glu=glu)
        p, _ = V.grow_hidden(m0, p0, dh, 2, 1e-3)
    else:
        p = p0
    if kind == "heis":
        H = V.ham(V.VMC_HEISENBERG, J=1.0, marshall=True)
        oh = O.ham(O.HEISENBERG, J=1.0, marshall=True)
    else:
        H = V.ham(V.VMC_TFIM, J=1.0, h=hx)
        oh = O.ham(O.TFIM, J=1.0, h=hx)
    return torch, O, V, spec, gm, om, om_emul, p, H, oh, ns, bf16


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", FULL, ids=lambda c: c[0])
def test_full_size_step(case):
    torch, O, V, spec, gm, om, om_emul, p, H, oh, ns, bf16 = _setup(case)
    N = spec.N
    cfg, lp, ph, e, g, st = [t.clone() for t in V.vmc_step(gm, p, H, ns, seed=1, counter=0)]
    torch.cuda.synchronize()
    pick = np.array([i for i in PICK if i < ns])
    p64 = p.cpu().numpy().astype(np.float64)
    c = cfg.cpu().numpy()[pick]
    lpg, phg = lp.cpu().numpy()[pick], ph.cpu().numpy()[pick]
    eg = e.cpu().numpy()[pick]
    assert np.isfinite(e.cpu().numpy()).all() and st.cpu().numpy()[3] == 0

    # sampling decisions and log psi of the sampled rows
    uni = O.philox_uniforms(1, 0, ns, N)[pick]
    if bf16:
        check_samples(O, om_emul, p64, c, uni, spec.Lx, spec.Ly, 1e-4)
        elp, eph = O.logpsi(om_emul, p64, c)
        assert rel_max(lpg, elp) < 2e-4
    else:
        check_samples(O, om, p64, c, uni, spec.Lx, spec.Ly, 1e-5)
    rlp, rph = O.logpsi(om, p64, c)
    tol = 1e-2 if bf16 else 1e-5
    assert rel_max(lpg, rlp) < tol
    if spec.is_complex:
        assert np.max(np.abs(phg - rph)) / max(np.max(np.abs(rph)), 1.0) < tol

    # local energy of the sampled rows
    eg_c = eg[:, 0] + 1j * eg[:, 1]
    if N <= 100:
        ref = O.local_energy(om, p64, oh, c)
        assert rel_l2(eg_c, ref) < tol
        assert np.max(np.abs(eg_c - ref) / np.maximum(np.abs(ref), N)) < tol
    else:
        # two rows against the oracle's full re-evaluation of every connected
        # configuration (about a minute of the host's cores)
        ref = O.local_energy(om, p64, oh, c[:2])
        assert np.max(np.abs(eg_c[:2] - ref) / np.maximum(np.abs(ref), N)) < tol
        # every connected configuration of two rows through the teacher-forced path
        for k in range(2):
            conn, coef, diag = _heisenberg_connections(c[k], spec.Lx, spec.Ly)
            lpc_, phc_ = V.rnn_logpsi(gm, p, torch.from_numpy(conn).cuda())
            torch.cuda.synchronize()
            lpc_, phc_ = lpc_.cpu().numpy().astype(np.float64), phc_.cpu().numpy().astype(np.float64)
            ratio = np.exp(0.5 * (lpc_ - lpg[k]) + 1j * (phc_ - phg[k]))
            e_tf = diag + np.sum(coef * ratio)
            assert abs(e_tf - eg_c[k]) / max(abs(e_tf), N) < 1e-5
            # a few of those connected configurations pinned to the oracle's emulation
            olp, _ = O.logpsi(om_emul, p64, conn[:4])
            assert rel_max(lpc_[:4], olp) < 2e-4

    # gradient restricted to the sampled rows against the oracle with the same E
    w = torch.zeros(ns, dtype=torch.float64, device="cuda")
    w[torch.from_numpy(pick).cuda()] = 1.0 / len(pick)
    gw, stw = V.vmc_grad(gm, p, cfg, e, weights=w)
    torch.cuda.synchronize()
    rg, rst = O.grad(om, p64, c, eg)
    assert np.allclose(stw.cpu().numpy()[:3], rst[:3], rtol=1e-12, atol=1e-12)
    err = rel_l2(gw.cpu().numpy(), rg)
    assert err < tol, "gradient relative l2 error %.3g" % err


def _heisenberg_connections(sigma, Lx, Ly):
    """Connected configurations of the Marshall-rotated Heisenberg model (the
    anti-aligned bonds), their coefficients and the diagonal, from the
    Hamiltonian's definition (J = 1): H = 1/4 sum Z Z + off-diagonal -1/2 per
    anti-aligned bond after the rotation."""
    bonds = []
    for j in range(Ly):
        for i in range(Lx):
            a = j * Lx + i
            if i + 1 < Lx:
                bonds.append((a, a + 1))
            if j + 1 < Ly:
                bonds.append((a, a + Lx))
    s = 1 - 2 * sigma.astype(np.int64)
    diag = 0.25 * sum(s[a] * s[b] for a, b in bonds)
    conn, coef = [], []
    for a, b in bonds:
        if sigma[a] != sigma[b]:
            t = sigma.copy()
            t[a] ^= 1
            t[b] ^= 1
            conn.append(t)
            coef.append(-0.5)
    return np.array(conn, dtype=np.uint8), np.array(coef), diag


@pytest.mark.parametrize("case", [FULL[2], FULL[3]], ids=lambda c: c[0])
def test_full_size_gradient_in_chunks(case):
    """The bench's step at full size, its gradient again in sample chunks of a
    quarter of the set (each in a workspace for one chunk): the statistics bit
    for bit, the gradient within the FP32 rounding of the per-position partial
    sums over different sample ranges."""
    torch, O, V, spec, gm, om, om_emul, p, H, oh, ns, bf16 = _setup(case)
    cfg, lp, ph, e, g, st = V.vmc_step(gm, p, H, ns, seed=7, counter=3)
    g, st = g.clone(), st.clone()
    w = torch.full((ns,), 1.0 / ns, dtype=torch.float64, device=p.device)
    g1, s1 = V.vmc_grad_chunked(gm, p, cfg, e, w, chunk=(ns + 3) // 4)
    torch.cuda.synchronize()
    assert torch.equal(s1, st)
    err = rel_l2(g1.cpu().numpy(), g.cpu().numpy())
    assert err < 1e-5, err
