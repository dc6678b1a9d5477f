"""Edge cases of the path through the C ABI, against the FP64 oracle: a
single sample, the longest chain the library accepts (N = 1024), a transverse
field of zero (no off-diagonal term), and a large sample count with ragged
tiles (sampled rows checked)."""
import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import check_samples, lib_and_oracle, rel_l2, rel_max, torch_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bf16", [False, True], ids=["fp32", "bf16"])
def test_single_sample(bf16):
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    spec, gm, om = lib_and_oracle(2, 3, 3, 16, True, True, bf16)
    p = synth.xavier_params(spec, 5, bias_scale=0.2)
    pd = torch.from_numpy(p).cuda()
    H = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True)
    cfg, lp, ph, e, g, st = [t.clone() for t in V.vmc_step(gm, pd, H, 1, seed=2, counter=0)]
    torch.cuda.synchronize()
    c = cfg.cpu().numpy()
    p64 = p.astype(np.float64)
    check_samples(O, om, p64, c, O.philox_uniforms(2, 0, 1, spec.N), 3, 3, 1e-4 if bf16 else 1e-5)
    rlp, rph = O.logpsi(om, p64, c)
    tol = 2e-4 if bf16 else 1e-5
    assert rel_max(lp.cpu().numpy(), rlp) < tol
    _, _, om64 = lib_and_oracle(2, 3, 3, 16, True, True, False)
    re = O.local_energy(om64, p64, O.ham(O.HEISENBERG, J=1.0, marshall=True), c)
    eg = e.cpu().numpy()
    assert abs(eg[0, 0] + 1j * eg[0, 1] - re[0]) / max(abs(re[0]), spec.N) < (1e-2 if bf16 else 1e-5)
    # one sample: E - Ebar = 0, so the covariance gradient vanishes exactly
    assert np.all(g.cpu().numpy() == 0.0)
    assert st.cpu().numpy()[2] == 0.0


def test_longest_chain():
    """1D, N = 1024 sites (the largest lattice accepted), d_h = 16: sampling
    from given uniforms, log psi and the local energy of two samples."""
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    N = 1024
    spec, gm, om = lib_and_oracle(1, N, 1, 16, False, False)
    p = synth.xavier_params(spec, 9, bias_scale=0.1)
    pd = torch.from_numpy(p).cuda()
    ns = 66
    uni = synth.uniforms(ns, N, 4)
    cfg, lp, _ = V.rnn_sample(gm, pd, ns, uniforms=torch.from_numpy(uni).cuda())
    H = V.ham(V.VMC_TFIM, 1.0, 1.0)
    e = V.local_energy(gm, pd, H, cfg[:2].contiguous())
    torch.cuda.synchronize()
    c = cfg.cpu().numpy()
    p64 = p.astype(np.float64)
    check_samples(O, om, p64, c[:8], uni[:8].astype(np.float64), N, 1, 1e-5)
    rlp, _ = O.logpsi(om, p64, c[:8])
    assert rel_max(lp.cpu().numpy()[:8], rlp) < 1e-5
    re = O.local_energy(om, p64, O.ham(O.TFIM, J=1.0, h=1.0), c[:2])
    eg = e.cpu().numpy()
    assert rel_l2(eg[:, 0] + 1j * eg[:, 1], re) < 1e-5


def test_zero_field():
    """TFIM with h = 0: no connected configuration contributes, E_loc is the
    bond sum -J sum s_a s_b exactly."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    spec, gm, _ = lib_and_oracle(2, 4, 5, 32, False, True)
    pd = torch.from_numpy(synth.xavier_params(spec, 2)).cuda()
    c = synth.configs(77, spec.N, 6)
    e = V.local_energy(gm, pd, V.ham(V.VMC_TFIM, 0.7, 0.0), torch.from_numpy(c).cuda())
    torch.cuda.synchronize()
    s = (1 - 2 * c.astype(np.int64)).reshape(77, 5, 4)
    diag = -0.7 * ((s[:, :, 1:] * s[:, :, :-1]).sum((1, 2)) + (s[:, 1:, :] * s[:, :-1, :]).sum((1, 2)))
    eg = e.cpu().numpy()
    assert np.array_equal(eg[:, 0], diag.astype(np.float64)) and np.all(eg[:, 1] == 0.0)


def test_many_samples_ragged():
    """2^17 + 3 samples (ragged last tile everywhere) in one vmc_step; sampled
    rows, including the last, against the oracle."""
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    spec, gm, om = lib_and_oracle(1, 12, 1, 32, True, False)
    p = synth.xavier_params(spec, 8, bias_scale=0.1)
    pd = torch.from_numpy(p).cuda()
    ns = (1 << 17) + 3
    H = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True)
    cfg, lp, ph, e, g, st = V.vmc_step(gm, pd, H, ns, seed=3, counter=1)
    torch.cuda.synchronize()
    pick = np.array([0, 1, 77777, ns - 2, ns - 1])
    c = cfg.cpu().numpy()[pick]
    p64 = p.astype(np.float64)
    uni = O.philox_uniforms(3, 1, ns, spec.N)[pick]
    check_samples(O, om, p64, c, uni, 12, 1, 1e-5)
    rlp, rph = O.logpsi(om, p64, c)
    assert rel_max(lp.cpu().numpy()[pick], rlp) < 1e-5
    re = O.local_energy(om, p64, O.ham(O.HEISENBERG, J=1.0, marshall=True), c)
    eg = e.cpu().numpy()[pick]
    assert rel_l2(eg[:, 0] + 1j * eg[:, 1], re) < 1e-5
    stats = st.cpu().numpy()
    assert np.isfinite(stats).all() and stats[3] == 0
    assert np.isfinite(g.cpu().numpy()).all()


def test_largest_2d_lattice():
    """2D 29x29, bfloat16, d_h = 128 with GLU: the largest square lattice whose
    tiles fit the LDS at that width (30x30 is refused, see test_abi).  Sampling
    from given uniforms and log psi against the oracle's bf16 emulation; the
    local energy of one sample against its connected configurations through the
    teacher-forced path, a few of them pinned to the oracle."""
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    L = 29
    spec, gm, om = lib_and_oracle(2, L, L, 128, False, True, True)
    N = spec.N
    p = synth.xavier_params(spec, 12, bias_scale=0.1)
    pd = torch.from_numpy(p).cuda()
    ns = 6
    uni = synth.uniforms(ns, N, 5)
    cfg, lp, _ = V.rnn_sample(gm, pd, ns, uniforms=torch.from_numpy(uni).cuda())
    torch.cuda.synchronize()
    c = cfg.cpu().numpy()
    lpg = lp.cpu().numpy().astype(np.float64)
    p64 = p.astype(np.float64)
    check_samples(O, om, p64, c, uni.astype(np.float64), L, L, 1e-3)
    rlp, _ = O.logpsi(om, p64, c)
    assert rel_max(lpg, rlp) < 2e-4
    hx = 1.0
    e = V.local_energy(gm, pd, V.ham(V.VMC_TFIM, 1.0, hx), cfg[:1].contiguous())
    torch.cuda.synchronize()
    eg = e.cpu().numpy()[0]
    # TFIM: one connection per site (that spin flipped), coefficient -h
    conn = np.repeat(c[:1], N, axis=0)
    conn[np.arange(N), np.arange(N)] ^= 1
    lpc, _ = V.rnn_logpsi(gm, pd, torch.from_numpy(conn).cuda())
    torch.cuda.synchronize()
    lpc = lpc.cpu().numpy().astype(np.float64)
    s = (1 - 2 * c[0].astype(np.int64)).reshape(L, L)
    diag = -((s[:, 1:] * s[:, :-1]).sum() + (s[1:, :] * s[:-1, :]).sum())
    e_tf = diag - hx * np.sum(np.exp(0.5 * (lpc - lpg[0])))
    assert abs(e_tf - eg[0]) / max(abs(e_tf), N) < 1e-5 and eg[1] == 0.0
    olp, _ = O.logpsi(om, p64, conn[[0, N // 2, N - 1]])
    assert rel_max(lpc[[0, N // 2, N - 1]], olp) < 2e-4
