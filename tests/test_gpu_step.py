"""vmc_step (one fused VMC step) against the three separate calls and the
oracle, through the C ABI."""
import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import check_samples, lib_and_oracle, rel_l2, torch_gpu

pytestmark = pytest.mark.gpu

STEP_CASES = [
    (2, 4, 4, 16, False, True, "tfim", False),
    (2, 5, 3, 20, True, True, "heis", False),
    (1, 20, 1, 16, False, False, "tfim", True),
    (2, 4, 4, 128, False, True, "tfim", True),
]


@pytest.mark.parametrize("case", STEP_CASES, ids=lambda c: "%dD_%dx%d_dh%d_c%d_g%d_%s_bf%d" % c)
def test_step_equals_separate_calls(case):
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    dims, Lx, Ly, dh, cplx, glu, kind, bf16 = case
    spec, gm, om = lib_and_oracle(dims, Lx, Ly, dh, cplx, glu, bf16)
    p = torch.from_numpy(synth.xavier_params(spec, 61, bias_scale=0.2)).cuda()
    H = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True) if kind == "heis" else V.ham(V.VMC_TFIM, 1.0, 2.0)
    ns = 150
    cfg, lp, ph, e, g, st = [t.clone() for t in V.vmc_step(gm, p, H, ns, seed=5, counter=3)]
    cfg2, lp2, ph2 = V.rnn_sample(gm, p, ns, seed=5, counter=3)
    e2 = V.local_energy(gm, p, H, cfg2)
    g2, st2 = V.vmc_grad(gm, p, cfg2, e2)
    torch.cuda.synchronize()
    assert torch.equal(cfg, cfg2) and torch.equal(lp, lp2)
    if cplx:
        assert torch.equal(ph, ph2)
    assert torch.equal(e, e2)
    assert torch.equal(g, g2) and torch.equal(st, st2)
    if not bf16:
        c = cfg.cpu().numpy()
        p64 = p.cpu().numpy().astype(np.float64)
        oh = O.ham(O.HEISENBERG, J=1.0, marshall=True) if kind == "heis" else O.ham(O.TFIM, J=1.0, h=2.0)
        re = O.local_energy(om, p64, oh, c)
        eg = e.cpu().numpy()
        assert rel_l2(eg[:, 0] + 1j * eg[:, 1], re) < 1e-5
        rg, rst = O.grad(om, p64, c, eg)
        assert rel_l2(g.cpu().numpy(), rg) < 1e-5
        uni = O.philox_uniforms(5, 3, ns, spec.N)
        check_samples(O, om, p64, c, uni, spec.Lx, spec.Ly, 1e-5)


@pytest.mark.parametrize("case", [STEP_CASES[1], STEP_CASES[3]], ids=lambda c: "%dD_%dx%d_dh%d_c%d_g%d_%s_bf%d" % c)
def test_step_graph_replay(case):
    """A vmc_step captured in a HIP graph (no allocation, no host sync and no
    memset inside the call) replays to the eager result, bit for bit, on every
    replay, with eager work and synchronisations between the replays."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    dims, Lx, Ly, dh, cplx, glu, kind, bf16 = case
    spec, gm, _ = lib_and_oracle(dims, Lx, Ly, dh, cplx, glu, bf16)
    p = torch.from_numpy(synth.xavier_params(spec, 71, bias_scale=0.2)).cuda()
    H = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True) if kind == "heis" else V.ham(V.VMC_TFIM, 1.0, 2.0)
    ns = 150
    ws = V.Workspace()
    ws.get(V.workspace_size(gm, H, ns))

    def outs():
        return (torch.empty((ns, spec.N), dtype=torch.uint8, device="cuda"),
                torch.empty(ns, dtype=torch.float32, device="cuda"),
                torch.empty(ns, dtype=torch.float32, device="cuda"),
                torch.empty((ns, 2), dtype=torch.float64, device="cuda"),
                torch.empty(V.param_count(gm), dtype=torch.float64, device="cuda"),
                torch.empty(4, dtype=torch.float64, device="cuda"))

    ref = V.vmc_step(gm, p, H, ns, seed=9, counter=4, ws=ws, out=outs())
    torch.cuda.synchronize()
    got = outs()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        V.vmc_step(gm, p, H, ns, seed=9, counter=4, ws=ws, out=got)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        V.vmc_step(gm, p, H, ns, seed=9, counter=4, ws=ws, out=got)
    for rep in range(3):
        for t in got:
            t.zero_()
        ws.buf.fill_(7)  # the workspace holds no state between calls
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), "replay %d" % rep
