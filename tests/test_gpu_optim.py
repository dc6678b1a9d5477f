"""Adam (vmc_adam) against the oracle's Adam step, its learning-rate
schedules, the device-resident Philox counter of vmc_step under HIP-graph
replay, and the synchronous finiteness check, through the C ABI."""
import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import lib_and_oracle, torch_gpu

pytestmark = pytest.mark.gpu


def test_adam_matches_oracle():
    """Five Adam steps on float32 storage against the oracle's FP64 steps
    (the difference is the float32 rounding of parameters and moments)."""
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    rng = np.random.default_rng(3)
    n = 100003  # ragged against the 256-thread blocks
    p = rng.standard_normal(n).astype(np.float32)
    grads = [rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 1, n) for _ in range(5)]
    pd = torch.from_numpy(p.copy()).cuda()
    md = torch.zeros(n, dtype=torch.float32, device="cuda")
    vd = torch.zeros(n, dtype=torch.float32, device="cuda")
    td = torch.zeros(1, dtype=torch.int64, device="cuda")
    cfg = V.adam_cfg(lr0=1e-3)
    rp, rm, rv = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        V.adam(pd, torch.from_numpy(g).cuda(), md, vd, td, cfg)
        rp, rm, rv = O.adam(rp, g, rm, rv, t, 1e-3)
    torch.cuda.synchronize()
    assert td.item() == 5
    assert np.max(np.abs(pd.cpu().numpy() - rp) / np.maximum(np.abs(rp), 1e-2)) < 1e-5
    # the moments are float32 running sums: their rounding is relative to the
    # gradients summed, not to the (possibly cancelled) result
    gscale = np.max(np.abs(np.stack(grads)), axis=0)
    assert np.max(np.abs(md.cpu().numpy() - rm) / (0.1 * gscale)) < 1e-5
    assert np.max(np.abs(vd.cpu().numpy() - rv) / np.maximum(np.abs(rv), 1e-3 * gscale ** 2)) < 1e-5


def test_adam_schedules():
    """Under a constant gradient every bias-corrected Adam step is
    lr(k) * g / (|g| + eps), so the parameter change of update k exposes the
    learning rate of the schedule (Table III: two stages, inverse-time decay)."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    n = 64
    g = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    for cfg, lr in ((V.adam_cfg(lr0=5e-3, lr1=5e-4, t_switch=3), lambda k: 5e-3 if k < 3 else 5e-4),
                    (V.adam_cfg(lr0=5e-4, tau=2.0), lambda k: 5e-4 / (1 + k / 2.0)),
                    (V.adam_cfg(lr0=5e-4, t_decay=4, tau=5.0), lambda k: 5e-4 / (1 + max(0, k - 4) / 5.0))):
        p = torch.zeros(n, dtype=torch.float32, device="cuda")
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        t = torch.full((1,), 0, dtype=torch.int64, device="cuda")
        prev = 0.0
        for k in range(8):
            V.adam(p, g, m, v, t, cfg)
            cur = float(p[0].item())
            step = prev - cur
            assert abs(step - lr(k) * 0.5 / (0.5 + 1e-8)) < 2e-7 * (1 + k) + 1e-3 * lr(k), (k, step, lr(k))
            prev = cur


def test_step_counter_on_device_replays_fresh_samples():
    """vmc_step with a device-resident counter, captured once in a HIP graph:
    replay k equals the eager step at counter c0 + k, successive replays
    differ, and the counter advances by one per replay."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    spec, gm, _ = lib_and_oracle(2, 4, 4, 32, False, True, True)
    p = torch.from_numpy(synth.xavier_params(spec, 5, bias_scale=0.2)).cuda()
    H = V.ham(V.VMC_TFIM, 1.0, 3.0)
    ns = 150
    ws = V.Workspace()
    ws.get(V.workspace_size(gm, H, ns))
    ref = [[t.clone() for t in V.vmc_step(gm, p, H, ns, seed=4, counter=c, ws=ws)] for c in (10, 11, 12)]
    torch.cuda.synchronize()
    ctr = torch.full((1,), 10, dtype=torch.int64, device="cuda")
    out = [t.clone() for t in ref[0]]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on a side stream (launch attributes)
        V.vmc_step(gm, p, H, ns, seed=4, counter=999, ws=ws, out=out, counter_dev=ctr)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert ctr.item() == 11
    ctr.fill_(10)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        V.vmc_step(gm, p, H, ns, seed=4, counter=999, ws=ws, out=out, counter_dev=ctr)
    torch.cuda.synchronize()
    assert ctr.item() == 10  # capture launches nothing
    prev_cfg = None
    for k in range(3):
        ws.buf.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref[k], out):
            assert torch.equal(a, b), "replay %d" % k
        if prev_cfg is not None:
            assert not torch.equal(prev_cfg, out[0])
        prev_cfg = out[0].clone()
        assert ctr.item() == 11 + k


def test_check_finite():
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    x = torch.randn(100001, device="cuda")
    assert V.check_finite(x) == 0
    x[5] = float("nan")
    x[77777] = float("inf")
    x[100000] = float("-inf")
    with pytest.raises(V.VmcError) as ei:
        V.check_finite(x)
    assert ei.value.status == V.VMC_ENONFINITE


def test_nonfinite_parameters_propagate_to_stats():
    """The asynchronous step does not stop on non-finite parameters: every
    local energy is non-finite and stats[3] counts all samples."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    spec, gm, _ = lib_and_oracle(1, 12, 1, 16, False, False)
    p = torch.from_numpy(synth.xavier_params(spec, 5, bias_scale=0.2)).cuda()
    p[3] = float("nan")
    H = V.ham(V.VMC_TFIM, 1.0, 1.0)
    _, _, _, e, g, st = V.vmc_step(gm, p, H, 64, seed=1, counter=0)
    torch.cuda.synchronize()
    assert st[3].item() == 64
    with pytest.raises(V.VmcError):
        V.check_finite(p)
