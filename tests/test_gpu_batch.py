"""Several uneven problems in one HIP graph (StepBatch): 1D TFIM chains of
lengths drawn from 32..128 with fields in [0.5, 1.5], d_h = 64, each with
its own weights, replayed as one graph over concurrent streams.  Every
replay equals the eager per-problem vmc_step bit for bit, and sampled rows
of every problem match the FP64 oracle."""
import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import check_samples, lib_and_oracle, rel_l2, rel_max, torch_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bf16", [False, True], ids=["fp32", "bf16"])
def test_uneven_chains_one_graph(bf16):
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    chains = synth.uneven_chains(6, 3)
    ns = 96
    problems, specs = [], []
    for c, (N, h) in enumerate(chains):
        spec, gm, _ = lib_and_oracle(1, N, 1, 64, False, False, bf16)
        p = torch.from_numpy(synth.xavier_params(spec, 100 + c, bias_scale=0.2)).cuda()
        problems.append(dict(model=gm, params=p, ham=V.ham(V.VMC_TFIM, 1.0, h), ns=ns, seed=11, counter=c))
        specs.append(spec)
    eager = []
    for pb in problems:
        eager.append([t.clone() for t in V.vmc_step(pb["model"], pb["params"], pb["ham"], ns, seed=11,
                                                     counter=pb["counter"])])
    torch.cuda.synchronize()
    batch = V.StepBatch(problems, streams=3).capture()
    for rep in range(2):
        for outs in batch.outputs:
            for t in outs:
                t.zero_()
        torch.cuda.synchronize()
        batch.replay()
        torch.cuda.synchronize()
        for i, (ref, got) in enumerate(zip(eager, batch.outputs)):
            for a, b in zip(ref, got):
                assert torch.equal(a, b), "problem %d, replay %d" % (i, rep)
    tol = 1e-2 if bf16 else 1e-5
    pick = np.array([0, 1, ns - 1])
    for c, (pb, spec) in enumerate(zip(problems, specs)):
        N, h = chains[c]
        _, _, om = lib_and_oracle(1, N, 1, 64, False, False, False)
        cfg, lp, _, e, _, _ = [t.cpu().numpy() for t in batch.outputs[c]]
        p64 = pb["params"].cpu().numpy().astype(np.float64)
        rlp, _ = O.logpsi(om, p64, cfg[pick])
        assert rel_max(lp[pick], rlp) < tol
        if not bf16:
            uni = O.philox_uniforms(11, c, ns, N)[pick]
            check_samples(O, om, p64, cfg[pick], uni, N, 1, 1e-5)
        ref = O.local_energy(om, p64, O.ham(O.TFIM, J=1.0, h=h), cfg[pick])
        assert rel_l2(e[pick, 0] + 1j * e[pick, 1], ref) < tol


# ------------------------------------------------------- vmc_step_batched

def _batched_case(torch, V, lens, fields, dh, cplx, bf16, seed0, kind="tfim"):
    ps, hams, models = [], [], []
    for c, (N, h) in enumerate(zip(lens, fields)):
        spec, gm, _ = lib_and_oracle(1, N, 1, dh, cplx, False, bf16)
        ps.append(synth.xavier_params(spec, seed0 + c, bias_scale=0.2))
        models.append(gm)
        if kind == "lrtfim":
            hams.append(V.ham(V.VMC_LRTFIM, J=1.0, h=h, alpha=0.5 + 0.1 * c))
        elif kind == "cluster":
            hams.append(V.ham(V.VMC_CLUSTER, J=h))
        else:
            hams.append(V.ham(V.VMC_TFIM, J=1.0, h=h))
    params = torch.from_numpy(np.stack(ps)).cuda()
    return models, hams, params


BATCH_CASES = [
    # lengths (ragged, unsorted), d_h, complex, bf16, kind
    ([33, 7, 64, 20, 47, 2], 64, False, False, "tfim"),
    ([33, 7, 64, 20, 47, 2], 64, False, True, "tfim"),
    ([40, 12, 25], 16, True, False, "lrtfim"),
    ([9, 3, 30, 4], 32, True, True, "cluster"),
    ([5, 21], 130, False, False, "tfim"),      # streamed weights (d_h padded to 256)
]


@pytest.mark.parametrize("case", BATCH_CASES, ids=lambda c: "%s_dh%d_c%d_bf%d" % (c[4], c[1], c[2], c[3]))
def test_batched_step_equals_per_problem_steps(case):
    """vmc_step_batched: problem k equals vmc_step on it alone (Philox key
    seed + k) bit for bit, for every output."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    lens, dh, cplx, bf16, kind = case
    fields = [0.5 + 0.13 * c for c in range(len(lens))]
    models, hams, params = _batched_case(torch, V, lens, fields, dh, cplx, bf16, 200, kind)
    m = models[0]
    ns = 131
    out = [t.clone() for t in V.vmc_step_batched(m, lens, hams, params, ns, seed=21, counter=5)]
    torch.cuda.synchronize()
    for k, (N, gm, H) in enumerate(zip(lens, models, hams)):
        cfg, lp, ph, e, g, st = V.vmc_step(gm, params[k].contiguous(), H, ns, seed=21 + k, counter=5)
        torch.cuda.synchronize()
        assert torch.equal(V.batch_configs(out[0], k, ns, N), cfg), k
        assert torch.equal(out[1][k], lp) and torch.equal(out[3][k], e), k
        if cplx:
            assert torch.equal(out[2][k], ph), k
        assert torch.equal(out[4][k], g) and torch.equal(out[5][k], st), k


def test_batched_graph_replay_with_device_counter():
    """A captured batched step with a device-resident counter replays to the
    eager batched steps at counters c, c+1."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    lens = [30, 9, 17]
    models, hams, params = _batched_case(torch, V, lens, [0.7, 1.0, 1.3], 64, False, True, 300)
    m, ns = models[0], 96
    ws = V.Workspace()
    ref = [[t.clone() for t in V.vmc_step_batched(m, lens, hams, params, ns, seed=3, counter=c, ws=ws)]
           for c in (8, 9)]
    out = [t.clone() for t in ref[0]]
    ctr = torch.full((1,), 8, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        V.vmc_step_batched(m, lens, hams, params, ns, seed=3, ws=ws, out=out, counter_dev=ctr)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ctr.fill_(8)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        V.vmc_step_batched(m, lens, hams, params, ns, seed=3, ws=ws, out=out, counter_dev=ctr)
    for k in range(2):
        ws.buf.fill_(5)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref[k], out):
            assert torch.equal(a, b), "replay %d" % k
    assert ctr.item() == 10


@pytest.mark.parametrize("bf16", [True, False], ids=["bf16", "fp32"])
def test_c5_full_config_batched(bf16):
    """The uneven-batch workload at its full size through the launches the
    bench times: 32 TFIM chains, N uniform in 32..128, h uniform in
    [0.5, 1.5], d_h = 64, 2048 samples each.  Every problem equals its own
    vmc_step bit for bit; sampled rows of every chain match the FP64 oracle
    (sampling decisions, log psi, local energy)."""
    torch = torch_gpu()
    from oracle import oracle as O
    from paper_2507_18700_amd import vmcrnn as V
    chains = synth.uneven_chains(32, 3)
    lens = [n for n, _ in chains]
    fields = [h for _, h in chains]
    models, hams, params = _batched_case(torch, V, lens, fields, 64, False, bf16, 100)
    ns = 2048
    out = [t.cpu() for t in V.vmc_step_batched(models[0], lens, hams, params, ns, seed=1, counter=0)]
    torch.cuda.synchronize()
    tol = 1e-2 if bf16 else 1e-5
    pick = np.array([0, 777, ns - 1])
    for k, (N, h) in enumerate(chains):
        if k % 4 == 0:  # a quarter of the problems against their own step (the rest: parity below)
            ref = V.vmc_step(models[k], params[k].contiguous(), hams[k], ns, seed=1 + k, counter=0)
            torch.cuda.synchronize()
            assert torch.equal(V.batch_configs(out[0], k, ns, N), ref[0].cpu())
            assert torch.equal(out[4][k], ref[4].cpu()) and torch.equal(out[3][k], ref[3].cpu())
        _, _, om = lib_and_oracle(1, N, 1, 64, False, False, False)
        cfg = V.batch_configs(out[0], k, ns, N).numpy()[pick]
        p64 = params[k].cpu().numpy().astype(np.float64)
        rlp, _ = O.logpsi(om, p64, cfg)
        assert rel_max(out[1][k].numpy()[pick], rlp) < tol
        if not bf16:
            uni = O.philox_uniforms(1 + k, 0, ns, N)[pick]
            check_samples(O, om, p64, cfg, uni, N, 1, 1e-5)
        e = out[3][k].numpy()[pick]
        ref_e = O.local_energy(om, p64, O.ham(O.TFIM, J=1.0, h=h), cfg)
        assert np.max(np.abs(e[:, 0] + 1j * e[:, 1] - ref_e) / np.maximum(np.abs(ref_e), N)) < tol
