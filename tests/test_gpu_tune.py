"""The launch tuning table and the autotuner, through the C ABI: every
candidate choice (row tile of the sampling / log psi launches, persistent
work-groups per compute unit of the suffix-chain launch) gives the same
output bits as the built-in choice, for vmc_step and for the separate calls;
the autotuner leaves a valid candidate in the table and the outputs of one
step."""
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import lib_and_oracle, torch_gpu

pytestmark = pytest.mark.gpu

CASES = [
    (2, 4, 4, 128, False, True, "tfim", True),   # bf16 d_h = 128: row tiles 64 / 48
    (2, 5, 3, 20, True, True, "heis", False),    # fp32 d_h = 32 (padded): 64 / 32
    (1, 20, 1, 16, False, False, "tfim", True),  # one option only
    (2, 3, 3, 256, True, True, "heis", True),    # bf16 d_h = 256: one option (48 rows)
]


def _setup(case):
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    dims, Lx, Ly, dh, cplx, glu, kind, bf16 = case
    spec, gm, _ = lib_and_oracle(dims, Lx, Ly, dh, cplx, glu, bf16)
    p = torch.from_numpy(synth.xavier_params(spec, 71, bias_scale=0.2)).cuda()
    H = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True) if kind == "heis" else V.ham(V.VMC_TFIM, 1.0, 2.0)
    return torch, V, gm, p, H


def _all_outputs(torch, V, gm, p, H, ns):
    step = [t.clone() for t in V.vmc_step(gm, p, H, ns, seed=9, counter=2)]
    c2, l2, f2 = [t.clone() for t in V.rnn_sample(gm, p, ns, seed=9, counter=2)]
    lt, ft = [t.clone() for t in V.rnn_logpsi(gm, p, c2)]
    e2 = V.local_energy(gm, p, H, c2).clone()
    g2, s2 = [t.clone() for t in V.vmc_grad(gm, p, c2, e2)]
    torch.cuda.synchronize()
    return step + [c2, l2, f2, lt, ft, e2, g2, s2]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dD_%dx%d_dh%d_c%d_g%d_%s_bf%d" % c)
def test_every_tuning_same_bits(case):
    torch, V, gm, p, H = _setup(case)
    ns = 333  # several row tiles with a ragged tail under every option
    V.reset_tuning(gm)
    ref = _all_outputs(torch, V, gm, p, H, ns)
    opts = V.row_tile_options(gm)
    try:
        for rt in opts:
            for wpc in (1, 3, 4):
                V.set_tuning(gm, row_tile=rt, chain_wgs_per_cu=wpc)
                assert V.get_tuning(gm) == {"row_tile": rt, "chain_wgs_per_cu": wpc}
                got = _all_outputs(torch, V, gm, p, H, ns)
                for k, (a, b) in enumerate(zip(got, ref)):
                    assert torch.equal(a, b), "output %d differs under row_tile %d, %d wgs/cu" % (k, rt, wpc)
    finally:
        V.reset_tuning(gm)


@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: "%dD_%dx%d_dh%d_c%d_g%d_%s_bf%d" % c)
def test_autotune_step(case):
    torch, V, gm, p, H = _setup(case)
    ns = 500
    V.reset_tuning(gm)
    ref = [t.clone() for t in V.vmc_step(gm, p, H, ns, seed=4, counter=1)]
    try:
        out, t = V.autotune_step(gm, p, H, ns, seed=4, counter=1, reps=2)
        torch.cuda.synchronize()
        assert t["row_tile"] in V.row_tile_options(gm) and 1 <= t["chain_wgs_per_cu"] <= 4
        assert V.get_tuning(gm) == t
        for a, b in zip(out, ref):
            assert torch.equal(a, b)
        # a step under the stored choice
        again = [x.clone() for x in V.vmc_step(gm, p, H, ns, seed=4, counter=1)]
        torch.cuda.synchronize()
        for a, b in zip(again, ref):
            assert torch.equal(a, b)
    finally:
        V.reset_tuning(gm)


def test_step_batch_autotune():
    """StepBatch tunes each distinct model shape, then its graph replays to the
    eager result."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    problems = []
    for c, (n, h) in enumerate([(32, 0.7), (48, 1.2), (32, 1.0)]):
        spec = synth.ModelSpec(dims=1, Lx=n, Ly=1, d_h=64)
        problems.append(dict(model=V.model(dims=1, Lx=n, d_h=64, precision=V.VMC_BF16),
                             params=torch.from_numpy(synth.xavier_params(spec, 100 + c)).cuda(),
                             ham=V.ham(V.VMC_TFIM, 1.0, h), ns=300 + 100 * c, seed=3, counter=c))
    b = V.StepBatch(problems, streams=2)
    try:
        b.run_eager()
        torch.cuda.synchronize()
        ref = [[t.clone() for t in o] for o in b.outputs]
        tuning = b.autotune(reps=1)
        assert len(tuning) == 2
        b.capture()
        for _ in range(2):
            b.replay()
            torch.cuda.synchronize()
            for o, r in zip(b.outputs, ref):
                for x, y in zip(o, r):
                    assert torch.equal(x, y)
    finally:
        for pb in problems:
            V.reset_tuning(pb["model"])
