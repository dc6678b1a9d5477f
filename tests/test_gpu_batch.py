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
