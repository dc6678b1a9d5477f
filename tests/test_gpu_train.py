"""The training driver on the GPU: graph-replayed steps equal eager steps
(device-resident Philox counter and Adam step), moments carried through the
width growth, a short Static run that approaches the free-fermion ground
energy of the 1D TFIM (Eq. (6)), and the early-stopping stages."""
import numpy as np
import pytest

from tests import exact
from tests.gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def test_graph_replay_equals_eager_training():
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    from paper_2507_18700_amd.train import Trainer, adaptive_stages
    H = V.ham(V.VMC_TFIM, J=1.0, h=1.0)
    runs = []
    for graph in (True, False):
        tr = Trainer(dict(dims=1, Lx=10), H, 64, adaptive_stages(8, 16, 12), V.adam_cfg(lr0=5e-3), graph=graph)
        res = tr.run(check_every=5)
        runs.append((res, tr.params.cpu().numpy(), tr.mom_m.cpu().numpy(), tr.t_dev.item(), tr.ctr_dev.item()))
    (ra, pa, ma, ta, ca), (rb, pb, mb, tb, cb) = runs
    assert ta == tb == 24 and ca == cb == 24
    assert ra.stage_steps == rb.stage_steps == [12, 12]
    assert np.array_equal(ra.energy, rb.energy) and np.array_equal(ra.variance, rb.variance)
    assert np.array_equal(pa, pb) and np.array_equal(ma, mb)
    assert len(np.unique(ra.energy)) > 20  # every step drew fresh samples


def test_growth_carries_parameters_and_moments():
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    from paper_2507_18700_amd.train import Trainer, adaptive_stages
    H = V.ham(V.VMC_TFIM, J=1.0, h=1.0)
    tr = Trainer(dict(dims=1, Lx=8), H, 32, adaptive_stages(4, 8, 6), V.adam_cfg(lr0=1e-2), noise_std=0.0)
    tr.stages = tr.stages[:1]
    tr.run(check_every=3)
    p0, m0, v0, model0 = tr.params.clone(), tr.mom_m.clone(), tr.mom_v.clone(), tr.m
    tr._grow(8)
    torch.cuda.synchronize()
    assert tr.m.d_h == 8 and tr.t_dev.item() == 6
    # noise 0: the old entries are copied, the new ones are zero (moments too)
    n_old = V.param_count(model0)
    assert np.isclose(np.sort(np.abs(tr.params.cpu().numpy()))[-n_old:].sum(),
                      np.sort(np.abs(p0.cpu().numpy())).sum(), rtol=1e-6)
    assert np.count_nonzero(tr.mom_m.cpu().numpy()) == np.count_nonzero(m0.cpu().numpy())
    assert np.isclose(np.abs(tr.mom_v.cpu().numpy()).sum(), np.abs(v0.cpu().numpy()).sum(), rtol=1e-6)


def test_static_training_approaches_the_ground_energy():
    """1D TFIM, N = 8, h = 1: a few thousand Adam steps bring the variational
    energy within 1e-3 (relative) of the free-fermion E_0, and never below it
    beyond the statistical error."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    from paper_2507_18700_amd.train import Trainer, static_stages
    N = 8
    e0 = exact.free_fermion_e0(N, 1.0, 1.0)
    tr = Trainer(dict(dims=1, Lx=N), V.ham(V.VMC_TFIM, J=1.0, h=1.0), 256, static_stages(32, 3000),
                 V.adam_cfg(lr0=5e-3, lr1=1e-3, t_switch=1500))
    tr.run(check_every=500)
    E, dE, var, _ = tr.evaluate(100000, batch=50000)
    assert E >= e0 - 5 * dE
    assert (E - e0) / abs(e0) < 1e-3, (E, e0)


def test_early_stopping_stages():
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    from paper_2507_18700_amd.train import EarlyStop, Stage, Trainer
    H = V.ham(V.VMC_TFIM, J=1.0, h=1.0)
    rule = EarlyStop(window=10, patience=15, max_steps_per_stage=400)
    tr = Trainer(dict(dims=1, Lx=8), H, 64, [Stage(4, 0), Stage(8, 0)], V.adam_cfg(lr0=1e-2), early_stop=rule)
    res = tr.run(check_every=20)
    assert len(res.stage_steps) == 2
    # each stage ran at least one full window plus the patience, and stopped at a check boundary
    assert all(25 <= s <= 400 and s % 20 == 0 for s in res.stage_steps)
    assert tr.t_dev.item() == sum(res.stage_steps)


def test_evaluate_at_fp32_equals_an_fp32_model():
    """evaluate(precision=FP32) on a BF16 model samples and scores the same
    parameters exactly as a model built at FP32 does (the evaluation of
    BF16-trained states in FP32)."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    from paper_2507_18700_amd.train import Trainer, static_stages
    H = V.ham(V.VMC_HEISENBERG, J=1.0, h=0.0, marshall=True)
    kw = dict(dims=2, Lx=3, Ly=3, glu=True)
    a = Trainer(dict(kw, precision=V.VMC_BF16), H, 64, static_stages(32, 4), V.adam_cfg(lr0=1e-3), seed=5)
    a.run(check_every=4)
    b = Trainer(dict(kw, precision=V.VMC_FP32), H, 64, static_stages(32, 0), V.adam_cfg(lr0=1e-3), seed=5)
    b.params.copy_(a.params)
    ra = a.evaluate(3000, batch=1000, precision=V.VMC_FP32)
    rb = b.evaluate(3000, batch=1000)
    rc = a.evaluate(3000, batch=1000)
    assert ra == rb
    assert ra != rc and abs(ra[0] - rc[0]) < 1e-2 * abs(ra[0])


def test_restart_adam_at_each_width():
    """restart_adam: after a doubling the moments are zero and the step
    count restarts, so that at the end the count equals the last stage's
    steps; without it the count runs on over the stages."""
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    from paper_2507_18700_amd.train import Trainer, adaptive_stages
    H = V.ham(V.VMC_TFIM, J=1.0, h=1.0)
    counts = []
    for restart in (True, False):
        tr = Trainer(dict(dims=1, Lx=8), H, 32, adaptive_stages(4, 8, 6), V.adam_cfg(lr0=1e-2),
                     restart_adam=restart)
        tr.stages = tr.stages[:1]
        tr.run(check_every=3)
        tr._grow(8)
        torch.cuda.synchronize()
        if restart:
            assert not tr.mom_m.any() and not tr.mom_v.any()
        else:
            assert tr.mom_m.any() and tr.mom_v.any()
        counts.append(tr.t_dev.item())
    assert counts == [0, 6]

