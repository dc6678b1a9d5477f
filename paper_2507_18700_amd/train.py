"""VMC training driver for Static and Adaptive RNN wave functions.

Follows the paper's training scheme: VMC steps (Sec. III) with the Adam
optimiser (App. B), a fixed hidden width (Static) or a sequence of widths
that double at fixed step intervals (Adaptive, Sec. II B and Fig. 2), where
the parameters and the Adam moments of the smaller model are carried into
the larger one by grow_hidden (App. B); or widths that double when an
early-stopping criterion on the moving average of the energy variance fires
(Sec. III B, App. B).

This module holds only schedule logic on the host.  Every step of the path
runs in the library's kernels: vmc_step (sampling, local energy, gradient),
vmc_adam (the update, with its step count in device memory) and grow_hidden
(the width transitions).  The step of each stage is captured once as a HIP
graph (the Philox counter and the Adam step live in device memory, so every
replay draws fresh samples and applies the right learning rate) and
replayed; the energy statistics of every step go to a device-side history
that the host reads every `check_every` steps.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import synth
from . import vmcrnn as V


@dataclass
class EarlyStop:
    """Early stopping on the moving average (window `window`) of the energy
    variance sigma^2 (per_spin: sigma^2 / N): an improvement is a drop of the
    average below the best value so far by more than
    delta(d_h) = 10^(-log2(d_h)/2) (App. B); the criterion fires after
    `patience` steps without improvement, counted from the first step with a
    full window."""
    window: int = 500
    patience: int = 10000
    max_steps_per_stage: int = 10 ** 7
    per_spin: bool = False

    @staticmethod
    def delta(d_h):
        return 10.0 ** (-0.5 * math.log2(d_h))


class EarlyStopState:
    """Running state of the criterion for one stage (host arithmetic on the
    variance history only)."""

    def __init__(self, rule, d_h):
        self.rule = rule
        self.delta = rule.delta(d_h)
        self.vals = []
        self.best = math.inf
        self.wait = 0
        self.fired_at = None
        self.wsum = 0.0  # running sum of the last `window` values

    def update(self, variances):
        """Feed the per-step variances (in order); returns the index (within
        the stage) of the step at which the criterion fired, or None."""
        w = self.rule.window
        for v in variances:
            self.vals.append(float(v))
            n = len(self.vals)
            if n % 10000 == 0:  # exact sum now and then, so that rounding does not drift
                self.wsum = math.fsum(self.vals[-w:])
            else:
                self.wsum += self.vals[-1] - (self.vals[-1 - w] if n > w else 0.0)
            if self.fired_at is not None or n < w:
                continue
            avg = self.wsum / w
            if avg < self.best - self.delta:
                self.best = avg
                self.wait = 0
            else:
                self.wait += 1
                if self.wait >= self.rule.patience:
                    self.fired_at = len(self.vals) - 1
        return self.fired_at


@dataclass
class Stage:
    d_h: int
    steps: int = 0              # fixed number of steps, or 0 with early stopping
    adam: V.AdamCfg = None      # learning-rate schedule for this stage (None: the trainer's)


def static_stages(d_h, steps):
    return [Stage(d_h, steps)]


def adaptive_stages(d_start, d_final, steps_per_stage):
    out, d = [], d_start
    while d <= d_final:
        out.append(Stage(d, steps_per_stage))
        d *= 2
    return out


def interval_stages(d_start, d_final, total_steps, interval):
    """Widths doubling every `interval` steps from d_start to d_final; the
    last width runs the rest of total_steps (Sec. III: the 1D, long-range and
    cluster Adaptive runs double at a fixed step count)."""
    out = adaptive_stages(d_start, d_final, interval)
    rest = total_steps - interval * (len(out) - 1)
    if rest <= 0:
        raise ValueError("total_steps must exceed (number of widths - 1) x interval")
    out[-1].steps = rest
    return out


@dataclass
class TrainResult:
    energy: np.ndarray = field(default_factory=lambda: np.zeros(0))      # Re E per step
    variance: np.ndarray = field(default_factory=lambda: np.zeros(0))    # sigma^2 per step
    d_h: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    stage_steps: list = field(default_factory=list)
    wall_s: float = 0.0
    samples: int = 0


class Trainer:
    """Trains one RNN wave function with VMC + Adam through the C ABI.

    model: dict(dims, Lx, Ly, is_complex, glu, precision); ham: vmc_ham;
    ns: samples per step; stages: list of Stage; adam: AdamCfg (learning
    rate as a function of the global step, Table III); noise_std: std of the
    padding noise of grow_hidden (Sec. II B); early_stop: EarlyStop, used by
    stages with steps = 0."""

    def __init__(self, model, ham, ns, stages, adam, seed=0, sample_seed=1, noise_std=1e-3, grow_seed=2,
                 early_stop=None, init_params=None, graph=True, device="cuda", restart_adam=False):
        self.mkw = dict(model)
        self.ham = ham
        self.ns = ns
        self.stages = stages
        self.adam = adam
        self.seed = seed
        self.sample_seed = sample_seed
        self.noise_std = noise_std
        self.grow_seed = grow_seed
        self.early_stop = early_stop or EarlyStop()
        self.graph = graph
        self.restart_adam = restart_adam
        self.dev = torch.device(device)
        d0 = stages[0].d_h
        self.m = self._model(d0)
        if init_params is None:
            spec = synth.ModelSpec(dims=self.mkw["dims"], Lx=self.mkw["Lx"], Ly=self.mkw.get("Ly", 1), d_h=d0,
                                   is_complex=bool(self.mkw.get("is_complex", False)),
                                   glu=bool(self.mkw.get("glu", False)))
            init_params = synth.xavier_params(spec, seed)
        self.params = torch.as_tensor(init_params, dtype=torch.float32).to(self.dev).contiguous()
        self.mom_m = torch.zeros_like(self.params)
        self.mom_v = torch.zeros_like(self.params)
        self.t_dev = torch.zeros(1, dtype=torch.int64, device=self.dev)      # Adam steps done
        self.ctr_dev = torch.zeros(1, dtype=torch.int64, device=self.dev)    # Philox counter

    def _model(self, d_h):
        k = self.mkw
        return V.model(dims=k["dims"], Lx=k["Lx"], Ly=k.get("Ly", 1), d_h=d_h, is_complex=k.get("is_complex", False),
                       glu=k.get("glu", False), precision=k.get("precision", V.VMC_FP32))

    def _grow(self, new_dh):
        p, mm, vv, to = V.grow_hidden(self.m, self.params, new_dh, self.grow_seed + new_dh, self.noise_std,
                                      self.mom_m, self.mom_v)
        self.params, self.mom_m, self.mom_v, self.m = p, mm, vv, to
        if self.restart_adam:  # a fresh optimiser state for the new width (moments 0, step count 0)
            self.mom_m.zero_()
            self.mom_v.zero_()
            self.t_dev.zero_()

    def _stage_buffers(self, hist_len):
        ns, m, dev = self.ns, self.m, self.dev
        self.ws = V.Workspace(dev)
        self.ws.get(V.workspace_size(m, self.ham, ns))
        self.out = (torch.empty((ns, m.N), dtype=torch.uint8, device=dev),
                    torch.empty(ns, dtype=torch.float32, device=dev),
                    torch.empty(ns, dtype=torch.float32, device=dev),
                    torch.empty((ns, 2), dtype=torch.float64, device=dev),
                    torch.empty(V.param_count(m), dtype=torch.float64, device=dev),
                    torch.empty(4, dtype=torch.float64, device=dev))
        self.hist = torch.zeros((hist_len, 4), dtype=torch.float64, device=dev)
        self.hist_idx = torch.zeros(1, dtype=torch.int64, device=dev)

    def _step(self, cfg):
        """One training step: VMC step, record its statistics, Adam update."""
        V.vmc_step(self.m, self.params, self.ham, self.ns, seed=self.sample_seed, ws=self.ws, out=self.out,
                   counter_dev=self.ctr_dev)
        self.hist.index_copy_(0, self.hist_idx, self.out[5].view(1, 4))
        self.hist_idx.add_(1)
        V.adam(self.params, self.out[4], self.mom_m, self.mom_v, self.t_dev, cfg)

    def run(self, check_every=500, log=None):
        res = TrainResult()
        energies, variances, dhs = [], [], []
        t0 = time.perf_counter()
        N = self.m.N
        for si, st in enumerate(self.stages):
            if si > 0:
                self._grow(st.d_h)
            cfg = st.adam or self.adam
            fixed = st.steps > 0
            budget = st.steps if fixed else self.early_stop.max_steps_per_stage
            chunk = min(check_every, budget)
            self._stage_buffers(chunk)
            es = None if fixed else EarlyStopState(self.early_stop, st.d_h)
            graph = None
            done = 0
            while done < budget:
                n = min(chunk, budget - done)
                self.hist_idx.zero_()
                if self.graph and n == chunk:
                    if graph is None:
                        # warm-up on a side stream (launch attributes), then capture one step;
                        # the warm-up is a real training step and is recorded like the others
                        side = torch.cuda.Stream()
                        side.wait_stream(torch.cuda.current_stream())
                        with torch.cuda.stream(side):
                            self._step(cfg)
                        torch.cuda.current_stream().wait_stream(side)
                        torch.cuda.synchronize()
                        graph = torch.cuda.CUDAGraph()
                        with torch.cuda.graph(graph):
                            self._step(cfg)
                        n_run = n - 1
                    else:
                        n_run = n
                    for _ in range(n_run):
                        graph.replay()
                else:
                    for _ in range(n):
                        self._step(cfg)
                h = self.hist[:n].cpu().numpy()  # synchronises
                energies.append(h[:, 0])
                variances.append(h[:, 2])
                dhs.append(np.full(n, st.d_h, np.int32))
                done += n
                if log:
                    log("d_h %d step %d/%s E %.8f var/N %.3e" % (st.d_h, done, budget if fixed else "-",
                                                                 h[-1, 0], h[-1, 2] / N))
                if es is not None and es.update(h[:, 2] / N if self.early_stop.per_spin else h[:, 2]) is not None:
                    break
            res.stage_steps.append(done)
            del graph
        torch.cuda.synchronize()
        res.wall_s = time.perf_counter() - t0
        res.energy = np.concatenate(energies)
        res.variance = np.concatenate(variances)
        res.d_h = np.concatenate(dhs)
        res.samples = int(res.energy.size) * self.ns
        return res

    def evaluate(self, n_samples, batch=100000, seed=12345, precision=None):
        """Energy and variance of the trained state from n_samples fresh
        samples (Tables I and II use 10^6): (E, error bar of E, sigma^2,
        error bar of sigma^2), error bars from the Gaussian assumption.
        precision: evaluate the same parameters at another operand precision
        (e.g. a BF16-trained state in FP32); default: the training one."""
        m = self.m
        if precision is not None:
            k = dict(self.mkw)
            k["precision"] = precision
            m = V.model(dims=k["dims"], Lx=k["Lx"], Ly=k.get("Ly", 1), d_h=self.m.d_h,
                        is_complex=k.get("is_complex", False), glu=k.get("glu", False), precision=precision)
        es = []
        k = 0
        while k < n_samples:
            b = min(batch, n_samples - k)
            cfg, _, _ = V.rnn_sample(m, self.params, b, seed=seed, counter=k // batch)
            e = V.local_energy(m, self.params, self.ham, cfg)
            es.append(e.cpu().numpy())
            k += b
        e = np.concatenate(es)
        z = e[:, 0] + 1j * e[:, 1]
        mean = z.mean()
        var = float(np.mean(np.abs(z - mean) ** 2))
        n = len(z)
        return float(mean.real), math.sqrt(var / n), var, var * math.sqrt(2.0 / (n - 1))


def _main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="VMC training of an RNN wave function (Static, Adaptive or "
                                             "Adaptive with early stopping), Table III settings")
    ap.add_argument("--ham", default="tfim", choices=["tfim", "heisenberg", "lrtfim", "cluster"])
    ap.add_argument("--N", type=int, default=20, help="chain length, or Lx of a 2D lattice")
    ap.add_argument("--Ly", type=int, default=1, help="> 1: 2D zig-zag RNN with GLU on an N x Ly lattice")
    ap.add_argument("--mode", default="static", choices=["static", "adaptive", "early"])
    ap.add_argument("--d-final", type=int, default=256)
    ap.add_argument("--d-start", type=int, default=2)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--stage-steps", type=int, default=0,
                    help="adaptive: steps between doublings (the last width runs the rest); 0: equal stages")
    ap.add_argument("--ns", type=int, default=100)
    ap.add_argument("--lr", type=float, default=None,
                    help="learning rate (default 5e-4; early stopping: the rate from d_h = 64 on, default 1e-4)")
    ap.add_argument("--lr-first", type=float, default=None,
                    help="static/adaptive: rate of the first half (two-value schedule); early: rate below d_h = 64")
    ap.add_argument("--decay-start", type=int, default=0, help="step from which the rate decays")
    ap.add_argument("--decay-tau", type=float, default=0.0, help="lr / (1 + (k - start) / tau); 0: no decay")
    ap.add_argument("--h", type=float, default=1.0)
    ap.add_argument("--J", type=float, default=1.0)
    ap.add_argument("--alpha", type=float, default=0.1)
    ap.add_argument("--marshall", action="store_true", help="Heisenberg with the Marshall sign rule")
    ap.add_argument("--complex", action="store_true")
    ap.add_argument("--bf16", action="store_true", help="BF16 MFMA operands")
    ap.add_argument("--eval-samples", type=int, default=10 ** 6)
    ap.add_argument("--eval-fp32", action="store_true", help="evaluate the trained parameters with FP32 operands")
    ap.add_argument("--check-every", type=int, default=500, help="steps between host reads of the history")
    ap.add_argument("--patience", type=int, default=10000, help="early stopping: steps without improvement")
    ap.add_argument("--max-stage-steps", type=int, default=10 ** 7, help="early stopping: cap per width")
    ap.add_argument("--stop-per-spin", action="store_true", help="early stopping on sigma^2/N instead of sigma^2")
    ap.add_argument("--restart-adam", action="store_true",
                    help="fresh Adam state at each width change instead of the carried (zero-padded) one")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--quiet", action="store_true")
    a = ap.parse_args()
    kinds = {"tfim": V.VMC_TFIM, "heisenberg": V.VMC_HEISENBERG, "lrtfim": V.VMC_LRTFIM, "cluster": V.VMC_CLUSTER}
    H = V.ham(kinds[a.ham], J=a.J, h=a.h, marshall=a.marshall, alpha=a.alpha)
    decay = dict(t_decay=a.decay_start, tau=a.decay_tau)
    if a.mode == "static":
        stages = static_stages(a.d_final, a.steps)
    elif a.mode == "adaptive":
        n_st = int(round(math.log2(a.d_final / a.d_start))) + 1
        try:
            stages = (interval_stages(a.d_start, a.d_final, a.steps, a.stage_steps) if a.stage_steps
                      else adaptive_stages(a.d_start, a.d_final, a.steps // n_st))
        except ValueError as e:
            ap.error(str(e))
    else:
        # early stopping (Table III): 0.01 below d_h = 64, 1e-4 from d_h = 64 on
        hi = V.adam_cfg(lr0=a.lr_first if a.lr_first is not None else 1e-2, **decay)
        lo = V.adam_cfg(lr0=a.lr if a.lr is not None else 1e-4, **decay)
        stages = [Stage(d, 0, hi if d < 64 else lo)
                  for d in (2 ** k for k in range(int(math.log2(a.d_start)), int(math.log2(a.d_final)) + 1))]
    lr = a.lr if a.lr is not None else 5e-4
    if a.lr_first is not None and a.mode != "early":
        adam = V.adam_cfg(lr0=a.lr_first, lr1=lr, t_switch=a.steps // 2, **decay)
    else:
        adam = V.adam_cfg(lr0=lr, **decay)
    two_d = a.Ly > 1
    model = dict(dims=2 if two_d else 1, Lx=a.N, Ly=a.Ly, is_complex=a.complex, glu=two_d,
                 precision=V.VMC_BF16 if a.bf16 else V.VMC_FP32)
    tr = Trainer(model, H, a.ns, stages, adam, seed=a.seed,
                 early_stop=EarlyStop(patience=a.patience, max_steps_per_stage=a.max_stage_steps,
                                      per_spin=a.stop_per_spin), restart_adam=a.restart_adam)
    res = tr.run(check_every=a.check_every, log=None if a.quiet else (lambda s: print(s, flush=True)))
    n_sites = a.N * a.Ly
    out = dict(ham=a.ham, N=a.N, Ly=a.Ly, mode=a.mode, stages=[s.d_h for s in stages], stage_steps=res.stage_steps,
               ns=a.ns, train_wall_s=round(res.wall_s, 2), train_samples_per_s=round(res.samples / res.wall_s, 1),
               ms_per_step=round(1e3 * res.wall_s / max(1, res.energy.size), 4),
               last_energy_mean_1000=float(res.energy[-1000:].mean()),
               stage_end_energy=[float(res.energy[:e][-min(100, n):].mean())
                                 for e, n in zip(np.cumsum(res.stage_steps), res.stage_steps)],
               precision="bf16" if a.bf16 else "fp32")
    if a.eval_samples > 0:
        E, dE, var, dvar = tr.evaluate(a.eval_samples, precision=V.VMC_FP32 if a.eval_fp32 else None)
        out["eval_precision"] = "fp32" if (a.eval_fp32 or not a.bf16) else "bf16"
        out.update(energy=E, energy_err=dE, var_per_spin=var / n_sites, var_per_spin_err=dvar / n_sites,
                   eval_samples=a.eval_samples)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    _main()
