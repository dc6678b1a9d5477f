"""Throughput of one VMC step (sample + local energy + gradient) of the 2D GRU
RNN wave function on one MI355X.

Workload: 2D transverse-field Ising model on a 10x10 open square lattice,
J = 1, h = 3; zig-zag 2D GRU with GLU, positive amplitudes; d_h = 64 weights
(Xavier-uniform, seed 0) grown to d_h = 128 by grow_hidden (noise std 1e-3,
seed 2); Ns = 10000 samples per step drawn with the on-device Philox stream
(seed 1, counter = step).  A step is one vmc_step call: sampling, the local
energy (all 100 spin flips of every sample in one launch) and the gradient,
sharing one forward pass; parameters are resident in HBM before the timed
region.

Prints one JSON line.  `roofline` is for the dominant kernel (the batched
suffix-chain launch of local_energy), timed with HIP events on its stream;
`cpu_baseline` is the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "VMC samples/s (sample+E_loc+grad), 2D RNN 10×10 d_h=128; BF16 vs FP32"
LX = LY = 10
N = LX * LY
DH0, DH = 64, 128
NS = 10000
H_FIELD, J_COUP = 3.0, 1.0
PEAK_TF = {"bf16": 2500.0, "fp32": 157.3}


# HBM traffic of the chain kernel, measured with rocprofv3 counters
# (FETCH_SIZE, WRITE_SIZE, scaled by the same counters on a plain copy of
# known size); valid only for the engine sources it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rnn_engine_chain_tfim2d_10x10_dh128_bf16.json")
ENGINE_SOURCES = ["engine_impl.h", "engine.hip", "engine_bf16_2d.hip", "common.h", "kernels.h"]


def engine_source_hash():
    h = hashlib.sha256()
    for f in ENGINE_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_18700_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Bytes per chain launch from the committed counter summary, or None if
    it was taken on other engine sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    return t.get("bytes_per_launch") if t.get("engine_source_hash") == engine_source_hash() else None


def copy_calibration(nbytes):
    """A plain device copy of known size (the counter calibration run)."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_bytes": nbytes, "launches": 3, "ms_last": round(dt * 1e3, 3),
                      "engine_source_hash": engine_source_hash()}))


def site_flops(dh, n_out=2):
    # 2D cell [2dh -> 3dh] + GLU [dh -> 2dh] + heads [dh -> n_out], 2 flops per MAC
    return 2 * (2 * dh) * (3 * dh) + 2 * dh * (2 * dh) + 2 * dh * n_out


def build_params(torch, V, synth):
    spec0 = synth.ModelSpec(dims=2, Lx=LX, Ly=LY, d_h=DH0, glu=True)
    p0 = torch.from_numpy(synth.xavier_params(spec0, 0)).cuda()
    m0 = V.model(dims=2, Lx=LX, Ly=LY, d_h=DH0, glu=True)
    p1, _ = V.grow_hidden(m0, p0, DH, 2, 1e-3)
    return p1


def run_gpu(torch, V, params, precision, steps, warmup, tune=True):
    m = V.model(dims=2, Lx=LX, Ly=LY, d_h=DH, glu=True,
                precision=V.VMC_BF16 if precision == "bf16" else V.VMC_FP32)
    H = V.ham(V.VMC_TFIM, J=J_COUP, h=H_FIELD)
    ws = V.Workspace()
    ws.get(V.workspace_size(m, H, NS))
    dev = params.device
    cfg = torch.empty((NS, N), dtype=torch.uint8, device=dev)
    lp = torch.empty(NS, dtype=torch.float32, device=dev)
    ph = torch.empty(NS, dtype=torch.float32, device=dev)
    e = torch.empty((NS, 2), dtype=torch.float64, device=dev)
    g = torch.empty(V.param_count(m), dtype=torch.float64, device=dev)
    st = torch.empty(4, dtype=torch.float64, device=dev)

    def step(i):
        V.vmc_step(m, params, H, NS, seed=1, counter=i, ws=ws, out=(cfg, lp, ph, e, g, st))

    # launch choices from the autotuner (untimed set-up; no choice changes a result bit)
    tuning = None
    if tune:
        _, tuning = V.autotune_step(m, params, H, NS, seed=1, counter=0, ws=ws, out=(cfg, lp, ph, e, g, st), reps=2)
    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    V.chain_timing(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record()
    for i in range(steps):
        step(warmup + i)
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    chain_ms, launches = V.chain_time()
    V.chain_timing(False)
    ms = t0.elapsed_time(t1) / steps
    # the configurations and energies of the last step, for the accuracy check
    return dict(ms_per_step=ms, wall_s=wall, chain_ms=chain_ms / max(launches, 1), launches=launches, tuning=tuning,
                cfg=cfg.clone(), e=e.clone(), stats=st.clone(), counter=warmup + steps - 1)


def cpu_baseline(torch, params, cfg, e_gpu, n_sub):
    """FP64 oracle (test infrastructure) on the first n_sub samples of the same
    step: sampling from the same Philox uniforms, the local energy of every
    sample and the gradient; also the energy-per-site error of the GPU."""
    import numpy as np
    from oracle import oracle as O
    om = O.model(dims=2, Lx=LX, Ly=LY, d_h=DH, glu=True)
    p = params.cpu().numpy().astype(np.float64)
    c = cfg[:n_sub].cpu().numpy()
    t = time.perf_counter()
    uni = O.philox_uniforms(1, 0, n_sub, N)
    O.sample(om, p, uni)
    eo = O.local_energy(om, p, O.ham(O.TFIM, J=J_COUP, h=H_FIELD), c)
    O.grad(om, p, c, eo)
    dt = time.perf_counter() - t
    eg = e_gpu[:n_sub].cpu().numpy()
    err = abs(eg[:, 0].mean() - eo.real.mean()) / N
    return dict(value=n_sub / dt, unit="samples/s", cores=O.num_threads(), kind="oracle",
                sample="first %d of the %d samples of one step (FP64 sample + E_loc with full "
                       "re-evaluation + gradient), %.1f s" % (n_sub, NS, dt)), err


def _timed(torch, fn, reps):
    """Milliseconds per call of fn (one call untimed first), HIP events on the current stream."""
    fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def zigzag_pos(Lx, Ly):
    """Order position of every lattice site (zig-zag: even rows left to right)."""
    import numpy as np
    pos = np.zeros(Lx * Ly, dtype=np.int64)
    for j in range(Ly):
        for i in range(Lx):
            pos[j * Lx + i] = j * Lx + (i if j % 2 == 0 else Lx - 1 - i)
    return pos


def other_workloads(torch, V, synth, reps=3):
    """The other configurations of the path, each timed as one vmc_step (or
    the batch graph) after the autotuner; C4 also times local_energy on
    configurations with 74 % anti-aligned bonds and reports the connection
    count and the chain kernel's fraction of the bf16 peak."""
    import numpy as np
    out = {}

    def step_rate(m, p, H, ns, name, extra=None):
        ws = V.Workspace()
        ws.get(V.workspace_size(m, H, ns))
        res = V.vmc_step(m, p, H, ns, seed=1, counter=0, ws=ws)
        V.autotune_step(m, p, H, ns, seed=1, counter=0, ws=ws, out=res, reps=1)
        ms = _timed(torch, lambda: V.vmc_step(m, p, H, ns, seed=1, counter=1, ws=ws, out=res), reps)
        out[name] = dict(samples_per_s=round(ns / (ms * 1e-3), 1), ms_per_step=round(ms, 3), ns=ns, **(extra or {}))
        return ws, res

    # C1: 1D TFIM N=20, J=h=1, d_h=16, Ns=1000 (FP32 path)
    spec = synth.ModelSpec(dims=1, Lx=20, d_h=16)
    m = V.model(dims=1, Lx=20, d_h=16, precision=V.VMC_FP32)
    step_rate(m, torch.from_numpy(synth.xavier_params(spec, 0)).cuda(), V.ham(V.VMC_TFIM, 1.0, 1.0), 1000,
              "c1_tfim1d_N20_dh16_fp32")
    # C2: 1D Heisenberg N=50 (Marshall), complex RNN d_h 32 -> 64, Ns=10^4 (FP32)
    spec = synth.ModelSpec(dims=1, Lx=50, d_h=32, is_complex=True)
    m0 = V.model(dims=1, Lx=50, d_h=32, is_complex=True)
    p2, m2 = V.grow_hidden(m0, torch.from_numpy(synth.xavier_params(spec, 0)).cuda(), 64, 2, 1e-3)
    step_rate(m2, p2, V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True), 10000, "c2_heis1d_N50_dh64_cplx_fp32")
    # C4: 2D Heisenberg 16x16 (Marshall), complex RNN + GLU d_h=256, Ns=4096 (BF16)
    spec = synth.ModelSpec(dims=2, Lx=16, Ly=16, d_h=256, is_complex=True, glu=True)
    m4 = V.model(dims=2, Lx=16, Ly=16, d_h=256, is_complex=True, glu=True, precision=V.VMC_BF16)
    p4 = torch.from_numpy(synth.xavier_params(spec, 0)).cuda()
    H4 = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True)
    ws4, _ = step_rate(m4, p4, H4, 4096, "c4_heis2d_16x16_dh256_cplx_bf16")
    cfg = synth.neel_like_configs(4096, 16, 16, 5, 0.74)
    a = cfg.reshape(4096, 16, 16)
    anti_h, anti_v = a[:, :, 1:] != a[:, :, :-1], a[:, 1:, :] != a[:, :-1, :]
    pos = zigzag_pos(16, 16).reshape(16, 16)
    first_h = np.minimum(pos[:, 1:], pos[:, :-1])[None].repeat(4096, 0)
    first_v = np.minimum(pos[1:, :], pos[:-1, :])[None].repeat(4096, 0)
    suffix = (255 - first_h)[anti_h].sum() + (255 - first_v)[anti_v].sum()
    nconn = (anti_h.sum() + anti_v.sum()) / 4096.0
    dcfg = torch.from_numpy(cfg).cuda()
    e = V.local_energy(m4, p4, H4, dcfg, ws=ws4)
    torch.cuda.synchronize()
    V.chain_timing(True)
    ms = _timed(torch, lambda: V.local_energy(m4, p4, H4, dcfg, ws=ws4, out=e), reps)
    chain_ms, launches = V.chain_time()
    V.chain_timing(False)
    chain_ms /= max(launches, 1)
    f_site = 16 * 256 * 256 + 2 * 256 * 4
    out["c4_local_energy_74pct_anti"] = dict(
        configs_per_s=round(4096 / (ms * 1e-3), 1), ms=round(ms, 3), mean_connections=round(float(nconn), 1),
        chain_ms=round(chain_ms, 3),
        chain_frac_of_bf16_peak=round(float(suffix) * f_site / (chain_ms * 1e-3) / 1e12 / PEAK_TF["bf16"], 4))
    # C5: 32 uneven 1D TFIM chains (N 32..128, h 0.5..1.5), d_h=64, Ns=2048 each, BF16, one graph
    problems = []
    for c, (n, h) in enumerate(synth.uneven_chains(32, 3)):
        spec = synth.ModelSpec(dims=1, Lx=n, d_h=64)
        problems.append(dict(model=V.model(dims=1, Lx=n, d_h=64, precision=V.VMC_BF16),
                             params=torch.from_numpy(synth.xavier_params(spec, 100 + c)).cuda(),
                             ham=V.ham(V.VMC_TFIM, 1.0, h), ns=2048, seed=1, counter=0))
    b = V.StepBatch(problems, streams=8)
    b.run_eager()
    b.autotune(reps=1)
    b.capture()
    ms = _timed(torch, b.replay, reps)
    out["c5_32_uneven_tfim1d_dh64_bf16"] = dict(samples_per_s=round(32 * 2048 / (ms * 1e-3), 1),
                                                 ms_per_batch_step=round(ms, 3), chains=32)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-samples", type=int, default=768)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="built-in launch choices instead of the autotuner's")
    ap.add_argument("--no-other", action="store_true", help="skip the other workloads (C1, C2, C4, C5)")
    ap.add_argument("--only-other", action="store_true",
                    help="only the other workloads, printed as their own JSON line (profiling runs)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    import torch
    from paper_2507_18700_amd import synth, vmcrnn as V
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.only_other:
        print(json.dumps({"other_workloads": other_workloads(torch, V, synth)}))
        return
    params = build_params(torch, V, synth)
    torch.cuda.synchronize()
    print("bench: params ready (%d floats), timing BF16 path" % params.numel(), file=sys.stderr, flush=True)
    bf = run_gpu(torch, V, params, "bf16", args.steps, args.warmup, tune=not args.no_tune)
    print("bench: bf16 %.2f ms/step" % bf["ms_per_step"], file=sys.stderr, flush=True)
    fp = None
    if not args.no_fp32:
        fp = run_gpu(torch, V, params, "fp32", max(1, min(args.steps, 3)), 1, tune=not args.no_tune)
        print("bench: fp32 %.2f ms/step" % fp["ms_per_step"], file=sys.stderr, flush=True)

    flops_chain = NS * (N * (N - 1) // 2) * site_flops(DH)
    flops_step = NS * (N + N * (N - 1) // 2 + 2 * N) * site_flops(DH)
    achieved = flops_chain / (bf["chain_ms"] * 1e-3) / 1e12
    value = NS / (bf["ms_per_step"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(bf["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "2D TFIM 10x10 open, J=1, h=3; zig-zag 2D GRU + GLU, positive RNN, "
                               "d_h 64->128 via grow_hidden; Ns=10000 per step; sample + E_loc + grad",
                   "Lx": LX, "Ly": LY, "d_h": DH, "ns": NS, "precision": "bf16 MFMA operands, fp32 accumulate, "
                                                                         "fp64 cross-sample reductions"},
        "roofline": {"bound": "mfma", "kernel": "rnn_engine<BF16,2,128> chain launch (suffix chains of local_energy)",
                     "achieved": round(achieved, 2), "peak": PEAK_TF["bf16"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TF["bf16"], 4), "traffic": measured_traffic(),
                     "flops_per_launch": flops_chain, "avg_launch_ms": round(bf["chain_ms"], 3)},
        "step_flops_algorithmic": flops_step,
        "step_frac_of_bf16_peak": round(flops_step / (bf["ms_per_step"] * 1e-3) / 1e12 / PEAK_TF["bf16"], 4),
        "tuning": bf["tuning"],
    }
    if fp is not None:
        out["fp32"] = {"value": round(NS / (fp["ms_per_step"] * 1e-3), 1), "ms_per_step": round(fp["ms_per_step"], 3),
                       "chain_avg_launch_ms": round(fp["chain_ms"], 3),
                       "chain_frac_of_fp32_peak": round(flops_chain / (fp["chain_ms"] * 1e-3) / 1e12 / PEAK_TF["fp32"], 4),
                       "bf16_speedup": round(fp["ms_per_step"] / bf["ms_per_step"], 3), "tuning": fp["tuning"]}
    if not args.no_other:
        print("bench: other workloads", file=sys.stderr, flush=True)
        out["other_workloads"] = other_workloads(torch, V, synth)
    if not args.no_cpu:
        cb, err_bf = cpu_baseline(torch, params, bf["cfg"], bf["e"], args.cpu_samples)
        out["cpu_baseline"] = cb
        acc = {"energy_per_site_err_bf16": err_bf}
        if fp is not None:
            # same configurations through the FP32 path
            m32 = V.model(dims=2, Lx=LX, Ly=LY, d_h=DH, glu=True, precision=V.VMC_FP32)
            e32 = V.local_energy(m32, params, V.ham(V.VMC_TFIM, J=J_COUP, h=H_FIELD), bf["cfg"])
            _, err32 = cpu_baseline(torch, params, bf["cfg"], e32, min(32, args.cpu_samples))
            acc["energy_per_site_err_fp32_first32"] = err32
        acc["reference"] = "FP64 oracle on the first samples of the last timed step"
        out["accuracy"] = acc
    print(json.dumps(out))


if __name__ == "__main__":
    main()
