"""Throughput of one VMC step (sample + local energy + gradient) of the 2D GRU
RNN wave function on one MI355X.

Workload: 2D transverse-field Ising model on a 10x10 open square lattice,
J = 1, h = 3; zig-zag 2D GRU with GLU, positive amplitudes; d_h = 64 weights
(Xavier-uniform, seed 0) grown to d_h = 128 by grow_hidden (noise std 1e-3,
seed 2); Ns = 10000 samples per step drawn with the on-device Philox stream
(seed 1).  A step is one vmc_step call: sampling, the local energy (all 100
spin flips of every sample in one launch) and the gradient, sharing one
forward pass; parameters are resident in HBM before the timed region.

Timing: the step is captured once as a HIP graph whose Philox counter lives
in device memory (every replay draws fresh samples, counter = replay index);
W untimed replays, then K timed replays, each bracketed by HIP events on the
stream; ms_per_step is the median.  The dominant kernel (the batched
suffix-chain launch of local_energy) is timed with the library's HIP events
on its stream over K eager steps of the same workload.

Prints one JSON line.  `roofline` is for the dominant kernel; `cpu_baseline`
is the FP64 oracle on a bounded sample of the last timed step; `accuracy`
states the error of every result against the FP64 oracle on that sample.
"""
import argparse
import hashlib
import json
import os
import platform
import re
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
# Transcendental issue rate of gfx950 (v_exp_f32, v_rcp_f32): half rate, 8 lanes
# per clock per SIMD: 256 CUs x 4 SIMDs x 8 x 2.4 GHz.
PEAK_TRANS_T = 256 * 4 * 8 * 2.4e9 / 1e12


# HBM traffic of the chain kernel, measured with rocprofv3 counters
# (FETCH_SIZE, WRITE_SIZE, scaled by the same counters on a plain copy of
# known size); valid only for the engine code it was measured on (the hash
# covers the code: comments and whitespace do not enter it).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rnn_engine_chain_tfim2d_10x10_dh128_bf16.json")
ENGINE_SOURCES = ["engine_impl.h", "engine.hip", "engine_bf16_2d.hip", "common.h", "kernels.h"]


def engine_source_hash():
    h = hashlib.sha256()
    for f in ENGINE_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_18700_amd", "csrc", f)) as fh:
            src = fh.read()
        # (the engine sources hold no string literal with a comment marker)
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def build_params(torch, V, synth):
    spec0 = synth.ModelSpec(dims=2, Lx=LX, Ly=LY, d_h=DH0, glu=True)
    p0 = torch.from_numpy(synth.xavier_params(spec0, 0)).cuda()
    m0 = V.model(dims=2, Lx=LX, Ly=LY, d_h=DH0, glu=True)
    p1, _ = V.grow_hidden(m0, p0, DH, 2, 1e-3)
    return p1


def step_outputs(torch, V, m, ns, dev):
    return (torch.empty((ns, m.N), dtype=torch.uint8, device=dev), torch.empty(ns, dtype=torch.float32, device=dev),
            torch.empty(ns, dtype=torch.float32, device=dev), torch.empty((ns, 2), dtype=torch.float64, device=dev),
            torch.empty(V.param_count(m), dtype=torch.float64, device=dev),
            torch.empty(4, dtype=torch.float64, device=dev))


def replay_times(torch, fn_replay, steps, warmup):
    """Median and mean milliseconds of `steps` timed replays after `warmup`
    untimed ones; each replay bracketed by HIP events on the current stream
    (no host synchronisation between replays), plus the host wall time."""
    import numpy as np
    for _ in range(warmup):
        fn_replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    wall0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn_replay()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return float(np.median(t)), float(t.mean()), wall


def capture(torch, fn):
    """One untimed call on a side stream (launch attributes), then a HIP graph of fn."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def run_gpu(torch, V, params, precision, steps, warmup, tune=True):
    m = V.model(dims=2, Lx=LX, Ly=LY, d_h=DH, glu=True,
                precision=V.VMC_BF16 if precision == "bf16" else V.VMC_FP32)
    H = V.ham(V.VMC_TFIM, J=J_COUP, h=H_FIELD)
    ws = V.Workspace()
    ws.get(V.workspace_size(m, H, NS))
    out = step_outputs(torch, V, m, NS, params.device)
    # launch choices from the autotuner (untimed set-up; no choice changes a result bit)
    tuning = None
    if tune:
        _, tuning = V.autotune_step(m, params, H, NS, seed=1, counter=0, ws=ws, out=out, reps=2)
    # the dominant kernel: library events around the chain launch of eager steps
    for i in range(warmup):
        V.vmc_step(m, params, H, NS, seed=1, counter=i, ws=ws, out=out)
    torch.cuda.synchronize()
    V.chain_timing(True)
    for i in range(steps):
        V.vmc_step(m, params, H, NS, seed=1, counter=warmup + i, ws=ws, out=out)
    torch.cuda.synchronize()
    chain_ms, launches = V.chain_time()
    V.chain_timing(False)
    # the headline: graph replays with the device-resident counter
    ctr = torch.zeros(1, dtype=torch.int64, device=params.device)
    g = capture(torch, lambda: V.vmc_step(m, params, H, NS, seed=1, ws=ws, out=out, counter_dev=ctr))
    ctr.zero_()
    med, mean, wall = replay_times(torch, g.replay, steps, warmup)
    assert int(ctr.item()) == warmup + steps
    # the configurations and energies of the last replay (counter warmup + steps - 1)
    return dict(ms_per_step=med, ms_mean=mean, wall_s=wall, chain_ms=chain_ms / max(launches, 1), launches=launches,
                tuning=tuning, m=m, out=[t.clone() for t in out], counter=warmup + steps - 1, ws=ws)


def accuracy_and_cpu(torch, V, params, bf, n_sub, n_one):
    """The FP64 oracle (test infrastructure) on the first n_sub samples of
    the last timed step: its own sampling from the same Philox uniforms, the
    local energies of the GPU's configurations (full re-evaluation) and the
    gradient with the GPU's energies (timed: the CPU baseline, all threads,
    then n_one samples on one thread); and the error of every GPU result on
    those samples."""
    import numpy as np
    from oracle import oracle as O
    om = O.model(dims=2, Lx=LX, Ly=LY, d_h=DH, glu=True)
    oh = O.ham(O.TFIM, J=J_COUP, h=H_FIELD)
    p = params.cpu().numpy().astype(np.float64)
    cfg_all, lp_all, _, e_all, _, _ = [t.cpu().numpy() for t in bf["out"]]
    c, lpg, eg = cfg_all[:n_sub], lp_all[:n_sub].astype(np.float64), e_all[:n_sub]
    w = np.full(n_sub, 1.0 / n_sub)

    def oracle_leg(n):
        uni = O.philox_uniforms(1, bf["counter"], n, N)
        cfg_o, _, _ = O.sample(om, p, uni)
        eo = O.local_energy(om, p, oh, c[:n])
        go, _ = O.grad(om, p, c[:n], eg[:n], np.full(n, 1.0 / n))
        return uni, cfg_o, eo, go

    threads = O.num_threads()
    t = time.perf_counter()
    uni, cfg_o, eo, go = oracle_leg(n_sub)
    dt = time.perf_counter() - t
    O.set_threads(1)
    t = time.perf_counter()
    oracle_leg(n_one)
    dt1 = time.perf_counter() - t
    O.set_threads(threads)
    cpu = dict(value=round(n_sub / dt, 2), unit="samples/s", cores=threads, kind="oracle",
               value_1core=round(n_one / dt1, 3), cpu=cpu_model(), nproc=os.cpu_count(),
               sample="oracle sampling from the Philox uniforms of the last timed step (counter %d), local energy "
                      "of the GPU's configurations with every connected configuration re-evaluated, and the "
                      "gradient, on the first %d of its %d samples (%.1f s on %d threads); one thread: %d samples, "
                      "%.1f s" % (bf["counter"], n_sub, NS, dt, threads, n_one, dt1))
    # errors of every result against the oracle on the same samples
    egc = eg[:, 0] + 1j * eg[:, 1]
    rlp, _, lpc, _ = O.logpsi(om, p, c, conditionals=True)
    p0 = np.exp(lpc[:, :, 0])
    near = (np.abs(uni - p0) < 1e-5).any(axis=1)
    diff = (egc.real - eo.real) / N
    var_g = np.mean(np.abs(egc - egc.mean()) ** 2)
    var_o = np.mean(np.abs(eo - eo.mean()) ** 2)
    # gradient of these samples alone (weights 1/n_sub) and its cancellation factor
    wd = torch.zeros(NS, dtype=torch.float64, device=params.device)
    wd[:n_sub] = 1.0 / n_sub
    gg, _ = V.vmc_grad(bf["m"], params, bf["out"][0], bf["out"][3], weights=wd, ws=bf["ws"])
    gg = gg.cpu().numpy()
    st = O.stats(eg, w)
    _, gabs = O.surrogate_grad_abs(om, p, c, w * (eg[:, 0] - st[0]))
    acc = dict(
        samples=n_sub,
        sample_divergence_frac=float(np.mean((cfg_o != c).any(axis=1))),
        near_tie_rows_1e5=int(near.sum()),
        logpsi_max_rel=float(np.max(np.abs(lpg - rlp) / np.abs(rlp))),
        eloc_l2_rel=float(np.linalg.norm(egc - eo) / np.linalg.norm(eo)),
        eloc_max_rel=float(np.max(np.abs(egc - eo) / np.maximum(np.abs(eo), N))),
        energy_per_site_err=float(abs(diff.mean())),
        energy_per_site_err_stderr=float(diff.std() / np.sqrt(n_sub)),
        energy_per_site_err_rms_per_sample=float(np.sqrt(np.mean(diff ** 2))),
        variance_rel_err=float(abs(var_g - var_o) / var_o),
        grad_l2_rel=float(np.linalg.norm(gg - go) / np.linalg.norm(go)),
        grad_kappa=float(np.linalg.norm(gabs) / np.linalg.norm(go)),
        reference="FP64 oracle on the first samples of the last timed step (sample divergence: the GPU's "
                  "sampling decisions against the oracle's own samples from the same uniforms)")
    return cpu, acc


def other_workloads(torch, V, synth, steps=5, warmup=2):
    """The other configurations of the path, each a graph-replayed step after
    the autotuner (median of `steps` replays): C1, C2 (1D, transcendental
    bound: reported against the transcendental issue rate), C4 (with the
    local energy on configurations with 74 % anti-aligned bonds and the chain
    kernel's fraction of the bf16 peak) and C5 through vmc_step_batched."""
    import numpy as np
    out = {}

    def trans_1d(dh, row_sites):
        # sigmoid(u), sigmoid(r), tanh(c): an exp and a reciprocal each, per unit and row-site
        return 6.0 * dh * row_sites

    def graph_step(m, p, H, ns, name, dh, rows_sites_fn):
        ws = V.Workspace()
        ws.get(V.workspace_size(m, H, ns))
        res = V.vmc_step(m, p, H, ns, seed=1, counter=0, ws=ws)
        V.autotune_step(m, p, H, ns, seed=1, counter=0, ws=ws, out=res, reps=1)
        ctr = torch.zeros(1, dtype=torch.int64, device=p.device)
        g = capture(torch, lambda: V.vmc_step(m, p, H, ns, seed=1, ws=ws, out=res, counter_dev=ctr))
        med, mean, _ = replay_times(torch, g.replay, steps, warmup)
        rs = rows_sites_fn(res[0].cpu().numpy())
        tr = trans_1d(dh, rs) / (med * 1e-3) / 1e12
        out[name] = dict(samples_per_s=round(ns / (med * 1e-3), 1), ms_per_step=round(med, 4), ns=ns,
                         roofline={"bound": "alu", "achieved": round(tr, 3), "peak": round(PEAK_TRANS_T, 2),
                                   "unit": "Tops/s (exp, rcp)", "frac": round(tr / PEAK_TRANS_T, 4)})
        return ws, res

    def tfim_rows(Nc, ns):
        return lambda cfg: ns * (Nc + Nc * (Nc - 1) / 2)

    def heis1d_rows(Nc, ns):
        def f(cfg):
            anti = cfg[:, 1:] != cfg[:, :-1]  # bond (k, k+1): chain over positions k+1..N-1
            return ns * Nc + float((anti * (Nc - 1 - np.arange(Nc - 1))[None, :]).sum())
        return f

    # C1: 1D TFIM N=20, J=h=1, d_h=16, Ns=1000 (FP32 path)
    spec = synth.ModelSpec(dims=1, Lx=20, d_h=16)
    m = V.model(dims=1, Lx=20, d_h=16, precision=V.VMC_FP32)
    graph_step(m, torch.from_numpy(synth.xavier_params(spec, 0)).cuda(), V.ham(V.VMC_TFIM, 1.0, 1.0), 1000,
               "c1_tfim1d_N20_dh16_fp32", 16, tfim_rows(20, 1000))
    # C2: 1D Heisenberg N=50 (Marshall), complex RNN d_h 32 -> 64, Ns=10^4 (FP32)
    spec = synth.ModelSpec(dims=1, Lx=50, d_h=32, is_complex=True)
    m0 = V.model(dims=1, Lx=50, d_h=32, is_complex=True)
    p2, m2 = V.grow_hidden(m0, torch.from_numpy(synth.xavier_params(spec, 0)).cuda(), 64, 2, 1e-3)
    graph_step(m2, p2, V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True), 10000, "c2_heis1d_N50_dh64_cplx_fp32", 64,
               heis1d_rows(50, 10000))
    # C4: 2D Heisenberg 16x16 (Marshall), complex RNN + GLU d_h=256, Ns=4096 (BF16)
    spec = synth.ModelSpec(dims=2, Lx=16, Ly=16, d_h=256, is_complex=True, glu=True)
    m4 = V.model(dims=2, Lx=16, Ly=16, d_h=256, is_complex=True, glu=True, precision=V.VMC_BF16)
    p4 = torch.from_numpy(synth.xavier_params(spec, 0)).cuda()
    H4 = V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True)
    ws4 = V.Workspace()
    ws4.get(V.workspace_size(m4, H4, 4096))
    res4 = V.vmc_step(m4, p4, H4, 4096, seed=1, counter=0, ws=ws4)
    V.autotune_step(m4, p4, H4, 4096, seed=1, counter=0, ws=ws4, out=res4, reps=1)
    ctr4 = torch.zeros(1, dtype=torch.int64, device="cuda")
    g4 = capture(torch, lambda: V.vmc_step(m4, p4, H4, 4096, seed=1, ws=ws4, out=res4, counter_dev=ctr4))
    med4, _, _ = replay_times(torch, g4.replay, 2, 1)
    out["c4_heis2d_16x16_dh256_cplx_bf16"] = dict(samples_per_s=round(4096 / (med4 * 1e-3), 1),
                                                  ms_per_step=round(med4, 3), ns=4096)
    del g4
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
    ms = _timed(torch, lambda: V.local_energy(m4, p4, H4, dcfg, ws=ws4, out=e), 2)
    chain_ms, launches = V.chain_time()
    V.chain_timing(False)
    chain_ms /= max(launches, 1)
    f_site = 16 * 256 * 256 + 2 * 256 * 4
    out["c4_local_energy_74pct_anti"] = dict(
        configs_per_s=round(4096 / (ms * 1e-3), 1), ms=round(ms, 3), mean_connections=round(float(nconn), 1),
        chain_ms=round(chain_ms, 3),
        chain_frac_of_bf16_peak=round(float(suffix) * f_site / (chain_ms * 1e-3) / 1e12 / PEAK_TF["bf16"], 4))
    del ws4, res4
    # C5: 32 uneven 1D TFIM chains (N 32..128, h 0.5..1.5), d_h=64, Ns=2048 each, BF16, one batched step
    chains = synth.uneven_chains(32, 3)
    lens = [n for n, _ in chains]
    hams = [V.ham(V.VMC_TFIM, 1.0, h) for _, h in chains]
    params = torch.from_numpy(np.stack([synth.xavier_params(synth.ModelSpec(dims=1, Lx=n, d_h=64), 100 + c)
                                        for c, n in enumerate(lens)])).cuda()
    m5 = V.model(dims=1, Lx=max(lens), d_h=64, precision=V.VMC_BF16)
    ws5 = V.Workspace()
    res5 = V.vmc_step_batched(m5, lens, hams, params, 2048, seed=1, counter=0, ws=ws5)
    V.chain_timing(True)
    for i in range(steps):
        V.vmc_step_batched(m5, lens, hams, params, 2048, seed=1, counter=i, ws=ws5, out=res5)
    torch.cuda.synchronize()
    c5_chain, n5 = V.chain_time()
    V.chain_timing(False)
    ctr5 = torch.zeros(1, dtype=torch.int64, device="cuda")
    g5 = capture(torch, lambda: V.vmc_step_batched(m5, lens, hams, params, 2048, seed=1, ws=ws5, out=res5,
                                                   counter_dev=ctr5))
    med5, _, _ = replay_times(torch, g5.replay, steps, warmup)
    rows = sum(2048 * (n + n * (n - 1) / 2) for n in lens)
    tr = trans_1d(64, rows) / (med5 * 1e-3) / 1e12
    chain_rows = sum(2048 * n * (n - 1) / 2 for n in lens)
    f1d = 6 * 64 * 64 + 2 * 64 * 2
    out["c5_32_uneven_tfim1d_dh64_bf16"] = dict(
        samples_per_s=round(32 * 2048 / (med5 * 1e-3), 1), ms_per_batch_step=round(med5, 3), chains=32,
        entry="vmc_step_batched (one sampling, one suffix-chain, one reverse-sweep launch for all chains)",
        chain_ms=round(c5_chain / max(n5, 1), 3),
        chain_frac_of_bf16_peak=round(chain_rows * f1d / (c5_chain / max(n5, 1) * 1e-3) / 1e12 / PEAK_TF["bf16"], 4),
        roofline={"bound": "alu", "achieved": round(tr, 3), "peak": round(PEAK_TRANS_T, 2),
                  "unit": "Tops/s (exp, rcp)", "frac": round(tr / PEAK_TRANS_T, 4)})
    return out


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-samples", type=int, default=2048)
    ap.add_argument("--cpu-samples-1core", type=int, default=12)
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
    print("bench: bf16 %.2f ms/step (median of %d graph replays)" % (bf["ms_per_step"], args.steps),
          file=sys.stderr, flush=True)
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
        "timing": {"ms_per_step_median": round(bf["ms_per_step"], 3), "ms_per_step_mean": round(bf["ms_mean"], 3),
                   "wall_s_timed_region": round(bf["wall_s"], 3),
                   "method": "median of HIP-graph replays (device-resident Philox counter), events per replay"},
        "roofline": {"bound": "mfma", "kernel": "rnn_engine<BF16,2,128> chain launch (suffix chains of local_energy)",
                     "achieved": round(achieved, 2), "peak": PEAK_TF["bf16"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TF["bf16"], 4), "traffic": measured_traffic(),
                     "flops_per_launch": flops_chain, "avg_launch_ms": round(bf["chain_ms"], 3),
                     "timed_launches": bf["launches"]},
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
        print("bench: oracle leg", file=sys.stderr, flush=True)
        cb, acc = accuracy_and_cpu(torch, V, params, bf, args.cpu_samples, args.cpu_samples_1core)
        out["cpu_baseline"] = cb
        out["accuracy"] = {"bf16": acc}
        if fp is not None:
            _, acc32 = accuracy_and_cpu(torch, V, params, fp, 32, 1)
            out["accuracy"]["fp32_first32"] = acc32
    print(json.dumps(out))


if __name__ == "__main__":
    main()
