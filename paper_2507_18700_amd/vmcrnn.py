"""Python binding of libvmcrnn.so (the C ABI of include/vmcrnn.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory (outputs and the workspace) and
the current HIP stream.  The functions have the names of the C entry points.
If the library is not built, every call raises; there is no CPU fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; VMCRNN_LIB names another build of the same sources
LIB_PATH = os.environ.get("VMCRNN_LIB") or os.path.join(_HERE, "libvmcrnn.so")

VMC_FP32, VMC_BF16 = 0, 1
VMC_TFIM, VMC_HEISENBERG, VMC_LRTFIM, VMC_CLUSTER = 0, 1, 2, 3
VMC_EINVAL, VMC_EUNSUPPORTED, VMC_ENOSPACE, VMC_EDEVICE, VMC_ENONFINITE = -1, -2, -3, -4, -5

EXPORTS = ("vmc_param_count", "vmc_workspace_size", "rnn_sample", "rnn_logpsi", "rnn_logpsi_grad", "local_energy",
           "vmc_grad", "vmc_energy_stats", "vmc_grad_chunk", "vmc_step", "vmc_step_batched", "vmc_batched_workspace_size", "vmc_step_noalloc",
           "vmc_noalloc_scratch_bytes", "vmc_adam", "vmc_check_finite",
           "grow_hidden", "vmc_row_tile_options",
           "vmc_set_tuning", "vmc_get_tuning", "vmc_autotune_step", "vmc_chain_timing", "vmc_chain_time",
           "vmc_status_str")


class VmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class Model(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("d_h", ctypes.c_int32), ("is_complex", ctypes.c_int32), ("glu", ctypes.c_int32),
                ("precision", ctypes.c_int32)]

    @property
    def N(self):
        return self.Lx * self.Ly


class Ham(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("marshall", ctypes.c_int32), ("J", ctypes.c_double),
                ("h", ctypes.c_double), ("alpha", ctypes.c_double)]


class AdamCfg(ctypes.Structure):
    _fields_ = [("lr0", ctypes.c_double), ("lr1", ctypes.c_double), ("t_switch", ctypes.c_int64),
                ("t_decay", ctypes.c_int64), ("tau", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("row_tile", ctypes.c_int32), ("chain_wgs_per_cu", ctypes.c_int32)]


def model(dims=1, Lx=4, Ly=1, d_h=16, is_complex=False, glu=False, precision=VMC_FP32):
    return Model(dims, Lx, Ly if dims == 2 else 1, d_h, int(is_complex), int(glu), int(precision))


def ham(kind=VMC_TFIM, J=1.0, h=1.0, marshall=False, alpha=0.0):
    return Ham(kind, int(marshall), float(J), float(h), float(alpha))


def adam_cfg(lr0=1e-3, lr1=None, t_switch=0, t_decay=0, tau=0.0, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam settings; lr(k) = (k < t_switch ? lr0 : lr1) / (1 + max(0, k - t_decay) / tau)."""
    return AdamCfg(float(lr0), float(lr0 if lr1 is None else lr1), int(t_switch), int(t_decay), float(tau),
                   float(beta1), float(beta2), float(eps))


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvmcrnn.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i64, u64, sz, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
        L.vmc_param_count.restype = i64
        L.vmc_param_count.argtypes = [P(Model)]
        L.vmc_workspace_size.restype = ctypes.c_int
        L.vmc_workspace_size.argtypes = [P(Model), P(Ham), i64, P(sz)]
        L.rnn_sample.restype = ctypes.c_int
        L.rnn_sample.argtypes = [P(Model), vp, i64, u64, u64, vp, vp, vp, vp, vp, sz, vp]
        L.rnn_logpsi.restype = ctypes.c_int
        L.rnn_logpsi.argtypes = [P(Model), vp, i64, vp, vp, vp, vp, sz, vp]
        L.rnn_logpsi_grad.restype = ctypes.c_int
        L.rnn_logpsi_grad.argtypes = [P(Model), vp, i64, vp, vp, vp, vp, vp, sz, vp]
        L.local_energy.restype = ctypes.c_int
        L.local_energy.argtypes = [P(Model), vp, P(Ham), i64, vp, vp, vp, sz, vp]
        L.vmc_grad.restype = ctypes.c_int
        L.vmc_grad.argtypes = [P(Model), vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.vmc_energy_stats.restype = ctypes.c_int
        L.vmc_energy_stats.argtypes = [i64, vp, vp, vp, vp]
        L.vmc_grad_chunk.restype = ctypes.c_int
        L.vmc_grad_chunk.argtypes = [P(Model), vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.vmc_step.restype = ctypes.c_int
        L.vmc_step.argtypes = [P(Model), vp, P(Ham), i64, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.vmc_step_batched.restype = ctypes.c_int
        L.vmc_step_batched.argtypes = [ctypes.c_int32, P(Model), P(ctypes.c_int32), P(Ham), vp, i64, u64, u64, vp, vp,
                                       vp, vp, vp, vp, vp, vp, sz, vp]
        L.vmc_batched_workspace_size.restype = ctypes.c_int
        L.vmc_batched_workspace_size.argtypes = [ctypes.c_int32, P(Model), P(ctypes.c_int32), P(Ham), i64, P(sz)]
        L.vmc_step_noalloc.restype = ctypes.c_int
        L.vmc_step_noalloc.argtypes = [P(Model), vp, P(Ham), i64, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.vmc_noalloc_scratch_bytes.restype = sz
        L.vmc_noalloc_scratch_bytes.argtypes = []
        L.vmc_adam.restype = ctypes.c_int
        L.vmc_adam.argtypes = [i64, vp, vp, vp, vp, vp, P(AdamCfg), vp]
        L.vmc_check_finite.restype = ctypes.c_int
        L.vmc_check_finite.argtypes = [vp, i64, P(i64), vp, sz, vp]
        L.grow_hidden.restype = ctypes.c_int
        L.grow_hidden.argtypes = [P(Model), vp, ctypes.c_int32, u64, d, vp, vp, vp, vp, vp, vp]
        L.vmc_row_tile_options.restype = ctypes.c_int
        L.vmc_row_tile_options.argtypes = [P(Model), P(ctypes.c_int32), P(ctypes.c_int32)]
        L.vmc_set_tuning.restype = ctypes.c_int
        L.vmc_set_tuning.argtypes = [P(Model), P(Tuning)]
        L.vmc_get_tuning.restype = ctypes.c_int
        L.vmc_get_tuning.argtypes = [P(Model), P(Tuning)]
        L.vmc_autotune_step.restype = ctypes.c_int
        L.vmc_autotune_step.argtypes = [P(Model), vp, P(Ham), i64, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp,
                                        ctypes.c_int32, P(Tuning)]
        L.vmc_chain_timing.restype = ctypes.c_int
        L.vmc_chain_timing.argtypes = [ctypes.c_int]
        L.vmc_chain_time.restype = ctypes.c_int
        L.vmc_chain_time.argtypes = [P(d), P(i64)]
        L.vmc_status_str.restype = ctypes.c_char_p
        L.vmc_status_str.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise VmcError(status, lib().vmc_status_str(status).decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, shape=None):
    """Checks a device argument before any launch: the C ABI cannot check
    lengths, so a short or mis-typed buffer would be read or written past
    its end on the GPU."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError("%s must be a contiguous %s tensor on the GPU" % (name, dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


def _params(m, params):
    return _dev(params, torch.float32, "params", (param_count(m),))


def _configs(m, configs):
    _dev(configs, torch.uint8, "configs")
    if configs.dim() != 2 or configs.shape[1] != m.N or configs.shape[0] < 1:
        raise ValueError("configs must have shape [n, N=%d] with n >= 1, got %s" % (m.N, tuple(configs.shape)))
    return configs.shape[0]


def _step_out(m, ns, out):
    """Checks a caller-supplied (configs, logp, phase, eloc, grad, stats) tuple."""
    cfg, lp, ph, e, g, st = out
    _dev(cfg, torch.uint8, "configs", (ns, m.N))
    _dev(lp, torch.float32, "logp", (ns,))
    if ph is not None:
        _dev(ph, torch.float32, "phase", (ns,))
    _dev(e, torch.float64, "eloc", (ns, 2))
    _dev(g, torch.float64, "grad", (param_count(m),))
    _dev(st, torch.float64, "stats", (4,))
    return out


def param_count(m):
    n = lib().vmc_param_count(ctypes.byref(m))
    if n < 0:
        raise VmcError(-1, "invalid model descriptor")
    return n


def workspace_size(m, H, ns):
    out = ctypes.c_size_t(0)
    _check(lib().vmc_workspace_size(ctypes.byref(m), None if H is None else ctypes.byref(H), ns,
                                    ctypes.byref(out)))
    return out.value


class Workspace:
    """Caller-owned device scratch passed to every call (grows on demand)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _ws(ws, m, H, ns):
    need = workspace_size(m, H, ns)
    if ws is None:
        dev = torch.cuda.current_device()
        ws = _default_ws.setdefault(dev, Workspace("cuda:%d" % dev))
    buf = ws.get(need)
    return buf, buf.numel()


def rnn_sample(m, params, ns, seed=0, counter=0, uniforms=None, ws=None, out=None):
    """Autoregressive sampling; returns (configs uint8 [ns,N], logp [ns], phase [ns])."""
    _params(m, params)
    dev = params.device
    if uniforms is not None:
        _dev(uniforms, torch.float32, "uniforms", (ns, m.N))
    if out is None:
        out = (torch.empty((ns, m.N), dtype=torch.uint8, device=dev),
               torch.empty(ns, dtype=torch.float32, device=dev),
               torch.empty(ns, dtype=torch.float32, device=dev))
    cfg, lp, ph = out
    _dev(cfg, torch.uint8, "configs", (ns, m.N))
    _dev(lp, torch.float32, "logp", (ns,))
    if ph is not None:
        _dev(ph, torch.float32, "phase", (ns,))
    buf, nb = _ws(ws, m, None, ns)
    _check(lib().rnn_sample(ctypes.byref(m), _ptr(params), ns, seed, counter, _ptr(uniforms), _ptr(cfg),
                            _ptr(lp), _ptr(ph), _ptr(buf), nb, _stream()))
    return cfg, lp, ph


def rnn_logpsi(m, params, configs, ws=None):
    """Teacher-forced (logp [nc], phase [nc]) of given configurations."""
    _params(m, params)
    nc = _configs(m, configs)
    lp = torch.empty(nc, dtype=torch.float32, device=params.device)
    ph = torch.empty(nc, dtype=torch.float32, device=params.device)
    buf, nb = _ws(ws, m, None, nc)
    _check(lib().rnn_logpsi(ctypes.byref(m), _ptr(params), nc, _ptr(configs), _ptr(lp), _ptr(ph), _ptr(buf),
                            nb, _stream()))
    return lp, ph


def rnn_logpsi_grad(m, params, configs, dlogp, dphase=None, ws=None, out=None):
    """Vector-Jacobian product of rnn_logpsi: sum_s dlogp_s d logP_s + dphase_s d phi_s,
    float64 [P]."""
    _params(m, params)
    nc = _configs(m, configs)
    _dev(dlogp, torch.float32, "dlogp", (nc,))
    if dphase is not None:
        _dev(dphase, torch.float32, "dphase", (nc,))
    g = out if out is not None else torch.empty(param_count(m), dtype=torch.float64, device=params.device)
    _dev(g, torch.float64, "grad", (param_count(m),))
    buf, nb = _ws(ws, m, None, nc)
    _check(lib().rnn_logpsi_grad(ctypes.byref(m), _ptr(params), nc, _ptr(configs), _ptr(dlogp), _ptr(dphase),
                                 _ptr(g), _ptr(buf), nb, _stream()))
    return g


class LogPsi(torch.autograd.Function):
    """(log P, phi) of given configurations as a differentiable function of the
    flat parameters: forward rnn_logpsi, backward rnn_logpsi_grad (the
    hand-written reverse sweep)."""

    @staticmethod
    def forward(ctx, params, configs, m):
        lp, ph = rnn_logpsi(m, params, configs)
        ctx.save_for_backward(params, configs)
        ctx.m = m
        return lp, ph

    @staticmethod
    def backward(ctx, glp, gph):
        params, configs = ctx.saved_tensors
        if glp is None:
            glp = torch.zeros(configs.shape[0], dtype=torch.float32, device=params.device)
        gph = None if (gph is None or not ctx.m.is_complex) else gph.float().contiguous()
        g = rnn_logpsi_grad(ctx.m, params, configs, glp.float().contiguous(), gph)
        return g.to(params.dtype), None, None


def logpsi(m, params, configs):
    """Differentiable (log P [nc], phase [nc]); see LogPsi."""
    return LogPsi.apply(params, configs, m)


def local_energy(m, params, H, configs, ws=None, out=None):
    """Local energies [ns, 2] float64 (real, imaginary)."""
    _params(m, params)
    ns = _configs(m, configs)
    e = out if out is not None else torch.empty((ns, 2), dtype=torch.float64, device=params.device)
    _dev(e, torch.float64, "eloc", (ns, 2))
    buf, nb = _ws(ws, m, H, ns)
    _check(lib().local_energy(ctypes.byref(m), _ptr(params), ctypes.byref(H), ns, _ptr(configs), _ptr(e),
                              _ptr(buf), nb, _stream()))
    return e


def vmc_grad(m, params, configs, eloc, weights=None, ws=None, out=None):
    """Covariance energy gradient; returns (grad float64 [P], stats float64 [4])."""
    _params(m, params)
    ns = _configs(m, configs)
    _dev(eloc, torch.float64, "eloc", (ns, 2))
    if weights is not None:
        _dev(weights, torch.float64, "weights", (ns,))
    if out is None:
        out = (torch.empty(param_count(m), dtype=torch.float64, device=params.device),
               torch.empty(4, dtype=torch.float64, device=params.device))
    g, st = out
    _dev(g, torch.float64, "grad", (param_count(m),))
    _dev(st, torch.float64, "stats", (4,))
    buf, nb = _ws(ws, m, None, ns)
    _check(lib().vmc_grad(ctypes.byref(m), _ptr(params), ns, _ptr(configs), _ptr(eloc), _ptr(weights), _ptr(g),
                          _ptr(st), _ptr(buf), nb, _stream()))
    return g, st


def energy_stats(eloc, weights=None, out=None):
    """Re Ebar, Im Ebar, var and the non-finite count of a set of local
    energies, as vmc_grad forms them; returns stats float64 [4]."""
    if not (isinstance(eloc, torch.Tensor) and eloc.dim() == 2 and eloc.shape[1] == 2):
        raise ValueError("eloc must be a [ns, 2] tensor")
    ns = eloc.shape[0]
    if ns < 1:
        raise ValueError("eloc holds no sample")
    _dev(eloc, torch.float64, "eloc", (ns, 2))
    if weights is not None:
        _dev(weights, torch.float64, "weights", (ns,))
    st = out if out is not None else torch.empty(4, dtype=torch.float64, device=eloc.device)
    _dev(st, torch.float64, "stats", (4,))
    _check(lib().vmc_energy_stats(ns, _ptr(eloc), _ptr(weights), _ptr(st), _stream()))
    return st


def vmc_grad_chunked(m, params, configs, eloc, weights, chunk, out=None):
    """vmc_grad of a sample set in chunks of at most `chunk` samples, each in
    a workspace sized for one chunk: the set's statistics first, then every
    chunk's contribution added to the gradient by the library.  weights
    float64 [ns] (1/ns for an unweighted set) is required.  Returns
    (grad float64 [P], stats float64 [4])."""
    _params(m, params)
    ns = _configs(m, configs)
    _dev(eloc, torch.float64, "eloc", (ns, 2))
    _dev(weights, torch.float64, "weights", (ns,))
    if not isinstance(chunk, int) or chunk < 1:
        raise ValueError("chunk must be a positive int")
    if out is None:
        out = (torch.empty(param_count(m), dtype=torch.float64, device=params.device),
               torch.empty(4, dtype=torch.float64, device=params.device))
    g, st = out
    _dev(g, torch.float64, "grad", (param_count(m),))
    energy_stats(eloc, weights, out=st)
    g.zero_()
    buf, nb = _ws(None, m, None, min(chunk, ns))
    for s0 in range(0, ns, chunk):
        n = min(chunk, ns - s0)
        _check(lib().vmc_grad_chunk(ctypes.byref(m), _ptr(params), n, _ptr(configs[s0:s0 + n]),
                                    _ptr(eloc[s0:s0 + n]), _ptr(weights[s0:s0 + n]), _ptr(st), _ptr(g),
                                    _ptr(buf), nb, _stream()))
    return g, st


def vmc_step(m, params, H, ns, seed=0, counter=0, uniforms=None, ws=None, out=None, counter_dev=None):
    """One VMC step (sample, local energy, gradient with w = 1/ns) sharing one
    forward pass; returns (configs, logp, phase, eloc, grad, stats).
    counter_dev: optional one-element uint64 (int64) device tensor that
    replaces `counter` and is advanced by one at the end of the step, so that
    replays of a captured graph draw fresh samples."""
    _params(m, params)
    dev = params.device
    if uniforms is not None:
        _dev(uniforms, torch.float32, "uniforms", (ns, m.N))
    if counter_dev is not None and not (isinstance(counter_dev, torch.Tensor) and counter_dev.is_cuda and
                                        counter_dev.dtype in (torch.int64, torch.uint64) and
                                        counter_dev.numel() == 1):
        raise TypeError("counter_dev must be a one-element int64/uint64 tensor on the GPU")
    if out is None:
        out = (torch.empty((ns, m.N), dtype=torch.uint8, device=dev),
               torch.empty(ns, dtype=torch.float32, device=dev),
               torch.empty(ns, dtype=torch.float32, device=dev),
               torch.empty((ns, 2), dtype=torch.float64, device=dev),
               torch.empty(param_count(m), dtype=torch.float64, device=dev),
               torch.empty(4, dtype=torch.float64, device=dev))
    cfg, lp, ph, e, g, st = _step_out(m, ns, out)
    buf, nb = _ws(ws, m, H, ns)
    _check(lib().vmc_step(ctypes.byref(m), _ptr(params), ctypes.byref(H), ns, seed, counter, _ptr(counter_dev),
                          _ptr(uniforms), _ptr(cfg), _ptr(lp), _ptr(ph), _ptr(e), _ptr(g), _ptr(st), _ptr(buf), nb,
                          _stream()))
    return cfg, lp, ph, e, g, st


def _batch_args(m, chain_lens, hams):
    n = len(chain_lens)
    if n < 1 or len(hams) != n:
        raise ValueError("one Hamiltonian per chain")
    lens = (ctypes.c_int32 * n)(*[int(c) for c in chain_lens])
    hs = (Ham * n)(*hams)
    return n, lens, hs


def batched_workspace_size(m, chain_lens, hams, ns):
    n, lens, hs = _batch_args(m, chain_lens, hams)
    out = ctypes.c_size_t(0)
    _check(lib().vmc_batched_workspace_size(n, ctypes.byref(m), lens, hs, ns, ctypes.byref(out)))
    return out.value


def vmc_step_batched(m, chain_lens, hams, params, ns, seed=0, counter=0, ws=None, out=None, counter_dev=None):
    """One VMC step of several 1D problems (own chain lengths, couplings and
    weights, the cell shape of m) in shared launches.  params: [nprob, P]
    float32.  Returns (configs [nprob, ns * Nmax] uint8, logp [nprob, ns],
    phase [nprob, ns], eloc [nprob, ns, 2], grad [nprob, P], stats
    [nprob, 4]); batch_configs() gives problem k's [ns, N_k] view.  Problem k
    equals vmc_step on it alone with seed + k."""
    n, lens, hs = _batch_args(m, chain_lens, hams)
    P = param_count(m)
    _dev(params, torch.float32, "params", (n, P))
    nmax = max(int(c) for c in chain_lens)
    dev = params.device
    if out is None:
        out = (torch.empty((n, ns * nmax), dtype=torch.uint8, device=dev),
               torch.empty((n, ns), dtype=torch.float32, device=dev),
               torch.empty((n, ns), dtype=torch.float32, device=dev),
               torch.empty((n, ns, 2), dtype=torch.float64, device=dev),
               torch.empty((n, P), dtype=torch.float64, device=dev),
               torch.empty((n, 4), dtype=torch.float64, device=dev))
    cfg, lp, ph, e, g, st = out
    _dev(cfg, torch.uint8, "configs", (n, ns * nmax))
    _dev(lp, torch.float32, "logp", (n, ns))
    if ph is not None:
        _dev(ph, torch.float32, "phase", (n, ns))
    _dev(e, torch.float64, "eloc", (n, ns, 2))
    _dev(g, torch.float64, "grad", (n, P))
    _dev(st, torch.float64, "stats", (n, 4))
    if counter_dev is not None:
        _dev(counter_dev, torch.int64, "counter_dev", (1,))
    need = batched_workspace_size(m, chain_lens, hams, ns)
    if ws is None:
        d = torch.cuda.current_device()
        ws = _default_ws.setdefault(d, Workspace("cuda:%d" % d))
    buf = ws.get(need)
    _check(lib().vmc_step_batched(n, ctypes.byref(m), lens, hs, _ptr(params), ns, seed, counter, _ptr(counter_dev),
                                  _ptr(cfg), _ptr(lp), _ptr(ph), _ptr(e), _ptr(g), _ptr(st), _ptr(buf), buf.numel(),
                                  _stream()))
    return out


def batch_configs(configs, k, ns, n_k):
    """Problem k's configurations [ns, n_k] inside the batched configs array."""
    return configs[k, :ns * n_k].view(ns, n_k)


def vmc_step_noalloc(m, params, H, ns, out, seed=0, counter=0, uniforms=None, counter_dev=None):
    """vmc_step with the library's fixed device workspace (no allocation in
    the library); `out` = (configs, logp, phase, eloc, grad, stats) must be
    given.  Calls on one GPU share that workspace and must not overlap."""
    _params(m, params)
    if uniforms is not None:
        _dev(uniforms, torch.float32, "uniforms", (ns, m.N))
    if counter_dev is not None:
        _dev(counter_dev, torch.int64, "counter_dev", (1,))
    cfg, lp, ph, e, g, st = _step_out(m, ns, out)
    _check(lib().vmc_step_noalloc(ctypes.byref(m), _ptr(params), ctypes.byref(H), ns, seed, counter,
                                  _ptr(counter_dev), _ptr(uniforms), _ptr(cfg), _ptr(lp), _ptr(ph), _ptr(e), _ptr(g),
                                  _ptr(st), _stream()))
    return out


def noalloc_scratch_bytes():
    return lib().vmc_noalloc_scratch_bytes()


def adam(params, grad, m_mom, v_mom, t_dev, cfg):
    """Adam update of the float32 parameters (in place) from a float64
    gradient; m_mom, v_mom float32 moments; t_dev a one-element int64 device
    tensor of updates done (advanced by the call)."""
    n = params.numel()
    _dev(params, torch.float32, "params")
    _dev(grad, torch.float64, "grad", (n,))
    _dev(m_mom, torch.float32, "m", (n,))
    _dev(v_mom, torch.float32, "v", (n,))
    _dev(t_dev, torch.int64, "t_dev", (1,))
    _check(lib().vmc_adam(n, _ptr(params), _ptr(grad), _ptr(m_mom), _ptr(v_mom), _ptr(t_dev), ctypes.byref(cfg),
                          _stream()))


def check_finite(x, ws=None):
    """Number of non-finite entries of a float32 device tensor (synchronous);
    raises VmcError(VMC_ENONFINITE) if there are any."""
    _dev(x, torch.float32, "x")
    if ws is None:
        dev = torch.cuda.current_device()
        ws = _default_ws.setdefault(dev, Workspace("cuda:%d" % dev))
    buf = ws.get(256)
    cnt = ctypes.c_int64(0)
    _check(lib().vmc_check_finite(_ptr(x), x.numel(), ctypes.byref(cnt), _ptr(buf), buf.numel(), _stream()))
    return cnt.value


def grow_hidden(m, params, new_dh, seed, noise_std, m_mom=None, v_mom=None):
    """Grown parameters (and moments if given) at hidden width new_dh."""
    _params(m, params)
    to = Model(m.dims, m.Lx, m.Ly, new_dh, m.is_complex, m.glu, m.precision)
    n1 = param_count(to)
    p1 = torch.empty(n1, dtype=torch.float32, device=params.device)
    mm = vv = None
    if m_mom is not None or v_mom is not None:
        _dev(m_mom, torch.float32, "m", (params.numel(),))
        _dev(v_mom, torch.float32, "v", (params.numel(),))
        mm = torch.empty_like(p1)
        vv = torch.empty_like(p1)
    _check(lib().grow_hidden(ctypes.byref(m), _ptr(params), new_dh, seed, float(noise_std), _ptr(p1),
                             _ptr(m_mom), _ptr(v_mom), _ptr(mm), _ptr(vv), _stream()))
    if mm is not None:
        return p1, mm, vv, to
    return p1, to


def row_tile_options(m):
    """Row-tile heights the model shape can run with (built-in first)."""
    opts = (ctypes.c_int32 * 2)()
    n = ctypes.c_int32(0)
    _check(lib().vmc_row_tile_options(ctypes.byref(m), opts, ctypes.byref(n)))
    return [opts[i] for i in range(n.value)]


def set_tuning(m, row_tile=0, chain_wgs_per_cu=0):
    """Set the launch choices of this model shape (0 = built-in); reset_tuning restores all."""
    _check(lib().vmc_set_tuning(ctypes.byref(m), ctypes.byref(Tuning(int(row_tile), int(chain_wgs_per_cu)))))


def reset_tuning(m):
    _check(lib().vmc_set_tuning(ctypes.byref(m), None))


def get_tuning(m):
    """The launch choices in effect for this model shape, as a dict."""
    t = Tuning()
    _check(lib().vmc_get_tuning(ctypes.byref(m), ctypes.byref(t)))
    return {"row_tile": t.row_tile, "chain_wgs_per_cu": t.chain_wgs_per_cu}


def autotune_step(m, params, H, ns, seed=0, counter=0, uniforms=None, ws=None, out=None, reps=3):
    """Autotuner: times vmc_step under each candidate launch choice, keeps the
    fastest in the library's table and returns (outputs of vmc_step, choice)."""
    _params(m, params)
    dev = params.device
    if uniforms is not None:
        _dev(uniforms, torch.float32, "uniforms", (ns, m.N))
    if out is None:
        out = (torch.empty((ns, m.N), dtype=torch.uint8, device=dev),
               torch.empty(ns, dtype=torch.float32, device=dev),
               torch.empty(ns, dtype=torch.float32, device=dev),
               torch.empty((ns, 2), dtype=torch.float64, device=dev),
               torch.empty(param_count(m), dtype=torch.float64, device=dev),
               torch.empty(4, dtype=torch.float64, device=dev))
    cfg, lp, ph, e, g, st = _step_out(m, ns, out)
    buf, nb = _ws(ws, m, H, ns)
    t = Tuning()
    _check(lib().vmc_autotune_step(ctypes.byref(m), _ptr(params), ctypes.byref(H), ns, seed, counter,
                                   _ptr(uniforms), _ptr(cfg), _ptr(lp), _ptr(ph), _ptr(e), _ptr(g), _ptr(st),
                                   _ptr(buf), nb, _stream(), int(reps), ctypes.byref(t)))
    return out, {"row_tile": t.row_tile, "chain_wgs_per_cu": t.chain_wgs_per_cu}


def _shape_key(m):
    return "d%d_%dx%d_h%d_p%d_g%d_c%d" % (m.dims, m.Lx, m.Ly, m.d_h, m.precision, m.glu, m.is_complex)


def save_tuning(path, models):
    """Write the tuning in effect for each model shape to a JSON cache file."""
    import json
    data = {_shape_key(m): get_tuning(m) for m in models}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load_tuning(path, models):
    """Apply the cached tuning of every listed model shape found in the file;
    returns the number applied."""
    import json
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for m in models:
        t = data.get(_shape_key(m))
        if t is not None:
            set_tuning(m, t["row_tile"], t["chain_wgs_per_cu"])
            n += 1
    return n


def chain_timing(enable):
    """Start (and reset) or stop event timing of the suffix-chain launch."""
    _check(lib().vmc_chain_timing(int(bool(enable))))


def chain_time():
    """(total milliseconds, number of timed launches) of the suffix-chain kernel."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().vmc_chain_time(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


class StepBatch:
    """One VMC step of several independent problems (uneven chains, other
    couplings) replayed as one HIP graph.  Each problem is a dict with keys
    model, params, ham, ns and optionally seed, counter; each gets its own
    workspace and outputs (`outputs[i]` = (configs, logp, phase, eloc, grad,
    stats) of problem i).  The problems are spread over `streams` side
    streams, longest first (work ~ ns * N^2) onto the least loaded stream,
    so that their launches overlap on the GPU; capture() records everything
    once, replay() runs the whole batch."""

    def __init__(self, problems, streams=4):
        self.problems = problems
        self.outputs = []
        self.workspaces = []
        for pb in problems:
            m, ns, dev = pb["model"], pb["ns"], pb["params"].device
            ws = Workspace(dev)
            ws.get(workspace_size(m, pb["ham"], ns))
            self.workspaces.append(ws)
            self.outputs.append((torch.empty((ns, m.N), dtype=torch.uint8, device=dev),
                                 torch.empty(ns, dtype=torch.float32, device=dev),
                                 torch.empty(ns, dtype=torch.float32, device=dev),
                                 torch.empty((ns, 2), dtype=torch.float64, device=dev),
                                 torch.empty(param_count(m), dtype=torch.float64, device=dev),
                                 torch.empty(4, dtype=torch.float64, device=dev)))
        nstream = max(1, min(streams, len(problems)))
        self.streams = [torch.cuda.Stream() for _ in range(nstream)]
        load = [0.0] * nstream
        self.assign = [[] for _ in range(nstream)]
        order = sorted(range(len(problems)), key=lambda i: -problems[i]["ns"] * problems[i]["model"].N ** 2)
        for i in order:
            k = min(range(nstream), key=lambda j: load[j])
            self.assign[k].append(i)
            load[k] += problems[i]["ns"] * problems[i]["model"].N ** 2
        self.graph = None

    def _issue(self):
        main = torch.cuda.current_stream()
        for s, idx in zip(self.streams, self.assign):
            s.wait_stream(main)
            with torch.cuda.stream(s):
                for i in idx:
                    pb = self.problems[i]
                    vmc_step(pb["model"], pb["params"], pb["ham"], pb["ns"], seed=pb.get("seed", 0),
                             counter=pb.get("counter", 0), ws=self.workspaces[i], out=self.outputs[i])
        for s in self.streams:
            main.wait_stream(s)

    def autotune(self, reps=2):
        """Run the autotuner once per distinct model shape of the batch (on its
        largest problem, alone on the current stream) before capture; returns
        {shape: tuning}.  The tuning lives in the library's table, so the
        captured launches use it."""
        pick = {}
        for i, pb in enumerate(self.problems):
            k = _shape_key(pb["model"])
            if k not in pick or pb["ns"] > self.problems[pick[k]]["ns"]:
                pick[k] = i
        self.tuning = {}
        for k, i in sorted(pick.items()):
            pb = self.problems[i]
            _, self.tuning[k] = autotune_step(pb["model"], pb["params"], pb["ham"], pb["ns"], seed=pb.get("seed", 0),
                                              counter=pb.get("counter", 0), ws=self.workspaces[i],
                                              out=self.outputs[i], reps=reps)
        return self.tuning

    def run_eager(self):
        self._issue()

    def capture(self):
        self._issue()  # warm-up outside the graph (launch attributes, library load)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._issue()
        return self

    def replay(self):
        self.graph.replay()
