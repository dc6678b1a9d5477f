"""ctypes front end of the FP64 CPU oracle (``oracle.c``).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the bench may import this module; the product path never does.  All arrays
are host numpy arrays (float64 parameters, uint8 configurations in lattice
order).  The functions follow the paper section by section; see ``oracle.c``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile liboracle.so with gcc (OpenMP over samples, no BLAS)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class Model(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("d_h", ctypes.c_int32), ("is_complex", ctypes.c_int32),
                ("glu", ctypes.c_int32), ("bf16", ctypes.c_int32)]


class Ham(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("marshall", ctypes.c_int32),
                ("J", ctypes.c_double), ("h", ctypes.c_double), ("alpha", ctypes.c_double)]


TFIM, HEISENBERG, LRTFIM, CLUSTER = 0, 1, 2, 3

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, u8, i64 = ctypes.c_double, ctypes.c_uint8, ctypes.c_int64
        L.ora_param_count.restype = i64
        L.ora_param_count.argtypes = [P(Model)]
        L.ora_logpsi.argtypes = [P(Model), P(d), i64, P(u8), P(d), P(d), P(d), P(d)]
        L.ora_sample.argtypes = [P(Model), P(d), i64, P(d), P(u8), P(d), P(d)]
        L.ora_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.ora_philox_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i64, ctypes.c_int32, P(d)]
        L.ora_local_energy.argtypes = [P(Model), P(d), P(Ham), i64, P(u8), P(d)]
        L.ora_bond_count.restype = ctypes.c_int32
        L.ora_bond_count.argtypes = [P(Model)]
        L.ora_stats.argtypes = [i64, P(d), P(d), P(d)]
        L.ora_surrogate_grad.argtypes = [P(Model), P(d), i64, P(u8), P(d), P(d), P(d)]
        L.ora_grad.argtypes = [P(Model), P(d), i64, P(u8), P(d), P(d), P(d), P(d)]
        L.ora_grow_hidden.argtypes = [P(Model), P(d), ctypes.c_int32, ctypes.c_uint64, d,
                                      P(d), P(d), P(d), P(d), P(d)]
        L.ora_num_threads.restype = ctypes.c_int32
        L.ora_round_bf16.restype = d
        L.ora_round_bf16.argtypes = [d]
        L.ora_adam.argtypes = [i64, P(d), P(d), P(d), P(d), i64, d, d, d, d]
        L.ora_surrogate_grad_abs.argtypes = [P(Model), P(d), i64, P(u8), P(d), P(d), P(d), P(d)]
        L.ora_set_threads.argtypes = [ctypes.c_int32]
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def model(dims=1, Lx=4, Ly=1, d_h=4, is_complex=False, glu=False, bf16=False):
    return Model(dims, Lx, Ly if dims == 2 else 1, d_h, int(is_complex), int(glu), int(bf16))


def ham(kind=TFIM, J=1.0, h=1.0, marshall=False, alpha=0.0):
    return Ham(kind, int(marshall), J, h, alpha)


def n_sites(m):
    return m.Lx * m.Ly


def param_count(m):
    return lib().ora_param_count(ctypes.byref(m))


def logpsi(m, params, configs, conditionals=False):
    """log P and phi of each configuration; optionally the per-position
    log-conditionals and phase conditionals, both [nc, N, 2]."""
    params, configs = _f64(params), _u8(configs)
    nc = configs.shape[0]
    N = n_sites(m)
    lp = np.zeros(nc)
    ph = np.zeros(nc)
    lpc = np.zeros((nc, N, 2)) if conditionals else None
    phc = np.zeros((nc, N, 2)) if conditionals else None
    lib().ora_logpsi(ctypes.byref(m), _p(params), nc, _p(configs, ctypes.c_uint8), _p(lp), _p(ph),
                     _p(lpc), _p(phc))
    if conditionals:
        return lp, ph, lpc, phc
    return lp, ph


def sample(m, params, uniforms):
    params, uniforms = _f64(params), _f64(uniforms)
    ns = uniforms.shape[0]
    N = n_sites(m)
    cfg = np.zeros((ns, N), np.uint8)
    lp = np.zeros(ns)
    ph = np.zeros(ns)
    lib().ora_sample(ctypes.byref(m), _p(params), ns, _p(uniforms), _p(cfg, ctypes.c_uint8),
                     _p(lp), _p(ph))
    return cfg, lp, ph


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


def philox_uniforms(seed, counter, ns, N):
    u = np.zeros((ns, N))
    lib().ora_philox_uniforms(seed, counter, ns, N, _p(u))
    return u


def local_energy(m, params, h, configs):
    params, configs = _f64(params), _u8(configs)
    ns = configs.shape[0]
    e = np.zeros((ns, 2))
    lib().ora_local_energy(ctypes.byref(m), _p(params), ctypes.byref(h), ns,
                           _p(configs, ctypes.c_uint8), _p(e))
    return e[:, 0] + 1j * e[:, 1]


def bond_count(m):
    return lib().ora_bond_count(ctypes.byref(m))


def _eloc_arr(eloc):
    eloc = np.asarray(eloc)
    if np.iscomplexobj(eloc) or eloc.ndim == 1:
        return _f64(np.stack([eloc.real, np.imag(eloc)], axis=1))
    return _f64(eloc)


def stats(eloc, weights=None):
    e = _eloc_arr(eloc)
    w = None if weights is None else _f64(weights)
    st = np.zeros(4)
    lib().ora_stats(e.shape[0], _p(e), _p(w), _p(st))
    return st


def surrogate_grad(m, params, configs, a, b=None):
    params, configs = _f64(params), _u8(configs)
    g = np.zeros(param_count(m))
    lib().ora_surrogate_grad(ctypes.byref(m), _p(params), configs.shape[0],
                             _p(configs, ctypes.c_uint8), _p(_f64(a)),
                             _p(None if b is None else _f64(b)), _p(g))
    return g


def surrogate_grad_abs(m, params, configs, a, b=None):
    """(gradient, per-entry sum over samples of |per-sample contribution|)."""
    params, configs = _f64(params), _u8(configs)
    g = np.zeros(param_count(m))
    ga = np.zeros(param_count(m))
    lib().ora_surrogate_grad_abs(ctypes.byref(m), _p(params), configs.shape[0], _p(configs, ctypes.c_uint8),
                                 _p(_f64(a)), _p(None if b is None else _f64(b)), _p(g), _p(ga))
    return g, ga


def set_threads(n):
    lib().ora_set_threads(int(n))


def grad(m, params, configs, eloc, weights=None):
    params, configs = _f64(params), _u8(configs)
    e = _eloc_arr(eloc)
    w = None if weights is None else _f64(weights)
    g = np.zeros(param_count(m))
    st = np.zeros(4)
    lib().ora_grad(ctypes.byref(m), _p(params), configs.shape[0], _p(configs, ctypes.c_uint8),
                   _p(e), _p(w), _p(g), _p(st))
    return g, st


def grow_hidden(m, params, new_dh, seed, noise_std, m_mom=None, v_mom=None):
    params = _f64(params)
    to = Model(m.dims, m.Lx, m.Ly, new_dh, m.is_complex, m.glu, m.bf16)
    n1 = param_count(to)
    p1 = np.zeros(n1)
    m1 = np.zeros(n1) if m_mom is not None else None
    v1 = np.zeros(n1) if v_mom is not None else None
    lib().ora_grow_hidden(ctypes.byref(m), _p(params), new_dh, seed, noise_std, _p(p1),
                          _p(None if m_mom is None else _f64(m_mom)),
                          _p(None if v_mom is None else _f64(v_mom)), _p(m1), _p(v1))
    if m_mom is not None or v_mom is not None:
        return p1, m1, v1
    return p1


def adam(params, grad, m_mom, v_mom, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 on float64 copies; returns (p, m, v)."""
    p, g, m1, v1 = _f64(params).copy(), _f64(grad), _f64(m_mom).copy(), _f64(v_mom).copy()
    lib().ora_adam(p.size, _p(p), _p(g), _p(m1), _p(v1), int(t), float(lr), float(beta1), float(beta2), float(eps))
    return p, m1, v1


def num_threads():
    return lib().ora_num_threads()


def round_bf16(x):
    return lib().ora_round_bf16(float(x))
