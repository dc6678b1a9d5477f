"""Seeded synthetic inputs: parameters, uniforms and configurations.

This module only draws numbers; it holds none of the method's arithmetic.  It
serves the tests, the bench and users who want initial weights for a VMC run.

Parameter blocks follow the flat layout of the library (row-major [out][in]):
  1D GRU (App. A of the paper): W_g [dh, dh+2], b_g, W_r [dh, dh+2], b_r,
                                W_h [dh, dh], b_h, W_in [dh, 2], b_in
  2D GRU (App. A):              W [dh, 2dh+4], b, W_g [dh, 2dh+4], b_g, U [dh, 2dh]
  GLU (App. A, optional):       W_1 [dh, dh], b_1, W_2 [dh, dh], b_2
  amplitude head (Eq. (3)):     U_a [2, dh], c_a [2]
  phase head (Eq. (5), cRNN):   U_p [2, dh], c_p [2]
The paper does not state its initialisation; Xavier-uniform weights with bound
sqrt(6 / (fan_in + fan_out)) and zero biases are used unless a bias scale is
given (tests draw nonzero biases so that every term is exercised).
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class ModelSpec:
    dims: int = 1
    Lx: int = 4
    Ly: int = 1
    d_h: int = 4
    is_complex: bool = False
    glu: bool = False

    @property
    def N(self):
        return self.Lx * (self.Ly if self.dims == 2 else 1)


def blocks(spec):
    """[(name, shape)] of the flat parameter vector, in layout order."""
    d = spec.d_h
    out = []
    if spec.dims == 1:
        out += [("W_g", (d, d + 2)), ("b_g", (d,)), ("W_r", (d, d + 2)), ("b_r", (d,)),
                ("W_h", (d, d)), ("b_h", (d,)), ("W_in", (d, 2)), ("b_in", (d,))]
    else:
        out += [("W", (d, 2 * d + 4)), ("b", (d,)), ("W_g", (d, 2 * d + 4)), ("b_g", (d,)),
                ("U", (d, 2 * d))]
    if spec.glu:
        out += [("W_1", (d, d)), ("b_1", (d,)), ("W_2", (d, d)), ("b_2", (d,))]
    out += [("U_a", (2, d)), ("c_a", (2,))]
    if spec.is_complex:
        out += [("U_p", (2, d)), ("c_p", (2,))]
    return out


def param_count(spec):
    return int(sum(int(np.prod(s)) for _, s in blocks(spec)))


def split(spec, flat):
    """Views of the flat vector by block name."""
    res, o = {}, 0
    for name, shape in blocks(spec):
        n = int(np.prod(shape))
        res[name] = flat[o:o + n].reshape(shape)
        o += n
    return res


def xavier_params(spec, seed, bias_scale=0.0, gain=1.0, dtype=np.float32):
    """Xavier-uniform weights (numpy PCG64 stream `seed`), biases uniform in
    [-bias_scale, bias_scale] (zero by default)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shape in blocks(spec):
        if len(shape) == 2:
            bound = gain * np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            if bias_scale > 0:
                parts.append(rng.uniform(-bias_scale, bias_scale, size=shape))
            else:
                parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(dtype)


def uniforms(ns, N, seed, dtype=np.float32):
    """Sampling uniforms in [0,1), [ns, N], indexed by sample and order position.
    Multiples of 2^-24, so that float32 and float64 hold the same values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.integers(0, 1 << 24, size=(ns, N), dtype=np.int64).astype(np.float64) / float(1 << 24)
    return u.astype(dtype)


def configs(ns, N, seed, p_one=0.5):
    """Random spin configurations in {0,1}, [ns, N] uint8 (lattice order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((ns, N)) < p_one).astype(np.uint8)


def neel_like_configs(ns, Lx, Ly, seed, anti_fraction):
    """Configurations on an Lx x Ly open lattice whose nearest-neighbour bonds
    are anti-aligned with probability close to `anti_fraction`: a Neel state
    with each spin flipped independently with probability q, where
    1 - 2q(1-q) = anti_fraction (bond-independent approximation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = 0.5 * (1.0 - np.sqrt(max(0.0, 2.0 * anti_fraction - 1.0)))
    ii, jj = np.meshgrid(np.arange(Lx), np.arange(Ly))
    neel = ((ii + jj) % 2).astype(np.uint8).ravel()
    flips = (rng.random((ns, Lx * Ly)) < q).astype(np.uint8)
    return (neel[None, :] ^ flips).astype(np.uint8)


def eloc_values(ns, seed, complex_=False, scale=1.0):
    """Synthetic local energies [ns, 2] (re, im) for gradient tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = np.zeros((ns, 2))
    e[:, 0] = scale * rng.standard_normal(ns)
    if complex_:
        e[:, 1] = scale * rng.standard_normal(ns)
    return e


def uneven_chains(count, seed, n_lo=32, n_hi=128, h_lo=0.5, h_hi=1.5):
    """A batch of independent 1D TFIM problems of uneven length: chain lengths
    uniform in {n_lo..n_hi} and transverse fields uniform in [h_lo, h_hi]
    (numpy PCG64 stream `seed`); returns [(N_c, h_c)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    hs = rng.uniform(h_lo, h_hi, size=count)
    return [(int(n), float(h)) for n, h in zip(ns, hs)]
