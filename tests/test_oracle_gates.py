"""Pins of the oracle's GRU gate algebra (App. A) by saturated gates.

A gate driven by a bias of +-60 is 0 or 1 to far below double rounding, and
the cell then reduces to a recursion simple enough to write down here: a
Markov chain in the previous spin, a product state, or a plain tanh RNN.
Each pin is chosen so that a plausible slip in the oracle fails it:
  - u and (1 - u) exchanged in the update (1D: h = (1-u) h + u c; 2D:
    h = u c + (1-u) U h'): the open and closed update gates swap their
    closed forms (Markov chain <-> product state);
  - the reset gate applied to h before W_h instead of to (W_h h + b_h):
    with r = 0 the candidate would keep b_h;
  - the GLU halves exchanged (g = (W_1 h + b_1) * sig(W_2 h + b_2)):
    a closed sigmoid half would then scale a large linear half;
  - the one-hot columns or the [h_hz; h_vt] blocks of U taken in the wrong
    order, or a weight matrix transposed: the recursions below index them
    by the documented layout ([out][in]).
CPU only."""
import math

import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests import exact

BIG = 60.0  # sigmoid(+-(60 - 12)) is 1 or 0 to about 1e-21


def _model(ora, spec):
    return ora.model(dims=spec.dims, Lx=spec.Lx, Ly=spec.Ly, d_h=spec.d_h,
                     is_complex=spec.is_complex, glu=spec.glu)


def _params(spec, seed):
    return synth.xavier_params(spec, seed, bias_scale=0.7, gain=1.5, dtype=np.float64)


def _log_softmax(l):
    mx = np.max(l)
    return l - mx - math.log(np.exp(l - mx).sum())


def _chain_logp(cfg, order, cond_logits):
    """log P of each configuration from per-position logit functions:
    cond_logits(c, n) -> the 2 logits at order position n of configuration c."""
    out = np.zeros(len(cfg))
    for s, c in enumerate(cfg):
        for n, site in enumerate(order):
            out[s] += _log_softmax(cond_logits(c, n))[c[site]]
    return out


def _zigzag(Lx, Ly):
    """Per order position: (site, horizontal predecessor site or -1, vertical
    predecessor site or -1); even rows run left to right."""
    res = []
    for n in range(Lx * Ly):
        j, k = divmod(n, Lx)
        i = k if j % 2 == 0 else Lx - 1 - k
        ih = i - 1 if j % 2 == 0 else i + 1
        hz = j * Lx + ih if 0 <= ih < Lx else -1
        vt = (j - 1) * Lx + i if j > 0 else -1
        res.append((j * Lx + i, hz, vt))
    return res


def _onehot(c, site):
    v = np.zeros(2)
    if site >= 0:
        v[c[site]] = 1.0
    return v


# ------------------------------------------------------------------ 1D cell

SPEC1 = synth.ModelSpec(dims=1, Lx=6, d_h=4)


def _check(ora, spec, p, want_fn, atol=1e-12):
    m = _model(ora, spec)
    cfg = exact.all_configs(spec.N)
    lp, _ = ora.logpsi(m, p, cfg)
    want = want_fn(cfg)
    assert np.max(np.abs(lp - want)) < atol
    return lp


def test_1d_update_open_reset_closed_is_markov_chain(ora):
    """u = 1, r = 0: c = tanh(W_in x + b_in) whatever W_h and b_h are, and
    h_n = c_n, so the conditional at n depends on sigma_{n-1} only."""
    spec = SPEC1
    p = _params(spec, 11)
    b = synth.split(spec, p)
    b["b_g"][:] = BIG
    b["b_r"][:] = -BIG

    def logits(c, n):
        x = np.zeros(2) if n == 0 else _onehot(c, n - 1)
        h = np.tanh(b["W_in"] @ x + b["b_in"])
        return b["U_a"] @ h + b["c_a"]

    lp = _check(ora, spec, p, lambda cfg: _chain_logp(cfg, range(spec.N), logits))
    # a reset gate placed before W_h would let b_h through: the closed form
    # above ignores b_h, and so must the oracle
    b["b_h"][:] += 0.9
    b["W_h"][:] *= -2.0
    lp2, _ = ora.logpsi(_model(ora, spec), p, exact.all_configs(spec.N))
    assert np.max(np.abs(lp2 - lp)) < 1e-12


def test_1d_update_closed_is_product_state(ora):
    """u = 0: h stays h_0 = 0, every conditional is softmax(c_a)."""
    spec = SPEC1
    p = _params(spec, 12)
    b = synth.split(spec, p)
    b["b_g"][:] = -BIG
    _check(ora, spec, p, lambda cfg: _chain_logp(cfg, range(spec.N), lambda c, n: b["c_a"].copy()))


def test_1d_reset_open_is_tanh_rnn(ora):
    """u = 1, r = 1: h_n = tanh(W_h h_{n-1} + b_h + W_in x_{n-1} + b_in), the
    tanh recursion of Eq. (2) with W_h on the hidden state."""
    spec = SPEC1
    p = _params(spec, 13)
    b = synth.split(spec, p)
    b["b_g"][:] = BIG
    b["b_r"][:] = BIG

    def want(cfg):
        out = np.zeros(len(cfg))
        for s, c in enumerate(cfg):
            h = np.zeros(spec.d_h)
            for n in range(spec.N):
                x = np.zeros(2) if n == 0 else _onehot(c, n - 1)
                h = np.tanh(b["W_h"] @ h + b["b_h"] + b["W_in"] @ x + b["b_in"])
                out[s] += _log_softmax(b["U_a"] @ h + b["c_a"])[c[n]]
        return out

    _check(ora, spec, p, want)


def test_1d_update_gate_selects_by_previous_spin(ora):
    """W_g acts only through its one-hot columns, +60 for sigma_{n-1} = 0 and
    -60 for sigma_{n-1} = 1; r = 0.  Then h_n = tanh(W_in e_0 + b_in) after a
    0 and h_n = h_{n-1} after a 1; at n = 0 (no input) u = 1/2 and
    h = tanh(b_in) / 2."""
    spec = SPEC1
    p = _params(spec, 14)
    b = synth.split(spec, p)
    d = spec.d_h
    b["W_g"][:, :d] = 0.0
    b["W_g"][:, d] = BIG
    b["W_g"][:, d + 1] = -BIG
    b["b_g"][:] = 0.0
    b["b_r"][:] = -BIG

    def want(cfg):
        out = np.zeros(len(cfg))
        for s, c in enumerate(cfg):
            h = 0.5 * np.tanh(b["b_in"])
            for n in range(spec.N):
                if n > 0 and c[n - 1] == 0:
                    h = np.tanh(b["W_in"][:, 0] + b["b_in"])
                out[s] += _log_softmax(b["U_a"] @ h + b["c_a"])[c[n]]
        return out

    _check(ora, spec, p, want)


def test_glu_halves(ora):
    """GLU g = (W_1 h + b_1) * sig(W_2 h + b_2) on the Markov-chain cell of
    the first pin: with W_2 = 0, b_2 = +60 the GLU is the affine map W_1 h +
    b_1; with b_2 = -60 it is 0 and every conditional is softmax(c_a)."""
    spec = synth.ModelSpec(dims=1, Lx=6, d_h=4, glu=True)
    p = _params(spec, 15)
    b = synth.split(spec, p)
    b["b_g"][:] = BIG
    b["b_r"][:] = -BIG
    b["W_2"][:] = 0.0
    b["b_2"][:] = BIG

    def logits(c, n):
        x = np.zeros(2) if n == 0 else _onehot(c, n - 1)
        h = np.tanh(b["W_in"] @ x + b["b_in"])
        return b["U_a"] @ (b["W_1"] @ h + b["b_1"]) + b["c_a"]

    _check(ora, spec, p, lambda cfg: _chain_logp(cfg, range(spec.N), logits))
    b["b_2"][:] = -BIG
    _check(ora, spec, p, lambda cfg: _chain_logp(cfg, range(spec.N), lambda c, n: b["c_a"].copy()))


# ------------------------------------------------------------------ 2D cell

SPEC2 = synth.ModelSpec(dims=2, Lx=3, Ly=3, d_h=3)


def test_2d_update_open_depends_on_neighbour_spins_only(ora):
    """u = 1: h = tanh(W [h'; s'] + b); with the hidden blocks of W zero the
    conditional at a site is a function of its two predecessor spins
    (one-hot columns in the order [x_hz; x_vt], absent = 0)."""
    spec = SPEC2
    p = _params(spec, 21)
    b = synth.split(spec, p)
    d = spec.d_h
    b["b_g"][:] = BIG
    b["W"][:, :2 * d] = 0.0
    zz = _zigzag(spec.Lx, spec.Ly)

    def logits(c, n):
        _, hz, vt = zz[n]
        x = np.concatenate([_onehot(c, hz), _onehot(c, vt)])
        h = np.tanh(b["W"][:, 2 * d:] @ x + b["b"])
        return b["U_a"] @ h + b["c_a"]

    _check(ora, spec, p, lambda cfg: _chain_logp(cfg, [z[0] for z in zz], logits))


def test_2d_update_closed_is_product_state(ora):
    """u = 0: h = U h' stays 0 from the first site on; every conditional is
    softmax(c_a)."""
    spec = SPEC2
    p = _params(spec, 22)
    b = synth.split(spec, p)
    b["b_g"][:] = -BIG
    zz = _zigzag(spec.Lx, spec.Ly)
    _check(ora, spec, p, lambda cfg: _chain_logp(cfg, [z[0] for z in zz], lambda c, n: b["c_a"].copy()))


def test_2d_update_gate_selects_candidate_or_carry(ora):
    """W_g acts only through its horizontal one-hot columns (+60 for a 0,
    -60 for a 1) and the hidden blocks of W are zero: after a horizontal 0
    h = tanh(W_x s' + b) (the candidate), after a horizontal 1
    h = U[:, :d] h_hz + U[:, d:] h_vt (the carry), at a row start (no
    horizontal neighbour) the average of the two."""
    spec = SPEC2
    p = _params(spec, 23)
    b = synth.split(spec, p)
    d = spec.d_h
    b["W"][:, :2 * d] = 0.0
    b["W_g"][:, :] = 0.0
    b["W_g"][:, 2 * d] = BIG
    b["W_g"][:, 2 * d + 1] = -BIG
    b["b_g"][:] = 0.0
    zz = _zigzag(spec.Lx, spec.Ly)

    def want(cfg):
        out = np.zeros(len(cfg))
        for s, c in enumerate(cfg):
            hs = {}
            for n, (site, hz, vt) in enumerate(zz):
                x = np.concatenate([_onehot(c, hz), _onehot(c, vt)])
                cand = np.tanh(b["W"][:, 2 * d:] @ x + b["b"])
                hh = hs[hz] if hz >= 0 else np.zeros(d)
                hv = hs[vt] if vt >= 0 else np.zeros(d)
                carry = b["U"][:, :d] @ hh + b["U"][:, d:] @ hv
                if hz < 0:
                    h = 0.5 * cand + 0.5 * carry
                elif c[hz] == 0:
                    h = cand
                else:
                    h = carry
                hs[site] = h
                out[s] += _log_softmax(b["U_a"] @ h + b["c_a"])[c[site]]
        return out

    _check(ora, spec, p, want)


def test_2d_update_open_is_tanh_rnn(ora):
    """u = 1: h = tanh(W[:, :d] h_hz + W[:, d:2d] h_vt + W[:, 2d:] s' + b),
    the 2D tanh recursion on the zig-zag predecessors."""
    spec = SPEC2
    p = _params(spec, 24)
    b = synth.split(spec, p)
    d = spec.d_h
    b["b_g"][:] = BIG
    zz = _zigzag(spec.Lx, spec.Ly)

    def want(cfg):
        out = np.zeros(len(cfg))
        for s, c in enumerate(cfg):
            hs = {}
            for site, hz, vt in zz:
                x = np.concatenate([_onehot(c, hz), _onehot(c, vt)])
                hh = hs[hz] if hz >= 0 else np.zeros(d)
                hv = hs[vt] if vt >= 0 else np.zeros(d)
                h = np.tanh(b["W"][:, :d] @ hh + b["W"][:, d:2 * d] @ hv + b["W"][:, 2 * d:] @ x + b["b"])
                hs[site] = h
                out[s] += _log_softmax(b["U_a"] @ h + b["c_a"])[c[site]]
        return out

    _check(ora, spec, p, want)


@pytest.mark.parametrize("dims", [1, 2])
def test_phase_head_closed_form(ora, dims):
    """Complex RNN with the update gate closed (h = 0): phi = sum_n
    pi * softsign(c_p)[sigma_n] (Eq. (5)), with its own head bias c_p."""
    spec = synth.ModelSpec(dims=dims, Lx=3, Ly=2 if dims == 2 else 1, d_h=3, is_complex=True)
    p = _params(spec, 25)
    b = synth.split(spec, p)
    b["b_g"][:] = -BIG
    m = _model(ora, spec)
    cfg = exact.all_configs(spec.N)
    _, ph = ora.logpsi(m, p, cfg)
    zph = np.pi * b["c_p"] / (1.0 + np.abs(b["c_p"]))
    n1 = cfg.sum(1)
    assert np.max(np.abs(ph - (n1 * zph[1] + (spec.N - n1) * zph[0]))) < 1e-12
