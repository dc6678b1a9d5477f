"""Pins of the oracle's local energies of the long-range TFIM (Eq. (8)) and
of the 1D cluster state (Eq. (9)), and of its Adam step (App. B), against
facts fixed by the paper and by mathematics: Hamiltonians built from Pauli
Kronecker products, the cluster ground energy -n, limits of the long-range
exponent, product-state closed forms and the first Adam step.  CPU only."""
import math

import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests import exact


def _make(ora, N, d_h, cplx, seed, glu=False):
    spec = synth.ModelSpec(dims=1, Lx=N, d_h=d_h, is_complex=cplx, glu=glu)
    m = ora.model(dims=1, Lx=N, d_h=d_h, is_complex=cplx, glu=glu)
    p = synth.xavier_params(spec, seed, bias_scale=0.3, gain=1.5, dtype=np.float64)
    return spec, m, p


CASES = [
    ("lrtfim", dict(J=0.8, h=1.1, alpha=0.1), 6, False),
    ("lrtfim", dict(J=1.0, h=0.7, alpha=1.7), 7, True),
    ("cluster", dict(J=1.0), 6, True),
    ("cluster", dict(J=0.6), 5, False),
    ("cluster", dict(J=1.0), 3, True),
    ("cluster", dict(J=1.0), 4, True),
]


def _hams(ora, kind, kw, N):
    if kind == "lrtfim":
        return ora.ham(ora.LRTFIM, J=kw["J"], h=kw["h"], alpha=kw["alpha"]), \
            exact.lrtfim(N, kw["J"], kw["h"], kw["alpha"])
    return ora.ham(ora.CLUSTER, J=kw["J"]), exact.cluster(N, kw["J"])


@pytest.mark.parametrize("kind,kw,N,cplx", CASES, ids=lambda x: str(x))
def test_local_energy_is_h_psi_over_psi(ora, kind, kw, N, cplx):
    """(H psi)(sigma) = E_loc(sigma) psi(sigma) for every configuration, and
    sum_sigma P E_loc = <psi|H|psi>, with H from Pauli Kronecker products."""
    spec, m, p = _make(ora, N, 4, cplx, seed=N)
    h_ora, h_ex = _hams(ora, kind, kw, N)
    cfg = exact.all_configs(N)
    lp, ph = ora.logpsi(m, p, cfg)
    psi = np.exp(0.5 * lp + 1j * ph)
    e = ora.local_energy(m, p, h_ora, cfg)
    hpsi = h_ex @ psi
    assert np.max(np.abs(hpsi - e * psi)) < 1e-12
    assert abs(np.sum(np.exp(lp) * e) - np.vdot(psi, hpsi)) < 1e-12


@pytest.mark.parametrize("n", [3, 4, 6, 8])
def test_cluster_ground_energy_is_minus_n(n):
    """The n terms of Eq. (9), as written, commute and are independent, so the
    ground energy is -n (the value the paper quotes for n = 64)."""
    H = exact.cluster(n)
    assert abs(exact.ground_energy(H) - (-n)) < 1e-10
    assert abs(H - H.conj().T).max() < 1e-15


def test_cluster_zero_weights_closed_form(ora):
    """All parameters zero: psi uniform, every ratio 1, so
    E_loc = -J sum_terms prod_Z s_z; its mean over all configurations is -J
    (only the X_{n-1} X_n term has no Z)."""
    N, J = 6, 0.9
    spec, m, _ = _make(ora, N, 3, True, 0)
    p = np.zeros(ora.param_count(m))
    cfg = exact.all_configs(N)
    e = ora.local_energy(m, p, ora.ham(ora.CLUSTER, J=J), cfg)
    s = 1.0 - 2.0 * cfg
    want = -J * (sum(s[:, k] for k in range(1, N - 3 + 1)) + s[:, 0] + 1.0 + s[:, N - 2] * s[:, N - 1])
    assert np.max(np.abs(e - want)) < 1e-12
    assert abs(e.mean() - (-J)) < 1e-12


def test_lrtfim_limits(ora):
    """alpha -> infinity leaves the nearest-neighbour TFIM of Eq. (6); alpha =
    0 gives the all-to-all coupling -J ((sum s)^2 - N) / 2."""
    N = 7
    spec, m, p = _make(ora, N, 4, True, 3)
    cfg = synth.configs(40, N, 1)
    e_nn = ora.local_energy(m, p, ora.ham(ora.TFIM, J=0.8, h=1.3), cfg)
    e_lr = ora.local_energy(m, p, ora.ham(ora.LRTFIM, J=0.8, h=1.3, alpha=200.0), cfg)
    assert np.max(np.abs(e_lr - e_nn)) < 1e-12
    e0 = ora.local_energy(m, p, ora.ham(ora.LRTFIM, J=0.8, h=1.3, alpha=0.0), cfg)
    s = 1.0 - 2.0 * cfg
    diag = -0.8 * (s.sum(1) ** 2 - N) / 2.0
    e_nn_off = e_nn - (-0.8 * (s[:, :-1] * s[:, 1:]).sum(1))
    assert np.max(np.abs(e0 - (diag + e_nn_off))) < 1e-11


def test_lrtfim_variational_bound(ora):
    """<psi|H|psi> >= E_0 of Eq. (8) by exact diagonalisation (N = 8)."""
    N = 8
    spec, m, p = _make(ora, N, 4, False, 5)
    cfg = exact.all_configs(N)
    lp, _ = ora.logpsi(m, p, cfg)
    e = ora.local_energy(m, p, ora.ham(ora.LRTFIM, J=1.0, h=1.0, alpha=0.1), cfg)
    e0 = exact.ground_energy(exact.lrtfim(N, 1.0, 1.0, 0.1))
    assert np.sum(np.exp(lp) * e).real >= e0 - 1e-12


def test_adam_first_step_and_constant_gradient(ora):
    """With zero moments, the first Adam step is lr * g / (|g| + eps) per
    entry (bias-corrected moments are g and g^2); under a constant gradient
    every later step is the same."""
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    m = np.zeros(50)
    v = np.zeros(50)
    p1, m1, v1 = ora.adam(p, g, m, v, 1, lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    q, mm, vv = p1, m1, v1
    for t in range(2, 6):
        q2, mm, vv = ora.adam(q, g, mm, vv, t, lr, eps=eps)
        assert np.allclose(q - q2, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)
        q = q2


def test_adam_minimises_a_quadratic(ora):
    """Adam on f(p) = |p - c|^2 / 2 (gradient p - c) reaches c."""
    c = np.linspace(-1.0, 2.0, 7)
    p = np.zeros(7)
    m = np.zeros(7)
    v = np.zeros(7)
    for t in range(1, 3001):
        p, m, v = ora.adam(p, p - c, m, v, t, 1e-2)
    assert np.max(np.abs(p - c)) < 1e-3
