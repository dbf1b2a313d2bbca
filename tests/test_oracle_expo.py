"""Pins of the oracle's exact propagation in homogeneous media (CPU).

``expo_advance`` is checked against things it does not compute itself: the
RK4 time-marching solver (already pinned) converging at fourth order, the
steady state reached for long times, the closed form of the spatial mean
of the fluence, and the semigroup property including the source term.
"""
import numpy as np

from oracle import pn


def _setup(seed, n=8, N=2, src=True):
    rng = np.random.default_rng(seed)
    M = (N + 1) ** 2
    psi0 = rng.standard_normal((M, n, n, n))
    q = rng.standard_normal((M, n, n, n)) if src else None
    return psi0, q


def _hom(n, mua, mus, g):
    return (np.full((n, n, n), mua), np.full((n, n, n), mus), np.full((n, n, n), g))


def test_matches_rk4_marching_at_fourth_order():
    """K RK4 steps of the marching solver approach the exact propagation
    with error ~ dt^4: halving dt divides the error by about 16."""
    n, N, dx, c = 8, 2, 0.5, 0.3
    mua, mus, g = 0.2, 2.0, 0.7
    psi0, q = _setup(1, n, N)
    T = 2.0
    ex = pn.expo_advance(n, N, dx, c, mua, mus, g, psi0, q, T)
    errs = []
    for K in (16, 32):
        st = pn.solve(n, N, dx, c, T / K, *_hom(n, mua, mus, g), psi0, q, 0, 0.01, 1.0, K)["state"]
        errs.append(np.linalg.norm(st - ex) / np.linalg.norm(ex))
    assert errs[1] < 2e-6
    assert 12.0 < errs[0] / errs[1] < 20.0, errs


def test_long_time_limit_is_the_steady_state():
    """For c mu_a T >> 1 the propagated state is the steady state of the
    periodic homogeneous problem (oracle GMRES, pinned to a direct solve)."""
    n, N, dx, c = 8, 3, 0.5, 0.3
    mua, mus, g = 0.5, 3.0, 0.8
    psi0, q = _setup(2, n, N)
    T = 400.0                       # exp(-c mu_a T) = exp(-60)
    ex = pn.expo_advance(n, N, dx, c, mua, mus, g, psi0, q, T)
    ss = pn.steady_state(n, N, dx, c, *_hom(n, mua, mus, g), q, 0, 0.01, 1.0, tol=1e-13)
    assert np.linalg.norm(ex - ss) <= 1e-10 * np.linalg.norm(ss)


def test_mean_fluence_closed_form():
    """The k = 0 fluence mode obeys dphi/dt = c (-mu_a phi + q0): its mean
    is exp(-c mu_a T) phi(0) + (1 - exp(-c mu_a T)) q0 / mu_a."""
    n, N, dx, c = 8, 2, 0.5, 0.3
    mua, mus, g = 0.3, 2.0, 0.6
    psi0, q = _setup(3, n, N)
    T = 3.7
    ex = pn.expo_advance(n, N, dx, c, mua, mus, g, psi0, q, T)
    e = np.exp(-c * mua * T)
    want = e * psi0[0].mean() + (1 - e) * q[0].mean() / mua
    assert abs(ex[0].mean() - want) <= 1e-13 * max(1.0, abs(want))


def test_semigroup_with_source():
    """Propagating by T1 then T2 equals propagating by T1 + T2 (the source
    term composes through the integral of the exponential)."""
    n, N, dx, c = 8, 2, 0.5, 0.3
    mua, mus, g = 0.1, 1.5, 0.9
    psi0, q = _setup(4, n, N)
    a = pn.expo_advance(n, N, dx, c, mua, mus, g, psi0, q, 1.3)
    a = pn.expo_advance(n, N, dx, c, mua, mus, g, a, q, 2.1)
    b = pn.expo_advance(n, N, dx, c, mua, mus, g, psi0, q, 3.4)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
