"""Pins of the oracle's exact propagation in homogeneous media and of its
time-dependent-source step (CPU).

``expo_advance`` is checked against things it does not compute itself: the
RK4 time-marching solver (already pinned) converging at fourth order, the
steady state reached for long times, the closed form of the spatial mean
of the fluence, and the semigroup property including the source term. The
time-dependent source step is checked against the classic RK4 solve for a
constant profile and against the closed form of a single mode under a
linearly ramped source (fourth-order convergence).
"""
import numpy as np

import rte_inputs as ri

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


# ------------------------------------------------ time-dependent sources ---

def test_constant_profile_equals_autonomous_rk4():
    """A constant profile s = 1 gives the classic RK4 solve of the constant
    source (two independent formulations of the same step)."""
    n, N, dx, c = 8, 2, 0.5, 0.3
    rng = np.random.default_rng(11)
    M = (N + 1) ** 2
    psi0 = rng.standard_normal((M, n, n, n))
    q = rng.standard_normal((M, n, n, n))
    mua, mus, g = rng.uniform(0.05, 0.2, (n, n, n)), rng.uniform(1, 3, (n, n, n)), rng.uniform(0.5, 0.9, (n, n, n))
    dt = 0.2 * dx / c
    a = pn.solve(n, N, dx, c, dt, mua, mus, g, psi0, q, 2, 0.01, 1.0, 4)["state"]
    b = pn.solve(n, N, dx, c, dt, mua, mus, g, psi0, q, 2, 0.01, 1.0, 4,
                 q_profile=([1.0, 1.0], 10.0))["state"]
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_linear_profile_single_mode_fourth_order():
    """One Fourier mode with a source ramping linearly in time: the exact
    solution is the exponential of the generator augmented by the ramp
    ``[[M, c q, 0], [0, 0, 1], [0, 0, 0]]``; the time-dependent RK4 step
    converges to it at fourth order."""
    from scipy.linalg import expm
    n, N, dx, c = 8, 2, 0.5, 0.3
    M = (N + 1) ** 2
    rng = np.random.default_rng(12)
    v = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    w = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = (1, 2, -1)
    mua, mus, g = 0.1, 2.0, 0.8
    sig = [mua + mus * (1 - g ** l) for l in range(N + 1)]
    k = pn.wavenumbers(n, dx)
    kv = (k[f[0]], k[f[1]], k[f[2]])
    U = pn.real_basis_transform(N)
    T, alpha, beta = 2.0, 0.5, 1.5           # s(t) = alpha + beta t

    def exact(kvec, a0, qa):
        G = np.zeros((M + 2, M + 2), complex)
        G[:M, :M] = pn.mode_matrix(N, kvec, sig, c)
        G[:M, M] = c * qa
        G[M, M + 1] = 1.0
        z = np.concatenate([a0, [alpha, beta]])
        return (expm(T * G) @ z)[:M]

    aR = U.conj() @ exact(kv, U.T @ v, U.T @ w)
    aRm = U.conj() @ exact(tuple(-t for t in kv), U.T @ v.conj(), U.T @ w.conj())
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ph = np.exp(2j * np.pi * (f[0] * x + f[1] * y + f[2] * z) / n)
    ref = np.array([(0.5 * (aR[a] * ph + aRm[a] * ph.conj())).real for a in range(M)])
    psi0 = ri.fourier_mode_ic(n, N, f, v)
    q = ri.fourier_mode_ic(n, N, f, w)
    ma, ms, gg = (np.full((n, n, n), x_) for x_ in (mua, mus, g))
    prof = ([alpha, alpha + beta * 10.0], 10.0)   # linear over [0, 10]
    errs = []
    for K in (8, 16):
        st = pn.solve(n, N, dx, c, T / K, ma, ms, gg, psi0, q, 0, 0.01, 1.0, K, q_profile=prof)["state"]
        errs.append(np.linalg.norm(st - ref) / np.linalg.norm(ref))
    assert errs[1] < 1e-5
    assert 12.0 < errs[0] / errs[1] < 20.0, errs
