"""Pins of the oracle's discrete adjoint (CPU).

The adjoint is checked against things it does not compute itself: the
forward operator (dot-product identity), central finite differences of the
forward solver, and the second-order Taylor remainder.
"""
import numpy as np
import pytest

import rte_inputs as ri
from oracle import pn


def _tiny(seed=0, n=8, N=2, W=1):
    rng = np.random.default_rng(seed)
    mu_a = rng.uniform(0.05, 0.3, (n, n, n))
    mu_s = rng.uniform(1.0, 4.0, (n, n, n))
    g = rng.uniform(0.5, 0.9, (n, n, n))
    return rng, n, N, W, mu_a, mu_s, g


def test_operator_transpose_dot_product():
    """<L x, y> = <x, L^T y> for the linear part of the operator (no
    source), heterogeneous medium with absorbing layer; L applied by the
    complex-basis oracle operator, L^T by the real-basis transpose."""
    rng, n, N, W, mu_a, mu_s, g = _tiny(1)
    M = (N + 1) ** 2
    dx, c = 0.5, 0.3
    U = pn.real_basis_transform(N)
    Sig, _ = pn.potentials(mu_a, mu_s, g, N, W, 0.01, 1.0)
    k = pn.wavenumbers(n, dx)
    x = rng.standard_normal((M, n, n, n))
    y = rng.standard_normal((M, n, n, n))
    Lx = pn.to_real_basis(pn.operator(pn.to_complex_basis(x, U).astype(complex), Sig, None,
                                      pn.coupling_matrices(N), k, c), U)
    LTy = pn.operator_transpose(y, Sig, pn.real_coupling(N), k, c)
    lhs, rhs = float((Lx * y).sum()), float((x * LTy).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def _loss(wl_args, det, target, mu_a, mu_s, scheme="rk4"):
    n, N, dx, c, dt, g, psi0, W, steps = wl_args
    out = pn.solve(n, N, dx, c, dt, mu_a, mu_s, g, psi0, None, W, 0.01, 1.0, steps,
                   det_index=det, return_state=False, scheme=scheme)
    r = out["readings"]
    return float(((r - target) ** 2).sum()), r


@pytest.mark.parametrize("scheme", ["rk4", "euler"])
def test_adjoint_matches_central_differences(scheme):
    """dJ/dmu_a and dJ/dmu_s from the reverse sweep equal central finite
    differences of the forward solver at interior voxels (FP64), for the
    RK4 scheme and the first-order step of eq. (11)."""
    rng, n, N, W, mu_a, mu_s, g = _tiny(2)
    dx, c = 0.5, 0.3
    dt = 0.2 * dx / c
    steps = 6
    psi0 = ri.gaussian_ic(n, N, sigma=1.0)
    det = np.array([(3 * n + 4) * n + 2, (5 * n + 2) * n + 5], np.int64)
    target = rng.uniform(0.0, 0.01, (steps, det.size))
    args = (n, N, dx, c, dt, g, psi0, W, steps)
    J0, r = _loss(args, det, target, mu_a, mu_s, scheme)
    djdr = 2.0 * (r - target)
    ga, gs = pn.adjoint_gradient(n, N, dx, c, dt, mu_a, mu_s, g, psi0, None, W, 0.01, 1.0,
                                 steps, det, djdr, scheme=scheme)
    for (z, y, x) in [(3, 3, 3), (4, 2, 5), (5, 5, 2)]:
        for grad, which in ((ga, "a"), (gs, "s")):
            eps = 1e-5
            ma, ms = mu_a.copy(), mu_s.copy()
            base = ma if which == "a" else ms
            h = eps * base[z, y, x]
            base[z, y, x] += h
            Jp, _ = _loss(args, det, target, ma, ms, scheme)
            base[z, y, x] -= 2 * h
            Jm, _ = _loss(args, det, target, ma, ms, scheme)
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - grad[z, y, x]) <= 1e-6 * max(abs(fd), 1e-12) + 1e-14, (which, fd, grad[z, y, x])
    # zero inside the absorbing layer
    assert np.all(ga[0] == 0.0) and np.all(gs[:, :, n - 1] == 0.0)


def test_taylor_remainder_is_second_order():
    """J(mu + e d) - J(mu) - e <grad, d> shrinks as e^2 along a random
    direction d supported inside the real domain."""
    rng, n, N, W, mu_a, mu_s, g = _tiny(3)
    dx, c = 0.5, 0.3
    dt = 0.2 * dx / c
    steps = 5
    psi0 = ri.gaussian_ic(n, N, sigma=1.0)
    det = np.array([(2 * n + 3) * n + 3, (4 * n + 4) * n + 5], np.int64)
    target = np.zeros((steps, det.size))
    args = (n, N, dx, c, dt, g, psi0, W, steps)
    J0, r = _loss(args, det, target, mu_a, mu_s)
    ga, gs = pn.adjoint_gradient(n, N, dx, c, dt, mu_a, mu_s, g, psi0, None, W, 0.01, 1.0,
                                 steps, det, 2.0 * (r - target))
    omega = pn.pml_depth(n, W) == 0
    da = rng.standard_normal((n, n, n)) * omega * mu_a
    ds = rng.standard_normal((n, n, n)) * omega * mu_s
    lin = float((ga * da).sum() + (gs * ds).sum())
    rem = []
    for e in (1e-2, 5e-3):
        Je, _ = _loss(args, det, target, mu_a + e * da, mu_s + e * ds)
        rem.append(abs(Je - J0 - e * lin))
    assert 3.0 < rem[0] / rem[1] < 5.0, rem
