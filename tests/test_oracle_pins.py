"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names the passage of the paper it pins and the independent fact
it uses (quadrature of scipy's spherical harmonics, Gauss-Legendre nodes,
closed-form dispersion, matrix exponentials, conservation laws). All run on
the CPU in seconds.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy.special import sph_harm_y

import rte_inputs as ri
from oracle import pn


# ------------------------------------------------------------- helpers ---

def _quad(L):
    nt = L // 2 + 1
    nph = L + 1
    x, wx = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(nph) / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    return T.ravel(), P.ravel(), np.outer(wx, np.full(nph, 2 * np.pi / nph)).ravel()


def _Y(N, T, P):
    rows = []
    for l in range(N + 1):
        for m in range(-l, l + 1):
            rows.append(sph_harm_y(l, m, T, P))
    return np.array(rows)


def _lw(N):
    return np.array([2 * l + 1 for l in range(N + 1) for _ in range(2 * l + 1)], float)


# --------------------------------------------------- eq. (6) coupling ---

@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_coupling_equals_quadrature_projection(N):
    """C-P1, eq. (6): the streaming coefficients equal the projection of
    s_j Y_b onto Y_a (exact quadrature of scipy's Condon-Shortley harmonics),
    rescaled to psi-coordinates by sqrt((2l_b+1)/(2l_a+1)) (eq. 3 weights)."""
    Bs = pn.coupling_matrices(N)
    T, P, W = _quad(2 * N + 3)
    Y = _Y(N, T, P)
    s = (np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T))
    lw = _lw(N)
    for j in range(3):
        Q = (Y.conj() * (W * s[j])) @ Y.T
        Q = Q * np.sqrt(lw[None, :] / lw[:, None])
        assert np.abs(Q - Bs[j]).max() < 1e-13


@pytest.mark.parametrize("N", [1, 3, 5, 7])
def test_m0_block_eigenvalues_are_gauss_legendre_nodes(N):
    """C-P3, alpha of eq. (6): the m=0 block of B_z is a Jacobi matrix of
    the Legendre recurrence, so its eigenvalues are the N+1 Gauss-Legendre
    nodes."""
    Bz = pn.coupling_matrices(N)[2]
    idx = [pn.sh_index(l, 0) for l in range(N + 1)]
    ev = np.sort(np.linalg.eigvals(Bz[np.ix_(idx, idx)]).real)
    nodes = np.sort(np.polynomial.legendre.leggauss(N + 1)[0])
    assert np.abs(ev - nodes).max() < 1e-13


@pytest.mark.parametrize("N", [1, 3, 7])
def test_streaming_spectrum_is_rotation_invariant(N):
    """C-P4, beta of eq. (6): spec(khat . B) = spec(B_z) for any unit khat,
    since s.khat is a rotated s_z."""
    Bx, By, Bz = pn.coupling_matrices(N)
    rng = np.random.default_rng(N)
    ref = np.sort(np.linalg.eigvals(Bz).real)
    for _ in range(3):
        kh = rng.standard_normal(3)
        kh /= np.linalg.norm(kh)
        ev = np.linalg.eigvals(kh[0] * Bx + kh[1] * By + kh[2] * Bz)
        assert np.abs(ev.imag).max() < 1e-10
        assert np.abs(np.sort(ev.real) - ref).max() < 1e-12


@pytest.mark.parametrize("N", [1, 3, 5, 7])
def test_real_basis_tables_real_and_symmetric(N):
    """C-P2: in the real basis the streaming matrices are real, and in
    orthonormal coordinates they are symmetric (s_j is a real multiplication
    operator); nnz 6/70/214/438 for N=1/3/5/7 across the three matrices."""
    U = pn.real_basis_transform(N)
    M = (N + 1) ** 2
    assert np.abs(U @ U.conj().T - np.eye(M)).max() < 1e-13
    c = np.sqrt(_lw(N))
    nnz = 0
    for B in pn.coupling_matrices(N):
        R = U.conj() @ B @ U.T
        assert np.abs(R.imag).max() < 1e-14
        O = (c[:, None] * R.real) / c[None, :]
        assert np.abs(O - O.T).max() < 1e-14
        nnz += int((np.abs(R.real) > 1e-12).sum())
    assert nnz == {1: 6, 3: 70, 5: 214, 7: 438}[N]


def test_real_basis_low_order_moments_are_fluence_and_flux():
    """Real basis (eq. 3 weights): psi^R_00 is the fluence and
    (psi^R_{1,1}, psi^R_{1,-1}, psi^R_{1,0}) the flux vector J, checked by
    building the radiance from random moments and integrating it over the
    sphere with an independent quadrature."""
    N = 3
    U = pn.real_basis_transform(N)
    rng = np.random.default_rng(7)
    psiR = rng.standard_normal((N + 1) ** 2)
    psi = U.T @ psiR
    T, P, W = _quad(2 * N + 4)
    Y = _Y(N, T, P)
    cl = np.sqrt(_lw(N) / (4 * np.pi))
    rad = ((cl * psi)[:, None] * Y).sum(0)
    assert np.abs(rad.imag).max() < 1e-12
    rad = rad.real
    s = (np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T))
    assert abs((W * rad).sum() - psiR[0]) < 1e-12
    J = [(W * s[j] * rad).sum() for j in range(3)]
    assert np.allclose(J, [psiR[pn.sh_index(1, 1)], psiR[pn.sh_index(1, -1)],
                           psiR[pn.sh_index(1, 0)]], atol=1e-12)
    back = pn.to_real_basis(pn.to_complex_basis(
        rng.standard_normal(((N + 1) ** 2, 2, 2, 2)), U), U)
    assert back.shape == ((N + 1) ** 2, 2, 2, 2)


# ---------------------------------------------------- eq. (2) and (5) ---

@pytest.mark.parametrize("g", [0.0, 0.5, 0.9, 0.95])
def test_hg_legendre_moments_are_powers_of_g(g):
    """C-P6, eqs. (2) and (5): the Legendre moments of the HG phase function
    are exactly g^l, which is the diagonal in-scatter factor per degree."""
    mom = pn.hg_legendre_moments(g, 8, nodes=2000 if g > 0.9 else 400)
    assert np.abs(mom - g ** np.arange(9)).max() < 1e-9


# ------------------------------------------------------- spectral grid ---

def test_wavenumbers_nyquist_zero():
    """Sec. II.A reading: k = 2 pi f/(n dx), Nyquist entry zero."""
    k = pn.wavenumbers(8, 0.5)
    assert k[4] == 0.0
    assert np.allclose(k[:4], 2 * np.pi * np.arange(4) / 4.0)
    assert np.allclose(k[5:], -2 * np.pi * np.arange(3, 0, -1) / 4.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("f", [1, 3, 7])
def test_p1_continuity_is_exact_spectral_divergence(axis, f):
    """C-P7 and C-P5 (first row): with no loss and no source the P_1 system
    gives d(phi)/dt = -c div J, and for a band-limited sin field (|f| < n/2)
    the spectral derivative is exact to rounding."""
    n, N, dx, c = 16, 1, 0.5, 0.3
    U = pn.real_basis_transform(N)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    coord = (x, y, z)[axis] * dx
    kk = 2 * np.pi * f / (n * dx)
    psiR = np.zeros((4, n, n, n))
    comp = (pn.sh_index(1, 1), pn.sh_index(1, -1), pn.sh_index(1, 0))[axis]
    psiR[comp] = np.sin(kk * coord)
    psi = pn.to_complex_basis(psiR, U).astype(complex)
    Sig = np.zeros((2, n, n, n))
    out = pn.to_real_basis(pn.operator(psi, Sig, None, pn.coupling_matrices(N),
                                       pn.wavenumbers(n, dx), c), U)
    assert np.abs(out[0] + c * kk * np.cos(kk * coord)).max() < 1e-12
    assert np.abs(out[1:]).max() < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_p1_flux_equation_gradient(axis):
    """C-P5 (second row): dJ/dt = -c grad(phi)/3 - c mu_1 J for P_1, with
    mu_1 = mu_a + mu_s (1 - g); checked on phi = cos(k.r), J = 0."""
    n, N, dx, c = 16, 1, 0.5, 0.3
    mua, mus, g = 0.02, 3.0, 0.8
    U = pn.real_basis_transform(N)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    coord = (x, y, z)[axis] * dx
    kk = 2 * np.pi * 5 / (n * dx)
    psiR = np.zeros((4, n, n, n))
    psiR[0] = np.cos(kk * coord)
    psiR[pn.sh_index(1, 0)] = 0.25      # a uniform J_z to see the mu_1 loss
    ma, ms, gg = ri.homogeneous_maps(n, mua, mus, g)
    Sig, _ = pn.potentials(ma, ms, gg, N, 0, 0.01, 1.0)
    psi = pn.to_complex_basis(psiR, U).astype(complex)
    out = pn.to_real_basis(pn.operator(psi, Sig, None, pn.coupling_matrices(N),
                                       pn.wavenumbers(n, dx), c), U)
    mu1 = mua + mus * (1 - g)
    expect_J = [np.zeros_like(coord) for _ in range(3)]
    expect_J[axis] = expect_J[axis] + c * kk * np.sin(kk * coord) / 3.0
    expect_J[2] = expect_J[2] - c * mu1 * 0.25
    got = (out[pn.sh_index(1, 1)], out[pn.sh_index(1, -1)], out[pn.sh_index(1, 0)])
    for j in range(3):
        assert np.abs(got[j] - expect_J[j]).max() < 1e-12
    assert np.abs(out[0] + c * mua * np.cos(kk * coord)).max() < 1e-12


def test_p1_dispersion_closed_form():
    """C-P5: eigenvalues of the P_1 mode generator are
    -c(mu_a+mu_1)/2 +- c sqrt((mu_1-mu_a)^2/4 - |k|^2/3) and -c mu_1 (twice)."""
    mua, mus, g, c = 0.01, 10.0, 0.9, 0.3
    mu1 = mua + mus * (1 - g)
    for kv in [(0.3, -1.2, 0.7), (2.0, 0.0, 0.0), (0.01, 0.02, 0.0)]:
        kk = np.linalg.norm(kv)
        ev = np.linalg.eigvals(pn.mode_matrix(1, kv, [mua, mua + mus * (1 - g)], c))
        disc = np.sqrt(complex((mu1 - mua) ** 2 / 4 - kk * kk / 3))
        ref = np.array([-c * (mua + mu1) / 2 + c * disc, -c * (mua + mu1) / 2 - c * disc,
                        -c * mu1, -c * mu1])
        for r in ref:
            assert np.abs(ev - r).min() < 1e-12
        for e in ev:
            assert np.abs(ref - e).min() < 1e-12


# ---------------------------------------------------- time integration ---

def _mode_state(n, N, f, v, U, R_k, R_mk):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ph = np.exp(2j * np.pi * (f[0] * x + f[1] * y + f[2] * z) / n)
    vc = U.T @ v
    vcm = U.T @ v.conj()
    pc = 0.5 * ((R_k @ vc)[:, None, None, None] * ph
                + (R_mk @ vcm)[:, None, None, None] * ph.conj())
    return pn.to_real_basis(pc, U)


@pytest.mark.parametrize("N", [1, 3])
def test_single_mode_equals_rk4_polynomial_and_expm(N):
    """C-P8: in a homogeneous periodic medium a single Fourier mode evolves
    as R(dt M(k))^n (R = RK4 stability polynomial, M(k) the block-tridiagonal
    mode generator) to rounding, and approaches expm(t M(k)) with fourth-order
    global error (halving dt cuts the error about 16x)."""
    n, dx, c = 8, 0.5, 0.3
    M = (N + 1) ** 2
    rng = np.random.default_rng(N)
    v = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = (1, -2, 3)
    mua, mus, g = 0.01, 2.0, 0.9
    ma, ms, gg = ri.homogeneous_maps(n, mua, mus, g)
    sig = [mua + mus * (1 - g ** l) for l in range(N + 1)]
    k = pn.wavenumbers(n, dx)
    kv = (k[f[0]], k[f[1]], k[f[2]])
    mkv = tuple(-t for t in kv)
    U = pn.real_basis_transform(N)
    psi0 = ri.fourier_mode_ic(n, N, f, v)
    T = 4.0
    errs = []
    for steps in (8, 16):
        dt = T / steps
        out = pn.solve(n, N, dx, c, dt, ma, ms, gg, psi0, None, 0, 0.01, 1.0, steps)
        Rk = np.linalg.matrix_power(pn.rk4_poly(dt * pn.mode_matrix(N, kv, sig, c)), steps)
        Rmk = np.linalg.matrix_power(pn.rk4_poly(dt * pn.mode_matrix(N, mkv, sig, c)), steps)
        exact_poly = _mode_state(n, N, f, v, U, Rk, Rmk)
        assert np.abs(out["state"] - exact_poly).max() < 1e-13 * max(1, np.abs(exact_poly).max())
        Ek = scipy.linalg.expm(T * pn.mode_matrix(N, kv, sig, c))
        Emk = scipy.linalg.expm(T * pn.mode_matrix(N, mkv, sig, c))
        exact = _mode_state(n, N, f, v, U, Ek, Emk)
        errs.append(np.abs(out["state"] - exact).max())
    ratio = errs[0] / errs[1]
    assert 12.0 < ratio < 20.0, errs


def test_single_mode_forward_euler():
    """Eq. (11) (first-order explicit step, sign reading R1): a single
    Fourier mode evolves as (I + dt M(k))^n exactly."""
    n, N, dx, c = 8, 2, 0.5, 0.3
    M = (N + 1) ** 2
    rng = np.random.default_rng(9)
    v = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = (2, 1, -3)
    mua, mus, g = 0.05, 3.0, 0.8
    ma, ms, gg = ri.homogeneous_maps(n, mua, mus, g)
    sig = [mua + mus * (1 - g ** l) for l in range(N + 1)]
    k = pn.wavenumbers(n, dx)
    kv = (k[f[0]], k[f[1]], k[f[2]])
    U = pn.real_basis_transform(N)
    dt, steps = 0.05, 7
    out = pn.solve(n, N, dx, c, dt, ma, ms, gg, ri.fourier_mode_ic(n, N, f, v), None, 0,
                   0.01, 1.0, steps, scheme="euler")
    I = np.eye(M)
    Rk = np.linalg.matrix_power(I + dt * pn.mode_matrix(N, kv, sig, c), steps)
    Rmk = np.linalg.matrix_power(I + dt * pn.mode_matrix(N, tuple(-t for t in kv), sig, c), steps)
    ref = _mode_state(n, N, f, v, U, Rk, Rmk)
    assert np.abs(out["state"] - ref).max() < 1e-13 * np.abs(ref).max()


def test_k0_decay_and_integrated_fluence():
    """C-P9: a uniform field in a homogeneous medium has only the k=0 mode;
    each degree decays by the scalar RK4 factor R(-c dt Sigma_l) per step
    exactly, the l=0 moment approaches exp(-c mu_a t), and the integrated
    fluence is the geometric series dt * sum_n R^n."""
    n, N, dx, c = 4, 3, 0.5, 0.3
    mua, mus, g = 0.05, 4.0, 0.7
    steps = 30
    dt = 0.2 * dx / c
    ma, ms, gg = ri.homogeneous_maps(n, mua, mus, g)
    psi0 = np.ones(((N + 1) ** 2, n, n, n))
    out = pn.solve(n, N, dx, c, dt, ma, ms, gg, psi0, None, 0, 0.01, 1.0, steps)
    for l in range(N + 1):
        z = -c * dt * (mua + mus * (1 - g ** l))
        R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
        for m in range(-l, l + 1):
            assert np.allclose(out["state"][pn.sh_index(l, m)], R ** steps, rtol=1e-13)
    z = -c * dt * mua
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    t = steps * dt
    assert abs(out["fluence"][0, 0, 0] - math.exp(-c * mua * t)) < 1e-9
    geo = dt * R * (1 - R ** steps) / (1 - R)
    assert np.allclose(out["phi_int"], geo, rtol=1e-13)
    assert np.allclose(out["readings"], 0.0) or out["readings"].size == 0


def test_photon_number_conserved_without_absorption():
    """C-P10: with mu_a = 0 and no boundary layer the l=0 loss is zero and
    the k=0 derivative vanishes, so sum_r psi_0^0 is constant to rounding
    for any heterogeneous mu_s, g."""
    n, N = 8, 3
    rng = np.random.default_rng(11)
    mus = rng.uniform(1, 10, (n, n, n))
    g = rng.uniform(0.5, 0.95, (n, n, n))
    mua = np.zeros((n, n, n))
    psi0 = rng.standard_normal(((N + 1) ** 2, n, n, n))
    out = pn.solve(n, N, 0.5, 0.3, 0.2 * 0.5 / 0.3, mua, mus, g, psi0, None, 0,
                   0.01, 1.0, 20)
    assert abs(out["fluence"].sum() - psi0[0].sum()) < 1e-11 * np.abs(psi0[0]).sum()


# --------------------------------------- tiny grids, dense operator ---

def _dense_L(n, N, dx, c, Sig):
    M = (N + 1) ** 2
    B = pn.coupling_matrices(N)
    k = pn.wavenumbers(n, dx)
    size = M * n ** 3
    L = np.zeros((size, size), complex)
    for i in range(size):
        e = np.zeros(size, complex)
        e[i] = 1.0
        L[:, i] = pn.operator(e.reshape(M, n, n, n), Sig, None, B, k, c, workers=1).ravel()
    return L


def test_dense_operator_symmetric_part_is_the_loss():
    """C-P11: on a tiny heterogeneous grid with a boundary layer, the dense
    operator L (columns = operator applied to unit vectors), written in
    orthonormal coordinates, has symmetric part exactly -c Sigma (streaming
    is skew-adjoint), so energy never increases; one oracle step equals
    R(dt L) u."""
    n, N, dx, c = 4, 2, 0.5, 0.3
    M = (N + 1) ** 2
    rng = np.random.default_rng(3)
    mua = rng.uniform(0.01, 0.1, (n, n, n))
    mus = rng.uniform(1, 10, (n, n, n))
    g = rng.uniform(0.6, 0.95, (n, n, n))
    W = 1
    Sig, _ = pn.potentials(mua, mus, g, N, W, 0.01, 1.0)
    L = _dense_L(n, N, dx, c, Sig)
    cl = np.repeat(np.sqrt(_lw(N)), n ** 3)
    O = (cl[:, None] * L) / cl[None, :]
    sym = 0.5 * (O + O.conj().T)
    lofa = np.repeat([pn.sh_lm(a)[0] for a in range(M)], n ** 3)
    D = -c * Sig[lofa, np.tile(np.arange(n ** 3) // (n * n), M),
                 np.tile((np.arange(n ** 3) // n) % n, M),
                 np.tile(np.arange(n ** 3) % n, M)]
    assert np.abs(sym - np.diag(D)).max() < 1e-13
    assert np.linalg.eigvalsh(sym).max() <= 1e-14
    dt = 0.2 * dx / c
    U = pn.real_basis_transform(N)
    psiR = rng.standard_normal((M, n, n, n))
    out = pn.solve(n, N, dx, c, dt, mua, mus, g, psiR, None, W, 0.01, 1.0, 1)
    u = pn.to_complex_basis(psiR, U).ravel()
    R = pn.rk4_poly(dt * L)
    ref = pn.to_real_basis((R @ u).reshape(M, n, n, n), U)
    assert np.abs(out["state"] - ref).max() < 1e-13


def test_steady_state_matches_direct_solve():
    """C-P11: with a constant source, marching approaches the steady state
    u* = -L^{-1} c q (q zeroed in the layer) of the dense operator."""
    n, N, dx, c = 4, 1, 0.5, 0.3
    M = (N + 1) ** 2
    rng = np.random.default_rng(5)
    mua = rng.uniform(0.3, 0.5, (n, n, n))
    mus = rng.uniform(1, 2, (n, n, n))
    g = np.full((n, n, n), 0.5)
    W = 1
    Sig, omega = pn.potentials(mua, mus, g, N, W, 0.01, 1.0)
    L = _dense_L(n, N, dx, c, Sig)
    U = pn.real_basis_transform(N)
    qR = rng.standard_normal((M, n, n, n))
    qc = pn.to_complex_basis(qR, U) * omega[None]
    ustar = np.linalg.solve(L, -c * qc.ravel())
    ref = pn.to_real_basis(ustar.reshape(M, n, n, n), U)
    dt = 0.2 * dx / c
    out = pn.solve(n, N, dx, c, dt, mua, mus, g, None, qR, W, 0.01, 1.0, 3000)
    assert np.abs(out["state"] - ref).max() < 1e-10 * np.abs(ref).max()
    assert out["residual"][-1] < 1e-12
    # the Krylov steady state (library GMRES on the oracle operator) equals
    # the direct dense solve
    ss = pn.steady_state(n, N, dx, c, mua, mus, g, qR, W, 0.01, 1.0, tol=1e-13)
    assert np.abs(ss - ref).max() < 1e-10 * np.abs(ref).max()


# ------------------------------------------------------ boundary layer ---

def test_pml_profile_special_values():
    """Sec. II.B / III.B reading: zero depth inside the real domain,
    depth W at the grid faces, mu_b = mu0 + (mu1-mu0)(1-cos(pi d/W))/2,
    rising monotonically to mu1 at depth W; the layer switches off
    scattering so Sigma_l = mu_b for every l there."""
    n, W = 16, 4
    d = pn.pml_depth(n, W)
    assert d[W:n - W, W:n - W, W:n - W].max() == 0
    assert d[0, 8, 8] == W and d[8, 8, n - 1] == W and d[0, 0, 0] == W
    assert d[W - 1, 8, 8] == 1 and d[8, n - W, 8] == 1
    mub = pn.pml_profile(n, W, 0.01, 1.0)
    assert mub[0, 8, 8] == pytest.approx(1.0, abs=1e-15)
    assert mub[W - 1, 8, 8] == pytest.approx(0.01 + 0.99 * 0.5 * (1 - math.cos(math.pi / W)))
    line = mub[8, 8, :W + 1][::-1]
    assert np.all(np.diff(line) > 0)
    mua, mus, g = ri.homogeneous_maps(n, 0.02, 7.0, 0.9)
    Sig, omega = pn.potentials(mua, mus, g, 3, W, 0.01, 1.0)
    for l in range(4):
        assert np.allclose(Sig[l][omega], 0.02 + 7.0 * (1 - 0.9 ** l))
        assert np.allclose(Sig[l][~omega], mub[~omega])


def test_outputs_bookkeeping():
    """Readings are psi_0^0 at the detector voxels after every step, the
    integrated fluence is dt times their running sum and the residual is
    the relative change of the fluence between consecutive steps."""
    wl = ri.workload("p3_adjoint", n=8, steps=3)
    wl.det_index = np.array([0, 17, 300], np.int64)
    args = (wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g, wl.psi0,
            None, wl.W, wl.mu0, wl.mu1)
    fl = [wl.psi0[0]] + [pn.solve(*args, s)["fluence"] for s in (1, 2, 3)]
    out = pn.solve(*args, 3, det_index=wl.det_index)
    for s in range(3):
        assert np.array_equal(out["readings"][s], fl[s + 1].ravel()[wl.det_index])
        assert out["residual"][s] == pytest.approx(
            np.linalg.norm(fl[s + 1] - fl[s]) / np.linalg.norm(fl[s + 1]), rel=1e-12)
    assert np.allclose(out["phi_int"], wl.dt * (fl[1] + fl[2] + fl[3]), rtol=1e-14)
