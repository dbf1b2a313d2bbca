"""FP64 reference solver for the pseudospectral P_N radiative transport step.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

What it computes (Powell, Cox & Arridge, "A pseudospectral method for
solution of the radiative transport equation", arXiv:1801.06364):

* the transport equation, eq. (1), with the Henyey-Greenstein phase
  function, eq. (2);
* radiance and source expanded in complex spherical harmonics with weights
  sqrt((2l+1)/4pi), eqs. (3)-(4); the addition theorem, eq. (5), makes the
  in-scattering diagonal, ``mu_s g^l psi_l^m``;
* the coupled first-order system eq. (6), truncated at ``l > N`` (Sec. II.A);
* spatial derivatives taken spectrally with the transform of eq. (8) on a
  periodic grid (Sec. II, II.A);
* the boundary layer of eq. (12): outside the real domain the scattering
  is switched off, the source is zero and a smooth (half-cosine) isotropic
  loss ``mu_b`` is applied (Sec. II.B, Sec. III.B);
* time marching with the classic four-stage Runge-Kutta tableau (the paper
  writes a first-order explicit step, eq. (11); the workloads here use RK4).

Readings of the paper that this module takes (the paper is silent or its
printed signs disagree with its own eqs. (1) and (6)):

* sign: ``d psi/dt = c (-[s.grad psi] - (mu_t - mu_s g^l) psi + q)``, the
  form eqs. (1) and (6) give; eqs. (9)-(11) print other signs;
* wavenumbers ``k = 2 pi f / (n dx)`` with the Nyquist entry set to zero;
* forward transform unnormalised with ``exp(-i k.r)`` (eq. 8), inverse
  scaled by ``1/n^3``;
* the layer depth of a voxel is its Chebyshev (max-norm) distance in voxels
  from the real domain, and ``mu_b = mu0 + (mu1 - mu0)(1 - cos(pi d/W))/2``.

Layout: moment fields are ``[a][z][y][x]`` with ``a = l*l + l + m``.
The oracle runs in the COMPLEX basis of eq. (3); inputs and outputs are
converted to and from the real basis (no Condon-Shortley phase) through a
unitary matrix computed by quadrature.

Everything here is float64 / complex128.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft
from scipy.special import sph_harm_y

WORKERS = os.cpu_count() or 1


# ----------------------------------------------------------- indexing ---

def sh_index(l: int, m: int) -> int:
    """Flat moment index of (l, m): ``l*l + l + m``."""
    return l * l + l + m


def sh_lm(a: int):
    """Inverse of :func:`sh_index`."""
    l = int(math.isqrt(a))
    return l, a - l * l - l


# ------------------------------------------------ eq. (6) coefficients ---

def alpha(l: int, m: int) -> float:
    """alpha_l^m = sqrt((l+m)(l-m)), eq. (6)."""
    v = (l + m) * (l - m)
    assert v >= 0, (l, m)
    return math.sqrt(v)


def beta(l: int, m: int) -> float:
    """beta_l^m = sqrt((l+m)(l+m-1)), eq. (6)."""
    v = (l + m) * (l + m - 1)
    assert v >= 0, (l, m)
    return math.sqrt(v)


def coupling_matrices(N: int):
    """Complex-basis streaming matrices ``(Bx, By, Bz)`` of eq. (6).

    Row ``(l, m)`` of ``B_j`` holds the coefficient of ``d/dj psi_{l'}^{m'}``
    in the streaming part of eq. (6), divided by ``2l+1``, so that the
    streaming term is ``sum_j B_j d/dj psi``. Terms that reach ``l' > N``
    are dropped (P_N closure, Sec. II.A); terms that reach ``|m'| > l'`` have
    zero coefficient and are skipped.
    """
    M = (N + 1) ** 2
    Bx = np.zeros((M, M), complex)
    By = np.zeros((M, M), complex)
    Bz = np.zeros((M, M), complex)

    def ok(l, m):
        return 0 <= l <= N and -l <= m <= l

    for l in range(N + 1):
        w = 1.0 / (2 * l + 1)
        for m in range(-l, l + 1):
            a = sh_index(l, m)
            # d/dz [ alpha_{l+1}^m psi_{l+1}^m + alpha_l^m psi_{l-1}^m ]
            if ok(l + 1, m):
                Bz[a, sh_index(l + 1, m)] += w * alpha(l + 1, m)
            if ok(l - 1, m):
                Bz[a, sh_index(l - 1, m)] += w * alpha(l, m)
            # -1/2 (d/dx - i d/dy) [ beta_l^m psi_{l-1}^{m-1}
            #                       - beta_{l+1}^{-m+1} psi_{l+1}^{m-1} ]
            terms = []
            if ok(l - 1, m - 1):
                terms.append((sh_index(l - 1, m - 1), -0.5 * beta(l, m), -1j))
            if ok(l + 1, m - 1):
                terms.append((sh_index(l + 1, m - 1),
                              0.5 * beta(l + 1, -m + 1), -1j))
            # -1/2 (d/dx + i d/dy) [ -beta_l^{-m} psi_{l-1}^{m+1}
            #                       + beta_{l+1}^{m+1} psi_{l+1}^{m+1} ]
            if ok(l - 1, m + 1):
                terms.append((sh_index(l - 1, m + 1), 0.5 * beta(l, -m), 1j))
            if ok(l + 1, m + 1):
                terms.append((sh_index(l + 1, m + 1),
                              -0.5 * beta(l + 1, m + 1), 1j))
            for b, coef, ycoef in terms:
                Bx[a, b] += w * coef
                By[a, b] += w * coef * ycoef
    return Bx, By, Bz


# ------------------------------------------------------- real basis -----

def _sphere_quadrature(L: int):
    """Nodes/weights exact for polynomials of degree <= L on the sphere:
    Gauss-Legendre in cos(theta) times the trapezoid rule in phi."""
    nt = L // 2 + 1
    nph = L + 1
    x, wx = np.polynomial.legendre.leggauss(nt)
    theta = np.arccos(x)
    phi = 2 * np.pi * np.arange(nph) / nph
    T, P = np.meshgrid(theta, phi, indexing="ij")
    Wt = np.outer(wx, np.full(nph, 2 * np.pi / nph))
    return T.ravel(), P.ravel(), Wt.ravel()


def complex_sh(N: int, theta, phi):
    """Rows ``Y_l^m(theta, phi)`` for all ``a``, Condon-Shortley phase."""
    M = (N + 1) ** 2
    Y = np.zeros((M, theta.size), complex)
    for l in range(N + 1):
        for m in range(-l, l + 1):
            Y[sh_index(l, m)] = sph_harm_y(l, m, theta, phi)
    return Y


def real_sh(N: int, theta, phi):
    """Real harmonics without Condon-Shortley phase:
    ``sqrt2 N P_l^m cos(m phi)`` (m>0), ``Y_l^0`` (m=0),
    ``sqrt2 N P_l^|m| sin(|m| phi)`` (m<0)."""
    M = (N + 1) ** 2
    Y = np.zeros((M, theta.size))
    for l in range(N + 1):
        for m in range(-l, l + 1):
            yc = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                Y[sh_index(l, m)] = math.sqrt(2) * (-1) ** m * yc.real
            elif m < 0:
                Y[sh_index(l, m)] = math.sqrt(2) * (-1) ** m * yc.imag
            else:
                Y[sh_index(l, m)] = yc.real
    return Y


def real_basis_transform(N: int) -> np.ndarray:
    """Unitary ``U`` with ``Y^R_a = sum_b U[a,b] Y_b``, by exact quadrature
    of ``<Y^R_a, Y_b>`` over the sphere."""
    T, P, Wq = _sphere_quadrature(2 * N + 2)
    YR = real_sh(N, T, P)
    Y = complex_sh(N, T, P)
    return (YR * Wq) @ Y.conj().T


def to_complex_basis(psi_real: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Complex-basis moments of a real-basis field: ``psi = U^T psi^R``
    (same weights, so the radiance is unchanged)."""
    return np.tensordot(U.T, psi_real, axes=(1, 0))


def to_real_basis(psi: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Real-basis moments ``conj(U) psi``; the imaginary part of a physical
    (real) radiance is zero up to rounding and is dropped."""
    return np.tensordot(U.conj(), psi, axes=(1, 0)).real


# --------------------------------------------------- grid and medium ----

def wavenumbers(n: int, dx: float) -> np.ndarray:
    """``k = 2 pi f / (n dx)`` in FFT order, Nyquist entry set to zero."""
    k = 2 * np.pi * np.fft.fftfreq(n, d=dx)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def pml_depth(n: int, W: int) -> np.ndarray:
    """Max-norm distance (voxels) of each voxel from the real domain
    ``[W, n-W)^3``; zero inside it."""
    i = np.arange(n)
    d1 = np.maximum(np.maximum(W - i, i - (n - 1 - W)), 0)
    return np.maximum(np.maximum(d1[:, None, None], d1[None, :, None]),
                      d1[None, None, :])


def pml_profile(n: int, W: int, mu0: float, mu1: float) -> np.ndarray:
    """Half-cosine layer attenuation ``mu_b`` (Sec. II.B, Sec. III.B): rises
    smoothly from ``mu0`` at the real-domain edge to ``mu1`` at depth ``W``.
    Zero where the depth is zero (inside the real domain)."""
    d = pml_depth(n, W).astype(float)
    if W == 0:
        return np.zeros_like(d)
    mub = mu0 + (mu1 - mu0) * 0.5 * (1.0 - np.cos(np.pi * d / W))
    return np.where(d > 0, mub, 0.0)


def potentials(mu_a, mu_s, g, N: int, W: int, mu0: float, mu1: float):
    """Per-degree loss ``Sigma_l(r)`` and real-domain mask (eqs. 6, 12).

    Inside the real domain ``Sigma_l = mu_t - mu_s g^l`` with
    ``mu_t = mu_a + mu_s``; in the layer ``Sigma_l = mu_b`` for every ``l``
    (no scattering there)."""
    n = mu_a.shape[0]
    d = pml_depth(n, W)
    omega = d == 0
    mub = pml_profile(n, W, mu0, mu1)
    Sig = np.empty((N + 1,) + mu_a.shape)
    for l in range(N + 1):
        inside = mu_a + mu_s - mu_s * g ** l
        Sig[l] = np.where(omega, inside, mub)
    return Sig, omega


# --------------------------------------------------------- operator -----

def _pairs(B):
    """Non-zero (a, b) entries of the three streaming matrices."""
    Bx, By, Bz = B
    nz = (np.abs(Bx) + np.abs(By) + np.abs(Bz)) > 0
    return [(a, b, Bx[a, b], By[a, b], Bz[a, b])
            for a, b in zip(*np.nonzero(nz))]


def operator(psi, Sig, q, B, k, c, workers=None):
    """Right-hand side ``d psi/dt`` of the semi-discrete system (eq. 9 with
    the sign reading above):
    ``c * (-IFFT[sum_j i k_j B_j FFT(psi)] - Sigma_l psi + q)``."""
    workers = workers or WORKERS
    M = psi.shape[0]
    N = int(math.isqrt(M)) - 1
    psih = sfft.fftn(psi, axes=(1, 2, 3), workers=workers)
    kz = k[:, None, None]
    ky = k[None, :, None]
    kx = k[None, None, :]
    shat = np.zeros_like(psih)
    for a, b, bx, by, bz in _pairs(B):
        shat[a] += 1j * (kx * bx + ky * by + kz * bz) * psih[b]
    del psih
    s = sfft.ifftn(shat, axes=(1, 2, 3), workers=workers)
    del shat
    out = np.empty_like(psi)
    for l in range(N + 1):
        for m in range(-l, l + 1):
            a = sh_index(l, m)
            out[a] = -s[a] - Sig[l] * psi[a]
            if q is not None:
                out[a] += q[a]
    out *= c
    return out


def rk4_step(psi, f, dt):
    """Classic four-stage Runge-Kutta step (Butcher tableau 1/2, 1/2, 1;
    weights 1/6, 1/3, 1/3, 1/6)."""
    k = f(psi)
    acc = k.copy()
    k = f(psi + (0.5 * dt) * k)
    acc += 2.0 * k
    k = f(psi + (0.5 * dt) * k)
    acc += 2.0 * k
    k = f(psi + dt * k)
    acc += k
    return psi + (dt / 6.0) * acc


def full_moments(a, M):
    """Inputs may give only the K <= M leading moments; pad with zeros."""
    if a is None:
        return None
    a = np.asarray(a, float)
    if a.shape[0] == M:
        return a
    out = np.zeros((M,) + a.shape[1:])
    out[:a.shape[0]] = a
    return out


def euler_step(psi, f, dt):
    """First-order explicit step of eq. (11) (with the sign reading of the
    right-hand side): ``psi + dt f(psi)``."""
    return psi + dt * f(psi)


def source_profile(samples, delta):
    """Temporal profile s(t) of a source ``q(r) s(t)`` (eq. 4 lets q depend
    on time): linear between ``samples[i]`` at ``t = i * delta`` (t from the
    start of the run), the last value after the last sample."""
    samples = np.asarray(samples, float)
    knots = delta * np.arange(samples.size)
    return lambda t: np.interp(t, knots, samples)


def source_moments(s_of_t, t0, h, knots):
    """``m_j = int_0^h (h - tau)^j / j! s(t0 + tau) dtau`` for j = 0..3, by
    adaptive quadrature (SciPy ``quad``) split at the profile's knots."""
    from scipy.integrate import quad
    pts = [k - t0 for k in knots if 0.0 < k - t0 < h]
    out = []
    for j in range(4):
        f = (lambda tau, j=j: (h - tau) ** j / math.factorial(j) * s_of_t(t0 + tau))
        val, _ = quad(f, 0.0, h, points=pts or None, epsabs=0.0, epsrel=1e-13, limit=200)
        out.append(val)
    return out


def rk4_source_step(psi, lin, cq, h, m):
    """One fourth-order step of ``d psi/dt = L psi + c q s(t)``: the
    variation-of-constants formula with ``exp(h L)`` truncated after
    ``(hL)^4 / 4!`` and the source integral after ``L^3``,
    ``sum_j (hL)^j psi / j! + sum_j L^j (c q) m_j``, m_j the source moments
    of the step. For constant s it is the classic RK4 step of an affine
    system."""
    out = psi.copy()
    term = psi
    for j in range(1, 5):
        term = (h / j) * lin(term)
        out = out + term
    v = cq
    for j in range(4):
        out = out + m[j] * v
        if j < 3:
            v = lin(v)
    return out


def solve(n, N, dx, c, dt, mu_a, mu_s, g, psi0_real, q_real, W, mu0, mu1,
          steps, det_index=(), workers=None, return_state=True, scheme="rk4",
          q_profile=None):
    """March ``steps`` RK4 steps from ``psi0_real`` (real-basis moments).

    ``q_profile = (samples, delta)`` makes the source ``q(r) s(t)`` with s
    from :func:`source_profile` (t = 0 at the start); RK4 then takes
    :func:`rk4_source_step` with the step's source moments and forward Euler
    uses ``s`` at the start of each step.

    Returns a dict with ``fluence`` (psi_0^0 after the last step),
    ``readings`` ``[steps][n_det]`` (psi_0^0 at the detector voxels after
    every step), ``phi_int`` (sum over steps of ``dt * psi_0^0``),
    ``residual`` ``[steps]`` (``||phi_n - phi_{n-1}|| / ||phi_n||``),
    ``peak`` ``[steps]`` (max |psi_0^0| over the grid after every step) and,
    if asked, ``state`` (real-basis moments after the last step)."""
    M = (N + 1) ** 2
    B = coupling_matrices(N)
    U = real_basis_transform(N)
    k = wavenumbers(n, dx)
    Sig, omega = potentials(mu_a, mu_s, g, N, W, mu0, mu1)
    psi0_real = full_moments(psi0_real, M)
    q_real = full_moments(q_real, M)
    if psi0_real is None:
        psi = np.zeros((M, n, n, n), complex)
    else:
        psi = to_complex_basis(psi0_real, U).astype(complex)
    q = None
    if q_real is not None:
        q = to_complex_basis(q_real, U) * omega[None]
    det = np.asarray(det_index, dtype=np.int64)
    readings = np.zeros((steps, det.size))
    residual = np.zeros(steps)
    peak = np.zeros(steps)
    phi_int = np.zeros((n, n, n))
    prev = psi[0].real.copy()

    def f(y):
        return operator(y, Sig, q, B, k, c, workers)

    stepper = euler_step if scheme == "euler" else rk4_step
    if q_profile is not None:
        s_of_t = source_profile(*q_profile)
        knots = q_profile[1] * np.arange(len(q_profile[0]))
        cq = c * q if q is not None else np.zeros_like(psi)

        def lin(y):
            return operator(y, Sig, None, B, k, c, workers)

        def stepper(y, _f, h, step=[0]):
            t0 = step[0] * h
            step[0] += 1
            if scheme == "euler":
                return y + h * (lin(y) + s_of_t(t0) * cq)
            return rk4_source_step(y, lin, cq, h, source_moments(s_of_t, t0, h, knots))
    for s in range(steps):
        psi = stepper(psi, f, dt)
        phi = psi[0].real
        readings[s] = phi.ravel()[det]
        peak[s] = np.abs(phi).max()
        phi_int += dt * phi
        nrm = np.linalg.norm(phi)
        residual[s] = np.linalg.norm(phi - prev) / nrm if nrm > 0 else 0.0
        prev = phi.copy()
    out = dict(fluence=psi[0].real.copy(), readings=readings,
               phi_int=phi_int, residual=residual, peak=peak)
    if return_state:
        out["state"] = to_real_basis(psi, U)
    return out


# ----------------------------------------- single-mode algebra (pins) ---

def mode_matrix(N: int, kvec, sig_l, c: float) -> np.ndarray:
    """Generator ``M(k) = -c (i k.B + diag(Sigma_l(a)))`` of one Fourier
    mode in a homogeneous medium (complex basis)."""
    Bx, By, Bz = coupling_matrices(N)
    kx, ky, kz = kvec
    M = (N + 1) ** 2
    D = np.array([sig_l[sh_lm(a)[0]] for a in range(M)], float)
    return -c * (1j * (kx * Bx + ky * By + kz * Bz) + np.diag(D))


def rk4_poly(Z: np.ndarray) -> np.ndarray:
    """Stability polynomial of classic RK4, ``I + Z + Z^2/2 + Z^3/6 + Z^4/24``."""
    I = np.eye(Z.shape[0], dtype=complex)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    return I + Z + Z2 / 2 + Z3 / 6 + Z3 @ Z / 24


# --------------------------------------------------- phase function -----

def hg_phase(mu, g):
    """Henyey-Greenstein phase function of eq. (2), ``mu = s.s'``."""
    return (1.0 - g * g) / (4 * np.pi * (1.0 + g * g - 2 * g * mu) ** 1.5)


def hg_legendre_moments(g: float, L: int, nodes: int = 400) -> np.ndarray:
    """``2 pi int p(mu) P_l(mu) dmu`` for l = 0..L by Gauss-Legendre
    quadrature (the diagonal scattering factor the addition theorem, eq. 5,
    puts on degree l)."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    p = hg_phase(x, g)
    out = np.zeros(L + 1)
    for l in range(L + 1):
        Pl = np.polynomial.legendre.Legendre.basis(l)(x)
        out[l] = 2 * np.pi * np.sum(w * p * Pl)
    return out


# ------------------------------------------- discrete adjoint (reverse) ---

def real_coupling(N: int):
    """Real-basis streaming matrices ``conj(U) B_j U^T`` (real up to
    rounding), from the eq. (6) matrices and the quadrature-built U."""
    U = real_basis_transform(N)
    return tuple((U.conj() @ B @ U.T).real for B in coupling_matrices(N))


def _spectral_derivative(f, k, axis):
    """d f / d x_axis of a real periodic field (axis 0 = z, 1 = y, 2 = x),
    via the FFT with the Nyquist wavenumber zero."""
    shape = [1, 1, 1]
    shape[axis] = k.size
    fh = sfft.fftn(f, axes=(axis,), workers=WORKERS)
    return sfft.ifftn(1j * k.reshape(shape) * fh, axes=(axis,), workers=WORKERS).real


def operator_transpose(y, Sig, BR, k, c):
    """Transpose (Euclidean, real basis) of the linear part of the operator:
    ``L = -c (sum_j B_j d_j + Sigma)``; with ``d_j^T = -d_j`` (periodic,
    skew spectral derivative) ``L^T y = -c (-sum_j B_j^T d_j y + Sigma y)``."""
    M = y.shape[0]
    N = int(math.isqrt(M)) - 1
    out = np.zeros_like(y)
    for j, axis in ((0, 2), (1, 1), (2, 0)):      # B_x acts along x (axis 2)
        BT = BR[j].T
        d = np.stack([_spectral_derivative(y[b], k, axis) for b in range(M)])
        out -= np.tensordot(BT, d, axes=(1, 0))
    for l in range(N + 1):
        for m in range(-l, l + 1):
            a = sh_index(l, m)
            out[a] += Sig[l] * y[a]
    return -c * out


def adjoint_gradient(n, N, dx, c, dt, mu_a, mu_s, g, psi0_real, q_real, W, mu0,
                     mu1, steps, det_index, dj_dr, scheme="rk4"):
    """Gradient of a loss J(readings) with respect to mu_a(r), mu_s(r) by the
    reverse mode of the classic RK4 scheme that :func:`solve` integrates.

    ``dj_dr[s, d]`` is dJ/d(reading of detector d after step s + 1). Forward
    states are produced by the complex-basis solver; the reverse sweep runs
    in the real basis with :func:`operator_transpose`. Returns
    ``(grad_mu_a, grad_mu_s)``, each ``(n, n, n)``, zero in the layer
    (there the loss is ``mu_b`` for every degree, eq. 12)."""
    M = (N + 1) ** 2
    B = coupling_matrices(N)
    BR = real_coupling(N)
    U = real_basis_transform(N)
    k = wavenumbers(n, dx)
    Sig, omega = potentials(mu_a, mu_s, g, N, W, mu0, mu1)
    psi0_real = full_moments(psi0_real, M)
    q_real = full_moments(q_real, M)
    q = None
    if q_real is not None:
        q = to_complex_basis(q_real, U) * omega[None]

    def f(y):
        return operator(y, Sig, q, B, k, c)

    psi = (to_complex_basis(psi0_real, U).astype(complex)
           if psi0_real is not None else np.zeros((M, n, n, n), complex))
    states = [psi]
    stepper = euler_step if scheme == "euler" else rk4_step
    for _ in range(steps):
        psi = stepper(psi, f, dt)
        states.append(psi)
    det = np.asarray(det_index, np.int64)
    lofa = np.array([sh_lm(a)[0] for a in range(M)])
    gsig = np.zeros((N + 1, n, n, n))

    def add_grad(kbar, y):
        # d f / d Sigma_l = -c y_a for the moments a of degree l
        prod = -c * kbar * y
        for l in range(N + 1):
            gsig[l] += prod[lofa == l].sum(axis=0)

    lam = np.zeros((M, n, n, n))

    def inject(s):
        flat = lam[0].reshape(-1)
        np.add.at(flat, det, dj_dr[s])

    inject(steps - 1)
    for s in range(steps - 1, -1, -1):
        u = states[s]
        if scheme == "euler":
            # u' = u + dt f(u): adjoint lam + dt L^T lam, gradient (dt lam, u)
            kb0 = dt * lam
            add_grad(kb0, to_real_basis(u, U))
            lam = lam + operator_transpose(kb0, Sig, BR, k, c)
            if s >= 1:
                inject(s - 1)
            continue
        k1 = f(u)
        k2 = f(u + 0.5 * dt * k1)
        k3 = f(u + 0.5 * dt * k2)
        ys = [to_real_basis(u, U), to_real_basis(u + 0.5 * dt * k1, U),
              to_real_basis(u + 0.5 * dt * k2, U), to_real_basis(u + dt * k3, U)]
        kb = [dt / 6 * lam, dt / 3 * lam, dt / 3 * lam, dt / 6 * lam]
        ub = lam.copy()
        # stage 4: y4 = u + dt k3
        yb = operator_transpose(kb[3], Sig, BR, k, c)
        add_grad(kb[3], ys[3])
        ub += yb
        kb[2] = kb[2] + dt * yb
        # stage 3: y3 = u + dt/2 k2
        yb = operator_transpose(kb[2], Sig, BR, k, c)
        add_grad(kb[2], ys[2])
        ub += yb
        kb[1] = kb[1] + 0.5 * dt * yb
        # stage 2: y2 = u + dt/2 k1
        yb = operator_transpose(kb[1], Sig, BR, k, c)
        add_grad(kb[1], ys[1])
        ub += yb
        kb[0] = kb[0] + 0.5 * dt * yb
        # stage 1: y1 = u
        yb = operator_transpose(kb[0], Sig, BR, k, c)
        add_grad(kb[0], ys[0])
        ub += yb
        lam = ub
        if s >= 1:
            inject(s - 1)
    gmua = gsig.sum(axis=0) * omega
    gmus = sum((1.0 - g ** l) * gsig[l] for l in range(N + 1)) * omega
    return gmua, gmus


# --------------------------------------------------------- steady state ---

def steady_state(n, N, dx, c, mu_a, mu_s, g, q_real, W, mu0, mu1, tol=1e-12,
                 workers=None):
    """Steady state of the semi-discrete system: the u with ``f(u) = 0``,
    i.e. ``(S + Sigma) u = q`` in the real basis (the time-marched solution
    approaches it; Sec. II.A). Solved with SciPy's GMRES on the oracle's
    operator (a library Krylov routine as the solver step); returns the
    real-basis state."""
    import scipy.sparse.linalg as spla
    M = (N + 1) ** 2
    B = coupling_matrices(N)
    U = real_basis_transform(N)
    k = wavenumbers(n, dx)
    Sig, omega = potentials(mu_a, mu_s, g, N, W, mu0, mu1)
    qR = full_moments(q_real, M) * omega[None]
    size = M * n ** 3

    def A(xflat):
        x = to_complex_basis(xflat.reshape(M, n, n, n), U).astype(complex)
        # f(x) = c (-(S + Sigma) x) for q = 0, so (S + Sigma) x = -f(x) / c
        fx = operator(x, Sig, None, B, k, c, workers)
        return (-to_real_basis(fx, U) / c).ravel()

    op = spla.LinearOperator((size, size), matvec=A, dtype=float)
    b = qR.ravel()
    x, info = spla.gmres(op, b, rtol=tol, atol=0.0, restart=60, maxiter=400)
    if info != 0:
        raise RuntimeError(f"oracle steady-state GMRES did not converge (info={info})")
    return x.reshape(M, n, n, n)


# ------------------------------------------ exponential propagation ------

def expo_advance(n, N, dx, c, mu_a, mu_s, g, psi0_real, q_real, T):
    """Advance the semi-discrete system by a time ``T`` exactly, in a
    homogeneous medium on the periodic grid (no boundary layer). Each Fourier
    mode obeys ``da/dt = M(k) a + c q(k)`` with the mode generator
    ``M(k) = -c (i k.B + Sigma)`` (integrating the time-domain form
    analytically, Sec. II.A; exponential integrators for homogeneous media,
    Sec. IV), so ``a(T) = exp(T M) a(0) + int_0^T exp(s M) ds c q``. Both
    terms are read off the matrix exponential (SciPy's ``expm``) of the
    augmented generator ``[[T M, T c q], [0, 0]]`` of each mode.

    ``mu_a``, ``mu_s``, ``g`` are scalars; ``psi0_real`` / ``q_real`` hold
    the leading real-basis moments (or None). Returns the real-basis state.
    """
    from scipy.linalg import expm
    M = (N + 1) ** 2
    B = coupling_matrices(N)
    U = real_basis_transform(N)
    k = wavenumbers(n, dx)
    sig = [mu_a + mu_s * (1.0 - g ** l) for l in range(N + 1)]
    p0 = full_moments(psi0_real, M)
    q0 = full_moments(q_real, M)
    a = (np.zeros((M, n, n, n), complex) if p0 is None
         else sfft.fftn(to_complex_basis(p0, U).astype(complex), axes=(1, 2, 3)))
    qh = (np.zeros((M, n, n, n), complex) if q0 is None
          else sfft.fftn(to_complex_basis(q0, U).astype(complex), axes=(1, 2, 3)))
    from threadpoolctl import threadpool_limits
    Bx, By, Bz = B
    D = np.diag([sig[sh_lm(i)[0]] for i in range(M)]).astype(complex)
    out = np.empty_like(a)
    G = np.zeros((M + 1, M + 1), complex)
    # small dense products: one BLAS thread is far faster than many
    with threadpool_limits(limits=1):
        for z in range(n):
            for y in range(n):
                for x in range(n):
                    # T M(k), M(k) = -c (i k.B + Sigma): the mode generator
                    G[:M, :M] = (-c * T) * (1j * (k[x] * Bx + k[y] * By + k[z] * Bz) + D)
                    G[:M, M] = (T * c) * qh[:, z, y, x]
                    E = expm(G)
                    out[:, z, y, x] = E[:M, :M] @ a[:, z, y, x] + E[:M, M]
    return to_real_basis(sfft.ifftn(out, axes=(1, 2, 3)), U)
