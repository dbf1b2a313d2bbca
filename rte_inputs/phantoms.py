"""Seeded phantoms, initial conditions, sources and detectors.

Every generator is deterministic given its arguments (NumPy PCG64 through
``numpy.random.default_rng(seed)``). Units: mm, ps, mm^-1.

Grid convention: voxel ``(z, y, x)`` sits at ``r = (x, y, z) * dx``; the
real domain is the cube of voxel indices ``[W, n - W)`` on every axis and the
``W`` outer voxel layers form the absorbing boundary layer.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


def _moments(N: int) -> int:
    return (N + 1) * (N + 1)


# ---------------------------------------------------------------- maps ---

def homogeneous_maps(n: int, mu_a: float, mu_s: float, g: float):
    """Constant optical maps ``(mu_a, mu_s, g)``, each ``(n, n, n)`` float64."""
    shape = (n, n, n)
    return (np.full(shape, float(mu_a)), np.full(shape, float(mu_s)),
            np.full(shape, float(g)))


def sphere_maps(n: int, W: int, count: int, seed: int,
                radius: tuple = (4, 16),
                background: tuple = (0.01, 10.0, 0.9),
                mu_a_range: tuple = (0.005, 0.1),
                mu_s_range: tuple = (5.0, 20.0),
                g_range: tuple = (0.8, 0.95)):
    """Background medium with ``count`` spherical inclusions.

    Radii are integers drawn uniformly from ``radius`` (inclusive, voxels)
    and clipped so a sphere fits in the real domain; each centre is uniform
    among positions that keep the whole sphere inside ``[W, n-W)``. Later
    spheres overwrite earlier ones. A voxel belongs to a sphere when its
    squared index distance to the centre is ``<= r*r``.
    """
    rng = np.random.default_rng(seed)
    mu_a, mu_s, g = homogeneous_maps(n, *background)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                          indexing="ij")
    inner = n - 2 * W
    for _ in range(count):
        r = int(rng.integers(radius[0], radius[1] + 1))
        r = max(0, min(r, (inner - 1) // 2))
        lo, hi = W + r, n - W - 1 - r
        cz, cy, cx = (int(rng.integers(lo, hi + 1)) for _ in range(3))
        a = rng.uniform(*mu_a_range)
        s = rng.uniform(*mu_s_range)
        gg = rng.uniform(*g_range)
        inside = (z - cz) ** 2 + (y - cy) ** 2 + (x - cx) ** 2 <= r * r
        mu_a[inside] = a
        mu_s[inside] = s
        g[inside] = gg
    return mu_a, mu_s, g


def _gaussian_random_field(n: int, corr: float, seed: int) -> np.ndarray:
    """Zero-mean unit-variance periodic Gaussian random field.

    White noise is smoothed by a Gaussian kernel of standard deviation
    ``corr / sqrt(2)`` voxels, so that the field's autocorrelation is a
    Gaussian of standard deviation ``corr`` voxels; it is then rescaled to
    unit sample variance.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n))
    f = np.fft.fftfreq(n)
    s = corr / np.sqrt(2.0)
    kern = np.exp(-2.0 * (np.pi * s) ** 2 * (f[:, None, None] ** 2 +
                                             f[None, :, None] ** 2 +
                                             f[None, None, :] ** 2))
    field_ = np.fft.ifftn(np.fft.fftn(noise) * kern).real
    field_ -= field_.mean()
    field_ /= field_.std()
    return field_


def lognormal_maps(n: int, seeds=(3, 13), corr: float = 20.0,
                   mean_mu_a: float = 0.01, mean_mu_s: float = 10.0,
                   sigma: float = 0.5, g: float = 0.85):
    """Log-normal ``mu_a`` and ``mu_s`` (mean-preserving), constant ``g``."""
    ga = _gaussian_random_field(n, corr, seeds[0])
    gs = _gaussian_random_field(n, corr, seeds[1])
    mu_a = mean_mu_a * np.exp(sigma * ga - 0.5 * sigma * sigma)
    mu_s = mean_mu_s * np.exp(sigma * gs - 0.5 * sigma * sigma)
    return mu_a, mu_s, np.full((n, n, n), float(g))


# ------------------------------------------------- initial conditions ---

def gaussian_ic(n: int, N: int, center=None, sigma: float = 1.0):
    """Isotropic Gaussian pulse: only the ``a = 0`` moment is non-zero,
    ``exp(-|i - c|^2 / (2 sigma^2))`` in voxel units."""
    if center is None:
        center = (n // 2, n // 2, n // 2)
    cz, cy, cx = center
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                          indexing="ij")
    psi = np.zeros((_moments(N), n, n, n))
    psi[0] = np.exp(-((z - cz) ** 2 + (y - cy) ** 2 + (x - cx) ** 2)
                    / (2.0 * sigma * sigma))
    return psi


def delta_ic(n: int, N: int, center=None):
    """Isotropic point pulse: ``a = 0`` moment is 1 at one voxel."""
    if center is None:
        center = (n // 2, n // 2, n // 2)
    psi = np.zeros((_moments(N), n, n, n))
    psi[(0,) + tuple(center)] = 1.0
    return psi


def fourier_mode_ic(n: int, N: int, freq, vec):
    """Real single-Fourier-mode state ``Re(exp(i k.r) vec[a])``.

    ``freq = (fx, fy, fz)`` are integer frequencies (k_j = 2 pi f_j / (n dx));
    ``vec`` is a complex vector of length ``(N+1)**2`` in the real basis.
    """
    fx, fy, fz = freq
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                          indexing="ij")
    ph = np.exp(2j * np.pi * (fx * x + fy * y + fz * z) / n)
    vec = np.asarray(vec, dtype=complex)
    return np.real(vec[:, None, None, None] * ph[None])


# -------------------------------------------------------------- source ---

def collimated_slab_source(n: int, N: int, W: int):
    """Time-constant source directed along +z on the real-domain voxels of
    the slab ``z = W``: ``q_{l,0} = 1`` for every ``l <= N`` (the truncated
    expansion of a +z delta in angle), all other moments zero."""
    q = np.zeros((_moments(N), n, n, n))
    for l in range(N + 1):
        q[l * l + l, W, W:n - W, W:n - W] = 1.0
    return q


# ----------------------------------------------------------- detectors ---

def outer_layer_detectors(n: int, W: int, count: int, seed: int):
    """Distinct voxels on the outermost layer of the real domain.

    A voxel qualifies when all its indices are in ``[W, n-W)`` and at least
    one index equals ``W`` or ``n-1-W``. Returned as sorted linear indices.
    """
    i = np.arange(n)
    inside = (i >= W) & (i < n - W)
    edge = (i == W) | (i == n - 1 - W)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    ok = inside[z] & inside[y] & inside[x] & (edge[z] | edge[y] | edge[x])
    cand = np.flatnonzero(ok.ravel())
    rng = np.random.default_rng(seed)
    pick = rng.choice(cand, size=min(count, cand.size), replace=False)
    return np.sort(pick).astype(np.int64)


# ----------------------------------------------------------- workloads ---

@dataclass
class Workload:
    """One solve: grid, order, medium, initial state, source, detectors.

    ``psi0`` / ``q`` hold the leading K <= (N+1)^2 real-basis moments
    (shape (K, n, n, n)); the remaining moments are zero."""
    name: str
    n: int
    N: int
    precision: str            # "f64" | "f32"
    dx: float                 # mm
    c: float                  # mm/ps
    dt: float                 # ps
    W: int                    # boundary-layer width, voxels
    mu0: float                # layer attenuation at the real-domain edge
    mu1: float                # layer attenuation at the grid edge
    steps: int
    mu_a: np.ndarray
    mu_s: np.ndarray
    g: np.ndarray
    psi0: Optional[np.ndarray]
    q: Optional[np.ndarray]
    det_index: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    steady_tol: float = 0.0
    scheme: str = "rk4"       # "rk4" | "euler"

    @property
    def M(self) -> int:
        return _moments(self.N)


def _dt(dx, c, courant=0.2):
    return courant * dx / c


def workload(name: str, n: Optional[int] = None, steps: Optional[int] = None,
             precision: Optional[str] = None) -> Workload:
    """Build a named workload; ``n``/``steps``/``precision`` override the
    full-size values (the boundary layer scales as ``n/8``, the inclusion
    radii with ``n``)."""
    c = 0.3
    if name == "p1_gauss":          # P_1, 32^3, FP64, homogeneous, 100 steps
        n = n or 32
        dx = 0.5 * 32 / n
        W = n // 4
        mu_a, mu_s, g = homogeneous_maps(n, 0.01, 10.0, 0.9)
        return Workload(name, n, 1, precision or "f64", dx, c, _dt(dx, c), W,
                        0.01, 1.0, steps if steps is not None else 100,
                        mu_a, mu_s, g, gaussian_ic(n, 0), None)
    if name == "p7_spheres":        # P_7, 128^3, FP32, 5 inclusions, 2000 steps
        n = n or 128
        dx = 0.25
        W = n // 8
        s = n / 128.0
        r = (max(1, int(round(4 * s))), max(1, int(round(16 * s))))
        mu_a, mu_s, g = sphere_maps(n, W, 5, seed=2, radius=r)
        det = outer_layer_detectors(n, W, 32, seed=2)
        return Workload(name, n, 7, precision or "f32", dx, c, _dt(dx, c), W,
                        0.01, 1.0, steps if steps is not None else 2000,
                        mu_a, mu_s, g, delta_ic(n, 0), None, det)
    if name == "p5_steady":         # P_5, 256^3, FP32, log-normal, steady state
        n = n or 256
        dx = 0.25
        W = n // 8
        corr = 20.0 * n / 256.0
        mu_a, mu_s, g = lognormal_maps(n, corr=corr)
        return Workload(name, n, 5, precision or "f32", dx, c, _dt(dx, c), W,
                        0.01, 1.0, steps if steps is not None else 20000,
                        mu_a, mu_s, g, None, collimated_slab_source(n, 5, W),
                        np.zeros(0, np.int64), steady_tol=1e-6)
    if name == "p3_adjoint":        # P_3, 96^3, FP32, inclusions, 1000 steps
        n = n or 96
        dx = 0.25
        W = n // 8
        s = n / 96.0
        r = (max(1, int(round(3 * s))), max(1, int(round(12 * s))))
        mu_a, mu_s, g = sphere_maps(n, W, 5, seed=5, radius=r)
        det = outer_layer_detectors(n, W, 16, seed=5)
        return Workload(name, n, 3, precision or "f32", dx, c, _dt(dx, c), W,
                        0.01, 1.0, steps if steps is not None else 1000,
                        mu_a, mu_s, g, gaussian_ic(n, 0), None, det)
    if name == "paper_pml_steady":  # P_7, 64^3, 50 mm cube, half-cosine layer, Euler
        # steady state with an absorbing layer as in the paper's second
        # experiment: a 35.5 mm real domain inside a 50 mm grid, mu_a 0.01,
        # mu_s 10, g 0.95, constant isotropic Gaussian source (1/e diameter
        # 1.5 mm) offset 8 mm along x, forward Euler with dt 0.04 ps
        n = n or 64
        L = 50.0
        dx = L / n
        W = int(round((L - 35.5) / 2 / dx))
        mu_a, mu_s, g = homogeneous_maps(n, 0.01, 10.0, 0.95)
        sigma = 0.75 / np.sqrt(2.0) / dx            # exp(-r^2/(2 s^2)) = 1/e at r = 0.75 mm
        centre = (n // 2, n // 2, n // 2 + int(round(8.0 / dx)))
        q = gaussian_ic(n, 0, center=centre, sigma=sigma)
        return Workload(name, n, 7, precision or "f32", dx, c, 0.04, W, 0.01, 1.0,
                        steps if steps is not None else 25000, mu_a, mu_s, g, None, q,
                        np.zeros(0, np.int64), scheme="euler")
    if name == "paper_transient":  # P_21, 64^3, 50 mm cube, two regions, no layer, Euler
        # transient without absorbing layer as in the paper's first
        # experiment: 50 mm grid, mu_a 0.01, g 0.9, mu_s 1.0 except 5.0 in
        # the slab x <= 15 mm (x measured from the low-x face), isotropic
        # Gaussian initial fluence (1/e diameter 1.5 mm) at the centre,
        # forward Euler with dt 0.1 ps, 400 steps; fluence read along the
        # x axis through the centre
        n = n or 64
        L = 50.0
        dx = L / n
        mu_a, mu_s, g = homogeneous_maps(n, 0.01, 1.0, 0.9)
        xs = np.arange(n) * dx
        mu_s[:, :, xs <= 15.0] = 5.0
        sigma = 0.75 / np.sqrt(2.0) / dx
        psi0 = gaussian_ic(n, 0, sigma=sigma)
        c0 = n // 2
        det = np.array([(c0 * n + c0) * n + x for x in range(0, n, max(1, n // 16))], np.int64)
        return Workload(name, n, 21, precision or "f32", dx, c, 0.1, 0, 0.01, 1.0,
                        steps if steps is not None else 400, mu_a, mu_s, g, psi0, None, det,
                        scheme="euler")
    raise KeyError(name)


WORKLOADS = ("p1_gauss", "p7_spheres", "p5_steady", "p3_adjoint", "paper_pml_steady",
             "paper_transient")


# ------------------------------------------------------------- serving ---

@dataclass
class RequestSpec:
    """One solve request of the serving trace (inputs built on demand)."""
    rid: int
    n: int
    N: int
    steps: int
    nspheres: int             # 0: homogeneous background
    seed: int
    gap: float                # unit-mean exponential inter-arrival gap

    def workload(self, precision: str = "f32") -> Workload:
        n = self.n
        W = n // 8
        dx, c = 0.25, 0.3
        if self.nspheres == 0:
            mu_a, mu_s, g = homogeneous_maps(n, 0.01, 10.0, 0.9)
        else:
            r = (max(1, n // 32), max(1, n // 8))
            mu_a, mu_s, g = sphere_maps(n, W, self.nspheres, self.seed, radius=r)
        psi0 = gaussian_ic(n, 0)        # only the isotropic moment is non-zero
        return Workload(f"req{self.rid}", n, self.N, precision, dx, c, _dt(dx, c), W, 0.01,
                        1.0, self.steps, mu_a, mu_s, g, psi0, None)


def serving_requests(count: int = 256, seed: int = 4, sizes=(32, 48, 64, 96, 128),
                     orders=(1, 3, 5, 7), steps=(200, 1000)):
    """Seeded request trace: grid uniform in ``sizes``, P_N order uniform in
    ``orders``, step count uniform in ``steps`` (inclusive), half
    homogeneous and half with 1-5 spherical inclusions, Poisson arrivals
    (unit-mean exponential gaps, scaled by the server to the wanted rate)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        N = int(rng.choice(orders))
        st = int(rng.integers(steps[0], steps[1] + 1))
        ns = 0 if rng.random() < 0.5 else int(rng.integers(1, 6))
        out.append(RequestSpec(i, n, N, st, ns, int(rng.integers(1 << 30)),
                               float(rng.exponential(1.0))))
    return out
