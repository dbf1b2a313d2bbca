// Host-side FP64 tables for the P_N stepper: streaming coefficients of
// eq. (6) rotated to the real harmonic basis, FFT twiddles, wavenumbers and
// the per-degree losses with the absorbing layer of eq. (12).
#include <algorithm>
#include <cmath>
#include <complex>

#include "rte_internal.h"

namespace rte {

namespace {

using cplx = std::complex<double>;

inline int idx(int l, int m) { return l * l + l + m; }

// alpha_l^m and beta_l^m of eq. (6).
inline double alpha_c(int l, int m) {
  const double v = double(l + m) * double(l - m);
  return v > 0 ? std::sqrt(v) : 0.0;
}
inline double beta_c(int l, int m) {
  const double v = double(l + m) * double(l + m - 1);
  return v > 0 ? std::sqrt(v) : 0.0;
}

inline bool valid(int N, int l, int m) { return l >= 0 && l <= N && m >= -l && m <= l; }

// Complex-basis streaming coefficients of eq. (6): the coefficient of
// d/dj psi_{l'}^{m'} in the equation for psi_l^m, divided by 2l+1.
void complex_streaming(int N, std::vector<cplx>& Bx, std::vector<cplx>& By,
                       std::vector<cplx>& Bz) {
  const int M = (N + 1) * (N + 1);
  Bx.assign(M * M, 0.0);
  By.assign(M * M, 0.0);
  Bz.assign(M * M, 0.0);
  for (int l = 0; l <= N; ++l) {
    const double w = 1.0 / (2 * l + 1);
    for (int m = -l; m <= l; ++m) {
      const int a = idx(l, m);
      // z-derivative: alpha terms couple (l, m) with (l +- 1, m).
      if (valid(N, l + 1, m)) Bz[a * M + idx(l + 1, m)] += w * alpha_c(l + 1, m);
      if (valid(N, l - 1, m)) Bz[a * M + idx(l - 1, m)] += w * alpha_c(l, m);
      // (d/dx - i d/dy) acting on order m-1, weight -1/2.
      struct Term { int l2, m2; double c; double ysign; };
      Term terms[4] = {
          {l - 1, m - 1, -0.5 * beta_c(l, m), -1.0},
          {l + 1, m - 1, +0.5 * beta_c(l + 1, -m + 1), -1.0},
          // (d/dx + i d/dy) acting on order m+1, weight -1/2.
          {l - 1, m + 1, +0.5 * beta_c(l, -m), +1.0},
          {l + 1, m + 1, -0.5 * beta_c(l + 1, m + 1), +1.0},
      };
      for (const Term& t : terms) {
        if (!valid(N, t.l2, t.m2)) continue;
        const int b = idx(t.l2, t.m2);
        Bx[a * M + b] += w * t.c;
        By[a * M + b] += w * t.c * cplx(0.0, t.ysign);
      }
    }
  }
}

// Unitary U with Y^R_a = sum_b U[a, b] Y_b (real harmonics without the
// Condon-Shortley phase in terms of the complex ones with it):
//   m > 0: Y^R_{l,m}  = ((-1)^m Y_l^m + Y_l^{-m}) / sqrt2
//   m < 0: Y^R_{l,-u} = ((-1)^u Y_l^u - Y_l^{-u}) / (i sqrt2),  u = -m
//   m = 0: Y^R_{l,0}  = Y_l^0
void real_from_complex(int N, std::vector<cplx>& U) {
  const int M = (N + 1) * (N + 1);
  U.assign(M * M, 0.0);
  const double r2 = 1.0 / std::sqrt(2.0);
  for (int l = 0; l <= N; ++l) {
    U[idx(l, 0) * M + idx(l, 0)] = 1.0;
    for (int u = 1; u <= l; ++u) {
      const double sg = (u % 2) ? -1.0 : 1.0;
      const int ap = idx(l, u), am = idx(l, -u);
      U[ap * M + ap] = sg * r2;
      U[ap * M + am] = r2;
      U[am * M + ap] = cplx(0.0, -sg * r2);   // sg / (i sqrt2)
      U[am * M + am] = cplx(0.0, r2);         // -1 / (i sqrt2)
    }
  }
}

}  // namespace

bool coupling_dense(int N, std::vector<double>& bx, std::vector<double>& by,
                    std::vector<double>& bz) {
  if (!order_built(N, 0)) return false;
  const int M = (N + 1) * (N + 1);
  std::vector<cplx> B[3];
  complex_streaming(N, B[0], B[1], B[2]);
  std::vector<cplx> U;
  real_from_complex(N, U);
  // non-zeros of each row of U (at most two: the orders +-|m| of degree l)
  std::vector<std::vector<int>> unz(M);
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b)
      if (U[a * M + b] != 0.0) unz[a].push_back(b);
  // Moments transform as psi^R = conj(U) psi, psi = U^T psi^R, so the
  // real-basis matrix is conj(U) B U^T (products over the non-zeros of U).
  std::vector<double>* out[3] = {&bx, &by, &bz};
  for (int j = 0; j < 3; ++j) {
    std::vector<cplx> T(size_t(M) * M, 0.0);
    for (int a = 0; a < M; ++a)
      for (int c = 0; c < M; ++c) {
        cplx s = 0.0;
        for (int b : unz[a]) s += std::conj(U[a * M + b]) * B[j][size_t(b) * M + c];
        T[size_t(a) * M + c] = s;
      }
    out[j]->assign(size_t(M) * M, 0.0);
    for (int a = 0; a < M; ++a)
      for (int d = 0; d < M; ++d) {
        cplx s = 0.0;
        for (int c : unz[d]) s += T[size_t(a) * M + c] * U[d * M + c];
        if (std::abs(s.imag()) > 1e-13) return false;   // must be real
        (*out[j])[size_t(a) * M + d] = std::abs(s.real()) < 1e-15 ? 0.0 : s.real();
      }
  }
  // Every non-zero must sit in a slot of its row.
  for (int l = 0; l <= N; ++l)
    for (int m = -l; m <= l; ++m) {
      const int a = idx(l, m);
      const SlotList sl = slots_of(N, l, m);
      for (int b = 0; b < M; ++b) {
        const bool nz = bx[a * M + b] != 0.0 || by[a * M + b] != 0.0 || bz[a * M + b] != 0.0;
        bool in = false;
        for (int s = 0; s < sl.count; ++s) in = in || (sl.b[s] == b);
        if (nz && !in) return false;
      }
    }
  return true;
}

namespace {
// Real harmonic Y^R_{l,m}(theta, phi) of the basis above (no Condon-Shortley
// phase, orthonormal on the sphere): N_lm P_l^|m|(cos theta) times
// sqrt2 cos(m phi) (m > 0), 1 (m = 0) or sqrt2 sin(|m| phi) (m < 0).
double real_sh(int l, int m, double ct, double phi) {
  const int am = m < 0 ? -m : m;
  // P_am^am = (2 am - 1)!! (1 - x^2)^(am/2), then upward in l
  const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  double pmm = 1.0;
  for (int i = 1; i <= am; ++i) pmm *= double(2 * i - 1) * st;
  double p = pmm;
  if (l > am) {
    double pm1 = ct * double(2 * am + 1) * pmm;
    double pm0 = pmm;
    for (int ll = am + 2; ll <= l; ++ll) {
      const double pn = (double(2 * ll - 1) * ct * pm1 - double(ll + am - 1) * pm0) / double(ll - am);
      pm0 = pm1;
      pm1 = pn;
    }
    p = pm1;
  }
  double ratio = 1.0;   // (l - am)! / (l + am)!
  for (int i = l - am + 1; i <= l + am; ++i) ratio /= double(i);
  const double nlm = std::sqrt(double(2 * l + 1) / (4.0 * M_PI) * ratio);
  if (m > 0) return std::sqrt(2.0) * nlm * p * std::cos(m * phi);
  if (m < 0) return std::sqrt(2.0) * nlm * p * std::sin(am * phi);
  return nlm * p;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
}
}  // namespace

bool rotation_x90(int N, std::vector<double>& D) {
  if (N < 0 || N > kDenseOrder) return false;
  // D_ab = int Y_a(s) Y_b(X^-1 s) ds for X the rotation by +90 degrees
  // about x (y -> z, z -> -y), so X^-1 s = (s_x, s_z, -s_y); block per
  // degree, exact quadrature (degree <= 2N in cos theta and in phi)
  std::vector<double> gx, gw;
  const int q = N + 2, P = 2 * N + 2;
  gauss_legendre(q, gx, gw);
  size_t off = 0;
  D.clear();
  for (int l = 0; l <= N; ++l) {
    const int d = 2 * l + 1;
    std::vector<double> blk(size_t(d) * d, 0.0);
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < P; ++j) {
        const double ct = gx[i], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        const double phi = 2.0 * M_PI * (j + 0.5) / P;
        const double wq = gw[i] * 2.0 * M_PI / P;
        const double sx = st * std::cos(phi), sy = st * std::sin(phi), sz = ct;
        // X^-1 s
        const double rx = sx, ry = sz, rz = -sy;
        const double rct = rz, rphi = std::atan2(ry, rx);
        for (int ma = -l; ma <= l; ++ma) {
          const double ya = real_sh(l, ma, ct, phi) * wq;
          for (int mb = -l; mb <= l; ++mb) blk[size_t(ma + l) * d + (mb + l)] += ya * real_sh(l, mb, rct, rphi);
        }
      }
    for (int a = 0; a < d * d; ++a) D.push_back(std::fabs(blk[a]) < 1e-15 ? 0.0 : blk[a]);
    off += size_t(d) * d;
  }
  // self-check of the representation against the streaming matrices:
  // D (k.B) D^T = (X k).B for k = x, y, z
  std::vector<double> b[3];
  if (!coupling_dense(N, b[0], b[1], b[2])) return false;
  const int M = (N + 1) * (N + 1);
  std::vector<double> Dd(size_t(M) * M, 0.0);
  size_t o = 0;
  for (int l = 0; l <= N; ++l) {
    const int d = 2 * l + 1, a0 = l * l;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) Dd[size_t(a0 + i) * M + a0 + j] = D[o + size_t(i) * d + j];
    o += size_t(d) * d;
  }
  // X e_x = e_x, X e_y = e_z, X e_z = -e_y
  const double Xc[3][3] = {{1, 0, 0}, {0, 0, -1}, {0, 1, 0}};   // columns are X e_j
  for (int jx = 0; jx < 3; ++jx) {
    for (int a = 0; a < M; ++a)
      for (int c = 0; c < M; ++c) {
        double lhs = 0.0;
        for (int p = 0; p < M; ++p) {
          const double dap = Dd[size_t(a) * M + p];
          if (dap == 0.0) continue;
          for (int r = 0; r < M; ++r) lhs += dap * b[jx][size_t(p) * M + r] * Dd[size_t(c) * M + r];
        }
        double rhs = 0.0;
        for (int i = 0; i < 3; ++i) rhs += Xc[i][jx] * b[i][size_t(a) * M + c];
        if (std::fabs(lhs - rhs) > 1e-11) return false;
      }
  }
  return true;
}

bool coupling_table(int N, std::vector<int>& code, std::vector<double>& val) {
  std::vector<double> b[3];
  if (!coupling_dense(N, b[0], b[1], b[2])) return false;
  const int M = (N + 1) * (N + 1);
  code.assign(size_t(M) * kMaxSlots, -1);
  val.assign(size_t(M) * kMaxSlots, 0.0);
  for (int l = 0; l <= N; ++l)
    for (int m = -l; m <= l; ++m) {
      const int a = idx(l, m);
      const SlotList sl = slots_of(N, l, m);
      int k = 0;
      for (int s = 0; s < sl.count; ++s)
        for (int ax = 0; ax < 3; ++ax) {
          const double v = b[ax][size_t(a) * M + sl.b[s]];
          if (v == 0.0) continue;
          if (k == kMaxSlots) return false;
          code[size_t(a) * kMaxSlots + k] = (sl.b[s] << 2) | ax;
          val[size_t(a) * kMaxSlots + k] = v;
          ++k;
        }
    }
  return true;
}

void twiddles(int n, std::vector<double>& tw) {
  tw.assign(2 * size_t(n), 0.0);
  for (int t = 0; t < n; ++t) {
    // Reduce the angle to the first octant so cos/sin are evaluated on
    // |x| <= pi/4 and symmetric entries are exactly symmetric.
    const long long p = 8LL * t;             // angle = 2 pi t / n = (pi/4) p / n
    long long oct = p / n;                   // octant 0..7
    const long long rem = p - oct * n;       // angle within octant, (pi/4) rem/n
    double c, s;
    const double th = (M_PI / 4.0) * double(rem) / double(n);
    const double ct = std::cos(th), st = std::sin(th);
    const double ctc = std::cos(M_PI / 4.0 - th), stc = std::sin(M_PI / 4.0 - th);
    switch (oct) {
      case 0: c = ct;   s = st;   break;
      case 1: c = stc;  s = ctc;  break;
      case 2: c = -st;  s = ct;   break;
      case 3: c = -ctc; s = stc;  break;
      case 4: c = -ct;  s = -st;  break;
      case 5: c = -stc; s = -ctc; break;
      case 6: c = st;   s = -ct;  break;
      default: c = ctc; s = -stc; break;
    }
    tw[2 * t] = c;          // exp(-i angle) = cos - i sin
    tw[2 * t + 1] = -s;
  }
}

void wavenumbers(int n, double dx, std::vector<double>& k) {
  k.assign(n, 0.0);
  for (int f = 0; f < n; ++f) {
    int ff = f <= (n - 1) / 2 ? f : f - n;
    if (2 * f == n) ff = 0;                   // Nyquist -> 0
    k[f] = 2.0 * M_PI * double(ff) / (double(n) * dx);
  }
}

void potentials(int n, int N, int W, double mu0, double mu1,
                const double* mu_a, const double* mu_s, const double* g,
                std::vector<double>& sig, std::vector<uint8_t>& inside) {
  const size_t V = size_t(n) * n * n;
  sig.assign(size_t(N + 1) * V, 0.0);
  inside.assign(V, 0);
  auto depth1 = [&](int i) {
    int d = 0;
    if (W - i > d) d = W - i;
    if (i - (n - 1 - W) > d) d = i - (n - 1 - W);
    return d;
  };
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const size_t v = (size_t(z) * n + y) * n + x;
        int d = depth1(x);
        d = depth1(y) > d ? depth1(y) : d;
        d = depth1(z) > d ? depth1(z) : d;
        if (d == 0) {
          inside[v] = 1;
          double gl = 1.0;
          for (int l = 0; l <= N; ++l) {
            sig[size_t(l) * V + v] = mu_a[v] + mu_s[v] * (1.0 - gl);
            gl *= g[v];
          }
        } else {
          const double mub = mu0 + (mu1 - mu0) * 0.5 * (1.0 - std::cos(M_PI * double(d) / double(W)));
          for (int l = 0; l <= N; ++l) sig[size_t(l) * V + v] = mub;
        }
      }
}

bool grid_supported(int n) {
  switch (n) {
    case 16: case 32: case 48: case 64: case 96: case 128: case 256: return true;
    default: return false;
  }
}

}  // namespace rte
