// Compile-time streaming coefficients of eq. (6) in the real harmonic basis.
//
// Same definitions as the host tables (rte_tables.cpp): the complex-basis
// coefficient of d/dj psi_{l'}^{m'} in the equation for psi_l^m, divided by
// 2l+1, rotated to real harmonics without the Condon-Shortley phase by
// B^R = conj(U) B U^T. Here every entry is a constant expression, so kernels
// that apply the coupling many times per point (the exact propagation) carry
// the values as instruction constants instead of loading them.
#pragma once

#include "rte_internal.h"

namespace rte {
namespace ct {

struct Cx {
  double re, im;
};
constexpr Cx cx_add(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
constexpr Cx cx_mul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
constexpr Cx cx_conj(Cx a) { return {a.re, -a.im}; }

// Square root by Newton's iteration (exact to rounding for the small
// integer arguments used here).
constexpr double sqrt_ct(double x) {
  if (x <= 0) return 0.0;
  double r = x > 1 ? x : 1.0;
  for (int i = 0; i < 200; ++i) {
    const double nr = 0.5 * (r + x / r);
    if (nr == r) break;
    r = nr;
  }
  return r;
}

constexpr double alpha_ct(int l, int m) {
  const double v = double(l + m) * double(l - m);
  return v > 0 ? sqrt_ct(v) : 0.0;
}
constexpr double beta_ct(int l, int m) {
  const double v = double(l + m) * double(l + m - 1);
  return v > 0 ? sqrt_ct(v) : 0.0;
}
constexpr bool valid_ct(int N, int l, int m) { return l >= 0 && l <= N && m >= -l && m <= l; }

// Complex-basis coefficient (axis 0 = x, 1 = y, 2 = z) of psi_{l2}^{m2} in
// the equation for psi_l^m.
constexpr Cx complex_coef(int N, int axis, int l, int m, int l2, int m2) {
  if (!valid_ct(N, l, m) || !valid_ct(N, l2, m2)) return {0.0, 0.0};
  const double w = 1.0 / (2 * l + 1);
  if (axis == 2) {
    double v = 0.0;
    if (l2 == l + 1 && m2 == m) v += w * alpha_ct(l + 1, m);
    if (l2 == l - 1 && m2 == m) v += w * alpha_ct(l, m);
    return {v, 0.0};
  }
  // (d/dx -+ i d/dy) terms acting on orders m -+ 1 (weight -1/2 each)
  double c = 0.0, ys = 0.0;
  if (l2 == l - 1 && m2 == m - 1) { c += -0.5 * beta_ct(l, m); ys = -1.0; }
  if (l2 == l + 1 && m2 == m - 1) { c += 0.5 * beta_ct(l + 1, -m + 1); ys = -1.0; }
  if (l2 == l - 1 && m2 == m + 1) { c += 0.5 * beta_ct(l, -m); ys = 1.0; }
  if (l2 == l + 1 && m2 == m + 1) { c += -0.5 * beta_ct(l + 1, m + 1); ys = 1.0; }
  if (axis == 0) return {w * c, 0.0};
  return {0.0, w * c * ys};
}

// Row of U (Y^R_a = sum_b U[a, b] Y_b) for real index (l, m): up to two
// complex orders with their coefficients.
struct URow {
  int count;
  int m[2];
  Cx c[2];
};
constexpr URow urow(int l, int m) {
  constexpr double r2 = 0.70710678118654752440;   // 1 / sqrt 2
  URow r{0, {0, 0}, {{0, 0}, {0, 0}}};
  if (m == 0) {
    r.count = 1;
    r.m[0] = 0;
    r.c[0] = {1.0, 0.0};
    return r;
  }
  const int u = m > 0 ? m : -m;
  const double sg = (u % 2) ? -1.0 : 1.0;
  r.count = 2;
  r.m[0] = u;
  r.m[1] = -u;
  if (m > 0) {
    r.c[0] = {sg * r2, 0.0};
    r.c[1] = {r2, 0.0};
  } else {
    r.c[0] = {0.0, -sg * r2};
    r.c[1] = {0.0, r2};
  }
  return r;
}

// Real-basis coefficient B^R_axis[a][d], a = (l, m), d = (l2, m2).
constexpr double real_coef(int N, int axis, int a, int d) {
  const int l = isqrt_c(a), m = a - l * l - l;
  const int l2 = isqrt_c(d), m2 = d - l2 * l2 - l2;
  const URow ra = urow(l, m), rd = urow(l2, m2);
  Cx s{0.0, 0.0};
  for (int i = 0; i < ra.count; ++i)
    for (int j = 0; j < rd.count; ++j)
      s = cx_add(s, cx_mul(cx_mul(cx_conj(ra.c[i]), complex_coef(N, axis, l, ra.m[i], l2, rd.m[j])), rd.c[j]));
  return s.re;
}

}  // namespace ct
}  // namespace rte
