// Device building blocks for the P_N stepper on gfx950: complex helpers,
// radix-2/3/4/8 butterflies and a Stockham auto-sort FFT of compile-time
// length executed by a group of P lanes of one wavefront on data staged in
// LDS.
//
// An FFT of length L is owned by P = L / E lanes of ONE 64-lane wavefront;
// each lane holds E elements in registers per stage (E = 8 for powers of
// two, 24 when L has a factor 3). Every stage only exchanges data among
// lanes of the same wavefront, so stages synchronise with a wavefront
// barrier instead of a workgroup barrier. Lengths, radices and twiddle
// spans are template constants; the LDS layout enters through an element
// accessor (affine, or bank-swizzled by a GF(2)-linear map), so each access
// costs at most one XOR beyond a per-lane base.
#pragma once

#include <hip/hip_runtime.h>

namespace rte {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

template <typename V>
__device__ __forceinline__ V cmk(decltype(V::x) re, decltype(V::x) im) {
  V r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return cmk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return cmk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return cmk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return cmk<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V::x) s) { return cmk<V>(a.x * s, a.y * s); }
// a * (DIR * i); DIR = -1 for the forward transform, +1 for the inverse.
template <typename V, int DIR> __device__ __forceinline__ V cmul_i(V a) {
  if constexpr (DIR > 0) return cmk<V>(-a.y, a.x);
  else return cmk<V>(a.y, -a.x);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ plans ----
// Radix sequence for length L = 2^a 3^b (b <= 1): a radix-3 stage first,
// then radix-8 stages, then one radix-4 or radix-2 stage for the rest.
constexpr int plan_count(int L) {
  int c = 0, m = L;
  if (m % 3 == 0) { ++c; m /= 3; }
  while (m % 8 == 0) { ++c; m /= 8; }
  if (m == 4 || m == 2) ++c;
  return c;
}
constexpr int plan_radix(int L, int st) {
  int m = L, s = 0;
  if (m % 3 == 0) { if (s == st) return 3; ++s; m /= 3; }
  while (m % 8 == 0) { if (s == st) return 8; ++s; m /= 8; }
  if (m == 4) return 4;
  if (m == 2) return 2;
  return 0;
}
constexpr bool plan_ok(int L) {
  int m = L;
  if (m % 3 == 0) m /= 3;
  while (m % 8 == 0) m /= 8;
  return m == 1 || m == 2 || m == 4;
}
// Elements per lane: must be a multiple of every radix of the plan.
constexpr int elems_per_lane(int L) { return (L % 3 == 0) ? 24 : (L >= 8 ? 8 : L); }

// In-register DFT of size R: v[q] <- sum_r v[r] exp(DIR 2 pi i q r / R).
template <typename V, int R, int DIR> struct Bfly;

template <typename V, int DIR> struct Bfly<V, 2, DIR> {
  static __device__ __forceinline__ void run(V* v) {
    const V t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
  }
};

template <typename V, int DIR> struct Bfly<V, 3, DIR> {
  static __device__ __forceinline__ void run(V* v) {
    using T = decltype(V::x);
    const T h = T(0.86602540378443864676);   // sqrt(3)/2
    const V t = cadd(v[1], v[2]);
    const V m = cmk<V>(v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y);
    const V d = cscale(cmul_i<V, DIR>(csub(v[1], v[2])), h);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, d);
    v[2] = csub(m, d);
  }
};

template <typename V, int DIR> struct Bfly<V, 4, DIR> {
  static __device__ __forceinline__ void run(V* v) {
    const V t0 = cadd(v[0], v[2]);
    const V t1 = csub(v[0], v[2]);
    const V t2 = cadd(v[1], v[3]);
    const V t3 = cmul_i<V, DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <typename V, int DIR> struct Bfly<V, 8, DIR> {
  static __device__ __forceinline__ void run(V* v) {
    using T = decltype(V::x);
    const T r2 = T(0.70710678118654752440);
    V a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = cadd(v[r], v[r + 4]);
      b[r] = csub(v[r], v[r + 4]);
    }
    // b[r] *= exp(DIR i pi r / 4)
    {
      const V x = b[1];
      b[1] = cmk<V>((x.x - T(DIR) * x.y) * r2, (x.y + T(DIR) * x.x) * r2);
      b[2] = cmul_i<V, DIR>(b[2]);
      const V y = b[3];
      b[3] = cmk<V>((-y.x - T(DIR) * y.y) * r2, (-y.y + T(DIR) * y.x) * r2);
    }
    Bfly<V, 4, DIR>::run(a);
    Bfly<V, 4, DIR>::run(b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = a[q];
      v[2 * q + 1] = b[q];
    }
  }
};

// 16-point DFT, v[q] <- sum_r v[r] exp(DIR 2 pi i q r / 16): radix 4 over
// r = 4 r1 + r2, internal twiddles exp(DIR 2 pi i q1 r2 / 16), radix 4 over
// r2; output q = q1 + 4 q2.
template <typename V, int DIR> struct Bfly<V, 16, DIR> {
  static __device__ __forceinline__ void run(V* v) {
    using T = decltype(V::x);
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);   // cos, sin(pi/8)
    const T r2 = T(0.70710678118654752440);
    const T dr = T(DIR);
    V y[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      y[b][0] = v[b];
      y[b][1] = v[b + 4];
      y[b][2] = v[b + 8];
      y[b][3] = v[b + 12];
      Bfly<V, 4, DIR>::run(y[b]);
    }
    // y[r2][q1] *= exp(DIR 2 pi i q1 r2 / 16)
    auto rot = [dr](V a, T c, T s) { return cmk<V>(a.x * c - dr * a.y * s, a.y * c + dr * a.x * s); };
    auto r8 = [dr, r2](V a) { return cmk<V>((a.x - dr * a.y) * r2, (a.y + dr * a.x) * r2); };
    auto r38 = [dr, r2](V a) { return cmk<V>((-a.x - dr * a.y) * r2, (-a.y + dr * a.x) * r2); };
    y[1][1] = rot(y[1][1], c1, s1);
    y[1][2] = r8(y[1][2]);
    y[1][3] = rot(y[1][3], s1, c1);
    y[2][1] = r8(y[2][1]);
    y[2][2] = cmul_i<V, DIR>(y[2][2]);
    y[2][3] = r38(y[2][3]);
    y[3][1] = rot(y[3][1], s1, c1);
    y[3][2] = r38(y[3][2]);
    y[3][3] = rot(y[3][3], -c1, -s1);   // exp(DIR i 9 pi / 8)
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1) {
      V t[4] = {y[0][q1], y[1][q1], y[2][q1], y[3][q1]};
      Bfly<V, 4, DIR>::run(t);
#pragma unroll
      for (int q2 = 0; q2 < 4; ++q2) v[q1 + 4 * q2] = t[q2];
    }
  }
};

// Element accessors. An FFT pass addresses element i of FFT f through an
// accessor `at` with i split as i = a + b: `a` holds the lane-dependent
// part and `b` a compile-time part whose bits are disjoint from those of a
// (for power-of-two lengths). at.lane(f, a) returns the per-lane state of
// one access pattern and at.elem(lane, b) the element's LDS address, so a
// swizzled layout costs one XOR per access (kXor: the layout needs the
// disjoint split; otherwise it is affine and any split works).
//
// Affine layout: element i of FFT f at p0 + f FS + i IS.
template <typename V, int FS, int IS>
struct AffineAt {
  static constexpr bool kXor = false;
  V* p0;
  struct Lane { V* q; };
  __device__ __forceinline__ Lane lane(int f, int a) const { return {p0 + f * FS + a * IS}; }
  __device__ __forceinline__ V* elem(Lane l, int b) const { return l.q + b * IS; }
};

// One Stockham stage of radix R on an FFT of length L. Lane p (of
// P = L/E) performs butterflies j = p + i P, i < E / R, after the previous
// stages have combined spans of NS; butterfly j reads elements j + r L/R and
// writes o + r NS, o = (j / NS) NS R + j % NS. tw holds exp(-2 pi i t / NTAB),
// t < NTAB.
template <typename V, int L, int R, int NS, int NTAB, int DIR, typename At>
__device__ __forceinline__ void fft_stage(const At& at, int f, int p, const V* tw, bool act) {
  constexpr int E = elems_per_lane(L);
  constexpr int P = L / E;
  constexpr int NB = E / R;
  constexpr int LR = L / R;
  constexpr int SPAN = (NTAB / (NS * R));
  static_assert(E % R == 0, "radix must divide elements per lane");
  static_assert(!At::kXor || (L & (L - 1)) == 0, "swizzled layouts need power-of-two lengths");
  V v[NB][R];
  if (act) {
    // reads: j + r LR = p + (i P + r LR), the constant part a multiple of P
    const auto lr = at.lane(f, p);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = *at.elem(lr, i * P + r * LR);
    }
  }
  wave_sync();
  if (act) {
    // writes: o + r NS split into a lane part and a constant part (power-of-two
    // lengths: NS and P are powers of two, so one divides the other)
    constexpr bool kSplit = (L & (L - 1)) == 0;
    int aw = 0;
    if constexpr (!kSplit) aw = 0;
    else if constexpr (NS <= P) aw = (p / NS) * NS * R + p % NS;
    else aw = p;
    const auto lw = at.lane(f, aw);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = p + i * P;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw[r * k * SPAN];
          if constexpr (DIR > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Bfly<V, R, DIR>::run(v[i]);
      int ob;
      if constexpr (!kSplit) ob = (j / NS) * NS * R + k;
      else if constexpr (NS <= P) ob = i * P * R;
      else ob = ((i * P) / NS) * NS * R + (i * P) % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) *at.elem(lw, ob + r * NS) = v[i][r];
    }
  }
  wave_sync();
}

template <typename V, int L, int NTAB, int DIR, int ST = 0, int NS = 1, typename At>
__device__ __forceinline__ void fft_stages(const At& at, int f, int p, const V* tw, bool act) {
  if constexpr (ST < plan_count(L)) {
    constexpr int R = plan_radix(L, ST);
    fft_stage<V, L, R, NS, NTAB, DIR>(at, f, p, tw, act);
    fft_stages<V, L, NTAB, DIR, ST + 1, NS * R>(at, f, p, tw, act);
  }
}

// Run COUNT FFTs of length L through accessor `at` with every wavefront of a
// BLOCK-thread workgroup holding 64 / P of them at a time.
template <typename V, int L, int NTAB, int DIR, int COUNT, int BLOCK, typename At>
__device__ __forceinline__ void fft_batch(const V* tw, const At& at) {
  static_assert(plan_ok(L), "unsupported FFT length");
  constexpr int P = L / elems_per_lane(L);
  static_assert(64 % P == 0 && (P & (P - 1)) == 0, "an FFT must fit one wavefront");
  constexpr int PER_WAVE = 64 / P;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  constexpr int per_round = (BLOCK / 64) * PER_WAVE;
  const int g = lane / P;
  const int p = lane - g * P;
  for (int f0 = 0; f0 < COUNT; f0 += per_round) {
    const int f = f0 + wave * PER_WAVE + g;
    const bool act = f < COUNT;
    int fa = act ? f : 0, pp = p;
    // opaque copies: the per-lane index arithmetic of the stages is redone
    // in every round instead of being hoisted (and held in registers) across
    // rounds and calls; the mask restores what is known of the lane index
    asm volatile("" : "+v"(fa), "+v"(pp));
    pp &= P - 1;
    fft_stages<V, L, NTAB, DIR>(at, fa, pp, tw, act);
  }
}

// Bank swizzle of an FFT of length L stored contiguously in LDS: element i
// sits at i ^ ((i >> 3) & 15) (a permutation inside each aligned block of
// 16). A Stockham stage with eight elements per lane writes every lane's
// eight outputs to consecutive slots (stride 8 across the lanes), which
// without it puts the 16 lanes of one LDS cycle on two bank pairs; with it
// every read and write of the radix-8 and radix-2 stages of a length-64..256
// transform is conflict-free. Lengths that are not a power of two >= 64 keep
// the plain order.
template <int L>
__device__ __forceinline__ int fft_swz(int i) {
  if constexpr (L >= 64 && (L & (L - 1)) == 0) return i ^ ((i >> 3) & 15);
  else return i;
}

// Contiguous FFTs of length L with the swizzle above: element i of FFT f at
// p0 + f PITCH + fft_swz<L>(i) (the swizzle is linear over GF(2), so it
// splits over the disjoint parts a and b).
template <typename V, int L, int PITCH>
struct SwzAt {
  static constexpr bool kXor = (L >= 64 && (L & (L - 1)) == 0);
  V* p0;
  struct Lane { V* q; int x; };
  __device__ __forceinline__ Lane lane(int f, int a) const { return {p0 + f * PITCH, fft_swz<L>(a)}; }
  __device__ __forceinline__ V* elem(Lane l, int b) const {
    if constexpr (kXor) return l.q + (l.x ^ fft_swz<L>(b));
    else return l.q + l.x + b;
  }
};

// Element-wise copy of COUNT items by a BLOCK-thread workgroup with up to
// 16 loads per thread in flight before the matching stores, so global
// latency overlaps instead of serialising load -> store pairs.
template <int COUNT, int BLOCK, typename Ld, typename St>
__device__ __forceinline__ void staged_copy(Ld ld, St st) {
  constexpr int ITER = (COUNT + BLOCK - 1) / BLOCK;
  constexpr int CHUNK = ITER < 16 ? ITER : 16;
  for (int it0 = 0; it0 < ITER; it0 += CHUNK) {
    decltype(ld(0)) tmp[CHUNK];
#pragma unroll
    for (int c = 0; c < CHUNK; ++c) {
      const int i = int(threadIdx.x) + (it0 + c) * BLOCK;
      if (it0 + c < ITER && (COUNT % BLOCK == 0 || i < COUNT)) tmp[c] = ld(i);
    }
#pragma unroll
    for (int c = 0; c < CHUNK; ++c) {
      const int i = int(threadIdx.x) + (it0 + c) * BLOCK;
      if (it0 + c < ITER && (COUNT % BLOCK == 0 || i < COUNT)) st(i, tmp[c]);
    }
  }
}

}  // namespace rte
