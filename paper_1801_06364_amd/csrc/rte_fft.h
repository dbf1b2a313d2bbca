// Device building blocks for the P_N stepper on gfx950: complex helpers,
// radix-2/3/4/8 butterflies and a Stockham auto-sort FFT executed by a
// group of P lanes of one wavefront on data staged in LDS.
//
// An FFT of length L is owned by P = L / E lanes of ONE 64-lane wavefront;
// each lane holds E elements in registers per stage (E = 8 for powers of
// two, 24 when L has a factor 3). Because every stage only exchanges data
// among lanes of the same wavefront, stages synchronise with a wavefront
// barrier instead of a workgroup barrier.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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

// One Stockham stage of radix R on an FFT of length L stored at
// buf[i * stride]. Lane p (of P) performs butterflies j = p + i P,
// i < E / R. tw holds exp(-2 pi i t / ntab), t < ntab, and twmul = ntab / L.
template <typename V, int E, int R, int DIR>
__device__ __forceinline__ void fft_stage(V* buf, int stride, int L, int P, int p,
                                          int Ns, const V* tw, int twmul, bool act) {
  constexpr int NB = E / R;
  V v[NB][R];
  const int LR = L / R;
  if (act) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = p + i * P;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[(j + r * LR) * stride];
    }
  }
  wave_sync();
  if (act) {
    const int span = (L / (Ns * R)) * twmul;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = p + i * P;
      const int k = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw[r * k * span];
          if constexpr (DIR > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Bfly<V, R, DIR>::run(v[i]);
      const int o = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(o + r * Ns) * stride] = v[i][r];
    }
  }
  wave_sync();
}

// Full FFT: plan holds the radices, 4 bits each, first stage lowest.
template <typename V, int E, int DIR>
__device__ __forceinline__ void fft_lds(V* buf, int stride, int L, int P, int p,
                                        unsigned plan, const V* tw, int twmul, bool act) {
  int Ns = 1;
#pragma unroll 1
  for (int st = 0; st < 6; ++st) {
    const int R = (plan >> (4 * st)) & 15;
    if (R == 0) break;
    if (R == 8) {
      if constexpr (E % 8 == 0) fft_stage<V, E, 8, DIR>(buf, stride, L, P, p, Ns, tw, twmul, act);
    } else if (R == 4) {
      if constexpr (E % 4 == 0) fft_stage<V, E, 4, DIR>(buf, stride, L, P, p, Ns, tw, twmul, act);
    } else if (R == 2) {
      if constexpr (E % 2 == 0) fft_stage<V, E, 2, DIR>(buf, stride, L, P, p, Ns, tw, twmul, act);
    } else if (R == 3) {
      if constexpr (E % 3 == 0) fft_stage<V, E, 3, DIR>(buf, stride, L, P, p, Ns, tw, twmul, act);
    }
    Ns *= R;
  }
}

// Run `count` FFTs (index f, base pointer base_of(f)) with every wavefront
// of the workgroup holding 64 / P of them at a time.
template <typename V, int E, int DIR, typename BaseOf>
__device__ __forceinline__ void fft_batch(int count, int stride, int L, unsigned plan,
                                          const V* tw, int twmul, BaseOf base_of) {
  const int P = L / E;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int per_wave = 64 / P;
  const int per_round = (blockDim.x >> 6) * per_wave;
  const int g = lane / P;
  const int p = lane - g * P;
  for (int f0 = 0; f0 < count; f0 += per_round) {
    const int f = f0 + wave * per_wave + g;
    const bool act = (g < per_wave) && (f < count);
    V* base = base_of(act ? f : 0);
    fft_lds<V, E, DIR>(base, stride, L, P, p, plan, tw, twmul, act);
  }
}

}  // namespace rte
