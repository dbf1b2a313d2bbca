// Kernels of one RK stage of the P_N stepper, specialised at compile time
// for the grid size NN (points per axis) and the working precision T.
//
// One RK stage evaluates f(v) = c (w - Sigma_l v + q) with
// w = -IFFT[ i (k.B) FFT(v) ] (eqs. 6, 9, 10 with the sign form of eqs. 1
// and 6) in three sweeps over HBM:
//   F  k_fwd_plane  per (moment, z-plane): x real-to-complex FFT and y FFT of
//                   the plane in LDS, written to the half spectrum
//                   [b][z][ky][kx], kx in [0, n/2];
//   Z  k_zpass      per (ky, kx-tile): all moments of TT spectral columns in
//                   LDS; z FFT, the streaming coupling of eq. (10) in the real
//                   basis, inverse z FFT;
//   P  k_inv_plane  per (moment, z-plane): inverse y FFT, complex-to-real x
//                   FFT and the fused pointwise epilogue (loss, in-scatter,
//                   boundary layer, source, RK combine; after the last stage
//                   also the integrated fluence and fluence-change partials).
// k_end_step closes each step (detector readings, residual, stop flags).
//
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2. Tiles that share cache lines (neighbouring kx columns in Z, the moments
// of one z-plane that read the same loss map in P) are remapped so that
// consecutive logical tiles run on the same XCD.
#pragma once

#include <hip/hip_runtime.h>

#include "rte_fft.h"
#include "rte_internal.h"

#ifndef RTE_ZBUDGET
#define RTE_ZBUDGET (64 * 1024)
#endif

namespace rte {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

// Physical block id -> logical tile: XCD x (= bid % 8) receives a contiguous
// range of logical tiles, in dispatch order.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  const int x = bid % kXcds, local = bid / kXcds;
  return x * per + (x < rem ? x : rem) + local;
}

template <int NN> struct GridC {
  static constexpr int n = NN;
  static constexpr int H = NN / 2;
  static constexpr int Kp = NN / 2 + 1;
  static constexpr int E = elems_per_lane(NN);
  static_assert(elems_per_lane(NN / 2) == elems_per_lane(NN), "row/column lane shape");
};

// kx columns per Z-pass workgroup: largest power of two (<= 16) whose
// columns of all moments fit the LDS budget.
template <typename T, int NN, int N>
constexpr int z_tile() {
  constexpr long col = long((N + 1) * (N + 1)) * NN * 2 * sizeof(T);
  int tt = 1;
  while (tt < 16 && 2 * tt <= NN / 2 + 1 && (2 * tt) * col + NN * 2 * long(sizeof(T)) <= RTE_ZBUDGET) tt *= 2;
  return tt;
}

template <typename T, int NN>
constexpr size_t plane_lds() {
  using G = GridC<NN>;
  const size_t b = (size_t(NN) * G::Kp + NN) * 2 * sizeof(T);
  return b < 2 * kBlock * 8 ? 2 * kBlock * 8 : b;
}
template <typename T, int NN, int N>
constexpr size_t z_lds() {
  return (size_t(z_tile<T, NN, N>()) * (N + 1) * (N + 1) * NN + NN) * 2 * sizeof(T);
}

// ---------------------------------------------------------- F: forward ---

template <typename T, int NN>
__global__ void __launch_bounds__(kBlock)
k_fwd_plane(const T* __restrict__ src, typename cplx_of<T>::type* __restrict__ spec,
            const typename cplx_of<T>::type* __restrict__ twg, const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  using G = GridC<NN>;
  constexpr int n = NN, H = G::H, Kp = G::Kp;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + n;
  const int plane = blockIdx.x;            // b * n + z
  for (int i = threadIdx.x; i < n; i += kBlock) tw[i] = twg[i];
  const T* s = src + size_t(plane) * n * n;
  for (int i = threadIdx.x; i < n * H; i += kBlock) {
    const int y = i / H, j = i - y * H;
    pl[y * Kp + j] = *reinterpret_cast<const V*>(s + y * n + 2 * j);
  }
  __syncthreads();
  // x: n packed rows of length H (twiddle table of length n, stride 2)
  fft_batch<V, H, 1, 2 * H, -1, n>(tw, [&](int f) { return pl + f * Kp; });
  __syncthreads();
  // real-to-complex split: X_k from Z_k and Z_{H-k}
  constexpr int half = H / 2;
  for (int i = threadIdx.x; i < n * (half + 1); i += kBlock) {
    const int y = i / (half + 1), k = i - y * (half + 1);
    V* row = pl + y * Kp;
    if (k == 0) {
      const V z0 = row[0];
      row[0] = cmk<V>(z0.x + z0.y, T(0));
      row[H] = cmk<V>(z0.x - z0.y, T(0));
    } else {
      const int m = H - k;
      const V zk = row[k], zm = row[m];
      const V zmc = cconj(zm), zkc = cconj(zk);
      // X_k = (Z_k + conj Z_m)/2 - i w_k (Z_k - conj Z_m)/2,  w_k = exp(-2 pi i k / n)
      const V ek = cscale(cadd(zk, zmc), T(0.5));
      const V ok = cmul_i<V, -1>(cscale(csub(zk, zmc), T(0.5)));
      row[k] = cadd(ek, cmul(tw[k], ok));
      if (m != k) {
        const V em = cscale(cadd(zm, zkc), T(0.5));
        const V om = cmul_i<V, -1>(cscale(csub(zm, zkc), T(0.5)));
        row[m] = cadd(em, cmul(tw[m], om));
      }
    }
  }
  __syncthreads();
  // y: Kp columns of length n, stride Kp
  fft_batch<V, n, Kp, n, -1, Kp>(tw, [&](int f) { return pl + f; });
  __syncthreads();
  V* dst = spec + size_t(plane) * n * Kp;
  for (int i = threadIdx.x; i < n * Kp; i += kBlock) dst[i] = pl[i];
}

// ------------------------------------------------- Z: z FFT + coupling ---

template <typename V, typename T, int N, int A, int S>
struct RowAcc {
  static __device__ __forceinline__ void run(const V* in, const T* __restrict__ c, T kx, T ky,
                                             T kz, T& re, T& im) {
    constexpr int l = isqrt_c(A);
    constexpr int m = A - l * l - l;
    constexpr SlotList sl = slots_of(N, l, m);
    if constexpr (S < sl.count) {
      constexpr int b = sl.b[S];
      const T* t = c + (A * kMaxSlots + S) * 3;
      const T cf = t[0] * kx + t[1] * ky + t[2] * kz;
      re += cf * in[b].x;
      im += cf * in[b].y;
      RowAcc<V, T, N, A, S + 1>::run(in, c, kx, ky, kz, re, im);
    }
  }
};

template <typename V, typename T, int N, int A, int OSTRIDE>
struct Rows {
  static __device__ __forceinline__ void run(const V* in, V* out, const T* __restrict__ c, T kx,
                                             T ky, T kz, T sc) {
    if constexpr (A < (N + 1) * (N + 1)) {
      T re = 0, im = 0;
      RowAcc<V, T, N, A, 0>::run(in, c, kx, ky, kz, re, im);
      // w_hat = -i * sc * sum_b (k.B)[a,b] u_hat_b
      out[A * OSTRIDE] = cmk<V>(sc * im, -sc * re);
      Rows<V, T, N, A + 1, OSTRIDE>::run(in, out, c, kx, ky, kz, sc);
    }
  }
};

template <typename T, int NN, int N>
__global__ void __launch_bounds__(kBlock)
k_zpass(typename cplx_of<T>::type* __restrict__ spec, const typename cplx_of<T>::type* __restrict__ twg,
        const T* __restrict__ kv, const T* __restrict__ coef, T sc, const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  using G = GridC<NN>;
  constexpr int n = NN, Kp = G::Kp;
  constexpr int M = (N + 1) * (N + 1);
  constexpr int TT = z_tile<T, NN, N>();
  constexpr int NTILE = (Kp + TT - 1) / TT;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* col = tw + n;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int ky = tile / NTILE;
  const int kx0 = (tile - ky * NTILE) * TT;
  const int tc = min(TT, Kp - kx0);
  for (int i = threadIdx.x; i < n; i += kBlock) tw[i] = twg[i];
  // column element (b, kz, t) at spec[((b n + kz) n + ky) Kp + kx0 + t]
  V* gbase = spec + size_t(ky) * Kp + kx0;
  for (int i = threadIdx.x; i < M * TT * n; i += kBlock) {
    const int t = i % TT;
    const int kz = (i / TT) % n;
    const int b = i / (TT * n);
    if (t < tc) col[(b * TT + t) * n + kz] = gbase[(size_t(b) * n + kz) * n * Kp + t];
  }
  __syncthreads();
  auto base = [&](int f) { return col + f * n; };
  fft_batch<V, n, 1, n, -1, M * TT>(tw, base);
  __syncthreads();
  const T kyv = kv[ky];
  for (int pt = threadIdx.x; pt < TT * n; pt += kBlock) {
    const int t = pt / n, kz = pt - t * n;
    if (t >= tc) continue;
    V in[M];
#pragma unroll
    for (int b = 0; b < M; ++b) in[b] = col[(b * TT + t) * n + kz];
    Rows<V, T, N, 0, TT * n>::run(in, col + t * n + kz, coef, kv[kx0 + t], kyv, kv[kz], sc);
  }
  __syncthreads();
  fft_batch<V, n, 1, n, +1, M * TT>(tw, base);
  __syncthreads();
  for (int i = threadIdx.x; i < M * TT * n; i += kBlock) {
    const int t = i % TT;
    const int kz = (i / TT) % n;
    const int b = i / (TT * n);
    if (t < tc) gbase[(size_t(b) * n + kz) * n * Kp + t] = col[(b * TT + t) * n + kz];
  }
}

// ------------------------------------------- P: inverse + epilogue -------

template <typename T, int NN, bool FIRST, bool LAST>
__global__ void __launch_bounds__(kBlock)
k_inv_plane(const typename cplx_of<T>::type* __restrict__ spec, const T* vin, T* u, T* dst,
            const T* __restrict__ sig, const T* __restrict__ q, const int* __restrict__ qflag,
            double* __restrict__ phi_int, double* __restrict__ partial,
            const typename cplx_of<T>::type* __restrict__ twg, int M, T h, double dt,
            const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  using G = GridC<NN>;
  constexpr int n = NN, H = G::H, Kp = G::Kp;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + n;
  // logical order z-major, moment-minor: moments of one z-plane (which
  // share the loss maps) run back to back on one XCD
  const int lt = xcd_tile(blockIdx.x, gridDim.x);
  const int z = lt / M, b = lt - z * M;
  const int plane = b * n + z;
  for (int i = threadIdx.x; i < n; i += kBlock) tw[i] = twg[i];
  const V* srcp = spec + size_t(plane) * n * Kp;
  for (int i = threadIdx.x; i < n * Kp; i += kBlock) pl[i] = srcp[i];
  __syncthreads();
  fft_batch<V, n, Kp, n, +1, Kp>(tw, [&](int f) { return pl + f; });
  __syncthreads();
  // complex-to-real merge: Z_k = (X_k + conj X_{H-k}) + i conj(w_k) (X_k - conj X_{H-k})
  constexpr int half = H / 2;
  for (int i = threadIdx.x; i < n * (half + 1); i += kBlock) {
    const int y = i / (half + 1), k = i - y * (half + 1);
    V* row = pl + y * Kp;
    const int m = H - k;
    const V xk = row[k], xm = row[m];
    const V xmc = cconj(xm), xkc = cconj(xk);
    const V zk = cadd(cadd(xk, xmc), cmul_i<V, +1>(cmul(cconj(tw[k]), csub(xk, xmc))));
    if (k == 0) {
      row[0] = zk;
    } else {
      row[k] = zk;
      if (m != k) row[m] = cadd(cadd(xm, xkc), cmul_i<V, +1>(cmul(cconj(tw[m]), csub(xm, xkc))));
    }
  }
  __syncthreads();
  fft_batch<V, H, 1, 2 * H, +1, n>(tw, [&](int f) { return pl + f * Kp; });
  __syncthreads();
  // epilogue on (x_{2j}, x_{2j+1}) pairs
  const int l = isqrt_c(b);
  const size_t poff = size_t(plane) * n * n;
  const size_t voff = size_t(z) * n * n;
  const T* sg = sig + size_t(l) * n * n * n + voff;
  const bool hasq = (q != nullptr) && qflag[z];
  double acc_d = 0.0, acc_o = 0.0;
  for (int i = threadIdx.x; i < n * H; i += kBlock) {
    const int y = i / H, j = i - y * H;
    const int e = y * n + 2 * j;
    const V w = pl[y * Kp + j];
    const V uu = *reinterpret_cast<const V*>(u + poff + e);
    const V vv = FIRST ? uu : *reinterpret_cast<const V*>(vin + poff + e);
    const V ss = *reinterpret_cast<const V*>(sg + e);
    T src0 = -ss.x * vv.x, src1 = -ss.y * vv.y;
    if (hasq) {
      const V qq = *reinterpret_cast<const V*>(q + poff + e);
      src0 += qq.x;
      src1 += qq.y;
    }
    const V o = cmk<V>(uu.x + w.x + h * src0, uu.y + w.y + h * src1);
    *reinterpret_cast<V*>(dst + poff + e) = o;
    if (LAST && b == 0) {
      double2* pi = reinterpret_cast<double2*>(phi_int + voff + e);
      double2 acc = *pi;
      acc.x += dt * double(o.x);
      acc.y += dt * double(o.y);
      *pi = acc;
      const double d0 = double(o.x) - double(uu.x), d1 = double(o.y) - double(uu.y);
      acc_d += d0 * d0 + d1 * d1;
      acc_o += double(o.x) * double(o.x) + double(o.y) * double(o.y);
    }
  }
  if (LAST && b == 0) {
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);
    red[threadIdx.x] = acc_d;
    red[kBlock + threadIdx.x] = acc_o;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        red[threadIdx.x] += red[threadIdx.x + s];
        red[kBlock + threadIdx.x] += red[kBlock + threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partial[2 * z] = red[0];
      partial[2 * z + 1] = red[kBlock];
    }
  }
}

// ------------------------------------------------------- end of step ---

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_end_step(const T* __restrict__ u, const long long* __restrict__ det, int ndet,
           double* __restrict__ readings, double* __restrict__ resid, long long cap,
           const double* __restrict__ partial, int n, Ctl* ctl) {
  if (ctl->stop) return;
  const long long s = ctl->step;
  if (s < cap)
    for (int p = threadIdx.x; p < ndet; p += blockDim.x) readings[s * ndet + p] = double(u[det[p]]);
  if (threadIdx.x == 0) {
    double d2 = 0.0, o2 = 0.0;
    for (int z = 0; z < n; ++z) {
      d2 += partial[2 * z];
      o2 += partial[2 * z + 1];
    }
    const double r = o2 > 0.0 ? sqrt(d2 / o2) : 0.0;
    if (s < cap) resid[s] = r;
    ctl->last_resid = r;
    ctl->last_norm2 = o2;
    ctl->step = s + 1;
    if (!isfinite(d2) || !isfinite(o2) || o2 > ctl->growth_limit) ctl->stop = 2;
    else if (ctl->tol > 0.0 && r < ctl->tol) ctl->stop = 1;
  }
}

// ------------------------------------------------------------ launch ---

template <typename T, int NN, int N>
hipError_t prepare_t(const StepArgs& a) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, size_t bytes) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  };
  set(reinterpret_cast<const void*>(&k_fwd_plane<T, NN>), plane_lds<T, NN>());
  set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, true, false>), plane_lds<T, NN>());
  set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, false, false>), plane_lds<T, NN>());
  set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, false, true>), plane_lds<T, NN>());
  set(reinterpret_cast<const void*>(&k_zpass<T, NN, N>), z_lds<T, NN, N>());
  return e;
}

template <typename T, int NN, int N>
hipError_t enqueue_t(const StepArgs& a, hipEvent_t* ev) {
  using V = typename cplx_of<T>::type;
  using G = GridC<NN>;
  constexpr int M = (N + 1) * (N + 1);
  constexpr int TT = z_tile<T, NN, N>();
  constexpr int NTILE = (G::Kp + TT - 1) / TT;
  hipStream_t st = reinterpret_cast<hipStream_t>(a.stream);
  T* u = static_cast<T*>(a.u);
  T* v = static_cast<T*>(a.v);
  V* spec = static_cast<V*>(a.spec);
  const V* tw = static_cast<const V*>(a.tw);
  const T* kv = static_cast<const T*>(a.kv);
  const T* coef = static_cast<const T*>(a.coef);
  const T* sig = static_cast<const T*>(a.sig);
  const T* q = static_cast<const T*>(a.q);
  const Ctl* cctl = static_cast<const Ctl*>(a.ctl);
  const double n3 = double(NN) * NN * NN;
  const double alphas[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
  const dim3 blk(kBlock);
  const int planes = M * NN;
  const int zblocks = NN * NTILE;
  const size_t lp = plane_lds<T, NN>(), lz = z_lds<T, NN, N>();
  int mark = 0;
  auto rec = [&]() {
    if (ev) (void)hipEventRecord(ev[mark++], st);
  };
  rec();
  for (int s = 0; s < 4; ++s) {
    const double hs = alphas[s] * a.dt * a.c;
    const T* src = s == 0 ? u : v;
    hipLaunchKernelGGL((k_fwd_plane<T, NN>), dim3(planes), blk, lp, st, src, spec, tw, cctl);
    rec();
    hipLaunchKernelGGL((k_zpass<T, NN, N>), dim3(zblocks), blk, lz, st, spec, tw, kv, coef, T(hs / n3),
                       cctl);
    rec();
    if (s == 0)
      hipLaunchKernelGGL((k_inv_plane<T, NN, true, false>), dim3(planes), blk, lp, st, spec, src, u, v, sig,
                         q, a.qflag, a.phi_int, a.partial, tw, M, T(hs), a.dt, cctl);
    else if (s < 3)
      hipLaunchKernelGGL((k_inv_plane<T, NN, false, false>), dim3(planes), blk, lp, st, spec, src, u, v,
                         sig, q, a.qflag, a.phi_int, a.partial, tw, M, T(hs), a.dt, cctl);
    else
      hipLaunchKernelGGL((k_inv_plane<T, NN, false, true>), dim3(planes), blk, lp, st, spec, src, u, u, sig,
                         q, a.qflag, a.phi_int, a.partial, tw, M, T(hs), a.dt, cctl);
    rec();
  }
  hipLaunchKernelGGL((k_end_step<T>), dim3(1), blk, 0, st, u, a.det, a.ndet, a.readings, a.resid, a.cap,
                     a.partial, NN, static_cast<Ctl*>(a.ctl));
  rec();
  return hipGetLastError();
}

template <template <typename, int, int> class Fn, int NN, typename... Args>
hipError_t dispatch_tn(const StepArgs& a, Args... args) {
#define RTE_CASE_N(T)                                  \
  switch (a.N) {                                       \
    case 0: return Fn<T, NN, 0>::call(a, args...);     \
    case 1: return Fn<T, NN, 1>::call(a, args...);     \
    case 2: return Fn<T, NN, 2>::call(a, args...);     \
    case 3: return Fn<T, NN, 3>::call(a, args...);     \
    case 4: return Fn<T, NN, 4>::call(a, args...);     \
    case 5: return Fn<T, NN, 5>::call(a, args...);     \
    case 6: return Fn<T, NN, 6>::call(a, args...);     \
    case 7: return Fn<T, NN, 7>::call(a, args...);     \
    default: return hipErrorInvalidValue;              \
  }
  if (a.prec == 1) {
    RTE_CASE_N(double)
  } else {
    RTE_CASE_N(float)
  }
#undef RTE_CASE_N
}

template <typename T, int NN, int N> struct EnqueueFn {
  static hipError_t call(const StepArgs& a, hipEvent_t* ev) { return enqueue_t<T, NN, N>(a, ev); }
};
template <typename T, int NN, int N> struct PrepareFn {
  static hipError_t call(const StepArgs& a) { return prepare_t<T, NN, N>(a); }
};

// Defines the per-size entry points used by the runtime.
#define RTE_DEFINE_SIZE(NN)                                                              \
  int enqueue_step_n##NN(const StepArgs& a, void* ev) {                                  \
    return int(dispatch_tn<EnqueueFn, NN>(a, static_cast<hipEvent_t*>(ev)));             \
  }                                                                                      \
  int prepare_n##NN(const StepArgs& a) { return int(dispatch_tn<PrepareFn, NN>(a)); }

}  // namespace rte
