// MI355X (gfx950) P_N pseudospectral transport stepper: kernels, runtime and
// the C-ABI declared in include/rte.h.
//
// One RK stage evaluates f(v) = c (w - Sigma_l v + q) with
// w = -IFFT[ i (k.B) FFT(v) ] (eqs. 6, 9, 10 with the sign form of eqs. 1
// and 6) in three sweeps over HBM:
//   F  (k_fwd_plane)  per (moment, z-plane): x real-to-complex FFT and y FFT
//                     of the plane in LDS, written to the half spectrum;
//   Z  (k_zpass)      per (ky, kx-tile) column, all moments in LDS: z FFT,
//                     the streaming coupling of eq. (10) in the real basis,
//                     inverse z FFT;
//   P  (k_inv_plane)  per (moment, z-plane): inverse y FFT, complex-to-real
//                     x FFT and the fused pointwise epilogue (loss, source,
//                     boundary layer, RK combine; after the last stage also
//                     integrated fluence and the fluence-change partials).
// A one-block kernel closes each step (detector readings, residual, flags).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rte.h"
#include "rte_fft.h"
#include "rte_internal.h"

namespace rte {

// ------------------------------------------------------------- control ---

struct Ctl {
  long long step;       // steps applied since creation / last set_state
  int stop;             // 0 run, 1 converged (tol met), 2 unstable
  int pad;
  double tol;           // relative fluence change that stops a run (0: off)
  double growth_limit;  // ||phi||^2 above this flags runaway growth
  double last_resid;
  double last_norm2;
};

struct Geo {
  int n, H, Kp, M, N;   // H = n/2, Kp = n/2 + 1
  unsigned plan_row;    // radices of the length-H row FFT
  unsigned plan_col;    // radices of the length-n column FFT
  int TT;               // kx columns per Z-pass workgroup
  int ntile;            // Z-pass tiles per ky
};

__host__ __device__ inline size_t spec_off(const Geo& g, int b, int z, int ky, int kx) {
  return ((size_t(b) * g.n + z) * g.n + ky) * g.Kp + kx;
}

// ---------------------------------------------------------- F: forward ---

template <typename T, int E>
__global__ void __launch_bounds__(256)
k_fwd_plane(const T* __restrict__ src, typename cplx_of<T>::type* __restrict__ spec,
            const typename cplx_of<T>::type* __restrict__ twg, Geo g, const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + g.n;
  const int n = g.n, H = g.H, Kp = g.Kp;
  const int plane = blockIdx.x;            // b * n + z
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
  const T* s = src + size_t(plane) * n * n;
  for (int i = threadIdx.x; i < n * H; i += blockDim.x) {
    const int y = i / H, j = i - y * H;
    pl[y * Kp + j] = *reinterpret_cast<const V*>(s + size_t(y) * n + 2 * j);
  }
  __syncthreads();
  // x: n packed rows of length H
  fft_batch<V, E, -1>(n, 1, H, g.plan_row, tw, 2, [&](int f) { return pl + f * Kp; });
  __syncthreads();
  // real-to-complex split: X_k from Z_k and Z_{H-k}
  const int half = H / 2;
  for (int i = threadIdx.x; i < n * (half + 1); i += blockDim.x) {
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
  fft_batch<V, E, -1>(Kp, Kp, n, g.plan_col, tw, 1, [&](int f) { return pl + f; });
  __syncthreads();
  const int b = plane / n, z = plane - b * n;
  V* dst = spec + spec_off(g, b, z, 0, 0);
  for (int i = threadIdx.x; i < n * Kp; i += blockDim.x) dst[i] = pl[i];
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

template <typename V, typename T, int N, int A>
struct Rows {
  static __device__ __forceinline__ void run(const V* in, V* out, int ostride,
                                             const T* __restrict__ c, T kx, T ky, T kz, T sc) {
    if constexpr (A < (N + 1) * (N + 1)) {
      T re = 0, im = 0;
      RowAcc<V, T, N, A, 0>::run(in, c, kx, ky, kz, re, im);
      // w_hat = -i * sc * sum_b (k.B)[a,b] u_hat_b
      out[A * ostride] = cmk<V>(sc * im, -sc * re);
      Rows<V, T, N, A + 1>::run(in, out, ostride, c, kx, ky, kz, sc);
    }
  }
};

template <typename T, int E, int N>
__global__ void __launch_bounds__(256)
k_zpass(typename cplx_of<T>::type* __restrict__ spec, const typename cplx_of<T>::type* __restrict__ twg,
        const T* __restrict__ kv, const T* __restrict__ coef, Geo g, T sc,
        const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  constexpr int M = (N + 1) * (N + 1);
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* col = tw + g.n;
  const int n = g.n, TT = g.TT;
  const int ky = blockIdx.x / g.ntile;
  const int kx0 = (blockIdx.x - ky * g.ntile) * TT;
  const int tc = min(TT, g.Kp - kx0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
  for (int i = threadIdx.x; i < M * TT * n; i += blockDim.x) {
    const int t = i % TT;
    const int kz = (i / TT) % n;
    const int b = i / (TT * n);
    if (t < tc) col[(b * TT + t) * n + kz] = spec[spec_off(g, b, kz, ky, kx0 + t)];
  }
  __syncthreads();
  const int nfft = M * TT;
  auto base = [&](int f) { return col + f * n; };
  fft_batch<V, E, -1>(nfft, 1, n, g.plan_col, tw, 1, base);
  __syncthreads();
  const T kyv = kv[ky];
  for (int pt = threadIdx.x; pt < TT * n; pt += blockDim.x) {
    const int t = pt / n, kz = pt - t * n;
    if (t >= tc) continue;
    V in[M];
#pragma unroll
    for (int b = 0; b < M; ++b) in[b] = col[(b * TT + t) * n + kz];
    Rows<V, T, N, 0>::run(in, col + t * n + kz, TT * n, coef, kv[kx0 + t], kyv, kv[kz], sc);
  }
  __syncthreads();
  fft_batch<V, E, +1>(nfft, 1, n, g.plan_col, tw, 1, base);
  __syncthreads();
  for (int i = threadIdx.x; i < M * TT * n; i += blockDim.x) {
    const int t = i % TT;
    const int kz = (i / TT) % n;
    const int b = i / (TT * n);
    if (t < tc) spec[spec_off(g, b, kz, ky, kx0 + t)] = col[(b * TT + t) * n + kz];
  }
}

// ------------------------------------------- P: inverse + epilogue -------

template <typename T, int E, bool FIRST, bool LAST>
__global__ void __launch_bounds__(256)
k_inv_plane(const typename cplx_of<T>::type* __restrict__ spec, const T* vin, T* u, T* dst,
            const T* __restrict__ sig, const T* __restrict__ q, const int* __restrict__ qflag,
            double* __restrict__ phi_int, double* __restrict__ partial,
            const typename cplx_of<T>::type* __restrict__ twg, Geo g, T h, double dt,
            const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + g.n;
  const int n = g.n, H = g.H, Kp = g.Kp;
  const int plane = blockIdx.x;
  const int b = plane / n, z = plane - b * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
  const V* srcp = spec + spec_off(g, b, z, 0, 0);
  for (int i = threadIdx.x; i < n * Kp; i += blockDim.x) pl[i] = srcp[i];
  __syncthreads();
  fft_batch<V, E, +1>(Kp, Kp, n, g.plan_col, tw, 1, [&](int f) { return pl + f; });
  __syncthreads();
  // complex-to-real merge: Z_k = (X_k + conj X_{H-k}) + i conj(w_k) (X_k - conj X_{H-k})
  const int half = H / 2;
  for (int i = threadIdx.x; i < n * (half + 1); i += blockDim.x) {
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
  fft_batch<V, E, +1>(n, 1, H, g.plan_row, tw, 2, [&](int f) { return pl + f * Kp; });
  __syncthreads();
  // epilogue on (x_{2j}, x_{2j+1}) pairs
  const int l = isqrt_c(b);
  const size_t poff = size_t(plane) * n * n;
  const size_t voff = size_t(z) * n * n;
  const T* sg = sig + size_t(l) * n * n * n + voff;
  const bool hasq = (q != nullptr) && qflag[z];
  double acc_d = 0.0, acc_o = 0.0;
  for (int i = threadIdx.x; i < n * H; i += blockDim.x) {
    const int y = i / H, j = i - y * H;
    const size_t e = size_t(y) * n + 2 * j;
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
    red[blockDim.x + threadIdx.x] = acc_o;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        red[threadIdx.x] += red[threadIdx.x + s];
        red[blockDim.x + threadIdx.x] += red[blockDim.x + threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partial[2 * z] = red[0];
      partial[2 * z + 1] = red[blockDim.x];
    }
  }
}

// ------------------------------------------------------- end of step ---

template <typename T>
__global__ void __launch_bounds__(256)
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

// ------------------------------------------------------------ runtime ---

constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t u, v, spec, sig, q, qflag, tw, kv, coef, det, readings, resid, partial, phi_int, ctl, total;
};

inline bool config_ok(const rte_config* c) {
  if (!c) return false;
  if (!grid_supported(c->n)) return false;
  if (c->order_N < 0 || c->order_N > kMaxOrder) return false;
  if (c->precision != RTE_FP32 && c->precision != RTE_FP64) return false;
  if (c->pml_width < 0 || 2 * c->pml_width >= c->n) return false;
  if (!(c->dx_mm > 0) || !(c->c_mm_ps > 0) || !std::isfinite(c->dx_mm) || !std::isfinite(c->c_mm_ps))
    return false;
  if (!std::isfinite(c->dt_ps)) return false;
  if (c->pml_width > 0 && (!(c->pml_mu0 >= 0) || !(c->pml_mu1 >= 0))) return false;
  if (c->n_det < 0 || (c->n_det > 0 && !c->det_index)) return false;
  if (c->record_steps < 0) return false;
  // plane passes keep one n x (n/2+1) complex plane in LDS (160 KB per CU)
  const size_t s = c->precision == RTE_FP64 ? 16 : 8;
  if ((size_t(c->n) * (c->n / 2 + 1) + c->n) * s > 160 * 1024) return false;
  return true;
}

inline Layout layout_of(const rte_config* c, bool has_q) {
  Layout L{};
  const size_t n = c->n, M = size_t(c->order_N + 1) * (c->order_N + 1);
  const size_t s = c->precision == RTE_FP64 ? 8 : 4;
  const size_t V = n * n * n;
  size_t o = 0;
  L.u = o; o = up(o + M * V * s);
  L.v = o; o = up(o + M * V * s);
  L.spec = o; o = up(o + M * n * n * (n / 2 + 1) * 2 * s);
  L.sig = o; o = up(o + size_t(c->order_N + 1) * V * s);
  L.q = o; o = up(o + (has_q ? M * V * s : 0));
  L.qflag = o; o = up(o + n * sizeof(int));
  L.tw = o; o = up(o + n * 2 * s);
  L.kv = o; o = up(o + n * s);
  L.coef = o; o = up(o + M * kMaxSlots * 3 * s);
  L.det = o; o = up(o + size_t(c->n_det) * 8);
  L.readings = o; o = up(o + size_t(c->record_steps) * c->n_det * 8);
  L.resid = o; o = up(o + size_t(c->record_steps) * 8);
  L.partial = o; o = up(o + n * 2 * 8);
  L.phi_int = o; o = up(o + V * 8);
  L.ctl = o; o = up(o + sizeof(Ctl));
  L.total = o;
  return L;
}

inline unsigned fft_plan(int L) {
  unsigned plan = 0;
  int sh = 0, m = L;
  auto push = [&](int r) { plan |= unsigned(r) << sh; sh += 4; m /= r; };
  if (m % 3 == 0) push(3);
  while (m % 8 == 0) push(8);
  if (m == 4) push(4);
  if (m == 2) push(2);
  return m == 1 ? plan : 0u;
}

}  // namespace rte

struct rte_handle {
  rte_config cfg;
  rte::Geo geo;
  rte::Layout lay;
  int n, N, M, prec;
  double dt;
  bool has_q;
  hipStream_t stream;
  unsigned char* ws;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool graph_ready;
  bool use_graph;
  size_t lds_plane, lds_z;
  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

namespace rte {

template <typename T, int E, int N>
hipError_t set_lds_limits(rte_handle* h) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, size_t bytes) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  };
  set(reinterpret_cast<const void*>(&k_fwd_plane<T, E>), h->lds_plane);
  set(reinterpret_cast<const void*>(&k_inv_plane<T, E, true, false>), h->lds_plane);
  set(reinterpret_cast<const void*>(&k_inv_plane<T, E, false, false>), h->lds_plane);
  set(reinterpret_cast<const void*>(&k_inv_plane<T, E, false, true>), h->lds_plane);
  set(reinterpret_cast<const void*>(&k_zpass<T, E, N>), h->lds_z);
  return e;
}

template <typename T, int E, int N>
hipError_t enqueue_step_t(rte_handle* h, hipEvent_t* ev) {
  using V = typename cplx_of<T>::type;
  const Geo& g = h->geo;
  const Layout& L = h->lay;
  T* u = h->at<T>(L.u);
  T* v = h->at<T>(L.v);
  V* spec = h->at<V>(L.spec);
  const V* tw = h->at<V>(L.tw);
  const T* kv = h->at<T>(L.kv);
  const T* coef = h->at<T>(L.coef);
  const T* sig = h->at<T>(L.sig);
  const T* q = h->has_q ? h->at<T>(L.q) : nullptr;
  const int* qflag = h->at<int>(L.qflag);
  double* phi = h->at<double>(L.phi_int);
  double* partial = h->at<double>(L.partial);
  Ctl* ctl = h->at<Ctl>(L.ctl);
  const double c = h->cfg.c_mm_ps, dt = h->dt;
  const double n3 = double(g.n) * g.n * g.n;
  const double alphas[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
  const dim3 blk(256);
  const int planes = g.M * g.n;
  const int zblocks = g.n * g.ntile;
  int mark = 0;
  auto rec = [&]() {
    if (ev) (void)hipEventRecord(ev[mark++], h->stream);
  };
  rec();
  for (int s = 0; s < 4; ++s) {
    const double hs = alphas[s] * dt * c;
    const T* src = s == 0 ? u : v;
    hipLaunchKernelGGL((k_fwd_plane<T, E>), dim3(planes), blk, h->lds_plane, h->stream, src, spec, tw,
                       g, ctl);
    rec();
    hipLaunchKernelGGL((k_zpass<T, E, N>), dim3(zblocks), blk, h->lds_z, h->stream, spec, tw, kv, coef,
                       g, T(hs / n3), ctl);
    rec();
    if (s == 0)
      hipLaunchKernelGGL((k_inv_plane<T, E, true, false>), dim3(planes), blk, h->lds_plane, h->stream,
                         spec, src, u, v, sig, q, qflag, phi, partial, tw, g, T(hs), dt, ctl);
    else if (s < 3)
      hipLaunchKernelGGL((k_inv_plane<T, E, false, false>), dim3(planes), blk, h->lds_plane, h->stream,
                         spec, src, u, v, sig, q, qflag, phi, partial, tw, g, T(hs), dt, ctl);
    else
      hipLaunchKernelGGL((k_inv_plane<T, E, false, true>), dim3(planes), blk, h->lds_plane, h->stream,
                         spec, src, u, u, sig, q, qflag, phi, partial, tw, g, T(hs), dt, ctl);
    rec();
  }
  hipLaunchKernelGGL((k_end_step<T>), dim3(1), blk, 0, h->stream, u, h->at<long long>(L.det),
                     h->cfg.n_det, h->at<double>(L.readings), h->at<double>(L.resid),
                     (long long)h->cfg.record_steps, partial, g.n, ctl);
  rec();
  return hipGetLastError();
}

// Dispatch over precision, E (radix-3 grids use E = 24) and the order N.
template <template <typename, int, int> class Fn>
hipError_t dispatch(rte_handle* h) {
  const bool three = (h->n % 3) == 0;
#define RTE_CASE_N(T, E)                                   \
  switch (h->N) {                                          \
    case 0: return Fn<T, E, 0>::call(h);                   \
    case 1: return Fn<T, E, 1>::call(h);                   \
    case 2: return Fn<T, E, 2>::call(h);                   \
    case 3: return Fn<T, E, 3>::call(h);                   \
    case 4: return Fn<T, E, 4>::call(h);                   \
    case 5: return Fn<T, E, 5>::call(h);                   \
    case 6: return Fn<T, E, 6>::call(h);                   \
    case 7: return Fn<T, E, 7>::call(h);                   \
    default: return hipErrorInvalidValue;                  \
  }
  if (h->prec == RTE_FP64) {
    if (three) { RTE_CASE_N(double, 24) } else { RTE_CASE_N(double, 8) }
  } else {
    if (three) { RTE_CASE_N(float, 24) } else { RTE_CASE_N(float, 8) }
  }
#undef RTE_CASE_N
}

template <typename T, int E, int N> struct StepFn {
  static hipError_t call(rte_handle* h) { return enqueue_step_t<T, E, N>(h, nullptr); }
};
thread_local hipEvent_t* g_prof_events = nullptr;
template <typename T, int E, int N> struct ProfStepFn {
  static hipError_t call(rte_handle* h) { return enqueue_step_t<T, E, N>(h, g_prof_events); }
};
template <typename T, int E, int N> struct LdsFn {
  static hipError_t call(rte_handle* h) { return set_lds_limits<T, E, N>(h); }
};

int to_code(hipError_t e) { return e == hipSuccess ? RTE_OK : RTE_EDEVICE; }

template <typename T>
void convert_upload(std::vector<T>& tmp, const double* src, size_t count) {
  tmp.resize(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = T(src[i]);
}

template <typename T>
int upload_state_t(rte_handle* h, const double* psi) {
  const size_t cnt = size_t(h->M) * h->n * h->n * h->n;
  std::vector<T> tmp;
  if (psi) convert_upload(tmp, psi, cnt);
  else tmp.assign(cnt, T(0));
  hipError_t e = hipMemcpyAsync(h->at<T>(h->lay.u), tmp.data(), cnt * sizeof(T), hipMemcpyHostToDevice,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return to_code(e);
}

template <typename T>
int download_t(rte_handle* h, size_t off, size_t cnt, double* out) {
  std::vector<T> tmp(cnt);
  hipError_t e = hipMemcpyAsync(tmp.data(), h->ws + off, cnt * sizeof(T), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return RTE_EDEVICE;
  for (size_t i = 0; i < cnt; ++i) out[i] = double(tmp[i]);
  return RTE_OK;
}

int read_ctl(rte_handle* h, Ctl* c) {
  hipError_t e = hipMemcpyAsync(c, h->ws + h->lay.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return to_code(e);
}

int write_ctl(rte_handle* h, const Ctl* c) {
  hipError_t e = hipMemcpyAsync(h->ws + h->lay.ctl, c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return to_code(e);
}

int reset_run_state(rte_handle* h, double growth_limit) {
  Ctl c{};
  c.growth_limit = growth_limit;
  int rc = write_ctl(h, &c);
  if (rc) return rc;
  hipError_t e = hipMemsetAsync(h->ws + h->lay.phi_int, 0, size_t(h->n) * h->n * h->n * 8, h->stream);
  if (e == hipSuccess && h->cfg.record_steps > 0 && h->cfg.n_det > 0)
    e = hipMemsetAsync(h->ws + h->lay.readings, 0, size_t(h->cfg.record_steps) * h->cfg.n_det * 8, h->stream);
  if (e == hipSuccess && h->cfg.record_steps > 0)
    e = hipMemsetAsync(h->ws + h->lay.resid, 0, size_t(h->cfg.record_steps) * 8, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return to_code(e);
}

double growth_limit_of(const rte_handle* h, const double* psi0, const double* q,
                       const std::vector<double>& sig0) {
  const size_t V = size_t(h->n) * h->n * h->n;
  double f2 = 0.0, q2 = 0.0, smin = 1e300;
  for (size_t i = 0; i < V; ++i) {
    if (psi0) f2 += psi0[i] * psi0[i];
    if (q) q2 += q[i] * q[i];
    smin = std::min(smin, sig0[i]);
  }
  smin = std::max(smin, 1e-6);
  return 1e16 * (f2 + q2 / (smin * smin) + 1e-300);
}

template <typename T>
int upload_tables_t(rte_handle* h, const rte_medium* med, const std::vector<double>& sig,
                    const std::vector<uint8_t>& inside, const std::vector<double>& coef) {
  const int n = h->n;
  const size_t V = size_t(n) * n * n;
  const Layout& L = h->lay;
  std::vector<T> tmp;
  hipError_t e = hipSuccess;
  auto put = [&](size_t off, const void* p, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(h->ws + off, p, bytes, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  };
  convert_upload(tmp, sig.data(), sig.size());
  put(L.sig, tmp.data(), tmp.size() * sizeof(T));
  std::vector<double> tw, kv;
  twiddles(n, tw);
  convert_upload(tmp, tw.data(), tw.size());
  put(L.tw, tmp.data(), tmp.size() * sizeof(T));
  wavenumbers(n, h->cfg.dx_mm, kv);
  convert_upload(tmp, kv.data(), kv.size());
  put(L.kv, tmp.data(), tmp.size() * sizeof(T));
  convert_upload(tmp, coef.data(), coef.size());
  put(L.coef, tmp.data(), tmp.size() * sizeof(T));
  std::vector<int> qflag(n, 0);
  if (h->has_q) {
    std::vector<double> qm(size_t(h->M) * V);
    for (int a = 0; a < h->M; ++a)
      for (size_t i = 0; i < V; ++i) {
        const double val = inside[i] ? med->q[size_t(a) * V + i] : 0.0;
        qm[size_t(a) * V + i] = val;
        if (val != 0.0) qflag[i / (size_t(n) * n)] = 1;
      }
    convert_upload(tmp, qm.data(), qm.size());
    put(L.q, tmp.data(), tmp.size() * sizeof(T));
  }
  put(L.qflag, qflag.data(), qflag.size() * sizeof(int));
  if (h->cfg.n_det > 0) put(L.det, h->cfg.det_index, size_t(h->cfg.n_det) * 8);
  return to_code(e);
}

int enqueue_steps(rte_handle* h, int64_t k) {
  if (k <= 0) return RTE_OK;
  if (h->use_graph && !h->graph_ready) {
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = dispatch<StepFn>(h);
      e = hipStreamEndCapture(h->stream, &h->graph);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      h->use_graph = false;   // fall back to direct launches
    } else {
      h->graph_ready = true;
    }
  }
  for (int64_t i = 0; i < k; ++i) {
    hipError_t e = h->graph_ready ? hipGraphLaunch(h->exec, h->stream) : dispatch<StepFn>(h);
    if (e != hipSuccess) return RTE_EDEVICE;
  }
  return RTE_OK;
}

}  // namespace rte

// ================================================================ C-ABI ==

extern "C" {

size_t rte_workspace_bytes(const rte_config* cfg) {
  if (!rte::config_ok(cfg)) return 0;
  return rte::layout_of(cfg, true).total;
}

int rte_create(const rte_config* cfg, const rte_medium* med, void* dev_ws, size_t ws_bytes,
               void* hip_stream, rte_handle** out) {
  using namespace rte;
  if (!out) return RTE_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg) || !med || !med->mu_a || !med->mu_s || !med->g) return RTE_EINVAL;
  const int n = cfg->n, N = cfg->order_N, M = (N + 1) * (N + 1);
  const size_t V = size_t(n) * n * n;
  for (size_t i = 0; i < V; ++i) {
    if (!(med->mu_a[i] >= 0) || !(med->mu_s[i] >= 0) || !std::isfinite(med->mu_a[i]) ||
        !std::isfinite(med->mu_s[i]) || !(med->g[i] > -1.0 && med->g[i] < 1.0))
      return RTE_EINVAL;
  }
  for (int p = 0; p < cfg->n_det; ++p)
    if (cfg->det_index[p] < 0 || size_t(cfg->det_index[p]) >= V) return RTE_EINVAL;
  const bool has_q = med->q != nullptr;
  const Layout L = layout_of(cfg, has_q);
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) != 0 || ws_bytes < L.total) return RTE_ENOMEM;

  std::vector<double> coef;
  if (!coupling_slots(N, coef)) return RTE_EINVAL;
  std::vector<double> sig;
  std::vector<uint8_t> inside;
  potentials(n, N, cfg->pml_width, cfg->pml_mu0, cfg->pml_mu1, med->mu_a, med->mu_s, med->g, sig, inside);

  rte_handle* h = new (std::nothrow) rte_handle();
  if (!h) return RTE_ENOMEM;
  h->cfg = *cfg;
  h->n = n;
  h->N = N;
  h->M = M;
  h->prec = cfg->precision;
  h->dt = cfg->dt_ps > 0 ? cfg->dt_ps : 0.2 * cfg->dx_mm / cfg->c_mm_ps;
  h->has_q = has_q;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = reinterpret_cast<unsigned char*>(dev_ws);
  h->lay = L;
  h->graph_ready = false;
  const char* ng = std::getenv("RTE_NO_GRAPH");
  h->use_graph = (h->stream != nullptr) && !(ng && ng[0] == '1');
  Geo& g = h->geo;
  g.n = n;
  g.H = n / 2;
  g.Kp = n / 2 + 1;
  g.M = M;
  g.N = N;
  g.plan_row = fft_plan(n / 2);
  g.plan_col = fft_plan(n);
  const size_t cs = cfg->precision == RTE_FP64 ? 16 : 8;
  const size_t col_bytes = size_t(M) * n * cs;
  int TT = 1;
  while (TT < 16 && TT * 2 <= g.Kp && (size_t(2 * TT) * col_bytes + n * cs) <= 64 * 1024) TT *= 2;
  g.TT = TT;
  g.ntile = (g.Kp + TT - 1) / TT;
  h->lds_plane = (size_t(n) * g.Kp + n) * cs;
  h->lds_z = size_t(TT) * col_bytes + n * cs;
  if (h->lds_z > 160 * 1024 || g.plan_row == 0 || g.plan_col == 0) {
    delete h;
    return RTE_EINVAL;
  }
  // the reduction in the last inverse pass reuses the plane LDS
  h->lds_plane = std::max(h->lds_plane, size_t(2 * 256 * 8));

  hipError_t e = dispatch<LdsFn>(h);
  int rc = to_code(e);
  if (!rc) rc = h->prec == RTE_FP64 ? upload_tables_t<double>(h, med, sig, inside, coef)
                                    : upload_tables_t<float>(h, med, sig, inside, coef);
  if (!rc) rc = h->prec == RTE_FP64 ? upload_state_t<double>(h, med->psi0) : upload_state_t<float>(h, med->psi0);
  if (!rc) {
    std::vector<double> sig0(sig.begin(), sig.begin() + V);
    rc = reset_run_state(h, growth_limit_of(h, med->psi0, med->q, sig0));
  }
  h->cfg.det_index = nullptr;
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return RTE_OK;
}

int rte_step(rte_handle* h, int64_t nsteps) {
  if (!h || nsteps < 0) return RTE_EINVAL;
  return rte::enqueue_steps(h, nsteps);
}

int rte_run(rte_handle* h, int64_t max_steps, double steady_tol, int64_t* steps_taken) {
  using namespace rte;
  if (!h || max_steps < 0 || !(steady_tol > 0)) return RTE_EINVAL;
  Ctl c;
  int rc = read_ctl(h, &c);
  if (rc) return rc;
  const long long start = c.step;
  c.tol = steady_tol;
  if (c.stop == 1) c.stop = 0;
  rc = write_ctl(h, &c);
  if (rc) return rc;
  int64_t done = 0;
  const int64_t chunk = 64;
  while (done < max_steps) {
    const int64_t k = std::min(chunk, max_steps - done);
    rc = enqueue_steps(h, k);
    if (rc) return rc;
    rc = read_ctl(h, &c);
    if (rc) return rc;
    done += k;
    if (c.stop) break;
  }
  if (steps_taken) *steps_taken = c.step - start;
  const int stop = c.stop;
  c.tol = 0.0;
  if (c.stop == 1) c.stop = 0;
  rc = write_ctl(h, &c);
  if (rc) return rc;
  return stop == 2 ? RTE_EUNSTABLE : RTE_OK;
}

int rte_fluence(rte_handle* h, int which, double* out, size_t len) {
  using namespace rte;
  if (!h || !out) return RTE_EINVAL;
  const size_t V = size_t(h->n) * h->n * h->n;
  if (len < V) return RTE_EINVAL;
  if (which == RTE_FLUENCE_NOW)
    return h->prec == RTE_FP64 ? download_t<double>(h, h->lay.u, V, out) : download_t<float>(h, h->lay.u, V, out);
  if (which == RTE_FLUENCE_INTEGRATED) return download_t<double>(h, h->lay.phi_int, V, out);
  return RTE_EINVAL;
}

int rte_steps_done(rte_handle* h, int64_t* steps) {
  if (!h || !steps) return RTE_EINVAL;
  rte::Ctl c;
  int rc = rte::read_ctl(h, &c);
  if (rc) return rc;
  *steps = c.step;
  return c.stop == 2 ? RTE_EUNSTABLE : RTE_OK;
}

int rte_readings(rte_handle* h, double* out, size_t len, int64_t* rows) {
  if (!h || (!out && len)) return RTE_EINVAL;
  rte::Ctl c;
  int rc = rte::read_ctl(h, &c);
  if (rc) return rc;
  int64_t r = std::min<int64_t>(c.step, h->cfg.record_steps);
  if (h->cfg.n_det == 0) r = 0;
  else r = std::min<int64_t>(r, int64_t(len / size_t(h->cfg.n_det)));
  if (rows) *rows = r;
  if (r == 0) return RTE_OK;
  return rte::download_t<double>(h, h->lay.readings, size_t(r) * h->cfg.n_det, out);
}

int rte_residuals(rte_handle* h, double* out, size_t len, int64_t* rows) {
  if (!h || (!out && len)) return RTE_EINVAL;
  rte::Ctl c;
  int rc = rte::read_ctl(h, &c);
  if (rc) return rc;
  int64_t r = std::min<int64_t>(std::min<int64_t>(c.step, h->cfg.record_steps), int64_t(len));
  if (rows) *rows = r;
  if (r == 0) return RTE_OK;
  return rte::download_t<double>(h, h->lay.resid, size_t(r), out);
}

int rte_get_state(rte_handle* h, double* out, size_t len) {
  if (!h || !out) return RTE_EINVAL;
  const size_t cnt = size_t(h->M) * h->n * h->n * h->n;
  if (len < cnt) return RTE_EINVAL;
  return h->prec == RTE_FP64 ? rte::download_t<double>(h, h->lay.u, cnt, out)
                             : rte::download_t<float>(h, h->lay.u, cnt, out);
}

int rte_set_state(rte_handle* h, const double* in, size_t len) {
  if (!h || !in) return RTE_EINVAL;
  const size_t cnt = size_t(h->M) * h->n * h->n * h->n;
  if (len < cnt) return RTE_EINVAL;
  rte::Ctl c;
  int rc = rte::read_ctl(h, &c);
  if (rc) return rc;
  rc = h->prec == RTE_FP64 ? rte::upload_state_t<double>(h, in) : rte::upload_state_t<float>(h, in);
  if (rc) return rc;
  return rte::reset_run_state(h, c.growth_limit);
}

int rte_coupling_dense(int32_t order_N, double* bx, double* by, double* bz) {
  if (!bx || !by || !bz) return RTE_EINVAL;
  std::vector<double> X, Y, Z;
  if (!rte::coupling_dense(order_N, X, Y, Z)) return RTE_EINVAL;
  std::memcpy(bx, X.data(), X.size() * 8);
  std::memcpy(by, Y.data(), Y.size() * 8);
  std::memcpy(bz, Z.data(), Z.size() * 8);
  return RTE_OK;
}

int rte_profile_kernels(rte_handle* h, int64_t nsteps, double* ms, int64_t* counts) {
  using namespace rte;
  if (!h || !ms || !counts || nsteps < 0) return RTE_EINVAL;
  constexpr int kLaunches = 13;
  hipEvent_t ev[kLaunches + 1];
  for (int i = 0; i <= kLaunches; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) return RTE_EDEVICE;
  for (int c = 0; c < 4; ++c) {
    ms[c] = 0.0;
    counts[c] = 0;
  }
  int rc = RTE_OK;
  for (int64_t s = 0; s < nsteps && rc == RTE_OK; ++s) {
    g_prof_events = ev;
    hipError_t e = dispatch<ProfStepFn>(h);
    g_prof_events = nullptr;
    if (e == hipSuccess) e = hipEventSynchronize(ev[kLaunches]);
    if (e != hipSuccess) {
      rc = RTE_EDEVICE;
      break;
    }
    for (int i = 0; i < kLaunches; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) {
        rc = RTE_EDEVICE;
        break;
      }
      const int cls = i == kLaunches - 1 ? 3 : i % 3;
      ms[cls] += t;
      counts[cls] += 1;
    }
  }
  for (int i = 0; i <= kLaunches; ++i) (void)hipEventDestroy(ev[i]);
  return rc;
}

void rte_destroy(rte_handle* h) {
  if (!h) return;
  if (h->graph_ready) {
    (void)hipGraphExecDestroy(h->exec);
    (void)hipGraphDestroy(h->graph);
  }
  delete h;
}

const char* rte_strerror(int code) {
  switch (code) {
    case RTE_OK: return "ok";
    case RTE_EINVAL: return "invalid argument or unsupported configuration";
    case RTE_ENOMEM: return "workspace too small or misaligned";
    case RTE_EUNSTABLE: return "non-finite or runaway fluence detected";
    case RTE_EDEVICE: return "HIP runtime error";
    default: return "unknown error";
  }
}

}  // extern "C"
