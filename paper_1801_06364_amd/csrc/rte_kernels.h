// Kernels of one RK stage of the P_N stepper, specialised at compile time
// for the grid size NN (points per axis) and the working precision T.
//
// One RK stage evaluates f(v) = c (w - Sigma_l v + q) with the streaming
// term w = -(Bx d/dx + By d/dy + Bz d/dz) v of eq. (6), evaluated
// spectrally (eqs. 7-10; sign form of eqs. 1 and 6). Since the B_j are
// constant matrices, the z derivative can be taken per moment before the
// moments are mixed, which keeps every sweep over HBM coalesced:
//   F  k_fwd_plane  per (moment, z-plane): x real-to-complex FFT and y FFT of
//                   the plane in LDS -> xy spectrum S [b][z][ky][kx];
//   D  k_pencil     per (moment, ky, 16 kx columns): z FFT, times i k_z,
//                   inverse z FFT -> D = d/dz S (xy spectral, z physical);
//   C  k_couple     per spectral point, all moments in registers:
//                   W = -i (kx Bx + ky By) S - Bz D, written over S
//                   (k_couple_rt for orders beyond registers: a run-time
//                   slot table, W to a separate buffer);
//   P  k_inv_plane  per (moment, z-plane): inverse y FFT, complex-to-real x
//                   FFT and the fused pointwise epilogue (loss, in-scatter,
//                   boundary layer, source, RK combine; after the last stage
//                   also the integrated fluence and fluence-change partials);
//                   in a time step it also transforms its output plane
//                   forward (F of the next stage, fused).
// k_end_step closes each step (detector readings, residual, stop flags).
// Grids of 256 points split F and P into row and y-pencil passes. Also
// here: the exact propagation in homogeneous media (k_expo on the full 3D
// spectrum) and the vector kernels of the Krylov steady-state solver.
//
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2. Tiles that share data (neighbouring kx tiles in D, the moments of one
// z-plane that read the same loss map in P) are remapped so that
// consecutive logical tiles run on the same XCD. Planes and pencils sit in
// LDS in bank-swizzled layouts (PlaneLayout, fft_swz) so that the Stockham
// stages run without bank conflicts.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "rte_coupling_ct.h"
#include "rte_fft.h"
#include "rte_internal.h"

#ifndef RTE_PBLOCK
#define RTE_PBLOCK 512
#endif
#ifndef RTE_ZBLOCK
#define RTE_ZBLOCK 256
#endif
#ifndef RTE_CBLOCK
#define RTE_CBLOCK 256
#endif

namespace rte {

constexpr int kBlock = 256;        // end-of-step kernel
constexpr int kPBlock = RTE_PBLOCK;  // plane passes
constexpr int kZBlock = RTE_ZBLOCK;  // z-derivative pass
constexpr int kCBlock = RTE_CBLOCK;  // coupling pass
#ifndef RTE_FPPW
#define RTE_FPPW 1
#endif
constexpr int kFwdPlanes = RTE_FPPW;  // planes per forward-plane workgroup
constexpr int kXcds = 8;

// Physical block id -> logical tile: XCD x (= bid % 8) receives a contiguous
// range of logical tiles, in dispatch order.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  const int x = bid % kXcds, local = bid / kXcds;
  return x * per + (x < rem ? x : rem) + local;
}

// Batched launches: grid row blockIdx.y is a slot whose workspace lies
// bs bytes after the previous slot's; every pointer of the launch moves by
// blockIdx.y * bs (null pointers stay null). bs = 0: a single solve.
template <typename P>
__device__ __forceinline__ P* slot_ptr(P* p, long long bs) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  if (bs == 0 || p == nullptr) return p;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(p) + (long long)blockIdx.y * bs);
}

template <int NN> struct GridC {
  static constexpr int n = NN;
  static constexpr int H = NN / 2;
  static constexpr int E = elems_per_lane(NN);
  static_assert(elems_per_lane(NN / 2) == elems_per_lane(NN), "row/column lane shape");
};

// LDS layout of RB packed spectral rows of H = n/2 complex values (a whole
// plane when RB = n). Default: row pitch H + 1 (odd, so the strided column
// accesses of the y transform spread over the banks). The 128-point plane
// is transformed along both axes by radix-8 Stockham stages whose stride-8
// writes alias on that layout; it uses pitch H + 8 and stores column c of
// row r at c ^ ((c >> 3) & 7) ^ x(r >> 1), where the row term
// x(q) = ((q ^ (q >> 3)) & 7) | ((q & 4) << 1) spreads the 16 rows that one
// LDS cycle touches in every y stage over distinct banks and keeps the two
// rows one cycle touches in the x stages on complementary halves. Row blocks
// of the large-grid kernels (RB < n, x transforms only) use the in-row
// swizzle of contiguous FFTs.
template <int NN, int RB> struct PlaneLayout {
  static constexpr int H = NN / 2;
  static constexpr bool SWZ = (NN == 128 && RB == NN);
  static constexpr bool ROWSWZ = (RB < NN && H >= 64 && (H & (H - 1)) == 0);
  static constexpr int PITCH = SWZ ? H + 8 : H + 1;
  static constexpr int SIZE = RB * PITCH;
  // column swizzle and row-pair term of the 128-point plane (both linear
  // over GF(2), so they split over disjoint index parts)
  static __device__ __forceinline__ int cs(int c) { return c ^ ((c >> 3) & 7); }
  static __device__ __forceinline__ int rx(int r) {
    const int q = r >> 1;
    return ((q ^ (q >> 3)) & 7) | ((q << 1) & 8);
  }
  static __device__ __forceinline__ int pos(int row, int col) {
    if constexpr (SWZ) return row * PITCH + (cs(col) ^ rx(row));
    else if constexpr (ROWSWZ) return row * PITCH + fft_swz<H>(col);
    else return row * PITCH + col;
  }
  // x transforms of the 128-point plane: FFT f = row f, element i = column i
  template <typename V> struct XSwz {
    static constexpr bool kXor = true;
    V* p0;
    struct Lane { V* q; int x; };
    __device__ __forceinline__ Lane lane(int f, int a) const { return {p0 + f * PITCH, cs(a) ^ rx(f)}; }
    __device__ __forceinline__ V* elem(Lane l, int b) const { return l.q + (l.x ^ cs(b)); }
  };
  // y transforms of the 128-point plane: FFT f = column f, element i = row i
  template <typename V> struct YSwz {
    static constexpr bool kXor = true;
    V* p0;
    struct Lane { V* q; int x; };
    __device__ __forceinline__ Lane lane(int f, int a) const { return {p0 + a * PITCH, cs(f) ^ rx(a)}; }
    __device__ __forceinline__ V* elem(Lane l, int b) const { return l.q + b * PITCH + (l.x ^ rx(b)); }
  };
  // accessors of the row (x) and column (y) transforms
  template <typename V> static __device__ __forceinline__ auto xat(V* pl) {
    if constexpr (SWZ) return XSwz<V>{pl};
    else if constexpr (ROWSWZ) return SwzAt<V, H, PITCH>{pl};
    else return AffineAt<V, PITCH, 1>{pl};
  }
  template <typename V> static __device__ __forceinline__ auto yat(V* pl) {
    if constexpr (SWZ) return YSwz<V>{pl};
    else return AffineAt<V, 1, PITCH>{pl};
  }
};

template <typename T, int NN>
constexpr size_t plane_lds() {
  // twiddles (n) + the plane
  const size_t b = (size_t(PlaneLayout<NN, NN>::SIZE) + NN) * 2 * sizeof(T);
  return b < 2 * kPBlock * 8 ? 2 * kPBlock * 8 : b;
}
// ---------------------------------------------------------- F: forward ---

// Real-to-complex split of RB rows of packed x transforms Z (layout Lay):
// X_k = (Z_k + conj Z_m)/2 - i w_k (Z_k - conj Z_m)/2, m = H - k,
// w_k = exp(-2 pi i k / n); column 0 becomes the real pair (X_0, X_{n/2}).
// H/2 lanes per row: lane k > 0 does the pair (k, H - k), lane 0 column 0
// and the self-paired column H/2.
template <typename V, typename T, int NN, int RB, typename Lay, int BLOCK>
__device__ __forceinline__ void r2c_split(V* pl, const V* tw) {
  constexpr int H = NN / 2, half = H / 2;
  for (int i = threadIdx.x; i < RB * half; i += BLOCK) {
    const int y = i / half, kk = i - y * half;
    auto row = [&](int c) -> V& { return pl[Lay::pos(y, c)]; };
    auto pair = [&](int k) {
      const int m = H - k;
      const V zk = row(k), zm = row(m);
      const V zmc = cconj(zm), zkc = cconj(zk);
      const V ek = cscale(cadd(zk, zmc), T(0.5));
      const V ok = cmul_i<V, -1>(cscale(csub(zk, zmc), T(0.5)));
      row(k) = cadd(ek, cmul(tw[k], ok));
      if (m != k) {
        const V em = cscale(cadd(zm, zkc), T(0.5));
        const V om = cmul_i<V, -1>(cscale(csub(zm, zkc), T(0.5)));
        row(m) = cadd(em, cmul(tw[m], om));
      }
    };
    if (kk == 0) {
      const V z0 = row(0);
      row(0) = cmk<V>(z0.x + z0.y, z0.x - z0.y);   // packed (X_0, X_{n/2})
      pair(half);
    } else {
      pair(kk);
    }
  }
}

// The x transform of a real row has real kx = 0 and kx = n/2 entries; both
// have zero x wavenumber (the Nyquist one by the Nyquist rule), so every
// later operator treats them alike and they travel packed as one complex
// column kx = 0 holding (X_0, X_{n/2}). The half spectrum is therefore
// exactly n/2 columns wide: [b][z][ky][kx], kx in [0, n/2).
// Forward transform of one real plane held in LDS as n rows of H packed
// complex values (PlaneLayout): x real-to-complex FFT with the
// kx = 0 / n/2 packing, then y FFT of the H columns. Callers synchronise
// before (plane written) and read the spectrum after (ends synchronised).
template <typename V, typename T, int NN, int BLOCK>
__device__ __forceinline__ void forward_plane_lds(V* pl, const V* tw) {
  constexpr int n = NN, H = NN / 2;
  using Lay = PlaneLayout<NN, NN>;
  // x: n packed rows of length H (twiddle table of length n, stride 2)
  fft_batch<V, H, 2 * H, -1, n, BLOCK>(tw, Lay::xat(pl));
  __syncthreads();
  r2c_split<V, T, NN, n, Lay, BLOCK>(pl, tw);
  __syncthreads();
  // y: H columns of length n
  fft_batch<V, n, n, -1, H, BLOCK>(tw, Lay::yat(pl));
  __syncthreads();
}

template <typename T, int NN>
__global__ void __launch_bounds__(kPBlock)
k_fwd_plane(const T* __restrict__ src, typename cplx_of<T>::type* __restrict__ spec,
            const typename cplx_of<T>::type* __restrict__ twg, const Ctl* __restrict__ ctl, int nplanes) {
  using V = typename cplx_of<T>::type;
  using G = GridC<NN>;
  constexpr int n = NN, H = G::H;
  using Lay = PlaneLayout<NN, NN>;
  constexpr int CNT = n * H;                     // complex values per packed plane
  constexpr int ITER = (CNT + kPBlock - 1) / kPBlock;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + n;
  for (int i = threadIdx.x; i < n; i += kPBlock) tw[i] = twg[i];
  // kFwdPlanes consecutive planes per workgroup; the next plane's loads are
  // issued into registers before the current plane's FFTs, so HBM traffic
  // overlaps the LDS work
  const int p0 = blockIdx.x * kFwdPlanes;
  V pre[ITER];
  auto gload = [&](int plane) {
    const V* s = reinterpret_cast<const V*>(src + size_t(plane) * n * n);
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int i = int(threadIdx.x) + it * kPBlock;
      if (CNT % kPBlock == 0 || i < CNT) pre[it] = s[i];
    }
  };
  gload(p0);
  for (int k = 0; k < kFwdPlanes; ++k) {
    const int plane = p0 + k;                    // b * n + z
    if (plane >= nplanes) break;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int i = int(threadIdx.x) + it * kPBlock;
      if (CNT % kPBlock == 0 || i < CNT) pl[Lay::pos(i / H, i % H)] = pre[it];
    }
    __syncthreads();
    if (k + 1 < kFwdPlanes && plane + 1 < nplanes) gload(plane + 1);
    forward_plane_lds<V, T, NN, kPBlock>(pl, tw);
    V* dst = spec + size_t(plane) * n * H;
    staged_copy<n * H, kPBlock>([&](int i) { return pl[Lay::pos(i / H, i % H)]; },
                                [&](int i, V x) { dst[i] = x; });
    __syncthreads();
  }
}

// ------------------------------------------------ pencil passes (D, Y) ---

// Pencils of 16 (or fewer) kx columns of the xy spectrum along one axis, all
// points of that axis, staged in LDS with a padded column pitch (a 16-wide
// FP32 complex row segment is one 128-byte line).
//   PENCIL_ZDERIV: axis z; forward FFT, times i k_z / n (Nyquist k_z = 0),
//                  inverse FFT, written to the derivative buffer
//                  (tile = (b, ky, kx-tile));
//   PENCIL_YFWD / PENCIL_YINV: axis y, forward / inverse FFT in place
//                  (tile = (b, z, kx-tile); used where a whole plane does
//                  not fit in LDS);
//   PENCIL_ZFWD / PENCIL_ZINV: axis z, forward / inverse FFT in place (the
//                  full 3D spectrum of the exact propagation).
enum { PENCIL_ZDERIV = 0, PENCIL_YFWD = 1, PENCIL_YINV = 2, PENCIL_ZFWD = 3, PENCIL_ZINV = 4 };
constexpr bool pencil_z(int mode) { return mode == PENCIL_ZDERIV || mode == PENCIL_ZFWD || mode == PENCIL_ZINV; }
constexpr bool pencil_inverse(int mode) { return mode == PENCIL_YINV || mode == PENCIL_ZINV; }

#ifndef RTE_ZDW
#define RTE_ZDW 16
#endif
constexpr int zd_width(int H) {
  int t = RTE_ZDW;
  while (t > 1 && H % t != 0) t /= 2;
  return t;
}
template <typename T, int NN> struct ZdShape {
  static constexpr int TZ = zd_width(NN / 2);   // largest power of two <= RTE_ZDW dividing n/2
  static constexpr int PITCH = NN + 1;
  static constexpr int NTILE = (NN / 2) / TZ;
  static_assert(NTILE * TZ == NN / 2, "tiles must cover the half spectrum");
};

template <typename T, int NN>
constexpr size_t zd_lds() {
  using Z = ZdShape<T, NN>;
  return (size_t(Z::TZ) * Z::PITCH + NN) * 2 * sizeof(T);
}

template <typename T, int NN, int MODE>
__global__ void __launch_bounds__(kZBlock)
k_pencil(const typename cplx_of<T>::type* src, typename cplx_of<T>::type* dst,   // may alias (in place)
         const typename cplx_of<T>::type* __restrict__ twg, const T* __restrict__ kv,
         const Ctl* __restrict__ ctl, long long bs = 0) {
  using V = typename cplx_of<T>::type;
  using Z = ZdShape<T, NN>;
  constexpr int n = NN, H = NN / 2, TZ = Z::TZ, PITCH = Z::PITCH;
  // element stride along the pencil axis in the [b][z][ky][kx] spectrum
  constexpr size_t AX = pencil_z(MODE) ? size_t(n) * H : size_t(H);
  src = slot_ptr(src, bs);
  dst = slot_ptr(dst, bs);
  twg = slot_ptr(twg, bs);
  kv = slot_ptr(kv, bs);
  ctl = slot_ptr(ctl, bs);
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* col = tw + n;
  // logical tile = (b * n + w) * NTILE + kx-tile, w = ky (z pencils) or z
  // (y pencils); neighbouring tiles share an XCD
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bw = tile / Z::NTILE;
  const int kx0 = (tile - bw * Z::NTILE) * TZ;
  const int b = bw / n, w = bw - b * n;
  const size_t base = pencil_z(MODE) ? (size_t(b) * n * n + w) * H + kx0
                                            : (size_t(b) * n + w) * size_t(n) * H + kx0;
  for (int i = threadIdx.x; i < n; i += kZBlock) tw[i] = twg[i];
  // element i of pencil f (bank-swizzled within the pencil)
  const SwzAt<V, n, PITCH> at{col};
  staged_copy<n * TZ, kZBlock>(
      [&](int i) { return src[base + size_t(i / TZ) * AX + (i % TZ)]; },
      [&](int i, V x) { col[(i % TZ) * PITCH + fft_swz<n>(i / TZ)] = x; });
  __syncthreads();
  if constexpr (pencil_inverse(MODE)) {
    fft_batch<V, n, n, +1, TZ, kZBlock>(tw, at);
  } else {
    fft_batch<V, n, n, -1, TZ, kZBlock>(tw, at);
  }
  if constexpr (MODE == PENCIL_ZDERIV) {
    __syncthreads();
    const T inv_n = T(1) / T(n);
    for (int i = threadIdx.x; i < n * TZ; i += kZBlock) {
      const int t = i / n, kz = i - t * n;
      V* e = col + t * PITCH + fft_swz<n>(kz);
      const T k = kv[kz] * inv_n;
      const V x = *e;
      *e = cmk<V>(-k * x.y, k * x.x);     // times i k_z / n
    }
    __syncthreads();
    fft_batch<V, n, n, +1, TZ, kZBlock>(tw, at);
  }
  __syncthreads();
  staged_copy<n * TZ, kZBlock>(
      [&](int i) { return col[(i % TZ) * PITCH + fft_swz<n>(i / TZ)]; },
      [&](int i, V x) { dst[base + size_t(i / TZ) * AX + (i % TZ)] = x; });
}

// --------------------------------------------- row passes (large grids) ---

// Forward x transform of RB rows (rows r = (b n + z) n + y of the real
// field) per workgroup: real-to-complex with the kx = 0 / n/2 packing, into
// the spectrum buffer as [b][z][y][kx].
template <int NN> struct RowShape {
  static constexpr int RB = 16;                       // rows per workgroup
  static_assert(NN % RB == 0, "rows of a block must share a plane");
};

template <typename T, int NN>
constexpr size_t rows_lds() {
  const size_t b = (size_t(PlaneLayout<NN, RowShape<NN>::RB>::SIZE) + NN) * 2 * sizeof(T);
  return b < 2 * kPBlock * 8 ? 2 * kPBlock * 8 : b;
}

template <typename T, int NN>
__global__ void __launch_bounds__(kZBlock)
k_rows_fwd(const T* __restrict__ src, typename cplx_of<T>::type* __restrict__ spec,
           const typename cplx_of<T>::type* __restrict__ twg, const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2, RB = RowShape<NN>::RB;
  using Lay = PlaneLayout<NN, RB>;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + n;
  const size_t r0 = size_t(blockIdx.x) * RB;
  for (int i = threadIdx.x; i < n; i += kZBlock) tw[i] = twg[i];
  const V* s = reinterpret_cast<const V*>(src + r0 * n);
  staged_copy<RB * H, kZBlock>([&](int i) { return s[i]; },
                               [&](int i, V x) { pl[Lay::pos(i / H, i % H)] = x; });
  __syncthreads();
  fft_batch<V, H, 2 * H, -1, RB, kZBlock>(tw, Lay::xat(pl));
  __syncthreads();
  r2c_split<V, T, NN, RB, Lay, kZBlock>(pl, tw);
  __syncthreads();
  V* dst = spec + r0 * H;
  staged_copy<RB * H, kZBlock>([&](int i) { return pl[Lay::pos(i / H, i % H)]; },
                               [&](int i, V x) { dst[i] = x; });
}

// --------------------------------------------------- C: moment coupling ---

// For one spectral point (kx, ky, z) the streaming term of eq. (10) in the
// real basis is
//   W_a = s * ( -i (kx Bx + ky By)[a,b] S_b  -  Bz[a,b] D_b ),
// S the moments' xy spectra, D their z derivatives. Bx and By join orders
// |m| and |m| +- 1, Bz only equal orders (eq. 6; the real basis mixes m and
// -m only). So the rows with even |m| read S at odd |m| and D at even |m|,
// and the rows with odd |m| the other halves: two threads per point, one per
// parity class P, read every input exactly once between them, and each
// writes its rows over the D entries that only it reads.
__host__ __device__ constexpr int m_parity(int a) {
  const int l = isqrt_c(a), m = a - l * l - l;
  return (m < 0 ? -m : m) & 1;
}
__host__ __device__ constexpr int parity_rows(int N, int P) {
  int c = 0;
  for (int a = 0; a < (N + 1) * (N + 1); ++a) c += m_parity(a) == P;
  return c;
}

template <typename V, typename T, int N, int A, int S, int P>
struct RowAccP {
  // acc: (re, im) of the x and y sums of S, then of the z sum of D; the
  // coefficients are instruction constants (one axis per non-zero)
  static __device__ __forceinline__ void run(const V* sr, const V* dr, T* acc) {
    constexpr int l = isqrt_c(A);
    constexpr int m = A - l * l - l;
    constexpr SlotList sl = slots_of(N, l, m);
    if constexpr (S < sl.count) {
      constexpr int b = sl.b[S];
      constexpr double c0 = ct::real_coef(N, 0, A, b);
      constexpr double c1 = ct::real_coef(N, 1, A, b);
      constexpr double c2 = ct::real_coef(N, 2, A, b);
      static_assert((c0 == 0.0 && c1 == 0.0) || m_parity(b) != P, "x, y coupling within one |m| parity");
      static_assert(c2 == 0.0 || m_parity(b) == P, "z coupling across |m| parities");
      if constexpr (c0 != 0.0) {
        acc[0] += T(c0) * sr[b].x;
        acc[1] += T(c0) * sr[b].y;
      }
      if constexpr (c1 != 0.0) {
        acc[2] += T(c1) * sr[b].x;
        acc[3] += T(c1) * sr[b].y;
      }
      if constexpr (c2 != 0.0) {
        acc[4] += T(c2) * dr[b].x;
        acc[5] += T(c2) * dr[b].y;
      }
      RowAccP<V, T, N, A, S + 1, P>::run(sr, dr, acc);
    }
  }
};

// Shell L's inputs of class P: S at the other parity, D at this one.
template <typename V, int N, int P, int B, int END>
struct LoadShellP {
  static __device__ __forceinline__ void run(V* sr, V* dr, const V* __restrict__ sp, const V* dp, size_t ms) {
    if constexpr (B < END) {
      if constexpr (m_parity(B) != P) sr[B] = sp[B * ms];
      else dr[B] = dp[B * ms];
      LoadShellP<V, N, P, B + 1, END>::run(sr, dr, sp, dp, ms);
    }
  }
};
template <typename V, int L, int N, int P>
__device__ __forceinline__ void load_shell_p(V* sr, V* dr, const V* __restrict__ sp, const V* dp, size_t ms) {
  if constexpr (L <= N) LoadShellP<V, N, P, L * L, (L + 1) * (L + 1)>::run(sr, dr, sp, dp, ms);
}

// Rows in shell order a = l^2 + l + m. Output shell l reads input shells
// l - 1 and l + 1 only, so shell l + 1 is loaded when output shell l starts;
// a row's own D entry was loaded one shell earlier, before the row is
// written over it. At most three shells need to be live in registers (FP32
// P_7: 110 registers; a scheduling barrier before each shell's loads kept it
// at 108 but measured 1% slower).
template <typename V, typename T, int N, int A, int P>
struct RowsP {
  static __device__ __forceinline__ void run(V* sr, V* dr, const V* __restrict__ sp, V* dp, size_t ms, T kx,
                                             T ky, T sc) {
    if constexpr (A < (N + 1) * (N + 1)) {
      constexpr int l = isqrt_c(A);
      if constexpr (A == l * l && l >= 1) load_shell_p<V, l + 1, N, P>(sr, dr, sp, dp, ms);
      if constexpr (m_parity(A) == P) {
        T acc[6] = {0, 0, 0, 0, 0, 0};
        RowAccP<V, T, N, A, 0, P>::run(sr, dr, acc);
        const T re = kx * acc[0] + ky * acc[2], im = kx * acc[1] + ky * acc[3];
        // -i (re + i im) - (dre + i dim)
        dp[A * ms] = cmk<V>(sc * (im - acc[4]), sc * (-re - acc[5]));
      }
      RowsP<V, T, N, A + 1, P>::run(sr, dr, sp, dp, ms, kx, ky, sc);
    }
  }
};

template <typename V, typename T, int N, int P>
__device__ __forceinline__ void couple_point(const V* __restrict__ sp, V* dp, size_t ms, T kx, T ky, T sc) {
  constexpr int M = (N + 1) * (N + 1);
  V sr[M], dr[M];
  load_shell_p<V, 0, N, P>(sr, dr, sp, dp, ms);
  load_shell_p<V, 1, N, P>(sr, dr, sp, dp, ms);
  RowsP<V, T, N, 0, P>::run(sr, dr, sp, dp, ms, kx, ky, sc);
}

// Two blocks per kCBlock spectral points of the (z, ky) rows, one per parity
// class (uniform per wavefront); the moments of a point are strided by
// n^2 H. Coalesced along kx. W replaces D in dspec.
template <typename T, int NN, int N>
__global__ void __launch_bounds__(kCBlock)
k_couple(const typename cplx_of<T>::type* __restrict__ spec, typename cplx_of<T>::type* dspec,
         const T* __restrict__ kv, T sc, const Ctl* __restrict__ ctl, long long bs = 0) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2;
  constexpr size_t MS = size_t(n) * n * H;      // moment stride
  spec = slot_ptr(spec, bs);
  dspec = slot_ptr(dspec, bs);
  kv = slot_ptr(kv, bs);
  ctl = slot_ptr(ctl, bs);
  if (ctl->stop) return;
  const int cls = blockIdx.x & 1;
  const int pt = (blockIdx.x >> 1) * kCBlock + threadIdx.x;   // (z * n + ky) * H + kx
  if (pt >= n * n * H) return;
  const T kx = kv[pt % H], ky = kv[(pt / H) % n];
  if (cls == 0) {
    couple_point<V, T, N, 0>(spec + pt, dspec + pt, MS, kx, ky, sc);
  } else if constexpr (parity_rows(N, 1) > 0) {
    couple_point<V, T, N, 1>(spec + pt, dspec + pt, MS, kx, ky, sc);
  }
}

// High orders (more moments than registers hold): one thread per spectral
// point and row slice (blockIdx.y: the order groups |m| = g, g + kRtSlices,
// ..., so that the small grids of high orders still give every SIMD several
// wavefronts) walks its rows with the slot table, reading each input from
// the spectrum (neighbouring shells stay in the caches across rows) and
// writing W to a separate buffer, since later rows still need the inputs. All kMaxSlots
// loads of a row are issued before any is used (a padding slot, code -1,
// re-reads the row's first input and adds nothing), so a row costs one
// memory latency instead of one per input. Rows go by order group, degree
// ascending, (l, g) then (l, -g): their inputs are the degrees l +- 1 at
// orders g and g +- 1, so rows l and l + 2 of a group share half of them
// while they are still in L2 (and (l, +-g) share them in L1).
constexpr int kRtSlices = 4;

template <typename T, int NN>
__global__ void __launch_bounds__(kCBlock)
k_couple_rt(const typename cplx_of<T>::type* __restrict__ spec,
            const typename cplx_of<T>::type* __restrict__ dspec, typename cplx_of<T>::type* __restrict__ out,
            const T* __restrict__ kv, const int* __restrict__ code, const T* __restrict__ val, int M, T sc,
            const Ctl* __restrict__ ctl) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2;
  constexpr size_t MS = size_t(n) * n * H;
  if (ctl->stop) return;
  const int pt = blockIdx.x * kCBlock + threadIdx.x;   // (z * n + ky) * H + kx
  if (pt >= n * n * H) return;
  const int N = isqrt_c(M - 1);
  const T kx = kv[pt % H], ky = kv[(pt / H) % n];
  for (int g = int(blockIdx.y); g <= N; g += kRtSlices)
  for (int l = g; l <= N; ++l)
  for (int sg = 0; sg < (g > 0 ? 2 : 1); ++sg) {
    const int a = l * l + l + (sg ? -g : g);
    const int* cr = code + size_t(a) * kMaxSlots;
    const T* vr = val + size_t(a) * kMaxSlots;
    const int c0 = max(cr[0], 0);   // (moment 0, x) if a row had no slot
    V x[kMaxSlots];
    int ax[kMaxSlots];
    T w[kMaxSlots];
#pragma unroll
    for (int k = 0; k < kMaxSlots; ++k) {
      const int c = cr[k];
      const int cc = c >= 0 ? c : c0;
      ax[k] = c >= 0 ? (c & 3) : 3;
      w[k] = vr[k];
      x[k] = ((cc & 3) == 2 ? dspec : spec)[size_t(cc >> 2) * MS + pt];
    }
    // per-axis weights by selects (no branches, so the weight loads stay
    // ahead of the input loads)
    T acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kMaxSlots; ++k) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T wd = ax[k] == d ? w[k] : T(0);
        acc[2 * d] += wd * x[k].x;
        acc[2 * d + 1] += wd * x[k].y;
      }
    }
    const T re = kx * acc[0] + ky * acc[2], im = kx * acc[1] + ky * acc[3];
    out[size_t(a) * MS + pt] = cmk<V>(sc * (im - acc[4]), sc * (-re - acc[5]));
  }
}

// ------------------------------------------- P: inverse + epilogue -------

// Complex-to-real merge of RB packed spectral rows in LDS (layout Lay):
// Z_k = (X_k + conj X_{H-k}) + i conj(w_k) (X_k - conj X_{H-k}); column 0
// carries the real pair (X_0, X_{n/2}).
template <typename V, typename T, int NN, int RB, typename Lay, int BLOCK>
__device__ __forceinline__ void c2r_merge(V* pl, const V* tw) {
  constexpr int H = NN / 2, half = H / 2;
  // H/2 lanes per row: lane k > 0 does the pair (k, H - k), lane 0 column 0
  // and the self-paired column H/2
  for (int i = threadIdx.x; i < RB * half; i += BLOCK) {
    const int y = i / half, kk = i - y * half;
    auto row = [&](int c) -> V& { return pl[Lay::pos(y, c)]; };
    auto pair = [&](int k) {
      const int m = H - k;
      const V xk = row(k), xm = row(m);
      const V xmc = cconj(xm), xkc = cconj(xk);
      row(k) = cadd(cadd(xk, xmc), cmul_i<V, +1>(cmul(cconj(tw[k]), csub(xk, xmc))));
      if (m != k) row(m) = cadd(cadd(xm, xkc), cmul_i<V, +1>(cmul(cconj(tw[m]), csub(xm, xkc))));
    };
    if (kk == 0) {
      const V p0 = row(0);
      row(0) = cmk<V>(p0.x + p0.y, p0.x - p0.y);
      pair(half);
    } else {
      pair(kk);
    }
  }
}

#ifndef RTE_EPI_UNROLL
#define RTE_EPI_UNROLL 16
#endif
#ifndef RTE_PWAVES
#define RTE_PWAVES 1
#endif
constexpr int kEpiUnroll = RTE_EPI_UNROLL;   // epilogue elements per thread with loads in flight
constexpr int kPWaves = RTE_PWAVES;          // minimum waves per SIMD asked of the plane passes

// Epilogue modes of the inverse pass.
enum { EPI_MID = 0, EPI_FIRST = 1, EPI_LAST = 2, EPI_ADJ = 3, EPI_EULER = 4, EPI_APPLY = 5, EPI_SET = 6 };

// Pointwise epilogue of RB rows starting at row y0 of plane (b, z), on
// (x_{2j}, x_{2j+1}) pairs:
//   forward stages  o = u + w + h (-Sigma_l v + q)   -> dst
//     (EPI_FIRST: v = u; EPI_LAST: also phi_int += dt o (FP64) for the
//     fluence moment and the partial sums of (o - u)^2 and o^2);
//   EPI_ADJ         o = w - h Sigma_l v  -> dst, and u += o (u is the
//     adjoint accumulator; no source term in the transposed operator);
//   EPI_EULER       first and last stage at once (v = u, o -> u, bookkeeping);
//   EPI_APPLY       o = -w + Sigma_l v -> dst with w = -S v (h = 1): the
//     steady-state operator A v = (S + Sigma) v, for which the steady state
//     solves A u = q;
//   EPI_SET         o = w -> dst (the transformed field itself).
template <typename V, typename T, int NN, int RB, typename Lay, int BLOCK, int MODE, bool KEEP = false>
__device__ __forceinline__ void epilogue(V* pl, int y0, int b, int z, const T* vin, T* u,
                                         T* dst, const T* __restrict__ sig, const T* __restrict__ q,
                                         bool hasq, T qs, double* __restrict__ phi_int, T h, double dt,
                                         double& acc_d, double& acc_o) {
  constexpr int n = NN, H = NN / 2;
  const int l = isqrt_c(b);
  const size_t poff = (size_t(b) * n + z) * n * n + size_t(y0) * n;
  const size_t voff = size_t(z) * n * n + size_t(y0) * n;
  const T* sg = sig + size_t(l) * n * n * n + voff;
#pragma unroll kEpiUnroll
  for (int i = threadIdx.x; i < RB * H; i += BLOCK) {
    const int y = i / H, j = i - y * H;
    const int e = y * n + 2 * j;
    const V w = pl[Lay::pos(y, j)];
    if constexpr (MODE == EPI_SET) {
      *reinterpret_cast<V*>(dst + poff + e) = w;
      continue;
    }
    const V uu = MODE == EPI_APPLY ? cmk<V>(T(0), T(0)) : *reinterpret_cast<const V*>(u + poff + e);
    const V vv = (MODE == EPI_FIRST || MODE == EPI_EULER) ? uu : *reinterpret_cast<const V*>(vin + poff + e);
    const V ss = *reinterpret_cast<const V*>(sg + e);
    T src0 = -ss.x * vv.x, src1 = -ss.y * vv.y;
    if (MODE != EPI_ADJ && hasq) {
      const V qq = *reinterpret_cast<const V*>(q + poff + e);
      src0 += qs * qq.x;
      src1 += qs * qq.y;
    }
    if constexpr (MODE == EPI_APPLY) {
      *reinterpret_cast<V*>(dst + poff + e) = cmk<V>(-w.x + ss.x * vv.x, -w.y + ss.y * vv.y);
      continue;
    }
    if constexpr (MODE == EPI_ADJ) {
      const V o = cmk<V>(w.x + h * src0, w.y + h * src1);
      *reinterpret_cast<V*>(dst + poff + e) = o;
      *reinterpret_cast<V*>(u + poff + e) = cmk<V>(uu.x + o.x, uu.y + o.y);
      continue;
    }
    const V o = cmk<V>(uu.x + w.x + h * src0, uu.y + w.y + h * src1);
    *reinterpret_cast<V*>(dst + poff + e) = o;
    if constexpr (KEEP) pl[Lay::pos(y, j)] = o;   // the output plane, for the fused forward transform
    if ((MODE == EPI_LAST || MODE == EPI_EULER) && b == 0) {
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
}

// Deterministic block sum of two FP64 values (fixed tree), written to out[0..1].
template <int BLOCK>
__device__ __forceinline__ void block_sum2(unsigned char* smem, double a, double c, double* out) {
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  red[threadIdx.x] = a;
  red[BLOCK + threadIdx.x] = c;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      red[BLOCK + threadIdx.x] += red[BLOCK + threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    out[1] = red[BLOCK];
  }
}

// Weight of the source in stage `stage` of a step: 1 for a constant source,
// else the step's row of the profile table (step1 - 1 if given, else the
// control block's step counter; past the table, its last row).
__device__ __forceinline__ double source_weight(const Ctl* __restrict__ ctl, int stage, long long step1) {
  if (ctl->qw == nullptr) return 1.0;
  long long r = step1 > 0 ? step1 - 1 : ctl->step;
  if (r >= ctl->qw_rows) r = ctl->qw_rows - 1;
  return ctl->qw[r * ctl->qw_cols + stage];
}

// FUSE: the stage output plane, still in LDS, is transformed forward at
// once (x r2c + y FFT) and written as the next stage's xy spectrum to fspec
// (which may be the spectrum just read: each workgroup owns its plane), so
// the next stage needs no separate forward pass.
template <typename T, int NN, int MODE, bool FUSE = false>
__global__ void __launch_bounds__(kPBlock, kPWaves)
k_inv_plane(const typename cplx_of<T>::type* spec, const T* vin, T* u, T* dst,
            const T* __restrict__ sig, const T* __restrict__ q, const int* __restrict__ qflag,
            double* __restrict__ phi_int, double* __restrict__ partial,
            const typename cplx_of<T>::type* __restrict__ twg, int M, T h, double dt,
            const Ctl* __restrict__ ctl, int stage, long long step1, typename cplx_of<T>::type* fspec,
            long long bs = 0) {
  using V = typename cplx_of<T>::type;
  using G = GridC<NN>;
  constexpr int n = NN, H = G::H;
  using Lay = PlaneLayout<NN, NN>;
  spec = slot_ptr(spec, bs);
  vin = slot_ptr(vin, bs);
  u = slot_ptr(u, bs);
  dst = slot_ptr(dst, bs);
  sig = slot_ptr(sig, bs);
  q = slot_ptr(q, bs);
  qflag = slot_ptr(qflag, bs);
  phi_int = slot_ptr(phi_int, bs);
  partial = slot_ptr(partial, bs);
  twg = slot_ptr(twg, bs);
  ctl = slot_ptr(ctl, bs);
  fspec = slot_ptr(fspec, bs);
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + n;
  // logical order z-major, moment-minor: moments of one z-plane (which
  // share the loss maps) run back to back on one XCD
  const int lt = xcd_tile(blockIdx.x, gridDim.x);
  const int z = lt / M, b = lt - z * M;
  const int plane = b * n + z;
  for (int i = threadIdx.x; i < n; i += kPBlock) tw[i] = twg[i];
  const V* srcp = spec + size_t(plane) * n * H;
  staged_copy<n * H, kPBlock>([&](int i) { return srcp[i]; },
                              [&](int i, V x) { pl[Lay::pos(i / H, i % H)] = x; });
  __syncthreads();
  fft_batch<V, n, n, +1, H, kPBlock>(tw, Lay::yat(pl));
  __syncthreads();
  c2r_merge<V, T, NN, n, Lay, kPBlock>(pl, tw);
  __syncthreads();
  fft_batch<V, H, 2 * H, +1, n, kPBlock>(tw, Lay::xat(pl));
  __syncthreads();
  double acc_d = 0.0, acc_o = 0.0;
  const bool hasq = (q != nullptr) && qflag[z];
  const T qs = hasq ? T(source_weight(ctl, stage, step1)) : T(0);
  epilogue<V, T, NN, n, Lay, kPBlock, MODE, FUSE>(pl, 0, b, z, vin, u, dst, sig, q, hasq, qs, phi_int, h, dt,
                                                 acc_d, acc_o);
  if constexpr (FUSE) {
    __syncthreads();
    forward_plane_lds<V, T, NN, kPBlock>(pl, tw);
    V* fd = fspec + size_t(plane) * n * H;
    staged_copy<n * H, kPBlock>([&](int i) { return pl[Lay::pos(i / H, i % H)]; },
                                [&](int i, V x) { fd[i] = x; });
  }
  // (block_sum2 reuses the LDS: it synchronises first)
  if ((MODE == EPI_LAST || MODE == EPI_EULER) && b == 0) block_sum2<kPBlock>(smem, acc_d, acc_o, partial + 2 * z);
}

// Inverse x transform + epilogue of RB rows per workgroup (grids whose
// plane does not fit in LDS; the y transform ran before as a pencil pass).
// Logical order (z, row block, moment) so moments sharing loss rows are
// neighbours on one XCD. FUSE: the output rows, still in LDS, are
// transformed forward at once (x real-to-complex, as k_rows_fwd) and
// written as the next stage's row spectrum to fspec (which may be the
// spectrum just read: each workgroup owns its rows), so the next stage
// needs no separate row pass.
template <typename T, int NN, int MODE, bool FUSE = false>
__global__ void __launch_bounds__(kZBlock)
k_rows_inv(const typename cplx_of<T>::type* spec, const T* vin, T* u, T* dst,
           const T* __restrict__ sig, const T* __restrict__ q, const int* __restrict__ qflag,
           double* __restrict__ phi_int, double* __restrict__ partial,
           const typename cplx_of<T>::type* __restrict__ twg, int M, T h, double dt,
           const Ctl* __restrict__ ctl, int stage, long long step1, typename cplx_of<T>::type* fspec = nullptr) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2, RB = RowShape<NN>::RB, NB = NN / RB;
  using Lay = PlaneLayout<NN, RB>;
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  V* tw = reinterpret_cast<V*>(smem);
  V* pl = tw + n;
  const int lt = xcd_tile(blockIdx.x, gridDim.x);
  const int b = lt % M, zy = lt / M;
  const int z = zy / NB, yb = zy - z * NB;
  const int y0 = yb * RB;
  for (int i = threadIdx.x; i < n; i += kZBlock) tw[i] = twg[i];
  const V* srcp = spec + ((size_t(b) * n + z) * n + y0) * H;
  staged_copy<RB * H, kZBlock>([&](int i) { return srcp[i]; },
                               [&](int i, V x) { pl[Lay::pos(i / H, i % H)] = x; });
  __syncthreads();
  c2r_merge<V, T, NN, RB, Lay, kZBlock>(pl, tw);
  __syncthreads();
  fft_batch<V, H, 2 * H, +1, RB, kZBlock>(tw, Lay::xat(pl));
  __syncthreads();
  double acc_d = 0.0, acc_o = 0.0;
  const bool hasq = (q != nullptr) && qflag[z];
  const T qs = hasq ? T(source_weight(ctl, stage, step1)) : T(0);
  epilogue<V, T, NN, RB, Lay, kZBlock, MODE, FUSE>(pl, y0, b, z, vin, u, dst, sig, q, hasq, qs, phi_int, h, dt,
                                                  acc_d, acc_o);
  if constexpr (FUSE) {
    __syncthreads();
    fft_batch<V, H, 2 * H, -1, RB, kZBlock>(tw, Lay::xat(pl));
    __syncthreads();
    r2c_split<V, T, NN, RB, Lay, kZBlock>(pl, tw);
    __syncthreads();
    V* fd = fspec + ((size_t(b) * n + z) * n + y0) * H;
    staged_copy<RB * H, kZBlock>([&](int i) { return pl[Lay::pos(i / H, i % H)]; },
                                 [&](int i, V x) { fd[i] = x; });
  }
  // (block_sum2 reuses the LDS: it synchronises first)
  if ((MODE == EPI_LAST || MODE == EPI_EULER) && b == 0) block_sum2<kZBlock>(smem, acc_d, acc_o, partial + 2 * zy);
}

// ------------------------------------------------------- end of step ---

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_end_step(const T* __restrict__ u, const long long* __restrict__ det, int ndet,
           double* __restrict__ readings, double* __restrict__ resid, long long cap,
           const double* __restrict__ partial, int npart, Ctl* ctl, long long bs = 0) {
  __shared__ double red[2 * kBlock];
  u = slot_ptr(u, bs);
  det = slot_ptr(det, bs);
  readings = slot_ptr(readings, bs);
  resid = slot_ptr(resid, bs);
  partial = slot_ptr(partial, bs);
  ctl = slot_ptr(ctl, bs);
  if (ctl->stop) return;
  const long long s = ctl->step;
  if (s < cap)
    for (int p = threadIdx.x; p < ndet; p += kBlock) readings[s * ndet + p] = double(u[det[p]]);
  // deterministic: fixed per-thread strides, then a fixed tree
  double pd = 0.0, po = 0.0;
  for (int i = threadIdx.x; i < npart; i += kBlock) {
    pd += partial[2 * i];
    po += partial[2 * i + 1];
  }
  red[threadIdx.x] = pd;
  red[kBlock + threadIdx.x] = po;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      red[kBlock + threadIdx.x] += red[kBlock + threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double d2 = red[0], o2 = red[kBlock];
    const double r = o2 > 0.0 ? sqrt(d2 / o2) : 0.0;
    if (s < cap) resid[s] = r;
    ctl->last_resid = r;
    ctl->last_norm2 = o2;
    ctl->step = s + 1;
    if (!isfinite(d2) || !isfinite(o2) || o2 > ctl->growth_limit) ctl->stop = 2;
    else if (ctl->tol > 0.0 && r < ctl->tol) ctl->stop = 1;
    else if (ctl->limit > 0 && s + 1 >= ctl->limit) ctl->stop = 3;
  }
}

// ------------------------------------------------------------ launch ---

// ------------------------------------------------------ adjoint helpers ---

// Gradient accumulation of one adjoint stage, one thread per voxel:
//   g_mu_a(r) += wgt * sum_a (2l+1) xs_a(r) y_a(r)
//   g_mu_s(r) += wgt * sum_a (1 - g(r)^l) (2l+1) xs_a(r) y_a(r)
// inside the real domain (gin(r) = g(r) there, > 1 in the layer, where the
// loss does not depend on mu_a, mu_s). xs is the (2l+1)-scaled adjoint of the
// stage output, y the forward stage input, wgt = -c a h (stage coefficient).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_grad(const T* __restrict__ xs, const T* __restrict__ y, const double* __restrict__ gin,
           double* __restrict__ gmua, double* __restrict__ gmus, int N, long long nvox, double wgt) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nvox) return;
  const double g = gin[r];
  if (g > 1.0) return;
  double sa = 0.0, ss = 0.0, gl = 1.0;
  for (int l = 0; l <= N; ++l) {
    double acc = 0.0;
    for (int m = -l; m <= l; ++m) {
      const long long a = l * l + l + m;
      acc += double(xs[a * nvox + r]) * double(y[a * nvox + r]);
    }
    acc *= double(2 * l + 1);
    sa += acc;
    ss += (1.0 - gl) * acc;
    gl *= g;
  }
  gmua[r] += wgt * sa;
  gmus[r] += wgt * ss;
}

// Adjoint source of the detector readings: lam_0(det_p) += dJ/dr[p].
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_inject(T* __restrict__ lam, const long long* __restrict__ det, const double* __restrict__ djdr,
             int ndet) {
  for (int p = threadIdx.x; p < ndet; p += kBlock) lam[det[p]] += T(djdr[p]);
}

// ------------------------------------------- media and states from HBM ---

// Per-degree loss inside the real domain, Sigma_l = mu_a + mu_s (1 - g^l),
// from device FP64 maps (the same FP64 arithmetic as the host construction,
// without contraction, rounded once); voxels of the absorbing layer (gin > 1)
// keep their loss, which does not depend on the medium.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_set_loss(T* __restrict__ sig, const double* __restrict__ mua, const double* __restrict__ mus,
           const double* __restrict__ gin, int N, long long V) {
#pragma clang fp contract(off)
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < V; v += (long long)gridDim.x * kBlock) {
    const double g = gin[v];
    if (!(g <= 1.0)) continue;
    const double a = mua[v], s = mus[v];
    double gl = 1.0;
    for (int l = 0; l <= N; ++l) {
      sig[(long long)l * V + v] = T(a + s * (1.0 - gl));
      gl *= g;
    }
  }
}

// u <- psi (device FP64, the `given` leading entries), zero beyond
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_set_state_f64(T* __restrict__ u, const double* __restrict__ psi, long long given, long long total) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total; i += (long long)gridDim.x * kBlock)
    u[i] = i < given ? T(psi[i]) : T(0);
}

// Runaway-growth threshold 1e16 (E + source_term + 1e-300) with E the
// (2l+1)-weighted energy of u (one workgroup, fixed partition and tree:
// deterministic); the same rule as the host-side threshold of a state set
// from host memory.
template <typename T>
__global__ void __launch_bounds__(1024)
k_growth_limit(const T* __restrict__ u, int M, long long V, double source_term, Ctl* __restrict__ ctl) {
  __shared__ double red[1024];
  double e = 0.0;
  for (int a = 0; a < M; ++a) {
    const double wt = double(2 * isqrt_c(a) + 1);
    double s = 0.0;
    for (long long i = threadIdx.x; i < V; i += 1024) {
      const double x = double(u[(long long)a * V + i]);
      s += x * x;
    }
    e += wt * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) ctl->growth_limit = 1e16 * (red[0] + source_term + 1e-300);
}

// ------------------------------------------------- Krylov vector kernels ---

// Weighted inner products <x, y>_W = sum_a (2l+1) sum_r x_a(r) y_a(r) (the
// Euclidean product of orthonormal-basis coefficients, in which the
// streaming operator is skew and the steady-state operator positive real).
// k_wdots: per block partial sums of <basis_i, w>_W for i < count (fixed
// element partition and tree: deterministic); k_cols_sum adds the block
// partials in a fixed order. Every vector kernel returns at once while the
// control block's stop flag is set (a GMRES cycle that has converged skips
// its remaining queued Arnoldi steps).
constexpr int kDotBlocks = 1024;
constexpr int kMaxBasis = 32;

// 16-byte vectors of the working precision (4 floats or 2 doubles): the
// vector kernels stream every field with one 16-byte access per lane.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  using type = float4;
  static constexpr int W = 4;
  static __device__ __forceinline__ double get(const float4& v, int k) {
    return double(k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w);
  }
  static __device__ __forceinline__ void set(float4& v, int k, double x) {
    const float f = float(x);
    if (k == 0) v.x = f;
    else if (k == 1) v.y = f;
    else if (k == 2) v.z = f;
    else v.w = f;
  }
};
template <> struct Vec16<double> {
  using type = double2;
  static constexpr int W = 2;
  static __device__ __forceinline__ double get(const double2& v, int k) { return k == 0 ? v.x : v.y; }
  static __device__ __forceinline__ void set(double2& v, int k, double x) {
    if (k == 0) v.x = x;
    else v.y = x;
  }
};
constexpr int kVecGroup = 8;   // basis vectors whose loads are in flight together

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_wdots(const T* __restrict__ basis, long long stride, int count, const T* __restrict__ w, int M,
        long long n3, double* __restrict__ partial, const Ctl* __restrict__ ctl) {
  using VT = Vec16<T>;
  using V = typename VT::type;
  constexpr int W = VT::W;
  __shared__ double red[kBlock];
  if (ctl->stop) return;
  double acc[kMaxBasis];
#pragma unroll
  for (int i = 0; i < kMaxBasis; ++i) acc[i] = 0.0;
  const long long step = (long long)gridDim.x * kBlock;
  const long long nv = n3 / W;   // n3 is a multiple of 4 (even grid sizes)
  for (int a = 0; a < M; ++a) {
    const double wt = double(2 * isqrt_c(a) + 1);
    const V* wa = reinterpret_cast<const V*>(w + (long long)a * n3);
    for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < nv; r += step) {
      const V wv = wa[r];
      double we[W];
#pragma unroll
      for (int k = 0; k < W; ++k) we[k] = wt * VT::get(wv, k);
#pragma unroll
      for (int g = 0; g < kMaxBasis; g += kVecGroup) {
        if (g < count) {   // count is uniform over the grid
          V bv[kVecGroup];
#pragma unroll
          for (int i = 0; i < kVecGroup; ++i)
            if (g + i < count) bv[i] = reinterpret_cast<const V*>(basis + (g + i) * stride + (long long)a * n3)[r];
#pragma unroll
          for (int i = 0; i < kVecGroup; ++i)
            if (g + i < count) {
              // elements in index order, as the scalar loop summed them
#pragma unroll
              for (int k = 0; k < W; ++k) acc[g + i] += we[k] * VT::get(bv[i], k);
            }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxBasis; ++i) {
    if (i < count) {
      red[threadIdx.x] = acc[i];
      __syncthreads();
      for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) partial[(long long)blockIdx.x * kMaxBasis + i] = red[0];
      __syncthreads();
    }
  }
}

// One workgroup per basis vector i: each thread adds the partials of blocks
// t, t + kBlock, ... in order, then a fixed tree (deterministic).
template <typename T>   // instantiated per working precision (one copy per translation unit)
__global__ void __launch_bounds__(kBlock)
k_cols_sum(const double* __restrict__ partial, int nblocks, int count, double* __restrict__ out,
           const Ctl* __restrict__ ctl) {
  __shared__ double red[kBlock];
  const int i = blockIdx.x;
  if (ctl->stop || i >= count) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partial[(long long)b * kMaxBasis + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// w <- sgn * w + sum_i coef[i] * basis_i  (coef on the device)
// (len is a multiple of 4; per element the same operations in the same
// order as a scalar loop, so the result does not depend on the vector width)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_combine(T* __restrict__ w, double sgn, const T* __restrict__ basis, long long stride, int count,
          const double* __restrict__ coef, double cscale, long long len, const Ctl* __restrict__ ctl) {
  using VT = Vec16<T>;
  using V = typename VT::type;
  constexpr int W = VT::W;
  if (ctl->stop) return;
  V* wv = reinterpret_cast<V*>(w);
  const long long nv = len / W;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < nv; e += (long long)gridDim.x * kBlock) {
    const V w0 = wv[e];
    double x[W];
#pragma unroll
    for (int k = 0; k < W; ++k) x[k] = sgn * VT::get(w0, k);
#pragma unroll
    for (int g = 0; g < kMaxBasis; g += kVecGroup) {
      if (g < count) {
        V bv[kVecGroup];
#pragma unroll
        for (int i = 0; i < kVecGroup; ++i)
          if (g + i < count) bv[i] = reinterpret_cast<const V*>(basis + (g + i) * stride)[e];
#pragma unroll
        for (int i = 0; i < kVecGroup; ++i)
          if (g + i < count) {
            const double c = cscale * coef[g + i];
#pragma unroll
            for (int k = 0; k < W; ++k) x[k] += c * VT::get(bv[i], k);
          }
      }
    }
    V o;
#pragma unroll
    for (int k = 0; k < W; ++k) VT::set(o, k, x[k]);
    wv[e] = o;
  }
}

// dst = src / s[0]
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_scale_by(T* __restrict__ dst, const T* __restrict__ src, const double* __restrict__ s, long long len,
           const Ctl* __restrict__ ctl) {
  using VT = Vec16<T>;
  using V = typename VT::type;
  constexpr int W = VT::W;
  if (ctl->stop) return;
  const double inv = 1.0 / s[0];
  const V* sv = reinterpret_cast<const V*>(src);
  V* dv = reinterpret_cast<V*>(dst);
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < len / W; e += (long long)gridDim.x * kBlock) {
    const V x = sv[e];
    V o;
#pragma unroll
    for (int k = 0; k < W; ++k) VT::set(o, k, VT::get(x, k) * inv);
    dv[e] = o;
  }
}

// dst = b - dst (b may be null: zero right-hand side)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_rhs_minus(T* __restrict__ dst, const T* __restrict__ b, long long len, const Ctl* __restrict__ ctl) {
  if (ctl->stop) return;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < len; e += (long long)gridDim.x * kBlock)
    dst[e] = (b ? b[e] : T(0)) - dst[e];
}

// One Arnoldi step's small-matrix work on the device (a single thread):
// Hessenberg column j = first + second Gram-Schmidt coefficients and the
// new vector's norm, the previous Givens rotations applied to it, a new
// rotation that zeroes its subdiagonal, the rotated residual vector g
// updated; sets the stop flag once |g[j+1]| / ref <= tol (this includes a
// breakdown, norm 0, where the Krylov space holds the solution).
template <typename T>   // instantiated per working precision (one copy per translation unit)
__global__ void __launch_bounds__(64)
k_gm_update(GmDev* __restrict__ gm, int j, Ctl* __restrict__ ctl) {
  if (threadIdx.x != 0 || ctl->stop) return;
  const int m = gm->m;
  double hv[kMaxBasisVectors + 1];
  for (int i = 0; i <= j; ++i) hv[i] = gm->hv[i] + gm->h2[i];
  const double hn = sqrt(gm->hn2);
  hv[j + 1] = hn;
  gm->hn = hn;
  for (int i = 0; i < j; ++i) {
    const double t = gm->cs[i] * hv[i] + gm->sn[i] * hv[i + 1];
    hv[i + 1] = -gm->sn[i] * hv[i] + gm->cs[i] * hv[i + 1];
    hv[i] = t;
  }
  const double r = hypot(hv[j], hv[j + 1]);
  const double c = r > 0 ? hv[j] / r : 1.0, sn = r > 0 ? hv[j + 1] / r : 0.0;
  gm->cs[j] = c;
  gm->sn[j] = sn;
  hv[j] = r;
  const double gj = gm->g[j];
  gm->g[j + 1] = -sn * gj;
  gm->g[j] = c * gj;
  for (int i = 0; i <= j; ++i) gm->R[i * m + j] = hv[i];
  gm->jdone = j + 1;
  if (fabs(gm->g[j + 1]) / gm->ref <= gm->tol) ctl->stop = 1;
}

// ------------------------------------ E: exact propagation per mode ---

// In a homogeneous medium without boundary layer every Fourier mode k of
// the moment vector a obeys da/dt = M(k) a + c q(k) with
//   M(k) = -c (i k.B + Sigma),
// Sigma the per-degree loss. Over a time T the mode advances exactly by
//   a <- exp(T M) a + int_0^T exp(s M) ds c q,
// evaluated per spectral point, all moments in registers, as s substeps of
// length h = T / s of the truncated Taylor series of the augmented
// generator [[h M, h c q], [0, 0]]:
//   t_1 = h (M a + c q),  t_j = h M t_{j-1} / j,  a <- a + sum_{j<=J} t_j.
// With nu = c T (|k| + max Sigma) >= ||T M|| (k.B has spectral norm <= |k|
// in the (2l+1)-weighted norm, in which Sigma is diagonal), the point takes
// s = ceil(nu / theta) substeps and the fewest J terms whose remainder
// bound (nu/s)^(J+1) / (J+1)! exp(nu/s) is below eps; theta is chosen on
// the host so that J never exceeds kTaylorMax.
template <typename T> struct TaylorMax;
template <> struct TaylorMax<float> { static constexpr int value = kTaylorMaxF32; };
template <> struct TaylorMax<double> { static constexpr int value = kTaylorMaxF64; };

template <typename T> struct ExpoParams {
  T sig[kMaxOrder + 1];   // per-degree loss Sigma_l
  double ct;              // c T
  double sigmax;          // max_l Sigma_l
  double theta;           // largest per-substep norm bound
  double eps;             // truncation target
  T inv_n3;               // 1 / n^3 (unnormalised transforms)
};

// (B_j t)_A for j = x, y, z accumulated over the compile-time slots of row
// A with the coefficients as instruction constants (every non-zero entry
// of the real-basis matrices belongs to exactly one axis): acc holds
// (re, im) per axis.
template <typename V, typename T, int N, int A, int S>
struct ExpoRowAcc {
  static __device__ __forceinline__ void run(const V* t, T* acc) {
    constexpr int l = isqrt_c(A);
    constexpr int m = A - l * l - l;
    constexpr SlotList sl = slots_of(N, l, m);
    if constexpr (S < sl.count) {
      constexpr int b = sl.b[S];
      constexpr double c0 = ct::real_coef(N, 0, A, b);
      constexpr double c1 = ct::real_coef(N, 1, A, b);
      constexpr double c2 = ct::real_coef(N, 2, A, b);
      if constexpr (c0 != 0.0) {
        acc[0] += T(c0) * t[b].x;
        acc[1] += T(c0) * t[b].y;
      }
      if constexpr (c1 != 0.0) {
        acc[2] += T(c1) * t[b].x;
        acc[3] += T(c1) * t[b].y;
      }
      if constexpr (c2 != 0.0) {
        acc[4] += T(c2) * t[b].x;
        acc[5] += T(c2) * t[b].y;
      }
      ExpoRowAcc<V, T, N, A, S + 1>::run(t, acc);
    }
  }
};

// nt = h (M t / c + q) (q only for the first term: SRC), acc += nt, all
// moments of one point; M t / c = -i (k.B) t - Sigma t.
template <typename V, typename T, int N, int A, bool SRC>
struct ExpoApply {
  static __device__ __forceinline__ void run(const V* t, V* nt, V* acc, T kx, T ky, T kz,
                                             const ExpoParams<T>& p, T h, const V* __restrict__ qp,
                                             size_t ms) {
    if constexpr (A < (N + 1) * (N + 1)) {
      constexpr int l = isqrt_c(A);
      T r[6] = {0, 0, 0, 0, 0, 0};
      ExpoRowAcc<V, T, N, A, 0>::run(t, r);
      const T re = kx * r[0] + ky * r[2] + kz * r[4];
      const T im = kx * r[1] + ky * r[3] + kz * r[5];
      T ox = im - p.sig[l] * t[A].x;
      T oy = -re - p.sig[l] * t[A].y;
      if constexpr (SRC) {
        const V qq = qp[A * ms];
        ox += p.inv_n3 * qq.x;
        oy += p.inv_n3 * qq.y;
      }
      nt[A] = cmk<V>(h * ox, h * oy);
      acc[A] = cmk<V>(acc[A].x + nt[A].x, acc[A].y + nt[A].y);
      ExpoApply<V, T, N, A + 1, SRC>::run(t, nt, acc, kx, ky, kz, p, h, qp, ms);
    }
  }
};

constexpr int kEBlock = 256;

// One thread per point of the full spectrum [b][kz][ky][kx] (kx < n/2; the
// kx = 0 slot carries the kx = n/2 column too, which has the same zero
// wavenumber, and the propagation is complex-linear, so both advance
// together). qs (the source spectrum, same layout) may be null.
template <typename T, int NN, int N>
__global__ void __launch_bounds__(kEBlock)
k_expo(typename cplx_of<T>::type* __restrict__ spec, const typename cplx_of<T>::type* __restrict__ qs,
       const T* __restrict__ kv, ExpoParams<T> p) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2;
  constexpr int M = (N + 1) * (N + 1);
  constexpr size_t MS = size_t(n) * n * H;
  constexpr int JMAX = TaylorMax<T>::value;
  const int pt = blockIdx.x * kEBlock + threadIdx.x;   // (kz * n + ky) * H + kx
  if (pt >= n * n * H) return;
  const int kxi = pt % H;
  const int kyi = (pt / H) % n;
  const int kzi = pt / (n * H);
  const T kx = kv[kxi], ky = kv[kyi], kz = kv[kzi];
  const double kk = std::sqrt(double(kx) * kx + double(ky) * ky + double(kz) * kz);
  const double nu = p.ct * (kk + p.sigmax);
  const int s = nu > p.theta ? int(std::ceil(nu / p.theta)) : 1;
  const double nus = nu / s;
  int J = 1;
  double bound = 0.5 * nus * nus * std::exp(nus);
  while (bound > p.eps && J < JMAX) {
    ++J;
    bound *= nus / (J + 1);
  }
  const T h = T(p.ct / s);
  V a[M], t[M], nt[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const V x = spec[i * MS + pt];
    a[i] = cmk<V>(p.inv_n3 * x.x, p.inv_n3 * x.y);
  }
  const V* qp = qs ? qs + pt : nullptr;
  auto term = [&](const V* src, V* dst, T hj, bool first) __attribute__((always_inline)) {
    if (first && qp) ExpoApply<V, T, N, 0, true>::run(src, dst, a, kx, ky, kz, p, hj, qp, MS);
    else ExpoApply<V, T, N, 0, false>::run(src, dst, a, kx, ky, kz, p, hj, nullptr, MS);
  };
  for (int sub = 0; sub < s; ++sub) {
#pragma unroll
    for (int i = 0; i < M; ++i) t[i] = a[i];
    term(t, nt, h, true);
    // the latest term is in nt; alternate buffers to avoid copies
    for (int j = 2; j <= J; j += 2) {
      term(nt, t, h / T(j), false);
      if (j + 1 > J) break;
      term(t, nt, h / T(j + 1), false);
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i) spec[i * MS + pt] = a[i];
}

// ----------------------------- E': exact propagation by rotation to k = z ---

// Rotation covariance of the streaming matrices: for the rotation R taking
// khat to z, D(R) (k.B) D(R)^T = |k| B_z, with D(R) the real-harmonic
// representation of R (block diagonal per degree, orthogonal; it commutes
// with the per-degree loss). So exp(T M(k)) = D^T exp(T M_z(|k|)) D, and
// M_z(|k|) = -c (i |k| B_z + Sigma) couples only equal orders m: blocks of
// size N + 1 - |m| (degrees |m|..N). The block exponentials depend on |k|
// only, i.e. on the integer f^2 = fx^2 + fy^2 + fz^2 of the grid frequencies:
// k_expo_table builds, for every f^2 and m, E_m = exp(T M_z) and
// Phi_m = int_0^T exp(s M_z) ds c (whole blocks, by scaling and squaring),
// k_expo_frame rotates each point's moments and source to the k = z frame
// and back, and k_expo_blocks applies the blocks in that frame. D(R) = X^T Rz(-theta) X Rz(-phi): Rz rotates the (m, -m)
// pairs by m times the angle, X (rotation by 90 degrees about x, y -> z) is
// a constant per-degree matrix computed once on the host.

constexpr int expo_block(int N, int m) { return N + 1 - (m < 0 ? -m : m); }
// number of f^2 values: kx index < n/2, ky and kz frequencies |f| < n/2
constexpr int expo_nf2(int n) { return (n / 2 - 1) * (n / 2 - 1) * 3 + 1; }
// offset (in complex entries) of the E block of order |m| in one f^2 row;
// the Phi block follows it. Orders m and -m have the same B_z block, hence
// the same exponentials: one pair of blocks per m >= 0.
constexpr int expo_block_offset(int N, int m) {
  int o = 0;
  for (int mm = 0; mm < m; ++mm) o += 2 * expo_block(N, mm) * expo_block(N, mm);
  return o;
}
constexpr int expo_row_size(int N) { return expo_block_offset(N, N + 1); }
constexpr int xrot_size(int N) {
  int o = 0;
  for (int l = 0; l <= N; ++l) o += (2 * l + 1) * (2 * l + 1);
  return o;
}
// real-valued offset of the table behind X and the B_z couplings (even, so
// that complex entries stay aligned)
constexpr int expo_table_offset(int N) {
  const int o = xrot_size(N) + 2 * (N + 1) * (N + 1);
  return o + (o & 1);
}

// Block exponentials by scaling and squaring, one wavefront per (f^2, m)
// block, in FP64 for both working precisions (the FP64 vector rate equals
// the unpacked FP32 rate). Lane (i, j) = (lane / d, lane % d) of the d x d
// block (d = N + 1 - m <= 8: at most 64 lanes) holds E_ij = exp(h A)_ij and
// P_ij = (int_0^h exp(s A) ds)_ij, A = -i |k| B_z - Sigma on the degrees
// m..N (per unit c: h runs up to c T). With h0 = c T / 2^q, q the fewest
// halvings that bring nu = c T (|k| + max Sigma), a bound on ||c T A||,
// to 1/2 or below, a Taylor series of kExpoTerms terms gives E and P at h0
// (truncation below 2^-53); q doublings
//   P <- P + E P,   E <- E E
// give them at c T. exp(t A) is a contraction (A + A^H = -2 Sigma <= 0), so
// a doubling at most doubles the error it inherits. bz[2a], bz[2a+1]: B_z
// couplings of row a to (l-1, m) and (l+1, m).
constexpr int kExpoTableWaves = 4;   // blocks (wavefronts) per workgroup
constexpr int kExpoTerms = 14;       // 0.5^15 / 15! < 2^-53

__host__ __device__ constexpr int expo_halvings(double nu) {
  int q = 0;
  for (double x = nu; x > 0.5; x *= 0.5) ++q;
  return q;
}

template <typename T, int N>
__global__ void __launch_bounds__(64 * kExpoTableWaves)
k_expo_table(typename cplx_of<T>::type* __restrict__ tab, const T* __restrict__ bz, ExpoParams<T> p,
             double kunit, int nf2) {
  using V = typename cplx_of<T>::type;
  __shared__ double2 sE[kExpoTableWaves][64], sP[kExpoTableWaves][64];
  const int wv = int(threadIdx.x) >> 6, ln = int(threadIdx.x) & 63;
  const long long blk = (long long)blockIdx.x * kExpoTableWaves + wv;   // uniform per wavefront
  if (blk >= (long long)nf2 * (N + 1)) return;
  const int f2 = int(blk / (N + 1)), m = int(blk - (long long)f2 * (N + 1));
  const int d = N + 1 - m;
  const int i = ln / d, j = ln - i * d;
  const bool act = ln < d * d;
  const double kk = kunit * sqrt(double(f2));
  const int q = expo_halvings(p.ct * (kk + p.sigmax));
  const double h0 = ldexp(p.ct, -q);
  double lo = 0.0, hi = 0.0, sg = 0.0;
  if (act) {
    const int l = m + i, a = l * l + l + m;
    if (i > 0) lo = double(bz[2 * a]);
    if (i + 1 < d) hi = double(bz[2 * a + 1]);
    sg = double(p.sig[l]);
  }
  // neighbours (i -+ 1, j); a row without one has a zero coupling to it
  const int up = (act && i > 0) ? ln - d : ln, dn = (act && i + 1 < d) ? ln + d : ln;
  // Taylor terms X_t = (h0 A)^t / t! from X_0 = I
  double xr = (act && i == j) ? 1.0 : 0.0, xi = 0.0;
  double er = xr, ei = 0.0, pr = h0 * xr, pi = 0.0;
  for (int t = 1; t <= kExpoTerms; ++t) {
    const double ur = __shfl(xr, up), ui = __shfl(xi, up);
    const double vr = __shfl(xr, dn), vi = __shfl(xi, dn);
    const double re = lo * ur + hi * vr, im = lo * ui + hi * vi;
    // A x = -i |k| (re + i im) - Sigma x
    const double st = h0 / double(t);
    const double nr = st * (kk * im - sg * xr), ni = st * (-kk * re - sg * xi);
    xr = nr;
    xi = ni;
    er += xr;
    ei += xi;
    const double w = h0 / double(t + 1);
    pr += w * xr;
    pi += w * xi;
  }
  for (int r = 0; r < q; ++r) {
    sE[wv][ln] = make_double2(er, ei);
    sP[wv][ln] = make_double2(pr, pi);
    wave_sync();
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    if (act) {
      for (int k = 0; k < d; ++k) {
        const double2 eik = sE[wv][i * d + k], ekj = sE[wv][k * d + j], pkj = sP[wv][k * d + j];
        ar += eik.x * ekj.x - eik.y * ekj.y;
        ai += eik.x * ekj.y + eik.y * ekj.x;
        br += eik.x * pkj.x - eik.y * pkj.y;
        bi += eik.x * pkj.y + eik.y * pkj.x;
      }
    }
    wave_sync();   // every lane has read the block before the next writes
    pr += br;
    pi += bi;
    er = ar;
    ei = ai;
  }
  if (act) {
    V* out = tab + (size_t)f2 * expo_row_size(N) + expo_block_offset(N, m);
    out[i * d + j] = cmk<V>(T(er), T(ei));
    out[d * d + i * d + j] = cmk<V>(T(pr), T(pi));
  }
}

// Rotation of one degree shell L (2L+1 moments in registers): z-rotation
// of the (m, -m) pairs by m times an angle given as (cos m a, sin m a).
template <typename V, typename T, int L>
__device__ __forceinline__ void shell_rot_z(V* v, const T* cm, const T* sm) {
#pragma unroll
  for (int m = 1; m <= L; ++m) {
    const V xp = v[L + m], xq = v[L - m];
    v[L + m] = cmk<V>(cm[m] * xp.x - sm[m] * xq.x, cm[m] * xp.y - sm[m] * xq.y);
    v[L - m] = cmk<V>(sm[m] * xp.x + cm[m] * xq.x, sm[m] * xp.y + cm[m] * xq.y);
  }
}

// v <- X_L v (TRANS: X_L^T v), the degree-L block of X from LDS
template <typename V, typename T, int L, bool TRANS>
__device__ __forceinline__ void shell_rot_x(V* v, const T* xs) {
  constexpr int d = 2 * L + 1;
  constexpr int o = L * (2 * L - 1) * (2 * L + 1) / 3;   // sum_{l<L} (2l+1)^2
  V w[d];
#pragma unroll
  for (int i = 0; i < d; ++i) {
    T re = T(0), im = T(0);
#pragma unroll
    for (int j = 0; j < d; ++j) {
      const T c = TRANS ? xs[o + j * d + i] : xs[o + i * d + j];
      re += c * v[j].x;
      im += c * v[j].y;
    }
    w[i] = cmk<V>(re, im);
    // one row's matrix entries at a time (the scheduler would otherwise
    // load the whole (2L+1)^2 block ahead and run out of registers)
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < d; ++i) v[i] = w[i];
}

// (cos, sin) of m phi and m theta, m = 0..N, for the direction of k
// (k = 0: no rotation)
template <typename T, int N>
__device__ __forceinline__ void k_angles(T kx, T ky, T kz, T* cp, T* sp, T* ct, T* st) {
  const T kxy = std::sqrt(kx * kx + ky * ky);
  const T kr = std::sqrt(kxy * kxy + kz * kz);
  T cph = T(1), sph = T(0), cth = T(1), sth = T(0);
  if (kr > T(0)) {
    cth = kz / kr;
    sth = kxy / kr;
  }
  if (kxy > T(0)) {
    cph = kx / kxy;
    sph = ky / kxy;
  }
  cp[0] = ct[0] = T(1);
  sp[0] = st[0] = T(0);
#pragma unroll
  for (int m = 1; m <= N; ++m) {
    cp[m] = cp[m - 1] * cph - sp[m - 1] * sph;
    sp[m] = sp[m - 1] * cph + cp[m - 1] * sph;
    ct[m] = ct[m - 1] * cth - st[m - 1] * sth;
    st[m] = st[m - 1] * cth + ct[m - 1] * sth;
  }
}

// Shells L..N of one point: to the k = z frame, D(R) = X^T Rz(-theta) X
// Rz(-phi) (BACK: D(R)^T = Rz(phi) X^T Rz(theta) X), scaled by sc; one shell
// in registers at a time.
template <typename V, typename T, int N, bool BACK, int L = 0, int LAST = N>
__device__ __forceinline__ void frame_shells(V* v, size_t ms, const T* xs, const T* cp, const T* sp,
                                             const T* ct, const T* st, T sc) {
  if constexpr (L <= LAST) {
    constexpr int d = 2 * L + 1, a0 = L * L;
    V w[d];
#pragma unroll
    for (int i = 0; i < d; ++i) {
      const V x = v[(a0 + i) * ms];
      w[i] = cmk<V>(sc * x.x, sc * x.y);
    }
    if constexpr (L > 0) {
      T ns[L + 1];
      if constexpr (!BACK) {
#pragma unroll
        for (int m = 0; m <= L; ++m) ns[m] = -sp[m];
        shell_rot_z<V, T, L>(w, cp, ns);
        shell_rot_x<V, T, L, false>(w, xs);
#pragma unroll
        for (int m = 0; m <= L; ++m) ns[m] = -st[m];
        shell_rot_z<V, T, L>(w, ct, ns);
        shell_rot_x<V, T, L, true>(w, xs);
      } else {
        shell_rot_x<V, T, L, false>(w, xs);
        shell_rot_z<V, T, L>(w, ct, st);
        shell_rot_x<V, T, L, true>(w, xs);
        shell_rot_z<V, T, L>(w, cp, sp);
      }
    }
#pragma unroll
    for (int i = 0; i < d; ++i) v[(a0 + i) * ms] = w[i];
    frame_shells<V, T, N, BACK, L + 1, LAST>(v, ms, xs, cp, sp, ct, st, sc);
  }
}

// Shell L (= blockIdx.y, uniform per workgroup) of every point.
template <typename V, typename T, int N, bool BACK, int L = 0>
__device__ __forceinline__ void frame_shell_of(int sh, V* v, size_t ms, const T* xs, const T* cp, const T* sp,
                                               const T* ct, const T* st, T sc) {
  if constexpr (L <= N) {
    if (sh == L) frame_shells<V, T, N, BACK, L, L>(v, ms, xs, cp, sp, ct, st, sc);
    else frame_shell_of<V, T, N, BACK, L + 1>(sh, v, ms, xs, cp, sp, ct, st, sc);
  }
}

// Every point's moments (scaled by sc) to (BACK: from) its k = z frame, in
// place in the full spectrum [b][kz][ky][kx]. The rotation is block
// diagonal by degree, so the grid's second dimension runs over the degree
// shells: a thread holds one shell of one point (at most 2N + 1 values),
// which keeps the registers per thread low enough for the waves the
// streaming access needs.
template <typename T, int NN, int N, bool BACK>
__global__ void __launch_bounds__(kEBlock)
k_expo_frame(typename cplx_of<T>::type* __restrict__ v, const T* __restrict__ kv, const T* __restrict__ xrot,
             T sc) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2;
  constexpr size_t MS = size_t(n) * n * H;
  constexpr int XS = xrot_size(N);
  __shared__ T xs[XS];
  for (int i = threadIdx.x; i < XS; i += kEBlock) xs[i] = xrot[i];
  __syncthreads();
  const int pt = blockIdx.x * kEBlock + threadIdx.x;
  if (pt >= n * n * H) return;
  const int xi = pt % H, yi = (pt / H) % n, zi = pt / (n * H);
  T cp[N + 1], sp[N + 1], ct[N + 1], st[N + 1];
  k_angles<T, N>(kv[xi], kv[yi], kv[zi], cp, sp, ct, st);
  frame_shell_of<V, T, N, BACK>(int(blockIdx.y), v + pt, MS, xs, cp, sp, ct, st, sc);
}

// a <- E_m a + Phi_m q on the degrees m..N of orders m and -m (same
// blocks), for m = MM..N, with a and q (both in the k = z frame) read from
// and a written to the spectrum
template <typename V, typename T, int N, int MM = 0, int LAST = N>
__device__ __forceinline__ void expo_blocks(V* a, const V* q, size_t ms, const V* row) {
  if constexpr (MM <= LAST) {
    constexpr int d = N + 1 - MM;
    constexpr int NS = MM == 0 ? 1 : 2;   // the orders m and -m
    const V* E = row + expo_block_offset(N, MM);
    const V* P = E + d * d;
    V x[NS][d], y[NS][d];
#pragma unroll
    for (int sgn = 0; sgn < NS; ++sgn)
#pragma unroll
      for (int j = 0; j < d; ++j) {
        const int m = sgn ? -MM : MM;
        const int bj = (MM + j) * (MM + j) + (MM + j) + m;
        x[sgn][j] = a[bj * ms];
        y[sgn][j] = q ? q[bj * ms] : cmk<V>(T(0), T(0));
      }
    // rows one at a time (a run-time loop: unrolled, the compiler would load
    // all 2 d^2 table entries at once), each written as soon as it is formed
    // (the block's inputs are all in registers by then)
#pragma unroll 1
    for (int i = 0; i < d; ++i) {
      T re[NS], im[NS];
#pragma unroll
      for (int sgn = 0; sgn < NS; ++sgn) re[sgn] = im[sgn] = T(0);
#pragma unroll
      for (int j = 0; j < d; ++j) {
        const V e = E[i * d + j];
        const V f = q ? P[i * d + j] : cmk<V>(T(0), T(0));
#pragma unroll
        for (int sgn = 0; sgn < NS; ++sgn) {
          re[sgn] += e.x * x[sgn][j].x - e.y * x[sgn][j].y + f.x * y[sgn][j].x - f.y * y[sgn][j].y;
          im[sgn] += e.x * x[sgn][j].y + e.y * x[sgn][j].x + f.x * y[sgn][j].y + f.y * y[sgn][j].x;
        }
      }
      const int l = MM + i;
#pragma unroll
      for (int sgn = 0; sgn < NS; ++sgn) a[(l * l + l + (sgn ? -MM : MM)) * ms] = cmk<V>(re[sgn], im[sgn]);
    }
    expo_blocks<V, T, N, MM + 1, LAST>(a, q, ms, row);
  }
}

// Order m (= blockIdx.y, uniform per workgroup) of one point.
template <typename V, typename T, int N, int MM = 0>
__device__ __forceinline__ void expo_block_of(int m, V* a, const V* q, size_t ms, const V* row) {
  if constexpr (MM <= N) {
    if (m == MM) expo_blocks<V, T, N, MM, MM>(a, q, ms, row);
    else expo_block_of<V, T, N, MM + 1>(m, a, q, ms, row);
  }
}

// Thread -> spectral point. The block products read one table row per
// |k|^2; the four points (+-fy, +-fz) of a given kx share it. Lanes are
// grouped so that one wavefront instruction holds those four points for TX
// consecutive kx (sub-group s of a quad of 4 TX lanes takes y -> y' if s & 1,
// z -> z' if s & 2, with i' = n - i, and 0' = n/2 for the index pair whose
// frequency is 0): the four lanes that share a row read it in the same
// instruction, which fetches it once. A bijection of the points, so the
// results are those of any other order.
#ifndef RTE_EXPO_OCT
#define RTE_EXPO_OCT 0
#endif
template <int NN> struct ExpoQuad {
  static constexpr int H = NN / 2;
  static constexpr bool OCT = RTE_EXPO_OCT;   // also pair (y, z) with (z, y): eight points per row
  static constexpr int G = OCT ? 8 : 4;       // points per group
  static constexpr int TXMAX = 64 / G;
  static constexpr int TX = (H % TXMAX == 0) ? TXMAX : (H % 8 == 0 ? 8 : (H % 4 == 0 ? 4 : 1));
  static_assert(64 % (G * TX) == 0, "groups must tile a wavefront");
  static constexpr int C = NN / 2;                                 // classes per axis
  static constexpr int NCLS = OCT ? C * (C + 1) / 2 : C * C;       // (y, z) classes
  static constexpr int THREADS = NCLS * (H / TX) * G * TX;          // threads launched
  static __device__ __forceinline__ int mirror(int i) { return i == 0 ? NN / 2 : NN - i; }
  // point index (z n + y) H + x of thread t < THREADS, or -1 (an idle lane
  // of a diagonal class, whose swapped points are the same points)
  static __device__ __forceinline__ int point(int t) {
    const int Q = t / (G * TX), l = t - Q * G * TX;
    const int sub = l / TX, xl = l - sub * TX;
    constexpr int XT = H / TX;
    const int xt = Q % XT, cls = Q / XT;
    int yc, zc;
    if constexpr (OCT) {
      // cls -> (yc <= zc): row zc holds zc + 1 classes
      int z = int((sqrtf(8.f * cls + 1.f) - 1.f) * 0.5f);
      while ((z + 1) * (z + 2) / 2 <= cls) ++z;
      while (z * (z + 1) / 2 > cls) --z;
      zc = z;
      yc = cls - z * (z + 1) / 2;
      if (sub & 4) {
        if (yc == zc) return -1;
        const int tmp = yc;
        yc = zc;
        zc = tmp;
      }
    } else {
      yc = cls % C;
      zc = cls / C;
    }
    const int y = (sub & 1) ? mirror(yc) : yc, z = (sub & 2) ? mirror(zc) : zc;
    return (z * NN + y) * H + xt * TX + xl;
  }
};

template <typename T, int NN, int N>
__global__ void __launch_bounds__(kEBlock)
k_expo_blocks(typename cplx_of<T>::type* __restrict__ spec, const typename cplx_of<T>::type* __restrict__ qs,
              const typename cplx_of<T>::type* __restrict__ tab) {
  using V = typename cplx_of<T>::type;
  constexpr int n = NN, H = NN / 2;
  constexpr size_t MS = size_t(n) * n * H;
  const int t = blockIdx.x * kEBlock + threadIdx.x;
  if (t >= ExpoQuad<NN>::THREADS) return;
  const int pt = ExpoQuad<NN>::point(t);
  if (pt < 0) return;
  const int xi = pt % H, yi = (pt / H) % n, zi = pt / (n * H);
  auto freq = [](int i) { return i < n / 2 ? i : (i == n / 2 ? 0 : i - n); };
  const int fy = freq(yi), fz = freq(zi);
  const int f2 = xi * xi + fy * fy + fz * fz;
  // the blocks of different orders are independent: one order per grid row
  // (blockIdx.y), which keeps a thread's registers to one block
  expo_block_of<V, T, N>(int(blockIdx.y), spec + pt, qs ? qs + pt : nullptr, MS,
                         tab + (size_t)f2 * expo_row_size(N));
}

}  // namespace rte

#include "rte_plane128.h"
#include "rte_pencil.h"

namespace rte {

// One pencil pass over all M n (n/2) / TZ tiles: the register pencils of FP32
// 128^3 / 256^3 grids where they apply, k_pencil otherwise (ns slot rows,
// bs slot stride for batched launches).
template <typename T, int NN, int MODE>
void launch_pencil(hipStream_t st, const typename cplx_of<T>::type* src, typename cplx_of<T>::type* dst,
                   const typename cplx_of<T>::type* tw, const T* kv, const Ctl* ctl, int M, unsigned ns = 1,
                   long long bs = 0) {
  if constexpr (pen::use_reg<T, NN, MODE>()) {
    const int tiles = M * NN * pen::Shape<NN>::NTILE;
    hipLaunchKernelGGL((pen::k_pencil_reg<NN, MODE>), dim3(tiles, ns), dim3(pen::Shape<NN>::THREADS), 0, st, src, dst, tw, kv, ctl,
                       bs);
  } else {
    using Z = ZdShape<T, NN>;
    const int tiles = M * NN * Z::NTILE;
    hipLaunchKernelGGL((k_pencil<T, NN, MODE>), dim3(tiles, ns), dim3(kZBlock), (zd_lds<T, NN>()), st, src, dst,
                       tw, kv, ctl, bs);
  }
}

// ---------------------------------------------------------------- launch ---

// FP32 128^3 time steps and operator applications use the register-fused
// plane pass (rte_plane128.h); other sizes and FP64 the generic one.
template <typename T, int NN> constexpr bool plane128() { return std::is_same<T, float>::value && NN == 128; }

// Forward xy transform of `planes` real planes into the packed spectrum
// (plane grids): the FP32 128^3 path uses the same arithmetic as the forward
// half of its fused inverse pass.
template <typename T, int NN>
void launch_fwd_plane(hipStream_t st, const T* src, typename cplx_of<T>::type* spec,
                      const typename cplx_of<T>::type* tw, const Ctl* ctl, int planes) {
  if constexpr (plane128<T, NN>())
    hipLaunchKernelGGL(p128::k_fwd128<512>, dim3(planes), dim3(512), p128::kLds, st, src, spec, tw, ctl, planes);
  else
    hipLaunchKernelGGL((k_fwd_plane<T, NN>), dim3((planes + kFwdPlanes - 1) / kFwdPlanes), dim3(kPBlock),
                       (plane_lds<T, NN>()), st, src, spec, tw, ctl, planes);
}

// Grids up to 128 points per axis keep a whole plane in LDS (plane passes);
// larger grids split each plane pass into a row pass and a y-pencil pass.
template <int NN> constexpr bool split_planes() { return NN > 128; }

template <typename T, int NN, int N>
hipError_t prepare_t(const StepArgs& a) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, size_t bytes) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  };
  if constexpr (split_planes<NN>()) {
    set(reinterpret_cast<const void*>(&k_rows_fwd<T, NN>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_FIRST>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_MID>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_LAST>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_ADJ>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_EULER>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_APPLY>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_SET>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_FIRST, true>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_MID, true>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_LAST, true>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_rows_inv<T, NN, EPI_EULER, true>), rows_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_pencil<T, NN, PENCIL_YFWD>), zd_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_pencil<T, NN, PENCIL_YINV>), zd_lds<T, NN>());
  } else {
    set(reinterpret_cast<const void*>(&k_fwd_plane<T, NN>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_FIRST>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_MID>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_LAST>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_ADJ>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_EULER>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_APPLY>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_SET>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_FIRST, true>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_MID, true>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_LAST, true>), plane_lds<T, NN>());
    set(reinterpret_cast<const void*>(&k_inv_plane<T, NN, EPI_EULER, true>), plane_lds<T, NN>());
    if constexpr (plane128<T, NN>()) {
      set(reinterpret_cast<const void*>(&p128::k_fwd128<512>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_FIRST, false>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_MID, false>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_LAST, false>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_ADJ, false>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_EULER, false>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_APPLY, false>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_FIRST, true>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_MID, true>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_LAST, true>), p128::kLds);
      set(reinterpret_cast<const void*>(&p128::k_plane128<EPI_EULER, true>), p128::kLds);
    }
  }
  set(reinterpret_cast<const void*>(&k_pencil<T, NN, PENCIL_ZDERIV>), zd_lds<T, NN>());
  set(reinterpret_cast<const void*>(&k_pencil<T, NN, PENCIL_ZFWD>), zd_lds<T, NN>());
  set(reinterpret_cast<const void*>(&k_pencil<T, NN, PENCIL_ZINV>), zd_lds<T, NN>());
  return e;
}

// Number of per-block fluence-change partial sums written by the last
// stage (one per z-plane, or one per row block on split grids).
template <int NN> constexpr int partial_count() {
  return split_planes<NN>() ? NN * (NN / RowShape<NN>::RB) : NN;
}

// One stage: out = MODE-epilogue of (u, src) with the streaming term
// sgn * a h c (-B.grad src) (sgn = -1 gives the transposed streaming).
template <typename T, int NN, int N, int MODE, bool FUSE = false>
void enqueue_stage(const StepArgs& a, ProfRec* pr, double hs, double sgn, const T* src, T* u, T* out,
                   int stage = 0, long long step1 = 0) {
  using V = typename cplx_of<T>::type;
  constexpr int M = (N + 1) * (N + 1);
  hipStream_t st = reinterpret_cast<hipStream_t>(a.stream);
  V* spec = static_cast<V*>(a.spec);
  V* dspec = static_cast<V*>(a.dspec);
  const V* tw = static_cast<const V*>(a.tw);
  const T* kv = static_cast<const T*>(a.kv);
  const T* sig = static_cast<const T*>(a.sig);
  const T* q = static_cast<const T*>(a.q);
  const Ctl* cctl = static_cast<const Ctl*>(a.ctl);
  const double n2 = double(NN) * NN;
  const dim3 pblk(kPBlock), zblk(kZBlock), cblk(kCBlock);
  const int planes = M * NN;
  const int cblocks = (NN * NN * (NN / 2) + kCBlock - 1) / kCBlock;
  const int rblocks = M * NN * (NN / RowShape<NN>::RB);
  const size_t lp = plane_lds<T, NN>(), lr = rows_lds<T, NN>();
  // batched launches (plane grids, register coupling): grid rows = slots
  const unsigned ns = a.nslot > 1 ? unsigned(a.nslot) : 1u;
  const long long bs = ns > 1 ? a.sstride : 0;
  auto rec = [&](int cls) {
    if (pr && pr->count < kMaxProfLaunches) {
      (void)hipEventRecord(static_cast<hipEvent_t>(pr->ev[pr->count]), st);
      pr->cls[pr->count++] = cls;
    }
  };
  if constexpr (split_planes<NN>()) {
    // (fused stages find the row spectrum of src already written by the
    // previous inverse row pass)
    if constexpr (!FUSE) {
      hipLaunchKernelGGL((k_rows_fwd<T, NN>), dim3(rblocks), zblk, lr, st, src, spec, tw, cctl);
      rec(PROF_FWD_ROWS);
    }
    launch_pencil<T, NN, PENCIL_YFWD>(st, spec, spec, tw, kv, cctl, M);
    rec(PROF_Y_FWD);
  } else if constexpr (!FUSE) {
    // (fused stages find the spectrum of src already written by the
    // previous inverse pass)
    launch_fwd_plane<T, NN>(st, src, spec, tw, cctl, planes);
    rec(PROF_FWD_PLANE);
  }
  launch_pencil<T, NN, PENCIL_ZDERIV>(st, spec, dspec, tw, kv, cctl, M, ns, bs);
  rec(PROF_ZDERIV);
  V* coupled = dspec;   // the inverse passes read the coupled spectrum from here
  if constexpr (N <= kDenseOrder) {
    hipLaunchKernelGGL((k_couple<T, NN, N>), dim3(2 * cblocks, ns), cblk, 0, st, spec, dspec, kv,
                       T(sgn * hs / n2), cctl, bs);
  } else {
    coupled = static_cast<V*>(a.wspec);
    hipLaunchKernelGGL((k_couple_rt<T, NN>), dim3(cblocks, kRtSlices), cblk, 0, st, spec, dspec, coupled, kv, a.ctab,
                       static_cast<const T*>(a.cval), M, T(sgn * hs / n2), cctl);
  }
  rec(PROF_COUPLE);
  if constexpr (split_planes<NN>()) {
    launch_pencil<T, NN, PENCIL_YINV>(st, coupled, coupled, tw, kv, cctl, M);
    rec(PROF_Y_INV);
    hipLaunchKernelGGL((k_rows_inv<T, NN, MODE, FUSE>), dim3(rblocks), zblk, lr, st, coupled, src, u, out, sig,
                       q, a.qflag, a.phi_int, a.partial, tw, M, T(hs), a.dt, cctl, stage, step1,
                       FUSE ? spec : static_cast<V*>(nullptr));
    rec(PROF_INV_ROWS);
  } else if constexpr (plane128<T, NN>()) {
    hipLaunchKernelGGL((p128::k_plane128<MODE, FUSE>), dim3(planes, ns), pblk, p128::kLds, st, coupled, src, u,
                       out, sig, q, a.qflag, a.phi_int, a.partial, tw, M, T(hs), a.dt, cctl, stage, step1,
                       FUSE ? spec : static_cast<V*>(nullptr), bs);
    rec(PROF_INV_PLANE);
  } else {
    hipLaunchKernelGGL((k_inv_plane<T, NN, MODE, FUSE>), dim3(planes, ns), pblk, lp, st, coupled, src, u, out,
                       sig, q, a.qflag, a.phi_int, a.partial, tw, M, T(hs), a.dt, cctl, stage, step1,
                       FUSE ? spec : static_cast<V*>(nullptr), bs);
    rec(PROF_INV_PLANE);
  }
}

// Exact propagation over time op.coef: 3D forward transforms of the state
// (and of the source, into the derivative buffer), the per-point
// exponential, inverse transforms written over the state.
template <typename T, int NN, int N>
hipError_t enqueue_expo(const StepArgs& a, const OpArgs& op, ProfRec* pr) {
  using V = typename cplx_of<T>::type;
  using Z = ZdShape<T, NN>;
  constexpr int M = (N + 1) * (N + 1);
  constexpr int n = NN, H = NN / 2;
  hipStream_t st = reinterpret_cast<hipStream_t>(a.stream);
  V* spec = static_cast<V*>(a.spec);
  V* dspec = static_cast<V*>(a.dspec);
  const V* tw = static_cast<const V*>(a.tw);
  const T* kv = static_cast<const T*>(a.kv);
  const T* sig = static_cast<const T*>(a.sig);
  const T* q = static_cast<const T*>(a.q);
  T* u = static_cast<T*>(a.u);
  const Ctl* cctl = static_cast<const Ctl*>(a.ctl);
  const dim3 pblk(kPBlock), zblk(kZBlock);
  const int planes = M * n;
  const int pencils = M * n * Z::NTILE;
  const int rblocks = M * n * (n / RowShape<NN>::RB);
  const size_t lp = plane_lds<T, NN>(), lz = zd_lds<T, NN>(), lr = rows_lds<T, NN>();
  auto rec = [&](int cls) {
    if (pr && pr->count < kMaxProfLaunches) {
      (void)hipEventRecord(static_cast<hipEvent_t>(pr->ev[pr->count]), st);
      pr->cls[pr->count++] = cls;
    }
  };
  if (pr) {
    (void)hipEventRecord(static_cast<hipEvent_t>(pr->ev0), st);
    pr->count = 0;
  }
  auto forward = [&](const T* src, V* dst) {
    if constexpr (split_planes<NN>()) {
      hipLaunchKernelGGL((k_rows_fwd<T, NN>), dim3(rblocks), zblk, lr, st, src, dst, tw, cctl);
      rec(PROF_FWD_ROWS);
      hipLaunchKernelGGL((k_pencil<T, NN, PENCIL_YFWD>), dim3(pencils), zblk, lz, st, dst, dst, tw, kv, cctl);
      rec(PROF_Y_FWD);
    } else {
      hipLaunchKernelGGL((k_fwd_plane<T, NN>), dim3((planes + kFwdPlanes - 1) / kFwdPlanes), pblk, lp, st, src,
                         dst, tw, cctl, planes);
      rec(PROF_FWD_PLANE);
    }
    hipLaunchKernelGGL((k_pencil<T, NN, PENCIL_ZFWD>), dim3(pencils), zblk, lz, st, dst, dst, tw, kv, cctl);
    rec(PROF_Z_FWD);
  };
  if (q) forward(q, dspec);
  forward(u, spec);
  ExpoParams<T> p{};
  double smax = 0.0;
  for (int l = 0; l <= kMaxOrder; ++l) {
    p.sig[l] = T(l <= N ? op.sigl[l] : 0.0);
    if (l <= N) smax = op.sigl[l] > smax ? op.sigl[l] : smax;
  }
  p.ct = op.coef * a.c;
  p.sigmax = smax;
  p.theta = op.scale;
  p.eps = op.eps;
  p.inv_n3 = T(1.0 / (double(n) * n * n));
  const int eblocks = (n * n * H + kEBlock - 1) / kEBlock;
  if (op.count == 1) {
    // rotation data in the stage buffer v: X blocks, B_z couplings, then the
    // block-exponential table (layout checked on the host)
    const T* xrot = static_cast<const T*>(a.v);
    const T* bz = xrot + xrot_size(N);
    V* tab = reinterpret_cast<V*>(static_cast<T*>(a.v) + expo_table_offset(N));
    const int nf2 = expo_nf2(NN);
    const long long tblocks = (long long)nf2 * (N + 1);
    hipLaunchKernelGGL((k_expo_table<T, N>), dim3(unsigned((tblocks + kExpoTableWaves - 1) / kExpoTableWaves)),
                       dim3(64 * kExpoTableWaves), 0, st, tab, bz, p, op.kunit, nf2);
    rec(PROF_EXPO_TABLE);
    if (q)
      hipLaunchKernelGGL((k_expo_frame<T, NN, N, false>), dim3(eblocks, N + 1), dim3(kEBlock), 0, st, dspec, kv, xrot,
                         p.inv_n3);
    hipLaunchKernelGGL((k_expo_frame<T, NN, N, false>), dim3(eblocks, N + 1), dim3(kEBlock), 0, st, spec, kv, xrot,
                       p.inv_n3);
    hipLaunchKernelGGL((k_expo_blocks<T, NN, N>), dim3((ExpoQuad<NN>::THREADS + kEBlock - 1) / kEBlock, N + 1),
                       dim3(kEBlock), 0, st, spec, q ? dspec : nullptr, tab);
    hipLaunchKernelGGL((k_expo_frame<T, NN, N, true>), dim3(eblocks, N + 1), dim3(kEBlock), 0, st, spec, kv, xrot, T(1));
  } else {
    hipLaunchKernelGGL((k_expo<T, NN, N>), dim3(eblocks), dim3(kEBlock), 0, st, spec, q ? dspec : nullptr, kv, p);
  }
  rec(PROF_EXPO);
  hipLaunchKernelGGL((k_pencil<T, NN, PENCIL_ZINV>), dim3(pencils), zblk, lz, st, spec, spec, tw, kv, cctl);
  rec(PROF_Z_INV);
  if constexpr (split_planes<NN>()) {
    hipLaunchKernelGGL((k_pencil<T, NN, PENCIL_YINV>), dim3(pencils), zblk, lz, st, spec, spec, tw, kv, cctl);
    rec(PROF_Y_INV);
    hipLaunchKernelGGL((k_rows_inv<T, NN, EPI_SET>), dim3(rblocks), zblk, lr, st, spec, u, u, u, sig,
                       static_cast<const T*>(nullptr), a.qflag, a.phi_int, a.partial, tw, M, T(0), 0.0, cctl, 0,
                       0LL);
    rec(PROF_INV_ROWS);
  } else {
    hipLaunchKernelGGL((k_inv_plane<T, NN, EPI_SET>), dim3(planes), pblk, lp, st, spec, u, u, u, sig,
                       static_cast<const T*>(nullptr), a.qflag, a.phi_int, a.partial, tw, M, T(0), 0.0, cctl, 0,
                       0LL, static_cast<V*>(nullptr));
    rec(PROF_INV_PLANE);
  }
  return hipGetLastError();
}

constexpr double kRkAlpha[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};

template <typename T, int NN, int N>
hipError_t enqueue_t(const StepArgs& a, const OpArgs& op, ProfRec* pr) {
  hipStream_t st = reinterpret_cast<hipStream_t>(a.stream);
  const Ctl* cctl = static_cast<const Ctl*>(a.ctl);
  const double hc = a.dt * a.c;
  const long long nvox = (long long)NN * NN * NN;
  constexpr int M = (N + 1) * (N + 1);
  switch (op.kind) {
    case OP_STEP: {
      T* u = static_cast<T*>(a.u);
      T* v = static_cast<T*>(a.v);
      if (pr) {
        (void)hipEventRecord(static_cast<hipEvent_t>(pr->ev0), st);
        pr->count = 0;
      }
      const long long s1 = op.step1;
      bool done = false;
      if (op.fused) {
        // the spectrum of u (xy on plane grids, x on split grids) is in
        // place on entry; every inverse pass leaves that of its output for
        // the next stage (the last one that of the new u, for the next step)
        if (a.scheme == 1) {
          enqueue_stage<T, NN, N, EPI_EULER, true>(a, pr, hc, 1.0, u, u, u, 0, s1);
        } else {
          enqueue_stage<T, NN, N, EPI_FIRST, true>(a, pr, kRkAlpha[0] * hc, 1.0, u, u, v, 0, s1);
          enqueue_stage<T, NN, N, EPI_MID, true>(a, pr, kRkAlpha[1] * hc, 1.0, v, u, v, 1, s1);
          enqueue_stage<T, NN, N, EPI_MID, true>(a, pr, kRkAlpha[2] * hc, 1.0, v, u, v, 2, s1);
          enqueue_stage<T, NN, N, EPI_LAST, true>(a, pr, kRkAlpha[3] * hc, 1.0, v, u, u, 3, s1);
        }
        done = true;
      }
      if (done) {
      } else if (a.scheme == 1) {
        // forward Euler (eq. 11 with the sign reading): u <- u + dt f(u)
        enqueue_stage<T, NN, N, EPI_EULER>(a, pr, hc, 1.0, u, u, u, 0, s1);
      } else {
        enqueue_stage<T, NN, N, EPI_FIRST>(a, pr, kRkAlpha[0] * hc, 1.0, u, u, v, 0, s1);
        enqueue_stage<T, NN, N, EPI_MID>(a, pr, kRkAlpha[1] * hc, 1.0, v, u, v, 1, s1);
        enqueue_stage<T, NN, N, EPI_MID>(a, pr, kRkAlpha[2] * hc, 1.0, v, u, v, 2, s1);
        enqueue_stage<T, NN, N, EPI_LAST>(a, pr, kRkAlpha[3] * hc, 1.0, v, u, u, 3, s1);
      }
      const unsigned ns = a.nslot > 1 ? unsigned(a.nslot) : 1u;
      hipLaunchKernelGGL((k_end_step<T>), dim3(1, ns), dim3(kBlock), 0, st, u, a.det, a.ndet, a.readings, a.resid,
                         a.cap, a.partial, partial_count<NN>(), static_cast<Ctl*>(a.ctl),
                         ns > 1 ? a.sstride : 0LL);
      if (pr && pr->count < kMaxProfLaunches) {
        (void)hipEventRecord(static_cast<hipEvent_t>(pr->ev[pr->count]), st);
        pr->cls[pr->count++] = PROF_END;
      }
      break;
    }
    case OP_STAGE: {
      // forward stage op.stage (0..2) of the nested RK4 form from base state
      // op.u with stage input op.x, writing op.y (no bookkeeping)
      const int s = op.stage;
      const T* xin = static_cast<const T*>(op.x);
      T* u = static_cast<T*>(op.u);
      T* out = static_cast<T*>(op.y);
      if (s == 0) enqueue_stage<T, NN, N, EPI_FIRST>(a, nullptr, kRkAlpha[0] * hc, 1.0, u, u, out, 0, op.step1);
      else enqueue_stage<T, NN, N, EPI_MID>(a, nullptr, kRkAlpha[s] * hc, 1.0, xin, u, out, s, op.step1);
      break;
    }
    case OP_ADJ_STAGE: {
      // xs_out = coef h F~(xs_in) with the streaming sign flipped, acc += xs_out
      enqueue_stage<T, NN, N, EPI_ADJ>(a, nullptr, op.coef * hc, -1.0, static_cast<const T*>(op.x),
                                       static_cast<T*>(op.u), static_cast<T*>(op.y));
      break;
    }
    case OP_ADJ_GRAD: {
      const int blocks = int((nvox + kBlock - 1) / kBlock);
      hipLaunchKernelGGL((k_adj_grad<T>), dim3(blocks), dim3(kBlock), 0, st, static_cast<const T*>(op.x),
                         static_cast<const T*>(op.y), op.gin, op.gmua, op.gmus, N, nvox,
                         -a.c * op.coef * a.dt);
      break;
    }
    case OP_APPLY: {
      // y = (S + Sigma) x
      enqueue_stage<T, NN, N, EPI_APPLY>(a, nullptr, 1.0, 1.0, static_cast<const T*>(op.x),
                                         static_cast<T*>(op.y), static_cast<T*>(op.y));
      break;
    }
    case OP_WDOTS: {
      const long long len = (long long)M * nvox;
      hipLaunchKernelGGL((k_wdots<T>), dim3(kDotBlocks), dim3(kBlock), 0, st, static_cast<const T*>(op.x),
                         len, op.count, static_cast<const T*>(op.y), M, nvox, op.gmua, cctl);
      hipLaunchKernelGGL((k_cols_sum<T>), dim3(kMaxBasis), dim3(kBlock), 0, st, op.gmua, kDotBlocks, op.count,
                         op.gmus, cctl);
      break;
    }
    case OP_COMBINE: {
      const long long len = (long long)M * nvox;
      hipLaunchKernelGGL((k_combine<T>), dim3(kDotBlocks), dim3(kBlock), 0, st, static_cast<T*>(op.y),
                         op.coef, static_cast<const T*>(op.x), len, op.count, op.djdr, op.scale, len, cctl);
      break;
    }
    case OP_SCALE: {
      const long long len = (long long)M * nvox;
      hipLaunchKernelGGL((k_scale_by<T>), dim3(kDotBlocks), dim3(kBlock), 0, st, static_cast<T*>(op.y),
                         static_cast<const T*>(op.x), op.djdr, len, cctl);
      break;
    }
    case OP_RHS_MINUS: {
      const long long len = (long long)M * nvox;
      hipLaunchKernelGGL((k_rhs_minus<T>), dim3(kDotBlocks), dim3(kBlock), 0, st, static_cast<T*>(op.y),
                         static_cast<const T*>(op.x), len, cctl);
      break;
    }
    case OP_SET_LOSS: {
      hipLaunchKernelGGL((k_set_loss<T>), dim3(kDotBlocks), dim3(kBlock), 0, st, static_cast<T*>(const_cast<void*>(a.sig)),
                         static_cast<const double*>(op.x), op.djdr, op.gin, N, nvox);
      break;
    }
    case OP_SET_STATE: {
      hipLaunchKernelGGL((k_set_state_f64<T>), dim3(kDotBlocks), dim3(kBlock), 0, st, static_cast<T*>(a.u),
                         static_cast<const double*>(op.x), (long long)op.count * nvox, (long long)M * nvox);
      break;
    }
    case OP_GROWTH: {
      hipLaunchKernelGGL((k_growth_limit<T>), dim3(1), dim3(1024), 0, st, static_cast<const T*>(a.u), M, nvox,
                         op.scale, static_cast<Ctl*>(a.ctl));
      break;
    }
    case OP_GM_UPDATE: {
      hipLaunchKernelGGL((k_gm_update<T>), dim3(1), dim3(64), 0, st, static_cast<GmDev*>(op.u), op.count,
                         static_cast<Ctl*>(a.ctl));
      break;
    }
    case OP_FWD: {
      // spectrum of u for the fused step: the row spectrum on split grids,
      // the xy spectrum on plane grids
      if constexpr (split_planes<NN>()) {
        using V = typename cplx_of<T>::type;
        const int rblocks = M * NN * (NN / RowShape<NN>::RB);
        hipLaunchKernelGGL((k_rows_fwd<T, NN>), dim3(rblocks), dim3(kZBlock), (rows_lds<T, NN>()), st,
                           static_cast<const T*>(a.u), static_cast<V*>(a.spec), static_cast<const V*>(a.tw),
                           cctl);
      } else {
        using V = typename cplx_of<T>::type;
        constexpr int planes = M * NN;
        const T* src = static_cast<const T*>(a.u);
        V* spec = static_cast<V*>(a.spec);
        const V* tw = static_cast<const V*>(a.tw);
        launch_fwd_plane<T, NN>(st, src, spec, tw, cctl, planes);
      }
      break;
    }
    case OP_EXPO:
      if constexpr (N <= kDenseOrder) return enqueue_expo<T, NN, N>(a, op, pr);
      else return hipErrorInvalidValue;
    case OP_PSTEP: {
      // one step of the handle's scheme on op.u in place (op.y holds the
      // stage values); the source is the one in a (null: none)
      T* x = static_cast<T*>(op.u);
      T* tmp = static_cast<T*>(op.y);
      if (a.scheme == 1) {
        enqueue_stage<T, NN, N, EPI_FIRST>(a, nullptr, hc, 1.0, x, x, x);
      } else {
        enqueue_stage<T, NN, N, EPI_FIRST>(a, nullptr, kRkAlpha[0] * hc, 1.0, x, x, tmp);
        enqueue_stage<T, NN, N, EPI_MID>(a, nullptr, kRkAlpha[1] * hc, 1.0, tmp, x, tmp);
        enqueue_stage<T, NN, N, EPI_MID>(a, nullptr, kRkAlpha[2] * hc, 1.0, tmp, x, tmp);
        enqueue_stage<T, NN, N, EPI_MID>(a, nullptr, kRkAlpha[3] * hc, 1.0, tmp, x, x);
      }
      break;
    }
    case OP_ADJ_INJECT: {
      hipLaunchKernelGGL((k_adj_inject<T>), dim3(1), dim3(kBlock), 0, st, static_cast<T*>(op.u), a.det,
                         op.djdr, a.ndet);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
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
    default: break;                                    \
  }                                                    \
  if constexpr (NN <= kHighOrderMaxGrid) {             \
    if (a.N == kHighOrder) return Fn<T, NN, kHighOrder>::call(a, args...); \
  }                                                    \
  return hipErrorInvalidValue;
  if (a.prec == 1) {
    RTE_CASE_N(double)
  } else {
    RTE_CASE_N(float)
  }
#undef RTE_CASE_N
}

template <typename T, int NN, int N> struct EnqueueFn {
  static hipError_t call(const StepArgs& a, const OpArgs* op, ProfRec* pr) { return enqueue_t<T, NN, N>(a, *op, pr); }
};
template <typename T, int NN, int N> struct PrepareFn {
  static hipError_t call(const StepArgs& a) { return prepare_t<T, NN, N>(a); }
};

// Defines the per-size entry points used by the runtime.
#define RTE_DEFINE_SIZE(NN)                                                              \
  int enqueue_op_n##NN(const StepArgs& a, const OpArgs& op, void* pr) {                 \
    return int(dispatch_tn<EnqueueFn, NN>(a, &op, static_cast<ProfRec*>(pr)));           \
  }                                                                                      \
  int prepare_n##NN(const StepArgs& a) { return int(dispatch_tn<PrepareFn, NN>(a)); }

}  // namespace rte
