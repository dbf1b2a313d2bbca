// Pencil passes of FP32 128^3 and 256^3 grids with the FFT stages that
// touch HBM kept in registers.
//
// A workgroup owns TZ kx columns of one pencil (all n points along the
// pencil axis, z for the z derivative, y for the y passes of 256^3 grids).
// Thread (kx, j) loads the 16 points j + (n/16) r of its column straight
// from HBM (one row segment of TZ complex values per wavefront
// load) and applies the first radix-16 Stockham stage in registers; one
// exchange through LDS (row pitch TZ: the 16 lanes of one LDS cycle touch
// 16 consecutive columns of a row) feeds the last stage, whose outputs are
// in natural order. For the z derivative the product with i k_z / n and the
// first stage of the inverse transform follow in registers on exactly those
// outputs, then one more exchange and the inverse's last stage, written
// straight to HBM. Plans (verified against a direct DFT): 256 = 16 x 16 both
// ways; 128 = 16 x 8 forward, 8 x 16 inverse. Twiddles come from an LDS copy
// of the table exp(-2 pi i t / n).
#pragma once

namespace rte {
namespace pen {

#ifndef RTE_PEN_TZ128
#define RTE_PEN_TZ128 16
#endif
#ifndef RTE_PEN_TZ256
#define RTE_PEN_TZ256 16
#endif

// TZ columns per workgroup; J = n / 16 threads per column, one per radix-16
// butterfly of the first stage; LDS holds the whole n x TZ tile. TZ = 8 and
// 32 measured no faster than 16 at either size.
template <int NN> struct Shape;
template <> struct Shape<128> {
  static constexpr int TZ = RTE_PEN_TZ128, NTILE = 64 / TZ, J = 8, THREADS = J * TZ;
};
template <> struct Shape<256> {
  static constexpr int TZ = RTE_PEN_TZ256, NTILE = 128 / TZ, J = 16, THREADS = J * TZ;
};

// FP32 pencils of these grids and modes run here; the others (FP64, the
// full 3D transforms of the exact propagation) in k_pencil.
template <typename T, int NN, int MODE> constexpr bool use_reg() {
  return std::is_same<T, float>::value && (NN == 128 || NN == 256) &&
         (MODE == PENCIL_ZDERIV || (NN == 256 && (MODE == PENCIL_YFWD || MODE == PENCIL_YINV)));
}

template <int DIR> __device__ __forceinline__ float2 tw_dir(float2 w) {
  if constexpr (DIR > 0) w.y = -w.y;
  return w;
}

// x <- x * (i k / n)
__device__ __forceinline__ float2 times_ik(float2 x, float k) { return cmk<float2>(-k * x.y, k * x.x); }

template <int NN, int MODE>
__global__ void __launch_bounds__(Shape<NN>::THREADS)
k_pencil_reg(const float2* src, float2* dst,   // may alias (in place)
             const float2* __restrict__ twg, const float* __restrict__ kv, const Ctl* __restrict__ ctl,
             long long bs) {
  constexpr int n = NN, H = NN / 2, TZ = Shape<NN>::TZ, NTILE = Shape<NN>::NTILE;
  constexpr size_t AX = pencil_z(MODE) ? size_t(n) * H : size_t(H);
  constexpr int DIR = pencil_inverse(MODE) ? +1 : -1;
  src = slot_ptr(src, bs);
  dst = slot_ptr(dst, bs);
  twg = slot_ptr(twg, bs);
  kv = slot_ptr(kv, bs);
  ctl = slot_ptr(ctl, bs);
  if (ctl->stop) return;
  __shared__ float2 tw[n];
  __shared__ float2 col[n * TZ];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bw = tile / NTILE;
  const int kx0 = (tile - bw * NTILE) * TZ;
  const int b = bw / n, w = bw - b * n;
  const size_t base = pencil_z(MODE) ? (size_t(b) * n * n + w) * H + kx0 : (size_t(b) * n + w) * size_t(n) * H + kx0;
  const int tid = threadIdx.x, kx = tid % TZ, j = tid / TZ;
  for (int i = tid; i < n; i += Shape<NN>::THREADS) tw[i] = twg[i];
  const float2* s = src + base + kx;
  float2* d = dst + base + kx;
  constexpr float inv_n = 1.0f / float(n);
  if constexpr (NN == 256) {
    // j < 16: stage 1 radix 16 over rows j + 16 r, stage 2 radix 16 (butterfly j)
    float2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = s[size_t(j + 16 * r) * AX];
    Bfly<float2, 16, DIR>::run(x);
#pragma unroll
    for (int q = 0; q < 16; ++q) col[(16 * j + q) * TZ + kx] = x[q];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = col[(j + 16 * r) * TZ + kx];
#pragma unroll
    for (int r = 1; r < 16; ++r) x[r] = cmul(x[r], tw_dir<DIR>(tw[r * j]));
    Bfly<float2, 16, DIR>::run(x);   // element j + 16 q
    if constexpr (MODE == PENCIL_ZDERIV) {
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = times_ik(x[q], kv[j + 16 * q] * inv_n);
      Bfly<float2, 16, +1>::run(x);  // inverse stage 1 on the same elements: outputs 16 j + q
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 16; ++q) col[(16 * j + q) * TZ + kx] = x[q];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = col[(j + 16 * r) * TZ + kx];
#pragma unroll
      for (int r = 1; r < 16; ++r) x[r] = cmul(x[r], tw_dir<+1>(tw[r * j]));
      Bfly<float2, 16, +1>::run(x);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) d[size_t(j + 16 * q) * AX] = x[q];
  } else {
    // j < 8: stage 1 radix 16 over rows j + 8 r, stage 2 radix 8 (butterflies j, j + 8)
    float2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = s[size_t(j + 8 * r) * AX];
    Bfly<float2, 16, DIR>::run(x);
#pragma unroll
    for (int q = 0; q < 16; ++q) col[(16 * j + q) * TZ + kx] = x[q];
    __syncthreads();
    float2 a[8], c[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      a[r] = col[(j + 16 * r) * TZ + kx];
      c[r] = col[(j + 8 + 16 * r) * TZ + kx];
    }
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      a[r] = cmul(a[r], tw_dir<DIR>(tw[r * j]));
      c[r] = cmul(c[r], tw_dir<DIR>(tw[r * (j + 8)]));
    }
    Bfly<float2, 8, DIR>::run(a);   // elements j + 16 q
    Bfly<float2, 8, DIR>::run(c);   // elements j + 8 + 16 q
    if constexpr (MODE == PENCIL_ZDERIV) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = times_ik(a[q], kv[j + 16 * q] * inv_n);
        c[q] = times_ik(c[q], kv[j + 8 + 16 * q] * inv_n);
      }
      // inverse: radix 8 (stride 1) on the same elements -> 8 j' + q, then radix 16 (stride 8)
      Bfly<float2, 8, +1>::run(a);
      Bfly<float2, 8, +1>::run(c);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        col[(8 * j + q) * TZ + kx] = a[q];
        col[(8 * (j + 8) + q) * TZ + kx] = c[q];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = col[(j + 8 * r) * TZ + kx];
#pragma unroll
      for (int r = 1; r < 16; ++r) x[r] = cmul(x[r], tw_dir<+1>(tw[r * j]));
      Bfly<float2, 16, +1>::run(x);
#pragma unroll
      for (int q = 0; q < 16; ++q) d[size_t(j + 8 * q) * AX] = x[q];
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        d[size_t(j + 16 * q) * AX] = a[q];
        d[size_t(j + 8 + 16 * q) * AX] = c[q];
      }
    }
  }
}

}  // namespace pen
}  // namespace rte
