// Pencil passes of FP32 grids with the FFT stages that touch HBM kept in
// registers: the z derivative at 32^3, 64^3, 96^3, 128^3 and 256^3, the y
// passes of 256^3 grids.
//
// A workgroup owns TZ kx columns of one pencil (all n points along the
// pencil axis, z for the z derivative, y for the y passes of 256^3 grids).
// At 128 and 256, thread (kx, j) loads the 16 points j + (n/16) r of its
// column straight from HBM (one row segment of TZ complex values per
// wavefront load) and applies the first radix-16 Stockham stage in
// registers; one exchange through LDS (row pitch TZ: the 16 lanes of one LDS
// cycle touch 16 consecutive columns of a row) feeds the last stage, whose
// outputs are in natural order. For the z derivative the product with
// i k_z / n and the first stage of the inverse transform follow in registers
// on exactly those outputs, then one more exchange and the inverse's last
// stage, written straight to HBM. At 96, 64 and 32 four threads share a
// column, each loading the n/4 points j + 4 r. Plans (verified against a
// direct DFT): 256 = 16 x 16 both ways; 128 = 16 x 8 forward, 8 x 16
// inverse; 96 = 24 x 4, 64 = 16 x 4 and 32 = 8 x 4 both ways (the radix-24
// stage as 8 x 3 with constant twiddles). Twiddles between the stages come
// from an LDS copy of the table exp(-2 pi i t / n).
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
// 96, 64 and 32: J = 4 threads per column (radix-24 / 16 / 8 first stage),
// TZ = 16 kx columns per workgroup (one wavefront)
template <> struct Shape<96> {
  static constexpr int TZ = 16, NTILE = 48 / TZ, J = 4, THREADS = J * TZ;
};
template <> struct Shape<64> {
  static constexpr int TZ = 16, NTILE = 32 / TZ, J = 4, THREADS = J * TZ;
};
template <> struct Shape<32> {
  static constexpr int TZ = 16, NTILE = 16 / TZ, J = 4, THREADS = J * TZ;
};

// FP32 pencils of these grids and modes run here; the others (FP64, the
// full 3D transforms of the exact propagation) in k_pencil.
template <typename T, int NN, int MODE> constexpr bool use_reg() {
  return std::is_same<T, float>::value && (NN == 32 || NN == 64 || NN == 96 || NN == 128 || NN == 256) &&
         (MODE == PENCIL_ZDERIV || (NN == 256 && (MODE == PENCIL_YFWD || MODE == PENCIL_YINV)));
}

template <int DIR> __device__ __forceinline__ float2 tw_dir(float2 w) {
  if constexpr (DIR > 0) w.y = -w.y;
  return w;
}

// x <- x * (i k / n)
__device__ __forceinline__ float2 times_ik(float2 x, float k) { return cmk<float2>(-k * x.y, k * x.x); }

// cos(t pi / 12) from the closed forms of the multiples of 15 degrees
__host__ __device__ constexpr double cos_pi12(int t) {
  constexpr double c[7] = {1.0, 0.96592582628906828675, 0.86602540378443864676, 0.70710678118654752440,
                           0.5, 0.25881904510252076235, 0.0};
  t = ((t % 24) + 24) % 24;
  if (t > 12) t = 24 - t;
  return t <= 6 ? c[t] : -c[12 - t];
}

// exp(DIR 2 pi i t / 24)
template <int DIR> __device__ __forceinline__ float2 w24(int t) {
  return cmk<float2>(float(cos_pi12(t)), float(DIR) * float(cos_pi12(6 - t)));
}

// 24-point DFT in registers, x[q] <- sum_r x[r] exp(DIR 2 pi i q r / 24):
// r = a + 3 b, q = c + 8 d; radix 8 over b for each a, twiddles
// exp(DIR 2 pi i a c / 24), radix 3 over a.
template <int DIR> __device__ __forceinline__ void dft24(float2* x) {
  float2 y[3][8];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 8; ++b) y[a][b] = x[a + 3 * b];
    Bfly<float2, 8, DIR>::run(y[a]);
  }
#pragma unroll
  for (int c = 1; c < 8; ++c) {
    y[1][c] = cmul(y[1][c], w24<DIR>(c));
    y[2][c] = cmul(y[2][c], w24<DIR>(2 * c));
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    float2 z[3] = {y[0][c], y[1][c], y[2][c]};
    Bfly<float2, 3, DIR>::run(z);
#pragma unroll
    for (int d = 0; d < 3; ++d) x[c + 8 * d] = z[d];
  }
}

// R-point DFT in registers (natural order in and out) of the four-thread
// column plans
template <int R, int DIR> __device__ __forceinline__ void dft_col(float2* x) {
  if constexpr (R == 24) dft24<DIR>(x);
  else Bfly<float2, R, DIR>::run(x);
}

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
  // 96 / 64 / 32: the four row blocks of the tile sit PAD entries apart, so
  // that the four row groups of one wavefront access fall in different banks
  constexpr int PAD = (NN == 96 || NN == 64 || NN == 32) ? 16 : 0;
  __shared__ float2 tw[n];
  __shared__ float2 col[n * TZ + 4 * PAD];
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
  if constexpr (NN == 96 || NN == 64 || NN == 32) {
    static_assert(MODE == PENCIL_ZDERIV, "96-, 64- and 32-point register pencils do the z derivative only");
    // R = n / 4. Thread j < 4: stage 1 radix R over rows j + 4 r -> Y_j[k1];
    // stage 2 radix 4 over j for k1 = j + 4 t (t < R / 4) -> X[k1 + R k2],
    // with the twiddles exp(-2 pi i j k1 / n) applied after the exchange
    constexpr int R = NN / 4, NT = R / 4;
    auto at = [&](int blk, int row) { return (R * blk + row) * TZ + blk * PAD + kx; };
    float2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = s[size_t(j + 4 * r) * AX];
    dft_col<R, -1>(x);
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) col[at(j, k1)] = x[k1];
    __syncthreads();
    float2 y[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int k1 = j + 4 * t;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) y[t][jj] = col[at(jj, k1)];
#pragma unroll
      for (int jj = 1; jj < 4; ++jj) y[t][jj] = cmul(y[t][jj], tw_dir<-1>(tw[jj * k1]));
      Bfly<float2, 4, -1>::run(y[t]);   // element k1 + R k2
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) y[t][k2] = times_ik(y[t][k2], kv[k1 + R * k2] * inv_n);
      // inverse: radix 4 over k2 -> Z[k1][p], times exp(2 pi i k1 p / n)
      Bfly<float2, 4, +1>::run(y[t]);
#pragma unroll
      for (int p = 1; p < 4; ++p) y[t][p] = cmul(y[t][p], tw_dir<+1>(tw[k1 * p]));
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int p = 0; p < 4; ++p) col[at(p, j + 4 * t)] = y[t][p];
    __syncthreads();
    // thread p = j: radix R over k1 -> output rows p + 4 s
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) x[k1] = col[at(j, k1)];
    dft_col<R, +1>(x);
#pragma unroll
    for (int q = 0; q < R; ++q) d[size_t(j + 4 * q) * AX] = x[q];
  } else if constexpr (NN == 256) {
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
