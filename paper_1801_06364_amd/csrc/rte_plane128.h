// Inverse (and fused forward) plane pass of FP32 128^3 grids with the FFT
// stages that touch HBM or the pointwise epilogue kept in registers.
//
// Per (moment, z-plane) the pass applies the inverse y FFT (128 points), the
// complex-to-real merge and the inverse x FFT (64 packed points) of the xy
// spectrum, the pointwise epilogue (loss, in-scatter, boundary layer,
// source, RK combine; eqs. (9), (11), (12) with the nested RK4 coefficients)
// and, in a time step, the forward x FFT, real-to-complex split and forward
// y FFT of its output plane (the next stage's spectrum). Same inputs,
// outputs and epilogue modes as k_inv_plane; only the schedule differs:
//
//   column FFTs (128 = 16 x 8, Stockham): the first radix-16 stage of the
//     inverse reads its 16 inputs straight from HBM (rows j + 8r of column
//     kx, one 512-byte row segment per wavefront load), the last radix-8
//     stage of the forward writes its outputs straight to HBM;
//   row FFTs (64 = 8 x 8): four lanes per row, each owning the two
//     butterflies j and 8 - j (j = 0 with 4), so the complex-to-real merge
//     (X_k with X_{64-k}) runs in registers before the first stage and the
//     real-to-complex split after the last one; the inverse's last stage
//     leaves each lane the 4 consecutive reals the epilogue needs (one
//     16-byte access per field) and these are exactly the inputs of the
//     forward's first stage, so inverse -> epilogue -> forward needs no LDS.
//
// The plane sits in LDS with an odd row pitch (65 complex values), which
// keeps every access conflict-free (16 lanes of one LDS cycle touch either 16
// consecutive columns of one row or one column of 16 consecutive rows) with
// compile-time offsets from a per-lane base. Six plane-sized LDS writes and
// six reads per plane (instead of one per Stockham stage). Twiddles of the
// column stages depend on the wavefront only (scalar loads); the others come
// from the LDS table exp(-2 pi i t / 128).
#pragma once

namespace rte {
namespace p128 {

constexpr int n = 128, H = 64, PITCH = 65;
#ifndef RTE_P128_NT
#define RTE_P128_NT 1
#endif
#ifndef RTE_P128_XCD
#define RTE_P128_XCD 1
#endif
#ifndef RTE_P128_BATCH
#define RTE_P128_BATCH 2
#endif
constexpr int kEpiBatch = RTE_P128_BATCH;   // epilogue quads per thread with loads in flight
constexpr size_t kLds = size_t(n + n * PITCH) * sizeof(float2);

// Element at a 32-bit byte offset from a uniform base: the address stays a
// scalar base plus one lane register (global_load ... v_off, s_base).
template <typename E, typename P> __device__ __forceinline__ E& at_b(P* base, unsigned byte_off) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return *reinterpret_cast<E*>(const_cast<char*>(reinterpret_cast<C*>(base) + byte_off));
}
template <typename E, typename P> __device__ __forceinline__ E ld_b(P* base, unsigned byte_off) {
  return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + byte_off);
}
// Store of a stream that no kernel of the pass reads again (RTE_P128_NT:
// nontemporal).
__device__ __forceinline__ void st_stream(float4* p, float4 v) {
#if RTE_P128_NT
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<v4*>(p));
#else
  *p = v;
#endif
}
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
#if RTE_P128_NT
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<v2*>(p));
#else
  *p = v;
#endif
}

// w or conj(w): the tables hold exp(-2 pi i t / n); the inverse (DIR = +1)
// uses their conjugates.
template <int DIR> __device__ __forceinline__ float2 twid(float2 w) {
  if constexpr (DIR > 0) w.y = -w.y;
  return w;
}

// Complex-to-real merge of one packed spectral value with its partner
// X_{64-k}: (P + conj Q) + i conj(w) (P - conj Q), w = exp(-2 pi i k / 128).
__device__ __forceinline__ float2 merge_inv(float2 p, float2 q, float2 w) {
  const float dx = p.x - q.x, dy = p.y + q.y;
  const float ex = w.x * dx + w.y * dy, ey = w.x * dy - w.y * dx;
  return cmk<float2>(p.x + q.x - ey, p.y - q.y + ex);
}
// Real-to-complex split: (P + conj Q)/2 - i w (P - conj Q)/2.
__device__ __forceinline__ float2 split_fwd(float2 p, float2 q, float2 w) {
  const float ex = 0.5f * (p.x + q.x), ey = 0.5f * (p.y - q.y);
  const float ox = 0.5f * (p.y + q.y), oy = -0.5f * (p.x - q.x);   // -i (P - conj Q) / 2
  return cmk<float2>(ex + w.x * ox - w.y * oy, ey + w.x * oy + w.y * ox);
}

// Merge (FWD = false) or split (FWD = true) of the two butterflies of a row
// lane: a[r] = X[ja + 8 r], b[r] = X[jb + 8 r], twiddles wa[8 r] and wb[8 r]
// (the LDS table from offsets ja and jb). Lanes t > 0 (ja = t,
// jb = 8 - t) pair a[r] with b[7 - r]; lane t = 0 (ja = 0, jb = 4) pairs
// a[r] with a[8 - r] and b[r] with b[7 - r], X_32 with itself, and packs the
// real X_0 / X_64 column. The partner is chosen by a per-lane select so the
// wavefront runs one path.
template <bool FWD>
__device__ __forceinline__ void pair_rows(float2* a, float2* b, bool t0, const float2* wa, const float2* wb) {
  float2 oa[8], ob[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const float2 qa = t0 ? a[(8 - r) & 7] : b[7 - r];
    const float2 qb = t0 ? b[7 - r] : a[7 - r];
    if constexpr (FWD) {
      oa[r] = split_fwd(a[r], qa, wa[8 * r]);
      ob[r] = split_fwd(b[r], qb, wb[8 * r]);
    } else {
      oa[r] = merge_inv(a[r], qa, wa[8 * r]);
      ob[r] = merge_inv(b[r], qb, wb[8 * r]);
    }
  }
  const float2 z0 = cmk<float2>(a[0].x + a[0].y, a[0].x - a[0].y);
  if (t0) oa[0] = z0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    a[r] = oa[r];
    b[r] = ob[r];
  }
}

// Pointwise epilogue of 4 consecutive reals (one 16-byte access per field);
// same arithmetic as the pair loop of `epilogue`, in single precision with
// the FP64 integrated fluence and partial sums. po: offset in the moment
// fields, vo: offset in the per-voxel fields.
template <int MODE>
__device__ __forceinline__ float4 epi4(float4 w, float4 uu, float4 vv, float4 ss, float4 qq, float qs, float h) {
  float4 o;
  if constexpr (MODE == EPI_SET) return w;
  float s0 = -ss.x * vv.x, s1 = -ss.y * vv.y, s2 = -ss.z * vv.z, s3 = -ss.w * vv.w;
  if constexpr (MODE != EPI_ADJ) {
    s0 += qs * qq.x;
    s1 += qs * qq.y;
    s2 += qs * qq.z;
    s3 += qs * qq.w;
  }
  if constexpr (MODE == EPI_APPLY) {
    o.x = -w.x + ss.x * vv.x;
    o.y = -w.y + ss.y * vv.y;
    o.z = -w.z + ss.z * vv.z;
    o.w = -w.w + ss.w * vv.w;
  } else if constexpr (MODE == EPI_ADJ) {
    o.x = w.x + h * s0;
    o.y = w.y + h * s1;
    o.z = w.z + h * s2;
    o.w = w.w + h * s3;
  } else {
    o.x = uu.x + w.x + h * s0;
    o.y = uu.y + w.y + h * s1;
    o.z = uu.z + w.z + h * s2;
    o.w = uu.w + w.w + h * s3;
  }
  return o;
}

// Forward transform of one real plane (x real-to-complex FFT with the
// kx = 0 / 64 packing, then the y FFT) to the packed xy spectrum `fd` in
// HBM. On entry row lane t of row y = 16 wv + (ln & 15) holds the reals
// x = 4t + 16k .. 4t + 16k + 3 of its row as c0[k] = (x, x + 1), c1[k] =
// (x + 2, x + 3), i.e. elements 2t + 8k and 2t + 1 + 8k of the packed row;
// the twiddle table is in LDS and no lane reads the plane any more. Both the
// fused inverse pass and the standalone forward pass run this code, so a
// spectrum is bitwise the same whichever pass formed it.
__device__ __forceinline__ void forward_plane(float2* c0, float2* c1, float2* pl, const float2* tw,
                                              const float2* __restrict__ twg, float2* fd) {
  const int tid = threadIdx.x, ln = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int t = ln >> 4, y = 16 * wv + (ln & 15);
  const bool t0 = (t == 0);
  const int ja = t, jb = t0 ? 4 : 8 - t;
  float2* row = pl + y * PITCH;
  // ---- x, stage 1 (radix 8): butterflies 2t, 2t + 1 -> elements 8 j + k
  Bfly<float2, 8, -1>::run(c0);
  Bfly<float2, 8, -1>::run(c1);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    row[16 * t + k] = c0[k];
    row[16 * t + 8 + k] = c1[k];
  }
  wave_sync();
  // ---- x, stage 2 (radix 8, twiddles exp(-2 pi i 2 r j / 128)): butterflies (ja, jb), then the split
  {
    float2 a[8], bq[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      a[r] = row[ja + 8 * r];
      bq[r] = row[jb + 8 * r];
    }
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      a[r] = cmul(a[r], tw[2 * r * ja]);
      bq[r] = cmul(bq[r], tw[2 * r * jb]);
    }
    Bfly<float2, 8, -1>::run(a);
    Bfly<float2, 8, -1>::run(bq);
    pair_rows<true>(a, bq, t0, tw + ja, tw + jb);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      row[ja + 8 * r] = a[r];
      row[jb + 8 * r] = bq[r];
    }
  }
  __syncthreads();
  // ---- y, stage 1 (radix 16): column ln, butterfly wv, rows wv + 8 r -> 16 wv + k
  {
    float2 x[16];
    const float2* s = pl + wv * PITCH + ln;
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = s[8 * r * PITCH];
    Bfly<float2, 16, -1>::run(x);
    __syncthreads();
    float2* d = pl + 16 * wv * PITCH + ln;
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k * PITCH] = x[k];
  }
  __syncthreads();
  // ---- y, stage 2 (radix 8, twiddles exp(-2 pi i r j / 128)), to HBM
  const unsigned lo = unsigned(ln) * 8u;
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    const int jp = wv + 8 * hh;
    const float2* c = pl + jp * PITCH + ln;
    float2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = c[16 * r * PITCH];
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], twg[r * jp]);
    Bfly<float2, 8, -1>::run(v);
#pragma unroll
    for (int k = 0; k < 8; ++k) st_stream(&at_b<float2>(fd, lo + unsigned((jp + 16 * k) * H * 8)), v[k]);
  }
}

// Standalone forward transform of real planes (the spectrum of a state set
// from outside a time step): one plane per workgroup of 512 threads
// (BLOCK), plane index b n + z.
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK, 4)
k_fwd128(const float* __restrict__ src, float2* __restrict__ spec, const float2* __restrict__ twg,
         const Ctl* __restrict__ ctl, int nplanes) {
  if (ctl->stop) return;
  extern __shared__ __align__(16) unsigned char smem[];
  float2* tw = reinterpret_cast<float2*>(smem);
  float2* pl = tw + n;
  const int plane = blockIdx.x;
  if (plane >= nplanes) return;
  const int tid = threadIdx.x, ln = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int t = ln >> 4, y = 16 * wv + (ln & 15);
  if (tid < n) tw[tid] = twg[tid];
  const float* sp = src + size_t(plane) * n * n;
  const unsigned off = unsigned(y * n + 4 * t) * 4u;
  float2 c0[8], c1[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 x = ld_b<float4>(sp, off + 64u * unsigned(k));
    c0[k] = cmk<float2>(x.x, x.y);
    c1[k] = cmk<float2>(x.z, x.w);
  }
  __syncthreads();
  forward_plane(c0, c1, pl, tw, twg, spec + size_t(plane) * n * H);
}

template <int MODE, bool FUSE>
__global__ void __launch_bounds__(512, 4)
k_plane128(const float2* spec, const float* vin, float* u, float* dst, const float* __restrict__ sig,
           const float* __restrict__ q, const int* __restrict__ qflag, double* __restrict__ phi_int,
           double* __restrict__ partial, const float2* __restrict__ twg, int M, float h, double dt,
           const Ctl* __restrict__ ctl, int stage, long long step1, float2* fspec, long long bs) {
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
  float2* tw = reinterpret_cast<float2*>(smem);
  float2* pl = tw + n;
#if RTE_P128_XCD
  const int lt = xcd_tile(blockIdx.x, gridDim.x);
#else
  const int lt = blockIdx.x;
#endif
  const int z = lt / M, b = lt - z * M;
  const int plane = b * n + z;
  const int tid = threadIdx.x, ln = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront index (uniform)
  if (tid < n) tw[tid] = twg[tid];

  // ---- inverse y, stage 1 (radix 16, from HBM): column ln, butterfly wv
  {
    const float2* sp = spec + size_t(plane) * n * H + wv * H;
    const unsigned lo = unsigned(ln) * 8u;
    float2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = ld_b<float2>(sp, lo + unsigned(8 * r * H * 8));
    Bfly<float2, 16, +1>::run(x);
    float2* d = pl + 16 * wv * PITCH + ln;
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k * PITCH] = x[k];
  }
  __syncthreads();
  // ---- inverse y, stage 2 (radix 8, twiddles exp(+2 pi i r j / 128)): butterflies wv, wv + 8
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    const int jp = wv + 8 * hh;
    float2* c = pl + jp * PITCH + ln;
    float2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = c[16 * r * PITCH];
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], twid<+1>(twg[r * jp]));
    Bfly<float2, 8, +1>::run(v);
#pragma unroll
    for (int k = 0; k < 8; ++k) c[16 * k * PITCH] = v[k];
  }
  __syncthreads();

  // ---- rows: lane t of row y owns butterflies (ja, jb)
  const int t = ln >> 4, y = 16 * wv + (ln & 15);
  const bool t0 = (t == 0);
  const int ja = t, jb = t0 ? 4 : 8 - t;
  float2* row = pl + y * PITCH;

  // epilogue fields: uniform bases (scalar registers) and one 32-bit lane
  // offset shared by every field (set up before the row FFT: computing them
  // inside the epilogue made the middle-stage variant spill)
  constexpr bool kLast = (MODE == EPI_LAST || MODE == EPI_EULER);
  const int l = isqrt_c(b);
  constexpr bool kSrc = (MODE == EPI_FIRST || MODE == EPI_MID || MODE == EPI_LAST || MODE == EPI_EULER);
  const bool hasq = kSrc && (q != nullptr) && qflag[z];
  const float qs = hasq ? float(source_weight(ctl, stage, step1)) : 0.f;
  const size_t vbase = size_t(z) * n * n, pbase = size_t(b) * n * n * n + vbase;
  const float* ub = u + pbase;
  float* ubw = u + pbase;
  const float* vb = vin + pbase;
  float* db = dst + pbase;
  const float* sb = sig + size_t(l) * n * n * n + vbase;
  const float* qb = q + pbase;
  double* pb = phi_int + vbase;
  const unsigned off = unsigned(y * n + 4 * t) * 4u;   // bytes of a float field
  auto epi_load = [&](int k, float4& uu, float4& vv, float4& ss, float4& qq) {
    const unsigned e = off + 64u * unsigned(k);
    if constexpr (MODE != EPI_SET) {
      if constexpr (MODE != EPI_APPLY) uu = ld_b<float4>(ub, e);
      else uu = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (MODE == EPI_FIRST || MODE == EPI_EULER) vv = uu;
      else vv = ld_b<float4>(vb, e);
      ss = ld_b<float4>(sb, e);
      qq = hasq ? ld_b<float4>(qb, e) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  float2 a[8], bq[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    a[r] = row[ja + 8 * r];
    bq[r] = row[jb + 8 * r];
  }
  pair_rows<false>(a, bq, t0, tw + ja, tw + jb);
  // inverse x, stage 1 (radix 8): outputs 8 j + k
  Bfly<float2, 8, +1>::run(a);
  Bfly<float2, 8, +1>::run(bq);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    row[8 * ja + k] = a[k];
    row[8 * jb + k] = bq[k];
  }
  wave_sync();
  // inverse x, stage 2 (radix 8, twiddles exp(+2 pi i 2 r j / 128)): butterflies 2t, 2t + 1
  float2 c0[8], c1[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    c0[r] = row[2 * t + 8 * r];
    c1[r] = row[2 * t + 1 + 8 * r];
  }
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    c0[r] = cmul(c0[r], twid<+1>(tw[2 * r * (2 * t)]));
    c1[r] = cmul(c1[r], twid<+1>(tw[2 * r * (2 * t + 1)]));
  }
  Bfly<float2, 8, +1>::run(c0);
  Bfly<float2, 8, +1>::run(c1);
  wave_sync();

  // ---- epilogue: element 2t + 8k holds reals x = 4t + 16k, 4t + 16k + 1
  double acc_d = 0.0, acc_o = 0.0;
  {
    const bool fl = kLast && b == 0;
#pragma unroll
    for (int half = 0; half < 8 / kEpiBatch; ++half) {
      // (the compiler would otherwise hoist every batch's loads to the top
      // and run out of registers)
      if (half > 0) asm volatile("" ::: "memory");
      float4 uu[kEpiBatch], vv[kEpiBatch], ss[kEpiBatch], qq[kEpiBatch];
#pragma unroll
      for (int i = 0; i < kEpiBatch; ++i) {
        epi_load(kEpiBatch * half + i, uu[i], vv[i], ss[i], qq[i]);
      }
#pragma unroll
      for (int i = 0; i < kEpiBatch; ++i) {
        const int k = kEpiBatch * half + i;
        const unsigned e = off + 64u * unsigned(k);
        const float4 w4 = make_float4(c0[k].x, c0[k].y, c1[k].x, c1[k].y);
        const float4 o = epi4<MODE>(w4, uu[i], vv[i], ss[i], qq[i], qs, h);
        st_stream(&at_b<float4>(db, e), o);
        if constexpr (MODE == EPI_ADJ)
          at_b<float4>(ubw, e) = make_float4(uu[i].x + o.x, uu[i].y + o.y, uu[i].z + o.z, uu[i].w + o.w);
        if constexpr (kLast) {
          if (fl) {
            double4& pi = at_b<double4>(pb, 2u * e);
            double4 acc = pi;
            acc.x += dt * double(o.x);
            acc.y += dt * double(o.y);
            acc.z += dt * double(o.z);
            acc.w += dt * double(o.w);
            pi = acc;
            const double d0 = double(o.x) - double(uu[i].x), d1 = double(o.y) - double(uu[i].y);
            const double d2 = double(o.z) - double(uu[i].z), d3 = double(o.w) - double(uu[i].w);
            acc_d += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
            acc_o += double(o.x) * double(o.x) + double(o.y) * double(o.y) + double(o.z) * double(o.z) +
                     double(o.w) * double(o.w);
          }
        }
        c0[k] = cmk<float2>(o.x, o.y);
        c1[k] = cmk<float2>(o.z, o.w);
      }
    }
  }

  if constexpr (FUSE) forward_plane(c0, c1, pl, tw, twg, fspec + size_t(plane) * n * H);
  // (block_sum2 reuses the LDS: it synchronises first)
  if ((MODE == EPI_LAST || MODE == EPI_EULER) && b == 0) block_sum2<512>(smem, acc_d, acc_o, partial + 2 * z);
}

}  // namespace p128
}  // namespace rte
