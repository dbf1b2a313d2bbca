// Internal declarations shared by the host table builder and the HIP
// runtime of the P_N stepper (not part of the public C-ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace rte {

// Orders built: every N <= kDenseOrder on every grid, and the high order
// kHighOrder (484 moments, the paper's first experiment) on grids of at
// most kHighOrderMaxGrid points per axis.
constexpr int kDenseOrder = 7;
constexpr int kHighOrder = 21;
constexpr int kHighOrderMaxGrid = 64;
constexpr int kMaxOrder = kHighOrder;              // largest order of any table
constexpr bool order_built(int N, int n) {
  return (N >= 0 && N <= kDenseOrder) || (N == kHighOrder && n <= kHighOrderMaxGrid);
}
// Largest Taylor degree of the exact propagation per working precision.
constexpr int kTaylorMaxF32 = 14;
constexpr int kTaylorMaxF64 = 24;
constexpr int kMaxSlots = 12;                      // coupling slots per row

constexpr int isqrt_c(int a) {
  int l = 0;
  while ((l + 1) * (l + 1) <= a) ++l;
  return l;
}

// Candidate coupling partners of real-basis row (l, m). The streaming
// operator of eq. (6) moves degree l to l +- 1 and order m to m or m +- 1;
// in the real basis (cos / sin pairs) a row (l, m) can therefore only reach
// (l +- 1, m') with m' in {m-1, m, m+1, -m-1, -m, -m+1}. The slots list those
// partners (in range, de-duplicated, ascending l' then m'); the kernels
// unroll their coupling sums over these slots at compile time.
struct SlotList {
  int count;
  int b[kMaxSlots];
};

constexpr SlotList slots_of(int N, int l, int m) {
  SlotList s{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  for (int dl = -1; dl <= 1; dl += 2) {
    const int lp = l + dl;
    if (lp < 0 || lp > N) continue;
    const int cand[6] = {m - 1, m, m + 1, -m - 1, -m, -m + 1};
    // ascending, de-duplicated
    for (int mp = -lp; mp <= lp; ++mp) {
      bool hit = false;
      for (int c = 0; c < 6; ++c) hit = hit || (cand[c] == mp);
      if (hit) s.b[s.count++] = lp * lp + lp + mp;
    }
  }
  return s;
}

// ---------------------------------------------------------------- tables --

// Real-basis streaming matrices (dense M x M, row-major, FP64) built from
// the complex-basis coefficients of eq. (6) and the unitary change of basis
// to real harmonics without Condon-Shortley phase. Returns false if N is out
// of range or a non-zero entry falls outside the slot pattern.
bool coupling_dense(int N, std::vector<double>& bx, std::vector<double>& by,
                    std::vector<double>& bz);

// Real-harmonic representation of the rotation by +90 degrees about x
// (y -> z): one (2l+1)^2 block per degree l <= N, row-major, concatenated.
// Computed by exact quadrature and checked against the streaming matrices
// (D (k.B) D^T = (X k).B); false if the check fails or N is out of range.
bool rotation_x90(int N, std::vector<double>& D);

// Coupling slot table of the high-order pass: per row a, the non-zeros of
// the real-basis streaming matrices as codes (b << 2 | axis) in slot order,
// -1 after the last, and their FP64 values. Returns false for an order that
// is not built.
bool coupling_table(int N, std::vector<int>& code, std::vector<double>& val);

// Twiddles exp(-2 pi i t / n), t in [0, n), as interleaved (cos, sin) FP64.
void twiddles(int n, std::vector<double>& tw);

// Wavenumbers 2 pi f / (n dx) in FFT order with the Nyquist entry zero.
void wavenumbers(int n, double dx, std::vector<double>& k);

// Per-degree loss Sigma_l(r), [N+1][n^3], and the real-domain mask:
// mu_a + mu_s (1 - g^l) inside [W, n-W)^3, mu_b (half-cosine layer) outside.
void potentials(int n, int N, int W, double mu0, double mu1,
                const double* mu_a, const double* mu_s, const double* g,
                std::vector<double>& sig, std::vector<uint8_t>& inside);

// Supported grid sizes for the in-LDS plane passes.
bool grid_supported(int n);

// ------------------------------------------------------- step launcher --

// Krylov solver limits: basis vectors (restart + 1) and dot-product
// partial sums (blocks x basis vectors).
constexpr int kMaxBasisVectors = 32;
constexpr int kDotPartials = 1024 * kMaxBasisVectors;

// Device-side state of one GMRES restart cycle (in the Krylov workspace):
// the Arnoldi coefficients of the newest vector, the rotated Hessenberg
// matrix and the Givens rotations, so that an Arnoldi step needs no host
// round trip; the host reads the block once per cycle.
struct GmDev {
  double hv[kMaxBasisVectors + 1];   // <v_i, w> of the first Gram-Schmidt pass
  double h2[kMaxBasisVectors + 1];   // of the second pass
  double hn2;                        // squared norm of the orthogonalised vector
  double hn;                         // its norm (the normalisation divisor)
  double ref;                        // reference norm of the relative residual
  double tol;                        // stop when |g[j+1]| / ref <= tol
  double R[kMaxBasisVectors * kMaxBasisVectors];  // rotated Hessenberg, R[i * m + j], i <= j
  double cs[kMaxBasisVectors];
  double sn[kMaxBasisVectors];
  double g[kMaxBasisVectors + 1];    // rotated residual vector
  int m;                             // restart length (row stride of R)
  int jdone;                         // Arnoldi steps completed in this cycle
};

// Device control block: step counter and run/stop flags shared by every
// kernel of a step (kernels return at once when stop != 0).
struct Ctl {
  long long step;       // steps applied since creation / last set_state
  int stop;             // 0 run, 1 converged (tol met), 2 unstable, 3 step limit
                        // reached or slot idle (batched serving)
  int pad;
  double tol;           // relative fluence change that stops a run (0: off)
  double growth_limit;  // ||phi||^2 above this flags runaway growth
  double last_resid;
  double last_norm2;
  // time profile of the source: per-step stage weights [qw_rows][qw_cols]
  // (null: constant source, weight 1); steps past the table use its last row
  const double* qw;
  long long qw_rows;
  int qw_cols;
  int pad2;
  // batched serving: the slot's run ends (stop = 3) once step reaches
  // limit (0: no limit)
  long long limit;
};

// Everything one RK4 step needs, as plain device pointers (carved from the
// caller's workspace) and scalars. Field pointers are of the working
// precision (float or double) and complex spectra interleave (re, im).
struct StepArgs {
  int prec;                 // 0 = FP32, 1 = FP64
  int scheme;               // 0 = nested RK4, 1 = forward Euler
  int N, M;                 // order and moment count
  void* stream;             // hipStream_t
  void* u;                  // state [M][n^3]
  void* v;                  // stage state [M][n^3]
  void* spec;               // xy spectrum [M][n][n][n/2] complex (kx = 0 packs
                            // the real kx = 0 and kx = n/2 columns)
  void* dspec;              // its z derivative, same layout
  void* wspec;              // coupled spectrum (orders above kDenseOrder only)
  const int* ctab;          // coupling slots [M][kMaxSlots]: (b << 2 | axis), -1 ends
                            // (orders above kDenseOrder only)
  const void* cval;         // their coefficients [M][kMaxSlots] (working precision)
  const void* tw;           // twiddles exp(-2 pi i t / n), n complex
  const void* kv;           // wavenumbers, n
  const void* sig;          // per-degree loss [N+1][n^3]
  const void* q;            // source [M][n^3] or nullptr
  const int* qflag;         // per z-plane: source present
  double* phi_int;          // integrated fluence [n^3]
  double* partial;          // per z-plane fluence-change partial sums [n][2]
  double* readings;         // [cap][ndet]
  double* resid;            // [cap]
  const long long* det;     // [ndet]
  int ndet;
  long long cap;
  void* ctl;                // device control block
  double c, dt;
  // batched launches (serving): nslot solves of one configuration whose
  // workspaces lie sstride bytes apart, the pointers above being those of
  // slot 0; grid row blockIdx.y selects the slot (0 / 1: a single solve)
  int nslot;
  long long sstride;
};

// Kernel classes timed by the profiling entry point.
enum {
  PROF_FWD_PLANE = 0, PROF_ZDERIV, PROF_COUPLE, PROF_INV_PLANE, PROF_END,
  PROF_FWD_ROWS, PROF_Y_FWD, PROF_Y_INV, PROF_INV_ROWS,
  PROF_Z_FWD, PROF_EXPO, PROF_Z_INV, PROF_EXPO_TABLE, PROF_CLASSES
};
constexpr int kMaxProfLaunches = 32;

// Event record of one profiled step: ev0 before the first launch, ev[i]
// after launch i, whose kernel class is cls[i].
struct ProfRec {
  void* ev0;
  void* ev[kMaxProfLaunches];
  int cls[kMaxProfLaunches];
  int count;
};

// Device operations queued by the per-grid-size entry points.
enum {
  OP_STEP = 0,       // one RK4 step with readings / integrated fluence / flags
  OP_STAGE = 1,      // one forward stage into a given buffer (no bookkeeping)
  OP_ADJ_STAGE = 2,  // one transposed stage: y = coef h F~(x), u += y
  OP_ADJ_GRAD = 3,   // gradient accumulation from (x, y)
  OP_ADJ_INJECT = 4, // detector adjoint sources into u
  OP_APPLY = 5,      // y = (S + Sigma) x (steady-state operator)
  OP_WDOTS = 6,      // gmus[i] = <x_i, y>_W, i < count (x: count vectors)
  OP_COMBINE = 7,    // y = coef * y + scale * sum_i djdr[i] x_i
  OP_SCALE = 8,      // y = x / djdr[0]
  OP_RHS_MINUS = 9,  // y = x - y (x may be null)
  OP_EXPO = 10,      // u <- exact propagation over time coef (homogeneous medium)
  OP_PSTEP = 11,     // u <- one time step of u (y: stage scratch), no bookkeeping
  OP_FWD = 12,       // spectrum of u (the entry condition of a fused OP_STEP)
  OP_GM_UPDATE = 13, // GMRES: Hessenberg column count (= j + 1) from the GmDev at u;
                     // sets the control block's stop flag once converged
  OP_SET_LOSS = 14,  // loss maps inside the real domain from device FP64 mu_a (x) and
                     // mu_s (djdr), with g from gin (the layer keeps its loss)
  OP_SET_STATE = 15, // u <- device FP64 moments x (count leading moments, the rest 0)
  OP_GROWTH = 16     // growth threshold of the control block from the weighted energy of u
                     // and the source term (scale)
};
struct OpArgs {
  int kind;
  int stage;         // OP_STAGE: 0..2
  double coef;       // OP_ADJ_STAGE / OP_ADJ_GRAD: RK stage coefficient
  void* u;           // base state / accumulator
  const void* x;     // stage input
  void* y;           // stage output
  const double* gin; // g inside the real domain, > 1 in the layer
  double* gmua;      // gradient accumulators (FP64, n^3)
  double* gmus;
  const double* djdr;// adjoint sources of one step's readings (ndet); device
                     // coefficients of OP_COMBINE / OP_SCALE
  int count;         // OP_WDOTS / OP_COMBINE: number of basis vectors; OP_EXPO: 1 =
                     // rotation path
  double scale;      // OP_COMBINE; OP_EXPO: per-substep norm limit theta
  double eps;        // OP_EXPO: Taylor truncation target
  double sigl[kMaxOrder + 1];  // OP_EXPO: per-degree loss of the medium
  double kunit;      // OP_EXPO: 2 pi / (n dx); with count = 1 the rotation
                     // data sit in the stage buffer v
  int fused;         // OP_STEP: the spectrum of u is in place on entry and is
                     // left in place for the next step (plane grids)
  long long step1;   // OP_STEP / OP_STAGE: 1 + the step index whose source
                     // weights apply (0: the control block's step counter)
};

// Per-grid-size entry points (one translation unit per n). enqueue_op
// queues one operation; pr (a ProfRec*) is null except when profiling a
// step.
int launch_enqueue_op(int n, const StepArgs& a, const OpArgs& op, void* pr);
int launch_prepare(int n, const StepArgs& a);

}  // namespace rte
