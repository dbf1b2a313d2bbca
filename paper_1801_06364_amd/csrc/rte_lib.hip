// MI355X (gfx950) P_N pseudospectral transport stepper: runtime (handle,
// workspace carve-up, table upload, graph capture, run control) and the
// C-ABI declared in include/rte.h. The kernels live in rte_kernels.h, one
// translation unit per grid size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/rte.h"
#include "rte_internal.h"

namespace rte {
namespace {
// The library's static device scratch array: the Krylov workspace of the
// no-allocation GMRES entry point. Each GPU holds its own copy for the life
// of the process; its device address is looked up once per device (with
// that device current) and kept, since host code may not use the symbol
// itself as a device address.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
}  // namespace
}  // namespace rte

static __device__ __align__(256) unsigned char scratch[rte::kScratchBytes];

namespace rte {
namespace {
// Device address of `scratch` on device dev (null on failure, *err set).
void* scratch_on(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::call_once(g_scratch_once[dev], [dev] {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
  });
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace
}  // namespace rte


namespace rte {

// ------------------------------------------------------------ runtime ---

constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t u, v, spec, dspec, wspec, ctab, cval, sig, q, qflag, tw, kv, det, readings, resid, partial, phi_int,
      gin, ctl,
      total;
};

inline bool config_ok(const rte_config* c) {
  if (!c) return false;
  if (!grid_supported(c->n)) return false;
  if (!order_built(c->order_N, c->n)) return false;
  if (c->precision != RTE_FP32 && c->precision != RTE_FP64) return false;
  if (c->pml_width < 0 || 2 * c->pml_width >= c->n) return false;
  if (!(c->dx_mm > 0) || !(c->c_mm_ps > 0) || !std::isfinite(c->dx_mm) || !std::isfinite(c->c_mm_ps))
    return false;
  if (!std::isfinite(c->dt_ps)) return false;
  if (c->pml_width > 0 && (!(c->pml_mu0 >= 0) || !(c->pml_mu1 >= 0))) return false;
  if (c->n_det < 0 || (c->n_det > 0 && !c->det_index)) return false;
  if (c->record_steps < 0) return false;
  if (c->scheme != RTE_RK4 && c->scheme != RTE_EULER) return false;
  // grids up to 128 keep one n x (n/2+1) complex plane in LDS (160 KB per
  // CU); larger grids use row + pencil passes
  const size_t s = c->precision == RTE_FP64 ? 16 : 8;
  if (c->n <= 128 && (size_t(c->n) * (c->n / 2 + 1) + c->n) * s > 160 * 1024) return false;
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
  L.spec = o; o = up(o + M * n * n * (n / 2) * 2 * s);
  L.dspec = o; o = up(o + M * n * n * (n / 2) * 2 * s);
  // orders above kDenseOrder: coupled-spectrum buffer and slot table
  const bool high = c->order_N > kDenseOrder;
  L.wspec = o; o = up(o + (high ? M * n * n * (n / 2) * 2 * s : 0));
  L.ctab = o; o = up(o + (high ? M * kMaxSlots * sizeof(int) : 0));
  L.cval = o; o = up(o + (high ? M * kMaxSlots * s : 0));
  L.sig = o; o = up(o + size_t(c->order_N + 1) * V * s);
  L.q = o; o = up(o + (has_q ? M * V * s : 0));
  L.qflag = o; o = up(o + n * sizeof(int));
  L.tw = o; o = up(o + n * 2 * s);
  L.kv = o; o = up(o + n * s);
  L.det = o; o = up(o + size_t(c->n_det) * 8);
  L.readings = o; o = up(o + size_t(c->record_steps) * c->n_det * 8);
  L.resid = o; o = up(o + size_t(c->record_steps) * 8);
  L.partial = o; o = up(o + n * n * 2 * 8);
  L.phi_int = o; o = up(o + V * 8);
  L.gin = o; o = up(o + V * 8);
  L.ctl = o; o = up(o + sizeof(Ctl));
  L.total = o;
  return L;
}

int enqueue_op_n16(const StepArgs& a, const OpArgs& op, void* pr);
int enqueue_op_n32(const StepArgs& a, const OpArgs& op, void* pr);
int enqueue_op_n48(const StepArgs& a, const OpArgs& op, void* pr);
int enqueue_op_n64(const StepArgs& a, const OpArgs& op, void* pr);
int enqueue_op_n96(const StepArgs& a, const OpArgs& op, void* pr);
int enqueue_op_n128(const StepArgs& a, const OpArgs& op, void* pr);
int enqueue_op_n256(const StepArgs& a, const OpArgs& op, void* pr);
int prepare_n16(const StepArgs& a);
int prepare_n32(const StepArgs& a);
int prepare_n48(const StepArgs& a);
int prepare_n64(const StepArgs& a);
int prepare_n96(const StepArgs& a);
int prepare_n128(const StepArgs& a);
int prepare_n256(const StepArgs& a);

int launch_enqueue_op(int n, const StepArgs& a, const OpArgs& op, void* ev) {
  switch (n) {
    case 16: return enqueue_op_n16(a, op, ev);
    case 32: return enqueue_op_n32(a, op, ev);
    case 48: return enqueue_op_n48(a, op, ev);
    case 64: return enqueue_op_n64(a, op, ev);
    case 96: return enqueue_op_n96(a, op, ev);
    case 128: return enqueue_op_n128(a, op, ev);
    case 256: return enqueue_op_n256(a, op, ev);
    default: return int(hipErrorInvalidValue);
  }
}

int launch_prepare(int n, const StepArgs& a) {
  switch (n) {
    case 16: return prepare_n16(a);
    case 32: return prepare_n32(a);
    case 48: return prepare_n48(a);
    case 64: return prepare_n64(a);
    case 96: return prepare_n96(a);
    case 128: return prepare_n128(a);
    case 256: return prepare_n256(a);
    default: return int(hipErrorInvalidValue);
  }
}

}  // namespace rte

struct rte_handle {
  rte_config cfg;
  rte::Layout lay;
  rte::StepArgs args;
  int n, N, M, prec;
  int q_moments;
  double dt;
  bool has_q;
  hipStream_t stream;
  unsigned char* ws;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool graph_ready;
  bool use_graph;
  bool spec_valid;                  // spec holds the xy spectrum of u (fused steps' entry condition)
  const double* qw;                 // source time profile (device, caller-owned) or null
  long long qw_rows;
  int qw_cols;
  bool homogeneous;                 // constant maps, no boundary layer
  bool expo_taylor;                 // exact propagation by the per-point series only
  std::vector<double> rot_data;     // X blocks and B_z couplings of the rotation path
  bool batch_owned;                 // a slot of a batch: stepped by the batch, read-only here
  int device;                       // HIP device current at creation (the stream's device)
  double source_term;               // weighted source energy / (smallest loss)^2 (growth limit)
  uint64_t medium_hash;             // FNV-1a of the maps and source (snapshot compatibility)
  double sigl[rte::kMaxOrder + 1];  // per-degree loss (homogeneous media)
  template <typename P> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
};

namespace rte {

int to_code(hipError_t e) { return e == hipSuccess ? RTE_OK : RTE_EDEVICE; }

OpArgs step_op() {
  OpArgs op{};
  op.kind = OP_STEP;
  op.fused = 1;
  return op;
}

template <typename T>
void convert_upload(std::vector<T>& tmp, const double* src, size_t count) {
  tmp.resize(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = T(src[i]);
}

// State upload: the given leading moments converted to the working
// precision, the remaining moments cleared on the device.
template <typename T>
int upload_state_t(rte_handle* h, const double* psi, int moments) {
  const size_t V = size_t(h->n) * h->n * h->n;
  const size_t cnt = size_t(h->M) * V;
  const size_t given = psi ? size_t(moments) * V : 0;
  hipError_t e = hipSuccess;
  std::vector<T> tmp;
  if (given) {
    tmp.resize(given);
    for (size_t i = 0; i < given; ++i) tmp[i] = T(psi[i]);
    e = hipMemcpyAsync(h->at<T>(h->lay.u), tmp.data(), given * sizeof(T), hipMemcpyHostToDevice, h->stream);
  }
  if (e == hipSuccess && given < cnt)
    e = hipMemsetAsync(h->at<T>(h->lay.u) + given, 0, (cnt - given) * sizeof(T), h->stream);
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
  c.stop = h->batch_owned ? 3 : 0;   // a batch slot stays idle until the batch starts it
  c.qw = h->qw;
  c.qw_rows = h->qw_rows;
  c.qw_cols = h->qw_cols;
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

// FNV-1a over the bytes of the optical maps and the source moments: a
// snapshot restores only into a handle built from the same medium.
inline void fnv1a(uint64_t& h, const void* p, size_t bytes) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
}

uint64_t medium_hash_of(const rte_medium* med, size_t V, int q_moments) {
  uint64_t h = 1469598103934665603ull;
  fnv1a(h, med->mu_a, V * 8);
  fnv1a(h, med->mu_s, V * 8);
  fnv1a(h, med->g, V * 8);
  if (med->q) fnv1a(h, med->q, size_t(q_moments) * V * 8);
  return h;
}

// Weighted energy sum_a (2l+1) ||x_a||^2 of the leading `moments` moment
// fields of x (the squared norm of the orthonormal-basis coefficients, in
// which the streaming operator is skew and the loss non-negative, so the
// source-free solution never exceeds it).
double weighted_energy(const double* x, int moments, size_t V) {
  if (!x) return 0.0;
  double e = 0.0;
  for (int a = 0; a < moments; ++a) {
    const int l = isqrt_c(a);
    double s = 0.0;
    for (size_t i = 0; i < V; ++i) s += x[size_t(a) * V + i] * x[size_t(a) * V + i];
    e += double(2 * l + 1) * s;
  }
  return e;
}

// Runaway-growth threshold on ||phi||^2: the fluence is one component of
// the moment vector, so ||phi(t)||^2 stays below the initial weighted
// energy plus the steady response to the source (source energy over the
// smallest loss squared); the limit is that bound times 1e16.
double growth_limit_of(double state_energy, double source_term) {
  return 1e16 * (state_energy + source_term + 1e-300);
}

template <typename T>
int upload_tables_t(rte_handle* h, const rte_medium* med, const std::vector<double>& sig,
                    const std::vector<uint8_t>& inside) {
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
  std::vector<int> qflag(n, 0);
  if (h->has_q && !med->q) {
    // a batch slot keeps the source section of the common layout: cleared
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.q, 0, size_t(h->M) * V * sizeof(T), h->stream);
  } else if (h->has_q) {
    std::vector<double> qm(size_t(h->M) * V);
    for (int a = 0; a < h->M; ++a)
      for (size_t i = 0; i < V; ++i) {
        const double val = (inside[i] && a < h->q_moments) ? med->q[size_t(a) * V + i] : 0.0;
        qm[size_t(a) * V + i] = val;
        if (val != 0.0) qflag[i / (size_t(n) * n)] = 1;
      }
    convert_upload(tmp, qm.data(), qm.size());
    put(L.q, tmp.data(), tmp.size() * sizeof(T));
  }
  put(L.qflag, qflag.data(), qflag.size() * sizeof(int));
  {
    // g inside the real domain, 2 (> 1) in the layer: the adjoint gradient
    // of the loss with respect to mu_a, mu_s vanishes there (eq. 12)
    std::vector<double> gin(V);
    for (size_t i = 0; i < V; ++i) gin[i] = inside[i] ? med->g[i] : 2.0;
    put(L.gin, gin.data(), V * 8);
  }
  if (h->cfg.n_det > 0) put(L.det, h->cfg.det_index, size_t(h->cfg.n_det) * 8);
  if (h->N > kDenseOrder) {
    std::vector<int> code;
    std::vector<double> val;
    if (!coupling_table(h->N, code, val)) return RTE_EINVAL;
    put(L.ctab, code.data(), code.size() * sizeof(int));
    convert_upload(tmp, val.data(), val.size());
    put(L.cval, tmp.data(), tmp.size() * sizeof(T));
  }
  return to_code(e);
}

int enqueue_steps(rte_handle* h, int64_t k) {
  if (k <= 0) return RTE_OK;
  if (h->use_graph && !h->graph_ready) {
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = hipError_t(launch_enqueue_op(h->n, h->args, step_op(), nullptr));
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
  if (!h->spec_valid) {
    OpArgs f{};
    f.kind = OP_FWD;
    if (launch_enqueue_op(h->n, h->args, f, nullptr) != 0) return RTE_EDEVICE;
    h->spec_valid = true;
  }
  for (int64_t i = 0; i < k; ++i) {
    hipError_t e = h->graph_ready ? hipGraphLaunch(h->exec, h->stream)
                                  : hipError_t(launch_enqueue_op(h->n, h->args, step_op(), nullptr));
    if (e != hipSuccess) return RTE_EDEVICE;
  }
  return RTE_OK;
}

// ------------------------------------------------------------- adjoint ---

struct AdjLayout {
  size_t ckpt, seg, v1, v2, v3, lam, xa, xb, scratch, gmua, gmus, djdr, phi, partial, ctl, total;
  int64_t nckpt, every;
};

inline AdjLayout adj_layout(const rte_config* c, int64_t steps, int64_t every) {
  AdjLayout A{};
  const size_t n = c->n, M = size_t(c->order_N + 1) * (c->order_N + 1);
  const size_t s = c->precision == RTE_FP64 ? 8 : 4;
  const size_t V = n * n * n, F = M * V * s;
  A.every = every;
  A.nckpt = (steps + every - 1) / every;
  size_t o = 0;
  A.ckpt = o; o = up(o + size_t(A.nckpt) * F);
  A.seg = o; o = up(o + size_t(every) * F);
  A.v1 = o; o = up(o + F);
  A.v2 = o; o = up(o + F);
  A.v3 = o; o = up(o + F);
  A.lam = o; o = up(o + F);
  A.xa = o; o = up(o + F);
  A.xb = o; o = up(o + F);
  A.scratch = o; o = up(o + F);
  A.gmua = o; o = up(o + V * 8);
  A.gmus = o; o = up(o + V * 8);
  A.djdr = o; o = up(o + size_t(steps) * size_t(c->n_det) * 8);
  A.phi = o; o = up(o + V * 8);
  A.partial = o; o = up(o + n * n * 2 * 8);
  A.ctl = o; o = up(o + sizeof(Ctl));
  A.total = o;
  return A;
}

inline size_t state_bytes(const rte_handle* h) {
  return size_t(h->M) * h->n * h->n * h->n * (h->prec == RTE_FP64 ? 8 : 4);
}

}  // namespace rte

// ================================================================ C-ABI ==

extern "C" {

size_t rte_workspace_bytes(const rte_config* cfg) {
  if (!rte::config_ok(cfg)) return 0;
  return rte::layout_of(cfg, true).total;
}

}  // extern "C"

namespace rte {
// rte_create's body; batch_slot: a slot of a batch (the common layout with a
// source section, control block idle until the batch starts the slot).
int create_impl(const rte_config* cfg, const rte_medium* med, void* dev_ws, size_t ws_bytes,
                void* hip_stream, rte_handle** out, bool batch_slot) {
  if (!out) return RTE_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg) || !med || !med->mu_a || !med->mu_s || !med->g) return RTE_EINVAL;
  if (med->psi0_moments < 0 || med->q_moments < 0) return RTE_EINVAL;
  const int n = cfg->n, N = cfg->order_N, M = (N + 1) * (N + 1);
  const size_t V = size_t(n) * n * n;
  for (size_t i = 0; i < V; ++i) {
    if (!(med->mu_a[i] >= 0) || !(med->mu_s[i] >= 0) || !std::isfinite(med->mu_a[i]) ||
        !std::isfinite(med->mu_s[i]) || !(med->g[i] > -1.0 && med->g[i] < 1.0))
      return RTE_EINVAL;
  }
  for (int p = 0; p < cfg->n_det; ++p)
    if (cfg->det_index[p] < 0 || size_t(cfg->det_index[p]) >= V) return RTE_EINVAL;
  {
    // distinct detector voxels: the adjoint injects each reading's source
    // at its voxel, one thread per detector
    std::vector<int64_t> d(cfg->det_index, cfg->det_index + cfg->n_det);
    std::sort(d.begin(), d.end());
    if (std::adjacent_find(d.begin(), d.end()) != d.end()) return RTE_EINVAL;
  }
  const bool has_q = med->q != nullptr || batch_slot;
  const Layout L = layout_of(cfg, has_q);
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) != 0 || ws_bytes < L.total) return RTE_ENOMEM;

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
  h->q_moments = (med->q_moments > 0 && med->q_moments < M) ? med->q_moments : M;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = reinterpret_cast<unsigned char*>(dev_ws);
  h->lay = L;
  h->batch_owned = batch_slot;
  h->device = 0;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  {
    // set-up of the static scratch array on this device (once per device)
    hipError_t se = hipSuccess;
    (void)scratch_on(h->device, &se);
  }
  h->graph_ready = false;
  h->spec_valid = false;
  h->qw = nullptr;
  h->qw_rows = 0;
  h->qw_cols = 0;
  {
    const char* et = std::getenv("RTE_EXPO_SERIES");
    h->expo_taylor = et && et[0] == '1';
  }
  h->homogeneous = cfg->pml_width == 0;
  for (size_t i = 1; i < V && h->homogeneous; ++i)
    h->homogeneous = med->mu_a[i] == med->mu_a[0] && med->mu_s[i] == med->mu_s[0] && med->g[i] == med->g[0];
  for (int l = 0; l <= kMaxOrder; ++l) h->sigl[l] = l <= N ? sig[size_t(l) * V] : 0.0;
  const char* ng = std::getenv("RTE_NO_GRAPH");
  h->use_graph = (h->stream != nullptr) && !(ng && ng[0] == '1');
  StepArgs& A = h->args;
  A.prec = h->prec;
  A.scheme = cfg->scheme;
  A.N = N;
  A.M = M;
  A.stream = h->stream;
  A.u = h->ws + L.u;
  A.v = h->ws + L.v;
  A.spec = h->ws + L.spec;
  A.dspec = h->ws + L.dspec;
  A.wspec = N > kDenseOrder ? h->ws + L.wspec : nullptr;
  A.ctab = N > kDenseOrder ? h->at<int>(L.ctab) : nullptr;
  A.cval = N > kDenseOrder ? h->ws + L.cval : nullptr;
  A.tw = h->ws + L.tw;
  A.kv = h->ws + L.kv;
  A.sig = h->ws + L.sig;
  A.q = has_q ? h->ws + L.q : nullptr;
  A.nslot = 1;
  A.sstride = 0;
  A.qflag = h->at<int>(L.qflag);
  A.phi_int = h->at<double>(L.phi_int);
  A.partial = h->at<double>(L.partial);
  A.readings = h->at<double>(L.readings);
  A.resid = h->at<double>(L.resid);
  A.det = h->at<long long>(L.det);
  A.ndet = cfg->n_det;
  A.cap = cfg->record_steps;
  A.ctl = h->ws + L.ctl;
  A.c = cfg->c_mm_ps;
  A.dt = h->dt;
  int rc = to_code(hipError_t(launch_prepare(n, A)));
  if (!rc) rc = h->prec == RTE_FP64 ? upload_tables_t<double>(h, med, sig, inside)
                                    : upload_tables_t<float>(h, med, sig, inside);
  const int pm = (med->psi0_moments > 0 && med->psi0_moments < M) ? med->psi0_moments : M;
  if (!rc)
    rc = h->prec == RTE_FP64 ? upload_state_t<double>(h, med->psi0, pm) : upload_state_t<float>(h, med->psi0, pm);
  if (!rc) {
    double smin = 1e300;
    for (size_t i = 0; i < V; ++i) smin = std::min(smin, sig[i]);
    smin = std::max(smin, 1e-6);
    h->source_term = weighted_energy(med->q, med->q ? h->q_moments : 0, V) / (smin * smin);
    h->medium_hash = medium_hash_of(med, V, med->q ? h->q_moments : 0);
    // the configuration that fixes the meaning of a snapshot's bytes
    fnv1a(h->medium_hash, &n, sizeof n);
    fnv1a(h->medium_hash, &N, sizeof N);
    fnv1a(h->medium_hash, &cfg->precision, sizeof cfg->precision);
    fnv1a(h->medium_hash, &cfg->scheme, sizeof cfg->scheme);
    fnv1a(h->medium_hash, &cfg->pml_width, sizeof cfg->pml_width);
    fnv1a(h->medium_hash, &cfg->pml_mu0, sizeof cfg->pml_mu0);
    fnv1a(h->medium_hash, &cfg->pml_mu1, sizeof cfg->pml_mu1);
    fnv1a(h->medium_hash, &cfg->dx_mm, sizeof cfg->dx_mm);
    fnv1a(h->medium_hash, &cfg->c_mm_ps, sizeof cfg->c_mm_ps);
    fnv1a(h->medium_hash, &h->dt, sizeof h->dt);
    fnv1a(h->medium_hash, &cfg->record_steps, sizeof cfg->record_steps);
    fnv1a(h->medium_hash, &cfg->n_det, sizeof cfg->n_det);
    if (cfg->n_det > 0) fnv1a(h->medium_hash, cfg->det_index, size_t(cfg->n_det) * 8);
    rc = reset_run_state(h, growth_limit_of(weighted_energy(med->psi0, med->psi0 ? pm : 0, V), h->source_term));
  }
  h->cfg.det_index = nullptr;
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return RTE_OK;
}
}  // namespace rte

extern "C" {

int rte_create(const rte_config* cfg, const rte_medium* med, void* dev_ws, size_t ws_bytes,
               void* hip_stream, rte_handle** out) {
  return rte::create_impl(cfg, med, dev_ws, ws_bytes, hip_stream, out, false);
}

int rte_step(rte_handle* h, int64_t nsteps) {
  if (!h || nsteps < 0 || h->batch_owned) return RTE_EINVAL;
  return rte::enqueue_steps(h, nsteps);
}

int rte_run(rte_handle* h, int64_t max_steps, double steady_tol, int64_t* steps_taken) {
  using namespace rte;
  if (!h || max_steps < 0 || !(steady_tol > 0) || h->batch_owned) return RTE_EINVAL;
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
  if (!h || !in || h->batch_owned) return RTE_EINVAL;
  h->spec_valid = false;
  const size_t cnt = size_t(h->M) * h->n * h->n * h->n;
  if (len < cnt) return RTE_EINVAL;
  const int rc = h->prec == RTE_FP64 ? rte::upload_state_t<double>(h, in, h->M)
                                     : rte::upload_state_t<float>(h, in, h->M);
  if (rc) return rc;
  const size_t V = size_t(h->n) * h->n * h->n;
  return rte::reset_run_state(h, rte::growth_limit_of(rte::weighted_energy(in, h->M, V), h->source_term));
}

namespace {
// Snapshot layout (host bytes): header, then u in the working precision
// (bitwise), the FP64 integrated fluence [n^3], the whole record of
// readings [record_steps][n_det] and residuals [record_steps].
struct SnapHeader {
  char magic[8];
  uint64_t compat;        // hash of configuration, detectors, maps and source
  int64_t step;
  int32_t stop, pad;
  double growth_limit, last_resid, last_norm2;
};
constexpr char kSnapMagic[8] = {'R', 'T', 'E', 'S', 'N', 'A', 'P', '1'};

struct SnapSizes {
  size_t state, phi, readings, resid, total;
};
SnapSizes snap_sizes(const rte_handle* h) {
  SnapSizes z{};
  const size_t V = size_t(h->n) * h->n * h->n;
  z.state = rte::state_bytes(h);
  z.phi = V * 8;
  z.readings = size_t(h->cfg.record_steps) * size_t(h->cfg.n_det) * 8;
  z.resid = size_t(h->cfg.record_steps) * 8;
  z.total = sizeof(SnapHeader) + z.state + z.phi + z.readings + z.resid;
  return z;
}
}  // namespace

size_t rte_snapshot_bytes(const rte_handle* h) { return h ? snap_sizes(h).total : 0; }

int rte_snapshot(rte_handle* h, void* out, size_t len) {
  using namespace rte;
  if (!h || !out) return RTE_EINVAL;
  const SnapSizes z = snap_sizes(h);
  if (len < z.total) return RTE_EINVAL;
  Ctl c;
  int rc = read_ctl(h, &c);
  if (rc) return rc;
  SnapHeader hd{};
  std::memcpy(hd.magic, kSnapMagic, 8);
  hd.compat = h->medium_hash;
  hd.step = c.step;
  hd.stop = c.stop == 1 ? 0 : c.stop;   // a converged run's stop flag ends with its rte_run
  hd.growth_limit = c.growth_limit;
  hd.last_resid = c.last_resid;
  hd.last_norm2 = c.last_norm2;
  unsigned char* o = static_cast<unsigned char*>(out);
  std::memcpy(o, &hd, sizeof hd);
  o += sizeof hd;
  hipError_t e = hipMemcpyAsync(o, h->ws + h->lay.u, z.state, hipMemcpyDeviceToHost, h->stream);
  o += z.state;
  if (e == hipSuccess) e = hipMemcpyAsync(o, h->ws + h->lay.phi_int, z.phi, hipMemcpyDeviceToHost, h->stream);
  o += z.phi;
  if (e == hipSuccess && z.readings)
    e = hipMemcpyAsync(o, h->ws + h->lay.readings, z.readings, hipMemcpyDeviceToHost, h->stream);
  o += z.readings;
  if (e == hipSuccess && z.resid)
    e = hipMemcpyAsync(o, h->ws + h->lay.resid, z.resid, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return to_code(e);
}

int rte_restore(rte_handle* h, const void* in, size_t len) {
  using namespace rte;
  if (!h || !in || h->batch_owned) return RTE_EINVAL;
  const SnapSizes z = snap_sizes(h);
  if (len < z.total) return RTE_EINVAL;
  SnapHeader hd;
  const unsigned char* p = static_cast<const unsigned char*>(in);
  std::memcpy(&hd, p, sizeof hd);
  if (std::memcmp(hd.magic, kSnapMagic, 8) != 0 || hd.compat != h->medium_hash || hd.step < 0 ||
      hd.stop < 0 || hd.stop > 2)
    return RTE_EINVAL;
  p += sizeof hd;
  h->spec_valid = false;
  hipError_t e = hipMemcpyAsync(h->ws + h->lay.u, p, z.state, hipMemcpyHostToDevice, h->stream);
  p += z.state;
  if (e == hipSuccess) e = hipMemcpyAsync(h->ws + h->lay.phi_int, p, z.phi, hipMemcpyHostToDevice, h->stream);
  p += z.phi;
  if (e == hipSuccess && z.readings)
    e = hipMemcpyAsync(h->ws + h->lay.readings, p, z.readings, hipMemcpyHostToDevice, h->stream);
  p += z.readings;
  if (e == hipSuccess && z.resid)
    e = hipMemcpyAsync(h->ws + h->lay.resid, p, z.resid, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return RTE_EDEVICE;
  Ctl c{};
  c.step = hd.step;
  c.stop = hd.stop;
  c.growth_limit = hd.growth_limit;
  c.last_resid = hd.last_resid;
  c.last_norm2 = hd.last_norm2;
  c.qw = h->qw;
  c.qw_rows = h->qw_rows;
  c.qw_cols = h->qw_cols;
  return write_ctl(h, &c);
}

namespace {
// Profile s(t): linear between samples[i] at t = i * delta, last value after.
double profile_at(const double* sm, int64_t ns, double delta, double t) {
  if (t <= 0.0 || ns == 1) return sm[0];
  const double x = t / delta;
  const int64_t i = int64_t(std::floor(x));
  if (i >= ns - 1) return sm[ns - 1];
  const double f = x - double(i);
  return sm[i] + f * (sm[i + 1] - sm[i]);
}

// int_0^h (h - tau)^j s(t0 + tau) dtau, j = 0..3: the step is split at the
// sample knots, where s is linear, and each piece integrated by 3-point
// Gauss-Legendre (exact for the polynomial degree <= 4 of the integrand).
void profile_moments(const double* sm, int64_t ns, double delta, double t0, double h, double out[4]) {
  static const double gx[3] = {-0.7745966692414834, 0.0, 0.7745966692414834};
  static const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  for (int j = 0; j < 4; ++j) out[j] = 0.0;
  double a = 0.0;
  while (a < h) {
    // next knot after t0 + a (or the end of the step); a knot within
    // rounding of a counts as passed
    double k = std::floor((t0 + a) / delta) + 1.0;
    double tk = k * delta - t0;
    while (tk <= a + 1e-12 * h) {
      k += 1.0;
      tk = k * delta - t0;
    }
    const double b = tk < h ? tk : h;
    const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    for (int g = 0; g < 3; ++g) {
      const double tau = mid + half * gx[g];
      const double sv = profile_at(sm, ns, delta, t0 + tau) * gw[g] * half;
      double p = 1.0;
      for (int j = 0; j < 4; ++j) {
        out[j] += p * sv;
        p *= (h - tau);
      }
    }
    a = b;
  }
}
}  // namespace

int rte_set_source_profile(rte_handle* h, const double* samples, int64_t nsamples, double delta_ps,
                           int64_t rows, void* dev_table, size_t table_bytes) {
  using namespace rte;
  if (!h || h->batch_owned) return RTE_EINVAL;
  const int cols = h->cfg.scheme == RTE_EULER ? 1 : 4;
  if (samples == nullptr || rows == 0) {
    h->qw = nullptr;
    h->qw_rows = 0;
    h->qw_cols = 0;
  } else {
    if (nsamples < 1 || rows < 0 || !(delta_ps > 0) || !std::isfinite(delta_ps)) return RTE_EINVAL;
    for (int64_t i = 0; i < nsamples; ++i)
      if (!std::isfinite(samples[i])) return RTE_EINVAL;
    const size_t need = size_t(rows) * cols * 8;
    if (!dev_table || (reinterpret_cast<uintptr_t>(dev_table) % 8) != 0 || table_bytes < need) return RTE_ENOMEM;
    std::vector<double> w(size_t(rows) * cols);
    const double dt = h->dt;
    for (int64_t r = 0; r < rows; ++r) {
      const double t0 = double(r) * dt;
      if (cols == 1) {
        w[size_t(r)] = profile_at(samples, nsamples, delta_ps, t0);
        continue;
      }
      double m[4];
      profile_moments(samples, nsamples, delta_ps, t0, dt, m);
      // stage k of the nested step (coefficients 1/4, 1/3, 1/2, 1) carries
      // (j + 1) / h^(j + 1) int (h - tau)^j s, j = 3 - k
      for (int k = 0; k < 4; ++k) {
        const int j = 3 - k;
        w[size_t(r) * 4 + k] = double(j + 1) * m[j] / std::pow(dt, j + 1);
      }
    }
    hipError_t e = hipMemcpyAsync(dev_table, w.data(), need, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return RTE_EDEVICE;
    h->qw = static_cast<const double*>(dev_table);
    h->qw_rows = rows;
    h->qw_cols = cols;
  }
  Ctl c;
  int rc = read_ctl(h, &c);
  if (rc) return rc;
  c.qw = h->qw;
  c.qw_rows = h->qw_rows;
  c.qw_cols = h->qw_cols;
  return write_ctl(h, &c);
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

size_t rte_adjoint_workspace_bytes(const rte_config* cfg, int64_t steps, int64_t every) {
  if (!rte::config_ok(cfg) || steps <= 0 || every <= 0) return 0;
  return rte::adj_layout(cfg, steps, every).total;
}

int rte_forward_checkpointed(rte_handle* h, int64_t steps, int64_t every, void* adj_ws, size_t adj_bytes) {
  using namespace rte;
  if (!h || steps <= 0 || every <= 0 || h->batch_owned) return RTE_EINVAL;
  const AdjLayout A = adj_layout(&h->cfg, steps, every);
  if (!adj_ws || (reinterpret_cast<uintptr_t>(adj_ws) % kAlign) != 0 || adj_bytes < A.total) return RTE_ENOMEM;
  unsigned char* w = static_cast<unsigned char*>(adj_ws);
  const size_t F = state_bytes(h);
  for (int64_t i = 0; i < steps; ++i) {
    if (i % every == 0) {
      if (hipMemcpyAsync(w + A.ckpt + size_t(i / every) * F, h->ws + h->lay.u, F, hipMemcpyDeviceToDevice,
                         h->stream) != hipSuccess)
        return RTE_EDEVICE;
    }
    const int rc = enqueue_steps(h, 1);
    if (rc) return rc;
  }
  Ctl c;
  const int rc = read_ctl(h, &c);
  if (rc) return rc;
  return c.stop == 2 ? RTE_EUNSTABLE : RTE_OK;
}

}  // extern "C"

namespace rte {
namespace {
// The reverse sweep of rte_adjoint; dev: dj_dr and the gradients are device
// buffers (copied device to device) instead of host arrays.
int adjoint_run(rte_handle* h, int64_t steps, int64_t every, void* adj_ws, size_t adj_bytes,
                const double* dj_dr, double* grad_mu_a, double* grad_mu_s, bool dev) {
  if (!h || steps <= 0 || every <= 0 || !grad_mu_a || !grad_mu_s || h->batch_owned) return RTE_EINVAL;
  if (h->cfg.n_det > 0 && !dj_dr) return RTE_EINVAL;
  h->spec_valid = false;   // the recomputation and transposed stages reuse the spectrum buffers
  const AdjLayout A = adj_layout(&h->cfg, steps, every);
  if (!adj_ws || (reinterpret_cast<uintptr_t>(adj_ws) % kAlign) != 0 || adj_bytes < A.total) return RTE_ENOMEM;
  unsigned char* w = static_cast<unsigned char*>(adj_ws);
  const size_t F = state_bytes(h);
  const size_t V = size_t(h->n) * h->n * h->n;
  const int nd = h->cfg.n_det;
  hipStream_t st = h->stream;
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  if (nd > 0)
    ok(hipMemcpyAsync(w + A.djdr, dj_dr, size_t(steps) * nd * 8,
                      dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  ok(hipMemsetAsync(w + A.gmua, 0, V * 8, st));
  ok(hipMemsetAsync(w + A.gmus, 0, V * 8, st));
  ok(hipMemsetAsync(w + A.lam, 0, F, st));
  Ctl hc{};
  {
    const int rc = read_ctl(h, &hc);
    if (rc) return rc;
  }
  // the checkpointed run ended at the handle's current step
  const long long s0 = hc.step - steps;
  Ctl c0{};
  c0.growth_limit = 1e300;
  c0.qw = h->qw;
  c0.qw_rows = h->qw_rows;
  c0.qw_cols = h->qw_cols;
  ok(hipMemcpyAsync(w + A.ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice, st));
  ok(hipStreamSynchronize(st));
  if (e != hipSuccess) return RTE_EDEVICE;

  // recompute arguments: private bookkeeping buffers, no readings
  StepArgs R = h->args;
  R.readings = nullptr;
  R.resid = nullptr;
  R.cap = 0;
  R.ndet = 0;
  R.phi_int = reinterpret_cast<double*>(w + A.phi);
  R.partial = reinterpret_cast<double*>(w + A.partial);
  R.ctl = w + A.ctl;
  R.v = w + A.scratch;
  const StepArgs& H = h->args;
  auto op = [&](const StepArgs& sa, const OpArgs& o) {
    if (e == hipSuccess) e = hipError_t(launch_enqueue_op(h->n, sa, o, nullptr));
  };
  auto inject = [&](int64_t reading) {
    if (nd == 0) return;
    OpArgs o{};
    o.kind = OP_ADJ_INJECT;
    o.u = w + A.lam;
    o.djdr = reinterpret_cast<const double*>(w + A.djdr) + size_t(reading) * nd;
    op(H, o);
  };
  auto grad = [&](const void* x, const void* y, double coef) {
    OpArgs o{};
    o.kind = OP_ADJ_GRAD;
    o.x = x;
    o.y = const_cast<void*>(y);
    o.coef = coef;
    o.gin = h->at<double>(h->lay.gin);
    o.gmua = reinterpret_cast<double*>(w + A.gmua);
    o.gmus = reinterpret_cast<double*>(w + A.gmus);
    op(R, o);
  };
  auto adj_stage = [&](const void* x, void* y, double coef) {
    OpArgs o{};
    o.kind = OP_ADJ_STAGE;
    o.x = x;
    o.y = y;
    o.u = w + A.lam;
    o.coef = coef;
    op(R, o);
  };
  auto fwd_stage = [&](int s, int64_t nn, const void* un, const void* x, void* y) {
    OpArgs o{};
    o.kind = OP_STAGE;
    o.stage = s;
    o.step1 = s0 + nn + 1;
    o.u = const_cast<void*>(un);
    o.x = x;
    o.y = y;
    op(R, o);
  };

  // readings r_s (s = 0..steps-1) are psi_00 of u_{s+1}
  inject(steps - 1);
  for (int64_t j = A.nckpt - 1; j >= 0 && e == hipSuccess; --j) {
    const int64_t n0 = j * every, n1 = std::min(steps, n0 + every);
    unsigned char* seg = w + A.seg;
    ok(hipMemcpyAsync(seg, w + A.ckpt + size_t(j) * F, F, hipMemcpyDeviceToDevice, st));
    for (int64_t nn = n0; nn + 1 < n1; ++nn) {
      unsigned char* next = seg + size_t(nn - n0 + 1) * F;
      ok(hipMemcpyAsync(next, seg + size_t(nn - n0) * F, F, hipMemcpyDeviceToDevice, st));
      StepArgs S = R;
      S.u = next;
      OpArgs o{};
      o.kind = OP_STEP;
      o.step1 = s0 + nn + 1;
      op(S, o);
    }
    for (int64_t nn = n1 - 1; nn >= n0 && e == hipSuccess; --nn) {
      const void* un = seg + size_t(nn - n0) * F;
      if (h->args.scheme == RTE_EULER) {
        // u' = u + h F(u): lam <- lam + h F^T lam, gradient term (lam, u)
        grad(w + A.lam, un, 1.0);
        adj_stage(w + A.lam, w + A.xa, 1.0);
        if (nn >= 1) inject(nn - 1);
        continue;
      }
      fwd_stage(0, nn, un, un, w + A.v1);
      fwd_stage(1, nn, un, w + A.v1, w + A.v2);
      fwd_stage(2, nn, un, w + A.v2, w + A.v3);
      // transposed nested stages (coefficients 1, 1/2, 1/3, 1/4), each
      // preceded by the gradient term of its forward counterpart
      grad(w + A.lam, w + A.v3, 1.0);
      adj_stage(w + A.lam, w + A.xa, 1.0);
      grad(w + A.xa, w + A.v2, 0.5);
      adj_stage(w + A.xa, w + A.xb, 0.5);
      grad(w + A.xb, w + A.v1, 1.0 / 3.0);
      adj_stage(w + A.xb, w + A.xa, 1.0 / 3.0);
      grad(w + A.xa, un, 0.25);
      adj_stage(w + A.xa, w + A.xb, 0.25);
      if (nn >= 1) inject(nn - 1);
    }
  }
  if (e != hipSuccess) return RTE_EDEVICE;
  const hipMemcpyKind back = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  ok(hipMemcpyAsync(grad_mu_a, w + A.gmua, V * 8, back, st));
  ok(hipMemcpyAsync(grad_mu_s, w + A.gmus, V * 8, back, st));
  ok(hipStreamSynchronize(st));
  return to_code(e);
}

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7) == 0; }
}  // namespace
}  // namespace rte

extern "C" {

int rte_adjoint(rte_handle* h, int64_t steps, int64_t every, void* adj_ws, size_t adj_bytes,
                const double* dj_dr, double* grad_mu_a, double* grad_mu_s) {
  return rte::adjoint_run(h, steps, every, adj_ws, adj_bytes, dj_dr, grad_mu_a, grad_mu_s, false);
}

int rte_adjoint_device(rte_handle* h, int64_t steps, int64_t every, void* adj_ws, size_t adj_bytes,
                       const double* dj_dr, double* grad_mu_a, double* grad_mu_s) {
  using rte::aligned8;
  if (!aligned8(dj_dr) || !aligned8(grad_mu_a) || !aligned8(grad_mu_s)) return RTE_EINVAL;
  return rte::adjoint_run(h, steps, every, adj_ws, adj_bytes, dj_dr, grad_mu_a, grad_mu_s, true);
}

int rte_set_medium_device(rte_handle* h, const double* mu_a, const double* mu_s) {
  using namespace rte;
  if (!h || !mu_a || !mu_s || h->batch_owned || !aligned8(mu_a) || !aligned8(mu_s)) return RTE_EINVAL;
  OpArgs o{};
  o.kind = OP_SET_LOSS;
  o.x = mu_a;
  o.djdr = mu_s;
  o.gin = h->at<double>(h->lay.gin);
  if (launch_enqueue_op(h->n, h->args, o, nullptr) != 0) return RTE_EDEVICE;
  // constant maps are no longer known on the host (no exact propagation),
  // and snapshots taken under the previous medium no longer fit
  h->homogeneous = false;
  const uint64_t salt = 0x6d656469756d2121ULL;
  fnv1a(h->medium_hash, &salt, sizeof salt);
  return to_code(hipStreamSynchronize(h->stream));
}

int rte_set_state_device(rte_handle* h, const double* psi, int32_t moments) {
  using namespace rte;
  if (!h || h->batch_owned || moments < 0 || moments > h->M || (moments > 0 && !psi) || !aligned8(psi))
    return RTE_EINVAL;
  h->spec_valid = false;
  int rc = reset_run_state(h, 1e300);   // threshold replaced on the device below
  if (rc) return rc;
  OpArgs o{};
  o.kind = OP_SET_STATE;
  o.x = psi;
  o.count = moments;
  if (launch_enqueue_op(h->n, h->args, o, nullptr) != 0) return RTE_EDEVICE;
  OpArgs g{};
  g.kind = OP_GROWTH;
  g.scale = h->source_term;
  if (launch_enqueue_op(h->n, h->args, g, nullptr) != 0) return RTE_EDEVICE;
  return to_code(hipStreamSynchronize(h->stream));
}

int rte_readings_device(rte_handle* h, double* out, size_t len, int64_t* rows) {
  if (!h || (!out && len) || !rte::aligned8(out)) return RTE_EINVAL;
  rte::Ctl c;
  int rc = rte::read_ctl(h, &c);
  if (rc) return rc;
  int64_t r = std::min<int64_t>(c.step, h->cfg.record_steps);
  if (h->cfg.n_det == 0) r = 0;
  else r = std::min<int64_t>(r, int64_t(len / size_t(h->cfg.n_det)));
  if (rows) *rows = r;
  if (r == 0) return RTE_OK;
  hipError_t e = hipMemcpyAsync(out, h->ws + h->lay.readings, size_t(r) * h->cfg.n_det * 8,
                                hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return rte::to_code(e);
}

size_t rte_krylov_workspace_bytes(const rte_config* cfg, int32_t restart) {
  if (!rte::config_ok(cfg) || restart < 1 || restart + 1 > rte::kMaxBasisVectors) return 0;
  const size_t n = cfg->n, M = size_t(cfg->order_N + 1) * (cfg->order_N + 1);
  const size_t F = M * n * n * n * (cfg->precision == RTE_FP64 ? 8 : 4);
  size_t o = rte::up(size_t(restart + 3) * F);            // basis, right-hand side, stage scratch
  o = rte::up(o + size_t(rte::kDotPartials) * 8);         // dot partial sums
  o = rte::up(o + 2 * size_t(rte::kMaxBasisVectors) * 8); // device coefficients
  o = rte::up(o + sizeof(rte::GmDev));                     // device cycle state
  return o;
}

}  // extern "C"

namespace rte {
namespace {

// Restarted GMRES on the handle's state with the Krylov workspace kws (the
// caller's, or the library's static scratch array). Every Arnoldi step runs
// on the device without a host round trip: the Gram-Schmidt coefficients,
// the norm, the Givens update of the Hessenberg column and the convergence
// test (GmDev, k_gm_update) stay in device memory, and once a cycle has
// converged its remaining queued steps return at once (stop flag). The host
// synchronises twice per restart cycle: for the residual norm that decides
// whether to start a cycle, and to read the cycle's rotated Hessenberg
// system, which it solves (at most 31 unknowns) before the solution update.
// No heap allocation: the host arrays have the fixed maximum size.
int gmres_run(rte_handle* h, int32_t restart, int64_t max_iters, double tol, int32_t steps_per_apply, void* kws,
              size_t kbytes, int64_t* iters, double* rel_residual) {
  if (!h || restart < 1 || restart + 1 > kMaxBasisVectors || max_iters < 1 || !(tol > 0) || steps_per_apply < 0 ||
      h->batch_owned)
    return RTE_EINVAL;
  if (h->qw) return RTE_EINVAL;   // a steady state needs a constant source
  const size_t need = rte_krylov_workspace_bytes(&h->cfg, restart);
  if (!kws || (reinterpret_cast<uintptr_t>(kws) % kAlign) != 0 || kbytes < need) return RTE_ENOMEM;
  h->spec_valid = false;          // the operator applications reuse the spectrum buffers
  {
    // kernels skip their work once a run has stopped: clear the stop flag
    // (and the run bookkeeping, which a steady solve does not produce)
    Ctl c;
    int rc = read_ctl(h, &c);
    if (rc == RTE_OK) rc = reset_run_state(h, c.growth_limit);
    if (rc) return rc;
  }
  const int m = restart;
  const int K = steps_per_apply;
  const size_t F = state_bytes(h);
  unsigned char* w = static_cast<unsigned char*>(kws);
  unsigned char* basis = w;
  unsigned char* bvec = w + size_t(m + 1) * F;     // right-hand side of the propagator system
  unsigned char* tmp = w + size_t(m + 2) * F;      // stage values of the time steps
  double* partial = reinterpret_cast<double*>(w + up(size_t(m + 3) * F));
  double* dcoef = reinterpret_cast<double*>(w + up(up(size_t(m + 3) * F) + size_t(kDotPartials) * 8));
  double* dout = dcoef + kMaxBasisVectors;
  GmDev* gm = reinterpret_cast<GmDev*>(w + up(up(up(size_t(m + 3) * F) + size_t(kDotPartials) * 8) +
                                              2 * size_t(kMaxBasisVectors) * 8));
  int* dstop = &static_cast<Ctl*>(h->args.ctl)->stop;
  hipStream_t st = h->stream;
  hipError_t e = hipSuccess;
  StepArgs nosrc = h->args;
  nosrc.q = nullptr;
  auto op = [&](const StepArgs& args, OpArgs o) {
    if (e == hipSuccess) e = hipError_t(launch_enqueue_op(h->n, args, o, nullptr));
  };
  auto vec = [&](int i) { return static_cast<void*>(basis + size_t(i) * F); };
  auto steps_on = [&](const StepArgs& args, void* x) {   // K time steps of x in place
    for (int k = 0; k < K; ++k) {
      OpArgs o{};
      o.kind = OP_PSTEP;
      o.u = x;
      o.y = tmp;
      op(args, o);
    }
  };
  auto rhs_minus = [&](const void* b, void* y) {   // y = b - y
    OpArgs o{};
    o.kind = OP_RHS_MINUS;
    o.x = b;
    o.y = y;
    op(h->args, o);
  };
  // y = A x with A = S + Sigma, or y = x - P^K x with P one source-free time step
  auto apply = [&](const void* x, void* y) {
    if (K == 0) {
      OpArgs o{};
      o.kind = OP_APPLY;
      o.x = x;
      o.y = y;
      op(h->args, o);
    } else {
      if (e == hipSuccess) e = hipMemcpyAsync(y, x, F, hipMemcpyDeviceToDevice, st);
      steps_on(nosrc, y);
      rhs_minus(x, y);
    }
  };
  // out[0..count) (device) = <basis_0..count-1, y>_W
  auto wdots = [&](const void* base, int count, const void* y, double* out) {
    OpArgs o{};
    o.kind = OP_WDOTS;
    o.x = base;
    o.y = const_cast<void*>(y);
    o.count = count;
    o.gmua = partial;
    o.gmus = out;
    op(h->args, o);
  };
  // <x, x>_W on the host (synchronises)
  auto norm2 = [&](const void* x) {
    double v = 0.0;
    wdots(x, 1, x, dout);
    if (e == hipSuccess) e = hipMemcpyAsync(&v, dout, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return v;
  };
  // y = sgn * y + scale * sum_i c[i] basis_i, coefficients c on the device
  auto combine = [&](void* y, double sgn, int count, const double* c, double scale) {
    OpArgs o{};
    o.kind = OP_COMBINE;
    o.x = basis;
    o.y = y;
    o.coef = sgn;
    o.count = count;
    o.djdr = c;
    o.scale = scale;
    op(h->args, o);
  };
  auto scale_by = [&](void* y, const double* s) {   // y /= s[0] (device)
    OpArgs o{};
    o.kind = OP_SCALE;
    o.x = y;
    o.y = y;
    o.djdr = s;
    op(h->args, o);
  };
  const void* qv = h->has_q ? static_cast<const void*>(h->ws + h->lay.q) : nullptr;
  // right-hand side: q, or the K source-driven steps from zero
  const void* b = qv;
  if (K > 0) {
    if (e == hipSuccess) e = hipMemsetAsync(bvec, 0, F, st);
    if (h->has_q) steps_on(h->args, bvec);
    b = bvec;
  }
  auto residual_into = [&](void* r) {   // r = b - B u
    apply(h->ws + h->lay.u, r);
    rhs_minus(b, r);
  };
  const double bnorm = b ? std::sqrt(norm2(b)) : 0.0;
  const double ref = bnorm > 0 ? bnorm : 1.0;
  int64_t it = 0;
  double rel = 1.0;
  GmDev gh;                        // host copy of the cycle state
  double y[kMaxBasisVectors];
  while (e == hipSuccess) {
    residual_into(vec(0));
    const double beta = std::sqrt(norm2(vec(0)));
    rel = beta / ref;
    if (e != hipSuccess || rel <= tol || it >= max_iters || beta == 0.0) break;
    // cycle state: g = beta e_0; v_0 = r / beta
    std::memset(&gh, 0, sizeof gh);
    gh.g[0] = beta;
    gh.ref = ref;
    gh.tol = tol;
    gh.m = m;
    if (e == hipSuccess) e = hipMemcpyAsync(gm, &gh, sizeof gh, hipMemcpyHostToDevice, st);
    scale_by(vec(0), &gm->g[0]);
    const int jmax = int(std::min<int64_t>(m, max_iters - it));
    for (int j = 0; j < jmax; ++j) {
      apply(vec(j), vec(j + 1));
      // classical Gram-Schmidt, applied twice, against v_0..v_j
      wdots(basis, j + 1, vec(j + 1), gm->hv);
      combine(vec(j + 1), 1.0, j + 1, gm->hv, -1.0);
      wdots(basis, j + 1, vec(j + 1), gm->h2);
      combine(vec(j + 1), 1.0, j + 1, gm->h2, -1.0);
      wdots(vec(j + 1), 1, vec(j + 1), &gm->hn2);
      OpArgs o{};
      o.kind = OP_GM_UPDATE;
      o.u = gm;
      o.count = j;
      op(h->args, o);
      scale_by(vec(j + 1), &gm->hn);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&gh, gm, sizeof gh, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) break;
    const int j = gh.jdone;
    it += j;
    // a converged cycle left the stop flag set: clear it for the update
    // and the next cycle
    e = hipMemsetAsync(dstop, 0, sizeof(int), st);
    // solve the j x j triangular system R y = g and update u += sum y_i v_i
    for (int i = j - 1; i >= 0; --i) {
      double t = gh.g[i];
      for (int k = i + 1; k < j; ++k) t -= gh.R[i * m + k] * y[k];
      y[i] = t / gh.R[i * m + i];
    }
    if (j > 0) {
      if (e == hipSuccess) e = hipMemcpyAsync(dcoef, y, size_t(j) * 8, hipMemcpyHostToDevice, st);
      combine(h->ws + h->lay.u, 1.0, j, dcoef, 1.0);
    }
  }
  if (K > 0 && e == hipSuccess) {
    // report the residual of the steady-state equation A u = q itself
    OpArgs o{};
    o.kind = OP_APPLY;
    o.x = h->ws + h->lay.u;
    o.y = vec(0);
    op(h->args, o);
    rhs_minus(qv, vec(0));
    const double rn = norm2(vec(0));
    const double qn = qv ? norm2(qv) : 0.0;
    rel = std::sqrt(rn) / (qn > 0 ? std::sqrt(qn) : 1.0);
  }
  if (iters) *iters = it;
  if (rel_residual) *rel_residual = rel;
  if (e != hipSuccess) return RTE_EDEVICE;
  return std::isfinite(rel) ? RTE_OK : RTE_EUNSTABLE;
}

}  // namespace
}  // namespace rte

extern "C" {

size_t rte_static_scratch_bytes(void) { return rte::kScratchBytes; }

int rte_steady_gmres(rte_handle* h, int32_t restart, int64_t max_iters, double tol, int32_t steps_per_apply,
                     void* kws, size_t kbytes, int64_t* iters, double* rel_residual) {
  return rte::gmres_run(h, restart, max_iters, tol, steps_per_apply, kws, kbytes, iters, rel_residual);
}

int rte_steady_gmres_static(rte_handle* h, int32_t restart, int64_t max_iters, double tol,
                            int32_t steps_per_apply, int64_t* iters, double* rel_residual) {
  if (!h) return RTE_EINVAL;
  const size_t need = rte_krylov_workspace_bytes(&h->cfg, restart);
  if (need == 0) return RTE_EINVAL;
  if (need > rte::kScratchBytes) return RTE_ENOMEM;   // beyond the static array
  hipError_t err = hipSuccess;
  void* ws = rte::scratch_on(h->device, &err);
  if (!ws) return RTE_EDEVICE;
  return rte::gmres_run(h, restart, max_iters, tol, steps_per_apply, ws, rte::kScratchBytes, iters, rel_residual);
}

namespace {
// Largest per-substep norm theta for which the Taylor remainder bound
// theta^(m+1) / (m+1)! * exp(theta) stays below eps (bisection on its log).
double taylor_theta(int m, double eps) {
  double lo = 0.0, hi = 64.0;
  for (int it = 0; it < 200; ++it) {
    const double t = 0.5 * (lo + hi);
    const double lb = (m + 1) * std::log(t) - std::lgamma(double(m + 2)) + t;
    if (lb <= std::log(eps)) lo = t;
    else hi = t;
  }
  return lo;
}
}  // namespace

namespace {
int expo_run(rte_handle* h, double t_ps, rte::ProfRec* pr) {
  using namespace rte;
  if (!h || !std::isfinite(t_ps) || t_ps < 0 || h->batch_owned) return RTE_EINVAL;
  if (!h->homogeneous || h->N > kDenseOrder || h->qw) return RTE_EINVAL;
  if (t_ps == 0) return RTE_OK;
  h->spec_valid = false;
  const bool f64 = h->prec == RTE_FP64;
  const double eps = f64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
  const double theta = taylor_theta(f64 ? kTaylorMaxF64 : kTaylorMaxF32, eps);
  double smax = 0.0;
  for (int l = 0; l <= h->N; ++l) smax = std::max(smax, h->sigl[l]);
  const double kmax = std::sqrt(3.0) * M_PI / h->cfg.dx_mm;
  const double nu = h->cfg.c_mm_ps * t_ps * (kmax + smax);
  if (nu / theta > 1e6) return RTE_EINVAL;   // split into shorter advances
  Ctl c;
  int rc = read_ctl(h, &c);
  if (rc) return rc;
  if (c.stop == 2) return RTE_EUNSTABLE;
  if (c.stop) {
    c.stop = 0;
    rc = write_ctl(h, &c);
    if (rc) return rc;
  }
  OpArgs o{};
  o.kind = OP_EXPO;
  o.coef = t_ps;
  o.scale = theta;
  o.eps = eps;
  o.kunit = 2.0 * M_PI / (double(h->n) * h->cfg.dx_mm);
  for (int l = 0; l <= kMaxOrder; ++l) o.sigl[l] = h->sigl[l];
  hipError_t e = hipSuccess;
  if (!h->expo_taylor) {
    // rotation path: X blocks, B_z couplings and the block-exponential table
    // go to the stage buffer v if they fit (else the per-point series)
    const int N = h->N, M = h->M, n = h->n;
    const size_t s = f64 ? 8 : 4;
    size_t xs = 0;
    for (int l = 0; l <= N; ++l) xs += size_t(2 * l + 1) * (2 * l + 1);
    size_t toff = xs + 2 * size_t(M);
    toff += toff & 1;
    size_t row = 0;   // one pair of blocks per m >= 0 (m and -m share them)
    for (int m = 0; m <= N; ++m) {
      const size_t d = size_t(N + 1 - m);
      row += 2 * d * d;
    }
    const size_t nf2 = size_t(n / 2 - 1) * (n / 2 - 1) * 3 + 1;
    const size_t need = (toff + nf2 * row * 2) * s;
    const size_t have = size_t(M) * n * n * n * s;
    if (need <= have && h->rot_data.empty()) {
      // X blocks and B_z couplings, built (and self-checked) once per handle
      std::vector<double> X;
      std::vector<double> b[3];
      if (rotation_x90(N, X) && coupling_dense(N, b[0], b[1], b[2])) {
        std::vector<double>& data = h->rot_data;
        data = X;
        data.resize(toff, 0.0);
        for (int l = 0; l <= N; ++l)
          for (int m = -l; m <= l; ++m) {
            const int a = l * l + l + m;
            if (l >= 1 && std::abs(m) <= l - 1)
              data[xs + 2 * a] = b[2][size_t(a) * M + (l - 1) * (l - 1) + (l - 1) + m];
            if (l + 1 <= N) data[xs + 2 * a + 1] = b[2][size_t(a) * M + (l + 1) * (l + 1) + (l + 1) + m];
          }
      }
    }
    if (need <= have && !h->rot_data.empty()) {
      const std::vector<double>& data = h->rot_data;
      if (f64) {
        e = hipMemcpyAsync(h->ws + h->lay.v, data.data(), data.size() * 8, hipMemcpyHostToDevice, h->stream);
      } else {
        std::vector<float> df(data.begin(), data.end());
        e = hipMemcpyAsync(h->ws + h->lay.v, df.data(), df.size() * 4, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);   // df is freed at scope end
      }
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      o.count = 1;
    }
  }
  if (e == hipSuccess) e = hipError_t(launch_enqueue_op(h->n, h->args, o, pr));
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return to_code(e);
}

// Per-class sums of the event intervals of one recorded launch sequence.
int collect_profile(const rte::ProfRec& pr, double* ms, int64_t* counts) {
  for (int i = 0; i < pr.count; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, i == 0 ? static_cast<hipEvent_t>(pr.ev0) : static_cast<hipEvent_t>(pr.ev[i - 1]),
                            static_cast<hipEvent_t>(pr.ev[i])) != hipSuccess)
      return RTE_EDEVICE;
    ms[pr.cls[i]] += t;
    counts[pr.cls[i]] += 1;
  }
  return RTE_OK;
}
}  // namespace

int rte_expo_advance(rte_handle* h, double t_ps) { return expo_run(h, t_ps, nullptr); }

int rte_profile_expo(rte_handle* h, double t_ps, double* ms, int64_t* counts) {
  using namespace rte;
  if (!h || !ms || !counts) return RTE_EINVAL;
  for (int c = 0; c < PROF_CLASSES; ++c) {
    ms[c] = 0.0;
    counts[c] = 0;
  }
  ProfRec pr{};
  hipEvent_t e0;
  hipEvent_t ev[kMaxProfLaunches];
  if (hipEventCreate(&e0) != hipSuccess) return RTE_EDEVICE;
  int made = 0;
  for (; made < kMaxProfLaunches; ++made)
    if (hipEventCreate(&ev[made]) != hipSuccess) break;
  int rc = made == kMaxProfLaunches ? RTE_OK : RTE_EDEVICE;
  pr.ev0 = e0;
  for (int i = 0; i < made; ++i) pr.ev[i] = ev[i];
  if (rc == RTE_OK) rc = expo_run(h, t_ps, &pr);
  if (rc == RTE_OK) rc = collect_profile(pr, ms, counts);
  (void)hipEventDestroy(e0);
  for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
  return rc;
}

int rte_profile_kernels(rte_handle* h, int64_t nsteps, double* ms, int64_t* counts) {
  using namespace rte;
  if (!h || !ms || !counts || nsteps < 0 || h->batch_owned) return RTE_EINVAL;
  ProfRec pr{};
  hipEvent_t e0;
  hipEvent_t ev[kMaxProfLaunches];
  if (hipEventCreate(&e0) != hipSuccess) return RTE_EDEVICE;
  int made = 0;
  for (; made < kMaxProfLaunches; ++made)
    if (hipEventCreate(&ev[made]) != hipSuccess) break;
  pr.ev0 = e0;
  for (int i = 0; i < made; ++i) pr.ev[i] = ev[i];
  for (int c = 0; c < PROF_CLASSES; ++c) {
    ms[c] = 0.0;
    counts[c] = 0;
  }
  int rc = made == kMaxProfLaunches ? RTE_OK : RTE_EDEVICE;
  if (rc == RTE_OK && !h->spec_valid) {
    OpArgs f{};
    f.kind = OP_FWD;
    if (launch_enqueue_op(h->n, h->args, f, nullptr) != 0) rc = RTE_EDEVICE;
    else h->spec_valid = true;
  }
  for (int64_t s = 0; s < nsteps && rc == RTE_OK; ++s) {
    hipError_t e = hipError_t(launch_enqueue_op(h->n, h->args, step_op(), &pr));
    if (e == hipSuccess && pr.count > 0) e = hipEventSynchronize(ev[pr.count - 1]);
    if (e != hipSuccess) {
      rc = RTE_EDEVICE;
      break;
    }
    rc = collect_profile(pr, ms, counts);
  }
  (void)hipEventDestroy(e0);
  for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
  return rc;
}

void rte_destroy(rte_handle* h) {
  if (!h || h->batch_owned) return;   // a batch slot's handle belongs to its batch
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

// ====================================================== batched serving ==
//
// A batch holds `slots` solves of one configuration in one caller-owned
// workspace, slot s at offset s * stride with the common layout. One
// captured step graph per number of slot rows k launches every kernel of
// the time step once with k grid rows (the slot index), so all resident
// solves of the configuration advance in the same launches. A slot that is
// idle, finished or failed has a non-zero stop flag in its control block and
// its workgroups return at once. Slots are staged (tables and state uploaded
// on the batch's staging stream) from any thread, started in stream order on
// the compute stream by the next rte_batch_step, and observed through
// control-block copies taken after every queued chunk of steps.

namespace rte {

constexpr int kBatchRing = 4;   // chunks whose control-block copies can be in flight

__global__ void k_slot_start(Ctl* ctl, long long limit) {
  if (threadIdx.x == 0) {
    ctl->step = 0;
    ctl->tol = 0.0;
    ctl->limit = limit;
    ctl->stop = 0;
  }
}

enum {
  SLOT_FREE = RTE_SLOT_FREE, SLOT_STAGING = RTE_SLOT_STAGING, SLOT_STAGED = RTE_SLOT_STAGED,
  SLOT_RUNNING = RTE_SLOT_RUNNING, SLOT_DONE = RTE_SLOT_DONE, SLOT_FAILED = RTE_SLOT_FAILED
};

}  // namespace rte

struct rte_batch {
  rte_config cfg;
  int slots;
  size_t stride;
  unsigned char* ws;
  hipStream_t stream;   // compute: step graphs, slot starts
  hipStream_t stage;    // staging uploads
  hipStream_t read;     // result reads of finished slots
  std::vector<rte_handle*> h;
  std::vector<int> state;
  std::vector<long long> limit;
  std::vector<long long> start_seq;   // chunk sequence number at which the slot started
  std::vector<long long> final_step;
  std::vector<hipEvent_t> staged_ev;
  std::vector<hipGraph_t> graph;      // [k - 1]: k slot rows
  std::vector<hipGraphExec_t> exec;
  rte::Ctl* snap;                     // pinned [kBatchRing][slots]
  hipEvent_t ring_ev[rte::kBatchRing];
  long long ring_seq[rte::kBatchRing];
  int ring_rows[rte::kBatchRing];
  long long seq;                      // chunks queued
  size_t ctl_off;
  std::mutex mu;
};

namespace rte {
bool batch_config_ok(const rte_config* cfg) {
  // plane grids (the fused step) and the register coupling pass
  return config_ok(cfg) && cfg->n <= 128 && cfg->order_N <= kDenseOrder;
}
}  // namespace rte

extern "C" {

size_t rte_batch_slot_bytes(const rte_config* cfg) {
  if (!rte::batch_config_ok(cfg)) return 0;
  return rte::layout_of(cfg, true).total;
}

int rte_batch_create(const rte_config* cfg, int32_t slots, void* dev_ws, size_t ws_bytes, void* hip_stream,
                     rte_batch** out) {
  using namespace rte;
  if (!out) return RTE_EINVAL;
  *out = nullptr;
  if (!batch_config_ok(cfg) || slots < 1 || slots > 65535 || !hip_stream) return RTE_EINVAL;
  const Layout L = layout_of(cfg, true);
  if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) != 0 || ws_bytes / L.total < size_t(slots))
    return RTE_ENOMEM;
  rte_batch* b = new (std::nothrow) rte_batch();
  if (!b) return RTE_ENOMEM;
  b->cfg = *cfg;
  b->cfg.det_index = nullptr;
  b->slots = slots;
  b->stride = L.total;
  b->ws = static_cast<unsigned char*>(dev_ws);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ctl_off = L.ctl;
  b->h.assign(slots, nullptr);
  b->state.assign(slots, SLOT_FREE);
  b->limit.assign(slots, 0);
  b->start_seq.assign(slots, 0);
  b->final_step.assign(slots, 0);
  b->staged_ev.assign(slots, nullptr);
  b->graph.assign(slots, nullptr);
  b->exec.assign(slots, nullptr);
  b->snap = nullptr;
  b->seq = 0;
  hipError_t e = hipStreamCreateWithFlags(&b->stage, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->read, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->snap), sizeof(Ctl) * kBatchRing * slots);
  for (int i = 0; i < kBatchRing && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&b->ring_ev[i], hipEventDisableTiming);
    b->ring_seq[i] = -1;
    b->ring_rows[i] = 0;
  }
  for (int s = 0; s < slots && e == hipSuccess; ++s) e = hipEventCreateWithFlags(&b->staged_ev[s], hipEventDisableTiming);
  if (e == hipSuccess) {
    // every slot starts idle (stop = 3): launches that cover it skip it
    std::vector<Ctl> idle(slots);
    for (auto& c : idle) {
      c = Ctl{};
      c.stop = 3;
    }
    e = hipMemcpy2DAsync(b->ws + b->ctl_off, b->stride, idle.data(), sizeof(Ctl), sizeof(Ctl), size_t(slots),
                         hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  }
  if (e != hipSuccess) {
    rte_batch_destroy(b);
    return RTE_EDEVICE;
  }
  *out = b;
  return RTE_OK;
}

int rte_batch_admit(rte_batch* b, int32_t slot, const rte_medium* med, const int64_t* det_index, int64_t steps) {
  using namespace rte;
  if (!b || slot < 0 || slot >= b->slots || !med || steps < 1) return RTE_EINVAL;
  if (b->cfg.n_det > 0 && !det_index) return RTE_EINVAL;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->state[slot] != SLOT_FREE) return RTE_EINVAL;
    b->state[slot] = SLOT_STAGING;
  }
  rte_config cfg = b->cfg;
  cfg.det_index = b->cfg.n_det > 0 ? det_index : nullptr;
  rte_handle* h = nullptr;
  int rc = create_impl(&cfg, med, b->ws + size_t(slot) * b->stride, b->stride, b->stage, &h, true);
  if (rc == RTE_OK && hipEventRecord(b->staged_ev[slot], b->stage) != hipSuccess) rc = RTE_EDEVICE;
  std::lock_guard<std::mutex> lk(b->mu);
  if (rc != RTE_OK) {
    if (h) {
      h->batch_owned = false;
      rte_destroy(h);
    }
    b->state[slot] = SLOT_FREE;
    return rc;
  }
  h->stream = b->read;   // the slot handle's reads use the batch's read stream
  b->h[slot] = h;
  b->limit[slot] = steps;
  b->state[slot] = SLOT_STAGED;
  return RTE_OK;
}

int rte_batch_step(rte_batch* b, int64_t nsteps) {
  using namespace rte;
  if (!b || nsteps < 0) return RTE_EINVAL;
  std::lock_guard<std::mutex> lk(b->mu);
  hipError_t e = hipSuccess;
  // start staged slots, in stream order before the next chunk
  for (int s = 0; s < b->slots && e == hipSuccess; ++s) {
    if (b->state[s] != SLOT_STAGED) continue;
    e = hipStreamWaitEvent(b->stream, b->staged_ev[s], 0);
    if (e != hipSuccess) break;
    Ctl* c = reinterpret_cast<Ctl*>(b->ws + size_t(s) * b->stride + b->ctl_off);
    hipLaunchKernelGGL(k_slot_start, dim3(1), dim3(64), 0, b->stream, c, (long long)b->limit[s]);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    StepArgs a = b->h[s]->args;
    a.stream = b->stream;
    OpArgs f{};
    f.kind = OP_FWD;
    e = hipError_t(launch_enqueue_op(b->cfg.n, a, f, nullptr));
    b->state[s] = SLOT_RUNNING;
    b->start_seq[s] = b->seq;
  }
  if (e != hipSuccess) return RTE_EDEVICE;
  int rows = 0;
  for (int s = 0; s < b->slots; ++s)
    if (b->state[s] == SLOT_RUNNING) rows = s + 1;
  if (rows == 0 || nsteps == 0) return RTE_OK;
  if (!b->exec[rows - 1]) {
    // capture one step over `rows` slot rows (pointers of slot 0, stride)
    int s0 = 0;
    while (!b->h[s0]) ++s0;   // any staged slot gives the common layout
    StepArgs a = b->h[s0]->args;
    const ptrdiff_t shift = -ptrdiff_t(size_t(s0) * b->stride);
    auto mv = [&](auto* p) -> decltype(p) {
      using B = typename std::conditional<std::is_const<typename std::remove_pointer<decltype(p)>::type>::value,
                                          const unsigned char, unsigned char>::type;
      return p ? reinterpret_cast<decltype(p)>(reinterpret_cast<B*>(p) + shift) : p;
    };
    a.u = mv(a.u); a.v = mv(a.v); a.spec = mv(a.spec); a.dspec = mv(a.dspec); a.tw = mv(a.tw); a.kv = mv(a.kv);
    a.sig = mv(a.sig); a.q = mv(a.q); a.qflag = mv(a.qflag); a.phi_int = mv(a.phi_int); a.partial = mv(a.partial);
    a.readings = mv(a.readings); a.resid = mv(a.resid); a.det = mv(a.det); a.ctl = mv(a.ctl);
    a.stream = b->stream;
    a.nslot = rows;
    a.sstride = (long long)b->stride;
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = hipError_t(launch_enqueue_op(b->cfg.n, a, step_op(), nullptr));
      e = hipStreamEndCapture(b->stream, &b->graph[rows - 1]);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[rows - 1], b->graph[rows - 1], nullptr, nullptr, 0);
    if (e != hipSuccess) {
      b->exec[rows - 1] = nullptr;
      return RTE_EDEVICE;
    }
  }
  for (int64_t i = 0; i < nsteps && e == hipSuccess; ++i) e = hipGraphLaunch(b->exec[rows - 1], b->stream);
  if (e != hipSuccess) return RTE_EDEVICE;
  // control blocks of the slot rows after this chunk, into the pinned ring
  const int idx = int(b->seq % kBatchRing);
  if (b->ring_seq[idx] >= 0) e = hipEventSynchronize(b->ring_ev[idx]);   // at most kBatchRing chunks in flight
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(b->snap + size_t(idx) * b->slots, sizeof(Ctl), b->ws + b->ctl_off, b->stride, sizeof(Ctl),
                         size_t(rows), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ring_ev[idx], b->stream);
  if (e != hipSuccess) return RTE_EDEVICE;
  b->ring_seq[idx] = b->seq;
  b->ring_rows[idx] = rows;
  b->seq += 1;
  return RTE_OK;
}

int rte_batch_poll(rte_batch* b, int64_t* steps_done, int32_t* status, int32_t* in_flight) {
  using namespace rte;
  if (!b) return RTE_EINVAL;
  std::lock_guard<std::mutex> lk(b->mu);
  // newest chunk whose control-block copies have landed
  int best = -1, pending = 0;
  for (int i = 0; i < kBatchRing; ++i) {
    if (b->ring_seq[i] < 0) continue;
    const hipError_t q = hipEventQuery(b->ring_ev[i]);
    if (q == hipErrorNotReady) {
      ++pending;
      continue;
    }
    if (q != hipSuccess) return RTE_EDEVICE;
    if (best < 0 || b->ring_seq[i] > b->ring_seq[best]) best = i;
  }
  if (in_flight) *in_flight = pending;
  for (int s = 0; s < b->slots; ++s) {
    if (b->state[s] == SLOT_RUNNING && best >= 0 && b->ring_seq[best] >= b->start_seq[s] && s < b->ring_rows[best]) {
      const Ctl& c = b->snap[size_t(best) * b->slots + s];
      b->final_step[s] = c.step;
      if (c.stop == 3) b->state[s] = SLOT_DONE;
      else if (c.stop != 0) b->state[s] = SLOT_FAILED;
    }
    if (status) status[s] = b->state[s];
    if (steps_done)
      steps_done[s] = (b->state[s] == SLOT_RUNNING || b->state[s] == SLOT_DONE || b->state[s] == SLOT_FAILED)
                          ? b->final_step[s] : 0;
  }
  return RTE_OK;
}

int rte_batch_handle(rte_batch* b, int32_t slot, rte_handle** out) {
  using namespace rte;
  if (!b || !out || slot < 0 || slot >= b->slots) return RTE_EINVAL;
  std::lock_guard<std::mutex> lk(b->mu);
  if (b->state[slot] != SLOT_DONE && b->state[slot] != SLOT_FAILED) return RTE_EINVAL;
  *out = b->h[slot];
  return RTE_OK;
}

int rte_batch_release(rte_batch* b, int32_t slot) {
  using namespace rte;
  if (!b || slot < 0 || slot >= b->slots) return RTE_EINVAL;
  std::lock_guard<std::mutex> lk(b->mu);
  const int st = b->state[slot];
  if (st != SLOT_DONE && st != SLOT_FAILED && st != SLOT_STAGED) return RTE_EINVAL;
  if (b->h[slot]) {
    b->h[slot]->batch_owned = false;
    rte_destroy(b->h[slot]);
    b->h[slot] = nullptr;
  }
  b->state[slot] = SLOT_FREE;
  b->final_step[slot] = 0;
  return RTE_OK;
}

void rte_batch_destroy(rte_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->stage) (void)hipStreamSynchronize(b->stage);
  if (b->read) (void)hipStreamSynchronize(b->read);
  for (size_t k = 0; k < b->exec.size(); ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
  }
  for (auto* h : b->h)
    if (h) {
      h->batch_owned = false;
      rte_destroy(h);
    }
  for (auto ev : b->staged_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (int i = 0; i < rte::kBatchRing; ++i)
    if (b->ring_ev[i]) (void)hipEventDestroy(b->ring_ev[i]);
  if (b->snap) (void)hipHostFree(b->snap);
  if (b->stage) (void)hipStreamDestroy(b->stage);
  if (b->read) (void)hipStreamDestroy(b->read);
  delete b;
}

}  // extern "C"
