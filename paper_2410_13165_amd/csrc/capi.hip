// C ABI of the lattice Boltzmann library (declarations and contracts in
// include/lbm.h): argument checking, the host-side parameter maths
// (eps, m4, omega of Sec. 2.3 and Remark 5), buffer management and the
// stream-ordered launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "engine.hpp"
#include "fuse.hpp"

using namespace lbm;

struct lbm_handle {
  KParams kp{};
  int d = 0, q = 0;
  int64_t dims[kMaxDim] = {1, 1, 1, 1};
  int64_t nodes = 0;
  int precision = LBM_FP64;
  double m4 = 0.0, min_omega = 0.0;
  int entropy_stable = 0;
  hipStream_t stream = nullptr;
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_ctx = nullptr;
  void* buf[2] = {nullptr, nullptr};     // populations (or g in split mode)
  double* phib[2] = {nullptr, nullptr};  // split mode: phi
  double* partial = nullptr;             // kRedBlocks x kNumAcc
  double* result = nullptr;              // kNumAcc
  int cur = 0;
  int64_t step = 0;
  bool initialised = false;
  bool batch_member = false;  // stepped only through its lbm_batch
  std::string err;
  // how the current state was initialised (gradients w.r.t. phi0 need it)
  int init_kind = 0;  // 0 unknown, 1 analytic field, 2 device phi0 + FD gradient,
                      // 3 device phi0 + explicit gradient, 4 K = 1
  // tape of checkpoints for lbm_tape_gradient
  bool tape_active = false;
  int64_t tape_start = 0, tape_every = 0;
  std::vector<void*> tape_ckpt;
  // kernel timing (lbm_profile_begin / lbm_profile_end): 3 events per step
  std::vector<hipEvent_t> prof_ev;
  int64_t prof_cap = 0, prof_used = 0, prof_steps = 0;
  bool profiling = false;
  // two steps per bulk pass (float32, d = 3): scratch state for the wall rows
  int steps_per_pass = 1;
  void* fuse_buf = nullptr;     // state_bytes: populations (+ phi in split mode)
  double* xdata2 = nullptr;     // split mode: x_1-face data of the second step
  int device = 0;               // current device at lbm_create
  // non-finite checks every check_every steps (0: off)
  int64_t check_every = 0, last_check = 0;
  unsigned* nonfinite = nullptr;  // device counter
};

static thread_local std::string g_create_error;

// Scratch of lbm_step_static: a fixed device array that each GPU holds from
// the library's first use on it until the process ends.  Host code never
// uses the array's name as an address (on the host it only names the
// symbol); the device address comes from hipGetSymbolAddress, taken once per
// device with that device current (static_scratch_setup, from lbm_create).
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Resolve (once) the device address of `scratch` on the current device.
void static_scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) {
    g_scratch_ptr[dev] = ptr;
  } else {
    g_scratch_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
    (void)hipGetLastError();
  }
}

void* static_scratch(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace

namespace {

int fail(lbm_handle* h, int code, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_create_error = msg;
  return code;
}

int hip_fail(lbm_handle* h, hipError_t e, const char* what) {
  return fail(h, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* dev_alloc(lbm_handle* h, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (h->alloc) return h->alloc(bytes, h->alloc_ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(lbm_handle* h, void* p) {
  if (!p) return;
  if (h->free_fn)
    h->free_fn(p, h->alloc_ctx);
  else
    (void)hipFree(p);
}

size_t elem_size(int precision) { return precision == LBM_FP64 ? 8 : 4; }

// the split layout: float32 g_k plus 8 bytes of phi per node (float64, or a
// hi/lo pair of float32)
bool split_mode(int precision) {
  return precision == LBM_FP32_SPLIT || precision == LBM_FP32_HILO;
}

size_t pop_bytes(const lbm_handle* h) {
  return static_cast<size_t>(h->kp.pstride) * h->q * elem_size(h->precision);
}

size_t phi_bytes(const lbm_handle* h) { return static_cast<size_t>(h->nodes) * sizeof(double); }

void release(lbm_handle* h) {
  for (int i = 0; i < 2; ++i) {
    dev_free(h, h->buf[i]);
    dev_free(h, h->phib[i]);
    h->buf[i] = nullptr;
    h->phib[i] = nullptr;
  }
  dev_free(h, h->partial);
  dev_free(h, h->result);
  dev_free(h, h->nonfinite);
  h->nonfinite = nullptr;
  dev_free(h, h->kp.xdata);
  dev_free(h, h->fuse_buf);
  dev_free(h, h->xdata2);
  h->partial = h->result = nullptr;
  h->kp.xdata = nullptr;
  h->fuse_buf = nullptr;
  h->xdata2 = nullptr;
}

// Copy the analytic field into the kernel parameter block.
int setup_field(lbm_handle* h, const lbm_field* fld) {
  FieldDev& F = h->kp.field;
  std::memset(&F, 0, sizeof(F));
  F.kind = kFieldNone;
  if (!fld || fld->kind == LBM_FIELD_NONE) return LBM_OK;
  const int d = h->d;
  if (fld->kind == LBM_FIELD_TANH_BUBBLE) {
    if (!(fld->W > 0.0)) return fail(nullptr, LBM_EINVAL, "tanh field needs W > 0");
    F.kind = kFieldTanh;
    F.Rr = fld->Rr;
    F.W = fld->W;
    for (int a = 0; a < d; ++a) F.center[a] = fld->center[a];
    return LBM_OK;
  }
  if (fld->kind != LBM_FIELD_COS_SUM && fld->kind != LBM_FIELD_EXP_SUM)
    return fail(nullptr, LBM_EINVAL, "unknown field kind");
  if (fld->n_modes < 1 || fld->n_modes > kMaxModes)
    return fail(nullptr, LBM_EINVAL, "field n_modes must be in 1..16");
  if (!fld->amps || !fld->kvecs) return fail(nullptr, LBM_EINVAL, "field amps/kvecs missing");
  F.kind = fld->kind == LBM_FIELD_COS_SUM ? kFieldCos : kFieldExp;
  F.nmodes = fld->n_modes;
  const double hx = 0.5 * h->kp.dx;
  for (int j = 0; j < F.nmodes; ++j) {
    F.amp[j] = fld->amps[j];
    F.phase[j] = fld->phases ? fld->phases[j] : 0.0;
    double ku = 0.0;
    for (int a = 0; a < d; ++a) {
      const double k = fld->kvecs[j * d + a];
      if (!std::isfinite(k)) return fail(nullptr, LBM_EINVAL, "non-finite wave vector");
      F.kvec[j][a] = k;
      ku += k * h->kp.u[a];
      if (F.kind == kFieldCos) {
        F.rot[j][a][0] = std::cos(hx * k);
        F.rot[j][a][1] = std::sin(hx * k);
      } else {
        F.rot[j][a][0] = std::exp(-hx * k);
        F.rot[j][a][1] = std::exp(hx * k);
      }
    }
    F.ku[j] = ku;
  }
  return LBM_OK;
}

void setup_faces(KParams& kp, int d) {
  kp.nwfaces = 0;
  kp.wall_rows = 0;
  for (int a = 1; a < d; ++a) {
    if (kp.bc[a] == LBM_BC_PERIODIC) continue;
    long long cnt = 1;
    for (int b = 1; b < d; ++b) {
      if (b == a) continue;
      const bool inner = (b < a) && kp.bc[b] != LBM_BC_PERIODIC;
      cnt *= inner ? (kp.n[b] - 2) : kp.n[b];
    }
    for (int side = 0; side < 2; ++side) {
      kp.wface_axis[kp.nwfaces] = a;
      kp.wface_side[kp.nwfaces] = side;
      kp.wface_count[kp.nwfaces] = static_cast<int>(cnt);
      kp.wall_rows += static_cast<int>(cnt);
      ++kp.nwfaces;
    }
  }
}

size_t xdata_bytes(const lbm_handle* h) {
  if (h->kp.bc[0] == LBM_BC_PERIODIC || !split_mode(h->precision)) return 0;
  return sizeof(double) * 2 * (2 * h->d - 1) * static_cast<size_t>(h->kp.rows);
}

int sync_result(lbm_handle* h, double* host) {
  hipError_t e = hipMemcpyAsync(host, h->result, kNumAcc * sizeof(double), hipMemcpyDeviceToHost,
                                h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  return LBM_OK;
}

// FP32 mode: the deviations are taken from omega_k (mean(phi0) + R t).
int compute_reference(lbm_handle* h, const double* phi0) {
  if (h->precision != LBM_FP32) {
    h->kp.phi_ref = 0.0;
    return LBM_OK;
  }
  hipError_t e = launch_sum_phi0(h->kp, phi0, h->partial, h->result, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sum of phi0");
  double host[kNumAcc];
  int rc = sync_result(h, host);
  if (rc != LBM_OK) return rc;
  h->kp.phi_ref = host[0] / static_cast<double>(h->nodes);
  return LBM_OK;
}

size_t state_bytes(const lbm_handle* h) {
  return pop_bytes(h) + (split_mode(h->precision) ? phi_bytes(h) : 0);
}

// Device copy of the current state into a buffer of state_bytes(h).
hipError_t copy_state_out(lbm_handle* h, void* dst) {
  hipError_t e = hipMemcpyAsync(dst, h->buf[h->cur], pop_bytes(h), hipMemcpyDeviceToDevice,
                                h->stream);
  if (e == hipSuccess && split_mode(h->precision))
    e = hipMemcpyAsync(static_cast<char*>(dst) + pop_bytes(h), h->phib[h->cur], phi_bytes(h),
                       hipMemcpyDeviceToDevice, h->stream);
  return e;
}

double* blob_phi(const lbm_handle* h, void* blob) {
  return (split_mode(h->precision) && blob)
             ? reinterpret_cast<double*>(static_cast<char*>(blob) + pop_bytes(h))
             : nullptr;
}

int tape_push(lbm_handle* h) {
  void* b = dev_alloc(h, state_bytes(h));
  if (!b) return fail(h, LBM_ENOMEM, "checkpoint allocation failed");
  hipError_t e = copy_state_out(h, b);
  if (e != hipSuccess) {
    dev_free(h, b);
    return hip_fail(h, e, "checkpoint copy");
  }
  h->tape_ckpt.push_back(b);
  return LBM_OK;
}

void tape_clear(lbm_handle* h) {
  if (!h->tape_ckpt.empty()) (void)hipStreamSynchronize(h->stream);
  for (void* b : h->tape_ckpt) dev_free(h, b);
  h->tape_ckpt.clear();
  h->tape_active = false;
}

int set_state_impl(lbm_handle* h, const void* src_dev, int64_t step);

}  // namespace

extern "C" {

void lbm_params_default(lbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(lbm_params);
  p->dx = 1.0;
  p->g = 0.5;
  p->bc_order = 4;
  p->init_order = 3;
  p->precision = LBM_FP64;
  p->steps_per_pass = 2;
}

int lbm_create(int d, const int64_t* dims, double tau, const lbm_params* p, lbm_handle** out) {
  if (out) *out = nullptr;
  if (!out || !dims || !p) return fail(nullptr, LBM_EINVAL, "null argument");
  if (p->struct_size != sizeof(lbm_params))
    return fail(nullptr, LBM_EINVAL, "lbm_params.struct_size mismatch (use lbm_params_default)");
  if (d < 1 || d > kMaxDim) return fail(nullptr, LBM_EINVAL, "d must be in 1..4");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(nullptr, LBM_EINVAL, "tau must be > 0");
  if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(nullptr, LBM_EINVAL, "dx must be > 0");
  if (p->precision < LBM_FP64 || p->precision > LBM_FP32_HILO)
    return fail(nullptr, LBM_EINVAL, "unknown precision");
  if (p->init_order != 1 && p->init_order != 3)
    return fail(nullptr, LBM_EINVAL, "init_order must be 1 or 3");
  int64_t nodes = 1;
  int scheme = kNoWall;
  for (int a = 0; a < d; ++a) {
    if (dims[a] < 1) return fail(nullptr, LBM_EINVAL, "dims must be >= 1");
    if (dims[a] > (int64_t(1) << 30)) return fail(nullptr, LBM_EINVAL, "dimension too large");
    nodes *= dims[a];
    if (nodes > std::numeric_limits<int32_t>::max())
      return fail(nullptr, LBM_EINVAL, "more than 2^31-1 nodes");
    const int lo = p->bc[a][0], hi = p->bc[a][1];
    for (const int bc : {lo, hi})
      if (bc != LBM_BC_PERIODIC && bc != LBM_BC_FULLWAY && bc != LBM_BC_HALFWAY)
        return fail(nullptr, LBM_EINVAL, "unknown boundary code");
    if ((lo == LBM_BC_PERIODIC) != (hi == LBM_BC_PERIODIC))
      return fail(nullptr, LBM_EINVAL, "a periodic face needs a periodic opposite face");
    if (lo != LBM_BC_PERIODIC) {
      if (dims[a] < 2) return fail(nullptr, LBM_EINVAL, "a Dirichlet axis needs >= 2 nodes");
      for (const int bc : {lo, hi}) {
        const int sch = bc == LBM_BC_FULLWAY ? kFullWay : kHalfWay;
        if (scheme != kNoWall && scheme != sch)
          return fail(nullptr, LBM_EUNSUPPORTED,
                      "full-way and half-way faces cannot be mixed in one lattice");
        scheme = sch;
      }
    }
  }
  if (scheme == kFullWay && p->bc_order != 1 && p->bc_order != 3 && p->bc_order != 4)
    return fail(nullptr, LBM_EINVAL, "full-way order must be 1, 3 or 4");
  if (scheme == kHalfWay && (p->bc_order < 1 || p->bc_order > 4))
    return fail(nullptr, LBM_EINVAL, "half-way order must be 1..4");
  if (scheme != kNoWall && (!p->field || p->field->kind == LBM_FIELD_NONE))
    return fail(nullptr, LBM_EINVAL, "Dirichlet walls need an analytic field for their data");
  if (scheme != kNoWall && p->field->kind == LBM_FIELD_TANH_BUBBLE)
    return fail(nullptr, LBM_EUNSUPPORTED, "the tanh field supplies no wall derivatives");
  if (p->wall_data != LBM_WALL_JETS && p->wall_data != LBM_WALL_TANGENTIAL)
    return fail(nullptr, LBM_EINVAL, "unknown wall_data");
  if (p->steps_per_pass != 1 && p->steps_per_pass != 2)
    return fail(nullptr, LBM_EINVAL, "steps_per_pass must be 1 or 2");
  if (p->check_every < 0) return fail(nullptr, LBM_EINVAL, "check_every must be >= 0");
  if (p->wall_data == LBM_WALL_TANGENTIAL)
    for (int a = 0; a < d; ++a)
      if (p->bc[a][0] != LBM_BC_PERIODIC && !(std::fabs(p->u[a]) > 0.0))
        return fail(nullptr, LBM_EINVAL,
                    "tangential wall data need u_j != 0 on every Dirichlet axis j");

  lbm_handle* h = new (std::nothrow) lbm_handle();
  if (!h) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
  h->d = d;
  h->q = q_of(d);
  h->nodes = nodes;
  h->precision = p->precision;
  h->steps_per_pass =
      (p->steps_per_pass == 2 && (d == 3 || (d == 2 && !split_mode(p->precision)))) ? 2
                                                                                        : 1;
  h->stream = static_cast<hipStream_t>(p->stream);
  if (hipGetDevice(&h->device) != hipSuccess) {
    (void)hipGetLastError();
    h->device = -1;
  }
  h->alloc = p->alloc;
  h->free_fn = p->free_fn;
  h->alloc_ctx = p->alloc_ctx;
  if ((h->alloc == nullptr) != (h->free_fn == nullptr)) {
    delete h;
    return fail(nullptr, LBM_EINVAL, "alloc and free_fn must both be set or both be NULL");
  }

  KParams& kp = h->kp;
  kp.d = d;
  kp.q = h->q;
  int64_t st = 1;
  for (int a = 0; a < kMaxDim; ++a) {
    const int64_t n = a < d ? dims[a] : 1;
    h->dims[a] = n;
    kp.n[a] = static_cast<int>(n);
    kp.stride[a] = static_cast<int>(st);
    st *= n;
    kp.bc[a] = a < d ? p->bc[a][0] : 0;
    kp.origin[a] = a < d ? p->origin[a] : 0.0;
    kp.u[a] = a < d ? p->u[a] : 0.0;
    kp.inv_u[a] = (a < d && p->bc[a][0] != LBM_BC_PERIODIC && p->u[a] != 0.0) ? 1.0 / p->u[a] : 0.0;
    kp.shift[a] = (a < d && p->bc[a][0] == LBM_BC_HALFWAY) ? 0.5 : 0.0;
  }
  kp.wall_data = p->wall_data;
  kp.nodes = static_cast<int>(nodes);
  kp.rows = static_cast<int>(nodes / dims[0]);
  // population planes: the nodes, then (with walls on x_1) one slot per row
  // for the x_1-face wall data; 256-byte aligned
  kp.xoff = static_cast<int>(nodes);
  const int64_t plane = nodes + (p->bc[0][0] != LBM_BC_PERIODIC ? nodes / dims[0] : 0);
  if (plane > std::numeric_limits<int32_t>::max()) {
    delete h;
    return fail(nullptr, LBM_EINVAL, "more than 2^31-1 nodes plus wall slots");
  }
  kp.pstride = (plane + 63) / 64 * 64;
  kp.scheme = scheme;
  kp.P = p->bc_order;
  kp.K = p->init_order;
  kp.tau = tau;
  kp.s = 1.0 / tau;
  kp.s_f = static_cast<float>(kp.s);
  kp.oms_f = static_cast<float>(1.0 - kp.s);
  kp.dx = p->dx;
  kp.dt = p->dx;  // c = 1
  kp.R = p->R;
  kp.dtR = kp.dt * kp.R;
  kp.dtR_hi = static_cast<float>(kp.dtR);
  kp.dtR_lo = static_cast<float>(kp.dtR - static_cast<double>(kp.dtR_hi));
  setup_faces(kp, d);

  // eps and omega: eq. (meq), eq. (meq-4rd) with g, closed form eq. (omega_k-2)
  double u[kMaxDim] = {0, 0, 0, 0};
  for (int a = 0; a < d; ++a) {
    u[a] = p->u[a];
    if (!std::isfinite(u[a])) {
      delete h;
      return fail(nullptr, LBM_EINVAL, "non-finite u");
    }
  }
  double g = std::isnan(p->g) ? 0.5 : p->g;
  h->m4 = (d >= 2) ? (p->use_m4 ? p->m4 : m4_interpolated(d, u, g)) : 0.0;
  omega_closed_form(d, u, h->m4, kp.omega);
  h->min_omega = kp.omega[0];
  for (int k = 0; k < h->q; ++k) {
    kp.omega_f[k] = static_cast<float>(kp.omega[k]);
    kp.omega_lo[k] = static_cast<float>(kp.omega[k] - static_cast<double>(kp.omega_f[k]));
    h->min_omega = std::fmin(h->min_omega, kp.omega[k]);
  }
  h->entropy_stable = h->min_omega > 0.0 ? 1 : 0;
  for (int k = 0; k < h->q; ++k) {
    for (int a = 0; a < kMaxDim; ++a)
      kp.cv[k][a] = static_cast<signed char>(a < d ? vel_comp(d, k, a) : 0);
    kp.kbar[k] = opp_index(d, k);
  }

  if (int rc = setup_field(h, p->field); rc != LBM_OK) {
    delete h;
    return rc;
  }

  // device buffers
  const size_t pb = pop_bytes(h);
  for (int i = 0; i < 2; ++i) {
    h->buf[i] = dev_alloc(h, pb);
    if (split_mode(h->precision)) h->phib[i] = static_cast<double*>(dev_alloc(h, phi_bytes(h)));
  }
  h->partial = static_cast<double*>(dev_alloc(h, sizeof(double) * kRedBlocks * kNumAcc));
  h->result = static_cast<double*>(dev_alloc(h, sizeof(double) * kNumAcc));
  h->check_every = p->check_every;
  if (h->check_every > 0) h->nonfinite = static_cast<unsigned*>(dev_alloc(h, 256));
  if (xdata_bytes(h) > 0) kp.xdata = static_cast<double*>(dev_alloc(h, xdata_bytes(h)));
  bool ok = h->buf[0] && h->buf[1] && h->partial && h->result &&
            (h->check_every == 0 || h->nonfinite);
  if (xdata_bytes(h) > 0) ok = ok && kp.xdata;
  if (split_mode(h->precision)) ok = ok && h->phib[0] && h->phib[1];
  if (!ok) {
    release(h);
    delete h;
    return fail(nullptr, LBM_ENOMEM, "device allocation failed");
  }
  // Deterministic content for the padding between population planes.
  for (int i = 0; i < 2; ++i) {
    hipError_t e = hipMemsetAsync(h->buf[i], 0, pb, h->stream);
    if (e != hipSuccess) {
      int rc = hip_fail(nullptr, e, "hipMemsetAsync");
      release(h);
      delete h;
      return rc;
    }
  }

  if (kp.field.kind != kFieldNone) {
    int rc = compute_reference(h, nullptr);
    if (rc == LBM_OK) {
      hipError_t e = launch_init(kp, h->precision, h->buf[0], h->phib[0], nullptr, nullptr,
                                 h->stream);
      if (e != hipSuccess) rc = hip_fail(h, e, "initialisation kernel");
    }
    if (rc == LBM_OK) {
      hipError_t e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) rc = hip_fail(h, e, "hipStreamSynchronize");
    }
    if (rc != LBM_OK) {
      g_create_error = h->err;
      release(h);
      delete h;
      return rc;
    }
    h->initialised = true;
    h->init_kind = (p->init_order == 1) ? 4 : 1;
  }
  static_scratch_setup(h->device);
  h->cur = 0;
  h->step = 0;
  *out = h;
  return LBM_OK;
}

int lbm_set_initial(lbm_handle* h, const double* phi0_dev, const double* grad_phi0_dev) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (!phi0_dev) return fail(h, LBM_EINVAL, "phi0 is NULL");
  if (h->kp.K == 3 && !grad_phi0_dev) {
    for (int a = 0; a < h->d; ++a)
      if (h->kp.bc[a] != LBM_BC_PERIODIC)
        return fail(h, LBM_EINVAL, "finite-difference gradients need periodic axes");
  }
  // a tape recorded before belongs to the previous run
  tape_clear(h);
  int rc = compute_reference(h, phi0_dev);
  if (rc != LBM_OK) return rc;
  hipError_t e = launch_init(h->kp, h->precision, h->buf[0], h->phib[0], phi0_dev, grad_phi0_dev,
                             h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "initialisation kernel");
  h->cur = 0;
  h->step = 0;
  h->last_check = 0;
  h->initialised = true;
  h->init_kind = (h->kp.K == 1) ? 4 : (grad_phi0_dev ? 3 : 2);
  return LBM_OK;
}

}  // extern "C"

namespace {

// Checks shared by the stepping entry points.
int step_checks(lbm_handle* h, int64_t n) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (n < 0) return fail(h, LBM_EINVAL, "n must be >= 0");
  if (h->batch_member) return fail(h, LBM_EINVAL, "batch instances are stepped by lbm_batch_step");
  if (!h->initialised) return fail(h, LBM_EINVAL, "no initial state (call lbm_set_initial)");
  return LBM_OK;
}

// Pairs of steps in one bulk pass where the lattice allows it; while a tape
// records checkpoints every `every` steps, pairs only when every is even and
// the pair starts on an even offset, so that no checkpoint falls inside one.
bool use_pairs(const lbm_handle* h) {
  return h->steps_per_pass == 2 && (!h->tape_active || h->tape_every % 2 == 0);
}

// Scratch state of a two-step pass: the rows on and next to the Dirichlet
// walls of x_2 / x_3 pass through it, so lattices without such walls need none.
size_t pair_state_bytes(const lbm_handle* h) {
  return h->kp.wall_rows > 0 ? state_bytes(h) : 0;
}

// n steps with the two-step scratch at cbuf (pair_state_bytes) and the split
// mode's second x_1-face array at xd2 (xdata_bytes).
// Count the non-finite values of population plane 0 of the stored state
// (split mode: phi).  Post-collision, f*_0 = (1 - s) f_0 + omega_0 (s phi + dt R)
// carries every population of its node through phi; with omega_0 = 0 plane 1
// is counted as well.
hipError_t check_nonfinite(lbm_handle* h) {
  if (h->precision == LBM_FP32_SPLIT)
    return launch_count_nonfinite(h->phib[h->cur], true, h->nodes, h->nonfinite, h->stream);
  if (h->precision == LBM_FP32_HILO)  // hi and lo of every node
    return launch_count_nonfinite(h->phib[h->cur], false, 2 * h->nodes, h->nonfinite, h->stream);
  const bool dbl = h->precision == LBM_FP64;
  const size_t es = elem_size(h->precision);
  const int planes = h->kp.omega[0] == 0.0 ? 2 : 1;
  hipError_t e = hipSuccess;
  for (int k = 0; k < planes && e == hipSuccess; ++k)
    e = launch_count_nonfinite(static_cast<char*>(h->buf[h->cur]) + k * h->kp.pstride * es, dbl,
                               h->nodes, h->nonfinite, h->stream);
  return e;
}

int run_steps(lbm_handle* h, int64_t n, void* cbuf, double* xd2) {
  const bool pairs = use_pairs(h);
  bool checked = false;
  if (h->check_every > 0 && n > 0) {
    hipError_t e = launch_zero_count(h->nonfinite, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "non-finite counter");
  }
  int64_t i = 0;
  while (i < n) {
    const int src = h->cur, dst = 1 - h->cur;
    const bool aligned = !h->tape_active || (h->step - h->tape_start) % 2 == 0;
    const int64_t todo = (pairs && aligned && n - i >= 2) ? 2 : 1;
    hipEvent_t* ev = nullptr;
    if (h->profiling && h->prof_used < h->prof_cap) {
      ev = &h->prof_ev[3 * h->prof_used];
      ++h->prof_used;
      h->prof_steps += todo;
    }
    hipError_t e;
    if (todo == 2) {
      const FusedBufs fb{h->buf[src], h->buf[dst], cbuf, h->phib[src], h->phib[dst],
                         blob_phi(h, cbuf), xd2};
      e = launch_fused_pair(h->kp, h->precision, fb, h->step, h->stream, ev);
    } else {
      e = launch_step(h->kp, h->precision, h->buf[src], h->buf[dst], h->phib[src],
                      h->phib[dst], h->step, h->stream, ev);
    }
    if (e != hipSuccess) return hip_fail(h, e, "step kernel");
    h->cur = dst;
    h->step += todo;
    i += todo;
    if (h->tape_active && (h->step - h->tape_start) % h->tape_every == 0) {
      int rc = tape_push(h);
      if (rc != LBM_OK) return rc;
    }
    if (h->check_every > 0 && h->step - h->last_check >= h->check_every) {
      e = check_nonfinite(h);
      if (e != hipSuccess) return hip_fail(h, e, "non-finite check");
      h->last_check = h->step;
      checked = true;
    }
  }
  if (checked) {
    unsigned bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, h->nonfinite, sizeof(bad), hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "non-finite check readback");
    if (bad > 0)
      return fail(h, LBM_ENONFINITE,
                  std::to_string(bad) + " non-finite values in the state by step " +
                      std::to_string(h->step));
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_step(lbm_handle* h, int64_t n) {
  if (int rc = step_checks(h, n); rc != LBM_OK) return rc;
  if (use_pairs(h) && n >= 2) {
    if (pair_state_bytes(h) > 0 && !h->fuse_buf) {
      h->fuse_buf = dev_alloc(h, pair_state_bytes(h));
      if (!h->fuse_buf) return fail(h, LBM_ENOMEM, "scratch state for two-step passes");
    }
    if (xdata_bytes(h) > 0 && !h->xdata2) {
      h->xdata2 = static_cast<double*>(dev_alloc(h, xdata_bytes(h)));
      if (!h->xdata2) return fail(h, LBM_ENOMEM, "x-face data for two-step passes");
    }
  }
  return run_steps(h, n, h->fuse_buf, h->xdata2);
}

int lbm_step_static(lbm_handle* h, int64_t n) {
  if (int rc = step_checks(h, n); rc != LBM_OK) return rc;
  if (h->tape_active)
    return fail(h, LBM_EINVAL, "lbm_step_static cannot record a tape (checkpoints are allocated)");
  void* cbuf = nullptr;
  double* xd2 = nullptr;
  if (use_pairs(h) && n >= 2) {
    const size_t cb = (pair_state_bytes(h) + 255) / 256 * 256;
    const size_t need = cb + xdata_bytes(h);
    if (need > kStaticScratchBytes)
      return fail(h, LBM_EINVAL,
                  "lbm_step_static needs " + std::to_string(need) +
                      " bytes of scratch for this lattice; its fixed scratch holds " +
                      std::to_string(kStaticScratchBytes) + " (use lbm_step)");
    if (need > 0) {
      hipError_t err = hipSuccess;
      void* base = static_scratch(h->device, &err);
      if (!base) return hip_fail(h, err, "address of the static scratch");
      if (pair_state_bytes(h) > 0) cbuf = base;
      if (xdata_bytes(h) > 0) xd2 = reinterpret_cast<double*>(static_cast<char*>(base) + cb);
    }
  }
  return run_steps(h, n, cbuf, xd2);
}

int lbm_moments(lbm_handle* h, uint32_t what, double* phi_out_dev, double* scalars_host) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (what & ~static_cast<uint32_t>(LBM_MOM_ALL)) return fail(h, LBM_EINVAL, "unknown bits in what");
  const uint32_t scalar_bits = what & (LBM_MOM_SUMS | LBM_MOM_RMSE | LBM_MOM_ENTROPY);
  if ((what & LBM_MOM_PHI) && !phi_out_dev)
    return fail(h, LBM_EINVAL, "LBM_MOM_PHI needs phi_out_dev");
  if (scalar_bits && !scalars_host)
    return fail(h, LBM_EINVAL, "scalar moments need scalars_host");
  if (!h->initialised) return fail(h, LBM_EINVAL, "no initial state");
  if (what == 0) return LBM_OK;
  hipError_t e = launch_moments(h->kp, h->precision, h->buf[h->cur], h->phib[h->cur], h->step,
                                (what & LBM_MOM_PHI) ? phi_out_dev : nullptr, h->partial,
                                h->result, what, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "moments kernel");
  if (!scalar_bits) return LBM_OK;
  double acc[kNumAcc];
  int rc = sync_result(h, acc);
  if (rc != LBM_OK) return rc;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const bool sums = what & LBM_MOM_SUMS;
  const bool err = (what & LBM_MOM_RMSE) && h->kp.field.kind != kFieldNone;
  const bool ent = (what & LBM_MOM_ENTROPY) && (split_mode(h->precision) || h->kp.s != 1.0);
  scalars_host[0] = sums ? acc[0] : nan;
  scalars_host[1] = sums ? acc[1] : nan;
  scalars_host[2] = err ? acc[2] : nan;
  scalars_host[3] = ent ? acc[3] : nan;
  scalars_host[4] = sums ? acc[4] : nan;
  scalars_host[5] = sums ? acc[5] : nan;
  scalars_host[6] = err ? std::sqrt(acc[2] / static_cast<double>(h->nodes)) : nan;
  scalars_host[7] = static_cast<double>(h->step) * h->kp.dt;
  return LBM_OK;
}

int lbm_info(const lbm_handle* h, lbm_info_t* out) {
  if (!h || !out) return fail(nullptr, LBM_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->d = h->d;
  out->q = h->q;
  out->precision = h->precision;
  out->entropy_stable = h->entropy_stable;
  for (int a = 0; a < kMaxDim; ++a) out->dims[a] = a < h->d ? h->dims[a] : 0;
  out->nodes = h->nodes;
  out->step = h->step;
  for (int k = 0; k < h->q; ++k) out->omega[k] = h->kp.omega[k];
  out->m4 = h->m4;
  out->min_omega = h->min_omega;
  out->s = h->kp.s;
  out->dt = h->kp.dt;
  out->phi_ref = h->kp.phi_ref;
  const int es = static_cast<int>(elem_size(h->precision));
  out->bytes_per_lu = 2 * h->q * es + (split_mode(h->precision) ? 16 : 0);
  out->pstride = h->kp.pstride;
  out->steps_per_pass = h->steps_per_pass;
  return LBM_OK;
}

int64_t lbm_state_bytes(const lbm_handle* h) {
  if (!h) return -1;
  int64_t b = static_cast<int64_t>(pop_bytes(h));
  if (split_mode(h->precision)) b += static_cast<int64_t>(phi_bytes(h));
  return b;
}

int lbm_get_state(const lbm_handle* h, void* dst_dev) {
  if (!h || !dst_dev) return fail(nullptr, LBM_EINVAL, "null argument");
  lbm_handle* mh = const_cast<lbm_handle*>(h);
  hipError_t e = hipMemcpyAsync(dst_dev, h->buf[h->cur], pop_bytes(h), hipMemcpyDeviceToDevice,
                                h->stream);
  if (e == hipSuccess && split_mode(h->precision))
    e = hipMemcpyAsync(static_cast<char*>(dst_dev) + pop_bytes(h), h->phib[h->cur], phi_bytes(h),
                       hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(mh, e, "hipMemcpyAsync");
  return LBM_OK;
}

int lbm_set_state(lbm_handle* h, const void* src_dev, int64_t step) {
  if (!h || !src_dev) return fail(nullptr, LBM_EINVAL, "null argument");
  if (step < 0) return fail(h, LBM_EINVAL, "step must be >= 0");
  if (h->batch_member) return fail(h, LBM_EINVAL, "batch instances take their state from the batch");
  return set_state_impl(h, src_dev, step);
}

}  // extern "C"

namespace {
int set_state_impl(lbm_handle* h, const void* src_dev, int64_t step) {
  tape_clear(h);
  hipError_t e = hipMemcpyAsync(h->buf[h->cur], src_dev, pop_bytes(h), hipMemcpyDeviceToDevice,
                                h->stream);
  if (e == hipSuccess && split_mode(h->precision))
    e = hipMemcpyAsync(h->phib[h->cur], static_cast<const char*>(src_dev) + pop_bytes(h),
                       phi_bytes(h), hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync");
  h->step = step;
  h->last_check = step;
  h->initialised = true;
  h->init_kind = 0;
  return LBM_OK;
}

void destroy_events(lbm_handle* h) {
  for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
  h->prof_ev.clear();
  h->prof_cap = h->prof_used = h->prof_steps = 0;
  h->profiling = false;
}
}  // namespace

extern "C" {

int lbm_profile_begin(lbm_handle* h, int64_t max_launches) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (h->profiling) return fail(h, LBM_EINVAL, "profiling already active");
  if (max_launches < 1 || max_launches > (int64_t(1) << 20))
    return fail(h, LBM_EINVAL, "max_launches must be in 1..2^20");
  h->prof_ev.assign(static_cast<size_t>(3 * max_launches), nullptr);
  for (auto& e : h->prof_ev) {
    hipError_t rc = hipEventCreate(&e);
    if (rc != hipSuccess) {
      destroy_events(h);
      return hip_fail(h, rc, "hipEventCreate");
    }
  }
  h->prof_cap = max_launches;
  h->prof_used = 0;
  h->prof_steps = 0;
  h->profiling = true;
  return LBM_OK;
}

int lbm_profile_end(lbm_handle* h, double* bulk_ms, double* wall_ms, int64_t* steps,
                    int64_t* launches) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (!h->profiling) return fail(h, LBM_EINVAL, "profiling not active");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    destroy_events(h);
    return hip_fail(h, e, "hipStreamSynchronize");
  }
  double b = 0.0, w = 0.0;
  for (int64_t i = 0; i < h->prof_used; ++i) {
    float t01 = 0.0f, t12 = 0.0f;
    e = hipEventElapsedTime(&t01, h->prof_ev[3 * i], h->prof_ev[3 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t12, h->prof_ev[3 * i + 1], h->prof_ev[3 * i + 2]);
    if (e != hipSuccess) {
      destroy_events(h);
      return hip_fail(h, e, "hipEventElapsedTime");
    }
    b += t01;
    w += t12;
  }
  if (bulk_ms) *bulk_ms = b;
  if (wall_ms) *wall_ms = h->kp.wall_rows > 0 ? w : 0.0;
  if (steps) *steps = h->prof_steps;
  if (launches) *launches = h->prof_used;
  destroy_events(h);
  return LBM_OK;
}

int lbm_tape_begin(lbm_handle* h, int64_t every) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (!h->initialised) return fail(h, LBM_EINVAL, "no initial state");
  if (every < 1) return fail(h, LBM_EINVAL, "checkpoint interval must be >= 1");
  if (h->batch_member) return fail(h, LBM_EINVAL, "batch instances cannot record a tape");
  if (h->precision == LBM_FP32_HILO)
    return fail(h, LBM_EUNSUPPORTED, "tapes support LBM_FP64, LBM_FP32 and LBM_FP32_SPLIT");
  tape_clear(h);
  h->tape_start = h->step;
  h->tape_every = every;
  h->tape_active = true;
  int rc = tape_push(h);
  if (rc != LBM_OK) h->tape_active = false;
  return rc;
}

int lbm_tape_end(lbm_handle* h) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  tape_clear(h);
  return LBM_OK;
}

int lbm_tape_gradient(lbm_handle* h, const double* dl_dphi_dev, double* dl_dphi0_dev,
                      double* dl_dgrad0_dev, double* dl_dtau_host, double* dl_dwall_host) {
  if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
  if (!h->tape_active) return fail(h, LBM_EINVAL, "no active tape (call lbm_tape_begin)");
  if (!dl_dphi_dev) return fail(h, LBM_EINVAL, "dL/dphi is NULL");
  const bool want_wall = dl_dwall_host != nullptr;
  if (want_wall && (h->kp.scheme == kNoWall ||
                    (h->kp.field.kind != kFieldCos && h->kp.field.kind != kFieldExp)))
    return fail(h, LBM_EINVAL, "wall-data gradients need Dirichlet walls fed by a cos or exp field");
  const bool want_init = dl_dphi0_dev || dl_dgrad0_dev;
  const bool at_init = h->tape_start == 0 && h->init_kind != 0;
  if (want_init && !at_init)
    return fail(h, LBM_EINVAL, "initial-state gradients need a tape that starts at an initialisation");
  if (dl_dtau_host && h->precision != LBM_FP32_SPLIT && h->kp.s == 1.0)
    return fail(h, LBM_EUNSUPPORTED, "dL/dtau needs s != 1 with post-collision storage");
  const KParams& kp = h->kp;
  const int64_t N = h->step - h->tape_start;
  const int64_t K = h->tape_every;
  const int64_t nseg = (N + K - 1) / K;
  // segment i starts from checkpoint i; a tape that does not cover the steps
  // taken since lbm_tape_begin cannot be replayed
  if (N < 0 || K < 1 || h->tape_ckpt.empty() ||
      static_cast<int64_t>(h->tape_ckpt.size()) < std::max<int64_t>(nseg, 1))
    return fail(h, LBM_EINVAL, "the tape does not cover the current step");
  const bool want_tau = dl_dtau_host != nullptr;
  const size_t pb = pop_bytes(h), sb = state_bytes(h);
  const LaunchShape shp = step_shape(kp);

  std::vector<void*> owned;
  auto alloc = [&](size_t bytes) -> void* {
    void* b = dev_alloc(h, bytes);
    if (b) owned.push_back(b);
    return b;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(h->stream);
    for (void* b : owned) dev_free(h, b);
    owned.clear();
  };
  void* lam[2] = {alloc(pb), alloc(pb)};
  // adjoint passes of two steps (d = 3) pair the adjoint steps within each
  // segment; the wall-data contractions need every lambda^n, so single steps
  const bool pairs = h->steps_per_pass == 2 && h->d == 3 && !want_wall;
  const long long npart =
      std::max<long long>(shp.blocks, pairs ? adjoint_pair_blocks(kp, h->precision) : 0);
  double* partial = static_cast<double*>(alloc(sizeof(double) * npart));
  // dsteps[0]: sum over the steps of the dL/ds contractions; dsteps[1]: the
  // initialisation's tau term
  double* dsteps = static_cast<double*>(alloc(sizeof(double) * 2));
  double* partial_init = static_cast<double*>(alloc(sizeof(double) * 65536));
  double* partial_wall =
      want_wall ? static_cast<double*>(alloc(sizeof(double) * (wall_grad_partials() + 2 * kMaxModes)))
                : nullptr;
  std::vector<void*> seg;
  if (want_tau && N > 0)
    for (int64_t i = 1; i < std::min<int64_t>(K, N); ++i) seg.push_back(alloc(sb));
  bool ok = lam[0] && lam[1] && partial && dsteps && partial_init && (!want_wall || partial_wall);
  for (void* b : seg) ok = ok && b;
  if (!ok) {
    cleanup();
    return fail(h, LBM_ENOMEM, "adjoint buffers");
  }
  // lam[0] is written for every node by the seed and lam[1] by the first
  // adjoint step; the slots past the nodes are never read
  hipError_t e = hipMemsetAsync(partial, 0, sizeof(double) * npart, h->stream);
  if (e == hipSuccess && want_wall)
    e = hipMemsetAsync(partial_wall, 0, sizeof(double) * wall_grad_partials(), h->stream);
  if (e == hipSuccess) e = launch_adjoint_seed(kp, h->precision, dl_dphi_dev, lam[0], h->stream);
  int cur = 0;
  for (int64_t sgi = nseg - 1; sgi >= 0 && e == hipSuccess; --sgi) {
    const int64_t s0 = h->tape_start + sgi * K;
    const int64_t s1 = std::min<int64_t>(s0 + K, h->step);
    // forward states g^{s0} .. g^{s1-1} of this segment (only for dL/dtau)
    std::vector<void*> st;
    if (want_tau) {
      st.push_back(h->tape_ckpt[sgi]);
      // single steps: every state is stored, and a two-step pass that also
      // stores its intermediate state takes longer than the two single steps
      // (measured: split mode at 256^3, 1.17 ms against 2 x 0.57 ms)
      for (int64_t n = s0 + 1; n < s1 && e == hipSuccess; ++n) {
        void* src = st.back();
        void* dst = seg[n - s0 - 1];
        e = launch_step(kp, h->precision, src, dst, blob_phi(h, src), blob_phi(h, dst), n - 1,
                        h->stream);
        st.push_back(dst);
      }
    }
    for (int64_t n = s1 - 1; n >= s0 && e == hipSuccess;) {
      const void* g = want_tau ? st[n - s0] : nullptr;
      if (pairs && n - 1 >= s0) {
        const void* g2 = want_tau ? st[n - 1 - s0] : nullptr;
        e = launch_adjoint_pair(kp, h->precision, lam[cur], lam[1 - cur], g, g2, partial,
                                h->stream);
        n -= 2;
      } else {
        // lam[cur] holds lambda^{n+1}: the sensitivities of the wall values of step n+1
        if (want_wall) e = launch_wall_grad(kp, h->precision, lam[cur], n, partial_wall, h->stream);
        if (e == hipSuccess)
          e = launch_adjoint_step(kp, h->precision, lam[cur], lam[1 - cur], g,
                                want_tau ? blob_phi(h, const_cast<void*>(g)) : nullptr, partial,
                                h->stream);
        n -= 1;
      }
      cur = 1 - cur;
    }
  }
  // dL/ds (without the 1/(1-s) of the post-collision modes), summed over the steps
  if (e == hipSuccess && want_tau) e = launch_sum_partials(partial, npart, dsteps, h->stream);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(h, e, "adjoint kernels");
  }
  // lambda^{start} = dL/df at the start of the tape
  double init_tau = 0.0;
  if (want_init || (want_tau && at_init)) {
    const bool fd = h->init_kind == 2;
    double* dphi = dl_dphi0_dev ? dl_dphi0_dev : static_cast<double*>(alloc(phi_bytes(h)));
    double* dgrad = dl_dgrad0_dev;
    if (!dgrad && fd) dgrad = static_cast<double*>(alloc(phi_bytes(h) * h->d));
    if (!dphi || (fd && !dgrad)) {
      cleanup();
      return fail(h, LBM_ENOMEM, "adjoint buffers");
    }
    unsigned nb = 0;
    e = launch_adjoint_init(kp, h->precision, lam[cur], h->tape_ckpt[0],
                            blob_phi(h, h->tape_ckpt[0]), dphi, dgrad, fd, partial_init, &nb,
                            h->stream);
    if (e == hipSuccess) e = launch_sum_partials(partial_init, nb, dsteps + 1, h->stream);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(h, e, "adjoint initialisation kernel");
    }
    if (h->kp.K == 3 && want_tau) {
      e = hipMemcpyAsync(&init_tau, dsteps + 1, sizeof(double), hipMemcpyDeviceToHost,
                         h->stream);
    }
  }
  if (want_wall && e == hipSuccess) {
    double* sums = partial_wall + wall_grad_partials();
    double host[2 * kMaxModes];
    e = launch_sum_wall_grad(partial_wall, sums, h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) {
      const int M = kp.field.nmodes;
      for (int j = 0; j < M; ++j) {
        dl_dwall_host[j] = host[j];
        dl_dwall_host[M + j] = kp.field.kind == kFieldCos ? host[kMaxModes + j] : 0.0;
      }
    }
  }
  if (want_tau && e == hipSuccess) {
    double dlds = 0.0;
    e = hipMemcpyAsync(&dlds, dsteps, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) {
      if (h->precision != LBM_FP32_SPLIT) dlds /= (1.0 - kp.s);
      // s = 1/tau
      *dl_dtau_host = -dlds / (kp.tau * kp.tau) + (at_init ? init_tau : 0.0);
    }
  }
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(h, e, "adjoint readback");
  }
  cleanup();
  return LBM_OK;
}

int lbm_equilibrium_weights(int d, const double* u, double g, int use_m4, double m4,
                            double* omega_out, double* m4_out, double* min_omega_out) {
  if (d < 1 || d > kMaxDim || !u || !omega_out)
    return fail(nullptr, LBM_EINVAL, "d must be in 1..4 and u, omega_out non-NULL");
  if (std::isnan(g)) g = 0.5;
  const double mm = (d >= 2) ? (use_m4 ? m4 : m4_interpolated(d, u, g)) : 0.0;
  omega_closed_form(d, u, mm, omega_out);
  double mn = omega_out[0];
  for (int k = 1; k < q_of(d); ++k) mn = std::fmin(mn, omega_out[k]);
  if (m4_out) *m4_out = mm;
  if (min_omega_out) *min_omega_out = mn;
  return LBM_OK;
}

int lbm_stability_map(int d, int64_t count, const double* sigma_dev, const double* s_dev,
                      double g, int32_t m, double* rho_dev, double* min_omega_dev,
                      int32_t* unconverged_dev, void* stream) {
  if (d < 1 || d > kMaxDim) return fail(nullptr, LBM_EINVAL, "d must be in 1..4");
  if (count < 0 || count > INT32_MAX) return fail(nullptr, LBM_EINVAL, "count out of range");
  if (m < 1 || m > (1 << 20)) return fail(nullptr, LBM_EINVAL, "m must be in 1..2^20");
  long long nxi = 1;
  for (int a = 0; a < d; ++a) {
    nxi *= m;
    if (nxi > (1LL << 31)) return fail(nullptr, LBM_EINVAL, "m^d must be <= 2^31");
  }
  if (std::isnan(g)) g = 0.5;
  if (!std::isfinite(g)) return fail(nullptr, LBM_EINVAL, "g must be finite");
  if (count == 0) return LBM_OK;
  if (!sigma_dev || !s_dev || !rho_dev)
    return fail(nullptr, LBM_EINVAL, "sigma, s and rho must not be null");
  hipError_t e = launch_stability(d, count, sigma_dev, s_dev, g, m, nxi, rho_dev, min_omega_dev,
                                  unconverged_dev, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "stability kernel");
  return LBM_OK;
}

const char* lbm_last_error(const lbm_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

int lbm_destroy(lbm_handle* h) {
  if (!h) return LBM_OK;
  (void)hipStreamSynchronize(h->stream);
  destroy_events(h);
  tape_clear(h);
  release(h);
  delete h;
  return LBM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct lbm_batch {
  std::vector<lbm_handle*> inst;
  int d = 0, precision = 0;
  hipStream_t stream = nullptr;
  lbm_handle* owner = nullptr;  // instance 0: its allocator serves the tables
  KParams* d_kps = nullptr;
  void** d_bufs = nullptr;
  BatchTile* d_tiles = nullptr;
  int max_tiles = 0, ntiles = 0;
  int tx = 64, ty = 4;
  // two-step passes (d = 2, every instance with steps_per_pass = 2)
  bool pairs = false;
  BatchTile2* d_tiles2 = nullptr;
  int ntiles2 = 0, tiles2_cap = 0;
  int ychunk = 0;                // rows per tile of the two-step passes
  int form = LBM_BATCH_PER_PAIR;  // launch form of the two-step passes
  int* d_first = nullptr;        // resident form: first tile of each instance (count + 1)
  int* d_order = nullptr;        // resident form: instances, largest first
  int cur = 0;
  int64_t step = 0;
  std::string err;
};

namespace {

int bfail(lbm_batch* b, int code, const std::string& msg) {
  if (b)
    b->err = msg;
  else
    g_create_error = msg;
  return code;
}

int batch_tiles(lbm_batch* b, int tx, int ty) {
  std::vector<BatchTile> t;
  for (size_t i = 0; i < b->inst.size(); ++i)
    for (int r = 0; r < b->inst[i]->kp.rows; r += ty) t.push_back(BatchTile{static_cast<int>(i), r});
  if (static_cast<int>(t.size()) > b->max_tiles) return bfail(b, LBM_EINVAL, "tile table overflow");
  hipError_t e = hipMemcpyAsync(b->d_tiles, t.data(), sizeof(BatchTile) * t.size(),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("tile upload: ") + hipGetErrorString(e));
  b->ntiles = static_cast<int>(t.size());
  b->tx = tx;
  b->ty = ty;
  return LBM_OK;
}

// Tile table of the two-step passes (d = 2): every instance cut into x_1
// tiles of the pass's width and chunks of yc rows; yc = 0 picks 64 rows,
// halved (down to 8) while the table has fewer than four tiles per CU.  Also
// each instance's first tile and the instances ordered by size, largest
// first (resident form).  The tables are allocated for the largest table
// (8 rows) on the first call.
int batch_pair_tiles(lbm_batch* b, int yc) {
  bool all = b->d == 2;
  for (lbm_handle* h : b->inst) all = all && h->steps_per_pass == 2;
  if (!all) return LBM_OK;
  const int tw = batch_pair_tile_width(b->precision);
  auto count = [&](int c) {
    long long n = 0;
    for (lbm_handle* h : b->inst)
      n += static_cast<long long>((h->kp.n[0] + tw - 1) / tw) * ((h->kp.n[1] + c - 1) / c);
    return n;
  };
  if (yc == 0) {
    yc = 64;
    while (yc > 8 && count(yc) < 4 * device_cus()) yc /= 2;
  }
  if (yc < 8 || yc > 64) return bfail(b, LBM_EINVAL, "row chunk must be in 8..64");
  const long long cap = count(8);
  if (cap > std::numeric_limits<int32_t>::max())
    return bfail(b, LBM_EINVAL, "too many tiles in the batch");
  if (!b->d_tiles2) {
    const int cnt = static_cast<int>(b->inst.size());
    b->d_tiles2 = static_cast<BatchTile2*>(dev_alloc(b->owner, sizeof(BatchTile2) * cap));
    b->d_first = static_cast<int*>(dev_alloc(b->owner, sizeof(int) * (cnt + 1)));
    b->d_order = static_cast<int*>(dev_alloc(b->owner, sizeof(int) * cnt));
    if (!b->d_tiles2 || !b->d_first || !b->d_order) return bfail(b, LBM_ENOMEM, "batch tables");
    b->tiles2_cap = static_cast<int>(cap);
  }
  std::vector<BatchTile2> t;
  std::vector<int> first(b->inst.size() + 1, 0), order(b->inst.size());
  t.reserve(static_cast<size_t>(count(yc)));
  for (size_t i = 0; i < b->inst.size(); ++i) {
    const KParams& kp = b->inst[i]->kp;
    first[i] = static_cast<int>(t.size());
    for (int y = 0; y < kp.n[1]; y += yc)
      for (int x = 0; x < kp.n[0]; x += tw)
        t.push_back(BatchTile2{static_cast<int>(i), x, y, std::min(y + yc, kp.n[1])});
  }
  first[b->inst.size()] = static_cast<int>(t.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return b->inst[x]->nodes > b->inst[y]->nodes;
  });
  hipError_t e = hipMemcpyAsync(b->d_tiles2, t.data(), sizeof(BatchTile2) * t.size(),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_first, first.data(), sizeof(int) * first.size(),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_order, order.data(), sizeof(int) * order.size(),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("tile upload: ") + hipGetErrorString(e));
  b->ntiles2 = static_cast<int>(t.size());
  b->ychunk = yc;
  b->pairs = true;
  return LBM_OK;
}

int batch_upload(lbm_batch* b) {
  std::vector<KParams> kps(b->inst.size());
  std::vector<void*> bufs(2 * b->inst.size());
  for (size_t i = 0; i < b->inst.size(); ++i) {
    kps[i] = b->inst[i]->kp;
    bufs[2 * i] = b->inst[i]->buf[0];
    bufs[2 * i + 1] = b->inst[i]->buf[1];
  }
  hipError_t e = hipMemcpyAsync(b->d_kps, kps.data(), sizeof(KParams) * kps.size(),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_bufs, bufs.data(), sizeof(void*) * bufs.size(), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
  return LBM_OK;
}

// Tuning results, keyed by the device (architecture name, CU count), the
// dimension, the storage mode and the instances' sizes: in memory for the
// process, and in the file named by LBM_TUNE_CACHE when it is set (one line
// per key: FNV-1a hash of the key, form, row chunk, tx, ty, ms per step).
struct TuneEntry {
  int form = LBM_BATCH_PER_PAIR, ychunk = 0, tx = 64, ty = 4;
  double ms = 0.0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune_mem;
std::map<uint64_t, TuneEntry> g_tune_file;
bool g_tune_file_read = false;

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string tune_key(const lbm_batch* b) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  std::string k = arch + ";cus=" + std::to_string(device_cus()) + ";d=" + std::to_string(b->d) +
                  ";prec=" + std::to_string(b->precision) + ";dims=";
  for (const lbm_handle* h : b->inst) {
    for (int a = 0; a < b->d; ++a) k += std::to_string(h->dims[a]) + (a + 1 < b->d ? "x" : ",");
  }
  return k;
}

// the single-step block shapes (tx, ty) the tuner times
constexpr int kTuneShapes[3][2] = {{64, 4}, {128, 2}, {256, 1}};

// An entry is used only if it names a launch the tuner itself could have
// chosen: a file written by another build, edited or cut short could
// otherwise set a zero row step or a block the kernels were not built for.
bool tune_entry_valid(const TuneEntry& e) {
  const bool form = e.form == LBM_BATCH_PER_PAIR || e.form == LBM_BATCH_RESIDENT;
  const bool rows = e.ychunk == 0 || (e.ychunk >= 8 && e.ychunk <= 64);
  bool shape = false;
  for (const auto& sh : kTuneShapes) shape = shape || (e.tx == sh[0] && e.ty == sh[1]);
  return form && rows && shape && std::isfinite(e.ms) && e.ms >= 0.0;
}

// Lines that do not parse, or whose entry is not valid, are skipped.
void tune_file_load() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("LBM_TUNE_CACHE");
  if (!path || !*path) return;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    unsigned long long hash = 0;
    TuneEntry e;
    if (std::sscanf(line, "%llx %d %d %d %d %lf", &hash, &e.form, &e.ychunk, &e.tx, &e.ty,
                    &e.ms) == 6 &&
        tune_entry_valid(e))
      g_tune_file[hash] = e;
  }
  std::fclose(f);
}

bool tune_cache_get(const std::string& key, TuneEntry* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_mem.find(key);
  if (it != g_tune_mem.end()) {
    *out = it->second;
    return true;
  }
  tune_file_load();
  auto jt = g_tune_file.find(fnv1a(key));
  if (jt == g_tune_file.end()) return false;
  *out = jt->second;
  g_tune_mem[key] = jt->second;
  return true;
}

void tune_cache_put(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_mem[key] = e;
  const char* path = std::getenv("LBM_TUNE_CACHE");
  if (!path || !*path) return;
  if (std::FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%016llx %d %d %d %d %.6f\n", static_cast<unsigned long long>(fnv1a(key)),
                 e.form, e.ychunk, e.tx, e.ty, e.ms);
    std::fclose(f);
  }
}

int batch_run(lbm_batch* b, int64_t n, bool allow_pairs = true) {
  if (n <= 0) return LBM_OK;
  int64_t done = 0;
  if (allow_pairs && b->pairs && b->form == LBM_BATCH_RESIDENT && n >= 2) {
    // every pair of steps of the call in one launch, one block per instance
    for (int64_t np = n / 2; np > 0;) {
      const int chunk = static_cast<int>(std::min<int64_t>(np, 1 << 30));
      hipError_t e = launch_batch_resident(b->d_kps, b->d_bufs, b->d_tiles2, b->d_first,
                                           b->d_order, static_cast<int>(b->inst.size()),
                                           b->precision, b->cur, chunk, b->stream);
      if (e != hipSuccess)
        return bfail(b, LBM_EDEVICE, std::string("resident batch pass: ") + hipGetErrorString(e));
      b->cur = (b->cur + chunk) & 1;
      np -= chunk;
      done += 2 * static_cast<int64_t>(chunk);
    }
  } else if (allow_pairs && b->pairs) {
    for (int64_t np = n / 2; np > 0;) {
      const int chunk = static_cast<int>(std::min<int64_t>(np, 1 << 20));
      hipError_t e = launch_batch_pair(b->d_kps, b->d_bufs, b->d_tiles2, b->ntiles2,
                                       b->precision, b->cur, chunk, b->stream);
      if (e != hipSuccess)
        return bfail(b, LBM_EDEVICE, std::string("batch two-step pass: ") + hipGetErrorString(e));
      b->cur = (b->cur + chunk) & 1;
      np -= chunk;
      done += 2 * static_cast<int64_t>(chunk);
    }
  }
  while (done < n) {
    const int chunk = static_cast<int>(std::min<int64_t>(n - done, 1 << 20));
    hipError_t e = launch_batch(b->d, b->d_kps, b->d_bufs, b->d_tiles, b->ntiles, b->tx, b->ty,
                                b->precision, b->cur, chunk, b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch step: ") + hipGetErrorString(e));
    b->cur = (b->cur + chunk) & 1;
    done += chunk;
  }
  b->step += n;
  for (lbm_handle* h : b->inst) {
    h->cur = b->cur;
    h->step = b->step;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_create(int count, int d, const int64_t* dims, const double* tau,
                     const lbm_params* params, lbm_batch** out) {
  if (out) *out = nullptr;
  if (!out || !dims || !tau || !params || count < 1)
    return bfail(nullptr, LBM_EINVAL, "null argument or count < 1");
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return bfail(nullptr, LBM_ENOMEM, "host allocation failed");
  b->d = d;
  b->precision = params[0].precision;
  b->stream = static_cast<hipStream_t>(params[0].stream);
  auto abort_create = [&](int rc) {
    std::string msg = g_create_error;
    for (lbm_handle* h : b->inst) lbm_destroy(h);
    if (b->owner) {
      dev_free(b->owner, b->d_kps);
      dev_free(b->owner, b->d_bufs);
      dev_free(b->owner, b->d_tiles);
      dev_free(b->owner, b->d_tiles2);
      dev_free(b->owner, b->d_first);
      dev_free(b->owner, b->d_order);
    }
    delete b;
    g_create_error = msg;
    return rc;
  };
  int64_t total_rows = 0;
  for (int i = 0; i < count; ++i) {
    if (params[i].precision != b->precision || params[i].stream != params[0].stream)
      return abort_create(bfail(nullptr, LBM_EINVAL, "batch instances need one precision and one stream"));
    if (split_mode(params[i].precision))
      return abort_create(bfail(nullptr, LBM_EUNSUPPORTED, "batches support LBM_FP64 and LBM_FP32"));
    for (int a = 0; a < d; ++a)
      if (params[i].bc[a][0] != LBM_BC_PERIODIC || params[i].bc[a][1] != LBM_BC_PERIODIC)
        return abort_create(bfail(nullptr, LBM_EUNSUPPORTED, "batch instances must be periodic"));
    lbm_handle* h = nullptr;
    int rc = lbm_create(d, dims + static_cast<size_t>(i) * d, tau[i], &params[i], &h);
    if (rc != LBM_OK) return abort_create(rc);
    h->batch_member = true;
    b->inst.push_back(h);
    total_rows += h->kp.rows;
  }
  b->owner = b->inst[0];
  if (total_rows > std::numeric_limits<int32_t>::max())
    return abort_create(bfail(nullptr, LBM_EINVAL, "too many rows in the batch"));
  b->max_tiles = static_cast<int>(total_rows);
  b->d_kps = static_cast<KParams*>(dev_alloc(b->owner, sizeof(KParams) * count));
  b->d_bufs = static_cast<void**>(dev_alloc(b->owner, sizeof(void*) * 2 * count));
  b->d_tiles = static_cast<BatchTile*>(dev_alloc(b->owner, sizeof(BatchTile) * b->max_tiles));
  if (!b->d_kps || !b->d_bufs || !b->d_tiles)
    return abort_create(bfail(nullptr, LBM_ENOMEM, "batch tables"));
  int rc = batch_upload(b);
  if (rc == LBM_OK) rc = batch_tiles(b, 64, 4);
  if (rc == LBM_OK) rc = batch_pair_tiles(b, 0);
  if (rc != LBM_OK) {
    g_create_error = b->err;
    return abort_create(rc);
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_set_initial(lbm_batch* b, const double* phi0_dev, const double* grad_dev) {
  if (!b || !phi0_dev) return bfail(b, LBM_EINVAL, "null argument");
  int64_t off = 0;
  for (lbm_handle* h : b->inst) {
    int rc = lbm_set_initial(h, phi0_dev + off, grad_dev ? grad_dev + off * b->d : nullptr);
    if (rc != LBM_OK) return bfail(b, rc, h->err);
    off += h->nodes;
  }
  b->cur = 0;
  b->step = 0;
  return batch_upload(b);  // float32 references may have changed
}

int lbm_batch_step(lbm_batch* b, int64_t n) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "null batch");
  if (n < 0) return bfail(b, LBM_EINVAL, "n must be >= 0");
  for (lbm_handle* h : b->inst)
    if (!h->initialised) return bfail(b, LBM_EINVAL, "an instance has no initial state");
  return batch_run(b, n);
}

int lbm_batch_set_launch(lbm_batch* b, int form, int ychunk) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "null batch");
  if (form != LBM_BATCH_PER_PAIR && form != LBM_BATCH_RESIDENT)
    return bfail(b, LBM_EINVAL, "unknown launch form");
  if (ychunk != 0 && (ychunk < 8 || ychunk > 64))
    return bfail(b, LBM_EINVAL, "row chunk must be 0 or in 8..64");
  if (!b->pairs) return bfail(b, LBM_EUNSUPPORTED, "the batch does not use two-step passes");
  int rc = batch_pair_tiles(b, ychunk);
  if (rc != LBM_OK) return rc;
  b->form = form;
  return LBM_OK;
}

int lbm_batch_tune(lbm_batch* b, int trial_steps, int32_t* config_out, double* ms_per_step_out) {
  if (!b) return bfail(nullptr, LBM_EINVAL, "null batch");
  if (trial_steps < 1) return bfail(b, LBM_EINVAL, "trial_steps must be >= 1");
  for (lbm_handle* h : b->inst)
    if (!h->initialised) return bfail(b, LBM_EINVAL, "an instance has no initial state");
  const std::string key = tune_key(b);
  TuneEntry best;
  bool cached = tune_cache_get(key, &best);
  int rc = LBM_OK;
  if (!cached) {
    // keep the states: trials advance the lattices
    std::vector<void*> saved;
    auto cleanup = [&]() {
      (void)hipStreamSynchronize(b->stream);
      for (size_t i = 0; i < saved.size(); ++i) dev_free(b->inst[i], saved[i]);
    };
    for (lbm_handle* h : b->inst) {
      void* st = dev_alloc(h, state_bytes(h));
      if (!st) {
        cleanup();
        return bfail(b, LBM_ENOMEM, "tuning buffers");
      }
      saved.push_back(st);
      if (copy_state_out(h, st) != hipSuccess) {
        cleanup();
        return bfail(b, LBM_EDEVICE, "tuning state copy");
      }
    }
    const int cur0 = b->cur;
    const int64_t step0 = b->step;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      cleanup();
      return bfail(b, LBM_EDEVICE, "hipEventCreate");
    }
    // one trial: warm-up steps, then `steps` timed steps; ms per step
    auto trial = [&](int64_t steps, bool pairs, double* ms) -> int {
      int r = batch_run(b, pairs ? 2 : 1, pairs);
      if (r != LBM_OK) return r;
      (void)hipEventRecord(e0, b->stream);
      r = batch_run(b, steps, pairs);
      (void)hipEventRecord(e1, b->stream);
      if (r != LBM_OK) return r;
      if (hipEventSynchronize(e1) != hipSuccess) return bfail(b, LBM_EDEVICE, "tuning run");
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, e0, e1);
      *ms = t / static_cast<double>(steps);
      return LBM_OK;
    };
    // single-step block shapes (remainder steps, batches without pairs)
    double best_single = 1e300;
    for (const auto& sh : kTuneShapes) {
      rc = batch_tiles(b, sh[0], sh[1]);
      double ms = 0.0;
      if (rc == LBM_OK) rc = trial(trial_steps, false, &ms);
      if (rc != LBM_OK) break;
      if (ms < best_single) {
        best_single = ms;
        best.tx = sh[0];
        best.ty = sh[1];
        best.ms = ms;
      }
    }
    // launch forms and row chunks of the two-step passes
    if (rc == LBM_OK && b->pairs) {
      const int64_t steps2 = std::max<int64_t>(2, trial_steps + (trial_steps & 1));
      double best_pair = 1e300;
      for (int form : {LBM_BATCH_PER_PAIR, LBM_BATCH_RESIDENT}) {
        for (int yc : {8, 16, 32, 64}) {
          rc = batch_pair_tiles(b, yc);
          b->form = form;
          double ms = 0.0;
          if (rc == LBM_OK) rc = trial(steps2, true, &ms);
          if (rc != LBM_OK) break;
          if (ms < best_pair) {
            best_pair = ms;
            best.form = form;
            best.ychunk = yc;
            best.ms = ms;
          }
        }
        if (rc != LBM_OK) break;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // restore the states and the step counters
    for (size_t i = 0; i < b->inst.size() && rc == LBM_OK; ++i) {
      lbm_handle* h = b->inst[i];
      h->cur = cur0;
      if (set_state_impl(h, saved[i], step0) != LBM_OK) rc = bfail(b, LBM_EDEVICE, h->err);
    }
    b->cur = cur0;
    b->step = step0;
    cleanup();
    if (rc != LBM_OK) return rc;
    for (lbm_handle* h : b->inst) h->init_kind = 0;
    tune_cache_put(key, best);
  }
  rc = batch_tiles(b, best.tx, best.ty);
  if (rc == LBM_OK && b->pairs) {
    rc = batch_pair_tiles(b, best.ychunk);
    b->form = best.form;
  }
  if (rc != LBM_OK) return rc;
  if (config_out) {
    config_out[0] = b->pairs ? best.form : -1;
    config_out[1] = b->pairs ? best.ychunk : 0;
    config_out[2] = best.tx;
    config_out[3] = best.ty;
    config_out[4] = cached ? 1 : 0;
  }
  if (ms_per_step_out) *ms_per_step_out = best.ms;
  return LBM_OK;
}

lbm_handle* lbm_batch_instance(const lbm_batch* b, int i) {
  if (!b || i < 0 || i >= static_cast<int>(b->inst.size())) return nullptr;
  return b->inst[i];
}

int lbm_batch_moments(lbm_batch* b, double* scalars_host) {
  if (!b || !scalars_host) return bfail(b, LBM_EINVAL, "null argument");
  for (size_t i = 0; i < b->inst.size(); ++i) {
    int rc = lbm_moments(b->inst[i], LBM_MOM_SUMS | LBM_MOM_RMSE | LBM_MOM_ENTROPY, nullptr,
                         scalars_host + i * LBM_NSCALARS);
    if (rc != LBM_OK) return bfail(b, rc, b->inst[i]->err);
  }
  return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->owner) {
    dev_free(b->owner, b->d_kps);
    dev_free(b->owner, b->d_bufs);
    dev_free(b->owner, b->d_tiles);
    dev_free(b->owner, b->d_tiles2);
    dev_free(b->owner, b->d_first);
    dev_free(b->owner, b->d_order);
  }
  for (lbm_handle* h : b->inst) lbm_destroy(h);
  delete b;
  return LBM_OK;
}

}  // extern "C"
