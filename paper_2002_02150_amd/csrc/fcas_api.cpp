// fcas_api.cpp -- the C ABI (include/fcas.h): argument validation on the
// host, the context (network, tables, workspace), the segment registry and the
// launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fcas.h"
#include "grad_kernels.hpp"
#include "launch.hpp"
#include "pso_kernels.hpp"

using namespace fcas;

namespace {

constexpr int kDefaultGrid = 2048;   // persistent work-groups of a pass launch unless tuned

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FCAS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct TimedPair {
  hipEvent_t a, b;
};

// Device memory of fitness_eval_batch_static: point descriptors, work lists,
// pass-2 partials and FFT workspace of one call, in a fixed array that every
// GPU the library runs on holds until the process ends.  Host code never uses
// the array's name as an address: scratch_for_device() looks up each device's
// copy once, with that device current, and keeps the pointer.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (which must be current).
int scratch_for_device(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(FCAS_EINVAL, "device %d beyond the library's table", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return FCAS_OK;
}

}  // namespace

struct fcas_ctx {
  int device = 0;
  fcas_network net{};
  fcas_config cfg{};
  int prec = 0;          // 0 float, 1 double
  size_t elt = 8;        // bytes of one complex element of the FFT path
  NetDesc h_net{};
  NetDesc* d_net = nullptr;
  std::vector<SegDesc> h_segs;
  SegDesc* d_segs = nullptr;
  std::vector<void*> seg_y;
  std::vector<double*> seg_b;
  EvalDesc* d_evals = nullptr;
  int32_t* d_lists = nullptr;    // [kNumPlans][max_batch]
  int32_t* d_counts = nullptr;   // [kNumPlans]
  int32_t* d_lists2 = nullptr;   // second work-list set of pso_run (iterations alternate between the two)
  int32_t* d_counts2 = nullptr;
  void* d_part_g = nullptr;      // [max_batch][part_stride]
  int32_t* d_part_j = nullptr;
  int32_t* d_plan_parts2 = nullptr;
  int part_stride = 1;           // pass-2 partials per point: the most any admitted plan leaves
  int32_t* d_err = nullptr;
  unsigned long long* d_evaluated = nullptr;   // running total of points evaluated
  double* d_sigma2 = nullptr;    // [FCAS_MAX_DET] scratch for segment registration
  double* d_inject = nullptr;    // [kInjectScratch] partial sums of fcas_inject
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  void* d_scratch = nullptr;     // this device's copy of the static scratch array (not owned)
  GradBuffers grad{};
  double* d_pol_grad = nullptr;    // [max_batch][4] polish: gradient at the current points
  double* d_pol_cand = nullptr;    // [max_batch][4] polish trials
  int32_t* d_pol_seg = nullptr;    // [max_batch]
  double* d_pol_f = nullptr;       // [max_batch]
  int32_t* d_pol_j = nullptr;      // [max_batch]
  int plan_refs[kNumPlans] = {0};   // registered segments per plan
  int schedule = FCAS_SCHEDULE_FUSED;
  int n_cu = 0;                     // compute units of the device
  int fused_cap[kNumPlans] = {0};   // resident work-groups of each fused kernel (0 = not queried)
  int32_t* d_done = nullptr;        // [kNumPlans][2][max_batch] fused-schedule tile counters
  bool timing = false;
  std::vector<TimedPair> t_pass1, t_passm, t_pass2, t_fused;
  int grid1[kNumPlans], grid2[kNumPlans];   // persistent grid sizes of the two passes
  int chosen[kNumPlans];                     // plan used for new segments of each length (by default plan)
};

namespace {

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// In-band bins f_* < k/T <= min(f_high, fs/2), 1 <= k < N/2.
void band(const fcas_config& c, int64_t n, int* k_lo, int* k_hi) {
  const double T = (double)n / c.fs_hz;
  const int64_t lo = (int64_t)std::floor(c.f_low_hz * T) + 1;
  int64_t hi = (int64_t)std::floor(c.f_high_hz * T);
  if (hi > n / 2 - 1) hi = n / 2 - 1;
  *k_lo = (int)lo;
  *k_hi = (int)hi;
}

int validate_network(const fcas_network* net) {
  if (!net) return fail(FCAS_EINVAL, "network is NULL");
  if (net->n_det < 1 || net->n_det > FCAS_MAX_DET)
    return fail(FCAS_EINVAL, "n_det must be in [1, %d], got %d", FCAS_MAX_DET, net->n_det);
  for (int i = 0; i < net->n_det; ++i) {
    if (!finite_all(net->pos_m[i], 3) || !finite_all(&net->tensor[i][0][0], 9))
      return fail(FCAS_EINVAL, "detector %d has a non-finite position or tensor", i);
  }
  return FCAS_OK;
}

int validate_config(const fcas_config* c) {
  if (!c) return fail(FCAS_EINVAL, "config is NULL");
  if (!(c->fs_hz > 0) || !std::isfinite(c->fs_hz)) return fail(FCAS_EINVAL, "fs_hz must be positive");
  if (!(c->f_low_hz > 0) || !(c->f_high_hz > c->f_low_hz) || !std::isfinite(c->f_high_hz))
    return fail(FCAS_EINVAL, "need 0 < f_low_hz < f_high_hz");
  if (c->precision != FCAS_MIXED && c->precision != FCAS_FP64)
    return fail(FCAS_EINVAL, "precision must be FCAS_MIXED or FCAS_FP64");
  if (c->max_batch < 1 || c->max_batch > (1 << 24)) return fail(FCAS_EINVAL, "max_batch must be in [1, 2^24]");
  if (c->max_segments < 1 || c->max_segments > (1 << 20))
    return fail(FCAS_EINVAL, "max_segments must be in [1, 2^20]");
  if (plan_for_length(c->max_samples) < 0)
    return fail(FCAS_EUNSUPPORTED_N, "max_samples %lld has no FFT plan", (long long)c->max_samples);
  if (c->workspace_bytes < 0) return fail(FCAS_EINVAL, "workspace_bytes must be >= 0");
  if (c->schedule != FCAS_SCHEDULE_FUSED && c->schedule != FCAS_SCHEDULE_TWO_PASS)
    return fail(FCAS_EINVAL, "schedule must be FCAS_SCHEDULE_FUSED or FCAS_SCHEDULE_TWO_PASS");
  for (int d = 0; d < 4; ++d) {
    if (!std::isfinite(c->box_lo[d]) || !std::isfinite(c->box_hi[d]) || !(c->box_hi[d] >= c->box_lo[d]))
      return fail(FCAS_EINVAL, "search box coordinate %d must satisfy lo <= hi (finite)", d);
  }
  if (!(c->box_lo[2] > 0) || !(c->box_lo[3] > 0)) return fail(FCAS_EINVAL, "chirp times must be positive");
  return FCAS_OK;
}

int validate_batch(const fcas_ctx* ctx, int32_t n, const void* theta, const void* seg, const void* f,
                   const void* j) {
  if (!ctx) return fail(FCAS_EINVAL, "context is NULL");
  if (n < 0) return fail(FCAS_EINVAL, "n must be >= 0, got %d", n);
  if (n > ctx->cfg.max_batch)
    return fail(FCAS_ECAPACITY, "n = %d exceeds max_batch = %d", n, ctx->cfg.max_batch);
  if (n > 0 && (!theta || !seg || !f || !j)) return fail(FCAS_EINVAL, "NULL device pointer");
  return FCAS_OK;
}

int free_all(fcas_ctx* c) {
  for (void* p : c->seg_y) if (p) hipFree(p);
  for (double* p : c->seg_b) if (p) hipFree(p);
  void* bufs[] = {c->d_net, c->d_segs, c->d_evals, c->d_lists, c->d_counts, c->d_part_g,
                  c->d_part_j, c->d_plan_parts2, c->d_err, c->d_sigma2, c->d_inject, c->d_ws,
                  c->d_pol_grad, c->d_pol_cand, c->d_pol_seg, c->d_pol_f, c->d_pol_j, c->d_evaluated,
                  c->d_done, c->d_lists2, c->d_counts2};
  for (void* p : bufs) if (p) hipFree(p);
  free_grad_buffers(c->grad);
  for (auto& t : c->t_pass1) { hipEventDestroy(t.a); hipEventDestroy(t.b); }
  for (auto& t : c->t_passm) { hipEventDestroy(t.a); hipEventDestroy(t.b); }
  for (auto& t : c->t_pass2) { hipEventDestroy(t.a); hipEventDestroy(t.b); }
  for (auto& t : c->t_fused) { hipEventDestroy(t.a); hipEventDestroy(t.b); }
  return FCAS_OK;
}

template <typename T>
int dev_alloc(T** p, size_t bytes) {
  hipError_t e = hipMalloc((void**)p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(FCAS_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return FCAS_OK;
}

}  // namespace

extern "C" {

const char* fcas_last_error(void) { return g_last_error.c_str(); }

int fcas_supported_n(int64_t n_samples) { return plan_for_length(n_samples) >= 0 ? 1 : 0; }

int fcas_plan_count(void) { return kNumPlans; }

int fcas_plan_info(int32_t plan, int64_t* n_samples, int32_t* n1, int32_t* n2, int32_t* e1, int32_t* e2,
                   int32_t* cols, int32_t* rows) {
  if (plan < 0 || plan >= kNumPlans) return fail(FCAS_EINVAL, "plan %d out of range [0, %d)", plan, kNumPlans);
  const PlanInfo& pi = kPlans[plan];
  if (n_samples) *n_samples = pi.n;
  if (n1) *n1 = pi.n1;
  if (n2) *n2 = pi.n2;
  if (e1) *e1 = pi.e1;
  if (e2) *e2 = pi.e2;
  if (cols) *cols = pi.cols[0];
  if (rows) *rows = pi.rows[0];
  return FCAS_OK;
}

int fcas_select_plan(fcas_ctx* ctx, int32_t plan, int32_t grid1, int32_t grid2) {
  if (!ctx) return fail(FCAS_EINVAL, "context is NULL");
  if (plan < 0 || plan >= kNumPlans) return fail(FCAS_EINVAL, "plan %d out of range [0, %d)", plan, kNumPlans);
  if (grid1 < 0 || grid2 < 0 || grid1 > (1 << 20) || grid2 > (1 << 20))
    return fail(FCAS_EINVAL, "grid sizes must be in [0, 2^20]");
  ctx->chosen[plan_for_length(kPlans[plan].n)] = plan;
  ctx->grid1[plan] = grid1 > 0 ? grid1 : kDefaultGrid;
  ctx->grid2[plan] = grid2 > 0 ? grid2 : kDefaultGrid;
  return FCAS_OK;
}

int fcas_create(const fcas_network* net, const fcas_config* cfg, int device, fcas_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(FCAS_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_network(net);
  if (rc) return rc;
  rc = validate_config(cfg);
  if (rc) return rc;
  {
    int k_lo, k_hi;
    band(*cfg, cfg->max_samples, &k_lo, &k_hi);
    if (k_lo > k_hi) return fail(FCAS_EINVAL, "empty band at max_samples");
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return fail(FCAS_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(FCAS_EINVAL, "device %d out of range [0, %d)", device, ndev);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

  fcas_ctx* c = new fcas_ctx();
  c->device = device;
  c->net = *net;
  c->cfg = *cfg;
  c->prec = cfg->precision == FCAS_FP64 ? 1 : 0;
  for (int i = 0; i < kNumPlans; ++i) {
    c->grid1[i] = c->grid2[i] = kDefaultGrid;
    c->chosen[i] = i;
  }
  c->schedule = c->prec == 0 ? cfg->schedule : FCAS_SCHEDULE_TWO_PASS;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1)
    c->n_cu = 1;
  c->elt = c->prec ? 16 : 8;
  NetDesc& h = c->h_net;
  h.n_det = net->n_det;
  h.max_segments = cfg->max_segments;
  std::memcpy(h.pos, net->pos_m, sizeof h.pos);
  std::memcpy(h.ten, net->tensor, sizeof h.ten);
  std::memcpy(h.box_lo, cfg->box_lo, sizeof h.box_lo);
  std::memcpy(h.box_hi, cfg->box_hi, sizeof h.box_hi);
  h.f_star = cfg->f_low_hz;
  const int B = cfg->max_batch;
  const size_t slot_bytes = 2 * (size_t)cfg->max_samples * c->elt;
  size_t ws = cfg->workspace_bytes > 0 ? (size_t)cfg->workspace_bytes : (size_t)B * slot_bytes;
  const size_t ws_default_cap = (size_t)8 << 30;
  if (cfg->workspace_bytes == 0 && ws > ws_default_cap) ws = ws_default_cap;
  if (ws < slot_bytes) {
    delete c;
    return fail(FCAS_EINVAL, "workspace_bytes %zu below one evaluation (%zu)", ws, slot_bytes);
  }
  c->ws_bytes = ws;
  c->h_segs.assign(cfg->max_segments, SegDesc{});
  c->seg_y.assign(cfg->max_segments, nullptr);
  c->seg_b.assign(cfg->max_segments, nullptr);
  const size_t part_elt = c->prec ? 8 : 4;
  for (int i = 0; i < kNumPlans; ++i)
    if (kPlans[i].n <= cfg->max_samples) c->part_stride = std::max(c->part_stride, kPlans[i].parts2[c->prec]);
  if ((rc = dev_alloc(&c->d_net, sizeof(NetDesc))) || (rc = dev_alloc(&c->d_segs, sizeof(SegDesc) * cfg->max_segments)) ||
      (rc = dev_alloc(&c->d_evals, sizeof(EvalDesc) * B)) ||
      (rc = dev_alloc(&c->d_lists, sizeof(int32_t) * (size_t)kNumPlans * B)) ||
      (rc = dev_alloc(&c->d_counts, sizeof(int32_t) * kNumPlans)) ||
      (rc = dev_alloc(&c->d_lists2, sizeof(int32_t) * (size_t)kNumPlans * B)) ||
      (rc = dev_alloc(&c->d_counts2, sizeof(int32_t) * kNumPlans)) ||
      (rc = dev_alloc(&c->d_part_g, part_elt * (size_t)B * c->part_stride)) ||
      (rc = dev_alloc(&c->d_part_j, sizeof(int32_t) * (size_t)B * c->part_stride)) ||
      (rc = dev_alloc(&c->d_plan_parts2, sizeof(int32_t) * kNumPlans)) ||
      (rc = dev_alloc(&c->d_err, sizeof(int32_t))) || (rc = dev_alloc(&c->d_sigma2, sizeof(double) * FCAS_MAX_DET)) ||
      (rc = dev_alloc(&c->d_inject, sizeof(double) * kInjectScratch)) ||
      (rc = dev_alloc(&c->d_ws, ws)) || (rc = alloc_grad_buffers(c->grad, B, net->n_det)) ||
      (rc = dev_alloc(&c->d_pol_grad, sizeof(double) * 4 * B)) ||
      (rc = dev_alloc(&c->d_pol_cand, sizeof(double) * 4 * B)) ||
      (rc = dev_alloc(&c->d_pol_seg, sizeof(int32_t) * B)) || (rc = dev_alloc(&c->d_pol_f, sizeof(double) * B)) ||
      (rc = dev_alloc(&c->d_pol_j, sizeof(int32_t) * B)) ||
      (rc = dev_alloc(&c->d_evaluated, sizeof(unsigned long long))) ||
      (rc = dev_alloc(&c->d_done, sizeof(int32_t) * 2 * (size_t)kNumPlans * B))) {
    std::string msg = g_last_error;
    free_all(c);
    delete c;
    g_last_error = msg;
    return rc;
  }
  if ((rc = scratch_for_device(device, &c->d_scratch))) {
    std::string msg = g_last_error;
    free_all(c);
    delete c;
    g_last_error = msg;
    return rc;
  }
  int32_t parts2[kNumPlans];
  for (int i = 0; i < kNumPlans; ++i) parts2[i] = kPlans[i].parts2[c->prec];
  if ((e = hipMemcpy(c->d_net, &h, sizeof(NetDesc), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_segs, c->h_segs.data(), sizeof(SegDesc) * cfg->max_segments, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(c->d_plan_parts2, parts2, sizeof parts2, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(c->d_err, 0, sizeof(int32_t))) != hipSuccess ||
      (e = hipMemset(c->d_evaluated, 0, sizeof(unsigned long long))) != hipSuccess ||
      (e = hipMemset(c->d_counts, 0, sizeof(int32_t) * kNumPlans)) != hipSuccess ||
      (e = hipMemset(c->d_counts2, 0, sizeof(int32_t) * kNumPlans)) != hipSuccess) {
    rc = hip_fail(e, "context initialisation");
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return FCAS_OK;
}

int fcas_destroy(fcas_ctx* ctx) {
  if (!ctx) return fail(FCAS_EINVAL, "context is NULL");
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  free_all(ctx);
  delete ctx;
  return FCAS_OK;
}

size_t fcas_workspace_bytes(const fcas_ctx* ctx) { return ctx ? ctx->ws_bytes : 0; }

int fcas_set_segment(fcas_ctx* ctx, int32_t seg_id, int64_t n_samples, const double* d_xf, const double* d_psd,
                     void* hip_stream) {
  if (!ctx) return fail(FCAS_EINVAL, "context is NULL");
  if (seg_id < 0 || seg_id >= ctx->cfg.max_segments)
    return fail(FCAS_ENOSEG, "segment id %d out of range [0, %d)", seg_id, ctx->cfg.max_segments);
  const int default_plan = plan_for_length(n_samples);
  if (default_plan < 0)
    return fail(FCAS_EUNSUPPORTED_N, "segment length %lld has no FFT plan", (long long)n_samples);
  const int plan = ctx->chosen[default_plan];
  if (n_samples > ctx->cfg.max_samples)
    return fail(FCAS_EINVAL, "segment length %lld exceeds max_samples %lld", (long long)n_samples,
                (long long)ctx->cfg.max_samples);
  if (!d_xf || !d_psd) return fail(FCAS_EINVAL, "NULL device pointer");
  int k_lo, k_hi;
  band(ctx->cfg, n_samples, &k_lo, &k_hi);
  if (k_lo > k_hi) return fail(FCAS_EINVAL, "empty band for %lld samples", (long long)n_samples);
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const int D = ctx->net.n_det;
  const int K = k_hi - k_lo + 1;
  const int64_t half = n_samples / 2 + 1;
  const double df = ctx->cfg.fs_hz / (double)n_samples;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  // A re-registered segment replaces the old one: its buffers are freed and
  // the device descriptor is cleared first, so that if any later step fails
  // the id is left unregistered (evaluations then report it as a bad
  // segment) rather than pointing at freed memory.
  if (ctx->seg_y[seg_id]) {
    const SegDesc empty{};
    if ((e = hipMemcpy(ctx->d_segs + seg_id, &empty, sizeof empty, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "segment descriptor upload");
    hipFree(ctx->seg_y[seg_id]);
    hipFree(ctx->seg_b[seg_id]);
    ctx->seg_y[seg_id] = nullptr;
    ctx->seg_b[seg_id] = nullptr;
    ctx->plan_refs[ctx->h_segs[seg_id].plan]--;
    ctx->h_segs[seg_id] = SegDesc{};
  }
  void* y = nullptr;
  double* b = nullptr;
  int rc;
  if ((rc = dev_alloc(&y, (size_t)K * D * ctx->elt))) return rc;
  if ((rc = dev_alloc(&b, (size_t)K * sizeof(double)))) {
    hipFree(y);
    return rc;
  }
  if ((e = launch_segment_sigma(d_psd, D, half, k_lo, k_hi, df, ctx->d_sigma2, s)) != hipSuccess ||
      (e = launch_segment_prep(ctx->prec, d_xf, d_psd, ctx->d_sigma2, D, half, k_lo, k_hi, df, ctx->cfg.f_low_hz, y,
                               b, s)) != hipSuccess) {
    hipFree(y);
    hipFree(b);
    return hip_fail(e, "segment preparation launch");
  }
  double sigma2[FCAS_MAX_DET];
  if ((e = hipMemcpyAsync(sigma2, ctx->d_sigma2, sizeof(double) * D, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    hipFree(y);
    hipFree(b);
    return hip_fail(e, "segment preparation");
  }
  SegDesc sd{};
  sd.y = y;
  sd.b = b;
  sd.n = n_samples;
  sd.k_lo = k_lo;
  sd.k_hi = k_hi;
  sd.plan = plan;
  sd.registered = 1;
  sd.dk1 = (int32_t)(kPlans[plan].n / kPlans[plan].e1);
  sd.df = df;
  sd.j_lo = 0;
  sd.j_hi = n_samples;
  for (int i = 0; i < D; ++i) {
    if (!(sigma2[i] > 0) || !std::isfinite(sigma2[i])) {
      hipFree(y);
      hipFree(b);
      return fail(FCAS_EINVAL, "template norm of detector %d is not positive and finite (check the PSD)", i);
    }
    sd.sigma[i] = std::sqrt(sigma2[i]);
  }
  if ((e = hipMemcpy(ctx->d_segs + seg_id, &sd, sizeof sd, hipMemcpyHostToDevice)) != hipSuccess) {
    hipFree(y);
    hipFree(b);
    return hip_fail(e, "segment descriptor upload");
  }
  ctx->h_segs[seg_id] = sd;
  ctx->seg_y[seg_id] = y;
  ctx->seg_b[seg_id] = b;
  ctx->plan_refs[plan]++;
  return FCAS_OK;
}

int fcas_set_segment_range(fcas_ctx* ctx, int32_t seg_id, int64_t j_lo, int64_t j_hi) {
  if (!ctx) return fail(FCAS_EINVAL, "context is NULL");
  if (seg_id < 0 || seg_id >= ctx->cfg.max_segments)
    return fail(FCAS_ENOSEG, "segment id %d out of range [0, %d)", seg_id, ctx->cfg.max_segments);
  SegDesc& sd = ctx->h_segs[seg_id];
  if (!sd.registered) return fail(FCAS_ENOSEG, "segment %d is not registered", seg_id);
  if (j_lo < 0 || j_hi > sd.n || j_lo >= j_hi)
    return fail(FCAS_EINVAL, "need 0 <= j_lo < j_hi <= %lld, got [%lld, %lld)", (long long)sd.n, (long long)j_lo,
                (long long)j_hi);
  hipSetDevice(ctx->device);
  sd.j_lo = j_lo;
  sd.j_hi = j_hi;
  hipError_t e = hipMemcpy(ctx->d_segs + seg_id, &sd, sizeof sd, hipMemcpyHostToDevice);
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "segment descriptor upload");
}

}  // extern "C"

namespace {

hipError_t timed_launch(fcas_ctx* ctx, std::vector<TimedPair>& rec, hipStream_t s, int pass, int plan,
                        const PassArgs& a, int grid) {
  // with timing on, the launch itself records the two events at the kernel's
  // start and end (hipExtLaunchKernel)
  TimedPair tp{};
  if (ctx->timing) {
    hipEventCreate(&tp.a);
    hipEventCreate(&tp.b);
  }
  hipError_t e = pass == 1   ? launch_pass1(ctx->prec, plan, a, grid, s, tp.a, tp.b)
                 : pass == 3 ? launch_passm(ctx->prec, plan, a, grid, s, tp.a, tp.b)
                             : launch_pass2(ctx->prec, plan, a, grid, s, tp.a, tp.b);
  if (ctx->timing) rec.push_back(tp);
  return e;
}

// The device buffers one evaluation call works in: point descriptors,
// per-plan work lists and their counts, pass-2 partials and the FFT
// workspace.  A context owns one set (own_bufs); fitness_eval_batch_static
// carves another out of the library's static scratch array.
struct EvalBufs {
  EvalDesc* evals;
  int32_t* lists;        // [kNumPlans][list_stride]
  int32_t* counts;       // [kNumPlans]
  void* part_g;          // [list_stride][part_stride]
  int32_t* part_j;
  void* ws;
  size_t ws_bytes;
  int list_stride;
};

EvalBufs own_bufs(const fcas_ctx* ctx) {
  return EvalBufs{ctx->d_evals, ctx->d_lists, ctx->d_counts, ctx->d_part_g, ctx->d_part_j,
                  ctx->d_ws, ctx->ws_bytes, ctx->cfg.max_batch};
}

// Enqueues the per-point set-up: descriptors and, with build_lists, the
// per-plan work lists (their counts are zero between calls: the context starts
// with zeros and every finalize clears them once the passes are done).
int enqueue_setup(fcas_ctx* ctx, const EvalBufs& b, int32_t n, const double* d_theta, const int32_t* d_seg,
                  hipStream_t s, bool build_lists = true) {
  hipError_t e;
  if ((e = launch_setup(ctx->d_net, ctx->d_segs, d_theta, d_seg, n, b.evals, b.lists, b.counts, b.list_stride,
                        build_lists ? 1 : 0, ctx->d_err, s)) != hipSuccess)
    return hip_fail(e, "set-up launch");
  return FCAS_OK;
}

PassArgs pass_args(fcas_ctx* ctx, const EvalBufs& b, int plan, int cap) {
  PassArgs a{};
  a.segs = ctx->d_segs;
  a.evals = b.evals;
  a.list = b.lists + (size_t)plan * b.list_stride;
  a.count = b.counts + plan;
  a.ws = b.ws;
  a.part_g = b.part_g;
  a.part_j = b.part_j;
  a.part_stride = ctx->part_stride;
  a.n_det = ctx->net.n_det;
  a.chunk_begin = 0;
  a.cap = cap;
  return a;
}

// One persistent launch of the fused schedule for the points of `plan`.
int enqueue_fused(fcas_ctx* ctx, const EvalBufs& b, int plan, int n, int cap, hipStream_t s) {
  const PlanInfo& pi = kPlans[plan];
  if (ctx->fused_cap[plan] == 0) {
    const int nb = fused_blocks_per_cu(plan);
    if (nb < 1) return fail(FCAS_EHIP, "fused kernel of plan %d cannot be resident", plan);
    ctx->fused_cap[plan] = nb * ctx->n_cu;
  }
  const int T = pi.tiles1[0] + pi.tiles2[0];
  const int grid = std::min(ctx->fused_cap[plan], n * T);
  // pipeline lag: about two rounds of the grid between a tile and its consumer
  int lag = (2 * grid + T - 1) / T;
  int slots = 2 * lag + 2;
  if (slots > cap) {
    slots = cap;
    lag = slots - 1;
  }
  FusedArgs f{};
  f.p = pass_args(ctx, b, plan, cap);
  f.done1 = ctx->d_done + (size_t)plan * 2 * ctx->cfg.max_batch;
  f.done2 = f.done1 + ctx->cfg.max_batch;
  f.err = ctx->d_err;
  f.lag = lag;
  f.slots = slots;
  f.max_spin = 1 << 18;
  TimedPair tp{};
  if (ctx->timing) {
    hipEventCreate(&tp.a);
    hipEventCreate(&tp.b);
    hipEventRecord(tp.a, s);
  }
  hipError_t e = launch_fused_f32(plan, f, grid, s);
  if (ctx->timing) {
    hipEventRecord(tp.b, s);
    ctx->t_fused.push_back(tp);
  }
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "fused launch");
}

int enqueue_passes(fcas_ctx* ctx, const EvalBufs& b, int32_t n, double* d_fitness, int32_t* d_argmax,
                   hipStream_t s, bool fused_ok, bool timed, bool finalize = true);

// Enqueues set-up, the FFT passes of every plan in use, and finalize.
int enqueue_eval(fcas_ctx* ctx, const EvalBufs& b, int32_t n, const double* d_theta, const int32_t* d_seg,
                 double* d_fitness, int32_t* d_argmax, hipStream_t s, bool fused_ok = true, bool timed = true) {
  int rc = enqueue_setup(ctx, b, n, d_theta, d_seg, s);
  if (rc) return rc;
  if ((rc = enqueue_passes(ctx, b, n, d_fitness, d_argmax, s, fused_ok, timed))) {
    // the set-up appended to the work lists and only finalize clears their
    // counts: clear them here so that the next call starts from empty lists
    launch_zero_i32(b.counts, kNumPlans, s);
  }
  return rc;
}

int enqueue_eval(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg, double* d_fitness,
                 int32_t* d_argmax, hipStream_t s) {
  return enqueue_eval(ctx, own_bufs(ctx), n, d_theta, d_seg, d_fitness, d_argmax, s);
}

// The FFT passes of every plan in use, then (finalize) the finalize kernel,
// which clears the work-list counts.  Plans with a middle pass, or with passes
// of unequal work items, always run as separate launches (the fused schedule
// covers the other two-pass plans, when fused_ok).  With `timed` false no
// timing events are recorded whatever the context's setting.
int enqueue_passes(fcas_ctx* ctx, const EvalBufs& b, int32_t n, double* d_fitness, int32_t* d_argmax,
                   hipStream_t s, bool fused_ok, bool timed, bool finalize) {
  hipError_t e;
  int rc;
  const bool fused = fused_ok && ctx->schedule == FCAS_SCHEDULE_FUSED;
  if (fused && (e = launch_zero_i32(ctx->d_done, 2 * kNumPlans * ctx->cfg.max_batch, s)) != hipSuccess)
    return hip_fail(e, "zero tile counters");
  const bool was_timing = ctx->timing;
  ctx->timing = was_timing && timed;
  for (int plan = 0; plan < kNumPlans; ++plan) {
    if (ctx->plan_refs[plan] <= 0) continue;
    const PlanInfo& pi = kPlans[plan];
    const size_t slot_bytes = 2 * (size_t)pi.n * ctx->elt;
    int cap = (int)std::min<size_t>(b.ws_bytes / slot_bytes, (size_t)n);
    if (cap < 1) cap = 1;
    if (fused && pi.nm == 1 && pi.threads1[0] == pi.threads2[0]) {
      if ((rc = enqueue_fused(ctx, b, plan, n, cap, s))) {
        ctx->timing = was_timing;
        return rc;
      }
      continue;
    }
    PassArgs a = pass_args(ctx, b, plan, cap);
    for (int begin = 0; begin < n; begin += cap) {
      a.chunk_begin = begin;
      const int m = std::min(cap, n - begin);
      const int g1 = std::min(m * pi.tiles1[ctx->prec], ctx->grid1[plan]);
      const int g2 = std::min(m * pi.tiles2[ctx->prec], ctx->grid2[plan]);
      const char* what = nullptr;
      if ((e = timed_launch(ctx, ctx->t_pass1, s, 1, plan, a, g1)) != hipSuccess) what = "pass-1 launch";
      if (!what && pi.nm > 1) {
        const int gm = std::min(m * pi.tilesm[ctx->prec] * (2 / kPassmSeries), ctx->grid2[plan]);
        if ((e = timed_launch(ctx, ctx->t_passm, s, 3, plan, a, gm)) != hipSuccess) what = "middle-pass launch";
      }
      if (!what && (e = timed_launch(ctx, ctx->t_pass2, s, 2, plan, a, g2)) != hipSuccess) what = "pass-2 launch";
      if (what) {
        ctx->timing = was_timing;
        return hip_fail(e, what);
      }
    }
  }
  ctx->timing = was_timing;
  if (!finalize) return FCAS_OK;
  if ((e = launch_finalize(ctx->prec, b.evals, ctx->d_segs, b.part_g, b.part_j, n, ctx->part_stride,
                           ctx->d_plan_parts2, b.counts, ctx->d_evaluated, d_fitness, d_argmax, s)) != hipSuccess)
    return hip_fail(e, "finalize launch");
  return FCAS_OK;
}

}  // namespace

extern "C" {

int fitness_eval_batch(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg, double* d_fitness,
                       int32_t* d_argmax, void* hip_stream) {
  int rc = validate_batch(ctx, n, d_theta, d_seg, d_fitness, d_argmax);
  if (rc) return rc;
  if (n == 0) return FCAS_OK;
  hipSetDevice(ctx->device);
  return enqueue_eval(ctx, n, d_theta, d_seg, d_fitness, d_argmax, (hipStream_t)hip_stream);
}

int fitness_eval_batch_static(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg,
                              double* d_fitness, int32_t* d_argmax, void* hip_stream) {
  int rc = validate_batch(ctx, n, d_theta, d_seg, d_fitness, d_argmax);
  if (rc) return rc;
  if (n == 0) return FCAS_OK;
  if (!ctx->d_scratch) return fail(FCAS_EHIP, "no static scratch on device %d", ctx->device);
  // carve the call's buffers out of the scratch array, each 256-byte aligned
  const size_t part_elt = ctx->prec ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t o_counts = take(sizeof(int32_t) * kNumPlans);
  const size_t o_lists = take(sizeof(int32_t) * (size_t)kNumPlans * n);
  const size_t o_evals = take(sizeof(EvalDesc) * (size_t)n);
  const size_t o_pg = take(part_elt * (size_t)n * ctx->part_stride);
  const size_t o_pj = take(sizeof(int32_t) * (size_t)n * ctx->part_stride);
  size_t slot_max = 0;
  for (int plan = 0; plan < kNumPlans; ++plan)
    if (ctx->plan_refs[plan] > 0) slot_max = std::max(slot_max, 2 * (size_t)kPlans[plan].n * ctx->elt);
  if (off + std::max<size_t>(slot_max, 1) > kStaticScratchBytes)
    return fail(FCAS_ECAPACITY,
                "static scratch of %zu bytes: the tables of %d points take %zu and the longest registered segment "
                "needs %zu bytes of workspace",
                kStaticScratchBytes, n, off, slot_max);
  unsigned char* base = (unsigned char*)ctx->d_scratch;
  EvalBufs b{};
  b.counts = (int32_t*)(base + o_counts);
  b.lists = (int32_t*)(base + o_lists);
  b.evals = (EvalDesc*)(base + o_evals);
  b.part_g = base + o_pg;
  b.part_j = (int32_t*)(base + o_pj);
  b.ws = base + off;
  b.ws_bytes = kStaticScratchBytes - off;
  b.list_stride = n;
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  // the array keeps whatever the last call on this device left: the list
  // counts must start at zero
  hipError_t e = launch_zero_i32(b.counts, kNumPlans, s);
  if (e != hipSuccess) return hip_fail(e, "zero work-list counts");
  return enqueue_eval(ctx, b, n, d_theta, d_seg, d_fitness, d_argmax, s, false, false);
}

int fitness_grad_batch(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg, double* d_fitness,
                       int32_t* d_argmax, double* d_grad, void* hip_stream) {
  int rc = validate_batch(ctx, n, d_theta, d_seg, d_fitness, d_argmax);
  if (rc) return rc;
  if (n > 0 && !d_grad) return fail(FCAS_EINVAL, "NULL gradient pointer");
  if (n == 0) return FCAS_OK;
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  if ((rc = enqueue_eval(ctx, n, d_theta, d_seg, d_fitness, d_argmax, s))) return rc;
  hipError_t e = launch_gradient(ctx->prec, ctx->grad, ctx->d_net, ctx->d_segs, ctx->d_evals, d_theta, d_argmax, n,
                                 ctx->net.n_det, d_grad, s);
  if (e != hipSuccess) return hip_fail(e, "gradient launch");
  return FCAS_OK;
}

int fitness_polish(fcas_ctx* ctx, int32_t n, double* d_theta, const int32_t* d_seg, int32_t n_steps,
                   double step_frac, int32_t n_trials, double* d_fitness, int32_t* d_argmax, void* hip_stream) {
  int rc = validate_batch(ctx, n, d_theta, d_seg, d_fitness, d_argmax);
  if (rc) return rc;
  if (n_steps < 0 || n_trials < 1 || n_trials > 32) return fail(FCAS_EINVAL, "need n_steps >= 0, 1 <= n_trials <= 32");
  if (!(step_frac > 0) || !std::isfinite(step_frac)) return fail(FCAS_EINVAL, "step_frac must be positive");
  if ((int64_t)n * n_trials > ctx->cfg.max_batch)
    return fail(FCAS_ECAPACITY, "n * n_trials = %lld exceeds max_batch = %d", (long long)n * n_trials,
                ctx->cfg.max_batch);
  if (n == 0) return FCAS_OK;
  hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e;
  if ((rc = enqueue_eval(ctx, n, d_theta, d_seg, d_fitness, d_argmax, s))) return rc;
  for (int step = 0; step < n_steps; ++step) {
    // descriptors of the current points (their maximising samples are already in d_argmax)
    if (step > 0 && (rc = enqueue_setup(ctx, own_bufs(ctx), n, d_theta, d_seg, s, false))) return rc;
    if ((e = launch_gradient(ctx->prec, ctx->grad, ctx->d_net, ctx->d_segs, ctx->d_evals, d_theta, d_argmax, n,
                             ctx->net.n_det, ctx->d_pol_grad, s)) !=
            hipSuccess ||
        (e = launch_polish_trials(d_theta, ctx->d_pol_grad, d_seg, ctx->d_net, n, n_trials, step_frac,
                                  ctx->d_pol_cand, ctx->d_pol_seg, s)) != hipSuccess)
      return hip_fail(e, "polish launch");
    const int m = n * n_trials;
    // the trial batch reuses the evaluation buffers: its outputs go to the polish scratch arrays
    double* cand_f = ctx->d_pol_f;
    int32_t* cand_j = ctx->d_pol_j;
    if ((rc = enqueue_eval(ctx, m, ctx->d_pol_cand, ctx->d_pol_seg, cand_f, cand_j, s))) return rc;
    if ((e = launch_polish_select(d_theta, d_fitness, d_argmax, ctx->d_pol_cand, cand_f, cand_j, n, n_trials, s)) !=
        hipSuccess)
      return hip_fail(e, "polish select launch");
  }
  return FCAS_OK;
}

int fcas_inject(fcas_ctx* ctx, int64_t n_samples, const double* params, double snr, const double* d_psd,
                double* d_xf, void* hip_stream) {
  if (!ctx || !params || !d_psd || !d_xf) return fail(FCAS_EINVAL, "NULL argument");
  if (!finite_all(params, 8) || !std::isfinite(snr) || snr < 0) return fail(FCAS_EINVAL, "non-finite parameter");
  if (!(params[2] > 0) || !(params[3] > 0)) return fail(FCAS_EINVAL, "chirp times must be positive");
  if (params[6] < -1.0 || params[6] > 1.0) return fail(FCAS_EINVAL, "cos_iota must be in [-1, 1]");
  if (n_samples < 4 || (n_samples & 1)) return fail(FCAS_EINVAL, "n_samples must be even and >= 4");
  int k_lo, k_hi;
  band(ctx->cfg, n_samples, &k_lo, &k_hi);
  if (k_lo > k_hi) return fail(FCAS_EINVAL, "empty band for %lld samples", (long long)n_samples);
  hipSetDevice(ctx->device);
  hipError_t e = launch_inject(ctx->h_net, params, snr, n_samples, k_lo, k_hi, ctx->cfg.fs_hz / (double)n_samples,
                               d_psd, ctx->d_inject, ctx->d_sigma2, d_xf, (hipStream_t)hip_stream);
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "injection launch");
}

int fcas_device_error(fcas_ctx* ctx, int32_t* flags_out) {
  if (!ctx || !flags_out) return fail(FCAS_EINVAL, "NULL argument");
  hipSetDevice(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  if ((e = hipMemcpy(flags_out, ctx->d_err, sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "read error flags");
  if ((e = hipMemset(ctx->d_err, 0, sizeof(int32_t))) != hipSuccess) return hip_fail(e, "clear error flags");
  return FCAS_OK;
}

int fcas_evaluated(fcas_ctx* ctx, uint64_t* count_out) {
  if (!ctx || !count_out) return fail(FCAS_EINVAL, "NULL argument");
  hipSetDevice(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  unsigned long long v = 0;
  if ((e = hipMemcpy(&v, ctx->d_evaluated, sizeof v, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "read evaluation count");
  *count_out = (uint64_t)v;
  return FCAS_OK;
}

int fcas_set_timing(fcas_ctx* ctx, int enable) {
  if (!ctx) return fail(FCAS_EINVAL, "context is NULL");
  ctx->timing = enable != 0;
  return FCAS_OK;
}

int fcas_read_timing(fcas_ctx* ctx, const char* which, double* total_ms, int64_t* launches) {
  if (!ctx || !which || !total_ms || !launches) return fail(FCAS_EINVAL, "NULL argument");
  std::vector<TimedPair>* rec = nullptr;
  if (!std::strcmp(which, "pass1")) rec = &ctx->t_pass1;
  else if (!std::strcmp(which, "passm")) rec = &ctx->t_passm;
  else if (!std::strcmp(which, "pass2")) rec = &ctx->t_pass2;
  else if (!std::strcmp(which, "fused")) rec = &ctx->t_fused;
  else return fail(FCAS_EINVAL, "unknown kernel name '%s' (timed: pass1, passm, pass2, fused)", which);
  hipSetDevice(ctx->device);
  double tot = 0.0;
  for (auto& t : *rec) {
    hipError_t e = hipEventSynchronize(t.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    hipEventElapsedTime(&ms, t.a, t.b);
    tot += ms;
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  *total_ms = tot;
  *launches = (int64_t)rec->size();
  rec->clear();
  return FCAS_OK;
}

}  // extern "C"

// precision dispatch of the pass launchers (the instantiations live in eval_f32.hip / eval_f64.hip)
namespace fcas {
hipError_t launch_pass1_f32(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_pass1_f64(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_passm_f32(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_passm_f64(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_pass2_f32(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_pass2_f64(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_finalize_f32(const EvalDesc*, const SegDesc*, const void*, const int32_t*, int, int, const int32_t*,
                               int32_t*, unsigned long long*, double*, int32_t*, hipStream_t);
hipError_t launch_finalize_f64(const EvalDesc*, const SegDesc*, const void*, const int32_t*, int, int, const int32_t*,
                               int32_t*, unsigned long long*, double*, int32_t*, hipStream_t);

hipError_t launch_pass1(int precision, int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  return precision ? launch_pass1_f64(plan, a, grid, s, e0, e1) : launch_pass1_f32(plan, a, grid, s, e0, e1);
}
hipError_t launch_passm(int precision, int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  return precision ? launch_passm_f64(plan, a, grid, s, e0, e1) : launch_passm_f32(plan, a, grid, s, e0, e1);
}
hipError_t launch_pass2(int precision, int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
  return precision ? launch_pass2_f64(plan, a, grid, s, e0, e1) : launch_pass2_f32(plan, a, grid, s, e0, e1);
}
hipError_t launch_finalize(int precision, const EvalDesc* evals, const SegDesc* segs, const void* part_g,
                           const int32_t* part_j, int n, int part_stride, const int32_t* plan_parts2,
                           int32_t* counts, unsigned long long* evaluated, double* fitness, int32_t* argmax,
                           hipStream_t s) {
  return precision ? launch_finalize_f64(evals, segs, part_g, part_j, n, part_stride, plan_parts2, counts, evaluated,
                                         fitness, argmax, s)
                   : launch_finalize_f32(evals, segs, part_g, part_j, n, part_stride, plan_parts2, counts, evaluated,
                                         fitness, argmax, s);
}
}  // namespace fcas

namespace {

int make_pso(const fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, PsoDev* d) {
  if (!ctx || !p || !s) return fail(FCAS_EINVAL, "NULL argument");
  if (p->n_runs < 1 || p->n_runs > (1 << 20)) return fail(FCAS_EINVAL, "n_runs must be in [1, 2^20]");
  if (p->n_particles < 1 || p->n_particles > 1024) return fail(FCAS_EINVAL, "n_particles must be in [1, 1024]");
  if (p->n_iter < 1) return fail(FCAS_EINVAL, "n_iter must be >= 1");
  const double pr[5] = {p->w0, p->w1, p->c1, p->c2, p->vmax};
  if (!finite_all(pr, 5) || !(p->vmax > 0)) return fail(FCAS_EINVAL, "PSO constants must be finite, vmax > 0");
  if (!s->x || !s->v || !s->pbest_x || !s->pbest_f || !s->pbest_j || !s->best_x || !s->best_f || !s->best_j ||
      !s->iteration)
    return fail(FCAS_EINVAL, "NULL swarm state array");
  d->n_runs = p->n_runs;
  d->n_particles = p->n_particles;
  d->n_iter = p->n_iter;
  d->w0 = p->w0;
  d->w1 = p->w1;
  d->c1 = p->c1;
  d->c2 = p->c2;
  d->vmax = p->vmax;
  d->seed = p->seed;
  for (int k = 0; k < 4; ++k) {
    d->lo[k] = ctx->cfg.box_lo[k];
    d->span[k] = ctx->cfg.box_hi[k] - ctx->cfg.box_lo[k];
  }
  d->x = s->x;
  d->v = s->v;
  d->pbest_x = s->pbest_x;
  d->pbest_f = s->pbest_f;
  d->pbest_j = s->pbest_j;
  d->best_x = s->best_x;
  d->best_f = s->best_f;
  d->best_j = s->best_j;
  d->iteration = s->iteration;
  return FCAS_OK;
}

}  // namespace

extern "C" {

int pso_init(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, double* d_theta_out,
             void* hip_stream) {
  PsoDev d{};
  int rc = make_pso(ctx, p, s, &d);
  if (rc) return rc;
  if (!d_theta_out) return fail(FCAS_EINVAL, "NULL theta output");
  hipSetDevice(ctx->device);
  hipError_t e = launch_pso_init(d, d_theta_out, (hipStream_t)hip_stream);
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "pso_init launch");
}

int pso_step(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, const double* d_fitness,
             const int32_t* d_argmax, double* d_theta_next, void* hip_stream) {
  PsoDev d{};
  int rc = make_pso(ctx, p, s, &d);
  if (rc) return rc;
  if (!d_fitness || !d_argmax || !d_theta_next) return fail(FCAS_EINVAL, "NULL device pointer");
  hipSetDevice(ctx->device);
  hipError_t e = launch_pso_step(d, d_fitness, d_argmax, d_theta_next, (hipStream_t)hip_stream);
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "pso_step launch");
}

int pso_run(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, int32_t n_iter, double* d_theta,
            const int32_t* d_seg, double* d_fitness, int32_t* d_argmax, void* hip_stream) {
  PsoDev d{};
  int rc = make_pso(ctx, p, s, &d);
  if (rc) return rc;
  if (n_iter < 0) return fail(FCAS_EINVAL, "n_iter must be >= 0, got %d", n_iter);
  const int64_t n64 = (int64_t)d.n_runs * d.n_particles;
  if (n64 > ctx->cfg.max_batch)
    return fail(FCAS_ECAPACITY, "n_runs * n_particles = %lld exceeds max_batch = %d", (long long)n64,
                ctx->cfg.max_batch);
  const int n = (int)n64;
  if ((rc = validate_batch(ctx, n, d_theta, d_seg, d_fitness, d_argmax))) return rc;
  if (n_iter == 0) return FCAS_OK;
  hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e;
  if (d.n_particles > kTailMaxParticles) {
    // runs too large for one work-group of the fused tail: separate launches
    for (int it = 0; it < n_iter; ++it) {
      if ((rc = enqueue_eval(ctx, own_bufs(ctx), n, d_theta, d_seg, d_fitness, d_argmax, st, true, false)))
        return rc;
      if ((e = launch_pso_step(d, d_fitness, d_argmax, d_theta, st)) != hipSuccess)
        return hip_fail(e, "pso_step launch");
    }
    return FCAS_OK;
  }
  // Iteration it evaluates from work-list set it % 2; the tail kernel that
  // ends it clears that set's counts and appends the next points to the other.
  EvalBufs b[2] = {own_bufs(ctx), own_bufs(ctx)};
  b[1].lists = ctx->d_lists2;
  b[1].counts = ctx->d_counts2;
  auto clear_counts = [&]() {
    launch_zero_i32(b[0].counts, kNumPlans, st);
    launch_zero_i32(b[1].counts, kNumPlans, st);
  };
  if ((rc = enqueue_setup(ctx, b[0], n, d_theta, d_seg, st))) return rc;
  for (int it = 0; it < n_iter; ++it) {
    const EvalBufs& cur = b[it & 1];
    const EvalBufs& nxt = b[(it + 1) & 1];
    if ((rc = enqueue_passes(ctx, cur, n, d_fitness, d_argmax, st, true, false, false))) {
      clear_counts();
      return rc;
    }
    TailArgs t{};
    t.net = ctx->d_net;
    t.segs = ctx->d_segs;
    t.evals = cur.evals;
    t.part_g = cur.part_g;
    t.part_j = cur.part_j;
    t.part_stride = ctx->part_stride;
    t.list_stride = nxt.list_stride;
    t.plan_parts2 = ctx->d_plan_parts2;
    t.counts_cur = cur.counts;
    t.lists_next = nxt.lists;
    t.counts_next = nxt.counts;
    t.evaluated = ctx->d_evaluated;
    t.fitness = d_fitness;
    t.argmax = d_argmax;
    t.theta = d_theta;
    t.seg_ids = d_seg;
    t.err = ctx->d_err;
    t.setup = it + 1 < n_iter ? 1 : 0;
    if ((e = launch_pso_tail(ctx->prec, d, t, st)) != hipSuccess) {
      clear_counts();
      return hip_fail(e, "PSO tail launch");
    }
  }
  return FCAS_OK;
}

int pso_best(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, double* d_out_f,
             double* d_out_theta, int32_t* d_out_j, int32_t* d_out_run, void* hip_stream) {
  PsoDev d{};
  int rc = make_pso(ctx, p, s, &d);
  if (rc) return rc;
  if (!d_out_f || !d_out_theta || !d_out_j || !d_out_run) return fail(FCAS_EINVAL, "NULL device pointer");
  hipSetDevice(ctx->device);
  hipError_t e =
      launch_pso_best(d, d.n_runs, d.n_runs, d_out_f, d_out_theta, d_out_j, d_out_run, (hipStream_t)hip_stream);
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "pso_best launch");
}

int pso_best_segments(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, int32_t runs_per_segment,
                      int32_t runs_used, double* d_out_f, double* d_out_theta, int32_t* d_out_j, int32_t* d_out_run,
                      void* hip_stream) {
  PsoDev d{};
  int rc = make_pso(ctx, p, s, &d);
  if (rc) return rc;
  if (runs_per_segment < 1 || d.n_runs % runs_per_segment != 0)
    return fail(FCAS_EINVAL, "runs_per_segment = %d must divide n_runs = %d", runs_per_segment, d.n_runs);
  if (runs_used < 1 || runs_used > runs_per_segment)
    return fail(FCAS_EINVAL, "runs_used = %d must be in [1, runs_per_segment = %d]", runs_used, runs_per_segment);
  if (!d_out_f || !d_out_theta || !d_out_j || !d_out_run) return fail(FCAS_EINVAL, "NULL device pointer");
  hipSetDevice(ctx->device);
  hipError_t e = launch_pso_best(d, runs_per_segment, runs_used, d_out_f, d_out_theta, d_out_j, d_out_run,
                                 (hipStream_t)hip_stream);
  return e == hipSuccess ? FCAS_OK : hip_fail(e, "pso_best_segments launch");
}

}  // extern "C"
