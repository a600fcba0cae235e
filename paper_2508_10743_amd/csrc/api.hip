// C ABI of libdarc: argument validation, workspace sizing, the coordinate-
// descent sweep (Eq. (3), Algorithm 1 of the paper) and kernel timing.
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "darc.h"
#include "darc_kernels.hpp"

using namespace darc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return DARC_OK;
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DARC_EHIP, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

constexpr long long kMaxVoxels = 1ll << 29;

int check_dims(const char* fn, int n, int d0, int d1, int d2) {
  if (n < 0) return fail(DARC_EINVAL, "%s: n = %d < 0", fn, n);
  if (d0 < 2 || d1 < 2 || d2 < 2)
    return fail(DARC_EINVAL, "%s: every dim must be >= 2 (got %d x %d x %d)", fn, d0, d1, d2);
  const long long V = static_cast<long long>(d0) * d1 * d2;
  if (V > kMaxVoxels)
    return fail(DARC_EINVAL, "%s: %lld voxels exceed the limit of %lld", fn, V, kMaxVoxels);
  return DARC_OK;
}

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

int check_ws(const char* fn, void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return DARC_OK;
  if (!ws) return fail(DARC_EWORKSPACE, "%s: workspace of %zu bytes required, got NULL", fn, need);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(DARC_EWORKSPACE, "%s: workspace must be 256-byte aligned", fn);
  if (ws_bytes < need)
    return fail(DARC_EWORKSPACE, "%s: workspace of %zu bytes is smaller than %zu", fn, ws_bytes,
                need);
  return DARC_OK;
}

size_t field_bytes(int n, int d0, int d1, int d2) {
  return static_cast<size_t>(n) * 3 * d0 * d1 * d2 * sizeof(float);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

#define DARC_TRY(expr)          \
  do {                          \
    const int rc__ = (expr);    \
    if (rc__ != DARC_OK) return rc__; \
  } while (0)

// ------------------------------------------------------------- kernel timing

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};

bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_event_pool;
long long g_prof_counts[KC_NUM];
double g_prof_ms[KC_NUM];

const char* const kClassNames[KC_NUM] = {
    "exp_fwd_step", "exp_bwd_step", "warp", "warp_bwd", "mse", "lncc_fwd", "lncc_bwd",
    "gauss", "diffusion", "adam", "center", "atlas", "fill", "misc", "iter_fused"};

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

namespace darc {

void prof_begin(hipStream_t s, int cls) {
  if (!g_prof_on) return;
  hipEvent_t a = take_event();
  if (!a) return;
  (void)hipEventRecord(a, s);
  g_prof_recs.push_back(ProfRec{cls, a, nullptr});
}

void prof_end(hipStream_t s, int cls) {
  if (!g_prof_on || g_prof_recs.empty()) return;
  ProfRec& r = g_prof_recs.back();
  if (r.cls != cls || r.b != nullptr) return;
  hipEvent_t b = take_event();
  if (!b) return;
  (void)hipEventRecord(b, s);
  r.b = b;
}

// ------------------------------------------------------------ tuning table

namespace {
struct TuneEntry {
  int kind, d0, d1, d2, n, tz;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
}  // namespace

int tuned_tz(int kind, const Geom& g, int n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int fallback = 0;  // the entry for every shape (dims and n zero), if set
  for (const TuneEntry& e : g_tune) {
    if (e.kind != kind) continue;
    if (e.d0 == g.d0 && e.d1 == g.d1 && e.d2 == g.d2 && e.n == n) return e.tz;
    if (e.d0 == 0 && e.d1 == 0 && e.d2 == 0 && e.n == 0) fallback = e.tz;
  }
  return fallback;
}

void set_tuned_tz(int kind, const Geom& g, int n, int tz) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (TuneEntry& e : g_tune)
    if (e.kind == kind && e.d0 == g.d0 && e.d1 == g.d1 && e.d2 == g.d2 && e.n == n) {
      e.tz = tz;
      return;
    }
  g_tune.push_back(TuneEntry{kind, g.d0, g.d1, g.d2, n, tz});
}

void clear_tuned() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

// Runs `body` twice on `s` and returns the faster time in ms (or -1).
template <class F>
float time_on(hipStream_t s, F body) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
  float best = -1.0f;
  body();  // warm-up
  for (int r = 0; r < 2; ++r) {
    (void)hipEventRecord(a, s);
    body();
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess) break;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) == hipSuccess && (best < 0.0f || ms < best)) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

}  // namespace darc

extern "C" {

int darc_abi_version(void) { return DARC_ABI_VERSION; }

const char* darc_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ Exp(v)

size_t darc_exp_svf_ws_bytes(int n, int d0, int d1, int d2, int n_sq, int has_ckpt) {
  if (n <= 0 || n_sq < 2 || has_ckpt) return 0;
  return field_bytes(n, d0, d1, d2);
}

int darc_exp_svf(const float* v, float* u, float* ckpt, int n, int d0, int d1, int d2, int n_sq,
                 void* ws, size_t ws_bytes, void* stream) {
  DARC_TRY(check_dims("darc_exp_svf", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!v || !u) return fail(DARC_EINVAL, "darc_exp_svf: v and u must not be NULL");
  if (u == v) return fail(DARC_EINVAL, "darc_exp_svf: u must not alias v");
  if (n_sq < 0 || n_sq > 16) return fail(DARC_EINVAL, "darc_exp_svf: n_sq = %d not in 0..16", n_sq);
  const size_t need = darc_exp_svf_ws_bytes(n, d0, d1, d2, n_sq, ckpt != nullptr);
  DARC_TRY(check_ws("darc_exp_svf", ws, ws_bytes, need));
  const Geom g = make_geom(d0, d1, d2);
  run_exp_fwd(v, u, n_sq >= 2 ? ckpt : nullptr, static_cast<float*>(ws), nullptr, g, n, n_sq,
              as_stream(stream));
  return check_launch("darc_exp_svf");
}

// gradient ping-pong buffers (plus two recompute buffers without
// checkpoints), then the adjoint's tile records
static size_t exp_bwd_fields(int n_sq, int has_ckpt) {
  const size_t nf = n_sq >= 3 ? 2 : (n_sq == 2 ? 1 : 0);
  return nf + ((!has_ckpt && n_sq >= 2) ? 2 : 0);
}

size_t darc_exp_svf_bwd_ws_bytes(int n, int d0, int d1, int d2, int n_sq, int has_ckpt) {
  if (n <= 0 || n_sq < 1 || d0 < 2 || d1 < 2 || d2 < 2) return 0;
  const size_t f = align256(field_bytes(n, d0, d1, d2));
  return exp_bwd_fields(n_sq, has_ckpt) * f +
         align256(exp_aux_bytes(make_geom(d0, d1, d2), n, n_sq));
}

int darc_exp_svf_bwd(const float* v, const float* ckpt, const float* g_u, float* g_v, int n, int d0,
                     int d1, int d2, int n_sq, void* ws, size_t ws_bytes, void* stream) {
  DARC_TRY(check_dims("darc_exp_svf_bwd", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!v || !g_u || !g_v) return fail(DARC_EINVAL, "darc_exp_svf_bwd: v, g_u, g_v must not be NULL");
  if (g_v == g_u) return fail(DARC_EINVAL, "darc_exp_svf_bwd: g_v must not alias g_u");
  if (n_sq < 0 || n_sq > 16)
    return fail(DARC_EINVAL, "darc_exp_svf_bwd: n_sq = %d not in 0..16", n_sq);
  const int has_ckpt = ckpt != nullptr;
  const size_t need = darc_exp_svf_bwd_ws_bytes(n, d0, d1, d2, n_sq, has_ckpt);
  DARC_TRY(check_ws("darc_exp_svf_bwd", ws, ws_bytes, need));
  const Geom g = make_geom(d0, d1, d2);
  char* w = static_cast<char*>(ws);
  const size_t f = align256(field_bytes(n, d0, d1, d2));
  const size_t nf = exp_bwd_fields(n_sq, has_ckpt);
  float* buf[4] = {nullptr, nullptr, nullptr, nullptr};
  for (size_t i = 0; i < nf; ++i) buf[i] = reinterpret_cast<float*>(w + i * f);
  int* aux = reinterpret_cast<int*>(w + nf * f);
  if (has_ckpt || n_sq < 2)
    run_exp_bwd(v, ckpt, g_u, g_v, buf[0], buf[1], aux, false, g, n, n_sq, as_stream(stream));
  else
    run_exp_bwd_recompute(v, g_u, g_v, buf[0], buf[1], buf[2], buf[3], aux, g, n, n_sq,
                          as_stream(stream));
  return check_launch("darc_exp_svf_bwd");
}

// -------------------------------------------------------------------- warp

int darc_warp3d(const float* img, const float* u, float* out, int n, int d0, int d1, int d2,
                void* stream) {
  DARC_TRY(check_dims("darc_warp3d", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!img || !u || !out) return fail(DARC_EINVAL, "darc_warp3d: NULL pointer");
  if (out == img) return fail(DARC_EINVAL, "darc_warp3d: out must not alias img");
  launch_warp(img, u, out, make_geom(d0, d1, d2), n, as_stream(stream));
  return check_launch("darc_warp3d");
}

int darc_warp3d_bwd(const float* img, const float* u, const float* g_out, float* g_u, int n, int d0,
                    int d1, int d2, void* stream) {
  DARC_TRY(check_dims("darc_warp3d_bwd", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!img || !u || !g_out || !g_u) return fail(DARC_EINVAL, "darc_warp3d_bwd: NULL pointer");
  launch_warp_bwd(img, u, g_out, g_u, make_geom(d0, d1, d2), n, as_stream(stream));
  return check_launch("darc_warp3d_bwd");
}

// --------------------------------------------------------- dissimilarities

size_t darc_sim_grad_ws_bytes(int metric, int n, int d0, int d1, int d2) {
  if (metric != DARC_LNCC || n <= 0) return 0;
  return static_cast<size_t>(n) * 4 * d0 * d1 * d2 * sizeof(float);
}

int darc_sim_grad(const float* warped, const float* atlas, int metric, int win, float eps,
                  double* loss, float* g_warped, int n, int d0, int d1, int d2, void* ws,
                  size_t ws_bytes, void* stream) {
  DARC_TRY(check_dims("darc_sim_grad", n, d0, d1, d2));
  if (metric != DARC_MSE && metric != DARC_LNCC && metric != DARC_L1)
    return fail(DARC_EINVAL, "darc_sim_grad: unknown metric %d", metric);
  if (metric == DARC_LNCC) {
    if (win < 1 || win % 2 == 0)
      return fail(DARC_EINVAL, "darc_sim_grad: window %d must be odd and positive", win);
    if (!lncc_window_supported(win))
      return fail(DARC_EUNSUPPORTED, "darc_sim_grad: window %d not built (3, 5, 7, 9, 11)", win);
    if (!(eps > 0.0f)) return fail(DARC_EINVAL, "darc_sim_grad: eps must be > 0");
  }
  if (n == 0) return ok();
  if (!warped || !atlas || !loss) return fail(DARC_EINVAL, "darc_sim_grad: NULL pointer");
  const Geom g = make_geom(d0, d1, d2);
  hipStream_t st = as_stream(stream);
  if (metric != DARC_LNCC) {
    launch_mse(warped, atlas, loss, 1, g_warped, g, n, metric == DARC_L1, st);
  } else {
    const size_t need = g_warped ? darc_sim_grad_ws_bytes(metric, n, d0, d1, d2) : 0;
    DARC_TRY(check_ws("darc_sim_grad", ws, ws_bytes, need));
    float* fields = g_warped ? static_cast<float*>(ws) : nullptr;
    launch_lncc_fwd(warped, atlas, fields, loss, 1, win, eps, g, n, st);
    if (g_warped) launch_lncc_bwd(fields, warped, atlas, g_warped, win, g, n, st);
  }
  return check_launch("darc_sim_grad");
}

}  // extern "C"

// ------------------------------------------- dissimilarity without allocation

namespace {

// The scratch of darc_sim_grad_noalloc: one array per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address): every use goes through
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = static_cast<size_t>(128) << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device, filled on first use

int scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return fail(DARC_EHIP, "darc_sim_grad_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.empty()) {
    int count = 0;
    e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1)
      return fail(DARC_EHIP, "darc_sim_grad_noalloc: hipGetDeviceCount: %s",
                  hipGetErrorString(e));
    g_scratch_ptr.assign(static_cast<size_t>(count), nullptr);
  }
  if (dev < 0 || dev >= static_cast<int>(g_scratch_ptr.size()))
    return fail(DARC_EHIP, "darc_sim_grad_noalloc: device %d out of range", dev);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DARC_EHIP, "darc_sim_grad_noalloc: hipGetSymbolAddress: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DARC_OK;
}

}  // namespace

extern "C" {

size_t darc_sim_grad_noalloc_max_bytes(void) { return kNoallocScratchBytes; }

int darc_sim_grad_noalloc(const float* warped, const float* atlas, int metric, int win, float eps,
                          double* loss, float* g_warped, int n, int d0, int d1, int d2,
                          void* stream) {
  DARC_TRY(check_dims("darc_sim_grad_noalloc", n, d0, d1, d2));
  const size_t need = (g_warped && n > 0) ? darc_sim_grad_ws_bytes(metric, n, d0, d1, d2) : 0;
  if (need > kNoallocScratchBytes)
    return fail(DARC_EWORKSPACE,
                "darc_sim_grad_noalloc: %d subjects of %d x %d x %d need %zu bytes of scratch, "
                "more than the %zu held per GPU; split the batch or use darc_sim_grad",
                n, d0, d1, d2, need, kNoallocScratchBytes);
  void* ws = nullptr;
  if (need > 0) DARC_TRY(scratch_for_current_device(&ws));
  const int rc = darc_sim_grad(warped, atlas, metric, win, eps, loss, g_warped, n, d0, d1, d2, ws,
                               need > 0 ? kNoallocScratchBytes : 0, stream);
  if (rc != DARC_OK) {
    // name this entry point in the message darc_sim_grad left
    const std::string msg = g_err;
    return fail(rc, "darc_sim_grad_noalloc: %s", msg.c_str());
  }
  return rc;
}

// ------------------------------------------------------------- smoothing

int darc_smooth3d(const float* in, float* out, int n, int ncomp, int d0, int d1, int d2, int mode,
                  float param, double* loss, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  DARC_TRY(check_dims("darc_smooth3d", n, d0, d1, d2));
  if (ncomp < 1) return fail(DARC_EINVAL, "darc_smooth3d: ncomp = %d < 1", ncomp);
  if (mode != DARC_GAUSS && mode != DARC_DIFFUSION)
    return fail(DARC_EINVAL, "darc_smooth3d: unknown mode %d", mode);
  if (mode == DARC_GAUSS) {
    if (!(param > 0.0f)) return fail(DARC_EINVAL, "darc_smooth3d: sigma must be > 0");
    const int r = gauss_radius(param);
    if (r < 1 || r > 8)
      return fail(DARC_EUNSUPPORTED, "darc_smooth3d: radius int(3 sigma + 0.5) = %d not in 1..8", r);
  }
  if (n == 0) return ok();
  if (!in) return fail(DARC_EINVAL, "darc_smooth3d: in must not be NULL");
  if (out == in) return fail(DARC_EINVAL, "darc_smooth3d: out must not alias in");
  const Geom g = make_geom(d0, d1, d2);
  hipStream_t st = as_stream(stream);
  if (mode == DARC_GAUSS) {
    if (!out) return fail(DARC_EINVAL, "darc_smooth3d: out must not be NULL");
    launch_gauss(in, out, param, g, n * ncomp, st);
  } else {
    if (!out && !loss) return fail(DARC_EINVAL, "darc_smooth3d: out and loss are both NULL");
    launch_diffusion(in, out, loss, 1, make_regw(g, ncomp, param), g, n, ncomp, st);
  }
  return check_launch("darc_smooth3d");
}

// ------------------------------------------------- Adam, centring, atlas

int darc_adam_step(float* v, float* m, float* s, const float* g, long long count, long long t,
                   float lr, double beta1, double beta2, float eps, void* stream) {
  if (count < 0) return fail(DARC_EINVAL, "darc_adam_step: count < 0");
  if (t < 1) return fail(DARC_EINVAL, "darc_adam_step: step t must be >= 1");
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
    return fail(DARC_EINVAL, "darc_adam_step: betas must lie in [0, 1)");
  if (!(eps > 0.0f)) return fail(DARC_EINVAL, "darc_adam_step: eps must be > 0");
  if (count == 0) return ok();
  if (!v || !m || !s || !g) return fail(DARC_EINVAL, "darc_adam_step: NULL pointer");
  launch_adam(v, v, m, s, g, count, t, lr, beta1, beta2, eps, as_stream(stream));
  return check_launch("darc_adam_step");
}

int darc_center(float* u, float* mean_out, int n, int d0, int d1, int d2, void* stream) {
  DARC_TRY(check_dims("darc_center", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!u) return fail(DARC_EINVAL, "darc_center: u must not be NULL");
  launch_center(u, mean_out, make_geom(d0, d1, d2), n, as_stream(stream));
  return check_launch("darc_center");
}

int darc_atlas_update(const float* images, const float* u, const float* mean, float* atlas, int n,
                      int d0, int d1, int d2, void* stream) {
  DARC_TRY(check_dims("darc_atlas_update", n, d0, d1, d2));
  if (n < 1) return fail(DARC_EINVAL, "darc_atlas_update: n must be >= 1");
  if (!images || !atlas) return fail(DARC_EINVAL, "darc_atlas_update: NULL pointer");
  if (!u && mean) return fail(DARC_EINVAL, "darc_atlas_update: mean given without u");
  launch_atlas(images, u, mean, atlas, make_geom(d0, d1, d2), n, as_stream(stream));
  return check_launch("darc_atlas_update");
}

int darc_atlas_median(const float* images, const float* u, const float* mean, float* atlas, int n,
                      int d0, int d1, int d2, void* stream) {
  DARC_TRY(check_dims("darc_atlas_median", n, d0, d1, d2));
  if (n < 1) return fail(DARC_EINVAL, "darc_atlas_median: n must be >= 1");
  if (median_threads(n) == 0)
    return fail(DARC_EUNSUPPORTED, "darc_atlas_median: n = %d > 512 subjects", n);
  if (!images || !u || !atlas) return fail(DARC_EINVAL, "darc_atlas_median: NULL pointer");
  launch_atlas_median(images, u, mean, atlas, make_geom(d0, d1, d2), n, as_stream(stream));
  return check_launch("darc_atlas_median");
}

}  // extern "C"

// ------------------------------------------------------- stochastic atlas

namespace {

struct SgdLayout {
  size_t fields, ga, m, s, sloss, total;
};

SgdLayout sgd_layout(int d0, int d1, int d2, int batch) {
  const size_t V = static_cast<size_t>(d0) * d1 * d2;
  SgdLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.fields = take(static_cast<size_t>(batch) * 4 * V * sizeof(float));
  L.ga = take(static_cast<size_t>(batch) * V * sizeof(float));
  L.m = take(V * sizeof(float));
  L.s = take(V * sizeof(float));
  L.sloss = take(static_cast<size_t>(batch) * sizeof(double));
  L.total = off;
  return L;
}

int check_sgd(const char* fn, int batch, int epochs, int win, float eps, float lr, double b1,
              double b2, float aeps) {
  if (batch < 1) return fail(DARC_EINVAL, "%s: atlas batch must be >= 1", fn);
  if (epochs < 1) return fail(DARC_EINVAL, "%s: epochs must be >= 1", fn);
  if (win < 1 || win % 2 == 0) return fail(DARC_EINVAL, "%s: window %d must be odd", fn, win);
  if (!lncc_window_supported(win))
    return fail(DARC_EUNSUPPORTED, "%s: window %d not built (3, 5, 7, 9, 11)", fn, win);
  if (!(eps > 0.0f)) return fail(DARC_EINVAL, "%s: eps must be > 0", fn);
  if (!(lr > 0.0f)) return fail(DARC_EINVAL, "%s: learning rate must be > 0", fn);
  if (!(b1 >= 0.0 && b1 < 1.0 && b2 >= 0.0 && b2 < 1.0))
    return fail(DARC_EINVAL, "%s: betas must lie in [0, 1)", fn);
  if (!(aeps > 0.0f)) return fail(DARC_EINVAL, "%s: adam eps must be > 0", fn);
  return DARC_OK;
}

// epochs x minibatches of one Adam step on the atlas each
void run_atlas_sgd(const float* warped, float* atlas, int n, const Geom& g, int batch, int epochs,
                   int win, float eps, float lr, double b1, double b2, float aeps, double* losses,
                   char* ws, hipStream_t s) {
  const SgdLayout L = sgd_layout(g.d0, g.d1, g.d2, batch);
  float* fields = reinterpret_cast<float*>(ws + L.fields);
  float* ga = reinterpret_cast<float*>(ws + L.ga);
  float* m = reinterpret_cast<float*>(ws + L.m);
  float* sv = reinterpret_cast<float*>(ws + L.s);
  double* sloss = reinterpret_cast<double*>(ws + L.sloss);
  launch_fill_f32(m, g.V, 0.0f, s);
  launch_fill_f32(sv, g.V, 0.0f, s);
  long long t = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int b0 = 0; b0 < n; b0 += batch) {
      const int nb = n - b0 < batch ? n - b0 : batch;
      ++t;
      launch_fill_f64(sloss, nb, 0.0, s);
      launch_lncc_atlas_grad(warped + static_cast<size_t>(b0) * g.V, atlas, fields, ga, sloss, 1,
                             win, eps, g, nb, s);
      if (losses) launch_sum_f64(sloss, nb, 1.0 / nb, losses + (t - 1), s);
      launch_adam_batch_mean(atlas, m, sv, ga, nb, g.V, t, lr, b1, b2, aeps, s);
    }
  }
}

}  // namespace

extern "C" {

size_t darc_atlas_sgd_ws_bytes(int n, int d0, int d1, int d2, int batch) {
  if (n < 1 || batch < 1 || d0 < 2 || d1 < 2 || d2 < 2) return 0;
  return sgd_layout(d0, d1, d2, batch < n ? batch : n).total;
}

int darc_atlas_sgd(const float* warped, float* atlas, int n, int d0, int d1, int d2, int batch,
                   int epochs, int win, float eps, float lr, double beta1, double beta2,
                   float adam_eps, double* losses, void* ws, size_t ws_bytes, void* stream) {
  DARC_TRY(check_dims("darc_atlas_sgd", n, d0, d1, d2));
  if (n < 1) return fail(DARC_EINVAL, "darc_atlas_sgd: n must be >= 1");
  DARC_TRY(check_sgd("darc_atlas_sgd", batch, epochs, win, eps, lr, beta1, beta2, adam_eps));
  if (!warped || !atlas) return fail(DARC_EINVAL, "darc_atlas_sgd: NULL pointer");
  const int b = batch < n ? batch : n;
  DARC_TRY(check_ws("darc_atlas_sgd", ws, ws_bytes, darc_atlas_sgd_ws_bytes(n, d0, d1, d2, b)));
  run_atlas_sgd(warped, atlas, n, make_geom(d0, d1, d2), b, epochs, win, eps, lr, beta1, beta2,
                adam_eps, losses, static_cast<char*>(ws), as_stream(stream));
  return check_launch("darc_atlas_sgd");
}

// ------------------------------------------------- one-shot segmentation

int darc_warp_labels(const unsigned char* labels, const float* u, unsigned char* out, int n,
                     int d0, int d1, int d2, void* stream) {
  DARC_TRY(check_dims("darc_warp_labels", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!labels || !u || !out) return fail(DARC_EINVAL, "darc_warp_labels: NULL pointer");
  launch_warp_labels(labels, u, out, make_geom(d0, d1, d2), n, as_stream(stream));
  return check_launch("darc_warp_labels");
}

size_t darc_segment_ws_bytes(int n, int d0, int d1, int d2, int n_sq) {
  if (n <= 0 || n_sq < 1 || n_sq > 16 || d0 < 2 || d1 < 2 || d2 < 2) return 0;
  return (n_sq >= 2 ? 2 : 1) * align256(field_bytes(n, d0, d1, d2));
}

int darc_segment(const unsigned char* labels, const float* v, unsigned char* out, int n, int d0,
                 int d1, int d2, int n_sq, void* ws, size_t ws_bytes, void* stream) {
  DARC_TRY(check_dims("darc_segment", n, d0, d1, d2));
  if (n_sq < 1 || n_sq > 16) return fail(DARC_EINVAL, "darc_segment: n_sq must be in 1..16");
  if (n == 0) return ok();
  if (!labels || !v || !out) return fail(DARC_EINVAL, "darc_segment: NULL pointer");
  DARC_TRY(check_ws("darc_segment", ws, ws_bytes, darc_segment_ws_bytes(n, d0, d1, d2, n_sq)));
  const Geom g = make_geom(d0, d1, d2);
  hipStream_t st = as_stream(stream);
  float* u = static_cast<float*>(ws);
  float* tmp = n_sq >= 2
                   ? reinterpret_cast<float*>(static_cast<char*>(ws) +
                                              align256(field_bytes(n, d0, d1, d2)))
                   : nullptr;
  run_exp_fwd(v, u, nullptr, tmp, nullptr, g, n, n_sq, st, /*negate=*/true);
  launch_warp_labels(labels, u, out, g, n, st);
  return check_launch("darc_segment");
}

int darc_dice_counts(const unsigned char* a, const unsigned char* b, int n, long long V,
                     int num_labels, unsigned long long* counts, void* stream) {
  if (n < 0 || V < 0) return fail(DARC_EINVAL, "darc_dice_counts: n and V must be >= 0");
  if (V > (1ll << 40)) return fail(DARC_EINVAL, "darc_dice_counts: V above 2^40");
  if (n > 65535) return fail(DARC_EINVAL, "darc_dice_counts: n above 65535");
  if (num_labels < 1 || num_labels > 256)
    return fail(DARC_EINVAL, "darc_dice_counts: num_labels must be in 1..256");
  if (n == 0 || V == 0) return ok();
  if (!a || !b || !counts) return fail(DARC_EINVAL, "darc_dice_counts: NULL pointer");
  launch_dice_counts(a, b, n, V, num_labels, counts, as_stream(stream));
  return check_launch("darc_dice_counts");
}

// ------------------------------------------------------ warm-start network

int darc_conv3d_kpad(int cin, int ksize) {
  if (cin < 1 || (ksize != 1 && ksize != 3)) return 0;
  return conv_kpad(cin, ksize == 3 ? 27 : 1);
}

int darc_conv3d(const unsigned short* x0, int c0, int up0, const unsigned short* x1, int c1,
                int n, int d0, int d1, int d2, int ksize, int stride, const unsigned short* w,
                const float* bias, int cout, int act, float slope, unsigned short* y_bf16,
                float* y_f32, void* stream) {
  DARC_TRY(check_dims("darc_conv3d", n, d0, d1, d2));
  if (c0 < 8 || c0 % 8 || c1 < 0 || c1 % 8)
    return fail(DARC_EINVAL, "darc_conv3d: channel counts must be multiples of 8 (c0 >= 8)");
  if (ksize != 1 && ksize != 3) return fail(DARC_EINVAL, "darc_conv3d: ksize must be 1 or 3");
  if (stride != 1 && stride != 2) return fail(DARC_EINVAL, "darc_conv3d: stride must be 1 or 2");
  if (cout < 1 || cout > 4096) return fail(DARC_EINVAL, "darc_conv3d: cout must be in 1..4096");
  if (up0 && (d0 % 2 || d1 % 2 || d2 % 2))
    return fail(DARC_EINVAL, "darc_conv3d: an upsampled x0 needs even dims");
  if ((y_bf16 == nullptr) == (y_f32 == nullptr))
    return fail(DARC_EINVAL, "darc_conv3d: exactly one of y_bf16 and y_f32 must be given");
  if (n == 0) return ok();
  if (!x0 || (c1 && !x1) || !w) return fail(DARC_EINVAL, "darc_conv3d: NULL pointer");
  ConvGeom cg{};
  cg.i0 = d0;
  cg.i1 = d1;
  cg.i2 = d2;
  cg.o0 = (d0 - 1) / stride + 1;
  cg.o1 = (d1 - 1) / stride + 1;
  cg.o2 = (d2 - 1) / stride + 1;
  cg.nvox = static_cast<long long>(n) * cg.o0 * cg.o1 * cg.o2;
  cg.stride = stride;
  cg.ntaps = ksize == 3 ? 27 : 1;
  cg.c0 = c0;
  cg.c1 = c1;
  cg.up0 = up0 ? 1 : 0;
  cg.kpad = conv_kpad(c0 + c1, cg.ntaps);
  cg.cout = cout;
  cg.act = act ? 1 : 0;
  cg.slope = slope;
  launch_conv3d(x0, x1, w, bias, y_bf16, y_f32, cg, as_stream(stream));
  return check_launch("darc_conv3d");
}

int darc_conv3d_grad(const unsigned short* dz, int cz, const unsigned short* x0, int c0, int up0,
                     const unsigned short* x1, int c1, int n, int d0, int d1, int d2, int stride,
                     const float* w, int cout, float* dw, float* db, float* dx,
                     unsigned short* wt, void* stream) {
  DARC_TRY(check_dims("darc_conv3d_grad", n, d0, d1, d2));
  if (c0 < 8 || c0 % 8 || c1 < 0 || c1 % 8 || cz < 8 || cz % 8 || cout < 1 || cout > cz)
    return fail(DARC_EINVAL, "darc_conv3d_grad: bad channel counts");
  if (stride != 1 && stride != 2) return fail(DARC_EINVAL, "darc_conv3d_grad: stride must be 1 or 2");
  if ((up0 || stride == 2) && (d0 % 2 || d1 % 2 || d2 % 2))
    return fail(DARC_EINVAL, "darc_conv3d_grad: odd dims with upsampling or stride 2");
  if (n == 0) return ok();
  if (!dz || !x0 || (c1 && !x1) || !w || !dw || (dx && !wt))
    return fail(DARC_EINVAL, "darc_conv3d_grad: NULL pointer");
  hipStream_t st = as_stream(stream);
  ConvGeom cg{};
  cg.i0 = d0;
  cg.i1 = d1;
  cg.i2 = d2;
  cg.stride = stride;
  cg.o0 = (d0 - 1) / stride + 1;
  cg.o1 = (d1 - 1) / stride + 1;
  cg.o2 = (d2 - 1) / stride + 1;
  cg.nvox = static_cast<long long>(n) * cg.o0 * cg.o1 * cg.o2;
  cg.ntaps = 27;
  cg.c0 = c0;
  cg.c1 = c1;
  cg.up0 = up0 ? 1 : 0;
  cg.kpad = conv_kpad(c0 + c1, 27);
  cg.cout = cout;
  launch_conv_wgrad(dz, cz, x0, x1, cg, dw, db, st);
  if (dx) {
    const int kt = conv_kpad(cz, 27);
    launch_pack_wt(w, c0 + c1, cout, cz, cg.kpad, kt, wt, st);
    ConvGeom g{};
    g.i0 = g.o0 = d0;
    g.i1 = g.o1 = d1;
    g.i2 = g.o2 = d2;
    g.nvox = static_cast<long long>(n) * d0 * d1 * d2;
    g.stride = 1;
    g.ntaps = 27;
    g.c0 = cz;
    g.dil0 = stride == 2;
    g.kpad = kt;
    g.cout = c0 + c1;
    g.ycl32 = 1;
    launch_conv3d(dz, nullptr, wt, nullptr, nullptr, dx, g, st);
  }
  return check_launch("darc_conv3d_grad");
}

}  // extern "C"

namespace {

struct UnetLayer {
  int cin, cout, stride, act;  // cin padded to a multiple of 8
};
// e0 e1 e2 e3 d2 d1 d0 out
const UnetLayer kUnet[8] = {{8, 16, 1, 1},   {16, 32, 2, 1}, {32, 64, 2, 1}, {64, 128, 2, 1},
                            {192, 64, 1, 1}, {96, 32, 1, 1}, {48, 16, 1, 1}, {16, 3, 1, 0}};

// Scratch of the network: BF16 activations (forward), then for training the
// prediction, two BF16 output gradients, one BF16 weight pack and the FP32
// gradients of the skip outputs.
struct UnetWs {
  size_t x, e0, e1, e2, e3, d2, d1, d0, fwd;                   // forward part
  size_t vp, dz, dz2, wt, ge2, ge1, ge0, total;  // training part
};

UnetWs unet_ws(int n, int d0, int d1, int d2) {
  const size_t V = static_cast<size_t>(d0) * d1 * d2 * n;
  UnetWs L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t h = sizeof(uint16_t), f = sizeof(float);
  L.x = take(V * 8 * h);
  L.e0 = take(V * 16 * h);
  L.e1 = take(V / 8 * 32 * h);
  L.e2 = take(V / 64 * 64 * h);
  L.e3 = take(V / 512 * 128 * h);
  L.d2 = take(V / 64 * 64 * h);
  L.d1 = take(V / 8 * 32 * h);
  L.d0 = take(V * 16 * h);
  L.fwd = off;
  L.vp = take(V * 3 * f);
  L.dz = take(V * 16 * h);
  L.dz2 = take(V * 16 * h);
  L.wt = take(static_cast<size_t>(192) * conv_kpad(64, 27) * h);
  // FP32 gradients of the skip outputs, accumulated from two convolutions
  L.ge2 = take(V / 64 * 64 * f);
  L.ge1 = take(V / 8 * 32 * f);
  L.ge0 = take(V * 16 * f);
  L.total = off;
  return L;
}

// Per layer: inputs (x0 with c0 channels, optionally doubled; x1 with c1),
// input level, BF16 output (or the FP32 velocity), and the forward geometry.
struct UnetStep {
  const uint16_t *x0, *x1;
  int c0, c1, up0, lev;
  uint16_t* y;
  ConvGeom cg;
  size_t wo, bo;
};

void unet_plan(char* base, const UnetWs& L, int n, int d0, int d1, int d2, UnetStep (&P)[8]) {
  auto buf = [&](size_t o) { return reinterpret_cast<uint16_t*>(base + o); };
  const struct {
    size_t x0;
    int c0, up0;
    size_t x1;
    int c1, lev;
    size_t y;
  } T[8] = {{L.x, 8, 0, 0, 0, 0, L.e0},       {L.e0, 16, 0, 0, 0, 0, L.e1},
            {L.e1, 32, 0, 0, 0, 1, L.e2},     {L.e2, 64, 0, 0, 0, 2, L.e3},
            {L.e3, 128, 1, L.e2, 64, 2, L.d2}, {L.d2, 64, 1, L.e1, 32, 1, L.d1},
            {L.d1, 32, 1, L.e0, 16, 0, L.d0}, {L.d0, 16, 0, 0, 0, 0, 0}};
  size_t wo = 0, bo = 0;
  for (int l = 0; l < 8; ++l) {
    const UnetLayer& U = kUnet[l];
    UnetStep& S = P[l];
    S.x0 = buf(T[l].x0);
    S.x1 = T[l].c1 ? buf(T[l].x1) : nullptr;
    S.c0 = T[l].c0;
    S.c1 = T[l].c1;
    S.up0 = T[l].up0;
    S.lev = T[l].lev;
    S.y = l < 7 ? buf(T[l].y) : nullptr;
    ConvGeom cg{};
    cg.i0 = d0 >> S.lev;
    cg.i1 = d1 >> S.lev;
    cg.i2 = d2 >> S.lev;
    cg.stride = U.stride;
    cg.o0 = (cg.i0 - 1) / U.stride + 1;
    cg.o1 = (cg.i1 - 1) / U.stride + 1;
    cg.o2 = (cg.i2 - 1) / U.stride + 1;
    cg.nvox = static_cast<long long>(n) * cg.o0 * cg.o1 * cg.o2;
    cg.ntaps = 27;
    cg.c0 = S.c0;
    cg.c1 = S.c1;
    cg.up0 = S.up0;
    cg.kpad = conv_kpad(U.cin, 27);
    cg.cout = U.cout;
    cg.act = U.act;
    cg.slope = 0.2f;
    S.cg = cg;
    S.wo = wo;
    S.bo = bo;
    wo += static_cast<size_t>(U.cout) * cg.kpad;
    bo += U.cout;
  }
}

void unet_run_forward(const uint16_t* w, const float* b, const float* atlas, const float* images,
                      float* v, int n, int d0, int d1, int d2, char* base, const UnetWs& L,
                      const UnetStep (&P)[8], hipStream_t st) {
  launch_pack_pair(atlas, images, reinterpret_cast<uint16_t*>(base + L.x),
                   static_cast<long long>(d0) * d1 * d2, n, 8, st);
  for (int l = 0; l < 8; ++l)
    launch_conv3d(P[l].x0, P[l].x1, w + P[l].wo, b + P[l].bo, P[l].y, l == 7 ? v : nullptr,
                  P[l].cg, st);
}

size_t unet_num_weights() {
  size_t t = 0;
  for (const UnetLayer& U : kUnet) t += static_cast<size_t>(U.cout) * conv_kpad(U.cin, 27);
  return t;
}

int unet_num_biases() {
  int t = 0;
  for (const UnetLayer& U : kUnet) t += U.cout;
  return t;
}

int check_unet(const char* fn, int n, int d0, int d1, int d2) {
  DARC_TRY(check_dims(fn, n, d0, d1, d2));
  if (d0 % 8 || d1 % 8 || d2 % 8 || d0 < 8 || d1 < 8 || d2 < 8)
    return fail(DARC_EINVAL, "%s: dims must be multiples of 8", fn);
  return DARC_OK;
}

// Gradient of the mean squared error of the prediction against v_target
// with respect to the FP32 weights: dw, db overwritten; loss += the error.
void unet_run_backward(const uint16_t* wq, const float* w, const float* b, const float* atlas,
                       const float* images, const float* target, int n, int d0, int d1, int d2,
                       char* base, const UnetWs& L, const UnetStep (&P)[8], float* dw, float* db,
                       double* loss, float* vpred, hipStream_t st) {
  auto f32 = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
  auto b16 = [&](size_t o) { return reinterpret_cast<uint16_t*>(base + o); };
  float* vp = vpred ? vpred : f32(L.vp);
  unet_run_forward(wq, b, atlas, images, vp, n, d0, d1, d2, base, L, P, st);
  const long long V = static_cast<long long>(d0) * d1 * d2;
  launch_fill_f32(dw, static_cast<long long>(unet_num_weights()), 0.0f, st);
  launch_fill_f32(db, unet_num_biases(), 0.0f, st);
  // FP32 gradients where a layer's output gradient has two sources (the
  // skip outputs e0, e1, e2); the others pass to the next layer fused into
  // BF16 (below)
  float* dy[7] = {f32(L.ge0), f32(L.ge1), f32(L.ge2), nullptr, nullptr, nullptr, nullptr};
  // BF16 output gradients of consecutive layers alternate between two
  // buffers: the input-gradient convolution of layer l reads layer l's and
  // writes layer l-1's, the activation adjoint fused into its epilogue
  uint16_t* dzb[2] = {b16(L.dz), b16(L.dz2)};
  uint16_t* wt = b16(L.wt);
  for (int l = 7; l >= 0; --l) {
    const UnetStep& S = P[l];
    const UnetLayer& U = kUnet[l];
    const int cz = (U.cout + 7) / 8 * 8;
    uint16_t* dz = dzb[(7 - l) & 1];
    // the output layer's gradient comes from the loss, written as BF16 by
    // the loss kernel (the output layer has no activation)
    if (l == 7) launch_mse_dz(vp, target, n, V, U.cout, cz, loss, dz, st);
    launch_conv_wgrad(dz, cz, S.x0, S.x1, S.cg, dw + S.wo, db + S.bo, st);
    if (l == 0) break;
    // input gradient: a stride-1 convolution of dz (on the dilated grid for
    // stride-2 layers) with flipped taps and exchanged channels
    const int kt = conv_kpad(cz, 27);
    launch_pack_wt(w + S.wo, U.cin, U.cout, cz, S.cg.kpad, kt, wt, st);
    ConvGeom g{};
    g.i0 = S.cg.i0;
    g.i1 = S.cg.i1;
    g.i2 = S.cg.i2;
    g.o0 = g.i0;
    g.o1 = g.i1;
    g.o2 = g.i2;
    g.nvox = static_cast<long long>(n) * g.i0 * g.i1 * g.i2;
    g.stride = 1;
    g.ntaps = 27;
    g.c0 = cz;
    g.c1 = 0;
    g.dil0 = U.stride == 2;
    g.kpad = kt;
    g.cout = U.cin;
    g.ycl32 = 1;
    g.slope = 0.2f;  // of layer l-1's leaky ReLU (every layer before the output's has one)
    uint16_t* dzn = dzb[(8 - l) & 1];
    if (S.c1) {  // concatenated input: split into the deeper and the skip tensor
      // layer 4 reads (e3, e2), layer 5 (d2, e1), layer 6 (d1, e0); the
      // epilogue writes the skip channels straight into their gradient and
      // sums the deeper tensor's channels over the 2 x 2 x 2 children of
      // each voxel of its half resolution (layer l-1's output), passed
      // through that layer's activation adjoint
      g.csplit = S.c0;
      g.y32b = dy[6 - l];
      g.hpool = 1;
      g.dz16 = dzn;
      g.acty = P[l - 1].y;
      launch_conv3d(dz, nullptr, wt, nullptr, nullptr, nullptr, g, st);
    } else {
      // the output layer (its input is d0), or a stride-2 encoder layer,
      // whose input's gradient already holds the skip part (accumulated)
      g.accum = l != 7;
      g.dz16 = dzn;
      g.acty = P[l - 1].y;
      launch_conv3d(dz, nullptr, wt, nullptr, nullptr, dy[l - 1], g, st);
    }
  }
}

}  // namespace

extern "C" {

int darc_unet_layout(int layer, int* cin, int* cout, int* kpad, size_t* w_offset,
                     size_t* b_offset) {
  if (layer < 0 || layer >= 8) return fail(DARC_EINVAL, "darc_unet_layout: layer must be 0..7");
  size_t wo = 0, bo = 0;
  for (int l = 0; l < layer; ++l) {
    wo += static_cast<size_t>(kUnet[l].cout) * conv_kpad(kUnet[l].cin, 27);
    bo += kUnet[l].cout;
  }
  if (cin) *cin = kUnet[layer].cin;
  if (cout) *cout = kUnet[layer].cout;
  if (kpad) *kpad = conv_kpad(kUnet[layer].cin, 27);
  if (w_offset) *w_offset = wo;
  if (b_offset) *b_offset = bo;
  return ok();
}

size_t darc_unet_num_weights(void) { return unet_num_weights(); }
int darc_unet_num_biases(void) { return unet_num_biases(); }

size_t darc_unet_ws_bytes(int n, int d0, int d1, int d2) {
  if (n < 1 || d0 < 8 || d1 < 8 || d2 < 8 || d0 % 8 || d1 % 8 || d2 % 8) return 0;
  return unet_ws(n, d0, d1, d2).fwd;
}

size_t darc_unet_train_ws_bytes(int n, int d0, int d1, int d2) {
  if (n < 1 || d0 < 8 || d1 < 8 || d2 < 8 || d0 % 8 || d1 % 8 || d2 % 8) return 0;
  return unet_ws(n, d0, d1, d2).total;
}

int darc_unet_forward(const unsigned short* w, const float* b, const float* atlas,
                      const float* images, float* v, int n, int d0, int d1, int d2, void* ws,
                      size_t ws_bytes, void* stream) {
  DARC_TRY(check_unet("darc_unet_forward", n, d0, d1, d2));
  if (n == 0) return ok();
  if (!w || !b || !atlas || !images || !v) return fail(DARC_EINVAL, "darc_unet_forward: NULL pointer");
  DARC_TRY(check_ws("darc_unet_forward", ws, ws_bytes, darc_unet_ws_bytes(n, d0, d1, d2)));
  const UnetWs L = unet_ws(n, d0, d1, d2);
  UnetStep P[8];
  char* base = static_cast<char*>(ws);
  unet_plan(base, L, n, d0, d1, d2, P);
  unet_run_forward(w, b, atlas, images, v, n, d0, d1, d2, base, L, P, as_stream(stream));
  return check_launch("darc_unet_forward");
}

int darc_unet_backward(const unsigned short* wq, const float* w, const float* b,
                       const float* atlas, const float* images, const float* v_target,
                       float* dw, float* db, double* loss, float* v_pred, int n, int d0, int d1,
                       int d2, void* ws, size_t ws_bytes, void* stream) {
  DARC_TRY(check_unet("darc_unet_backward", n, d0, d1, d2));
  if (n < 1) return fail(DARC_EINVAL, "darc_unet_backward: n must be >= 1");
  if (!wq || !w || !b || !atlas || !images || !v_target || !dw || !db || !loss)
    return fail(DARC_EINVAL, "darc_unet_backward: NULL pointer");
  DARC_TRY(check_ws("darc_unet_backward", ws, ws_bytes, darc_unet_train_ws_bytes(n, d0, d1, d2)));
  const UnetWs L = unet_ws(n, d0, d1, d2);
  UnetStep P[8];
  char* base = static_cast<char*>(ws);
  unet_plan(base, L, n, d0, d1, d2, P);
  unet_run_backward(wq, w, b, atlas, images, v_target, n, d0, d1, d2, base, L, P, dw, db, loss,
                    v_pred, as_stream(stream));
  return check_launch("darc_unet_backward");
}

int darc_unet_train_step(darc_unet_train* t, const float* atlas, const float* images,
                         const float* v_target, float lr, double beta1, double beta2, float eps,
                         double* loss, int n, int d0, int d1, int d2, void* ws, size_t ws_bytes,
                         void* stream) {
  DARC_TRY(check_unet("darc_unet_train_step", n, d0, d1, d2));
  if (!t || !t->w || !t->b || !t->mw || !t->sw || !t->mb || !t->sb || !t->wq || !t->dw || !t->db)
    return fail(DARC_EINVAL, "darc_unet_train_step: NULL pointer in the training state");
  if (t->step < 0) return fail(DARC_EINVAL, "darc_unet_train_step: step must be >= 0");
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0f))
    return fail(DARC_EINVAL, "darc_unet_train_step: bad Adam constants");
  DARC_TRY(darc_unet_backward(t->wq, t->w, t->b, atlas, images, v_target, t->dw, t->db, loss,
                              nullptr, n, d0, d1, d2, ws, ws_bytes, stream));
  hipStream_t st = as_stream(stream);
  const long long nw = static_cast<long long>(unet_num_weights());
  launch_adam(t->w, t->w, t->mw, t->sw, t->dw, nw, t->step + 1, lr, beta1, beta2, eps, st);
  launch_adam(t->b, t->b, t->mb, t->sb, t->db, unet_num_biases(), t->step + 1, lr, beta1, beta2,
              eps, st);
  launch_to_bf16(t->w, t->wq, nw, st);
  t->step += 1;
  return check_launch("darc_unet_train_step");
}

// ------------------------------------------------------------- resampling

int darc_down2(const float* in, float* out, int nchan, int d0, int d1, int d2, void* stream) {
  DARC_TRY(check_dims("darc_down2", nchan, d0, d1, d2));
  if (d0 % 2 || d1 % 2 || d2 % 2 || d0 < 4 || d1 < 4 || d2 < 4)
    return fail(DARC_EINVAL, "darc_down2: fine dims must be even and >= 4");
  if (nchan == 0) return ok();
  if (!in || !out || in == out) return fail(DARC_EINVAL, "darc_down2: bad pointers");
  launch_down2(in, out, make_geom(d0, d1, d2), nchan, as_stream(stream));
  return check_launch("darc_down2");
}

int darc_up2(const float* in, float* out, int nchan, int d0, int d1, int d2, float scale,
             void* stream) {
  DARC_TRY(check_dims("darc_up2", nchan, d0, d1, d2));
  if (d0 % 2 || d1 % 2 || d2 % 2 || d0 < 4 || d1 < 4 || d2 < 4)
    return fail(DARC_EINVAL, "darc_up2: fine dims must be even and >= 4");
  if (nchan == 0) return ok();
  if (!in || !out || in == out) return fail(DARC_EINVAL, "darc_up2: bad pointers");
  launch_up2(in, out, make_geom(d0, d1, d2), nchan, scale, as_stream(stream));
  return check_launch("darc_up2");
}

}  // extern "C"

// ------------------------------------------------------------------- sweep

namespace {

struct SweepLayout {
  int B;
  size_t ckpt, aux, uN, gU, gA, gB, gV, iw, fields, vtmp, uhat, sloss, bc, wall, sgd, bar, total;
};

SweepLayout sweep_layout(const darc_state* st, const darc_params* p) {
  SweepLayout L{};
  const int n = st->n;
  L.B = (p->batch <= 0 || p->batch > n) ? n : p->batch;
  const size_t V = static_cast<size_t>(st->d0) * st->d1 * st->d2;
  const size_t fb = static_cast<size_t>(L.B) * 3 * V * sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.ckpt = take(p->n_sq >= 2 ? static_cast<size_t>(p->n_sq - 1) * fb : 0);
  L.aux = take(exp_aux_bytes(make_geom(st->d0, st->d1, st->d2), L.B, p->n_sq));
  L.uN = take(fb);
  L.gU = take(fb);
  L.gA = take(fb);
  L.gB = take(fb);
  L.gV = take(fb);
  const bool lncc = p->metric == DARC_LNCC;
  L.iw = take(lncc ? static_cast<size_t>(L.B) * V * sizeof(float) : 0);
  L.fields = take(lncc ? static_cast<size_t>(L.B) * 4 * V * sizeof(float) : 0);
  L.vtmp = take(p->smooth_sigma > 0.0f ? fb : 0);
  L.uhat = take(st->u_hat ? 0 : static_cast<size_t>(n) * 3 * V * sizeof(float));
  L.sloss = take(static_cast<size_t>(n) * sizeof(double));
  L.bc = take(static_cast<size_t>(p->k2) * 2 * sizeof(float));
  const bool sgd = p->atlas_mode == DARC_ATLAS_SGD;
  const int ab = p->atlas_batch < n ? p->atlas_batch : n;
  L.wall = take(sgd ? static_cast<size_t>(n) * V * sizeof(float) : 0);
  L.sgd = take(sgd ? sgd_layout(st->d0, st->d1, st->d2, ab).total : 0);
  L.bar = take(2 * sizeof(int));  // barrier counter and error flag of the fused iteration
  L.total = off;
  return L;
}

int check_sweep(const darc_state* st, const darc_params* p) {
  if (!st || !p) return fail(DARC_EINVAL, "darc_sweep: state and params must not be NULL");
  DARC_TRY(check_dims("darc_sweep", st->n, st->d0, st->d1, st->d2));
  if (st->n < 1) return fail(DARC_EINVAL, "darc_sweep: n must be >= 1");
  if (!st->images || !st->v || !st->m || !st->s || !st->atlas)
    return fail(DARC_EINVAL, "darc_sweep: images, v, m, s and atlas must not be NULL");
  if (p->metric != DARC_MSE && p->metric != DARC_LNCC && p->metric != DARC_L1)
    return fail(DARC_EINVAL, "darc_sweep: unknown metric %d", p->metric);
  if (p->metric == DARC_LNCC) {
    if (p->win < 1 || p->win % 2 == 0)
      return fail(DARC_EINVAL, "darc_sweep: window %d must be odd and positive", p->win);
    if (!lncc_window_supported(p->win))
      return fail(DARC_EUNSUPPORTED, "darc_sweep: window %d not built (3, 5, 7, 9, 11)", p->win);
    if (!(p->ncc_eps > 0.0f)) return fail(DARC_EINVAL, "darc_sweep: ncc_eps must be > 0");
  }
  if (!(p->lam >= 0.0f)) return fail(DARC_EINVAL, "darc_sweep: lam must be >= 0");
  if (!(p->smooth_sigma >= 0.0f)) return fail(DARC_EINVAL, "darc_sweep: smooth_sigma must be >= 0");
  if (p->smooth_sigma > 0.0f) {
    const int r = gauss_radius(p->smooth_sigma);
    if (r < 1 || r > 8)
      return fail(DARC_EUNSUPPORTED, "darc_sweep: Gaussian radius %d not in 1..8", r);
  }
  if (p->n_sq < 1 || p->n_sq > 16) return fail(DARC_EINVAL, "darc_sweep: n_sq must be in 1..16");
  if (p->k2 < 0) return fail(DARC_EINVAL, "darc_sweep: k2 must be >= 0");
  if (p->atlas_mode == DARC_ATLAS_MEDIAN) {
    if (median_threads(st->n) == 0)
      return fail(DARC_EUNSUPPORTED, "darc_sweep: median atlas of n = %d > 512 subjects", st->n);
  } else if (p->atlas_mode == DARC_ATLAS_SGD) {
    if (p->metric != DARC_LNCC)
      return fail(DARC_EINVAL, "darc_sweep: the stochastic atlas update is for the LNCC metric");
    DARC_TRY(check_sgd("darc_sweep", p->atlas_batch, p->k3, p->win, p->ncc_eps, p->atlas_lr,
                       p->beta1, p->beta2, p->adam_eps));
    if (p->sgd_init != DARC_SGD_INIT_WARM && p->sgd_init != DARC_SGD_INIT_INITIAL)
      return fail(DARC_EINVAL, "darc_sweep: unknown sgd_init %d", p->sgd_init);
  } else if (p->atlas_mode != DARC_ATLAS_MEAN) {
    return fail(DARC_EINVAL, "darc_sweep: unknown atlas_mode %d", p->atlas_mode);
  }
  if (!(p->beta1 >= 0.0 && p->beta1 < 1.0 && p->beta2 >= 0.0 && p->beta2 < 1.0))
    return fail(DARC_EINVAL, "darc_sweep: betas must lie in [0, 1)");
  if (!(p->adam_eps > 0.0f)) return fail(DARC_EINVAL, "darc_sweep: adam_eps must be > 0");
  if (p->center_mode != DARC_CENTER_DISPLACEMENT && p->center_mode != DARC_CENTER_VELOCITY)
    return fail(DARC_EINVAL, "darc_sweep: unknown center_mode %d", p->center_mode);
  if (st->step < 0) return fail(DARC_EINVAL, "darc_sweep: step must be >= 0");
  if (p->fused != DARC_FUSED_AUTO && p->fused != DARC_FUSED_OFF && p->fused != DARC_FUSED_ON)
    return fail(DARC_EINVAL, "darc_sweep: unknown fused mode %d", p->fused);
  if (p->fused == DARC_FUSED_ON && (p->metric == DARC_LNCC || p->smooth_sigma > 0.0f))
    return fail(DARC_EUNSUPPORTED,
                "darc_sweep: the fused iteration covers MSE and L1 without smoothing of v");
  return DARC_OK;
}

// Whether a sweep batch of B subjects runs its inner iterations fused.
// DARC_FUSED_AUTO follows the autotuner's choice for the shape, and without
// one takes separate launches: on this GPU a grid barrier costs 5-8 us at 64-
// 128 blocks (every block's agent-scope fence writes back its XCD's L2), so
// the 16 barriers of an iteration outweigh the launches they replace (4 x
// 32^3: 1.79 ms per fused sweep against 0.78 separate).
bool use_fused(const darc_params* p, const Geom& g, int B) {
  if (p->fused == DARC_FUSED_OFF || p->metric == DARC_LNCC || p->smooth_sigma > 0.0f)
    return false;
  if (fused_resident_blocks(p->metric == DARC_L1) < 8) return false;
  if (p->fused == DARC_FUSED_ON) return true;
  return tuned_tz(TUNE_FUSED, g, B) == 1;
}

}  // namespace

extern "C" {

size_t darc_sizeof_state(void) { return sizeof(darc_state); }
size_t darc_sizeof_params(void) { return sizeof(darc_params); }

size_t darc_sweep_ws_bytes(const darc_state* st, const darc_params* p) {
  if (check_sweep(st, p) != DARC_OK) return 0;
  return sweep_layout(st, p).total;
}

int darc_sweep(darc_state* st, const darc_params* p, double* losses, void* ws, size_t ws_bytes,
               void* stream) {
  DARC_TRY(check_sweep(st, p));
  if (!losses) return fail(DARC_EINVAL, "darc_sweep: losses must not be NULL");
  const SweepLayout L = sweep_layout(st, p);
  DARC_TRY(check_ws("darc_sweep", ws, ws_bytes, L.total));
  hipStream_t s = as_stream(stream);
  const Geom g = make_geom(st->d0, st->d1, st->d2);
  const int n = st->n, k2 = p->k2, N = p->n_sq, B = L.B;
  const size_t fsv = 3 * static_cast<size_t>(g.V);
  char* w = static_cast<char*>(ws);
  float* ckpt = N >= 2 ? reinterpret_cast<float*>(w + L.ckpt) : nullptr;
  int* aux = reinterpret_cast<int*>(w + L.aux);
  float* uN = reinterpret_cast<float*>(w + L.uN);
  float* gU = reinterpret_cast<float*>(w + L.gU);
  float* gA = reinterpret_cast<float*>(w + L.gA);
  float* gB = reinterpret_cast<float*>(w + L.gB);
  float* gV = reinterpret_cast<float*>(w + L.gV);
  float* iw = reinterpret_cast<float*>(w + L.iw);
  float* fields = reinterpret_cast<float*>(w + L.fields);
  float* vtmp = reinterpret_cast<float*>(w + L.vtmp);
  float* uh = st->u_hat ? st->u_hat : reinterpret_cast<float*>(w + L.uhat);
  double* sloss = reinterpret_cast<double*>(w + L.sloss);
  float* bc = reinterpret_cast<float*>(w + L.bc);
  const RegW rw = make_regw(g, 3, p->lam);
  const bool lncc = p->metric == DARC_LNCC;
  const bool l1 = p->metric == DARC_L1;
  const bool smooth = p->smooth_sigma > 0.0f;

  launch_fill_f64(losses, static_cast<long long>(n) * k2 + 1, 0.0, s);
  long long step = st->step;
  const bool fused = use_fused(p, g, B);
  if (p->fused == DARC_FUSED_ON && !fused)
    return fail(DARC_EHIP, "darc_sweep: the fused iteration cannot be made resident");
  unsigned* bar = reinterpret_cast<unsigned*>(w + L.bar);
  int* err = reinterpret_cast<int*>(w + L.bar) + 1;
  if (fused) launch_fill_f32(reinterpret_cast<float*>(err), 1, 0.0f, s);
  if (p->reinit_v) {
    const long long cnt = static_cast<long long>(n) * fsv;
    launch_fill_f32(st->v, cnt, 0.0f, s);
    launch_fill_f32(st->m, cnt, 0.0f, s);
    launch_fill_f32(st->s, cnt, 0.0f, s);
    if (st->step_dev) launch_fill_f64(reinterpret_cast<double*>(st->step_dev), 1, 0.0, s);
    step = 0;
  }

  // step 1: K2 gradient steps per subject against the fixed atlas; subjects
  // are independent, so a launch covers a batch of them.
  for (int b0 = 0; b0 < n; b0 += B) {
    const int nb = n - b0 < B ? n - b0 : B;
    float* vb = st->v + b0 * fsv;
    float* mb = st->m + b0 * fsv;
    float* sb = st->s + b0 * fsv;
    const float* ib = st->images + static_cast<size_t>(b0) * g.V;
    for (int k = 0; k < k2; ++k) {
      double* lslot = losses + static_cast<size_t>(b0) * k2 + k;
      if (fused) {
        // one launch per inner iteration (capacity checked by use_fused)
        run_iter_fused(ib, st->atlas, vb, mb, sb, ckpt, aux, uN, gU, gA, gB, gV, lslot, k2, rw, g,
                       nb, N, st->step_dev, step, k, p->lr, p->beta1, p->beta2, p->adam_eps, l1,
                       bar, err, s);
        continue;
      }
      run_exp_fwd(vb, uN, ckpt, nullptr, aux, g, nb, N, s);
      if (!lncc) {
        launch_mse_fused(ib, st->atlas, uN, gU, lslot, k2, rw, g, nb, l1, s);
      } else {
        launch_warp(ib, uN, iw, g, nb, s);
        launch_lncc_fwd(iw, st->atlas, fields, lslot, k2, p->win, p->ncc_eps, g, nb, s);
        launch_lncc_bwd_fused(fields, iw, st->atlas, ib, uN, gU, lslot, k2, rw, p->win, g, nb, s);
      }
      run_exp_bwd(vb, ckpt, gU, gV, gA, gB, aux, true, g, nb, N, s);
      const long long cnt = static_cast<long long>(nb) * fsv;
      float* vdst = smooth ? vtmp : vb;
      if (st->step_dev)
        launch_adam_dev(vb, vdst, mb, sb, gV, cnt, st->step_dev, k, bc + 2 * k, p->lr, p->beta1,
                        p->beta2, p->adam_eps, s);
      else
        launch_adam(vb, vdst, mb, sb, gV, cnt, step + k + 1, p->lr, p->beta1, p->beta2,
                    p->adam_eps, s);
      if (smooth) launch_gauss(vtmp, vb, p->smooth_sigma, g, nb * 3, s);
    }
  }

  if (st->step_dev) launch_step_add(st->step_dev, k2, s);

  // step 2: u_i = Exp(v_i), centrality activation
  if (p->center_mode == DARC_CENTER_VELOCITY) launch_center(st->v, nullptr, g, n, s);
  for (int b0 = 0; b0 < n; b0 += B) {
    const int nb = n - b0 < B ? n - b0 : B;
    run_exp_fwd(st->v + b0 * fsv, uh + b0 * fsv, nullptr, gA, nullptr, g, nb, N, s);
  }
  if (p->center_mode == DARC_CENTER_DISPLACEMENT) launch_center(uh, nullptr, g, n, s);

  // step 3: the atlas update from the warped subjects
  if (p->atlas_mode == DARC_ATLAS_MEDIAN) {
    launch_atlas_median(st->images, uh, nullptr, st->atlas, g, n, s);
  } else if (p->atlas_mode == DARC_ATLAS_SGD) {
    float* wall = reinterpret_cast<float*>(w + L.wall);
    launch_warp(st->images, uh, wall, g, n, s);
    // Algorithm 1's A = initialize() read literally: restart from A^0
    if (p->sgd_init == DARC_SGD_INIT_INITIAL)
      launch_atlas(st->images, nullptr, nullptr, st->atlas, g, n, s);
    run_atlas_sgd(wall, st->atlas, n, g, p->atlas_batch < n ? p->atlas_batch : n, p->k3, p->win,
                  p->ncc_eps, p->atlas_lr, p->beta1, p->beta2, p->adam_eps, nullptr, w + L.sgd, s);
  } else {
    launch_atlas(st->images, uh, nullptr, st->atlas, g, n, s);
  }

  // group loss at the new atlas
  launch_fill_f64(sloss, n, 0.0, s);
  for (int b0 = 0; b0 < n; b0 += B) {
    const int nb = n - b0 < B ? n - b0 : B;
    const float* ib = st->images + static_cast<size_t>(b0) * g.V;
    if (!lncc) {
      launch_mse_fused(ib, st->atlas, uh + b0 * fsv, nullptr, sloss + b0, 1, rw, g, nb, l1, s);
    } else {
      launch_warp(ib, uh + b0 * fsv, iw, g, nb, s);
      launch_lncc_fwd(iw, st->atlas, nullptr, sloss + b0, 1, p->win, p->ncc_eps, g, nb, s);
      if (rw.on) launch_diffusion(uh + b0 * fsv, nullptr, sloss + b0, 1, rw, g, nb, 3, s);
    }
  }
  launch_sum_f64(sloss, n, 1.0 / n, losses + static_cast<size_t>(n) * k2, s);
  if (fused) flag_fused_error(err, losses + static_cast<size_t>(n) * k2, s);
  st->step = step + k2;
  return check_launch("darc_sweep");
}

// -------------------------------------------------------------- autotuning


int darc_autotune(darc_state* st, const darc_params* p, void* ws, size_t ws_bytes, void* stream,
                  int* chosen) {
  DARC_TRY(check_sweep(st, p));
  const SweepLayout L = sweep_layout(st, p);
  DARC_TRY(check_ws("darc_autotune", ws, ws_bytes, L.total));
  hipStream_t s = as_stream(stream);
  const Geom g = make_geom(st->d0, st->d1, st->d2);
  const int B = L.B, N = p->n_sq;
  char* w = static_cast<char*>(ws);
  float* ckpt = N >= 2 ? reinterpret_cast<float*>(w + L.ckpt) : nullptr;
  int* aux = reinterpret_cast<int*>(w + L.aux);
  float* uN = reinterpret_cast<float*>(w + L.uN);
  float* gU = reinterpret_cast<float*>(w + L.gU);
  float* gA = reinterpret_cast<float*>(w + L.gA);
  float* gB = reinterpret_cast<float*>(w + L.gB);
  float* gV = reinterpret_cast<float*>(w + L.gV);
  const int cands[4] = {8, 16, 32, 64};
  // the squaring kernels also try one plane per block without marching (-1)
  const int exp_cands[5] = {-1, 8, 16, 32, 64};
  int pick[2] = {0, 0};
  // squaring steps and their adjoint on the first batch (u_N stands in for dL/du)
  {
    float best = -1.0f;
    for (int tz : exp_cands) {
      set_tuned_tz(TUNE_EXP, g, B, tz);
      const float ms = time_on(s, [&] {
        run_exp_fwd(st->v, uN, ckpt, nullptr, aux, g, B, N, s);
        (void)hipMemcpyAsync(gU, uN, static_cast<size_t>(B) * 3 * g.V * sizeof(float),
                             hipMemcpyDeviceToDevice, s);
        run_exp_bwd(st->v, ckpt, gU, gV, gA, gB, aux, true, g, B, N, s);
      });
      if (ms >= 0.0f && (best < 0.0f || ms < best)) {
        best = ms;
        pick[0] = tz;
      }
    }
    set_tuned_tz(TUNE_EXP, g, B, pick[0]);
  }
  // window kernels: LNCC statistics and adjoint, or the Gaussian on v
  const bool lncc = p->metric == DARC_LNCC, smooth = p->smooth_sigma > 0.0f;
  if (lncc || smooth) {
    float* iw = reinterpret_cast<float*>(w + L.iw);
    float* fields = reinterpret_cast<float*>(w + L.fields);
    double* sloss = reinterpret_cast<double*>(w + L.sloss);
    const RegW rw = make_regw(g, 3, p->lam);
    float best = -1.0f;
    for (int tz : cands) {
      set_tuned_tz(TUNE_WINDOW, g, B, tz);
      set_tuned_tz(TUNE_WINDOW, g, 3 * B, tz);
      const float ms = time_on(s, [&] {
        if (lncc) {
          launch_warp(st->images, uN, iw, g, B, s);
          launch_lncc_fwd(iw, st->atlas, fields, sloss, 1, p->win, p->ncc_eps, g, B, s);
          launch_lncc_bwd_fused(fields, iw, st->atlas, st->images, uN, gU, sloss, 1, rw, p->win, g,
                                B, s);
        }
        if (smooth) launch_gauss(st->v, gA, p->smooth_sigma, g, 3 * B, s);
      });
      if (ms >= 0.0f && (best < 0.0f || ms < best)) {
        best = ms;
        pick[1] = tz;
      }
    }
    set_tuned_tz(TUNE_WINDOW, g, B, pick[1]);
    set_tuned_tz(TUNE_WINDOW, g, 3 * B, pick[1]);
  }
  // one inner iteration fused against separate launches (MSE / L1 without
  // smoothing); Adam's results go to scratch, so the state is left as it is
  int fused_pick = 0;
  if (!lncc && !smooth && fused_resident_blocks(p->metric == DARC_L1) >= 8) {
    const bool l1 = p->metric == DARC_L1;
    const RegW rw = make_regw(g, 3, p->lam);
    double* sloss = reinterpret_cast<double*>(w + L.sloss);
    unsigned* bar = reinterpret_cast<unsigned*>(w + L.bar);
    int* err = reinterpret_cast<int*>(w + L.bar) + 1;
    launch_fill_f32(reinterpret_cast<float*>(err), 1, 0.0f, s);
    const long long cnt = static_cast<long long>(B) * 3 * g.V;
    const float t_sep = time_on(s, [&] {
      run_exp_fwd(st->v, uN, ckpt, nullptr, aux, g, B, N, s);
      launch_mse_fused(st->images, st->atlas, uN, gU, sloss, 1, rw, g, B, l1, s);
      run_exp_bwd(st->v, ckpt, gU, gV, gA, gB, aux, true, g, B, N, s);
      launch_adam(st->v, gA, gB, uN, gV, cnt, 1, p->lr, p->beta1, p->beta2, p->adam_eps, s);
    });
    const float t_fused = time_on(s, [&] {
      run_iter_fused(st->images, st->atlas, st->v, st->m, st->s, ckpt, aux, uN, gU, gA, gB, gV,
                     sloss, 1, rw, g, B, N, nullptr, 0, 0, p->lr, p->beta1, p->beta2,
                     p->adam_eps, l1, bar, err, s, gA, gB, uN);
    });
    if (t_sep >= 0.0f && t_fused >= 0.0f) {
      fused_pick = t_fused < t_sep ? 1 : 2;
      set_tuned_tz(TUNE_FUSED, g, B, fused_pick);
    }
  }
  if (chosen) {
    chosen[0] = pick[0];
    chosen[1] = pick[1];
    chosen[2] = fused_pick;
  }
  return check_launch("darc_autotune");
}

int darc_autotune_clear(void) {
  clear_tuned();
  return ok();
}

int darc_set_launch_shape(int kind, int d0, int d1, int d2, int n, int value) {
  const bool every = d0 == 0 && d1 == 0 && d2 == 0 && n == 0;
  if (!every) DARC_TRY(check_dims("darc_set_launch_shape", n, d0, d1, d2));
  Geom g{};
  if (!every) g = make_geom(d0, d1, d2);
  bool okv = false;
  if (kind == DARC_SHAPE_SQUARING) okv = value == -1 || value == 1 || value == 8 || value == 16 ||
                                         value == 32 || value == 64 || value == 0;
  else if (kind == DARC_SHAPE_WINDOW) okv = value == 8 || value == 16 || value == 32 ||
                                            value == 64 || value == 96 || value == 0;
  else if (kind == DARC_SHAPE_FUSED) okv = value >= 0 && value <= 2;
  else return fail(DARC_EINVAL, "darc_set_launch_shape: unknown kind %d", kind);
  if (!okv) return fail(DARC_EINVAL, "darc_set_launch_shape: value %d not valid for kind %d", value,
                        kind);
  set_tuned_tz(kind, g, n, value);
  return ok();
}

int darc_fused_barrier_ticks(long long ticks) {
  set_barrier_ticks(ticks);
  return ok();
}

// ------------------------------------------------------------- timing API

int darc_profile_enable(int on) {
  g_prof_on = on != 0;
  return ok();
}

int darc_profile_reset(void) {
  for (const ProfRec& r : g_prof_recs) {
    if (r.a) g_event_pool.push_back(r.a);
    if (r.b) g_event_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  for (int i = 0; i < KC_NUM; ++i) {
    g_prof_counts[i] = 0;
    g_prof_ms[i] = 0.0;
  }
  return ok();
}

int darc_profile_num_classes(void) { return KC_NUM; }

const char* darc_profile_name(int cls) {
  if (cls < 0 || cls >= KC_NUM) return "";
  return kClassNames[cls];
}

int darc_profile_collect(long long* counts, double* ms, int max_classes) {
  for (const ProfRec& r : g_prof_recs) {
    if (r.a && r.b) {
      if (hipEventSynchronize(r.b) != hipSuccess) return check_launch("darc_profile_collect");
      float t = 0.0f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        g_prof_counts[r.cls] += 1;
        g_prof_ms[r.cls] += t;
      }
    }
    if (r.a) g_event_pool.push_back(r.a);
    if (r.b) g_event_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  const int m = max_classes < KC_NUM ? max_classes : KC_NUM;
  for (int i = 0; i < m; ++i) {
    if (counts) counts[i] = g_prof_counts[i];
    if (ms) ms[i] = g_prof_ms[i];
  }
  return ok();
}

}  // extern "C"
