// C ABI of the single-grid simulator: handle, validation, launches, hipGraph
// replay, autotuning of the step-kernel shape, checkpoints and timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace lbm {

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int validate_config(const lbm_config* c) {
  if (!c) return fail(LBM_E_INVALID, "config is NULL");
  if (c->nx < 16 || c->ny < 16 || c->nx > 65536 || c->ny > 65536)
    return fail(LBM_E_INVALID, "grid %d x %d outside [16, 65536]", c->nx, c->ny);
  if (c->dtype != LBM_F32 && c->dtype != LBM_F64)
    return fail(LBM_E_INVALID, "dtype must be LBM_F32 or LBM_F64 (got %d)", c->dtype);
  if (!(c->tau > 0.5) || !std::isfinite(c->tau))
    return fail(LBM_E_INVALID, "tau must be a finite number > 0.5 (got %g)", c->tau);
  if (!(c->drag_alpha >= 0.0) || !std::isfinite(c->drag_alpha))
    return fail(LBM_E_INVALID, "drag_alpha must be finite and >= 0 (got %g)", c->drag_alpha);
  if (c->has_force != 0 && c->has_force != 1) return fail(LBM_E_INVALID, "has_force must be 0 or 1");
  if (c->with_balance != 0 && c->with_balance != 1)
    return fail(LBM_E_INVALID, "with_balance must be 0 or 1");
  if (c->with_balance)
    if (int rc = balance_grid_ok(c->nx, c->ny)) return rc;
  if (c->layout != LBM_LAYOUT_PLANES && c->layout != LBM_LAYOUT_ROWS)
    return fail(LBM_E_INVALID, "layout must be LBM_LAYOUT_PLANES or LBM_LAYOUT_ROWS");
  if (c->force_scheme != LBM_FORCE_GUO && c->force_scheme != LBM_FORCE_EDM)
    return fail(LBM_E_INVALID, "force_scheme must be LBM_FORCE_GUO or LBM_FORCE_EDM");
  if (c->collision != LBM_COLLISION_BGK && c->collision != LBM_COLLISION_ENTROPIC)
    return fail(LBM_E_INVALID, "collision must be LBM_COLLISION_BGK or LBM_COLLISION_ENTROPIC");
  if (c->collision == LBM_COLLISION_ENTROPIC &&
      (c->has_force || c->drag_alpha != 0.0 || c->damp_f0 != 0.0 || c->force_scheme != LBM_FORCE_GUO))
    return fail(LBM_E_UNSUPPORTED, "the entropic collision runs unforced");
  if (!(c->damp_f0 >= 0.0) || !std::isfinite(c->damp_f0))
    return fail(LBM_E_INVALID, "damp_f0 must be finite and >= 0 (got %g)", c->damp_f0);
  if (c->force_scheme == LBM_FORCE_GUO) {
    if (c->damp_f0 != 0.0)
      return fail(LBM_E_INVALID, "the spectral damping needs force_scheme = LBM_FORCE_EDM");
    return LBM_OK;
  }
  if (c->drag_alpha != 0.0)
    return fail(LBM_E_UNSUPPORTED, "linear drag is not combined with the exact-difference forcing");
  if (c->damp_f0 > 0.0) {
    if (!(c->damp_kmin > 0.0) || !(c->damp_kmax >= c->damp_kmin) || !(c->damp_kmax <= kEdmMaxK))
      return fail(LBM_E_INVALID, "damped shell needs 0 < kmin <= kmax <= %d (got %g, %g)", kEdmMaxK,
                  c->damp_kmin, c->damp_kmax);
    const int m = c->nx < c->ny ? c->nx : c->ny;
    if (!(2.0 * c->damp_kmax < m))
      return fail(LBM_E_INVALID, "damped shell |k| <= %g does not fit a %d x %d grid", c->damp_kmax,
                  c->nx, c->ny);
    EdmModes md;
    if (int rc = edm_modes(*c, &md)) return rc;
  }
  return LBM_OK;
}

size_t elem_size(int dtype) { return dtype == LBM_F32 ? 4 : 8; }

}  // namespace lbm

using namespace lbm;

struct lbm_ctx_s {
  lbm_config cfg{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  void* pop[2] = {nullptr, nullptr};
  int cur = 0;
  void* fx = nullptr;
  void* fy = nullptr;
  double* hist[2][3] = {{nullptr}};
  int64_t hist_t[2] = {-1, -1};
  double* mom[3] = {nullptr, nullptr, nullptr};
  double* ftot[2] = {nullptr, nullptr};
  double* partials = nullptr;
  double* scalars_dev = nullptr;
  BalanceWs bal{};
  int64_t t = 0;
  lbm_tile tile{};   // shape of the bulk of the steps (one or two steps per launch)
  lbm_tile tile1{};  // single-step shape for history-recording and odd steps
  int graph_chunk = 64;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  double timed_ms = 0.0;
  int64_t timed_launches = 0;
  int64_t pending_launches = 0;
  size_t plane = 0;
  PopLayout lay{};
  EdmModes edm_md{};  // damped modes (exact-difference scheme)
  EdmWs edm{};
  // balance running beside the steps (lbm_balance_begin / lbm_balance_end)
  hipStream_t bal_stream = nullptr;
  hipEvent_t bal_snap = nullptr, bal_done = nullptr;
  double* bal_host = nullptr;  // pinned statistics of the running balance, then its 8 moment scalars
  bool bal_pending = false;
  int64_t bal_t = 0;
  std::vector<int32_t> bal_sizes;
};

namespace {

struct Layout {
  void* pop[2];
  void* fx;
  void* fy;
  double* hist[2][3];
  double* mom[3];
  double* ftot[2];
  double* partials;
  double* scalars;
  BalanceWs bal;
  EdmWs edm;
  size_t bytes;
};

Layout carve_ctx(const lbm_config& c, void* base, size_t cap) {
  Carver cv(base, cap);
  const size_t plane = static_cast<size_t>(c.nx) * c.ny;
  const size_t es = elem_size(c.dtype);
  Layout l{};
  for (int b = 0; b < 2; ++b) l.pop[b] = cv.take<char>(9 * plane * es);
  if (c.has_force) {
    l.fx = cv.take<char>(plane * es);
    l.fy = cv.take<char>(plane * es);
  }
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 3; ++k) l.hist[s][k] = cv.take<double>(plane);
  for (int k = 0; k < 3; ++k) l.mom[k] = cv.take<double>(plane);
  for (int k = 0; k < 2; ++k) l.ftot[k] = cv.take<double>(plane);
  l.partials = cv.take<double>(static_cast<size_t>(moment_blocks(c.nx, c.ny)) * 8 + 8);
  l.scalars = cv.take<double>(8);
  if (c.with_balance) l.bal = carve_balance(cv, c.nx, c.ny);
  EdmModes md;
  if (edm_modes(c, &md) == LBM_OK) l.edm = carve_edm(cv, c, md);
  l.bytes = cv.used + 256;
  return l;
}

std::mutex g_tune_mu;
std::map<std::string, lbm_tile> g_tune;

std::string tune_key(int dtype, int nx, int ny, bool force, int layout, int scheme = LBM_FORCE_GUO) {
  char b[160];
  snprintf(b, sizeof(b), "step dtype=%d nx=%d ny=%d force=%d layout=%d scheme=%d", dtype, nx, ny,
           force ? 1 : 0, layout, scheme);
  return b;
}

void tune_cache_load() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char* path = std::getenv("LBM_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    int dt, nx, ny, fo, lay, sch;
    lbm_tile t;
    if (std::sscanf(line, "step dtype=%d nx=%d ny=%d force=%d layout=%d scheme=%d : %d %d %d %d %d %d %d %d",
                    &dt, &nx, &ny, &fo, &lay, &sch, &t.bx, &t.by, &t.vx, &t.ry, &t.nt, &t.fuse,
                    &t.pf, &t.halo) == 14 &&
        (sch >= 2 ? entropic_tile_ok(t, nx, ny) : sch == 1 ? edm_tile_ok(t, nx, ny) : tile_ok(t, dt, nx, ny)))
      g_tune[tune_key(dt, nx, ny, fo != 0, lay, sch)] = t;
  }
  std::fclose(f);
}

void tune_cache_store() {
  const char* path = std::getenv("LBM_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_tune)
    std::fprintf(f, "%s : %d %d %d %d %d %d %d %d\n", kv.first.c_str(), kv.second.bx, kv.second.by,
                 kv.second.vx, kv.second.ry, kv.second.nt, kv.second.fuse, kv.second.pf, kv.second.halo);
  std::fclose(f);
}

bool cfg_forced(const lbm_config& c) { return c.has_force || c.drag_alpha > 0.0 || c.damp_f0 > 0.0; }
bool is_forced(const lbm_ctx_s* c) { return cfg_forced(c->cfg); }
bool is_edm(const lbm_ctx_s* c) { return c->cfg.force_scheme == LBM_FORCE_EDM; }
bool is_entropic(const lbm_ctx_s* c) { return c->cfg.collision == LBM_COLLISION_ENTROPIC; }
// single-step, one-site-per-thread shapes only
bool one_site_kernel(const lbm_ctx_s* c) { return is_edm(c) || is_entropic(c); }
int scheme_code(const lbm_config& c) { return c.force_scheme + 2 * c.collision; }
std::string ctx_key(const lbm_ctx_s* c) {
  return tune_key(c->cfg.dtype, c->cfg.nx, c->cfg.ny, is_forced(c), c->cfg.layout, scheme_code(c->cfg));
}
bool ctx_tile_ok(const lbm_ctx_s* c, const lbm_tile& t) {
  if (is_entropic(c)) return entropic_tile_ok(t, c->cfg.nx, c->cfg.ny);
  return is_edm(c) ? edm_tile_ok(t, c->cfg.nx, c->cfg.ny) : tile_ok(t, c->cfg.dtype, c->cfg.nx, c->cfg.ny);
}
bool cfg_tile_ok(const lbm_config& c, const lbm_tile& t) {
  if (c.collision == LBM_COLLISION_ENTROPIC) return entropic_tile_ok(t, c.nx, c.ny);
  return c.force_scheme == LBM_FORCE_EDM ? edm_tile_ok(t, c.nx, c.ny) : tile_ok(t, c.dtype, c.nx, c.ny);
}

}  // namespace

namespace lbm {
bool tuned_tile(int dtype, int nx, int ny, bool force, int layout, lbm_tile* out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_cache_load();
  auto it = g_tune.find(tune_key(dtype, nx, ny, force, layout));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}
}  // namespace lbm

namespace {

// One launch: the bulk shape (c->tile, one or two steps) or, with `single`
// or a moment record, the single-step shape.
int enqueue_step(lbm_ctx_s* c, int src, hipStream_t s, double* hr, double* hx, double* hy,
                 bool single = false) {
  StepParams p{};
  p.src = c->pop[src];
  p.dst = c->pop[1 - src];
  p.fx = c->fx;
  p.fy = c->fy;
  p.h_rho = hr;
  p.h_ux = hx;
  p.h_uy = hy;
  p.nx = c->cfg.nx;
  p.ny = c->cfg.ny;
  p.ps = c->lay.ps;
  p.rs = c->lay.rs;
  p.omega = 1.0 / c->cfg.tau;
  p.alpha = c->cfg.drag_alpha;
  const lbm_tile& t = (single || hr) ? c->tile1 : c->tile;
  if (is_edm(c)) return edm_step(c->cfg, c->edm, c->edm_md, p, t, s);
  if (is_entropic(c)) return entropic_step(c->cfg.dtype, p, t, s);
  return launch_step(c->cfg.dtype, is_forced(c), p, t, s);
}

// Single-step shape to pair with a bulk shape.
lbm_tile single_for(const lbm_ctx_s* c, const lbm_tile& bulk) {
  if (steps_per_launch(bulk) == 1) return bulk;
  return default_tile(c->cfg.dtype, c->cfg.nx, c->cfg.ny, c->cfg.layout);
}

void drop_graphs(lbm_ctx_s* c) {
  for (auto& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

int build_graph(lbm_ctx_s* c, int parity) {
  if (!c->cap_stream) LBM_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  LBM_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = LBM_OK;
  int src = parity;
  for (int i = 0; i < c->graph_chunk && rc == LBM_OK; ++i) {
    rc = enqueue_step(c, src, c->cap_stream, nullptr, nullptr, nullptr);
    src ^= 1;
  }
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (rc != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->gexec[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return LBM_OK;
}

hipEvent_t get_event(lbm_ctx_s* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int collect_timing(lbm_ctx_s* c) {
  for (auto& pr : c->ev_pending) {
    LBM_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    LBM_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    c->timed_ms += ms;
    c->ev_free.push_back(pr.first);
    c->ev_free.push_back(pr.second);
  }
  c->ev_pending.clear();
  c->timed_launches += c->pending_launches;
  c->pending_launches = 0;
  return LBM_OK;
}

// Work on c->stream after this point waits for a running balance: for calls that
// write the moment history, the current FP64 moments, the total force or the
// balance workspace, which the balance stream reads.
int wait_balance(lbm_ctx_s* c) {
  if (c->bal_pending) LBM_HIP(hipStreamWaitEvent(c->stream, c->bal_done, 0));
  return LBM_OK;
}

int balance_input(lbm_ctx_s* c, lbm_balance_input* out, double* deferred_scalars = nullptr);

int moments_into(lbm_ctx_s* c, void* rho, void* ux, void* uy, int out_dtype, double* r64,
                 double* ux64, double* uy64, double* ftx, double* fty, double* scalars8) {
  MomentParams m{};
  m.pop = c->pop[c->cur];
  m.fx = c->fx;
  m.fy = c->fy;
  m.rho = rho;
  m.ux = ux;
  m.uy = uy;
  m.out_dtype = out_dtype;
  m.rho64 = r64;
  m.ux64 = ux64;
  m.uy64 = uy64;
  m.ftx64 = ftx;
  m.fty64 = fty;
  m.partials = c->partials;
  m.nx = c->cfg.nx;
  m.ny = c->cfg.ny;
  m.ps = c->lay.ps;
  m.rs = c->lay.rs;
  m.alpha = c->cfg.drag_alpha;
  int rc = is_edm(c) ? edm_moments(c->cfg, c->edm, c->edm_md, m, c->stream)
                     : launch_moments(c->cfg.dtype, is_forced(c), m, c->stream);
  if (rc) return rc;
  if (!scalars8) return LBM_OK;
  rc = launch_reduce_scalars(c->partials, moment_blocks(c->cfg.nx, c->cfg.ny), c->scalars_dev,
                             c->stream);
  if (rc) return rc;
  LBM_HIP(hipMemcpyAsync(scalars8, c->scalars_dev, 8 * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  LBM_HIP(hipStreamSynchronize(c->stream));
  scalars8[LBM_S_TIME] = static_cast<double>(c->t);
  if (scalars8[LBM_S_NONFINITE] > 0.0 || !(scalars8[LBM_S_MINRHO] > 0.0))
    return fail(LBM_E_DIVERGED, "run diverged: %.0f non-finite sites, min rho %g at step %lld",
                scalars8[LBM_S_NONFINITE], scalars8[LBM_S_MINRHO], static_cast<long long>(c->t));
  return LBM_OK;
}

// Header of a saved state: 32 int64 words (256 bytes), unused words zero.
// Words: 0 format tag, 1 t, 2-3 the times of the two recorded moment levels,
// 4 nx, 5 ny, 6 dtype, 7 population layout, 8 total bytes of the state.
constexpr int64_t kStateTag = 0x4c424d33;
struct StateHeader {
  int64_t t, h0, h1, nx, ny, dtype, layout, bytes;
};
__global__ void k_write_header(int64_t* h, StateHeader s) {
  const int i = threadIdx.x;
  if (i < 32) {
    int64_t v = 0;
    if (i == 0) v = kStateTag;
    if (i == 1) v = s.t;
    if (i == 2) v = s.h0;
    if (i == 3) v = s.h1;
    if (i == 4) v = s.nx;
    if (i == 5) v = s.ny;
    if (i == 6) v = s.dtype;
    if (i == 7) v = s.layout;
    if (i == 8) v = s.bytes;
    h[i] = v;
  }
}

constexpr size_t kHeader = 256;

size_t state_bytes_of(const lbm_ctx_s* c) {
  return kHeader + 9 * c->plane * elem_size(c->cfg.dtype) + 6 * c->plane * sizeof(double);
}

}  // namespace

extern "C" {

const char* lbm_version(void) { return "lbm-mi355x 0.1 (gfx950, D2Q9 BGK + sub-volume balance)"; }

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_E_INVALID: return "invalid argument";
    case LBM_E_NOMEM: return "workspace too small";
    case LBM_E_HIP: return "HIP runtime error";
    case LBM_E_DIVERGED: return "simulation diverged";
    case LBM_E_STATE: return "call not possible in the current state";
    case LBM_E_UNSUPPORTED: return "unsupported request";
    case LBM_E_TIMEOUT: return "bounded barrier wait ran out";
    default: return "unknown status";
  }
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

int lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes) {
  if (int rc = validate_config(cfg)) return rc;
  if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
  *bytes = carve_ctx(*cfg, nullptr, 0).bytes;
  return LBM_OK;
}

int lbm_init(const lbm_config* cfg, void* ws, size_t ws_bytes, const double* rho0,
             const double* ux0, const double* uy0, const double* fx, const double* fy,
             lbm_ctx* out) {
  if (int rc = validate_config(cfg)) return rc;
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!ws) return fail(LBM_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(LBM_E_INVALID, "workspace must be 256-byte aligned");
  if (!rho0 || !ux0 || !uy0) return fail(LBM_E_INVALID, "initial fields must not be NULL");
  if (cfg->has_force && (!fx || !fy)) return fail(LBM_E_INVALID, "has_force = 1 needs fx and fy");
  if (!cfg->has_force && (fx || fy)) return fail(LBM_E_INVALID, "fx/fy given but has_force = 0");
  Layout l = carve_ctx(*cfg, nullptr, 0);
  if (ws_bytes < l.bytes)
    return fail(LBM_E_NOMEM, "workspace %zu bytes < %zu required", ws_bytes, l.bytes);
  l = carve_ctx(*cfg, ws, ws_bytes);
  lbm_ctx_s* c = new lbm_ctx_s();
  c->cfg = *cfg;
  c->stream = static_cast<hipStream_t>(cfg->stream);
  c->pop[0] = l.pop[0];
  c->pop[1] = l.pop[1];
  c->fx = l.fx;
  c->fy = l.fy;
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 3; ++k) c->hist[s][k] = l.hist[s][k];
  for (int k = 0; k < 3; ++k) c->mom[k] = l.mom[k];
  c->ftot[0] = l.ftot[0];
  c->ftot[1] = l.ftot[1];
  c->partials = l.partials;
  c->scalars_dev = l.scalars;
  c->bal = l.bal;
  c->plane = static_cast<size_t>(cfg->nx) * cfg->ny;
  c->lay = pop_layout(cfg->layout, cfg->nx, cfg->ny);
  c->edm = l.edm;
  if (int rc = edm_modes(*cfg, &c->edm_md)) {
    delete c;
    return rc;
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache_load();
    auto it = g_tune.find(ctx_key(c));
    if (it != g_tune.end())
      c->tile = it->second;
    else
      c->tile = one_site_kernel(c) ? edm_default_tile(cfg->nx)
                                   : default_tile(cfg->dtype, cfg->nx, cfg->ny, cfg->layout);
    c->tile1 = single_for(c, c->tile);
  }
  int rc = launch_init(cfg->dtype, c->pop[0], c->lay, rho0, ux0, uy0, cfg->nx, cfg->ny, c->stream);
  if (rc == LBM_OK) rc = edm_tables(*cfg, c->edm, c->edm_md, c->stream);
  if (rc == LBM_OK && cfg->has_force) {
    rc = launch_to_storage(cfg->dtype, c->fx, fx, c->plane, c->stream);
    if (rc == LBM_OK) rc = launch_to_storage(cfg->dtype, c->fy, fy, c->plane, c->stream);
  }
  if (rc != LBM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx c, int64_t n) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(LBM_E_INVALID, "n must be >= 0");
  if (n == 0) return LBM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int64_t nhist = n < 2 ? n : 2;
  const int64_t plain = n - nhist;
  const int spl = steps_per_launch(c->tile);
  const int64_t bulk = plain / spl;  // launches of the bulk shape
  if (c->timing && bulk > 0) {
    e0 = get_event(c);
    e1 = get_event(c);
    if (!e0 || !e1) return fail(LBM_E_HIP, "hipEventCreate failed");
    LBM_HIP(hipEventRecord(e0, c->stream));
  }
  int64_t left = bulk;
  if (c->graph_chunk > 0) {
    while (left >= c->graph_chunk) {
      if (!c->gexec[c->cur])
        if (int rc = build_graph(c, c->cur)) return rc;
      LBM_HIP(hipGraphLaunch(c->gexec[c->cur], c->stream));
      left -= c->graph_chunk;
      c->t += static_cast<int64_t>(c->graph_chunk) * spl;  // chunk is even: parity unchanged
    }
  }
  for (; left > 0; --left) {
    if (int rc = enqueue_step(c, c->cur, c->stream, nullptr, nullptr, nullptr)) return rc;
    c->cur ^= 1;
    c->t += spl;
  }
  if (c->timing && bulk > 0) {
    LBM_HIP(hipEventRecord(e1, c->stream));
    c->ev_pending.emplace_back(e0, e1);
    c->pending_launches += bulk;
  }
  for (int64_t i = bulk * spl; i < plain; ++i) {
    if (int rc = enqueue_step(c, c->cur, c->stream, nullptr, nullptr, nullptr, true)) return rc;
    c->cur ^= 1;
    c->t += 1;
  }
  if (nhist > 0)
    if (int rc = wait_balance(c)) return rc;
  for (int64_t i = 0; i < nhist; ++i) {
    const int slot = static_cast<int>(c->t & 1);
    if (int rc = enqueue_step(c, c->cur, c->stream, c->hist[slot][0], c->hist[slot][1],
                              c->hist[slot][2]))
      return rc;
    c->hist_t[slot] = c->t;
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

int lbm_moments(lbm_ctx c, void* rho, void* ux, void* uy, int32_t out_dtype, double* scalars8) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (out_dtype != LBM_F32 && out_dtype != LBM_F64)
    return fail(LBM_E_INVALID, "out_dtype must be LBM_F32 or LBM_F64");
  return moments_into(c, rho, ux, uy, out_dtype, nullptr, nullptr, nullptr, nullptr, nullptr,
                      scalars8);
}

static int validate_balance_request(int nx, int ny, const int32_t* sizes, int32_t nsizes,
                                    lbm_balance_stats* out, const int32_t* windows, int32_t nwin,
                                    double* wterms, const lbm_balance_extra* extra = nullptr) {
  if (nsizes < 0 || nsizes > kMaxSizes)
    return fail(LBM_E_INVALID, "nsizes must be in [0, %d]", kMaxSizes);
  if (nsizes > 0 && !sizes) return fail(LBM_E_INVALID, "sizes must not be NULL");
  if (nsizes > 0 && !out && !(extra && extra->sample_counts))
    return fail(LBM_E_INVALID, "out must not be NULL (without sampled windows)");
  if (int rc = validate_balance_extra(nsizes, out, extra)) return rc;
  const int m = nx < ny ? nx : ny;
  for (int k = 0; k < nsizes; ++k)
    if (sizes[k] < 1 || sizes[k] > m)
      return fail(LBM_E_INVALID, "box size %d outside [1, %d]", sizes[k], m);
  if (nwin < 0 || nwin > kMaxWindows)
    return fail(LBM_E_INVALID, "nwin must be in [0, %d]", kMaxWindows);
  if (nwin > 0 && (!windows || !wterms)) return fail(LBM_E_INVALID, "windows/wterms NULL");
  for (int k = 0; k < nwin; ++k) {
    const int x0 = windows[3 * k], y0 = windows[3 * k + 1], L = windows[3 * k + 2];
    if (x0 < 0 || x0 >= nx || y0 < 0 || y0 >= ny || L < 1 || L > m)
      return fail(LBM_E_INVALID, "window %d (%d, %d, %d) out of range", k, x0, y0, L);
  }
  return LBM_OK;
}

int lbm_subvolume_balance(lbm_ctx c, const int32_t* sizes, int32_t nsizes, lbm_balance_stats* out,
                          double* dmaps, const int32_t* windows, int32_t nwin, double* wterms,
                          double* term_fields) {
  return lbm_subvolume_balance_ex(c, sizes, nsizes, out, dmaps, windows, nwin, wterms, term_fields,
                                  nullptr);
}

int lbm_subvolume_balance_ex(lbm_ctx c, const int32_t* sizes, int32_t nsizes, lbm_balance_stats* out,
                             double* dmaps, const int32_t* windows, int32_t nwin, double* wterms,
                             double* term_fields, const lbm_balance_extra* extra) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (!c->cfg.with_balance) return fail(LBM_E_STATE, "handle was created with with_balance = 0");
  if (int rc = validate_balance_request(c->cfg.nx, c->cfg.ny, sizes, nsizes, out, windows, nwin,
                                        wterms, extra))
    return rc;
  if (int rc = wait_balance(c)) return rc;
  lbm_balance_input in{};
  if (int rc = balance_input(c, &in)) return rc;
  return run_balance(in, c->bal, sizes, nsizes, out, dmaps, windows, nwin, wterms, term_fields, extra);
}

int lbm_balance_begin(lbm_ctx c, const int32_t* sizes, int32_t nsizes) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (!c->cfg.with_balance) return fail(LBM_E_STATE, "handle was created with with_balance = 0");
  if (c->bal_pending) return fail(LBM_E_STATE, "a balance is running: lbm_balance_end first");
  if (nsizes < 1) return fail(LBM_E_INVALID, "nsizes must be in [1, %d]", kMaxSizes);
  lbm_balance_stats dummy{};
  if (int rc = validate_balance_request(c->cfg.nx, c->cfg.ny, sizes, nsizes, &dummy, nullptr, 0, nullptr))
    return rc;
  if (!c->bal_stream) {
    LBM_HIP(hipStreamCreateWithFlags(&c->bal_stream, hipStreamNonBlocking));
    LBM_HIP(hipEventCreateWithFlags(&c->bal_snap, hipEventDisableTiming));
    LBM_HIP(hipEventCreateWithFlags(&c->bal_done, hipEventDisableTiming));
    LBM_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->bal_host), (balance_stats_doubles() + 8) * sizeof(double),
                          hipHostMallocDefault));
  }
  lbm_balance_input in{};
  if (int rc = balance_input(c, &in, c->bal_host + balance_stats_doubles())) return rc;
  in.stream = c->bal_stream;
  LBM_HIP(hipEventRecord(c->bal_snap, c->stream));
  LBM_HIP(hipStreamWaitEvent(c->bal_stream, c->bal_snap, 0));
  if (int rc = run_balance_async(in, c->bal, sizes, nsizes, c->bal_host)) return rc;
  LBM_HIP(hipEventRecord(c->bal_done, c->bal_stream));
  c->bal_sizes.assign(sizes, sizes + nsizes);
  c->bal_pending = true;
  c->bal_t = c->t;
  return LBM_OK;
}

int lbm_balance_end(lbm_ctx c, lbm_balance_stats* out) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (!c->bal_pending) return fail(LBM_E_STATE, "no balance is running");
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  LBM_HIP(hipEventSynchronize(c->bal_done));
  c->bal_pending = false;
  fill_balance_stats(c->bal_host, c->bal_sizes.data(), static_cast<int>(c->bal_sizes.size()), out);
  // the moment check of lbm_balance_begin (its scalars were copied before the balance started)
  const double* sc = c->bal_host + balance_stats_doubles();
  if (sc[LBM_S_NONFINITE] > 0.0 || !(sc[LBM_S_MINRHO] > 0.0))
    return fail(LBM_E_DIVERGED, "run diverged: %.0f non-finite sites, min rho %g at step %lld", sc[LBM_S_NONFINITE],
                sc[LBM_S_MINRHO], static_cast<long long>(c->bal_t));
  return LBM_OK;
}

}  // extern "C"

namespace {
// The balance input at the current time t: FP64 moments of t (with the total
// force and, for the entropic collision, the effective viscosity), the recorded
// moments of t-1 and t-2.  Enqueued on c->stream; synchronises to check the
// moments (LBM_E_DIVERGED), or, with deferred_scalars (pinned host double[8]),
// only enqueues the copy of the moment scalars there for a later check.
int balance_input(lbm_ctx_s* c, lbm_balance_input* out, double* deferred_scalars) {
  const int64_t t = c->t;
  if (t < 2 || c->hist_t[(t - 1) & 1] != t - 1 || c->hist_t[(t - 2) & 1] != t - 2)
    return fail(LBM_E_STATE, "balance at t = %lld needs the moments of steps t-1 and t-2",
                static_cast<long long>(t));
  const bool forced = is_forced(c);
  double sc[8];
  int rc = moments_into(c, nullptr, nullptr, nullptr, LBM_F64, c->mom[0], c->mom[1], c->mom[2],
                        forced ? c->ftot[0] : nullptr, forced ? c->ftot[1] : nullptr,
                        deferred_scalars ? nullptr : sc);
  if (rc) return rc;
  if (deferred_scalars) {
    if (int rc2 = launch_reduce_scalars(c->partials, moment_blocks(c->cfg.nx, c->cfg.ny), c->scalars_dev,
                                        c->stream))
      return rc2;
    LBM_HIP(hipMemcpyAsync(deferred_scalars, c->scalars_dev, 8 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  }
  lbm_balance_input& in = *out;
  in.nx = c->cfg.nx;
  in.ny = c->cfg.ny;
  in.nu = (c->cfg.tau - 0.5) / 3.0;
  const int s2 = static_cast<int>((t - 2) & 1), s1 = static_cast<int>((t - 1) & 1);
  for (int k = 0; k < 3; ++k) {
    const double* lv[3] = {c->hist[s2][k], c->hist[s1][k], c->mom[k]};
    for (int j = 0; j < 3; ++j) {
      if (k == 0) in.rho[j] = lv[j];
      if (k == 1) in.ux[j] = lv[j];
      if (k == 2) in.uy[j] = lv[j];
    }
  }
  in.fx = forced ? c->ftot[0] : nullptr;
  in.fy = forced ? c->ftot[1] : nullptr;
  in.stream = c->stream;
  if (is_entropic(c)) {  // the effective viscosity at t (the handle is unforced: ftot is free)
    if (int rc2 = relaxation_fields(c->cfg.dtype, true, c->pop[c->cur], c->lay, c->cfg.nx, c->cfg.ny,
                                    c->cfg.tau, nullptr, c->ftot[0], c->stream))
      return rc2;
    in.nu_field = c->ftot[0];
  }
  return LBM_OK;
}

// Scratch of lbm_balance_fields_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch` itself (in
// host code the name is a stand-in, not a device address): the per-device address
// comes from hipGetSymbolAddress on the first call on that device, with the device
// current, and only that address reaches the kernels.
constexpr size_t kNoAllocScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void** out) {
  int dev = -1;
  LBM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LBM_E_UNSUPPORTED, "device %d beyond the %d the static scratch supports", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0)
      return fail(LBM_E_HIP, "static scratch address %p not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

int validate_fields_input(const lbm_balance_input* in) {
  if (!in) return fail(LBM_E_INVALID, "input is NULL");
  for (int k = 0; k < 3; ++k)
    if (!in->rho[k] || !in->ux[k] || !in->uy[k])
      return fail(LBM_E_INVALID, "level %d fields must not be NULL", k);
  if ((in->fx == nullptr) != (in->fy == nullptr))
    return fail(LBM_E_INVALID, "fx and fy must both be given or both be NULL");
  if (!std::isfinite(in->nu) || in->nu < 0.0) return fail(LBM_E_INVALID, "nu must be finite, >= 0");
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_balance_workspace_bytes(int32_t nx, int32_t ny, size_t* bytes) {
  if (nx < 16 || ny < 16 || nx > 65536 || ny > 65536)
    return fail(LBM_E_INVALID, "grid %d x %d outside [16, 65536]", nx, ny);
  if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
  if (int rc = balance_grid_ok(nx, ny)) return rc;
  *bytes = balance_ws_bytes(nx, ny);
  return LBM_OK;
}

int lbm_balance_fields(const lbm_balance_input* in, void* ws, size_t ws_bytes, const int32_t* sizes,
                       int32_t nsizes, lbm_balance_stats* out, double* dmaps,
                       const int32_t* windows, int32_t nwin, double* wterms, double* term_fields) {
  return lbm_balance_fields_ex(in, ws, ws_bytes, sizes, nsizes, out, dmaps, windows, nwin, wterms,
                               term_fields, nullptr);
}

int lbm_balance_fields_ex(const lbm_balance_input* in, void* ws, size_t ws_bytes, const int32_t* sizes,
                          int32_t nsizes, lbm_balance_stats* out, double* dmaps,
                          const int32_t* windows, int32_t nwin, double* wterms, double* term_fields,
                          const lbm_balance_extra* extra) {
  if (!in) return fail(LBM_E_INVALID, "input is NULL");
  size_t need = 0;
  if (int rc = lbm_balance_workspace_bytes(in->nx, in->ny, &need)) return rc;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(LBM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < need) return fail(LBM_E_NOMEM, "workspace %zu bytes < %zu required", ws_bytes, need);
  if (int rc = validate_fields_input(in)) return rc;
  if (int rc = validate_balance_request(in->nx, in->ny, sizes, nsizes, out, windows, nwin, wterms, extra))
    return rc;
  Carver cv(ws, ws_bytes);
  BalanceWs b = carve_balance(cv, in->nx, in->ny);
  return run_balance(*in, b, sizes, nsizes, out, dmaps, windows, nwin, wterms, term_fields, extra);
}

int lbm_balance_fields_noalloc(const lbm_balance_input* in, const int32_t* sizes, int32_t nsizes,
                               lbm_balance_stats* out, double* dmaps, const int32_t* windows,
                               int32_t nwin, double* wterms, double* term_fields) {
  if (!in) return fail(LBM_E_INVALID, "input is NULL");
  size_t need = 0;
  if (int rc = lbm_balance_workspace_bytes(in->nx, in->ny, &need)) return rc;
  if (need > kNoAllocScratchBytes)
    return fail(LBM_E_NOMEM,
                "a %d x %d balance needs %zu bytes of scratch; the static scratch holds %zu "
                "(square grids up to 591 x 591): use lbm_balance_fields with a workspace",
                in->nx, in->ny, need, kNoAllocScratchBytes);
  if (int rc = validate_fields_input(in)) return rc;
  if (int rc = validate_balance_request(in->nx, in->ny, sizes, nsizes, out, windows, nwin, wterms))
    return rc;
  void* ws = nullptr;
  if (int rc = noalloc_scratch(&ws)) return rc;
  Carver cv(ws, kNoAllocScratchBytes);
  BalanceWs b = carve_balance(cv, in->nx, in->ny);
  return run_balance(*in, b, sizes, nsizes, out, dmaps, windows, nwin, wterms, term_fields, nullptr);
}

int lbm_enstrophy(lbm_ctx c, double* enstrophy) {
  if (!c || !enstrophy) return fail(LBM_E_INVALID, "NULL argument");
  if (int rc = wait_balance(c)) return rc;
  if (int rc = moments_into(c, nullptr, nullptr, nullptr, LBM_F64, c->mom[0], c->mom[1], c->mom[2], nullptr,
                            nullptr, nullptr))
    return rc;
  return global_enstrophy(c->mom[1], c->mom[2], c->cfg.nx, c->cfg.ny, c->partials,
                          moment_blocks(c->cfg.nx, c->cfg.ny) * 8, c->scalars_dev, enstrophy, c->stream);
}

int lbm_relaxation(lbm_ctx c, double* alpha, double* nu_eff) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (!alpha && !nu_eff) return LBM_OK;
  return relaxation_fields(c->cfg.dtype, is_entropic(c), c->pop[c->cur], c->lay, c->cfg.nx, c->cfg.ny,
                           c->cfg.tau, alpha, nu_eff, c->stream);
}

int lbm_energy_spectrum(lbm_ctx c, double* spectrum, int32_t nshells) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (!c->cfg.with_balance) return fail(LBM_E_STATE, "handle was created with with_balance = 0");
  if (!spectrum_size_ok(c->cfg.nx, c->cfg.ny))
    return fail(LBM_E_UNSUPPORTED, "spectrum needs power-of-two extents in [16, 4096]");
  if (!spectrum) return fail(LBM_E_INVALID, "spectrum is NULL");
  if (nshells < 1 || nshells > LBM_MAX_SHELLS)
    return fail(LBM_E_INVALID, "nshells must be in [1, %d]", LBM_MAX_SHELLS);
  if (int rc = wait_balance(c)) return rc;
  if (int rc = moments_into(c, nullptr, nullptr, nullptr, LBM_F64, c->mom[0], c->mom[1], c->mom[2],
                            nullptr, nullptr, nullptr))
    return rc;
  // the balance's term, aux and table fields are free between balance calls
  char* base = reinterpret_cast<char*>(c->bal.terms);
  const size_t room = static_cast<size_t>(reinterpret_cast<char*>(c->bal.means) - base);
  return run_spectrum(c->cfg.nx, c->cfg.ny, c->mom[1], c->mom[2], base, room, spectrum, nshells,
                      c->stream);
}

int lbm_spectrum_workspace_bytes(int32_t nx, int32_t ny, size_t* bytes) {
  if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
  if (!spectrum_size_ok(nx, ny))
    return fail(LBM_E_UNSUPPORTED, "spectrum needs power-of-two extents in [16, 4096] (got %d x %d)", nx, ny);
  *bytes = spectrum_ws_bytes(nx, ny);
  return LBM_OK;
}

int lbm_spectrum_fields(int32_t nx, int32_t ny, const double* ux, const double* uy, void* ws, size_t ws_bytes,
                        double* spectrum, int32_t nshells, void* stream) {
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(LBM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  return run_spectrum(nx, ny, ux, uy, ws, ws_bytes, spectrum, nshells, static_cast<hipStream_t>(stream));
}

int lbm_time(lbm_ctx c, int64_t* t) {
  if (!c || !t) return fail(LBM_E_INVALID, "NULL argument");
  *t = c->t;
  return LBM_OK;
}

int lbm_state_bytes(lbm_ctx c, size_t* bytes) {
  if (!c || !bytes) return fail(LBM_E_INVALID, "NULL argument");
  *bytes = state_bytes_of(c);
  return LBM_OK;
}

int lbm_save(lbm_ctx c, void* dst) {
  if (!c || !dst) return fail(LBM_E_INVALID, "NULL argument");
  char* d = static_cast<char*>(dst);
  StateHeader sh{c->t, c->hist_t[0], c->hist_t[1], c->cfg.nx, c->cfg.ny, c->cfg.dtype, c->cfg.layout,
                 static_cast<int64_t>(state_bytes_of(c))};
  hipLaunchKernelGGL(k_write_header, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<int64_t*>(d), sh);
  LBM_HIP(hipGetLastError());
  const size_t pb = 9 * c->plane * elem_size(c->cfg.dtype);
  LBM_HIP(hipMemcpyAsync(d + kHeader, c->pop[c->cur], pb, hipMemcpyDeviceToDevice, c->stream));
  size_t off = kHeader + pb;
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 3; ++k) {
      LBM_HIP(hipMemcpyAsync(d + off, c->hist[s][k], c->plane * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
      off += c->plane * sizeof(double);
    }
  return LBM_OK;
}

int lbm_load(lbm_ctx c, const void* src) {
  if (!c || !src) return fail(LBM_E_INVALID, "NULL argument");
  const char* d = static_cast<const char*>(src);
  // only the header is read before it has been checked against this handle
  int64_t h[9];
  LBM_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  LBM_HIP(hipStreamSynchronize(c->stream));
  if (h[0] != kStateTag) return fail(LBM_E_INVALID, "not a saved state of this library (tag %llx)",
                                     static_cast<unsigned long long>(h[0]));
  const int64_t want[5] = {c->cfg.nx, c->cfg.ny, c->cfg.dtype, c->cfg.layout,
                           static_cast<int64_t>(state_bytes_of(c))};
  static const char* what[5] = {"nx", "ny", "dtype", "layout", "state bytes"};
  for (int k = 0; k < 5; ++k)
    if (h[4 + k] != want[k])
      return fail(LBM_E_INVALID, "saved state has %s = %lld, this handle %lld", what[k],
                  static_cast<long long>(h[4 + k]), static_cast<long long>(want[k]));
  if (h[1] < 0 || h[2] < -1 || h[3] < -1 || h[2] > h[1] || h[3] > h[1])
    return fail(LBM_E_INVALID, "saved state has inconsistent times (t %lld, history %lld, %lld)",
                static_cast<long long>(h[1]), static_cast<long long>(h[2]), static_cast<long long>(h[3]));
  if (int rc = wait_balance(c)) return rc;
  const size_t pb = 9 * c->plane * elem_size(c->cfg.dtype);
  LBM_HIP(hipMemcpyAsync(c->pop[0], d + kHeader, pb, hipMemcpyDeviceToDevice, c->stream));
  size_t off = kHeader + pb;
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 3; ++k) {
      LBM_HIP(hipMemcpyAsync(c->hist[s][k], d + off, c->plane * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
      off += c->plane * sizeof(double);
    }
  c->cur = 0;
  c->t = h[1];
  c->hist_t[0] = h[2];
  c->hist_t[1] = h[3];
  return LBM_OK;
}

int lbm_set_tile(lbm_ctx c, const lbm_tile* tile) {
  if (!c || !tile) return fail(LBM_E_INVALID, "NULL argument");
  if (!ctx_tile_ok(c, *tile))
    return fail(LBM_E_INVALID, "tile (%d,%d,vx %d,ry %d,nt %d,fuse %d,pf %d,halo %d) not valid for %d x %d%s",
                tile->bx, tile->by, tile->vx, tile->ry, tile->nt, tile->fuse, tile->pf, tile->halo, c->cfg.nx,
                c->cfg.ny,
                is_edm(c) ? " with the exact-difference step" : "");
  c->tile = *tile;
  c->tile1 = single_for(c, c->tile);
  drop_graphs(c);
  return LBM_OK;
}

int lbm_get_tile(lbm_ctx c, lbm_tile* tile) {
  if (!c || !tile) return fail(LBM_E_INVALID, "NULL argument");
  *tile = c->tile;
  return LBM_OK;
}

int lbm_set_tuned_tile(const lbm_config* cfg, const lbm_tile* tile) {
  if (int rc = validate_config(cfg)) return rc;
  if (!tile) return fail(LBM_E_INVALID, "tile is NULL");
  if (!cfg_tile_ok(*cfg, *tile)) return fail(LBM_E_INVALID, "tile not valid for %d x %d", cfg->nx, cfg->ny);
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_cache_load();
  g_tune[tune_key(cfg->dtype, cfg->nx, cfg->ny, cfg_forced(*cfg), cfg->layout, scheme_code(*cfg))] = *tile;
  tune_cache_store();
  return LBM_OK;
}

int lbm_autotune(lbm_ctx c, int32_t trial_steps, lbm_tile* chosen) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (trial_steps < 1 || trial_steps > 10000) return fail(LBM_E_INVALID, "trial_steps in [1, 10000]");
  constexpr int kCap = 1024;
  std::vector<lbm_tile> cand(kCap);
  int n = tile_candidates(c->cfg.dtype, c->cfg.nx, c->cfg.ny, is_forced(c), cand.data(), kCap);
  if (n > kCap) n = kCap;
  if (one_site_kernel(c)) {  // single-step, one-site-per-thread shapes
    int k = 0;
    for (int i = 0; i < n; ++i)
      if (ctx_tile_ok(c, cand[i])) cand[k++] = cand[i];
    n = k;
  }
  if (n < 1) return fail(LBM_E_UNSUPPORTED, "no step-kernel shape fits this grid");
  const lbm_tile saved = c->tile;
  hipEvent_t e0, e1;
  LBM_HIP(hipEventCreate(&e0));
  LBM_HIP(hipEventCreate(&e1));
  float best = 1e30f, best1 = 1e30f;  // milliseconds per step: any shape, single-step shapes
  lbm_tile best_t = saved, best_t1 = c->tile1;
  int rc = LBM_OK;
  for (int i = 0; i < n && rc == LBM_OK; ++i) {
    c->tile = cand[i];
    // src -> dst repeatedly: the state (src) is never modified
    rc = enqueue_step(c, c->cur, c->stream, nullptr, nullptr, nullptr);
    if (rc) break;
    if (hipEventRecord(e0, c->stream) != hipSuccess) {
      rc = fail(LBM_E_HIP, "hipEventRecord");
      break;
    }
    for (int k = 0; k < trial_steps && rc == LBM_OK; ++k)
      rc = enqueue_step(c, c->cur, c->stream, nullptr, nullptr, nullptr);
    if (rc) break;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(LBM_E_HIP, "hipEventRecord/Synchronize");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= static_cast<float>(steps_per_launch(cand[i]));
    if (ms < best) {
      best = ms;
      best_t = cand[i];
    }
    if (steps_per_launch(cand[i]) == 1 && ms < best1) {
      best1 = ms;
      best_t1 = cand[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tile = rc == LBM_OK ? best_t : saved;
  c->tile1 = steps_per_launch(c->tile) == 1 ? c->tile : best_t1;
  drop_graphs(c);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[ctx_key(c)] = best_t;
    tune_cache_store();
  }
  if (chosen) *chosen = best_t;
  return LBM_OK;
}

int lbm_set_graph(lbm_ctx c, int32_t chunk) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (chunk < 0 || chunk % 2 != 0 || chunk > 4096)
    return fail(LBM_E_INVALID, "chunk must be 0 or an even number <= 4096");
  c->graph_chunk = chunk;
  drop_graphs(c);
  return LBM_OK;
}

int lbm_step_timing(lbm_ctx c, int32_t enable) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  c->timing = enable != 0;
  return LBM_OK;
}

int lbm_step_time(lbm_ctx c, double* ms, int64_t* launches, int32_t reset) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (int rc = collect_timing(c)) return rc;
  if (ms) *ms = c->timed_ms;
  if (launches) *launches = c->timed_launches;
  if (reset) {
    c->timed_ms = 0.0;
    c->timed_launches = 0;
  }
  return LBM_OK;
}

int lbm_destroy(lbm_ctx c) {
  if (!c) return LBM_OK;
  if (c->bal_stream) (void)hipStreamSynchronize(c->bal_stream);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (auto& pr : c->ev_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto e : c->ev_free) (void)hipEventDestroy(e);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->bal_stream) {
    (void)hipEventDestroy(c->bal_snap);
    (void)hipEventDestroy(c->bal_done);
    (void)hipStreamDestroy(c->bal_stream);
    (void)hipHostFree(c->bal_host);
  }
  delete c;
  return LBM_OK;
}

int lbm_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src) return fail(LBM_E_INVALID, "NULL pointer");
  if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
    return fail(LBM_E_INVALID, "bytes and pointers must be multiples of 16");
  if (bytes == 0) return LBM_OK;
  return launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
