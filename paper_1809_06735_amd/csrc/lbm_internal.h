// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/lbm.h"

namespace lbm {

// ---- error reporting ---------------------------------------------------------
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int validate_config(const lbm_config* c);

#define LBM_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::lbm::hip_fail(e_, #call); \
  } while (0)

// ---- D2Q9 lattice -----------------------------------------------------------
// Velocities in the order rest, +x, +y, -x, -y, (+1,+1), (-1,+1), (-1,-1), (+1,-1);
// weights 4/9, 1/9 (axis), 1/36 (diagonal).
constexpr int Q = 9;
__host__ __device__ constexpr int cxq(int l) {
  return l == 1 || l == 5 || l == 8 ? 1 : (l == 3 || l == 6 || l == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cyq(int l) {
  return l == 2 || l == 5 || l == 6 ? 1 : (l == 4 || l == 7 || l == 8 ? -1 : 0);
}
__host__ __device__ constexpr double wq(int l) {
  return l == 0 ? 4.0 / 9.0 : (l <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Element strides of the population array: element (l, y, x) is at
// l * ps + y * rs + x.  LBM_LAYOUT_PLANES: [9][ny][nx] (ps = nx ny, rs = nx);
// LBM_LAYOUT_ROWS: [ny][9][nx] (ps = nx, rs = 9 nx).
struct PopLayout {
  size_t ps, rs;
};
inline PopLayout pop_layout(int layout, int nx, int ny) {
  if (layout == LBM_LAYOUT_ROWS) return PopLayout{static_cast<size_t>(nx), static_cast<size_t>(9) * nx};
  return PopLayout{static_cast<size_t>(nx) * ny, static_cast<size_t>(nx)};
}

// Simple bump allocator over a caller workspace.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    used = align_up(used, 256);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

// ---- step kernels ---------------------------------------------------------------
struct StepParams {
  const void* src;   // populations (deviation from the weights), [9][ny][nx]
  void* dst;
  const void* fx;    // external force, storage type, or null
  const void* fy;
  double* h_rho;     // optional FP64 moment record (pre-collision, time t)
  double* h_ux;
  double* h_uy;
  int nx, ny;
  size_t ps, rs;     // population layout strides
  double omega;      // 1/tau
  double alpha;      // drag
};

int launch_init(int dtype, void* pop, PopLayout lay, const double* rho0, const double* ux0,
                const double* uy0, int nx, int ny, hipStream_t s);
// One launch of the step kernel the tile selects: one step (fuse 0/1) or
// fuse = 2..6 steps (temporal blocking, no moment history).  Buffers: src ->
// dst either way.
int launch_step(int dtype, bool force, const StepParams& p, const lbm_tile& t, hipStream_t s);
int launch_step_fused(int dtype, bool force, const StepParams& p, const lbm_tile& t, hipStream_t s);
// Workgroups of a multi-step shape that the current device holds at once (its
// occupancy per CU times the CU count).
int fused_resident_groups(int dtype, bool force, const lbm_tile& t, int* groups);
bool fused_tile_ok(const lbm_tile& t, int dtype);
// columns of output per strip of a multi-step shape (bx, or bx - 2 (fuse - 1) with halo = 1)
int fused_strip_width(const lbm_tile& t);
size_t fused_lds_bytes(int W, int K, int dtype);
inline int steps_per_launch(const lbm_tile& t) { return t.fuse >= 2 ? t.fuse : 1; }
bool tile_ok(const lbm_tile& t, int dtype, int nx, int ny);
lbm_tile default_tile(int dtype, int nx, int ny, int layout);
// Shapes lbm_autotune times; returns how many there are (at most cap stored).
int tile_candidates(int dtype, int nx, int ny, bool force, lbm_tile* out, int cap);
// Step-kernel shape chosen by lbm_autotune for this grid (process table or the
// LBM_TUNE_CACHE file), if any.
bool tuned_tile(int dtype, int nx, int ny, bool force, int layout, lbm_tile* out);

// Moments of the populations at their time: writes rho, ux, uy (out_dtype, any
// may be null), optional FP64 copies and total force, and per-block partial
// reductions (7 doubles per block) into `partials`; nblocks returned.
struct MomentParams {
  const void* pop;
  const void* fx;
  const void* fy;
  void* rho;
  void* ux;
  void* uy;
  int out_dtype;
  double* rho64;     // optional FP64 copies (for the balance)
  double* ux64;
  double* uy64;
  double* ftx64;     // optional FP64 total force F_ext - alpha rho u
  double* fty64;
  double* partials;  // [nblocks][8]
  int nx, ny;
  size_t ps, rs;     // population layout strides
  double alpha;
};
int moment_blocks(int nx, int ny);
int launch_moments(int dtype, bool force, const MomentParams& p, hipStream_t s);
int launch_reduce_scalars(const double* partials, int nblocks, double* out8, hipStream_t s);
int launch_to_storage(int dtype, void* dst, const double* src, size_t n, hipStream_t s);

int launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// ---- entropic collision -----------------------------------------------------------
// One entropic step src -> dst (single-step shapes with one site per thread).
int entropic_step(int dtype, const StepParams& p, const lbm_tile& t, hipStream_t s);
bool entropic_tile_ok(const lbm_tile& t, int nx, int ny);  // one site per thread, <= 256 threads
// alpha and nu_eff of the populations `pop` (either output may be null); for the
// BGK collision alpha = 2 and nu_eff = (tau0 - 1/2) / 3 everywhere.
int relaxation_fields(int dtype, bool entropic, const void* pop, PopLayout lay, int nx, int ny, double tau0,
                      double* alpha, double* nu, hipStream_t s);

// ---- energy spectrum -------------------------------------------------------------
bool spectrum_size_ok(int nx, int ny);
size_t spectrum_ws_bytes(int nx, int ny);
// Synchronous; ux, uy device FP64 [ny][nx]; spectrum host [nshells].
int run_spectrum(int nx, int ny, const double* ux, const double* uy, void* ws, size_t ws_bytes,
                 double* spectrum, int nshells, hipStream_t s);

// ---- exact-difference forcing and spectral damping (Sec. 3, Eqs. 14-16) -------
// Damped modes: the integer wavevectors with kmin <= |k| <= kmax in the half
// plane ky > 0 or (ky == 0, kx > 0); each stands for itself and -k.
constexpr int kEdmMaxK = 4;
constexpr int kEdmMaxModes = 24;
struct EdmModes {
  int m = 0;   // number of modes (0: no damping)
  int km = 0;  // largest |kx| or |ky| among them
  double f0 = 0.0;  // damping rate over nx ny (the factor of the unnormalised sums)
  int8_t kx[kEdmMaxModes] = {};
  int8_t ky[kEdmMaxModes] = {};
};
int edm_modes(const lbm_config& c, EdmModes* out);
// Equal grids stepped by one set of launches (the run is the grid's y index):
// run r's populations, force fields, Fourier partials and coefficients sit r
// strides after run 0's; each run has its own 1/tau and damping rate.
constexpr int kEdmMaxRuns = 64;
struct EdmRuns {
  int n = 1;
  size_t pop_stride = 0;    // elements between runs' population arrays
  size_t force_stride = 0;  // elements between runs' force fields
  double omega[kEdmMaxRuns] = {};
  double f0[kEdmMaxRuns] = {};  // damp_f0 / (nx ny) per run
};
struct EdmWs {
  double* tabx = nullptr;  // [km+1][2][nx] cos, sin of 2 pi m x / nx (FP64)
  double* taby = nullptr;  // [km+1][2][ny] same in y
  void* tabx_t = nullptr;  // tabx in the storage type
  double* partials = nullptr;  // [dft blocks][4 m] per-workgroup Fourier sums
  void* coef = nullptr;    // [ny][km+1][4] per-row force coefficients (storage type)
};
EdmWs carve_edm(Carver& cv, const lbm_config& c, const EdmModes& md);
int edm_tables(const lbm_config& c, const EdmWs& w, const EdmModes& md, hipStream_t s);
bool edm_tile_ok(const lbm_tile& t, int nx, int ny);
lbm_tile edm_default_tile(int nx);
// One step: the damping force's Fourier reduction (when m > 0), then the
// exact-difference step kernel src -> dst (optional moment record in p.h_*).
int edm_step(const lbm_config& c, const EdmWs& w, const EdmModes& md, const StepParams& p,
             const lbm_tile& t, hipStream_t s);
// One step of runs.n equal grids: p describes run 0 (no moment record); w
// holds runs.n partial and coefficient blocks (carve_edm_runs).
int edm_step_runs(const lbm_config& c, const EdmWs& w, const EdmModes& md, const EdmRuns& runs,
                  const StepParams& p, const lbm_tile& t, hipStream_t s);
EdmWs carve_edm_runs(Carver& cv, const lbm_config& c, const EdmModes& md, int nruns);
// Partials and coefficients of run r of such a workspace.
EdmWs edm_run_view(const EdmWs& w, const lbm_config& c, const EdmModes& md, int r);
// Moments of the current populations as launch_moments, with the physical
// velocity (j + F/2)/rho and the total force F_ext + F^R.
int edm_moments(const lbm_config& c, const EdmWs& w, const EdmModes& md, const MomentParams& p,
                hipStream_t s);

// ---- balance --------------------------------------------------------------------
struct BalanceWs {
  double* terms;     // [13][ny][nx]
  double* aux;       // [8][ny][nx]: E, Omega, omega, sxx, syy, sxy, Hx, Hy
  double* sat;       // [ny+1][13][sat_ld(nx)]: rows of the 13 fields' prefix tables, 128-byte aligned
  double* rtot;      // [ny][13][nx / 128 rounded up]: row totals and carries of the scanned rows
  double* means;     // [16]
  double* partials;  // block partials
  size_t partials_cap;  // doubles of window partials before the field-sum partials
  double* stats;     // [kMaxSizes][3][6] per-size statistics of this call (all corners)
  double* sstats;    // same over the sampled windows
  double* pool;      // [2][kMaxSizes][3][6] pooled statistics (all corners, sampled)
  double* edges;     // [3][LBM_MAX_EDGES] histogram edges
  unsigned long long* hist;  // [2][kMaxSizes][3][LBM_MAX_EDGES + 1] counts
  double* wterms;    // [kMaxWindows][LBM_NWVALS]
  int32_t* windows;  // [kMaxWindows][3]
};
constexpr int kMaxWindows = 4096;
constexpr int kMaxSizes = 64;
size_t balance_ws_bytes(int nx, int ny);
BalanceWs carve_balance(Carver& c, int nx, int ny);
// The window walks address the 13 prefix tables with 32-bit element offsets:
// a grid is accepted for the balance only while 13 ld (ny + 1) < 2^32, ld =
// nx + 1 rounded up to 16 (square grids up to 18 175^2).  LBM_OK, or LBM_E_UNSUPPORTED with a message.
int balance_grid_ok(int nx, int ny);
// Pieces of the balance reused by the adjoint: the 13 term fields and the aux
// fields (E, Omega, omega, sigma_xx, sigma_yy, sigma_xy, H_x, H_y) of passes
// A-C, with the 13 fields' domain means in ws.means; domain means of nf
// consecutive fields; their mean-centred prefix tables
// (row-interleaved: table row y of field f starts at (y nf + f) ld, ld = nx + 1
// rounded up to 16, so the rows of all fields at one y are adjacent); and scaled
// box sums of field f of such a table for every corner shifted by `off`.
int balance_terms(const lbm_balance_input& in, const BalanceWs& ws);
// The same passes; where the two-site passes run (even width, 16-byte aligned
// fields: *table set) and table is non-null, they also scan their rows into
// ws.sat and ws.rtot for balance_table, and write the term planes only when
// planes is set.
int balance_terms(const lbm_balance_input& in, const BalanceWs& ws, bool planes, bool* table);
// The 13 fields' means and complete prefix table ws.sat (the term planes
// ws.terms too when planes is set, and always where the one-site passes run).
int balance_table(const lbm_balance_input& in, const BalanceWs& ws, bool planes);
int field_means(const double* g, int nf, int nx, int ny, double* partials, double* means,
                hipStream_t s);
int sat_build(const double* g, int nf, const double* means, double* sat, int nx, int ny,
              hipStream_t s);
int box_map(const double* sat, const double* means, int nf, int f, int L, int off, double scale,
            double* out, int nx, int ny, hipStream_t s);
enum { AUX_E = 0, AUX_OM2 = 1, AUX_W = 2, AUX_SXX = 3, AUX_SYY = 4, AUX_SXY = 5, AUX_HX = 6,
       AUX_HY = 7, AUX_N = 8 };
int run_balance(const lbm_balance_input& in, const BalanceWs& ws, const int32_t* sizes,
                int nsizes, lbm_balance_stats* out, double* dmaps, const int32_t* windows,
                int nwin, double* wterms, double* term_fields, const lbm_balance_extra* extra);
int validate_balance_extra(int nsizes, const lbm_balance_stats* out, const lbm_balance_extra* extra);
// The all-corner statistics of run_balance, enqueued on in.stream without waiting: the
// statistics (kMaxSizes x 18 doubles at most) land in host_stats (pinned) when the stream
// reaches the end; fill_balance_stats turns them into lbm_balance_stats.
int run_balance_async(const lbm_balance_input& in, const BalanceWs& ws, const int32_t* sizes, int nsizes,
                      double* host_stats);
void fill_balance_stats(const double* host_stats, const int32_t* sizes, int nsizes, lbm_balance_stats* out);
size_t balance_stats_doubles();
// Omega = 1/2 sum omega^2 of FP64 fields [ny][nx] (omega by Eq. 18); partials holds
// max_blocks doubles, dev_out one.  Synchronous.
int global_enstrophy(const double* ux, const double* uy, int nx, int ny, double* partials, int max_blocks,
                     double* dev_out, double* host_out, hipStream_t s);

}  // namespace lbm
