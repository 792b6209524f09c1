/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice-Boltzmann library.
 *
 * The library advances a periodic two-dimensional D2Q9 BGK lattice-Boltzmann
 * model (Tauzin et al., Computers & Fluids 172 (2018), Sec. 1, Eqs. 1-2 and
 * Eq. 5) with an optional static body force (Guo's forcing term) and linear
 * drag, or with the paper's own forced set-up (Sec. 3, Eqs. 14-16: the
 * exact-difference forcing and the spectral damping of the large scales), and
 * evaluates the sub-volume averaged kinetic-energy and enstrophy
 * balances with their balancing errors (Sec. 2, Eqs. 8-13; Sec. 3, Eqs. 17-18
 * and Table 1; Sec. 4, Eq. 20).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: LBM_OK (0) or a negative LBM_E_*
 *   code.  Nothing throws and nothing exits.  A failed call leaves a
 *   human-readable message in lbm_last_error() (per host thread).
 * - Fields are row-major [ny][nx] (x fastest) with periodic wrap in x and y.
 *   Lattice units: dx = dt = 1, c_s^2 = 1/3, nu = (tau - 1/2)/3.
 * - "device" pointers are HIP device memory on the current device; "host"
 *   pointers are ordinary host memory.  The caller owns every buffer it
 *   passes, including workspaces; the library only borrows them for the
 *   lifetime of the object that was created with them.  The library owns only
 *   its host-side handle, which the matching *_destroy call frees.
 * - Work is enqueued on the HIP stream given in the config (NULL: the null
 *   stream).  Calls documented as synchronous wait for that stream.
 * - Arguments are validated before anything is enqueued; an invalid argument
 *   gives LBM_E_INVALID and enqueues nothing.
 * - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define LBM_API __attribute__((visibility("default")))
#else
#define LBM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
  LBM_OK = 0,
  LBM_E_INVALID = -1,     /* bad argument (message says which)                     */
  LBM_E_NOMEM = -2,       /* workspace smaller than the *_workspace_bytes figure   */
  LBM_E_HIP = -3,         /* a HIP runtime call failed (message holds its text)    */
  LBM_E_DIVERGED = -4,    /* non-finite moment or rho <= 0 found (step in message) */
  LBM_E_STATE = -5,       /* call not possible in the current state                */
  LBM_E_UNSUPPORTED = -6, /* valid request this build does not handle              */
  LBM_E_TIMEOUT = -7      /* a persistent kernel's bounded barrier wait ran out    */
};

/* ---- storage types and population layouts ---------------------------------- */
enum { LBM_F32 = 0, LBM_F64 = 1 };
enum { LBM_LAYOUT_PLANES = 0, LBM_LAYOUT_ROWS = 1 };

/* ---- forcing schemes (lbm_config.force_scheme) ----------------------------- */
enum {
  LBM_FORCE_GUO = 0, /* Guo's forcing term with the half-force velocity; optional
                        linear drag                                             */
  LBM_FORCE_EDM = 1  /* exact-difference method (Kupershtokh), the scheme of
                        Sec. 3; optional spectral damping of Eq. 16             */
};

/* ---- collision operators (lbm_config.collision) ---------------------------- */
enum {
  LBM_COLLISION_BGK = 0,      /* Eq. 1: relaxation time tau                              */
  LBM_COLLISION_ENTROPIC = 1  /* the entropic scheme of Sec. 1: relaxation time
                                 tau_eff = 2 tau / alpha towards the minimiser of H (Eq. 6)
                                 at the site's rho, rho u; alpha per site from
                                 H(f + alpha (f^eq - f)) = H(f).  Unforced only.         */
};

/* ---- indices into the 8 global scalars returned by *_moments -------------- */
enum {
  LBM_S_MASS = 0,      /* sum rho                                */
  LBM_S_MOMX = 1,      /* sum rho u_x                            */
  LBM_S_MOMY = 2,      /* sum rho u_y                            */
  LBM_S_ENERGY = 3,    /* sum rho |u|^2 / 2                      */
  LBM_S_MAXSPEED = 4,  /* max |u|                                */
  LBM_S_MINRHO = 5,    /* min rho                                */
  LBM_S_NONFINITE = 6, /* number of sites with a non-finite moment */
  LBM_S_TIME = 7       /* time step t of the moments              */
};

/* ---- order of the 13 balance integrand fields ----------------------------- */
enum {
  LBM_T_LHS_E = 0, /* d_t E, E = rho|u|^2/2, three-level formula (Eq. 17)        */
  LBM_T_E1 = 1,    /* -div(E u)                         (Eq. 10, first term)     */
  LBM_T_E2 = 2,    /* -u.grad p, p = rho/3              (Eq. 10, second term)    */
  LBM_T_E3 = 3,    /* u.F                               (Eq. 10, third term)     */
  LBM_T_E4 = 4,    /* -sigma_ij d_j u_i                 (Eq. 10, fourth term)    */
  LBM_T_E5 = 5,    /* d_j(u_i sigma_ij)                 (Eq. 10, fifth term)     */
  LBM_T_LHS_Z = 6, /* d_t Omega, Omega = omega^2/2                               */
  LBM_T_Z1 = 7,    /* -div(Omega u)                     (Eq. 11, first term)     */
  LBM_T_Z2 = 8,    /* -Omega div u                      (Eq. 11, second term)    */
  LBM_T_Z3 = 9,    /* omega curl(F/rho)                 (Eq. 11, third term)     */
  LBM_T_Z4 = 10,   /* H_x d_y omega - H_y d_x omega     (Eq. 11, fourth term)    */
  LBM_T_Z5 = 11,   /* d_x(omega H_y) - d_y(omega H_x)   (Eq. 11, fifth term)     */
  LBM_T_USQ = 12,  /* |u|^2 (for the sub-volume Mach number, Eq. 20)             */
  LBM_NTERMS = 13
};

/* ---- one row of the explicit-window output: the 13 box means, then ----------- */
enum {
  LBM_W_DE = 13,   /* delta^E of the window   (Eq. 12)                            */
  LBM_W_DZ = 14,   /* delta^Omega             (Eq. 13)                            */
  LBM_W_MA = 15,   /* Ma_V                    (Eq. 20)                            */
  LBM_NWVALS = 16
};

/* Simulation parameters of one periodic grid. */
typedef struct {
  int32_t nx, ny;      /* grid extents, each >= 16 (the composed 8th-order stencils
                          of the balance reach 12 cells)                          */
  int32_t dtype;       /* population storage: LBM_F32 or LBM_F64.  The arithmetic
                          of the step follows the storage type; every reduction,
                          the balance and the box sums run in FP64.               */
  int32_t has_force;   /* 1: a static external force field is given to lbm_init */
  int32_t with_balance;/* 1: the workspace also holds the balance scratch, so
                          lbm_subvolume_balance can be called on this handle     */
  int32_t layout;      /* population layout in the workspace: LBM_LAYOUT_PLANES
                          ([9][ny][nx]) or LBM_LAYOUT_ROWS ([ny][9][nx], the nine
                          populations of a grid row contiguous)                    */
  double tau;          /* BGK relaxation time (Eq. 1), > 0.5 (Eq. 5: nu > 0)     */
  double drag_alpha;   /* linear drag coefficient alpha >= 0: force -alpha rho u
                          (LBM_FORCE_GUO only)                                   */
  int32_t force_scheme;/* LBM_FORCE_GUO or LBM_FORCE_EDM                         */
  int32_t collision;   /* LBM_COLLISION_BGK or LBM_COLLISION_ENTROPIC (the latter
                          needs has_force = 0, drag_alpha = 0, damp_f0 = 0 and
                          LBM_FORCE_GUO; else LBM_E_UNSUPPORTED)                  */
  /* Spectral damping of the large scales (Sec. 3, Eq. 16), LBM_FORCE_EDM only:
   *   F^R(x) = -damp_f0 sum_{kmin <= |k| <= kmax} u^(k) exp(2 pi i (kx x/nx + ky y/ny)),
   *   u^(k)  = (1/(nx ny)) sum_x u(x) exp(-2 pi i (kx x/nx + ky y/ny)),
   * over integer wavevectors k, the u^(k) being the Fourier-series
   * coefficients of the bare velocity u = j/rho of the pre-collision
   * populations of the same step: F^R = -damp_f0 P[u], P the projection on
   * those modes, so damp_f0 is a damping rate per step (1e-5 in the paper).
   * damp_f0 = 0: no damping.  Otherwise 0 < damp_kmin <= damp_kmax <= 4 and
   * 2 damp_kmax < min(nx, ny).                                              */
  double damp_f0;
  double damp_kmin, damp_kmax;
  void* stream;        /* hipStream_t to enqueue on, or NULL                     */
} lbm_config;

/* Statistics over all windows of one box side L (Sec. 3: mu_l, sigma_l).
 * Every corner (x0, y0) of the periodic grid defines one L x L window when
 * L < min(nx, ny); L == nx == ny is a single window.  delta^E and delta^Omega
 * follow Eqs. 12-13 (denominator: the largest |RHS term|); a zero denominator
 * gives NaN, counted in nan_* and left out of the other figures.  Ma is
 * sqrt(<|u|^2>_V)/c_s (Eq. 20).  std is the population standard deviation. */
typedef struct {
  int32_t L;
  int32_t reserved;
  int64_t count_dE, nan_dE, count_dZ, nan_dZ, count_Ma;
  double mean_dE, std_dE, min_dE, max_dE;
  double mean_dZ, std_dZ, min_dZ, max_dZ;
  double mean_Ma, std_Ma, min_Ma, max_Ma;
} lbm_balance_stats;

/* Step-kernel launch shape.
 * fuse = 0 or 1: one step per launch.  bx*by threads per workgroup (a
 *   multiple of 64, at most 1024); each thread updates vx consecutive sites
 *   in x (1, 2 or 4; nx must be a multiple of vx) on ry consecutive rows.
 * fuse = 2..6: that many steps per launch (temporal blocking; the
 *   intermediate states stay in LDS and registers, bit-identical to single
 *   steps).  A workgroup updates a strip of columns and a band of ry rows;
 *   by = vx = 1; pf = 1 issues the loads of the next row earlier in the row's
 *   iteration.  The fuse - 1 halo columns on each side of the strip are
 *   recomputed: halo = 0 gives them an extra wavefront (bx + 64 threads, a
 *   strip of bx columns, bx a multiple of 64 up to 512); halo = 1 packs them
 *   into the bx threads (a strip of bx - 2 (fuse - 1) columns, bx a multiple of
 *   64 up to 512), which spends no issue slots on a mostly idle wavefront.
 * nt = 1 writes the new populations with non-temporal stores.  halo must be 0
 * for single-step shapes.  lbm_step runs the two steps that record the moment
 * history (and any remainder of the bulk that is not a multiple of fuse) with
 * the single-step kernel. */
typedef struct {
  int32_t bx, by, vx, ry, nt;
  int32_t fuse, pf;
  int32_t halo;
} lbm_tile;

/* ---- library information --------------------------------------------------- */
LBM_API const char* lbm_version(void);
LBM_API const char* lbm_strerror(int status);
LBM_API const char* lbm_last_error(void);

/* ---- single grid ------------------------------------------------------------ */
typedef struct lbm_ctx_s* lbm_ctx;

/* Bytes of device workspace lbm_init needs for cfg (populations A/B, force,
 * moment history, reduction scratch and, if cfg->with_balance, the balance
 * scratch).  Host call, enqueues nothing. */
LBM_API int lbm_workspace_bytes(const lbm_config* cfg, size_t* bytes);

/* Create a handle and set the populations to the equilibrium (Eq. 2) of the
 * given fields: f_l(x, 0) = f^eq_l(rho0(x), u0(x)).
 *   ws, ws_bytes : device workspace, 256-byte aligned, >= lbm_workspace_bytes.
 *   rho0, ux0, uy0 : device FP64 [ny][nx] initial density and velocity.
 *   fx, fy : device FP64 [ny][nx] static external force when cfg->has_force,
 *            else must be NULL.  Copied into the workspace (storage type).
 *   out : receives the handle.  Time starts at t = 0.
 * Asynchronous on cfg->stream; the inputs may be freed after the stream has
 * passed this point. */
LBM_API int lbm_init(const lbm_config* cfg, void* ws, size_t ws_bytes,
             const double* rho0, const double* ux0, const double* uy0,
             const double* fx, const double* fy, lbm_ctx* out);

/* Advance n >= 0 time steps of Eq. 1 (pull streaming fused with BGK collision,
 * Guo forcing with the half-force velocity, implicit linear drag).  The last
 * two steps also record (rho, u) at times t+n-2 and t+n-1 for the time
 * derivative of the balance.  Asynchronous.
 * With LBM_FORCE_EDM a step is: (damping only) the Fourier coefficients of
 * the bare velocity over the damped modes, reduced in a fixed order; then
 * f*_l = f_l - (f_l - f^eq_l(rho, u))/tau + f^eq_l(rho, u + F/rho) - f^eq_l(rho, u)
 * with u = j/rho and F = F_ext + F^R, pull-streamed like the BGK step; the
 * recorded velocity is the scheme's physical one, (j + F/2)/rho.  Such a
 * handle takes single-step shapes with vx = 1 only (lbm_set_tile,
 * lbm_autotune). */
LBM_API int lbm_step(lbm_ctx ctx, int64_t n);

/* Moments at the current time t: rho = sum f, u = (sum f c + F/2)/rho with
 * F = F_ext - alpha rho u solved in closed form (u = j/rho when unforced);
 * with LBM_FORCE_EDM, F = F_ext + F^R(j/rho) of the current populations.
 *   rho, ux, uy : device [ny][nx] outputs of type out_dtype (LBM_F32/LBM_F64),
 *                 any of them may be NULL.
 *   scalars8 : host double[8] (LBM_S_* order) or NULL.  When given, the call
 *              synchronises and returns LBM_E_DIVERGED if a moment is
 *              non-finite or rho <= 0 somewhere (the scalars are still
 *              filled).  Without it the call is asynchronous. */
LBM_API int lbm_moments(lbm_ctx ctx, void* rho, void* ux, void* uy, int32_t out_dtype,
                double* scalars8);

/* Global enstrophy of the current moments: 1/2 sum_x omega(x)^2 with
 * omega = d_x u_y - d_y u_x by Eq. 18 on the periodic grid (FP64, fixed
 * summation order).  Synchronous. */
LBM_API int lbm_enstrophy(lbm_ctx ctx, double* enstrophy);

/* Sub-volume energy and enstrophy balance at the current time t (needs the
 * handle created with with_balance = 1 and the two preceding steps recorded:
 * t >= 2 and the last lbm_step / lbm_load left them, else LBM_E_STATE).
 *   sizes[nsizes] : host, box sides 1 <= L <= min(nx, ny).
 *   out[nsizes]   : host, statistics per L.
 *   dmaps : device FP64 [nsizes][3][ny][nx] maps of delta^E, delta^Omega, Ma
 *           per window corner (y0, x0), or NULL.  For L == nx == ny only
 *           element [0][0] of each map is meaningful.
 *   windows[nwin][3] : host (x0, y0, L) triples, or NULL with nwin = 0.
 *   wterms[nwin][LBM_NWVALS] : host, per window the box means of the 13 fields
 *           (LBM_T_* order) followed by its delta^E, delta^Omega and Ma_V
 *           (LBM_W_*; NaN delta for a zero denominator).
 *   term_fields : device FP64 [13][ny][nx] pointwise integrand fields, or NULL.
 * Synchronous.  Returns LBM_E_DIVERGED if the moments at t are not finite. */
LBM_API int lbm_subvolume_balance(lbm_ctx ctx, const int32_t* sizes, int32_t nsizes,
                          lbm_balance_stats* out, double* dmaps,
                          const int32_t* windows, int32_t nwin, double* wterms,
                          double* term_fields);

/* The statistics of lbm_subvolume_balance (all corners, no maps, windows or
 * term fields) computed beside the following steps instead of in line with
 * them: lbm_balance_begin takes the moments of the current time t (as
 * lbm_subvolume_balance does, with the same preconditions), then enqueues the
 * balance on a second stream of the library (default priority) and returns
 * without waiting for the device; steps enqueued afterwards run concurrently
 * with it.  lbm_balance_end waits for it and fills out[nsizes] with exactly
 * what lbm_subvolume_balance would have returned at t, and returns
 * LBM_E_DIVERGED (with the statistics filled) if the moments of t were not
 * finite or had rho <= 0 somewhere.
 * Until lbm_balance_end, work that would overwrite what the balance reads (the
 * two history-recording steps of lbm_step, another balance, lbm_energy_spectrum,
 * lbm_load) waits for it on the device; a second lbm_balance_begin gives
 * LBM_E_STATE.  sizes[nsizes] : host, 1 <= nsizes <= 64. */
LBM_API int lbm_balance_begin(lbm_ctx ctx, const int32_t* sizes, int32_t nsizes);
LBM_API int lbm_balance_end(lbm_ctx ctx, lbm_balance_stats* out);

/* Optional outputs of the balance for the statistics as the paper presents
 * them (Sec. 3, Table 1; PDFs of Figs. 6-8 and 11-13; pooling over the 25
 * configurations of Sec. 4-5).  Zero-initialise and set what is wanted. */
#define LBM_MAX_EDGES 1024
typedef struct {
  const double* edges;           /* host [3][nedges] bin edges of delta^E, delta^Omega and
                                    Ma_V, each row finite and strictly increasing; NULL:
                                    no histograms                                        */
  int32_t nedges;                /* 1..LBM_MAX_EDGES when edges is given                  */
  int32_t accumulate;            /* 0: statistics and histograms of this call's windows,
                                    starting a new pool; 1: pooled with every call since
                                    the last one with accumulate = 0, size slot k with size
                                    slot k (the caller keeps the sizes in the same order).
                                    The pool lives in the balance workspace.             */
  int64_t* hist;                 /* host [nsizes][3][nedges + 1] counts over all corners
                                    (needs out): bin 0 below edges[0], bin i in
                                    [edges[i-1], edges[i]), bin nedges at or above the last
                                    edge; NaN values are not counted (see nan_*).  NULL:
                                    none                                                  */
  const int32_t* sample_xy;      /* device [total][2] lower corners (x0, y0) of randomly
                                    placed windows, taken modulo (nx, ny); the first
                                    sample_counts[0] have side sizes[0], the next
                                    sample_counts[1] side sizes[1], ...                   */
  const int32_t* sample_counts;  /* host [nsizes] counts >= 0, or NULL: no sampled windows */
  lbm_balance_stats* sample_out; /* host [nsizes] statistics over the sampled windows
                                    (required with sample_counts)                         */
  int64_t* sample_hist;          /* host [nsizes][3][nedges + 1] over the sampled windows,
                                    or NULL                                               */
} lbm_balance_extra;

/* lbm_subvolume_balance with optional extras; `out` may be NULL (no all-corner
 * evaluation, then hist must be NULL) when extra is given.  extra = NULL is
 * lbm_subvolume_balance.  Synchronous. */
LBM_API int lbm_subvolume_balance_ex(lbm_ctx ctx, const int32_t* sizes, int32_t nsizes,
                             lbm_balance_stats* out, double* dmaps, const int32_t* windows,
                             int32_t nwin, double* wterms, double* term_fields,
                             const lbm_balance_extra* extra);

/* Kinetic-energy spectrum of the current velocity (the u of lbm_moments), as
 * in Sec. 4, Fig. 5 and Sec. 5, Fig. 10:
 *   E(s) = 1/2 sum_{k in shell s} |u^(k)|^2,  u^(k) = (1/(nx ny)) sum_x u(x) e^{-ik.x},
 * k the signed integer frequencies (-n/2 .. n/2 - 1 per axis), shell s the
 * wavevectors with (2s - 1)^2 <= 4|k|^2 < (2s + 1)^2 (|k| rounded half up).
 *   spectrum : host double[nshells], 1 <= nshells <= LBM_MAX_SHELLS; shells no
 *              wavevector reaches are 0.
 * nx and ny must be powers of two in [16, 4096] (else LBM_E_UNSUPPORTED).
 * Needs the handle created with with_balance = 1: the balance scratch holds the
 * transforms (the next balance call recomputes its fields).  Synchronous.  The
 * shell sums are FP64 atomics: their last bits may differ between calls. */
#define LBM_MAX_SHELLS 4096
LBM_API int lbm_energy_spectrum(lbm_ctx ctx, double* spectrum, int32_t nshells);
/* The same for caller fields ux, uy (device FP64 [ny][nx]) on `stream`, with a
 * device workspace of lbm_spectrum_workspace_bytes.  Synchronous. */
LBM_API int lbm_spectrum_workspace_bytes(int32_t nx, int32_t ny, size_t* bytes);
LBM_API int lbm_spectrum_fields(int32_t nx, int32_t ny, const double* ux, const double* uy, void* ws,
                        size_t ws_bytes, double* spectrum, int32_t nshells, void* stream);

/* Relaxation of the current populations: alpha (device FP64 [ny][nx], or NULL)
 * of the entropic collision they would undergo now, and the effective viscosity
 * nu_eff = c_s^2 (2 tau / alpha - 1/2) (Eq. 5 with tau_eff = 2 tau / alpha).  For
 * the BGK collision alpha = 2 and nu_eff = nu.  On an entropic handle the
 * balance uses this nu_eff field at level n.  Asynchronous. */
LBM_API int lbm_relaxation(lbm_ctx ctx, double* alpha, double* nu_eff);

/* Current time step. */
LBM_API int lbm_time(lbm_ctx ctx, int64_t* t);

/* Checkpoint: bytes of the state (a 256-byte header, the populations and the
 * recorded moment history), and asynchronous copies of it to / from caller
 * device memory of at least lbm_state_bytes bytes.  The header records the
 * time, the history times, nx, ny, dtype, layout and the state's size;
 * lbm_load reads the header first (synchronising the stream) and returns
 * LBM_E_INVALID, copying nothing, when any of these differs from the handle's,
 * so a state from another grid, dtype or layout is refused.  lbm_load then
 * restores exactly what lbm_save stored. */
LBM_API int lbm_state_bytes(lbm_ctx ctx, size_t* bytes);
LBM_API int lbm_save(lbm_ctx ctx, void* dst_device);
LBM_API int lbm_load(lbm_ctx ctx, const void* src_device);

/* Launch shape of the step kernel: set explicitly, or choose by timing every
 * candidate shape on this grid (trial_steps steps each, state unchanged) and
 * keep the fastest; `chosen` (host, may be NULL) receives it.  The choice is
 * remembered in a process-wide table keyed by (dtype, nx, ny, force) and, if
 * the environment variable LBM_TUNE_CACHE names a file, in that file. */
LBM_API int lbm_set_tile(lbm_ctx ctx, const lbm_tile* tile);
LBM_API int lbm_get_tile(lbm_ctx ctx, lbm_tile* tile);
LBM_API int lbm_autotune(lbm_ctx ctx, int32_t trial_steps, lbm_tile* chosen);
/* Record `tile` in the same process-wide table (and cache file) for the grid
 * described by cfg (dtype, nx, ny, forced or not, layout), as if lbm_autotune
 * had chosen it: later handles of that grid start with it and lbm_adjoint_run
 * uses it for its first forward pass.  Host call; LBM_E_INVALID for a shape
 * the grid does not accept. */
LBM_API int lbm_set_tuned_tile(const lbm_config* cfg, const lbm_tile* tile);

/* hipGraph replay of `chunk` (even, >= 2) step launches for long lbm_step
 * calls; chunk = 0 launches every step directly. */
LBM_API int lbm_set_graph(lbm_ctx ctx, int32_t chunk);

/* Device-timed step kernels: while enabled, lbm_step brackets its step
 * launches with HIP events on the handle's stream.  lbm_step_time
 * synchronises and returns the summed milliseconds and kernel launches since
 * the last reset (reset = 1 clears them afterwards). */
LBM_API int lbm_step_timing(lbm_ctx ctx, int32_t enable);
LBM_API int lbm_step_time(lbm_ctx ctx, double* ms, int64_t* launches, int32_t reset);

/* Free the handle (not the caller's workspace).  Synchronises its stream. */
LBM_API int lbm_destroy(lbm_ctx ctx);

/* ---- balance of caller-given fields ------------------------------------------ */
/* Inputs of the stateless balance: three time levels ordered (n-2, n-1, n). */
typedef struct {
  int32_t nx, ny;
  double nu;                /* kinematic viscosity (Eq. 5)                      */
  const double* rho[3];     /* device FP64 [ny][nx] per level                   */
  const double* ux[3];
  const double* uy[3];
  const double* fx;         /* device FP64 [ny][nx] total body force at level n, */
  const double* fy;         /* or NULL for none                                 */
  void* stream;
  const double* nu_field;   /* device FP64 [ny][nx] kinematic viscosity at level n
                               (in the stress of Eqs. 8-11), or NULL: nu everywhere */
} lbm_balance_input;

/* Device workspace of lbm_balance_fields for an nx x ny grid. */
LBM_API int lbm_balance_workspace_bytes(int32_t nx, int32_t ny, size_t* bytes);

/* The sub-volume balance of lbm_subvolume_balance on given fields (same
 * outputs, same window definition).  Synchronous. */
LBM_API int lbm_balance_fields(const lbm_balance_input* in, void* ws, size_t ws_bytes,
                       const int32_t* sizes, int32_t nsizes, lbm_balance_stats* out,
                       double* dmaps, const int32_t* windows, int32_t nwin,
                       double* wterms, double* term_fields);
/* lbm_balance_fields with the extras of lbm_subvolume_balance_ex (the pool of
 * accumulate = 1 lives in ws). */
LBM_API int lbm_balance_fields_ex(const lbm_balance_input* in, void* ws, size_t ws_bytes,
                          const int32_t* sizes, int32_t nsizes, lbm_balance_stats* out,
                          double* dmaps, const int32_t* windows, int32_t nwin,
                          double* wterms, double* term_fields, const lbm_balance_extra* extra);

/* For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc):
 * lbm_balance_fields without a workspace argument.  Its scratch is a static
 * device array of 96 MiB per GPU, held by the library until the process ends,
 * enough for grids up to about 590 x 590 (lbm_balance_workspace_bytes(nx, ny)
 * must not exceed it; larger grids return LBM_E_NOMEM before anything is
 * enqueued).  The call itself allocates no device memory and calls no
 * allocating library routine; the caller passes inputs and outputs exactly as
 * for lbm_balance_fields and gets the same results (the same kernels).  Every
 * call on one GPU uses that GPU's one array, so calls that overlap on one GPU
 * (other host threads, other streams) race; nothing depends on what a previous
 * call left there.  Synchronous on in->stream, whose device must be current. */
LBM_API int lbm_balance_fields_noalloc(const lbm_balance_input* in, const int32_t* sizes, int32_t nsizes,
                                       lbm_balance_stats* out, double* dmaps, const int32_t* windows,
                                       int32_t nwin, double* wterms, double* term_fields);

/* ---- batched ensemble ---------------------------------------------------------- */
/* Many independent grids (sizes, tau, drag and force may differ per run; the
 * storage type must be the same) advanced together.  Mode LBM_BATCH_PERSISTENT
 * runs `chunk` steps of every run in one launch of a persistent kernel whose
 * workgroups take equal slices of a (run, row-band) work list and meet at a
 * grid-wide barrier between steps; the barrier waits are bounded and report
 * LBM_E_TIMEOUT instead of hanging.  Mode LBM_BATCH_PER_STEP launches one
 * kernel per step over the same work list.  Mode LBM_BATCH_MULTI_STEP
 * advances every run by K steps per launch over the (run, strip, band) tiles
 * of the single-grid multi-step kernel (see lbm_tile.fuse), bit-identical to
 * single steps; step counts that are not a multiple of K end with single-step
 * launches.  Mode LBM_BATCH_PERSISTENT_MULTI runs those K-step tiles inside
 * one persistent launch per chunk: a round of K steps over every tile, then
 * a grid-wide barrier (bounded waits as above), bit-identical to the
 * multi-step mode; the steps of a chunk beyond a multiple of K are single-step
 * launches.  All modes are replayed from hipGraphs. */
enum { LBM_BATCH_PERSISTENT = 0, LBM_BATCH_PER_STEP = 1, LBM_BATCH_MULTI_STEP = 2,
       LBM_BATCH_PERSISTENT_MULTI = 3 };
typedef struct lbm_batch_s* lbm_batch;

/* cfgs[nruns]: per-run configuration; with_balance must be 0 and collision
 * LBM_COLLISION_BGK (LBM_E_UNSUPPORTED otherwise), stream is taken from
 * cfgs[0].  Every run has the same force_scheme.  LBM_FORCE_EDM runs (Sec. 3,
 * at most 64) share nx, ny, layout, has_force and the damped shell (tau,
 * damp_f0 and the force fields may differ); they step in
 * LBM_BATCH_PER_STEP mode only (set at init; the other modes, set_tile,
 * set_multi and autotune give LBM_E_UNSUPPORTED), each step one launch of
 * every run's Fourier sums, one of their coefficients and one of the step
 * kernel, bit-identical to the runs stepped alone. */
LBM_API int lbm_batch_workspace_bytes(const lbm_config* cfgs, int32_t nruns, size_t* bytes);
/* rho0/ux0/uy0/fx/fy: host arrays of nruns device FP64 pointers (fx/fy NULL,
 * or entries NULL for runs without force).  Every run starts at f^eq of its
 * fields (Eq. 2); time t = 0. */
LBM_API int lbm_batch_init(const lbm_config* cfgs, int32_t nruns, void* ws, size_t ws_bytes,
                   const double* const* rho0, const double* const* ux0,
                   const double* const* uy0, const double* const* fx,
                   const double* const* fy, lbm_batch* out);
/* mode: LBM_BATCH_PERSISTENT, LBM_BATCH_PER_STEP, LBM_BATCH_MULTI_STEP or
 * LBM_BATCH_PERSISTENT_MULTI; chunk: even number of steps per graph replay
 * (2..100000). */
LBM_API int lbm_batch_set_mode(lbm_batch b, int32_t mode, int32_t chunk);
/* Work-item shape: block_threads (256, 512 or 1024) threads per workgroup;
 * vx (1, 2 or 4, dividing every run's nx) sites per thread; band_rows (1..64)
 * groups of block_threads*vx consecutive sites per work item. */
LBM_API int lbm_batch_set_tile(lbm_batch b, int32_t block_threads, int32_t vx, int32_t band_rows);
/* Shape of the multi-step mode: t->fuse = K (2..6) steps per launch, t->bx =
 * workgroup width (a multiple of 64, at most 512: the strip width with
 * t->halo = 0, the strip plus its 2 (K - 1) halo columns with t->halo = 1, as
 * in lbm_tile), t->ry = band height (>= 8 rows), t->nt = non-temporal stores;
 * by = vx = 1.  The next-row loads are always issued early (pf = 1). */
LBM_API int lbm_batch_set_multi(lbm_batch b, const lbm_tile* t);
LBM_API int lbm_batch_get_multi(lbm_batch b, lbm_tile* t);
/* Time every (mode, block_threads, vx, band_rows) candidate, every
 * multi-step shape and the fastest of those in the persistent multi-step mode
 * over about trial_steps (even) steps and keep the fastest per step; the chosen mode is readable with lbm_batch_get_mode, the
 * multi-step shape with lbm_batch_get_multi.  The trials are real steps: the
 * ensemble advances by them and lbm_batch_time says so. */
LBM_API int lbm_batch_autotune(lbm_batch b, int32_t trial_steps, int32_t* block_threads,
                       int32_t* vx, int32_t* band_rows);
LBM_API int lbm_batch_get_mode(lbm_batch b, int32_t* mode, int32_t* chunk);
/* Advance every run by n steps (asynchronous). */
LBM_API int lbm_batch_step(lbm_batch b, int64_t n);
/* Moments of one run, as lbm_moments.  Synchronises to read the barrier error
 * flag first: LBM_E_TIMEOUT if a persistent launch gave up waiting. */
LBM_API int lbm_batch_moments(lbm_batch b, int32_t run, void* rho, void* ux, void* uy,
                      int32_t out_dtype, double* scalars8);
LBM_API int lbm_batch_time(lbm_batch b, int64_t* t);
/* Total lattice sites over all runs (one step updates this many sites). */
LBM_API int64_t lbm_batch_sites(lbm_batch b);
LBM_API int lbm_batch_destroy(lbm_batch b);

/* ---- adjoint ---------------------------------------------------------------------- */
/* Differentiable unforced run: f(0) = f^eq(rho = 1, u0), `steps` steps of
 * Eq. 1, then the loss J = mean over all box x box windows of
 * (RHS^Omega_V - LHS^Omega_V)^2 (Eq. 11 residual at the last step; a box of
 * side nx == ny is one window).  The gradient is obtained by a discrete
 * adjoint sweep: checkpoints of the populations every ckpt_every steps, each
 * segment recomputed forward and swept backward.  With two or more segments the
 * workspace size returned holds two segment buffers: a stream of the library's own
 * recomputes the next segment while the current one is swept.  A workspace smaller by
 * one segment buffer, (ckpt_every + 1) * 9 * nx * ny elements of the dtype rounded up
 * to 256 bytes, also works, without that overlap; results are the same bits. */
typedef struct {
  int32_t nx, ny;
  int32_t dtype;        /* LBM_F32 or LBM_F64 populations and adjoint states   */
  int32_t box;          /* window side L of the loss                           */
  int32_t ckpt_every;   /* K >= 1                                              */
  int32_t reserved;
  int64_t steps;        /* T >= 2                                              */
  double tau;
  void* stream;
} lbm_adjoint_config;

LBM_API int lbm_adjoint_workspace_bytes(const lbm_adjoint_config* cfg, size_t* bytes);

/* ux0, uy0 : device FP64 [ny][nx] initial velocity.
 * loss : host double, receives J.
 * grad_ux0, grad_uy0 : device FP64 [ny][nx] dJ/du0, or both NULL for the loss only.
 * grad_tau : host double dJ/dtau, or NULL.
 * Synchronous. */
LBM_API int lbm_adjoint_run(const lbm_adjoint_config* cfg, void* ws, size_t ws_bytes,
                    const double* ux0, const double* uy0, double* loss,
                    double* grad_ux0, double* grad_uy0, double* grad_tau);

/* ---- three dimensions: D3Q19 and D3Q27 --------------------------------------------- */
/* The same method in three dimensions: the LBGK update of Eq. 1 with the
 * equilibrium of Eq. 2 on the D3Q19 lattice (rest weight 1/3, six axis
 * velocities of weight 1/18, twelve edge diagonals of weight 1/36,
 * c_s^2 = 1/3) or the D3Q27 lattice (every velocity in {-1, 0, 1}^3; weights
 * 8/27, 2/27 for the axes, 1/54 for the edges, 1/216 for the corners, the same
 * c_s^2), Guo's forcing term with the half-force velocity, and the
 * balances of Sec. 2 in index form over cubic sub-volumes L^3.  In 3D the
 * enstrophy equation keeps the vortex-stretching term omega_i omega_j d_j u_i
 * (Sec. 2 drops it only because it vanishes in 2D).
 * Fields are row-major [nz][ny][nx] (x fastest), periodic in x, y and z. */
typedef struct {
  int32_t nx, ny, nz;  /* 16..4096 each                                         */
  int32_t dtype;       /* LBM_F32 or LBM_F64 population storage and step arithmetic */
  int32_t has_force;   /* 1: static body force (fx, fy, fz given to lbm3_init)   */
  int32_t with_balance;/* 1: reserve the balance scratch (lbm3_subvolume_balance) */
  double tau;          /* relaxation time > 1/2; nu = (tau - 1/2)/3              */
  void* stream;        /* hipStream_t to enqueue on, or NULL                     */
  int32_t lattice;     /* LBM3_D3Q19 (0) or LBM3_D3Q27 (1); populations are
                          row-interleaved [nz][ny][Q][nx], Q = 19 or 27          */
  int32_t reserved;    /* 0                                                      */
} lbm3_config;
enum { LBM3_D3Q19 = 0, LBM3_D3Q27 = 1 };

typedef struct lbm3_ctx_s* lbm3_ctx;

/* Scalars of lbm3_moments, in this order. */
enum {
  LBM3_S_MASS = 0, LBM3_S_MOMX = 1, LBM3_S_MOMY = 2, LBM3_S_MOMZ = 3, LBM3_S_ENERGY = 4,
  LBM3_S_MAXU = 5, LBM3_S_MINRHO = 6, LBM3_S_NONFINITE = 7, LBM3_S_TIME = 8, LBM3_NSCALARS = 9
};

/* Pointwise integrand fields of the 3D balance, in this order (term_fields):
 * d_t E, -div(E u), -u.grad p (p = rho/3), u.F, -sigma_ij d_j u_i,
 * d_j(u_i sigma_ij); d_t Omega, -div(Omega u), -Omega div u,
 * omega.curl(F/rho), H.curl(omega), div(H x omega), omega_i omega_j d_j u_i
 * (vortex stretching); |u|^2.  E = rho|u|^2/2, Omega = |omega|^2/2,
 * omega = curl u, sigma_ij = nu rho (d_j u_i + d_i u_j), H_i = d_j sigma_ij/rho;
 * space derivatives by Eq. 18 along each axis, d_t by Eq. 17. */
enum {
  LBM3_T_LHS_E = 0, LBM3_T_E1, LBM3_T_E2, LBM3_T_E3, LBM3_T_E4, LBM3_T_E5,
  LBM3_T_LHS_Z, LBM3_T_Z1, LBM3_T_Z2, LBM3_T_Z3, LBM3_T_Z4, LBM3_T_Z5, LBM3_T_Z6,
  LBM3_T_USQ, LBM3_NTERMS
};

/* Launch shape of the bulk of lbm3_step.  fuse = 1: one step per launch (the
 * other fields are ignored; the only shape of a D3Q27 handle).  fuse = 2..4
 * (D3Q19): that many steps per launch
 * (temporal blocking; bit-identical to one-step launches): workgroups of
 * bx * by lanes (a multiple of 64, at most 512, with 2 * 16 * bx * by values of
 * LDS at most 64 KiB) each update a tile of (bx - 2 (fuse - 1)) x
 * (by - 2 (fuse - 1)) columns over a band of bz planes. */
typedef struct {
  int32_t fuse, bx, by, bz;
} lbm3_tile;

/* Bytes of device workspace lbm3_init needs for cfg.  Host call. */
LBM_API int lbm3_workspace_bytes(const lbm3_config* cfg, size_t* bytes);

/* Create a 3D handle with f_l(x, 0) = f^eq_l(rho0(x), u0(x)).
 *   ws, ws_bytes : device workspace, 256-byte aligned, >= lbm3_workspace_bytes.
 *   rho0, ux0, uy0, uz0 : device FP64 [nz][ny][nx] initial fields.
 *   fx, fy, fz : device FP64 [nz][ny][nx] static force when cfg->has_force,
 *                else NULL; copied into the workspace.
 * Asynchronous on cfg->stream. */
LBM_API int lbm3_init(const lbm3_config* cfg, void* ws, size_t ws_bytes, const double* rho0,
                      const double* ux0, const double* uy0, const double* uz0, const double* fx,
                      const double* fy, const double* fz, lbm3_ctx* out);

/* Advance n >= 0 steps (pull streaming fused with the BGK collision and Guo's
 * term; the bulk in launches of the lbm3_tile shape, the remainder and the last
 * two steps one per launch); the last two steps record (rho, u) for the time
 * derivative of the balance.  Asynchronous. */
LBM_API int lbm3_step(lbm3_ctx ctx, int64_t n);

/* Moments at the current time: rho = sum f, u = (sum f c + F/2)/rho, evaluated
 * in the storage type and written as FP64.
 *   rho, ux, uy, uz : device FP64 [nz][ny][nx], any may be NULL.
 *   scalars9 : host double[LBM3_NSCALARS] or NULL; when given the call
 *              synchronises and returns LBM_E_DIVERGED for a non-finite
 *              moment or rho <= 0 (the scalars are still filled). */
LBM_API int lbm3_moments(lbm3_ctx ctx, double* rho, double* ux, double* uy, double* uz,
                         double* scalars9);

LBM_API int lbm3_time(lbm3_ctx ctx, int64_t* t);

/* Bulk launch shape (lbm3_tile); LBM_E_INVALID for a shape that does not fit. */
LBM_API int lbm3_set_tile(lbm3_ctx ctx, const lbm3_tile* tile);
LBM_API int lbm3_get_tile(lbm3_ctx ctx, lbm3_tile* tile);
/* Time every candidate shape (trial_launches launches each, per step, from the
 * current state without changing it) and keep the fastest.  Synchronous. */
LBM_API int lbm3_autotune(lbm3_ctx ctx, int32_t trial_launches, lbm3_tile* chosen);

/* The 3D sub-volume balance at the current time t (handle with
 * with_balance = 1, t >= 2 with the two preceding steps recorded, else
 * LBM_E_STATE).  For every box side L in sizes[nsizes] (host, 1 <= L <=
 * min(nx, ny, nz)) the statistics of delta^E, delta^Omega (Eqs. 12-13 with
 * the stretching term among the enstrophy terms) and Ma_V = sqrt(<|u|^2>)/c_s
 * over the L^3 cubes at every corner (z0, y0, x0), periodic; L == nx == ny == nz
 * is the single whole-domain cube.  out[nsizes] : host.
 *   term_fields : device FP64 [LBM3_NTERMS][nz][ny][nx] integrands, or NULL.
 * Synchronous. */
LBM_API int lbm3_subvolume_balance(lbm3_ctx ctx, const int32_t* sizes, int32_t nsizes,
                                   lbm_balance_stats* out, double* term_fields);

/* Release the handle (after the stream has drained); the workspace is the caller's. */
LBM_API int lbm3_destroy(lbm3_ctx ctx);

/* ---- bandwidth reference ----------------------------------------------------------- */
/* Plain device-to-device copy of `bytes` (a multiple of 16) with 16-byte
 * vector loads and stores, on `stream`: the achievable-bandwidth reference
 * for the step kernel.  Asynchronous. */
LBM_API int lbm_copy(void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
