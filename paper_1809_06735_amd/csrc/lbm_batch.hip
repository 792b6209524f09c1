// Batched ensemble: many independent periodic grids advanced together.
//
// The work of one time step of every run is a list of equal-size items, each a
// contiguous range of (threads * vx * ir) sites of one run in row-major order.
// Persistent mode: one kernel with an occupancy-sized grid (every workgroup
// resident at once) walks the item list for `chunk` steps; between steps the
// workgroups meet at a grid-wide barrier (an atomic counter with a bounded
// wait: a wait that runs out sets an error flag and the kernel exits instead
// of hanging).  Per-step mode: one ordinary launch per step over the same list.
// Multi-step mode: one launch advances every run by K steps, its workgroups
// taking the (run, strip, band) tiles of the single-grid multi-step kernel
// (temporal blocking through LDS).  Persistent multi-step mode: one persistent
// kernel whose workgroups take those tiles, K steps per round, with a grid
// barrier between rounds.  All modes are captured into hipGraphs and
// replayed.  The arithmetic per site is the single-grid step's (pull, BGK
// collide, Guo force, drag).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "lbm_fused.h"
#include "lbm_internal.h"
#include "lbm_site.h"

namespace lbm {
namespace {

constexpr int kBT = 256;    // smallest workgroup of the batch kernels (threads)
constexpr int kBTMax = 1024;

struct RunDesc {
  void* pop[2];
  const void* fx;
  const void* fy;
  size_t ps, rs;
  int nx, ny;
  double omega;
  double alpha;
  int forced;
  int pad;
};

// the grid barrier's counters, error flag, bounded wait and variant
struct BarrierArgs {
  unsigned* barrier;      // zeroed before each persistent launch
  int* error;             // set to 1 by a barrier wait that ran out
  unsigned spin_limit;
  int flavor;             // grid-barrier variant (see grid_barrier)
};

struct BatchArgs {
  const RunDesc* runs;
  const int* item_run;
  const int* item_start;
  int nitems;
  int ir;                 // site groups per thread per item
  int bt;                 // threads per workgroup (256, 512 or 1024)
  int parity0;            // buffer index holding the state at the first step
  int nsteps;
  BarrierArgs bar;
};

template <typename T, int VX>
__device__ __forceinline__ void process_item(const BatchArgs& a, int item, int par) {
  const RunDesc r = a.runs[a.item_run[item]];
  const int nx = r.nx, ny = r.ny;
  const size_t plane = static_cast<size_t>(nx) * ny;
  const T* __restrict__ src = static_cast<const T*>(r.pop[par]);
  T* __restrict__ dst = static_cast<T*>(r.pop[par ^ 1]);
  const T omega = T(r.omega);
  const T guo = T(1) - T(0.5) * T(r.omega);
  const T alpha = T(r.alpha);
  const int start = a.item_start[item];
  for (int k = 0; k < a.ir; ++k) {
    const size_t site =
        static_cast<size_t>(start) + (static_cast<size_t>(k) * a.bt + threadIdx.x) * VX;
    if (site >= plane) break;
    const int y = static_cast<int>(site / nx);
    const int x0 = static_cast<int>(site - static_cast<size_t>(y) * nx);
    const int yn = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    T d[9][VX];
    step_detail::pull_all<T, VX>(src, r.ps, r.rs, nx, x0, y, yn, yp, d);
    const size_t row = static_cast<size_t>(y) * nx + x0;
    T o[9][VX];
    if (r.forced) {
      T fx[VX], fy[VX];
      if (r.fx) {
        step_detail::load_aligned<T, VX>(static_cast<const T*>(r.fx) + row, fx);
        step_detail::load_aligned<T, VX>(static_cast<const T*>(r.fy) + row, fy);
      } else {
#pragma unroll
        for (int i = 0; i < VX; ++i) fx[i] = fy[i] = T(0);
      }
#pragma unroll
      for (int i = 0; i < VX; ++i) {
        T di[9], oi[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) di[l] = d[l][i];
        step_detail::SiteMoments<T, true> m(di, fx[i], fy[i], alpha);
        step_detail::collide_site<T, true>(di, m, omega, guo, oi);
#pragma unroll
        for (int l = 0; l < 9; ++l) o[l][i] = oi[l];
      }
    } else {
#pragma unroll
      for (int i = 0; i < VX; ++i) {
        T di[9], oi[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) di[l] = d[l][i];
        step_detail::SiteMoments<T, false> m(di, T(0), T(0), alpha);
        step_detail::collide_site<T, false>(di, m, omega, guo, oi);
#pragma unroll
        for (int l = 0; l < 9; ++l) o[l][i] = oi[l];
      }
    }
#pragma unroll
    for (int l = 0; l < 9; ++l)
      step_detail::store_aligned<T, VX, true>(dst + l * r.ps + static_cast<size_t>(y) * r.rs + x0, o[l]);
  }
}

// Grid-wide barrier number `gen` (1, 2, ...), three variants with the same
// meaning (every workgroup's writes before the barrier are visible to every
// workgroup after it; agent-scope release/acquire, which on this chip write
// back and invalidate the per-XCD L2 caches):
//   0: every wavefront fences; one counter
//   1: thread 0 of each workgroup carries the release/acquire; one counter
//   2: as 1, with the workgroups split into 8 groups (blockIdx % 8): the last
//      arrival of a group forwards to a global counter and, once all groups
//      arrived, releases its group through a per-group flag
// A wait that runs out of spins sets the error flag; every later barrier then
// fails at once, so every workgroup leaves the kernel.
// Words 0 .. 17 (x kCounterStride) hold the barrier's counters and flags,
// words 18 .. 25 the persistent multi-step kernel's tile tickets.
constexpr int kCounterStride = 64;  // unsigned words between counters (256 bytes)
constexpr int kTicketSlot = 18;
constexpr int kBarrierWords = kCounterStride * (kTicketSlot + 8);

// Polls with relaxed loads (an acquire load would invalidate the caches on
// every poll, under the feet of the workgroups still computing) and acquires
// once, by a fence, when the target is reached.
__device__ __forceinline__ bool spin_until(const BarrierArgs& a, unsigned* p, unsigned target) {
  unsigned spins = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++spins > a.spin_limit) {
      __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__device__ bool grid_barrier(const BarrierArgs& a, unsigned gen) {
  __shared__ int ok;
  if (a.flavor == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      good = 0;
    } else if (a.flavor != 2) {
      __hip_atomic_fetch_add(a.barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      good = spin_until(a, a.barrier, gen * gridDim.x);
    } else {
      const unsigned G = gridDim.x;
      const unsigned g = blockIdx.x & 7;
      const unsigned gsize = (G - g + 7) / 8;
      const unsigned ngroups = G < 8 ? G : 8;
      unsigned* cg = a.barrier + kCounterStride * (1 + g);
      unsigned* rel = a.barrier + kCounterStride * (9 + g);
      // arrivals only release (an acquire would invalidate the caches of the
      // workgroups still computing); the last arrival of the group acquires the
      // others' writes before it forwards them
      const unsigned prev = __hip_atomic_fetch_add(cg, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (prev + 1 == gen * gsize) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_fetch_add(a.barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        good = spin_until(a, a.barrier, gen * ngroups);
        if (good) __hip_atomic_store(rel, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        good = spin_until(a, rel, gen);
      }
    }
    ok = good;
  }
  __syncthreads();
  if (a.flavor == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok != 0;
}

// Persistent one-step mode: the work list is split into eight contiguous parts
// drawn from tickets, as the tiles of the persistent multi-step kernel below.
template <typename T, int VX>
__global__ void __launch_bounds__(kBTMax) k_batch_persistent(BatchArgs a) {
  __shared__ unsigned tk;
  const unsigned per_part = gridDim.x >> 3;
  const int part = blockIdx.x & 7;
  const int per = (a.nitems + 7) / 8;
  const int first = part * per;
  const unsigned count = static_cast<unsigned>(max(0, min(a.nitems, first + per) - first));
  unsigned* ticket = a.bar.barrier + kCounterStride * (kTicketSlot + part);
  for (int s = 0; s < a.nsteps; ++s) {
    const int par = (a.parity0 + s) & 1;
    const unsigned base = static_cast<unsigned>(s) * (count + per_part);  // modulo 2^32
    for (;;) {
      if (threadIdx.x == 0)
        tk = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base;
      __syncthreads();
      const unsigned k = tk;
      __syncthreads();  // every thread has read tk before thread 0 draws again
      if (k >= count) break;  // uniform over the workgroup
      process_item<T, VX>(a, first + static_cast<int>(k), par);
    }
    if (s + 1 < a.nsteps)
      if (!grid_barrier(a.bar, static_cast<unsigned>(s + 1))) return;
  }
}

template <typename T, int VX>
__global__ void __launch_bounds__(kBTMax) k_batch_step(BatchArgs a) {
  process_item<T, VX>(a, blockIdx.x, a.parity0);
}

// Multi-step mode: item it (XCD-aware numbering) is tile item_tile[it] of run
// item_run[it]; every run advances K steps from buffer `parity`.
struct FusedArgs {
  const RunDesc* runs;
  const int* item_run;
  const int* item_tile;
  int nitems;
  int per_xcd;
  int W, H;     // strip width (output columns) and band height
  int threads;  // W + 64 (halo wavefront) or W + 2 (K - 1) (packed halo)
  int halo;
  int parity;
};

template <typename T, int K, bool NT>
__global__ void __launch_bounds__(fused_detail::kFusedMaxThreads) k_batch_fused(FusedArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int it = (b & 7) * a.per_xcd + (b >> 3);
  if (it >= a.nitems) return;  // uniform over the workgroup
  const RunDesc r = a.runs[a.item_run[it]];
  StepParams p{};
  p.src = r.pop[a.parity];
  p.dst = r.pop[a.parity ^ 1];
  p.fx = r.fx;
  p.fy = r.fy;
  p.nx = r.nx;
  p.ny = r.ny;
  p.ps = r.ps;
  p.rs = r.rs;
  p.omega = r.omega;
  p.alpha = r.alpha;
  const int strips = (r.nx + a.W - 1) / a.W;
  T* const lds = reinterpret_cast<T*>(smem_raw);
  if (r.forced)
    fused_detail::fused_tile<T, K, true, NT, true>(p, lds, a.W, a.H, strips, a.item_tile[it], a.halo != 0);
  else
    fused_detail::fused_tile<T, K, false, NT, true>(p, lds, a.W, a.H, strips, a.item_tile[it], a.halo != 0);
}

// Persistent multi-step mode: `rounds` rounds of K steps, round r from buffer
// parity + r.  The tile list is split into eight contiguous parts, part x
// taken by the workgroups b with b % 8 == x (gridDim.x is a multiple of 8), so
// that a run's neighbouring tiles, whose halos overlap, tend to share an L2.
// Within a part the workgroups draw tiles from a ticket counter, so a
// workgroup that finishes early takes more.  Each workgroup draws until a
// ticket is past the part's end, so a round adds exactly (tiles + workgroups)
// of the part to its counter and round r's tickets start at r times that.
// Tiles are independent within a round, so which workgroup takes a tile does
// not change any result.  Correctness does not depend on where a workgroup
// runs: the grid barrier between rounds publishes every write to every
// workgroup.
template <typename T, int K, bool NT>
__global__ void __launch_bounds__(fused_detail::kFusedMaxThreads) k_batch_fused_persistent(FusedArgs a,
                                                                                          int rounds,
                                                                                          BarrierArgs bar) {
  extern __shared__ unsigned char smem_raw[];
  T* const lds = reinterpret_cast<T*>(smem_raw);
  __shared__ unsigned tk;
  const unsigned per_part = gridDim.x >> 3;
  const int part = blockIdx.x & 7;
  const int first = part * a.per_xcd;
  const unsigned count = static_cast<unsigned>(max(0, min(a.nitems, first + a.per_xcd) - first));
  unsigned* ticket = bar.barrier + kCounterStride * (kTicketSlot + part);
  for (int r = 0; r < rounds; ++r) {
    const int par = (a.parity + r) & 1;
    const unsigned base = static_cast<unsigned>(r) * (count + per_part);  // modulo 2^32
    for (;;) {
      if (threadIdx.x == 0)
        tk = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base;
      __syncthreads();
      const unsigned k = tk;  // rewritten only after the tile's barriers
      if (k >= count) break;  // uniform over the workgroup
      const int it = first + static_cast<int>(k);
      const RunDesc rd = a.runs[a.item_run[it]];
      StepParams p{};
      p.src = rd.pop[par];
      p.dst = rd.pop[par ^ 1];
      p.fx = rd.fx;
      p.fy = rd.fy;
      p.nx = rd.nx;
      p.ny = rd.ny;
      p.ps = rd.ps;
      p.rs = rd.rs;
      p.omega = rd.omega;
      p.alpha = rd.alpha;
      const int strips = (rd.nx + a.W - 1) / a.W;
      if (rd.forced)
        fused_detail::fused_tile<T, K, true, NT, true>(p, lds, a.W, a.H, strips, a.item_tile[it], a.halo != 0);
      else
        fused_detail::fused_tile<T, K, false, NT, true>(p, lds, a.W, a.H, strips, a.item_tile[it], a.halo != 0);
      __syncthreads();  // the next tile rewrites the LDS rows
    }
    if (r + 1 < rounds)
      if (!grid_barrier(bar, static_cast<unsigned>(r + 1))) return;
  }
}

template <typename T, int K>
const void* fused_persistent_fn(bool nt) {
  return nt ? reinterpret_cast<const void*>(&k_batch_fused_persistent<T, K, true>)
            : reinterpret_cast<const void*>(&k_batch_fused_persistent<T, K, false>);
}

template <typename T>
const void* fused_persistent_fn(int K, bool nt) {
  switch (K) {
    case 2: return fused_persistent_fn<T, 2>(nt);
    case 3: return fused_persistent_fn<T, 3>(nt);
    case 4: return fused_persistent_fn<T, 4>(nt);
    case 5: return fused_persistent_fn<T, 5>(nt);
    default: return fused_persistent_fn<T, 6>(nt);
  }
}

template <typename T, int K>
void launch_batch_fused_k(const FusedArgs& a, bool nt, hipStream_t s) {
  const size_t lds = fused_lds_bytes(a.W, K, sizeof(T) == 8 ? LBM_F64 : LBM_F32);
  if (nt)
    hipLaunchKernelGGL((k_batch_fused<T, K, true>), dim3(a.per_xcd * 8), dim3(a.threads), lds, s, a);
  else
    hipLaunchKernelGGL((k_batch_fused<T, K, false>), dim3(a.per_xcd * 8), dim3(a.threads), lds, s, a);
}

template <typename T>
void launch_batch_fused(int K, const FusedArgs& a, bool nt, hipStream_t s) {
  switch (K) {
    case 2: launch_batch_fused_k<T, 2>(a, nt, s); break;
    case 3: launch_batch_fused_k<T, 3>(a, nt, s); break;
    case 4: launch_batch_fused_k<T, 4>(a, nt, s); break;
    case 5: launch_batch_fused_k<T, 5>(a, nt, s); break;
    default: launch_batch_fused_k<T, 6>(a, nt, s); break;
  }
}

__global__ void k_batch_reset(unsigned* barrier) {
  for (int i = threadIdx.x; i < kBarrierWords; i += blockDim.x) barrier[i] = 0u;
}

template <typename T, int VX>
int occupancy_blocks(int bt, int* blocks) {
  int per_cu = 0;
  LBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<T, VX>, bt, 0));
  int dev = 0;
  LBM_HIP(hipGetDevice(&dev));
  int cus = 0;
  LBM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *blocks = std::max(1, per_cu * cus);
  return LBM_OK;
}

template <typename T>
int occupancy_for(int vx, int bt, int* blocks) {
  switch (vx) {
    case 1: return occupancy_blocks<T, 1>(bt, blocks);
    case 2: return occupancy_blocks<T, 2>(bt, blocks);
    default: return occupancy_blocks<T, 4>(bt, blocks);
  }
}

template <typename T, int VX>
void launch_batch_t(bool persistent, const BatchArgs& a, int grid, hipStream_t s) {
  if (persistent)
    hipLaunchKernelGGL((k_batch_persistent<T, VX>), dim3(grid), dim3(a.bt), 0, s, a);
  else
    hipLaunchKernelGGL((k_batch_step<T, VX>), dim3(a.nitems), dim3(a.bt), 0, s, a);
}

template <typename T>
void launch_batch_vx(int vx, bool persistent, const BatchArgs& a, int grid, hipStream_t s) {
  switch (vx) {
    case 1: launch_batch_t<T, 1>(persistent, a, grid, s); break;
    case 2: launch_batch_t<T, 2>(persistent, a, grid, s); break;
    default: launch_batch_t<T, 4>(persistent, a, grid, s); break;
  }
}

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_batch_s {
  int nruns = 0;
  int dtype = LBM_F32;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<lbm_config> cfg;
  std::vector<RunDesc> runs;     // host copy
  RunDesc* d_runs = nullptr;
  int* d_item_run = nullptr;
  int* d_item_start = nullptr;
  size_t item_cap = 0;
  int* d_fitem_run = nullptr;    // multi-step work list: (run, tile)
  int* d_fitem_tile = nullptr;
  size_t fitem_cap = 0;
  int nfitems = 0;
  int fgrid = 0;                 // persistent multi-step grid (a multiple of 8)
  lbm_tile ftile{256, 1, 1, 64, 1, 4, 1};  // multi-step shape: strip, band, K, nt
  unsigned* d_barrier = nullptr;
  int* d_error = nullptr;
  double* d_partials = nullptr;
  double* d_scalars = nullptr;
  int nitems = 0;
  int vx = 4;
  int ir = 1;
  int bt = 256;
  int mode = LBM_BATCH_PERSISTENT;
  int chunk = 100;
  int grid = 0;
  int cur = 0;
  int64_t t = 0;
  int64_t sites = 0;
  unsigned spin_limit = 1u << 22;
  int flavor = 2;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // exact-difference runs (every run LBM_FORCE_EDM on one grid size)
  bool edm = false;
  EdmModes edm_md{};
  EdmWs edm_ws{};
  EdmRuns edm_runs{};
  lbm_tile edm_tile{};
};

namespace {

struct BatchLayout {
  std::vector<void*> pop0, pop1, fx, fy;
  RunDesc* runs;
  int* item_run;
  int* item_start;
  int* fitem_run;
  int* fitem_tile;
  size_t fitem_cap;
  unsigned* barrier;
  int* error;
  double* partials;
  double* scalars;
  EdmWs edm;
  size_t item_cap;
  size_t bytes;
};

bool edm_batch(const lbm_config* cfgs) { return cfgs[0].force_scheme == LBM_FORCE_EDM; }

size_t max_items(const lbm_config* cfgs, int nruns) {
  // smallest item: kBT sites (vx = 1, ir = 1)
  size_t n = 0;
  for (int r = 0; r < nruns; ++r) {
    const size_t plane = static_cast<size_t>(cfgs[r].nx) * cfgs[r].ny;
    n += (plane + kBT - 1) / kBT;
  }
  return n;
}

// multi-step tiles: strips of >= 54 columns (64 lanes less 2 (K - 1) packed halo
// columns at K = 6), bands of >= 8 rows
constexpr int kMinFusedBand = 8;
constexpr int kMinFusedStrip = 64 - 2 * 5;
size_t max_fused_items(const lbm_config* cfgs, int nruns) {
  size_t n = 0;
  for (int r = 0; r < nruns; ++r)
    n += static_cast<size_t>((cfgs[r].nx + kMinFusedStrip - 1) / kMinFusedStrip) *
         ((cfgs[r].ny + kMinFusedBand - 1) / kMinFusedBand);
  return n;
}

BatchLayout carve_batch(const lbm_config* cfgs, int nruns, void* base, size_t cap) {
  Carver cv(base, cap);
  BatchLayout l{};
  const size_t es = cfgs[0].dtype == LBM_F32 ? 4 : 8;
  int maxblocks = 0;
  for (int r = 0; r < nruns; ++r) {
    const size_t plane = static_cast<size_t>(cfgs[r].nx) * cfgs[r].ny;
    l.pop0.push_back(cv.take<char>(9 * plane * es));
    l.pop1.push_back(cv.take<char>(9 * plane * es));
    if (cfgs[r].has_force) {
      l.fx.push_back(cv.take<char>(plane * es));
      l.fy.push_back(cv.take<char>(plane * es));
    } else {
      l.fx.push_back(nullptr);
      l.fy.push_back(nullptr);
    }
    maxblocks = std::max(maxblocks, moment_blocks(cfgs[r].nx, cfgs[r].ny));
  }
  l.runs = cv.take<RunDesc>(nruns);
  l.item_cap = max_items(cfgs, nruns);
  l.item_run = cv.take<int>(l.item_cap);
  l.item_start = cv.take<int>(l.item_cap);
  l.fitem_cap = max_fused_items(cfgs, nruns);
  l.fitem_run = cv.take<int>(l.fitem_cap);
  l.fitem_tile = cv.take<int>(l.fitem_cap);
  l.barrier = cv.take<unsigned>(kBarrierWords);
  l.error = cv.take<int>(64);
  l.partials = cv.take<double>(static_cast<size_t>(maxblocks) * 8 + 8);
  l.scalars = cv.take<double>(8);
  if (edm_batch(cfgs)) {
    EdmModes md{};
    if (edm_modes(cfgs[0], &md) == LBM_OK) l.edm = carve_edm_runs(cv, cfgs[0], md, nruns);
  }
  l.bytes = cv.used + 256;
  return l;
}

// Exact-difference runs: damped modes, per-run 1/tau and damping rate, the
// equal strides between the runs' buffers, the shared tables.
int setup_edm(lbm_batch_s* b, const BatchLayout& l) {
  b->edm = true;
  b->mode = LBM_BATCH_PER_STEP;
  b->edm_ws = l.edm;
  b->edm_tile = edm_default_tile(b->cfg[0].nx);
  EdmRuns& R = b->edm_runs;
  R.n = b->nruns;
  const size_t es = b->dtype == LBM_F32 ? 4 : 8;
  for (int r = 0; r < b->nruns; ++r) {
    EdmModes md{};
    if (int rc = edm_modes(b->cfg[r], &md)) return rc;
    if (r == 0) b->edm_md = md;
    R.omega[r] = b->runs[r].omega;
    R.f0[r] = md.f0;
    if (r > 0) {
      const auto gap = [&](const void* a, const void* z) {
        return static_cast<size_t>(static_cast<const char*>(z) - static_cast<const char*>(a)) / es;
      };
      const size_t st = gap(b->runs[0].pop[0], b->runs[1].pop[0]);
      bool ok = gap(b->runs[r - 1].pop[0], b->runs[r].pop[0]) == st &&
                gap(b->runs[r - 1].pop[1], b->runs[r].pop[1]) == st;
      if (b->cfg[0].has_force)
        ok = ok && gap(b->runs[r - 1].fx, b->runs[r].fx) == st && gap(b->runs[r - 1].fy, b->runs[r].fy) == st;
      if (!ok) return fail(LBM_E_UNSUPPORTED, "exact-difference runs are not equally spaced in the workspace");
      R.pop_stride = R.force_stride = st;
    }
  }
  return edm_tables(b->cfg[0], b->edm_ws, b->edm_md, b->stream);
}

int validate_batch(const lbm_config* cfgs, int32_t nruns) {
  if (!cfgs || nruns < 1 || nruns > 4096) return fail(LBM_E_INVALID, "need 1..4096 runs");
  for (int r = 0; r < nruns; ++r) {
    lbm_config c = cfgs[r];
    if (int rc = validate_config(&c)) return rc;
    if (c.dtype != cfgs[0].dtype) return fail(LBM_E_INVALID, "run %d: all runs need one dtype", r);
    if (c.with_balance) return fail(LBM_E_INVALID, "run %d: with_balance must be 0 in a batch", r);
    if (c.collision != LBM_COLLISION_BGK)
      return fail(LBM_E_UNSUPPORTED, "run %d: a batch runs the BGK collision only", r);
    if (c.force_scheme != cfgs[0].force_scheme)
      return fail(LBM_E_UNSUPPORTED, "run %d: all runs of a batch need one force scheme", r);
    if (c.force_scheme == LBM_FORCE_EDM) {
      // exact-difference runs share the grid, the layout, the force flag and the damped modes
      const lbm_config& a = cfgs[0];
      if (c.nx != a.nx || c.ny != a.ny || c.layout != a.layout || c.has_force != a.has_force ||
          (c.damp_f0 > 0.0) != (a.damp_f0 > 0.0) || c.damp_kmin != a.damp_kmin || c.damp_kmax != a.damp_kmax)
        return fail(LBM_E_UNSUPPORTED, "run %d: exact-difference runs of a batch need one grid, layout, "
                                       "force flag and damped shell", r);
      if (nruns > kEdmMaxRuns) return fail(LBM_E_UNSUPPORTED, "at most %d exact-difference runs", kEdmMaxRuns);
    }
    if (static_cast<size_t>(c.nx) * c.ny > 0x7fffffffu)
      return fail(LBM_E_INVALID, "run %d: grid too large for a batch", r);
  }
  return LBM_OK;
}

// work list and shape of the multi-step tiles, from buffer parity `par`
FusedArgs fused_args(const lbm_batch_s* b, int par) {
  FusedArgs f{};
  f.runs = b->d_runs;
  f.item_run = b->d_fitem_run;
  f.item_tile = b->d_fitem_tile;
  f.nitems = b->nfitems;
  f.per_xcd = (b->nfitems + 7) / 8;
  f.W = fused_strip_width(b->ftile);
  f.H = b->ftile.ry;
  f.halo = b->ftile.halo;
  f.threads = f.halo ? b->ftile.bx : f.W + 64;
  f.parity = par;
  return f;
}

int build_items(lbm_batch_s* b) {
  std::vector<int> ir_run, ir_start;
  const size_t per = static_cast<size_t>(b->bt) * b->vx * b->ir;
  for (int r = 0; r < b->nruns; ++r) {
    const size_t plane = static_cast<size_t>(b->cfg[r].nx) * b->cfg[r].ny;
    for (size_t s0 = 0; s0 < plane; s0 += per) {
      ir_run.push_back(r);
      ir_start.push_back(static_cast<int>(s0));
    }
  }
  if (ir_run.size() > b->item_cap) return fail(LBM_E_INVALID, "work list exceeds its capacity");
  b->nitems = static_cast<int>(ir_run.size());
  // multi-step tiles of every run
  std::vector<int> f_run, f_tile;
  for (int r = 0; r < b->nruns; ++r) {
    const int W = fused_strip_width(b->ftile);
    const int strips = (b->cfg[r].nx + W - 1) / W;
    const int bands = (b->cfg[r].ny + b->ftile.ry - 1) / b->ftile.ry;
    for (int t = 0; t < strips * bands; ++t) {
      f_run.push_back(r);
      f_tile.push_back(t);
    }
  }
  if (f_run.size() > b->fitem_cap) return fail(LBM_E_INVALID, "multi-step work list exceeds its capacity");
  b->nfitems = static_cast<int>(f_run.size());
  LBM_HIP(hipMemcpyAsync(b->d_item_run, ir_run.data(), ir_run.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  LBM_HIP(hipMemcpyAsync(b->d_item_start, ir_start.data(), ir_start.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  LBM_HIP(hipMemcpyAsync(b->d_fitem_run, f_run.data(), f_run.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  LBM_HIP(hipMemcpyAsync(b->d_fitem_tile, f_tile.data(), f_tile.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  LBM_HIP(hipStreamSynchronize(b->stream));
  int occ = 0;
  if (int rc = b->dtype == LBM_F32 ? occupancy_for<float>(b->vx, b->bt, &occ)
                                   : occupancy_for<double>(b->vx, b->bt, &occ))
    return rc;
  // every workgroup resident, eight equal groups
  b->grid = std::min(occ / 8 * 8, 8 * ((b->nitems + 7) / 8));
  // persistent multi-step: every workgroup resident, eight equal groups
  {
    const FusedArgs f = fused_args(b, 0);
    const void* fn = b->dtype == LBM_F32 ? fused_persistent_fn<float>(b->ftile.fuse, b->ftile.nt != 0)
                                         : fused_persistent_fn<double>(b->ftile.fuse, b->ftile.nt != 0);
    const size_t lds = fused_lds_bytes(f.W, b->ftile.fuse, b->dtype);
    int per_cu = 0, dev = 0, cus = 0;
    LBM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, f.threads, lds));
    LBM_HIP(hipGetDevice(&dev));
    LBM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int resident = (per_cu * cus) / 8 * 8;
    b->fgrid = std::min(resident, 8 * f.per_xcd);
  }
  return LBM_OK;
}

void drop_batch_graphs(lbm_batch_s* b) {
  for (auto& g : b->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

BarrierArgs barrier_args(const lbm_batch_s* b) {
  BarrierArgs g{};
  g.barrier = b->d_barrier;
  g.error = b->d_error;
  g.spin_limit = b->spin_limit;
  g.flavor = b->flavor;
  return g;
}

BatchArgs make_args(lbm_batch_s* b, int parity0, int nsteps) {
  BatchArgs a{};
  a.runs = b->d_runs;
  a.item_run = b->d_item_run;
  a.item_start = b->d_item_start;
  a.nitems = b->nitems;
  a.ir = b->ir;
  a.bt = b->bt;
  a.parity0 = parity0;
  a.nsteps = nsteps;
  a.bar = barrier_args(b);
  return a;
}

// Buffer swaps that n steps take in the current mode.
int step_launches(const lbm_batch_s* b, int n) {
  if (b->mode != LBM_BATCH_MULTI_STEP && b->mode != LBM_BATCH_PERSISTENT_MULTI) return n;
  return n / b->ftile.fuse + n % b->ftile.fuse;
}

// n % K remaining steps, one per-step launch each, from parity p; returns the
// parity after them
int enqueue_single_steps(lbm_batch_s* b, int p, int n, hipStream_t s, int* p_out) {
  for (int k = 0; k < n; ++k) {
    BatchArgs a = make_args(b, p, 1);
    if (b->dtype == LBM_F32) launch_batch_vx<float>(b->vx, false, a, 0, s);
    else launch_batch_vx<double>(b->vx, false, a, 0, s);
    LBM_HIP(hipGetLastError());
    p ^= 1;
  }
  *p_out = p;
  return LBM_OK;
}

// Enqueue `n` steps starting from buffer parity `par` on stream s.
int enqueue_steps(lbm_batch_s* b, int par, int n, hipStream_t s) {
  if (n <= 0) return LBM_OK;
  if (b->edm) {
    // one launch sequence per step for all runs: Fourier sums, coefficients, step
    const RunDesc& r0 = b->runs[0];
    StepParams p{};
    p.fx = r0.fx;
    p.fy = r0.fy;
    p.nx = r0.nx;
    p.ny = r0.ny;
    p.ps = r0.ps;
    p.rs = r0.rs;
    p.omega = r0.omega;
    for (int k = 0; k < n; ++k) {
      p.src = r0.pop[(par + k) & 1];
      p.dst = r0.pop[(par + k + 1) & 1];
      if (int rc = edm_step_runs(b->cfg[0], b->edm_ws, b->edm_md, b->edm_runs, p, b->edm_tile, s)) return rc;
    }
    return LBM_OK;
  }
  if (b->mode == LBM_BATCH_MULTI_STEP) {
    const int K = b->ftile.fuse;
    FusedArgs f = fused_args(b, par);
    int p = par;
    for (int k = 0; k + K <= n; k += K) {
      f.parity = p;
      if (b->dtype == LBM_F32) launch_batch_fused<float>(K, f, b->ftile.nt != 0, s);
      else launch_batch_fused<double>(K, f, b->ftile.nt != 0, s);
      LBM_HIP(hipGetLastError());
      p ^= 1;
    }
    return enqueue_single_steps(b, p, n % K, s, &p);
  }
  if (b->mode == LBM_BATCH_PERSISTENT_MULTI) {
    const int K = b->ftile.fuse;
    const int rounds = n / K;
    int p = par;
    if (rounds > 0) {
      if (b->fgrid < 8) return fail(LBM_E_UNSUPPORTED, "the multi-step tiles do not fit a persistent grid");
      hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, b->d_barrier);
      LBM_HIP(hipGetLastError());
      const FusedArgs f = fused_args(b, par);
      const size_t lds = fused_lds_bytes(f.W, K, b->dtype);
      const void* fn = b->dtype == LBM_F32 ? fused_persistent_fn<float>(K, b->ftile.nt != 0)
                                           : fused_persistent_fn<double>(K, b->ftile.nt != 0);
      FusedArgs fa = f;
      int rr = rounds;
      BarrierArgs bar = barrier_args(b);
      void* args[] = {&fa, &rr, &bar};
      LBM_HIP(hipLaunchKernel(fn, dim3(b->fgrid), dim3(f.threads), args, lds, s));
      p ^= rounds & 1;
    }
    return enqueue_single_steps(b, p, n % K, s, &p);
  }
  if (b->mode == LBM_BATCH_PERSISTENT) {
    if (b->grid < 8) return fail(LBM_E_UNSUPPORTED, "the work items do not fit a persistent grid");
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, b->d_barrier);
    LBM_HIP(hipGetLastError());
    BatchArgs a = make_args(b, par, n);
    if (b->dtype == LBM_F32) launch_batch_vx<float>(b->vx, true, a, b->grid, s);
    else launch_batch_vx<double>(b->vx, true, a, b->grid, s);
    LBM_HIP(hipGetLastError());
  } else {
    for (int k = 0; k < n; ++k) {
      BatchArgs a = make_args(b, (par + k) & 1, 1);
      if (b->dtype == LBM_F32) launch_batch_vx<float>(b->vx, false, a, 0, s);
      else launch_batch_vx<double>(b->vx, false, a, 0, s);
      LBM_HIP(hipGetLastError());
    }
  }
  return LBM_OK;
}

int build_batch_graph(lbm_batch_s* b, int par) {
  if (!b->cap_stream) LBM_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  LBM_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_steps(b, par, b->chunk, b->cap_stream);
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->gexec[par], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return LBM_OK;
}

int check_error_flag(lbm_batch_s* b) {
  int h = 0;
  LBM_HIP(hipMemcpyAsync(&h, b->d_error, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  LBM_HIP(hipStreamSynchronize(b->stream));
  if (h) return fail(LBM_E_TIMEOUT, "a grid-barrier wait of the persistent batch kernel ran out "
                                    "(workgroups not all resident?); the batch state is invalid");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(const lbm_config* cfgs, int32_t nruns, size_t* bytes) {
  if (int rc = validate_batch(cfgs, nruns)) return rc;
  if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
  *bytes = carve_batch(cfgs, nruns, nullptr, 0).bytes;
  return LBM_OK;
}

int lbm_batch_init(const lbm_config* cfgs, int32_t nruns, void* ws, size_t ws_bytes,
                   const double* const* rho0, const double* const* ux0, const double* const* uy0,
                   const double* const* fx, const double* const* fy, lbm_batch* out) {
  if (int rc = validate_batch(cfgs, nruns)) return rc;
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(LBM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (!rho0 || !ux0 || !uy0) return fail(LBM_E_INVALID, "initial field arrays must not be NULL");
  BatchLayout l = carve_batch(cfgs, nruns, nullptr, 0);
  if (ws_bytes < l.bytes) return fail(LBM_E_NOMEM, "workspace %zu < %zu", ws_bytes, l.bytes);
  for (int r = 0; r < nruns; ++r) {
    if (!rho0[r] || !ux0[r] || !uy0[r]) return fail(LBM_E_INVALID, "run %d: NULL initial field", r);
    const bool has = fx && fy && fx[r] && fy[r];
    if (cfgs[r].has_force && !has) return fail(LBM_E_INVALID, "run %d: has_force needs fx, fy", r);
    if (!cfgs[r].has_force && fx && fx[r]) return fail(LBM_E_INVALID, "run %d: force without has_force", r);
  }
  l = carve_batch(cfgs, nruns, ws, ws_bytes);
  lbm_batch_s* b = new lbm_batch_s();
  b->nruns = nruns;
  b->dtype = cfgs[0].dtype;
  b->stream = static_cast<hipStream_t>(cfgs[0].stream);
  b->cfg.assign(cfgs, cfgs + nruns);
  b->d_runs = l.runs;
  b->d_item_run = l.item_run;
  b->d_item_start = l.item_start;
  b->item_cap = l.item_cap;
  b->d_fitem_run = l.fitem_run;
  b->d_fitem_tile = l.fitem_tile;
  b->fitem_cap = l.fitem_cap;
  b->d_barrier = l.barrier;
  b->d_error = l.error;
  b->d_partials = l.partials;
  b->d_scalars = l.scalars;
  int common = 4;
  for (int r = 0; r < nruns; ++r) {
    while (common > 1 && cfgs[r].nx % common) common >>= 1;
    b->sites += static_cast<int64_t>(cfgs[r].nx) * cfgs[r].ny;
  }
  b->vx = b->dtype == LBM_F32 ? common : std::min(common, 2);
  if (const char* fl = std::getenv("LBM_BATCH_BARRIER")) {
    const int v = std::atoi(fl);
    if (v >= 0 && v <= 2) b->flavor = v;
  }
  int rc = LBM_OK;
  for (int r = 0; r < nruns && rc == LBM_OK; ++r) {
    RunDesc d{};
    d.pop[0] = l.pop0[r];
    d.pop[1] = l.pop1[r];
    d.fx = l.fx[r];
    d.fy = l.fy[r];
    d.nx = cfgs[r].nx;
    d.ny = cfgs[r].ny;
    const PopLayout lay = pop_layout(cfgs[r].layout, d.nx, d.ny);
    d.ps = lay.ps;
    d.rs = lay.rs;
    d.omega = 1.0 / cfgs[r].tau;
    d.alpha = cfgs[r].drag_alpha;
    d.forced = (cfgs[r].has_force || cfgs[r].drag_alpha > 0.0) ? 1 : 0;
    b->runs.push_back(d);
    rc = launch_init(b->dtype, d.pop[0], lay, rho0[r], ux0[r], uy0[r], d.nx, d.ny, b->stream);
    const size_t plane = static_cast<size_t>(d.nx) * d.ny;
    if (rc == LBM_OK && cfgs[r].has_force) {
      rc = launch_to_storage(b->dtype, l.fx[r], fx[r], plane, b->stream);
      if (rc == LBM_OK) rc = launch_to_storage(b->dtype, l.fy[r], fy[r], plane, b->stream);
    }
  }
  if (rc == LBM_OK && edm_batch(cfgs)) rc = setup_edm(b, l);
  if (rc == LBM_OK) {
    hipError_t e = hipMemcpyAsync(b->d_runs, b->runs.data(), sizeof(RunDesc) * nruns,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_error, 0, 64 * sizeof(int), b->stream);
    if (e != hipSuccess) rc = hip_fail(e, "batch setup copy");
  }
  if (rc == LBM_OK) rc = build_items(b);
  if (rc != LBM_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_set_mode(lbm_batch b, int32_t mode, int32_t chunk) {
  if (!b) return fail(LBM_E_INVALID, "batch is NULL");
  if (mode != LBM_BATCH_PERSISTENT && mode != LBM_BATCH_PER_STEP && mode != LBM_BATCH_MULTI_STEP &&
      mode != LBM_BATCH_PERSISTENT_MULTI)
    return fail(LBM_E_INVALID, "mode must be LBM_BATCH_PERSISTENT, _PER_STEP, _MULTI_STEP or _PERSISTENT_MULTI");
  if (chunk < 2 || chunk % 2 || chunk > 100000) return fail(LBM_E_INVALID, "chunk: even, 2..100000");
  if (b->edm && mode != LBM_BATCH_PER_STEP)
    return fail(LBM_E_UNSUPPORTED, "exact-difference runs step in LBM_BATCH_PER_STEP mode only");
  b->mode = mode;
  b->chunk = chunk;
  drop_batch_graphs(b);
  return LBM_OK;
}

int lbm_batch_set_tile(lbm_batch b, int32_t block_threads, int32_t vx, int32_t band_rows) {
  if (!b) return fail(LBM_E_INVALID, "batch is NULL");
  if (b->edm) return fail(LBM_E_UNSUPPORTED, "exact-difference runs use their step kernel's own shape");
  if (block_threads != 256 && block_threads != 512 && block_threads != 1024)
    return fail(LBM_E_INVALID, "block_threads must be 256, 512 or 1024");
  if (vx != 1 && vx != 2 && vx != 4) return fail(LBM_E_INVALID, "vx must be 1, 2 or 4");
  for (int r = 0; r < b->nruns; ++r)
    if (b->cfg[r].nx % vx) return fail(LBM_E_INVALID, "vx %d does not divide nx of run %d", vx, r);
  if (band_rows < 1 || band_rows > 64) return fail(LBM_E_INVALID, "site groups per item in 1..64");
  b->bt = block_threads;
  b->vx = vx;
  b->ir = band_rows;
  drop_batch_graphs(b);
  return build_items(b);
}

int lbm_batch_set_multi(lbm_batch b, const lbm_tile* t) {
  if (!b || !t) return fail(LBM_E_INVALID, "NULL argument");
  if (b->edm) return fail(LBM_E_UNSUPPORTED, "exact-difference runs have no multi-step mode");
  if (!fused_tile_ok(*t, b->dtype) || t->ry < kMinFusedBand)
    return fail(LBM_E_INVALID, "multi-step shape: fuse 2..6, halo 0 or 1, width a multiple of 64 up "
                               "to 512, band >= %d rows", kMinFusedBand);
  b->ftile = *t;
  b->ftile.pf = 1;
  drop_batch_graphs(b);
  return build_items(b);
}

int lbm_batch_get_multi(lbm_batch b, lbm_tile* t) {
  if (!b || !t) return fail(LBM_E_INVALID, "NULL argument");
  *t = b->ftile;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch b, int64_t n) {
  if (!b) return fail(LBM_E_INVALID, "batch is NULL");
  if (n < 0) return fail(LBM_E_INVALID, "n must be >= 0");
  while (n >= b->chunk) {
    if (!b->gexec[b->cur])
      if (int rc = build_batch_graph(b, b->cur)) return rc;
    LBM_HIP(hipGraphLaunch(b->gexec[b->cur], b->stream));
    n -= b->chunk;
    b->t += b->chunk;
    b->cur = (b->cur + step_launches(b, b->chunk)) & 1;
  }
  if (n > 0) {
    if (int rc = enqueue_steps(b, b->cur, static_cast<int>(n), b->stream)) return rc;
    b->cur = (b->cur + step_launches(b, static_cast<int>(n))) & 1;
    b->t += n;
  }
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch b, int32_t trial_steps, int32_t* block_threads, int32_t* vx,
                       int32_t* band_rows) {
  if (!b) return fail(LBM_E_INVALID, "batch is NULL");
  if (trial_steps < 2 || trial_steps > 1000 || trial_steps % 2)
    return fail(LBM_E_INVALID, "trial_steps: even, 2..1000");
  if (b->edm) return fail(LBM_E_UNSUPPORTED, "exact-difference runs have one launch shape (no autotuning)");
  const int saved_vx = b->vx, saved_ir = b->ir, saved_bt = b->bt, saved_mode = b->mode;
  const lbm_tile saved_f = b->ftile;
  hipEvent_t e0, e1;
  LBM_HIP(hipEventCreate(&e0));
  LBM_HIP(hipEventCreate(&e1));
  float best = 1e30f, best_multi = 1e30f;  // milliseconds per step
  int bvx = saved_vx, bir = saved_ir, bbt = saved_bt, bmode = saved_mode;
  lbm_tile bf = saved_f;  // fastest multi-step shape, kept whichever mode wins
  int rc = LBM_OK;
  // one timed trial of the current settings: a warm-up of two steps, then
  // `steps` steps; the ensemble really advances, the time counter records it
  auto trial = [&](int steps) -> int {
    if (int r = build_items(b)) return r;
    if (int r = enqueue_steps(b, b->cur, 2, b->stream)) return r;
    b->cur = (b->cur + step_launches(b, 2)) & 1;
    if (hipEventRecord(e0, b->stream) != hipSuccess) return fail(LBM_E_HIP, "event");
    if (int r = enqueue_steps(b, b->cur, steps, b->stream)) return r;
    b->cur = (b->cur + step_launches(b, steps)) & 1;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail(LBM_E_HIP, "event");
    b->t += 2 + steps;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= static_cast<float>(steps);
    if (ms < best) {
      best = ms;
      bvx = b->vx;
      bir = b->ir;
      bbt = b->bt;
      bmode = b->mode;
    }
    if (b->mode == LBM_BATCH_MULTI_STEP && ms < best_multi) {
      best_multi = ms;
      bf = b->ftile;
    }
    return LBM_OK;
  };
  const int modes[2] = {LBM_BATCH_PERSISTENT, LBM_BATCH_PER_STEP};
  const int bts[2] = {256, 1024};
  const int vxs[3] = {1, 2, 4};
  const int irs[3] = {1, 2, 4};
  for (int mode : modes) {
    for (int bt : bts) {
      for (int v : vxs) {
        bool fits = true;
        for (int r = 0; r < b->nruns; ++r) fits = fits && (b->cfg[r].nx % v == 0);
        if (!fits || (b->dtype == LBM_F64 && v == 4)) continue;
        for (int i : irs) {
          b->mode = mode;
          b->bt = bt;
          b->vx = v;
          b->ir = i;
          if ((rc = trial(trial_steps)) != LBM_OK) break;
        }
        if (rc) break;
      }
      if (rc) break;
    }
    if (rc) break;
  }
  // multi-step shapes (remainder steps use the fastest single-step work list)
  if (rc == LBM_OK) {
    const int kbvx = bvx, kbir = bir, kbbt = bbt;
    b->vx = kbvx;
    b->ir = kbir;
    b->bt = kbbt;
    b->mode = LBM_BATCH_MULTI_STEP;
    const int ws[3] = {128, 256, 512};
    const int hs[3] = {32, 64, 128};
    // the packed halo (halo = 1) from K = 4 on, as for one grid
    for (int K = 2; K <= 6 && rc == LBM_OK; ++K)
      for (int halo = 0; halo <= (K >= 4 ? 1 : 0) && rc == LBM_OK; ++halo)
      for (int w = 0; w < 3 && rc == LBM_OK; ++w)
        for (int h : hs) {
          lbm_tile t{ws[w], 1, 1, h, 1, K, 1, halo};
          if (!fused_tile_ok(t, b->dtype)) continue;
          b->ftile = t;
          // a whole number of K-step launches
          if ((rc = trial(K * ((trial_steps + K - 1) / K))) != LBM_OK) break;
          // the single-step work list is the one found above whatever wins here
          bvx = kbvx;
          bir = kbir;
          bbt = kbbt;
        }
    // the fastest multi-step shape inside one persistent launch
    if (rc == LBM_OK) {
      b->mode = LBM_BATCH_PERSISTENT_MULTI;
      b->ftile = bf;
      const int K = bf.fuse;
      rc = trial(K * ((trial_steps + K - 1) / K));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == LBM_OK) rc = check_error_flag(b);
  const bool ok = rc == LBM_OK;
  b->vx = ok ? bvx : saved_vx;
  b->ir = ok ? bir : saved_ir;
  b->bt = ok ? bbt : saved_bt;
  b->mode = ok ? bmode : saved_mode;
  b->ftile = ok ? bf : saved_f;
  drop_batch_graphs(b);
  if (int r2 = build_items(b)) return rc ? rc : r2;
  if (rc) return rc;
  if (block_threads) *block_threads = b->bt;
  if (vx) *vx = b->vx;
  if (band_rows) *band_rows = b->ir;
  return LBM_OK;
}

int lbm_batch_get_mode(lbm_batch b, int32_t* mode, int32_t* chunk) {
  if (!b) return fail(LBM_E_INVALID, "batch is NULL");
  if (mode) *mode = b->mode;
  if (chunk) *chunk = b->chunk;
  return LBM_OK;
}

int lbm_batch_moments(lbm_batch b, int32_t run, void* rho, void* ux, void* uy, int32_t out_dtype,
                      double* scalars8) {
  if (!b) return fail(LBM_E_INVALID, "batch is NULL");
  if (run < 0 || run >= b->nruns) return fail(LBM_E_INVALID, "run %d out of range", run);
  if (out_dtype != LBM_F32 && out_dtype != LBM_F64) return fail(LBM_E_INVALID, "bad out_dtype");
  if (int rc = check_error_flag(b)) return rc;
  const RunDesc& r = b->runs[run];
  MomentParams m{};
  m.pop = r.pop[b->cur];
  m.fx = r.fx;
  m.fy = r.fy;
  m.rho = rho;
  m.ux = ux;
  m.uy = uy;
  m.out_dtype = out_dtype;
  m.partials = b->d_partials;
  m.nx = r.nx;
  m.ny = r.ny;
  m.ps = r.ps;
  m.rs = r.rs;
  m.alpha = r.alpha;
  if (b->edm) {
    EdmModes md = b->edm_md;
    md.f0 = b->edm_runs.f0[run];
    const EdmWs w = edm_run_view(b->edm_ws, b->cfg[0], b->edm_md, run);
    if (int rc = edm_moments(b->cfg[run], w, md, m, b->stream)) return rc;
  } else if (int rc = launch_moments(b->dtype, r.forced != 0, m, b->stream)) {
    return rc;
  }
  if (!scalars8) return LBM_OK;
  if (int rc = launch_reduce_scalars(b->d_partials, moment_blocks(r.nx, r.ny), b->d_scalars, b->stream))
    return rc;
  LBM_HIP(hipMemcpyAsync(scalars8, b->d_scalars, 8 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  LBM_HIP(hipStreamSynchronize(b->stream));
  scalars8[LBM_S_TIME] = static_cast<double>(b->t);
  if (scalars8[LBM_S_NONFINITE] > 0.0 || !(scalars8[LBM_S_MINRHO] > 0.0))
    return fail(LBM_E_DIVERGED, "run %d diverged by step %lld", run, static_cast<long long>(b->t));
  return LBM_OK;
}

int lbm_batch_time(lbm_batch b, int64_t* t) {
  if (!b || !t) return fail(LBM_E_INVALID, "NULL argument");
  *t = b->t;
  return LBM_OK;
}

int64_t lbm_batch_sites(lbm_batch b) { return b ? b->sites : 0; }

int lbm_batch_destroy(lbm_batch b) {
  if (!b) return LBM_OK;
  (void)hipStreamSynchronize(b->stream);
  drop_batch_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return LBM_OK;
}

}  // extern "C"
