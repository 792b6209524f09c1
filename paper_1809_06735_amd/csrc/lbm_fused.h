// Device code of the multi-step (temporally blocked) D2Q9 update of one tile,
// shared by the single-grid kernel and the batched-ensemble kernel.
//
// A workgroup owns a strip of W columns and a band of H rows of the output
// and marches down its band one row per iteration.  Level s = 1..K of the
// iteration advances one row by one step: level 1 pulls its populations from
// the source state in HBM (x - c_l, periodic) and collides them with Eq. 1 /
// Eq. 2 and Guo forcing, exactly as the single-step kernel does; level s > 1
// collides the output of level s - 1.  A level's six populations with
// c_x != 0 go to the neighbouring columns through an LDS row (two rows used
// alternately, one barrier per level); the three with c_x = 0, and the rows
// of the previous iterations that the pull also needs (c_y = +1 from two rows
// back, c_y = 0 from one row back), stay in registers.  Level s runs one row
// behind level s - 1 and on one column fewer on each side, so level 1 covers
// the strip plus K - 1 halo columns per side and only level K writes to HBM.
// The intermediate states never leave the CU: K lattice updates cost one read
// and one write of every population plus one read of the force field, 80 B
// per site per launch in FP32.  Results are bit-identical to K single-step
// launches (same per-site arithmetic, same operand order).
//
// Every lane runs every level in every iteration, also where the level has no
// valid input yet (the first iterations of a band, the halo lanes beyond their
// level): those values are never read by a valid site nor stored, and without
// per-level branches the compiler keeps the carries in place instead of
// copying them at every branch merge (about 6 % fewer VALU instructions per
// iteration at K = 6).  Only the HBM store is guarded.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_internal.h"
#include "lbm_site.h"

namespace lbm {
namespace fused_detail {

using namespace step_detail;

// strips of at most 512 columns (one extra wave for the halo): the register
// budget of a 576-thread workgroup leaves room for the carries of 6 levels
constexpr int kFusedMaxThreads = 576;

template <typename T, bool NT>
__device__ __forceinline__ void put(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Registers that carry one level's input between rows: the pre-collision
// values that the pull takes from the same row (l = 0, 1, 3) and from the row
// above (c_y = +1: l = 2, 5, 6), two rows of the latter.  Which of the two
// holds the older row alternates with the iteration's parity, so no value is
// moved between registers.
template <typename T>
struct Carry {
  T c0 = T(0), c1 = T(0), c3 = T(0);
  T c2[2] = {T(0), T(0)}, c5[2] = {T(0), T(0)}, c6[2] = {T(0), T(0)};
};

// One tile (strip `tile % strips`, band `tile / strips`) of a K-step update of
// the grid p (src -> dst), strips of W columns.  Separate halo (packed =
// false): threads [0, W) own the strip columns, threads W + j, j < 2 (K - 1),
// the halo columns at distance j / 2 + 1 left (j even) or right (j odd) of the
// strip, blockDim.x = W + 64.  Packed halo: thread t owns column
// x0 - (K - 1) + t, so the strip and both halos are one contiguous run of
// W + 2 (K - 1) = blockDim.x lanes.  Either way lds holds 2 * 6 * (W + 2 (K - 1))
// values, indexed by the column's position in that run.  PF issues the next
// row's loads after the first exchange barrier instead of at the end of the
// iteration.  Every thread of the workgroup must call it (it contains barriers).
template <typename T, int K, bool FORCE, bool NT, bool PF>
__device__ __forceinline__ void fused_tile(const StepParams& p, T* const lds, int W, int H,
                                           int strips, int tile, bool packed) {
  const int stride = W + 2 * (K - 1);
  const int nx = p.nx, ny = p.ny;
  const int x0 = (tile % strips) * W;
  const int y0 = (tile / strips) * H;
  const int weff = min(W, nx - x0);
  const int heff = min(H, ny - y0);
  const int t = threadIdx.x;
  // column, LDS index and the highest level this thread takes part in
  int col = x0, li = 0, top = 0;
  if (packed) {
    // a level-s value exists on the columns at least s - 1 away from both ends
    const int n_act = weff + 2 * (K - 1);
    if (t < n_act) {
      top = min(min(t, n_act - 1 - t) + 1, K);
      col = x0 - (K - 1) + t;
      if (col < 0) col += nx;
      if (col >= nx) col -= nx;
      li = t;
    }
  } else if (t < weff) {
    col = x0 + t;
    li = t + K - 1;
    top = K;
  } else if (t >= W && t < W + 2 * (K - 1)) {
    const int j = t - W;
    const int dist = j / 2 + 1;
    top = K - dist;
    if ((j & 1) == 0) {
      col = x0 - dist;
      if (col < 0) col += nx;
      li = K - 1 - dist;
    } else {
      col = x0 + weff - 1 + dist;
      if (col >= nx) col -= nx;
      li = K - 2 + weff + dist;
    }
  }
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const T* __restrict__ gfx = static_cast<const T*>(p.fx);
  const T* __restrict__ gfy = static_cast<const T*>(p.fy);
  const T omega = T(p.omega);
  const T guo = T(1) - T(0.5) * T(p.omega);
  const T alpha = T(p.alpha);

  auto wrap_row = [ny](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
  // every thread loads (threads without a site read their strip's first
  // column), so the loads sit outside any divergent branch
  auto load_row = [&](int r, T (&d)[9], T& fx, T& fy) {
    const int rn = r == 0 ? ny - 1 : r - 1;
    const int rp = r == ny - 1 ? 0 : r + 1;
    T v[9][1];
    pull_all<T, 1>(src, p.ps, p.rs, nx, col, r, rn, rp, v);
#pragma unroll
    for (int l = 0; l < 9; ++l) d[l] = v[l][0];
    if constexpr (FORCE) {
      if (gfx) {
        const size_t i = static_cast<size_t>(r) * nx + col;
        fx = gfx[i];
        fy = gfy[i];
      } else {
        fx = fy = T(0);
      }
    }
  };

  Carry<T> cy[K - 1];        // inputs of levels 2..K
  T fhx[K - 1], fhy[K - 1];  // force at the rows of levels 2..K
#pragma unroll
  for (int s = 0; s < K - 1; ++s) fhx[s] = fhy[s] = T(0);
  T d[9];
  T fx = T(0), fy = T(0);
  const int last = heff + K - 2;
  load_row(wrap_row(y0 - (K - 1)), d, fx, fy);

  // iteration k: level s works on row y0 + k - (s - 1) and holds valid data
  // from k = 2 s - 1 - K on; level K writes rows y0 .. y0 + heff - 1.  E is the
  // parity of the iteration count, which fixes the LDS rows and carry roles.
  // neighbour slots of the LDS rows, clamped into the row for lanes whose
  // values nobody reads (a lane that is valid at a level has both neighbours)
  const int lm = li > 0 ? li - 1 : 0;
  const int lp = li + 1 < stride ? li + 1 : li;
  auto iteration = [&](auto parity, int k) {
    constexpr int E = decltype(parity)::value;
    // LDS row of the first exchange: exchanges alternate rows across levels and
    // iterations, K - 1 of them per iteration
    constexpr int P0 = ((K - 1) & 1) ? E : 0;
    T o[9];
    {
      SiteMoments<T, FORCE> m(d, FORCE ? fx : T(0), FORCE ? fy : T(0), alpha);
      collide_site<T, FORCE>(d, m, omega, guo, o);
    }
    const T fx1 = fx, fy1 = fy;
#pragma unroll
    for (int s = 2; s <= K; ++s) {
      // exchange level s - 1's x-moving populations
      T* const slot = lds + ((P0 + s) & 1) * 6 * stride;
      if (top >= s - 1) {
        slot[0 * stride + li] = o[1];
        slot[1 * stride + li] = o[3];
        slot[2 * stride + li] = o[5];
        slot[3 * stride + li] = o[6];
        slot[4 * stride + li] = o[7];
        slot[5 * stride + li] = o[8];
      }
      __syncthreads();
      if constexpr (PF) {
        if (s == 2 && k < last) load_row(wrap_row(y0 + k + 1), d, fx, fy);
      }
      {
        Carry<T>& c = cy[s - 2];
        const T n1 = slot[0 * stride + lm];
        const T n3 = slot[1 * stride + lp];
        const T n5 = slot[2 * stride + lm];
        const T n6 = slot[3 * stride + lp];
        const T n7 = slot[4 * stride + lp];
        const T n8 = slot[5 * stride + lm];
        const T q0 = o[0], q2 = o[2], q4 = o[4];
        {
          // level s at (col, y0 + k - (s - 1)): d_l = g_l(x - c_l) of level s - 1;
          // c2[E ^ 1] etc. hold the row two back
          const T d2[9] = {c.c0, c.c1, c.c2[E ^ 1], c.c3, q4, c.c5[E ^ 1], c.c6[E ^ 1], n7, n8};
          SiteMoments<T, FORCE> m(d2, FORCE ? fhx[s - 2] : T(0), FORCE ? fhy[s - 2] : T(0), alpha);
          collide_site<T, FORCE>(d2, m, omega, guo, o);
          if (s == K && top >= K && k >= K - 1) {
            T* const out = dst + static_cast<size_t>(y0 + k - (K - 1)) * p.rs + col;
#pragma unroll
            for (int l = 0; l < 9; ++l) put<T, NT>(out + l * p.ps, o[l]);
          }
        }
        c.c0 = q0;
        c.c1 = n1;
        c.c3 = n3;
        c.c2[E ^ 1] = q2;
        c.c5[E ^ 1] = n5;
        c.c6[E ^ 1] = n6;
      }
    }
    // force history: level s + 1 works next iteration on this iteration's level-s row
#pragma unroll
    for (int s = K - 2; s >= 1; --s) {
      fhx[s] = fhx[s - 1];
      fhy[s] = fhy[s - 1];
    }
    fhx[0] = fx1;
    fhy[0] = fy1;
    if constexpr (!PF) {
      if (k < last) load_row(wrap_row(y0 + k + 1), d, fx, fy);
    }
  };
  for (int k = 1 - K; k <= last; k += 2) {
    iteration(std::integral_constant<int, 0>(), k);
    if (k + 1 > last) break;
    iteration(std::integral_constant<int, 1>(), k + 1);
  }
}


}  // namespace fused_detail
}  // namespace lbm
