// Launch shapes of the D2Q9 step kernels: validation, the default shape and
// the candidates the autotuner times (host code only, kept apart from the
// kernels so that the kernels' sources change only with their device code).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_internal.h"

namespace lbm {

size_t fused_lds_bytes(int W, int K, int dtype) {
  return static_cast<size_t>(2) * 6 * (W + 2 * (K - 1)) * (dtype == LBM_F64 ? 8 : 4);
}

int fused_strip_width(const lbm_tile& t) { return t.halo ? t.bx - 2 * (t.fuse - 1) : t.bx; }

bool fused_tile_ok(const lbm_tile& t, int dtype) {
  if (t.fuse < 2 || t.fuse > 6 || t.by != 1 || t.vx != 1) return false;
  if (t.halo != 0 && t.halo != 1) return false;
  if (t.bx < 64 || t.bx % 64 != 0 || t.bx > 512) return false;
  if (t.ry < 1 || t.ry > 4096) return false;
  if ((t.nt != 0 && t.nt != 1) || (t.pf != 0 && t.pf != 1)) return false;
  return fused_lds_bytes(fused_strip_width(t), t.fuse, dtype) <= 64 * 1024;
}

bool tile_ok(const lbm_tile& t, int dtype, int nx, int ny) {
  (void)ny;
  if (t.fuse >= 2) return fused_tile_ok(t, dtype);
  if (t.fuse < 0 || t.pf != 0 || t.halo != 0) return false;
  const int threads = t.bx * t.by;
  if (t.bx < 1 || t.by < 1 || t.ry < 1 || threads > 1024 || threads % 64 != 0) return false;
  if (t.vx != 1 && t.vx != 2 && t.vx != 4) return false;
  if (nx % t.vx != 0) return false;
  if (t.nt != 0 && t.nt != 1) return false;
  return true;
}

lbm_tile default_tile(int dtype, int nx, int ny, int layout) {
  lbm_tile t{};
  t.fuse = 1;
  if (layout == LBM_LAYOUT_ROWS) {
    // measured best on MI355X for the row layout: one site per thread, wide
    // workgroups along x, non-temporal stores
    t.vx = 1;
    int bx = 64;
    while (bx < 512 && bx * 2 <= nx) bx *= 2;
    t.bx = bx;
    t.by = bx >= 256 ? 1 : 256 / bx;
    t.ry = 1;
    t.nt = 1;
    return t;
  }
  t.vx = (dtype == LBM_F32) ? 4 : 2;
  while (t.vx > 1 && nx % t.vx != 0) t.vx >>= 1;
  int bx = 64;
  while (bx < 256 && bx * 2 * t.vx <= nx) bx *= 2;
  t.bx = bx;
  t.by = 256 / bx;
  t.ry = ny >= 4096 ? 4 : 1;
  t.nt = 0;
  return t;
}

int tile_candidates(int dtype, int nx, int ny, bool force, lbm_tile* out, int cap) {
  int n = 0;
  auto add = [&](const lbm_tile& t) {
    if (n < cap) out[n] = t;
    ++n;
  };
  const int vxs[3] = {1, 2, 4};
  const int threads[3] = {128, 256, 512};
  const int rys[4] = {1, 2, 4, 8};
  for (int vx : vxs) {
    if (nx % vx) continue;
    for (int th : threads) {
      for (int bx = 64; bx <= th; bx *= 2) {
        if (bx * vx > nx && bx > 64) continue;
        const int by = th / bx;
        for (int ry : rys) {
          if (by * ry > ny) continue;
          for (int nt = 0; nt <= 1; ++nt) {
            lbm_tile t{bx, by, vx, ry, nt, 1, 0};
            if (tile_ok(t, dtype, nx, ny)) add(t);
          }
        }
      }
    }
  }
  // K = 2..6 steps per launch: strip width W (halo wavefront) or workgroup
  // width (packed halo), band height H; the early loads (pf = 1) pay off from
  // K = 3 on, the packed halo from K = 4 on.  Besides the fixed heights, the
  // heights whose workgroup count fills the device's resident workgroup slots
  // in one or two whole rounds: a band costs its H rows plus a fixed K - 1 rows
  // of pipeline fill, and a launch lasts as many rounds as its busiest CU
  // takes, so these avoid a partly filled last round.
  const int ws[4] = {128, 192, 256, 512};
  const int hs[8] = {8, 16, 24, 32, 48, 64, 128, 256};
  for (int k = 2; k <= 6; ++k)
  for (int halo = 0; halo <= (k >= 4 ? 1 : 0); ++halo)
  for (int w : ws) {
    if (w > nx + 64 && w > 128) continue;
    for (int nt = 0; nt <= 1; ++nt)
      for (int pf = k >= 3 ? 1 : 0; pf <= 1; ++pf) {
        lbm_tile t{w, 1, 1, 8, nt, k, pf, halo};
        if (!tile_ok(t, dtype, nx, ny)) continue;
        for (int h : hs) {
          if (h > ny && h > 32) continue;
          t.ry = h;
          add(t);
        }
        int slots = 0;
        if (fused_resident_groups(dtype, force, t, &slots) != LBM_OK || slots < 1) continue;
        const int strips = (nx + fused_strip_width(t) - 1) / fused_strip_width(t);
        int prev = 0;
        for (int rounds = 1; rounds <= 2; ++rounds) {
          const int bands = rounds * slots / strips;
          if (bands < 1) continue;
          const int h = (ny + bands - 1) / bands;
          if (h < 8 || h == prev || std::find(hs, hs + 8, h) != hs + 8) continue;
          t.ry = h;
          add(t);
          prev = h;
        }
      }
  }
  return n;
}

}  // namespace lbm
