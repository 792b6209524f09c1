// Three-dimensional extension for gfx950: D3Q19 and D3Q27 LBGK steps (Eq. 1
// with the equilibrium of Eq. 2 on either lattice and Guo's forcing term), moments, and the
// sub-volume kinetic-energy and enstrophy balances in 3D, where the enstrophy
// equation gains the vortex-stretching term omega_i omega_j d_j u_i (Sec. 2
// notes that 3D keeps it), averaged over cubes L^3 at every corner.
//
// Populations: row-interleaved [nz][ny][Q][nx], Q = 19 or 27 (the Q population
// rows of one (y, z) row of sites are contiguous), deviations from the weights, kept
// un-streamed (population l stored at x is f_l(x + c_l)): one step pulls from
// x - c_l, collides and writes at x, 19 + 19 values per update (152 B FP32),
// both streams non-temporal (each value is touched once per step).
// Balance: pass A (first derivatives at level n and the vorticity at the three
// levels) gives the pointwise terms and the stress, vorticity and F / rho;
// pass B differences products and the stress (e1, e5, z1, z3, H = div sigma / rho);
// pass C the terms through H (z4 = H . curl omega, z5 = div(H x omega)).  Each
// field is mean-centred into an FP64 summed-volume table (scans along x, y, z),
// and every cube's box mean is eight table lookups (each continued
// periodically through the table's totals).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "lbm_internal.h"
#include "lbm_reduce.h"

namespace lbm {
namespace {

using namespace reduce_detail;

constexpr int Q3 = 19;
__host__ __device__ constexpr int c3(int l, int a) {
  // rest; +-x, +-y, +-z; (+-1, +-1, 0), (+-1, 0, +-1), (0, +-1, +-1), opposite pairs adjacent
  constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                            {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  return t[l][a];
}
__host__ __device__ constexpr double w3(int l) { return l == 0 ? 1.0 / 3.0 : (l <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// D3Q27: every c in {-1, 0, 1}^3, weight the product of the D1Q3 weights (2/3 at
// rest, 1/6 moving): the D3Q19 velocities in their order, then the eight
// corners in opposite pairs.
__host__ __device__ constexpr int c27(int l, int a) {
  constexpr int t[8][3] = {{1, 1, 1},  {-1, -1, -1}, {1, 1, -1},  {-1, -1, 1},
                           {1, -1, 1}, {-1, 1, -1},  {-1, 1, 1},  {1, -1, -1}};
  return l < 19 ? c3(l, a) : t[l - 19][a];
}
__host__ __device__ constexpr double w27(int l) {
  return l == 0 ? 8.0 / 27.0 : (l <= 6 ? 2.0 / 27.0 : (l <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
}
// velocity component a and weight of population l of the lattice with Q populations
template <int Q>
__host__ __device__ constexpr int cq3(int l, int a) {
  return Q == 19 ? c3(l, a) : c27(l, a);
}
template <int Q>
__host__ __device__ constexpr double wq3(int l) {
  return Q == 19 ? w3(l) : w27(l);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Element (l, z, y, x) of the row-interleaved population array of Q populations.
template <int Q = Q3>
__device__ __forceinline__ size_t pop_at(int l, int z, int y, int x, int ny, int nx) {
  return ((static_cast<size_t>(z) * ny + y) * Q + l) * nx + x;
}

// ---- step ---------------------------------------------------------------------------------
struct Step3 {
  const void* src;
  void* dst;
  const void* fx;
  const void* fy;
  const void* fz;
  double* h[4];  // optional FP64 record of rho, ux, uy, uz (pre-collision, time t)
  int nx, ny, nz;
  double omega;
};

// 1/x: IEEE division in FP64; in FP32 the hardware reciprocal refined by one
// Newton step (within an ulp of the quotient, a third of the instructions).
template <typename T>
__device__ __forceinline__ T recip3(T x) {
  if constexpr (sizeof(T) == 4) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
  } else {
    return T(1) / x;
  }
}

// Moments and BGK collision with Guo's term of one site in deviation form,
// shared by the one-step and the multi-step kernels (same operations in the
// same order, so both give the same bits).  Opposite velocities l, lbar (stored
// next to each other) share the weight and the parts of omega d^eq + G that are
// even in c, and see the odd parts with opposite signs.  With cu = c.u,
// cF = c.F and g = 1 - omega/2:
//   even  S = w B0 + 3 w cu (1.5 omega rho cu + 3 g cF),
//         B0 = omega (drho - 1.5 rho |u|^2) - 3 g u.F,
//   odd   A = w (3 omega rho cu + 3 g cF),
// f*_l = (1 - omega) d_l + S + A, f*_lbar = (1 - omega) d_lbar + S - A.
template <typename T, bool FORCE>
__device__ __forceinline__ void collide3(const T (&d)[Q3], T Fx, T Fy, T Fz, T om, T (&o)[Q3], T& drho_out, T& ux,
                                         T& uy, T& uz) {
  const T drho = (((d[0] + (d[1] + d[2])) + ((d[3] + d[4]) + (d[5] + d[6]))) +
                  (((d[7] + d[8]) + (d[9] + d[10])) + ((d[11] + d[12]) + (d[13] + d[14])))) +
                 ((d[15] + d[16]) + (d[17] + d[18]));
  const T jx = ((d[1] - d[2]) + (d[7] - d[8])) + (((d[9] - d[10]) + (d[11] - d[12])) + (d[13] - d[14]));
  const T jy = ((d[3] - d[4]) + (d[7] - d[8])) + (((d[10] - d[9]) + (d[15] - d[16])) + (d[17] - d[18]));
  const T jz = ((d[5] - d[6]) + (d[11] - d[12])) + (((d[14] - d[13]) + (d[15] - d[16])) + (d[18] - d[17]));
  drho_out = drho;
  const T rho = T(1) + drho;
  const T inv = recip3<T>(rho);
  if constexpr (FORCE) {
    ux = (jx + T(0.5) * Fx) * inv;
    uy = (jy + T(0.5) * Fy) * inv;
    uz = (jz + T(0.5) * Fz) * inv;
  } else {
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
  }
  const T om1 = T(1) - om;
  const T b = drho - rho * (T(1.5) * ((ux * ux + uy * uy) + uz * uz));
  const T wa = T(w3(1)), we = T(w3(7));
  const T p3 = (T(1.5) * om) * rho;
  const T wRa = (T(3) * om * wa) * rho, wRe = (T(3) * om * we) * rho;
  T B0 = om * b;
  T g3 = T(0);
  if constexpr (FORCE) {
    g3 = T(3) * (T(1) - T(0.5) * om);
    B0 = B0 - g3 * ((ux * Fx + uy * Fy) + uz * Fz);
  }
  const T wBa = wa * B0, wBe = we * B0;
  o[0] = om1 * d[0] + T(w3(0)) * B0;
  auto pair = [&](int l, int lb, T cu, T cF, T w, T wB, T wR) {
    T S, A;
    if constexpr (FORCE) {
      const T gc = g3 * cF;
      S = (T(3) * w) * (cu * (p3 * cu + gc)) + wB;
      A = wR * cu + w * gc;
    } else {
      S = (T(3) * w) * (cu * (p3 * cu)) + wB;
      A = wR * cu;
    }
    o[l] = om1 * d[l] + (S + A);
    o[lb] = om1 * d[lb] + (S - A);
  };
  pair(1, 2, ux, Fx, wa, wBa, wRa);
  pair(3, 4, uy, Fy, wa, wBa, wRa);
  pair(5, 6, uz, Fz, wa, wBa, wRa);
  pair(7, 8, ux + uy, Fx + Fy, we, wBe, wRe);
  pair(9, 10, ux - uy, Fx - Fy, we, wBe, wRe);
  pair(11, 12, ux + uz, Fx + Fz, we, wBe, wRe);
  pair(13, 14, ux - uz, Fx - Fz, we, wBe, wRe);
  pair(15, 16, uy + uz, Fy + Fz, we, wBe, wRe);
  pair(17, 18, uy - uz, Fy - Fz, we, wBe, wRe);
}

// The same collision on D3Q27 (the pairs of the D3Q19 collision plus the four
// corner pairs of weight 1/216; axis weight 2/27, edge weight 1/54).
template <typename T, bool FORCE>
__device__ __forceinline__ void collide27(const T (&d)[27], T Fx, T Fy, T Fz, T om, T (&o)[27], T& drho_out,
                                          T& ux, T& uy, T& uz) {
  // c.v for a velocity with components in {-1, 0, 1}: signed sums, no products (the
  // loops below are unrolled, so the branches fold away)
  auto dot = [](int cx, int cy, int cz, T a, T b, T c) {
    T r = cx > 0 ? a : -a;
    if (cx == 0) r = cy > 0 ? b : -b;
    else if (cy != 0) r += cy > 0 ? b : -b;
    if (cx == 0 && cy == 0) r = cz > 0 ? c : -c;
    else if (cz != 0) r += cz > 0 ? c : -c;
    return r;
  };
  T drho = d[0], jx = T(0), jy = T(0), jz = T(0);
#pragma unroll
  for (int l = 1; l < 27; l += 2) {
    drho += d[l] + d[l + 1];
    const T df = d[l] - d[l + 1];
    if (c27(l, 0) != 0) jx += c27(l, 0) > 0 ? df : -df;
    if (c27(l, 1) != 0) jy += c27(l, 1) > 0 ? df : -df;
    if (c27(l, 2) != 0) jz += c27(l, 2) > 0 ? df : -df;
  }
  drho_out = drho;
  const T rho = T(1) + drho;
  const T inv = recip3<T>(rho);
  if constexpr (FORCE) {
    ux = (jx + T(0.5) * Fx) * inv;
    uy = (jy + T(0.5) * Fy) * inv;
    uz = (jz + T(0.5) * Fz) * inv;
  } else {
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
  }
  const T om1 = T(1) - om;
  const T b = drho - rho * (T(1.5) * ((ux * ux + uy * uy) + uz * uz));
  const T p3 = (T(1.5) * om) * rho;
  T B0 = om * b;
  T g3 = T(0);
  if constexpr (FORCE) {
    g3 = T(3) * (T(1) - T(0.5) * om);
    B0 = B0 - g3 * ((ux * Fx + uy * Fy) + uz * Fz);
  }
  o[0] = om1 * d[0] + T(w27(0)) * B0;
#pragma unroll
  for (int l = 1; l < 27; l += 2) {
    const T w = T(w27(l));
    const T cu = dot(c27(l, 0), c27(l, 1), c27(l, 2), ux, uy, uz);
    const T wR = (T(3) * om * w) * rho;
    T S, A;
    if constexpr (FORCE) {
      const T cF = dot(c27(l, 0), c27(l, 1), c27(l, 2), Fx, Fy, Fz);
      const T gc = g3 * cF;
      S = (T(3) * w) * (cu * (p3 * cu + gc)) + w * B0;
      A = wR * cu + w * gc;
    } else {
      S = (T(3) * w) * (cu * (p3 * cu)) + w * B0;
      A = wR * cu;
    }
    o[l] = om1 * d[l] + (S + A);
    o[l + 1] = om1 * d[l + 1] + (S - A);
  }
}

template <typename T, bool FORCE, int Q = Q3>
__global__ void __launch_bounds__(256) k3_step(Step3 p) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= p.nx) return;
  const int y = blockIdx.y, z = blockIdx.z;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  T d[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const int xs = wrap(x - cq3<Q>(l, 0), nx), ys = wrap(y - cq3<Q>(l, 1), ny), zs = wrap(z - cq3<Q>(l, 2), nz);
    d[l] = __builtin_nontemporal_load(src + pop_at<Q>(l, zs, ys, xs, ny, nx));
  }
  const size_t i = (static_cast<size_t>(z) * ny + y) * nx + x;
  T Fx = T(0), Fy = T(0), Fz = T(0);
  if constexpr (FORCE) {
    Fx = static_cast<const T*>(p.fx)[i];
    Fy = static_cast<const T*>(p.fy)[i];
    Fz = static_cast<const T*>(p.fz)[i];
  }
  T o[Q], drho, ux, uy, uz;
  if constexpr (Q == 19)
    collide3<T, FORCE>(d, Fx, Fy, Fz, T(p.omega), o, drho, ux, uy, uz);
  else
    collide27<T, FORCE>(d, Fx, Fy, Fz, T(p.omega), o, drho, ux, uy, uz);
#pragma unroll
  for (int l = 0; l < Q; ++l) __builtin_nontemporal_store(o[l], dst + pop_at<Q>(l, z, y, x, ny, nx));
  if (p.h[0]) {
    p.h[0][i] = 1.0 + double(drho);  // rho - 1 kept to the storage type's precision
    p.h[1][i] = double(ux);
    p.h[2][i] = double(uy);
    p.h[3][i] = double(uz);
  }
}

// ---- K steps per launch (temporal blocking) ---------------------------------------------
// A workgroup of bx * by lanes owns an (x, y) tile of (bx - 2 (K - 1)) x (by - 2 (K - 1))
// output columns and a band of bz planes, and marches up the band one plane per
// iteration; lane (lx, ly) holds column (x0 - (K - 1) + lx, y0 - (K - 1) + ly), so the
// tile and its K - 1 halo columns on every side are one run of lanes.  Level s = 1..K of
// an iteration advances one plane by one step: level 1 pulls from the source state in
// HBM exactly as the one-step kernel does, level s > 1 collides the output of level
// s - 1.  A level's 16 populations with c_x or c_y != 0 reach the neighbouring lanes
// through LDS (two buffers used alternately, one barrier per level); the pull in z is
// a delay in registers: level s works one plane below level s - 1, takes the c_z = -1
// populations of level s - 1's current plane, the c_z = 0 ones of its previous plane and
// the c_z = +1 ones of the plane before (two register sets whose roles alternate with the
// iteration's parity).  Level s exists on the lanes at least s - 1 away from the edges of
// the tile's run, and only level K writes to HBM: K updates cost one read and one write
// of every population and one read of the force, with the same per-site arithmetic as K
// one-step launches (bit-identical results).
struct Fused3 {
  const void* src;
  void* dst;
  const void* fx;
  const void* fy;
  const void* fz;
  int nx, ny, nz;
  int bx, by, bz;         // lanes in x and y, band height
  int tiles_x, tiles_y;   // output tiles of (bx - 2 (K - 1)) x (by - 2 (K - 1)) columns
  int total;              // tiles_x * tiles_y * bands
  double omega;
};

// the 16 populations with c_x or c_y != 0, in LDS slot order
__host__ __device__ constexpr int kXY[16] = {1, 2, 3, 4, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18};
// c_z = 0 (carried one iteration) and c_z = +1 (carried two iterations)
__host__ __device__ constexpr int kZ0[9] = {0, 1, 2, 3, 4, 7, 8, 9, 10};
__host__ __device__ constexpr int kZP[5] = {5, 11, 14, 15, 18};

template <typename T, int K>
struct Carry3 {
  T z0[9];       // level s - 1, previous plane, c_z = 0 populations (pulled in x, y)
  T zp[2][5];    // level s - 1, the two previous planes, c_z = +1 populations
  T f[3];        // force at level s's plane
};

template <typename T, int K, bool FORCE>
__global__ void __launch_bounds__(512) k3_step_fused(Fused3 p) {
  extern __shared__ unsigned char smem3[];
  T* const lds = reinterpret_cast<T*>(smem3);
  const int lanes = p.bx * p.by;
  const int ox = p.bx - 2 * (K - 1), oy = p.by - 2 * (K - 1);
  int b = blockIdx.x;
  if (b >= p.total) return;  // uniform over the workgroup
  const int tx = b % p.tiles_x;
  b /= p.tiles_x;
  const int ty = b % p.tiles_y;
  const int tz = b / p.tiles_y;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x0 = tx * ox, y0 = ty * oy, z0 = tz * p.bz;
  const int weff = min(ox, nx - x0), heff = min(oy, ny - y0), deff = min(p.bz, nz - z0);
  const int nax = weff + 2 * (K - 1), nay = heff + 2 * (K - 1);
  const int t = threadIdx.x;
  const int lx = t % p.bx, ly = t / p.bx;
  int top = 0, x = x0, y = y0;
  if (lx < nax && ly < nay) {
    top = min(min(min(lx, nax - 1 - lx), min(ly, nay - 1 - ly)) + 1, K);
    x = wrap(x0 - (K - 1) + lx, nx);
    y = wrap(y0 - (K - 1) + ly, ny);
  }
  const int xm = wrap(x - 1, nx), xp = wrap(x + 1, nx), ym = wrap(y - 1, ny), yp = wrap(y + 1, ny);
  const T* __restrict__ src = static_cast<const T*>(p.src);
  T* __restrict__ dst = static_cast<T*>(p.dst);
  const T* __restrict__ gfx = static_cast<const T*>(p.fx);
  const T* __restrict__ gfy = static_cast<const T*>(p.fy);
  const T* __restrict__ gfz = static_cast<const T*>(p.fz);
  const T om = T(p.omega);

  // level 1 input of plane zl: f_l(x - c_l) of the source state, and the force there
  auto load_plane = [&](int zl, T (&d)[Q3], T (&f)[3]) {
    const int z = wrap(zl, nz), zmn = wrap(zl - 1, nz), zpl = wrap(zl + 1, nz);
#pragma unroll
    for (int l = 0; l < Q3; ++l) {
      const int cx = c3(l, 0), cy = c3(l, 1), cz = c3(l, 2);
      const int xs = cx == 1 ? xm : (cx == -1 ? xp : x);
      const int ys = cy == 1 ? ym : (cy == -1 ? yp : y);
      const int zs = cz == 1 ? zmn : (cz == -1 ? zpl : z);
      d[l] = __builtin_nontemporal_load(src + pop_at(l, zs, ys, xs, ny, nx));
    }
    if constexpr (FORCE) {
      const size_t i = (static_cast<size_t>(z) * ny + y) * nx + x;
      f[0] = gfx[i];
      f[1] = gfy[i];
      f[2] = gfz[i];
    } else {
      f[0] = f[1] = f[2] = T(0);
    }
  };

  Carry3<T, K> cy[K - 1];  // inputs of levels 2..K
#pragma unroll
  for (int s = 0; s < K - 1; ++s) {
#pragma unroll
    for (int j = 0; j < 9; ++j) cy[s].z0[j] = T(0);
#pragma unroll
    for (int j = 0; j < 5; ++j) cy[s].zp[0][j] = cy[s].zp[1][j] = T(0);
    cy[s].f[0] = cy[s].f[1] = cy[s].f[2] = T(0);
  }
  T d[Q3], f1[3];
  const int last = deff + K - 2;
  load_plane(z0 - (K - 1), d, f1);

  // iteration k: level s works on plane z0 + k - (s - 1), with valid input from
  // k = 2 s - 1 - K on; level K writes planes z0 .. z0 + deff - 1.  E is the parity
  // of the iteration count (LDS buffers and the two c_z = +1 register sets).
  auto iteration = [&](auto parity, int k) {
    constexpr int E = decltype(parity)::value;
    constexpr int P0 = ((K - 1) & 1) ? E : 0;
    T o[Q3], drho, ux, uy, uz;
    if (top >= 1) collide3<T, FORCE>(d, f1[0], f1[1], f1[2], om, o, drho, ux, uy, uz);
    T fprev[3] = {f1[0], f1[1], f1[2]};
    // the next plane's level-1 input: its loads fly while levels 2..K run
    if (k < last) load_plane(z0 + k + 1, d, f1);
#pragma unroll
    for (int s = 2; s <= K; ++s) {
      T* const slot = lds + ((P0 + s) & 1) * 16 * lanes;
      if (top >= s - 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) slot[j * lanes + t] = o[kXY[j]];
      }
      __syncthreads();
      Carry3<T, K>& c = cy[s - 2];
      // force of level s's plane: level s - 1's force of the previous iteration
      const T fs[3] = {c.f[0], c.f[1], c.f[2]};
      c.f[0] = fprev[0];
      c.f[1] = fprev[1];
      c.f[2] = fprev[2];
      fprev[0] = fs[0];
      fprev[1] = fs[1];
      fprev[2] = fs[2];
      if (k >= 2 * s - 3 - K && top >= s) {  // level s - 1 held valid data
        // g_l: level s - 1's value of the current plane at (x - c_x, y - c_y)
        T g[Q3];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int l = kXY[j];
          g[l] = slot[j * lanes + t - c3(l, 0) - c3(l, 1) * p.bx];
        }
        g[0] = o[0];
        g[5] = o[5];
        g[6] = o[6];
        if (k >= 2 * s - 1 - K) {
          T dn[Q3];
#pragma unroll
          for (int l = 0; l < Q3; ++l) dn[l] = g[l];  // c_z = -1: the current plane
#pragma unroll
          for (int j = 0; j < 9; ++j) dn[kZ0[j]] = c.z0[j];
#pragma unroll
          for (int j = 0; j < 5; ++j) dn[kZP[j]] = c.zp[E ^ 1][j];
          collide3<T, FORCE>(dn, fs[0], fs[1], fs[2], om, o, drho, ux, uy, uz);
          if (s == K) {
            const int zo = z0 + k - (K - 1);
#pragma unroll
            for (int l = 0; l < Q3; ++l) __builtin_nontemporal_store(o[l], dst + pop_at(l, zo, y, x, ny, nx));
          }
        }
#pragma unroll
        for (int j = 0; j < 9; ++j) c.z0[j] = g[kZ0[j]];
#pragma unroll
        for (int j = 0; j < 5; ++j) c.zp[E ^ 1][j] = g[kZP[j]];
      }
    }
  };
  for (int k = 1 - K; k <= last; k += 2) {
    iteration(std::integral_constant<int, 0>(), k);
    if (k + 1 > last) break;
    iteration(std::integral_constant<int, 1>(), k + 1);
  }
}

template <typename T, int Q = Q3>
__global__ void __launch_bounds__(256) k3_init(T* __restrict__ pop, const double* __restrict__ r0,
                                               const double* __restrict__ u0, const double* __restrict__ v0,
                                               const double* __restrict__ w0, int nx, int ny, int nz) {
  const size_t plane = static_cast<size_t>(nx) * ny * nz;
  for (size_t i = blockIdx.x * size_t(256) + threadIdx.x; i < plane; i += size_t(gridDim.x) * 256) {
    const int x = static_cast<int>(i % nx);
    const int y = static_cast<int>((i / nx) % ny);
    const int z = static_cast<int>(i / (static_cast<size_t>(nx) * ny));
    const double rho = r0[i], ux = u0[i], uy = v0[i], uz = w0[i];
    const double usq15 = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const double cu = cq3<Q>(l, 0) * ux + cq3<Q>(l, 1) * uy + cq3<Q>(l, 2) * uz;
      const double dev = wq3<Q>(l) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - usq15));
      const int xs = wrap(x - cq3<Q>(l, 0), nx), ys = wrap(y - cq3<Q>(l, 1), ny), zs = wrap(z - cq3<Q>(l, 2), nz);
      pop[pop_at<Q>(l, zs, ys, xs, ny, nx)] = T(dev);
    }
  }
}

template <typename T>
__global__ void k3_to_storage(T* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    dst[i] = T(src[i]);
}

// ---- moments ---------------------------------------------------------------------------------
constexpr int kS3 = 8;  // mass, momx, momy, momz, energy, max |u|, min rho, non-finite
template <typename T, bool FORCE, int Q = Q3>
__global__ void __launch_bounds__(kRedThreads) k3_moments(const T* __restrict__ pop, const T* __restrict__ fx,
                                                          const T* __restrict__ fy, const T* __restrict__ fz,
                                                          int nx, int ny, int nz, double* r, double* u,
                                                          double* v, double* w, double* partials) {
  const size_t plane = static_cast<size_t>(nx) * ny * nz;
  double acc[kS3] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1e300, 0.0};
  for (size_t i = blockIdx.x * size_t(kRedThreads) + threadIdx.x; i < plane;
       i += size_t(gridDim.x) * kRedThreads) {
    const int x = static_cast<int>(i % nx);
    const int y = static_cast<int>((i / nx) % ny);
    const int z = static_cast<int>(i / (static_cast<size_t>(nx) * ny));
    // the same rounding as the step: moments in the storage type
    T tr = T(0), tx = T(0), ty = T(0), tz = T(0);
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const int xs = wrap(x - cq3<Q>(l, 0), nx), ys = wrap(y - cq3<Q>(l, 1), ny), zs = wrap(z - cq3<Q>(l, 2), nz);
      const T dl = pop[pop_at<Q>(l, zs, ys, xs, ny, nx)];
      tr += dl;
      if (cq3<Q>(l, 0)) tx += cq3<Q>(l, 0) * dl;
      if (cq3<Q>(l, 1)) ty += cq3<Q>(l, 1) * dl;
      if (cq3<Q>(l, 2)) tz += cq3<Q>(l, 2) * dl;
    }
    const T rho = T(1) + tr;
    T Fx = T(0), Fy = T(0), Fz = T(0);
    if constexpr (FORCE) {
      Fx = fx[i];
      Fy = fy[i];
      Fz = fz[i];
    }
    const T inv = T(1) / rho;
    const double R = 1.0 + double(tr);  // formed in FP64 (see the 2D moments)
    const double U = double((tx + T(0.5) * Fx) * inv), V = double((ty + T(0.5) * Fy) * inv),
                 Wv = double((tz + T(0.5) * Fz) * inv);
    if (r) r[i] = R;
    if (u) u[i] = U;
    if (v) v[i] = V;
    if (w) w[i] = Wv;
    const double s2 = U * U + V * V + Wv * Wv;
    acc[0] += R;
    acc[1] += R * U;
    acc[2] += R * V;
    acc[3] += R * Wv;
    acc[4] += 0.5 * R * s2;
    acc[5] = fmax(acc[5], sqrt(s2));
    acc[6] = fmin(acc[6], R);
    acc[7] += (isfinite(R) && isfinite(U) && isfinite(V) && isfinite(Wv)) ? 0.0 : 1.0;
  }
  __shared__ double sh[kRedThreads / 64][kS3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double red[kS3];
#pragma unroll
  for (int k = 0; k < kS3; ++k) red[k] = k == 5 ? wave_max(acc[k]) : (k == 6 ? wave_min(acc[k]) : wave_sum(acc[k]));
  if (lane == 0)
    for (int k = 0; k < kS3; ++k) sh[wv][k] = red[k];
  __syncthreads();
  if (threadIdx.x < kS3) {
    const int k = threadIdx.x;
    double a = sh[0][k];
    for (int q = 1; q < kRedThreads / 64; ++q) a = k == 5 ? fmax(a, sh[q][k]) : (k == 6 ? fmin(a, sh[q][k]) : a + sh[q][k]);
    partials[blockIdx.x * kS3 + k] = a;
  }
}

__global__ void __launch_bounds__(kRedThreads) k3_reduce_scalars(const double* __restrict__ part, int nb,
                                                                 double* out) {
  double a[kS3];
#pragma unroll
  for (int k = 0; k < kS3; ++k) a[k] = k == 6 ? 1e300 : 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads)
#pragma unroll
    for (int k = 0; k < kS3; ++k) {
      const double q = part[b * kS3 + k];
      a[k] = k == 5 ? fmax(a[k], q) : (k == 6 ? fmin(a[k], q) : a[k] + q);
    }
  __shared__ double sh[kRedThreads / 64][kS3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kS3; ++k) {
    const double r = k == 5 ? wave_max(a[k]) : (k == 6 ? wave_min(a[k]) : wave_sum(a[k]));
    if (lane == 0) sh[wv][k] = r;
  }
  __syncthreads();
  if (threadIdx.x < kS3) {
    const int k = threadIdx.x;
    double r = sh[0][k];
    for (int w = 1; w < kRedThreads / 64; ++w) r = k == 5 ? fmax(r, sh[w][k]) : (k == 6 ? fmin(r, sh[w][k]) : r + sh[w][k]);
    out[k] = r;
  }
}

// ---- balance --------------------------------------------------------------------------------
constexpr int NT3 = 14;  // lhs_E, e1..e5, lhs_Z, z1..z6, usq
static_assert(NT3 == LBM3_NTERMS, "term count");
enum { T3_LHS_E = 0, T3_E1, T3_E2, T3_E3, T3_E4, T3_E5, T3_LHS_Z, T3_Z1, T3_Z2, T3_Z3, T3_Z4, T3_Z5, T3_Z6,
       T3_USQ };
// aux: E, Omega, omega (3), sigma xx yy zz xy xz yz, F / rho (3), H (3)
enum { A3_E = 0, A3_OM2, A3_WX, A3_WY, A3_WZ, A3_SXX, A3_SYY, A3_SZZ, A3_SXY, A3_SXZ, A3_SYZ, A3_GX, A3_GY,
       A3_GZ, A3_HX, A3_HY, A3_HZ, NA3 };

struct Bal3 {
  const double* rho[3];
  const double* u[3][3];  // [level][component]
  const double* F[3];     // total force at n (or null)
  double nu;
  int nx, ny, nz;
  double* terms;  // [NT3][plane]
  double* aux;    // [NA3][plane]
};

struct Site3 {
  int x, y, z, nx, ny, nz;
  size_t i;
  __device__ size_t at(int dx, int dy, int dz) const {
    return (static_cast<size_t>(wrap(z + dz, nz)) * ny + wrap(y + dy, ny)) * nx + wrap(x + dx, nx);
  }
};

// Eq. 18 along axis a of the value that `val(j)` returns at linear index j.
template <typename Fn>
__device__ __forceinline__ double fd8(const Site3& s, int a, Fn val) {
  auto d = [&](int m) {
    return val(s.at(a == 0 ? m : 0, a == 1 ? m : 0, a == 2 ? m : 0)) -
           val(s.at(a == 0 ? -m : 0, a == 1 ? -m : 0, a == 2 ? -m : 0));
  };
  const double d1 = d(1), d2 = d(2), d3 = d(3), d4 = d(4);
  return (4.0 * d1 - d2 + (4.0 / 21.0) * d3 - (1.0 / 56.0) * d4) / 5.0;
}

// One workgroup per 256-site run of an x row.  Each plane's runs are dealt to the
// eight XCDs in contiguous bands (workgroup b runs on XCD b mod 8, and workgroups
// are started in order), plane after plane: all XCDs work on the same planes at a
// time, and an XCD's y neighbours, and most of its stencil planes, are rows its own
// L2 has just read.  The grid holds 8 * ceil(runs per plane / 8) * nz workgroups.
__device__ __forceinline__ bool site3(int nx, int ny, int nz, Site3& s) {
  const int gx = (nx + 255) / 256;
  const int per_plane = gx * ny, chunk = (per_plane + 7) / 8;
  const int k = static_cast<int>(blockIdx.x >> 3);
  const int q = static_cast<int>(blockIdx.x & 7) * chunk + k % chunk;   // run within the plane
  if (q >= per_plane) return false;
  s.x = (q % gx) * 256 + threadIdx.x;
  s.y = q / gx;
  s.z = k / chunk;
  s.nx = nx;
  s.ny = ny;
  s.nz = nz;
  if (s.x >= nx) return false;
  s.i = (static_cast<size_t>(s.z) * ny + s.y) * nx + s.x;
  return true;
}

// The passes write their fields with non-temporal stores: only later kernels read
// them, and kept out of L2 they do not evict the planes that the z differences reuse.
__global__ void __launch_bounds__(256) k3_bal_a(Bal3 a) {
  Site3 s;
  if (!site3(a.nx, a.ny, a.nz, s)) return;
  const size_t plane = static_cast<size_t>(a.nx) * a.ny * a.nz;
  const size_t i = s.i;
  double du[3][3];  // d_j u_i at level n
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double* f = a.u[2][c];
      du[c][j] = fd8(s, j, [&](size_t k) { return f[k]; });
    }
  double dr[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double* f = a.rho[2];
    dr[j] = fd8(s, j, [&](size_t k) { return f[k]; });
  }
  double en[3], ens[3];
  double wn[3];
#pragma unroll
  for (int lv = 0; lv < 3; ++lv) {
    double w[3];
    if (lv == 2) {
      w[0] = du[2][1] - du[1][2];
      w[1] = du[0][2] - du[2][0];
      w[2] = du[1][0] - du[0][1];
      wn[0] = w[0];
      wn[1] = w[1];
      wn[2] = w[2];
    } else {
      const double* ux = a.u[lv][0];
      const double* uy = a.u[lv][1];
      const double* uz = a.u[lv][2];
      w[0] = fd8(s, 1, [&](size_t k) { return uz[k]; }) - fd8(s, 2, [&](size_t k) { return uy[k]; });
      w[1] = fd8(s, 2, [&](size_t k) { return ux[k]; }) - fd8(s, 0, [&](size_t k) { return uz[k]; });
      w[2] = fd8(s, 0, [&](size_t k) { return uy[k]; }) - fd8(s, 1, [&](size_t k) { return ux[k]; });
    }
    const double vx = a.u[lv][0][i], vy = a.u[lv][1][i], vz = a.u[lv][2][i];
    en[lv] = 0.5 * a.rho[lv][i] * (vx * vx + vy * vy + vz * vz);
    ens[lv] = 0.5 * (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  }
  const double r = a.rho[2][i];
  const double v[3] = {a.u[2][0][i], a.u[2][1][i], a.u[2][2][i]};
  double F[3] = {0.0, 0.0, 0.0};
  if (a.F[0]) {
    F[0] = a.F[0][i];
    F[1] = a.F[1][i];
    F[2] = a.F[2][i];
  }
  const double nu = a.nu;
  double sg[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) sg[c][j] = nu * r * (du[c][j] + du[j][c]);
  double e4 = 0.0, z6 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      e4 -= sg[c][j] * du[c][j];
      z6 += wn[c] * wn[j] * du[c][j];
    }
  double* t = a.terms;
  __builtin_nontemporal_store((3.0 * en[2] - 4.0 * en[1] + en[0]) / 2.0, &t[T3_LHS_E * plane + i]);
  __builtin_nontemporal_store(-(v[0] * dr[0] + v[1] * dr[1] + v[2] * dr[2]) / 3.0, &t[T3_E2 * plane + i]);
  __builtin_nontemporal_store(v[0] * F[0] + v[1] * F[1] + v[2] * F[2], &t[T3_E3 * plane + i]);
  __builtin_nontemporal_store(e4, &t[T3_E4 * plane + i]);
  __builtin_nontemporal_store((3.0 * ens[2] - 4.0 * ens[1] + ens[0]) / 2.0, &t[T3_LHS_Z * plane + i]);
  __builtin_nontemporal_store(-ens[2] * (du[0][0] + du[1][1] + du[2][2]), &t[T3_Z2 * plane + i]);
  __builtin_nontemporal_store(z6, &t[T3_Z6 * plane + i]);
  __builtin_nontemporal_store(v[0] * v[0] + v[1] * v[1] + v[2] * v[2], &t[T3_USQ * plane + i]);
  double* x = a.aux;
  __builtin_nontemporal_store(en[2], &x[A3_E * plane + i]);
  __builtin_nontemporal_store(ens[2], &x[A3_OM2 * plane + i]);
  __builtin_nontemporal_store(wn[0], &x[A3_WX * plane + i]);
  __builtin_nontemporal_store(wn[1], &x[A3_WY * plane + i]);
  __builtin_nontemporal_store(wn[2], &x[A3_WZ * plane + i]);
  __builtin_nontemporal_store(sg[0][0], &x[A3_SXX * plane + i]);
  __builtin_nontemporal_store(sg[1][1], &x[A3_SYY * plane + i]);
  __builtin_nontemporal_store(sg[2][2], &x[A3_SZZ * plane + i]);
  __builtin_nontemporal_store(sg[0][1], &x[A3_SXY * plane + i]);
  __builtin_nontemporal_store(sg[0][2], &x[A3_SXZ * plane + i]);
  __builtin_nontemporal_store(sg[1][2], &x[A3_SYZ * plane + i]);
  __builtin_nontemporal_store(F[0] / r, &x[A3_GX * plane + i]);
  __builtin_nontemporal_store(F[1] / r, &x[A3_GY * plane + i]);
  __builtin_nontemporal_store(F[2] / r, &x[A3_GZ * plane + i]);
}

__device__ __forceinline__ int sig_index(int c, int j) {
  // symmetric stress component (c, j) in the aux layout
  if (c == j) return A3_SXX + c;
  const int lo = c < j ? c : j, hi = c < j ? j : c;
  return lo == 0 ? (hi == 1 ? A3_SXY : A3_SXZ) : A3_SYZ;
}

__global__ void __launch_bounds__(256) k3_bal_b(Bal3 a) {
  Site3 s;
  if (!site3(a.nx, a.ny, a.nz, s)) return;
  const size_t plane = static_cast<size_t>(a.nx) * a.ny * a.nz;
  const size_t i = s.i;
  const double* ax = a.aux;
  const double* const* u = a.u[2];
  double e1 = 0.0, e5 = 0.0, z1 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double* uj = u[j];
    e1 -= fd8(s, j, [&](size_t k) { return ax[A3_E * plane + k] * uj[k]; });
    z1 -= fd8(s, j, [&](size_t k) { return ax[A3_OM2 * plane + k] * uj[k]; });
    const double* s0 = ax + sig_index(0, j) * plane;
    const double* s1 = ax + sig_index(1, j) * plane;
    const double* s2 = ax + sig_index(2, j) * plane;
    e5 += fd8(s, j, [&](size_t k) { return u[0][k] * s0[k] + u[1][k] * s1[k] + u[2][k] * s2[k]; });
  }
  // curl(F / rho)
  const double* gx = ax + A3_GX * plane;
  const double* gy = ax + A3_GY * plane;
  const double* gz = ax + A3_GZ * plane;
  const double cg[3] = {fd8(s, 1, [&](size_t k) { return gz[k]; }) - fd8(s, 2, [&](size_t k) { return gy[k]; }),
                        fd8(s, 2, [&](size_t k) { return gx[k]; }) - fd8(s, 0, [&](size_t k) { return gz[k]; }),
                        fd8(s, 0, [&](size_t k) { return gy[k]; }) - fd8(s, 1, [&](size_t k) { return gx[k]; })};
  const double w[3] = {ax[A3_WX * plane + i], ax[A3_WY * plane + i], ax[A3_WZ * plane + i]};
  const double r = a.rho[2][i];
  double h[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double dv = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double* sc = ax + sig_index(c, j) * plane;
      dv += fd8(s, j, [&](size_t k) { return sc[k]; });
    }
    h[c] = dv / r;
  }
  double* t = a.terms;
  __builtin_nontemporal_store(e1, &t[T3_E1 * plane + i]);
  __builtin_nontemporal_store(e5, &t[T3_E5 * plane + i]);
  __builtin_nontemporal_store(z1, &t[T3_Z1 * plane + i]);
  __builtin_nontemporal_store(w[0] * cg[0] + w[1] * cg[1] + w[2] * cg[2], &t[T3_Z3 * plane + i]);
  double* x = a.aux;
  __builtin_nontemporal_store(h[0], &x[A3_HX * plane + i]);
  __builtin_nontemporal_store(h[1], &x[A3_HY * plane + i]);
  __builtin_nontemporal_store(h[2], &x[A3_HZ * plane + i]);
}

__global__ void __launch_bounds__(256) k3_bal_c(Bal3 a) {
  Site3 s;
  if (!site3(a.nx, a.ny, a.nz, s)) return;
  const size_t plane = static_cast<size_t>(a.nx) * a.ny * a.nz;
  const size_t i = s.i;
  const double* ax = a.aux;
  const double* wx = ax + A3_WX * plane;
  const double* wy = ax + A3_WY * plane;
  const double* wz = ax + A3_WZ * plane;
  const double* hx = ax + A3_HX * plane;
  const double* hy = ax + A3_HY * plane;
  const double* hz = ax + A3_HZ * plane;
  const double cw[3] = {fd8(s, 1, [&](size_t k) { return wz[k]; }) - fd8(s, 2, [&](size_t k) { return wy[k]; }),
                        fd8(s, 2, [&](size_t k) { return wx[k]; }) - fd8(s, 0, [&](size_t k) { return wz[k]; }),
                        fd8(s, 0, [&](size_t k) { return wy[k]; }) - fd8(s, 1, [&](size_t k) { return wx[k]; })};
  // div(H x omega), (H x omega) = (hy wz - hz wy, hz wx - hx wz, hx wy - hy wx)
  const double z5 = fd8(s, 0, [&](size_t k) { return hy[k] * wz[k] - hz[k] * wy[k]; }) +
                    fd8(s, 1, [&](size_t k) { return hz[k] * wx[k] - hx[k] * wz[k]; }) +
                    fd8(s, 2, [&](size_t k) { return hx[k] * wy[k] - hy[k] * wx[k]; });
  double* t = a.terms;
  __builtin_nontemporal_store(hx[i] * cw[0] + hy[i] * cw[1] + hz[i] * cw[2], &t[T3_Z4 * plane + i]);
  __builtin_nontemporal_store(z5, &t[T3_Z5 * plane + i]);
}

// ---- summed-volume tables ---------------------------------------------------------------------
// P[f][z][y][x] over (nz+1)(ny+1)(nx+1): sum of (g_f - mean_f) over z' < z, y' < y, x' < x.
struct Vol {
  double* P;
  const double* means;
  int nx, ny, nz;
  __host__ __device__ size_t sx() const { return static_cast<size_t>(nx) + 1; }
  __host__ __device__ size_t sy() const { return (static_cast<size_t>(ny) + 1) * sx(); }
  __host__ __device__ size_t sf() const { return (static_cast<size_t>(nz) + 1) * sy(); }
  __device__ double get(int f, int z, int y, int x) const { return P[f * sf() + z * sy() + y * sx() + x]; }
  // the periodic continuation to 0 <= z <= 2 nz (and y, x): each axis index is its
  // remainder plus, past the grid, one full period
  __device__ double Q(int f, int z, int y, int x) const {
    const int zs[2] = {z > nz ? z - nz : z, nz}, ys[2] = {y > ny ? y - ny : y, ny},
              xs[2] = {x > nx ? x - nx : x, nx};
    const int cz = z > nz ? 2 : 1, cy = y > ny ? 2 : 1, cx = x > nx ? 2 : 1;
    double v = 0.0;
    for (int a = 0; a < cz; ++a)
      for (int b = 0; b < cy; ++b)
        for (int c = 0; c < cx; ++c) v += get(f, zs[a], ys[b], xs[c]);
    return v;
  }
  __device__ double box_mean(int f, int x0, int y0, int z0, int L) const {
    const int x1 = x0 + L, y1 = y0 + L, z1 = z0 + L;
    const double s = Q(f, z1, y1, x1) - Q(f, z0, y1, x1) - Q(f, z1, y0, x1) - Q(f, z1, y1, x0) +
                     Q(f, z0, y0, x1) + Q(f, z0, y1, x0) + Q(f, z1, y0, x0) - Q(f, z0, y0, x0);
    return means[f] + s / (double(L) * double(L) * double(L));
  }
};

// x scan: one workgroup per (y, z, field) row, coalesced 256-value segments.
__global__ void __launch_bounds__(256) k3_sat_x(const double* __restrict__ g, Vol v) {
  __shared__ double wsum[4];
  const int y = blockIdx.x, z = blockIdx.y, f = blockIdx.z;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t plane = static_cast<size_t>(v.nx) * v.ny * v.nz;
  const double mean = v.means[f];
  const double* row = g + f * plane + (static_cast<size_t>(z) * v.ny + y) * v.nx;
  double* out = v.P + f * v.sf() + (z + 1) * v.sy() + (y + 1) * v.sx();
  double carry = 0.0;
  for (int x0 = 0; x0 < v.nx; x0 += 256) {
    const int x = x0 + threadIdx.x;
    double val = x < v.nx ? row[x] - mean : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double t = __shfl_up(val, off, 64);
      if (lane >= off) val += t;
    }
    if (lane == 63) wsum[wv] = val;
    __syncthreads();
    double before = 0.0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    const double total = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    if (x < v.nx) out[x + 1] = carry + (before + val);
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.0;
}

// The x scans and the y running sums of one (z, field) plane in one pass, for
// nx <= 256 * kXYChunks: the workgroup walks the plane's rows in order, scans each
// row as k3_sat_x does and adds the row's prefix sums to per-column running sums kept
// in registers, as k3_sat_y does (same operations in the same order: the same bits).
// The next row's values are loaded before the current row is scanned, and the wave
// totals alternate between two LDS slots so one barrier per row segment suffices.
constexpr int kXYChunks = 4;
__global__ void __launch_bounds__(256) k3_sat_xy(const double* __restrict__ g, Vol v) {
  __shared__ double wsum[2][4];
  const int z = blockIdx.x, f = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t plane = static_cast<size_t>(v.nx) * v.ny * v.nz;
  const double mean = v.means[f];
  const double* src = g + f * plane + static_cast<size_t>(z) * v.ny * v.nx;
  double* dst = v.P + f * v.sf() + (z + 1) * v.sy();
  double run[kXYChunks], cur[kXYChunks];
#pragma unroll
  for (int c = 0; c < kXYChunks; ++c) {
    run[c] = 0.0;
    const int x = c * 256 + threadIdx.x;
    cur[c] = x < v.nx ? src[x] : 0.0;
  }
  int par = 0;
  for (int y = 0; y < v.ny; ++y) {
    double nxt[kXYChunks];
    const double* nrow = src + static_cast<size_t>(y + 1 < v.ny ? y + 1 : y) * v.nx;
#pragma unroll
    for (int c = 0; c < kXYChunks; ++c) {
      const int x = c * 256 + threadIdx.x;
      nxt[c] = x < v.nx ? nrow[x] : 0.0;
    }
    double* out = dst + (y + 1) * v.sx();
    double carry = 0.0;
#pragma unroll
    for (int c = 0; c < kXYChunks; ++c) {
      if (c * 256 >= v.nx) break;
      const int x = c * 256 + threadIdx.x;
      double val = x < v.nx ? cur[c] - mean : 0.0;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(val, off, 64);
        if (lane >= off) val += t;
      }
      if (lane == 63) wsum[par][wv] = val;
      __syncthreads();
      double before = 0.0;
      for (int w = 0; w < wv; ++w) before += wsum[par][w];
      const double total = (wsum[par][0] + wsum[par][1]) + (wsum[par][2] + wsum[par][3]);
      if (x < v.nx) {
        run[c] += carry + (before + val);
        out[x + 1] = run[c];
      }
      carry += total;
      par ^= 1;
    }
    if (threadIdx.x == 0) out[0] = 0.0;
#pragma unroll
    for (int c = 0; c < kXYChunks; ++c) cur[c] = nxt[c];
  }
}

// zero faces: z = 0 planes and y = 0 rows of every field
__global__ void k3_sat_faces(Vol v, int nf) {
  const size_t face = v.sy();                                 // one z = 0 plane
  const size_t rows = static_cast<size_t>(v.nz) * v.sx();     // y = 0 rows of z >= 1
  const size_t per = face + rows;
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < per * nf; k += size_t(gridDim.x) * blockDim.x) {
    const size_t f = k / per, r = k % per;
    double* base = v.P + f * v.sf();
    if (r < face)
      base[r] = 0.0;
    else {
      const size_t q = r - face;
      base[(q / v.sx() + 1) * v.sy() + q % v.sx()] = 0.0;
    }
  }
}

// running sums along y, then along z: one thread per x column (coalesced), sequential in y / z
__global__ void __launch_bounds__(256) k3_sat_y(Vol v) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x > v.nx) return;
  const int z = blockIdx.y + 1, f = blockIdx.z;
  double* col = v.P + f * v.sf() + z * v.sy() + x;
  double run = 0.0;
  for (int y = 1; y <= v.ny; ++y) {
    run += col[y * v.sx()];
    col[y * v.sx()] = run;
  }
}

__global__ void __launch_bounds__(256) k3_sat_z(Vol v) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x > v.nx) return;
  const int y = blockIdx.y, f = blockIdx.z;
  double* col = v.P + f * v.sf() + y * v.sx() + x;
  double run = 0.0;
  for (int z = 1; z <= v.nz; ++z) {
    run += col[z * v.sy()];
    col[z * v.sy()] = run;
  }
}

// ---- windows -----------------------------------------------------------------------------------
constexpr int kW3Threads = 256;
constexpr int kW3MaxBlocks = 2048;
constexpr int kW3Vals = 18;  // 3 quantities x (n, mean, m2, min, max, nan)

__device__ void w3_errors(const double (&m)[NT3], double& dE, double& dZ, double& ma) {
  const double rE = (((m[T3_E1] + m[T3_E2]) + m[T3_E3]) + m[T3_E4]) + m[T3_E5];
  const double denE = fmax(fmax(fmax(fabs(m[T3_E1]), fabs(m[T3_E2])), fmax(fabs(m[T3_E3]), fabs(m[T3_E4]))),
                           fabs(m[T3_E5]));
  const double rZ = ((((m[T3_Z1] + m[T3_Z2]) + m[T3_Z3]) + m[T3_Z4]) + m[T3_Z5]) + m[T3_Z6];
  const double denZ = fmax(fmax(fmax(fabs(m[T3_Z1]), fabs(m[T3_Z2])), fmax(fabs(m[T3_Z3]), fabs(m[T3_Z4]))),
                           fmax(fabs(m[T3_Z5]), fabs(m[T3_Z6])));
  dE = denE > 0.0 ? fabs(rE - m[T3_LHS_E]) / denE : __builtin_nan("");
  dZ = denZ > 0.0 ? fabs(rZ - m[T3_LHS_Z]) / denZ : __builtin_nan("");
  ma = sqrt(m[T3_USQ]) * 1.7320508075688772;  // / c_s, c_s = 1/sqrt(3)
}

// Running count, mean and sum of squared deviations (Welford), merged pairwise
// by Chan's formula; min, max and the count of NaN values beside them.
struct Run3 {
  double n, mean, m2, mn, mx, nan;
  __device__ void init() {
    n = mean = m2 = nan = 0.0;
    mn = 1e300;
    mx = -1e300;
  }
  __device__ void add(double v) {
    if (!isfinite(v)) {
      nan += 1.0;
      return;
    }
    n += 1.0;
    const double d = v - mean;
    mean += d / n;
    m2 += d * (v - mean);
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  __device__ void merge(const Run3& b) {
    if (b.n > 0.0) {
      const double nn = n + b.n, d = b.mean - mean;
      mean += d * (b.n / nn);
      m2 += b.m2 + d * d * (n * b.n / nn);
      n = nn;
      mn = fmin(mn, b.mn);
      mx = fmax(mx, b.mx);
    }
    nan += b.nan;
  }
  __device__ void load(const double* p) { n = p[0], mean = p[1], m2 = p[2], mn = p[3], mx = p[4], nan = p[5]; }
  __device__ void store(double* p) const { p[0] = n, p[1] = mean, p[2] = m2, p[3] = mn, p[4] = mx, p[5] = nan; }
};

// Merge of a thread's three accumulators across its workgroup (a lane-independent
// butterfly in each wavefront, then the wavefronts in order) into the workgroup's partial.
// lane = index in the wavefront, wv = wavefront index, nwv wavefronts (at most 4).
__device__ void w3_block_partial(Run3 (&r)[3], int lane, int wv, int nwv, double* out) {
#pragma unroll
  for (int q = 0; q < 3; ++q)
    for (int off = 1; off < 64; off <<= 1) {
      Run3 o;
      o.n = __shfl_xor(r[q].n, off, 64);
      o.mean = __shfl_xor(r[q].mean, off, 64);
      o.m2 = __shfl_xor(r[q].m2, off, 64);
      o.mn = __shfl_xor(r[q].mn, off, 64);
      o.mx = __shfl_xor(r[q].mx, off, 64);
      o.nan = __shfl_xor(r[q].nan, off, 64);
      if ((lane & off) == 0) {
        r[q].merge(o);
      } else {
        o.merge(r[q]);
        r[q] = o;
      }
    }
  __shared__ double sh[4][kW3Vals];
  if (lane == 0)
    for (int q = 0; q < 3; ++q) r[q].store(&sh[wv][q * 6]);
  __syncthreads();
  if (wv == 0 && lane < 3) {
    const int q = lane;
    Run3 acc, b;
    acc.load(&sh[0][q * 6]);
    for (int w = 1; w < nwv; ++w) {
      b.load(&sh[w][q * 6]);
      acc.merge(b);
    }
    acc.store(out + q * 6);
  }
}

__global__ void __launch_bounds__(kW3Threads) k3_windows(Vol v, int L, size_t count, double* partials) {
  Run3 r[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) r[q].init();
  for (size_t k = blockIdx.x * size_t(kW3Threads) + threadIdx.x; k < count; k += size_t(gridDim.x) * kW3Threads) {
    const int x0 = static_cast<int>(k % v.nx);
    const int y0 = static_cast<int>((k / v.nx) % v.ny);
    const int z0 = static_cast<int>(k / (static_cast<size_t>(v.nx) * v.ny));
    double m[NT3];
    for (int f = 0; f < NT3; ++f) m[f] = v.box_mean(f, x0, y0, z0, L);
    double val[3];
    w3_errors(m, val[0], val[1], val[2]);
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q].add(val[q]);
  }
  w3_block_partial(r, threadIdx.x & 63, threadIdx.x >> 6, kW3Threads / 64,
                   partials + static_cast<size_t>(blockIdx.x) * kW3Vals);
}

// The corner's offsets in a table plane for the xy box [x0, x0 + L) x [y0, y0 + L),
// through the periodic continuation of x and y: a corner index past the grid is its
// remainder plus one full period (column nx, row ny of the table).
struct XYBox {
  size_t r0, r1, rt;   // rows y0, y1 (remainder) and ny, in plane 0
  int x0, x1s, nx;
  bool xw, yw;
  __device__ XYBox(const Vol& v, int x, int y, int L) {
    const int x1 = x + L, y1 = y + L;
    xw = x1 > v.nx;
    yw = y1 > v.ny;
    x0 = x;
    x1s = xw ? x1 - v.nx : x1;
    nx = v.nx;
    r0 = static_cast<size_t>(y) * v.sx();
    r1 = static_cast<size_t>(yw ? y1 - v.ny : y1) * v.sx();
    rt = static_cast<size_t>(v.ny) * v.sx();
  }
  // box sum of table plane p (one field, one z); the row totals are loaded by every
  // lane and selected, not multiplied, so a non-finite total reaches only wrapping boxes
  __device__ __forceinline__ double sum(const double* __restrict__ p) const {
    const double a00 = p[r0 + x0], a01 = p[r0 + x1s], a0t = p[r0 + nx];
    const double a10 = p[r1 + x0], a11 = p[r1 + x1s], a1t = p[r1 + nx];
    const double q11 = xw ? a11 + a1t : a11, q01 = xw ? a01 + a0t : a01;
    double s = (q11 - a10) - (q01 - a00);
    if (yw) {
      const double t0 = p[rt + x0], t1 = p[rt + x1s], tt = p[rt + nx];
      s += (xw ? t1 + tt : t1) - t0;
    }
    return s;
  }
};

// Window statistics of side L < the grid by walks along z.  Thread (x0, y0) of the
// 64 x 4 workgroup takes the cubes with corner (x0, y0, j + m L), m = 0, 1, ..., for
// j = blockIdx.z, blockIdx.z + jg, ... < L: the xy box sums of table plane z serve as the
// top of one cube and the bottom of the next, so a cube costs one plane of box sums
// (six table values per field, nine where the box wraps in y) instead of eight corners.
// The cube past nz takes planes z1 - nz and nz (one period of z).  A thread keeps its
// bottom-plane sums in its own LDS slots (no barrier), so the field loop need not be
// unrolled; the box means go straight into the sums and maxima of the error ratios, in
// the field order of the corner-by-corner kernel.
//
// Work items r = (j group, y tile, x tile) are dealt to the XCDs in contiguous chunks
// (workgroup b runs on XCD b mod 8): the tiles that read the same table rows (x0 + L,
// y0 + L) share an L2, and at most sizes one XCD walks one residue class of z.
__global__ void __launch_bounds__(256) k3_windows_walk(Vol v, int L, int tx, int ty, int jg, double* partials) {
  __shared__ double bp[NT3][256];
  const int n = tx * ty * jg, per = (n + 7) / 8;
  const int r = static_cast<int>(blockIdx.x & 7) * per + static_cast<int>(blockIdx.x >> 3);
  if (r >= n) return;   // no partial slot: the merge reads slots 0 .. n - 1
  const int bxi = r % tx, byi = (r / tx) % ty, bzi = r / (tx * ty);
  const int x0 = bxi * 64 + threadIdx.x;
  const int y0 = byi * 4 + threadIdx.y;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  Run3 acc[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) acc[q].init();
  if (x0 < v.nx && y0 < v.ny) {
    const XYBox bx(v, x0, y0, L);
    const double inv_vol = 1.0 / (double(L) * double(L) * double(L));
    const size_t sy = v.sy(), sf = v.sf();
    // one cube: bottom plane sums in bp, top plane sums from plane pa (plus pt past nz)
    auto cube = [&](const double* pa, const double* pt) {
      double rE = 0.0, denE = 0.0, rZ = 0.0, denZ = 0.0, lhsE = 0.0, lhsZ = 0.0, usq = 0.0;
#pragma unroll 1
      for (int f = 0; f < NT3; ++f) {
        double bn = bx.sum(pa + f * sf);
        if (pt) bn += bx.sum(pt + f * sf);
        const double m = v.means[f] + (bn - bp[f][tid]) * inv_vol;
        bp[f][tid] = bn;
        if (f == T3_LHS_E) lhsE = m;
        if (f == T3_LHS_Z) lhsZ = m;
        if (f == T3_USQ) usq = m;
        if (f >= T3_E1 && f <= T3_E5) {
          rE = f == T3_E1 ? m : rE + m;
          denE = f == T3_E1 ? fabs(m) : fmax(denE, fabs(m));
        }
        if (f >= T3_Z1 && f <= T3_Z6) {
          rZ = f == T3_Z1 ? m : rZ + m;
          denZ = f == T3_Z1 ? fabs(m) : fmax(denZ, fabs(m));
        }
      }
      acc[0].add(denE > 0.0 ? fabs(rE - lhsE) / denE : __builtin_nan(""));
      acc[1].add(denZ > 0.0 ? fabs(rZ - lhsZ) / denZ : __builtin_nan(""));
      acc[2].add(sqrt(usq) * 1.7320508075688772);
    };
    for (int j = bzi; j < L; j += jg) {
#pragma unroll 2
      for (int f = 0; f < NT3; ++f) bp[f][tid] = bx.sum(v.P + f * sf + static_cast<size_t>(j) * sy);
      int z0 = j;
      for (; z0 + L <= v.nz; z0 += L) cube(v.P + static_cast<size_t>(z0 + L) * sy, nullptr);
      if (z0 < v.nz)
        cube(v.P + static_cast<size_t>(z0 + L - v.nz) * sy, v.P + static_cast<size_t>(v.nz) * sy);
    }
  }
  w3_block_partial(acc, threadIdx.x, threadIdx.y, 4, partials + static_cast<size_t>(r) * kW3Vals);
}

// Fixed-order merge of the workgroup partials: thread t takes partials t, t + 256, ...;
// then pairs of threads, four wavefronts, in a fixed tree.
__global__ void __launch_bounds__(256) k3_windows_final(const double* __restrict__ partials, int nb, double* out) {
  __shared__ double sh[256][kW3Vals];
  Run3 r[3], o;
#pragma unroll
  for (int q = 0; q < 3; ++q) r[q].init();
  for (int k = threadIdx.x; k < nb; k += 256)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      o.load(partials + static_cast<size_t>(k) * kW3Vals + q * 6);
      r[q].merge(o);
    }
#pragma unroll
  for (int q = 0; q < 3; ++q) r[q].store(&sh[threadIdx.x][q * 6]);
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        o.load(&sh[threadIdx.x + h][q * 6]);
        r[q].merge(o);
        r[q].store(&sh[threadIdx.x][q * 6]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) r[q].store(out + q * 6);
}

int grid1(size_t n, int cap) { return static_cast<int>(std::max<size_t>(1, std::min<size_t>(cap, (n + 255) / 256))); }

}  // namespace
}  // namespace lbm

// ==== handle ====================================================================================
using namespace lbm;

struct lbm3_ctx_s {
  lbm3_config cfg{};
  int q = 19;  // populations per site: 19 (D3Q19) or 27 (D3Q27)
  hipStream_t stream = nullptr;
  void* pop[2] = {nullptr, nullptr};
  int cur = 0;
  void* f[3] = {nullptr, nullptr, nullptr};  // force, storage type
  double* f64[3] = {nullptr, nullptr, nullptr};
  double* hist[2][4] = {{nullptr}};
  int64_t hist_t[2] = {-1, -1};
  double* mom[4] = {nullptr};
  double* partials = nullptr;
  double* scalars = nullptr;
  double* terms = nullptr;
  double* aux = nullptr;
  double* sat = nullptr;
  double* means = nullptr;
  double* wpart = nullptr;
  double* wstat = nullptr;
  int64_t t = 0;
  size_t plane = 0;
  lbm3_tile tile{1, 0, 0, 0};  // bulk steps: one per launch, or fuse per launch
};

namespace {

struct Layout3 {
  void* pop[2];
  void* f[3];
  double* f64[3];
  double* hist[2][4];
  double* mom[4];
  double *partials, *scalars, *terms, *aux, *sat, *means, *wpart, *wstat;
  size_t bytes;
};

int moment_blocks3(size_t plane) { return grid1(plane, 1024); }

Layout3 carve3(const lbm3_config& c, void* base, size_t cap) {
  Carver cv(base, cap);
  const size_t plane = static_cast<size_t>(c.nx) * c.ny * c.nz;
  const size_t es = c.dtype == LBM_F64 ? 8 : 4;
  Layout3 l{};
  const size_t q = c.lattice == LBM3_D3Q27 ? 27 : 19;
  for (int b = 0; b < 2; ++b) l.pop[b] = cv.take<char>(q * plane * es);
  if (c.has_force)
    for (int k = 0; k < 3; ++k) {
      l.f[k] = cv.take<char>(plane * es);
      l.f64[k] = cv.take<double>(plane);
    }
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 4; ++k) l.hist[s][k] = cv.take<double>(plane);
  for (int k = 0; k < 4; ++k) l.mom[k] = cv.take<double>(plane);
  l.partials = cv.take<double>(static_cast<size_t>(moment_blocks3(plane)) * kS3 + 8);
  l.scalars = cv.take<double>(8);
  if (c.with_balance) {
    const size_t vol = (static_cast<size_t>(c.nx) + 1) * (c.ny + 1) * (c.nz + 1);
    l.terms = cv.take<double>(NT3 * plane);
    l.aux = cv.take<double>(NA3 * plane);
    l.sat = cv.take<double>(NT3 * vol);
    l.means = cv.take<double>(16);
    l.wpart = cv.take<double>(std::max<size_t>(static_cast<size_t>(kW3MaxBlocks) * kW3Vals, NT3 * 512));
    l.wstat = cv.take<double>(static_cast<size_t>(kMaxSizes) * kW3Vals);
  }
  l.bytes = cv.used + 256;
  return l;
}

int validate3(const lbm3_config* c) {
  if (!c) return fail(LBM_E_INVALID, "config is NULL");
  if (c->nx < 16 || c->ny < 16 || c->nz < 16 || c->nx > 4096 || c->ny > 4096 || c->nz > 4096)
    return fail(LBM_E_INVALID, "3D grid %d x %d x %d outside [16, 4096]^3", c->nx, c->ny, c->nz);
  if (c->ny > 65535 || c->nz > 65535) return fail(LBM_E_INVALID, "grid too large");
  if (c->dtype != LBM_F32 && c->dtype != LBM_F64) return fail(LBM_E_INVALID, "dtype must be LBM_F32 or LBM_F64");
  if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return fail(LBM_E_INVALID, "tau must be a finite number > 0.5");
  if (c->has_force != 0 && c->has_force != 1) return fail(LBM_E_INVALID, "has_force must be 0 or 1");
  if (c->with_balance != 0 && c->with_balance != 1) return fail(LBM_E_INVALID, "with_balance must be 0 or 1");
  if (c->lattice != LBM3_D3Q19 && c->lattice != LBM3_D3Q27)
    return fail(LBM_E_INVALID, "lattice must be LBM3_D3Q19 or LBM3_D3Q27");
  return LBM_OK;
}

int launch3_step(lbm3_ctx_s* c, bool record) {
  Step3 p{};
  p.src = c->pop[c->cur];
  p.dst = c->pop[1 - c->cur];
  p.fx = c->f[0];
  p.fy = c->f[1];
  p.fz = c->f[2];
  const int slot = static_cast<int>(c->t & 1);
  if (record)
    for (int k = 0; k < 4; ++k) p.h[k] = c->hist[slot][k];
  p.nx = c->cfg.nx;
  p.ny = c->cfg.ny;
  p.nz = c->cfg.nz;
  p.omega = 1.0 / c->cfg.tau;
  const dim3 grid((p.nx + 255) / 256, p.ny, p.nz), block(256);
  const bool force = c->cfg.has_force != 0;
  auto go = [&](auto tag, auto q) {
    using T = decltype(tag);
    constexpr int Q = decltype(q)::value;
    if (force)
      hipLaunchKernelGGL((k3_step<T, true, Q>), grid, block, 0, c->stream, p);
    else
      hipLaunchKernelGGL((k3_step<T, false, Q>), grid, block, 0, c->stream, p);
  };
  using Q19 = std::integral_constant<int, 19>;
  using Q27 = std::integral_constant<int, 27>;
  if (c->cfg.dtype == LBM_F64) {
    if (c->q == 27) go(double{}, Q27{});
    else go(double{}, Q19{});
  } else {
    if (c->q == 27) go(float{}, Q27{});
    else go(float{}, Q19{});
  }
  LBM_HIP(hipGetLastError());
  if (record) c->hist_t[slot] = c->t;
  c->cur ^= 1;
  c->t += 1;
  return LBM_OK;
}

size_t fused3_lds_bytes(const lbm3_tile& t, int dtype) {
  return static_cast<size_t>(2) * 16 * t.bx * t.by * (dtype == LBM_F64 ? 8 : 4);
}

bool tile3_ok(const lbm3_tile& t, int dtype, int q) {
  if (t.fuse == 1) return true;
  if (q != 19) return false;  // the multi-step kernel is written for D3Q19
  if (t.fuse < 2 || t.fuse > 4) return false;
  const int lanes = t.bx * t.by;
  if (t.bx <= 2 * (t.fuse - 1) || t.by <= 2 * (t.fuse - 1) || t.bz < 1 || t.bz > 65536) return false;
  if (lanes < 64 || lanes > 512 || lanes % 64 != 0) return false;
  return fused3_lds_bytes(t, dtype) <= 64 * 1024;
}

template <typename T, int K, bool FORCE>
void launch_fused3_t(const Fused3& p, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k3_step_fused<T, K, FORCE>), dim3(p.total), dim3(p.bx * p.by), lds, s, p);
}

template <typename T, bool FORCE>
void launch_fused3_k(int K, const Fused3& p, size_t lds, hipStream_t s) {
  switch (K) {
    case 2: launch_fused3_t<T, 2, FORCE>(p, lds, s); break;
    case 3: launch_fused3_t<T, 3, FORCE>(p, lds, s); break;
    default: launch_fused3_t<T, 4, FORCE>(p, lds, s); break;
  }
}

// One launch of `tile.fuse` steps (no moment record).
int launch3_fused(lbm3_ctx_s* c, const lbm3_tile& tl) {
  const int K = tl.fuse;
  Fused3 p{};
  p.src = c->pop[c->cur];
  p.dst = c->pop[1 - c->cur];
  p.fx = c->f[0];
  p.fy = c->f[1];
  p.fz = c->f[2];
  p.nx = c->cfg.nx;
  p.ny = c->cfg.ny;
  p.nz = c->cfg.nz;
  p.bx = tl.bx;
  p.by = tl.by;
  p.bz = tl.bz;
  const int ox = tl.bx - 2 * (K - 1), oy = tl.by - 2 * (K - 1);
  p.tiles_x = (p.nx + ox - 1) / ox;
  p.tiles_y = (p.ny + oy - 1) / oy;
  const long long total = static_cast<long long>(p.tiles_x) * p.tiles_y * ((p.nz + tl.bz - 1) / tl.bz);
  if (total > 0x7fffffffLL) return fail(LBM_E_INVALID, "too many workgroups for this shape");
  p.total = static_cast<int>(total);
  p.omega = 1.0 / c->cfg.tau;
  const size_t lds = fused3_lds_bytes(tl, c->cfg.dtype);
  const bool force = c->cfg.has_force != 0;
  if (c->cfg.dtype == LBM_F64) {
    if (force) launch_fused3_k<double, true>(K, p, lds, c->stream);
    else launch_fused3_k<double, false>(K, p, lds, c->stream);
  } else {
    if (force) launch_fused3_k<float, true>(K, p, lds, c->stream);
    else launch_fused3_k<float, false>(K, p, lds, c->stream);
  }
  LBM_HIP(hipGetLastError());
  c->cur ^= 1;
  c->t += K;
  return LBM_OK;
}

int moments3(lbm3_ctx_s* c, double* r, double* u, double* v, double* w, double* scalars) {
  const size_t plane = c->plane;
  const int nb = moment_blocks3(plane);
  const int nx = c->cfg.nx, ny = c->cfg.ny, nz = c->cfg.nz;
  const bool force = c->cfg.has_force != 0;
  auto go = [&](auto tag, auto q) {
    using T = decltype(tag);
    constexpr int Q = decltype(q)::value;
    const T* pop = static_cast<const T*>(c->pop[c->cur]);
    if (force)
      hipLaunchKernelGGL((k3_moments<T, true, Q>), dim3(nb), dim3(kRedThreads), 0, c->stream, pop,
                         static_cast<const T*>(c->f[0]), static_cast<const T*>(c->f[1]),
                         static_cast<const T*>(c->f[2]), nx, ny, nz, r, u, v, w, c->partials);
    else
      hipLaunchKernelGGL((k3_moments<T, false, Q>), dim3(nb), dim3(kRedThreads), 0, c->stream, pop, nullptr,
                         nullptr, nullptr, nx, ny, nz, r, u, v, w, c->partials);
  };
  using Q19 = std::integral_constant<int, 19>;
  using Q27 = std::integral_constant<int, 27>;
  if (c->cfg.dtype == LBM_F64) {
    if (c->q == 27) go(double{}, Q27{});
    else go(double{}, Q19{});
  } else {
    if (c->q == 27) go(float{}, Q27{});
    else go(float{}, Q19{});
  }
  LBM_HIP(hipGetLastError());
  if (!scalars) return LBM_OK;
  hipLaunchKernelGGL(k3_reduce_scalars, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, nb, c->scalars);
  LBM_HIP(hipGetLastError());
  LBM_HIP(hipMemcpyAsync(scalars, c->scalars, kS3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LBM_HIP(hipStreamSynchronize(c->stream));
  scalars[8] = static_cast<double>(c->t);
  if (scalars[7] > 0.0 || !(scalars[6] > 0.0))
    return fail(LBM_E_DIVERGED, "3D run diverged: %.0f non-finite sites, min rho %g at step %lld", scalars[7],
                scalars[6], static_cast<long long>(c->t));
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm3_workspace_bytes(const lbm3_config* cfg, size_t* bytes) {
  if (int rc = validate3(cfg)) return rc;
  if (!bytes) return fail(LBM_E_INVALID, "bytes is NULL");
  *bytes = carve3(*cfg, nullptr, 0).bytes;
  return LBM_OK;
}

int lbm3_init(const lbm3_config* cfg, void* ws, size_t ws_bytes, const double* rho0, const double* ux0,
              const double* uy0, const double* uz0, const double* fx, const double* fy, const double* fz,
              lbm3_ctx* out) {
  if (int rc = validate3(cfg)) return rc;
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(LBM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (!rho0 || !ux0 || !uy0 || !uz0) return fail(LBM_E_INVALID, "initial fields must not be NULL");
  if (cfg->has_force && (!fx || !fy || !fz)) return fail(LBM_E_INVALID, "has_force = 1 needs fx, fy, fz");
  if (!cfg->has_force && (fx || fy || fz)) return fail(LBM_E_INVALID, "force given but has_force = 0");
  Layout3 l = carve3(*cfg, nullptr, 0);
  if (ws_bytes < l.bytes) return fail(LBM_E_NOMEM, "workspace %zu bytes < %zu required", ws_bytes, l.bytes);
  l = carve3(*cfg, ws, ws_bytes);
  lbm3_ctx_s* c = new lbm3_ctx_s();
  c->cfg = *cfg;
  c->q = cfg->lattice == LBM3_D3Q27 ? 27 : 19;
  c->stream = static_cast<hipStream_t>(cfg->stream);
  c->plane = static_cast<size_t>(cfg->nx) * cfg->ny * cfg->nz;
  for (int b = 0; b < 2; ++b) c->pop[b] = l.pop[b];
  for (int k = 0; k < 3; ++k) {
    c->f[k] = l.f[k];
    c->f64[k] = l.f64[k];
  }
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 4; ++k) c->hist[s][k] = l.hist[s][k];
  for (int k = 0; k < 4; ++k) c->mom[k] = l.mom[k];
  c->partials = l.partials;
  c->scalars = l.scalars;
  c->terms = l.terms;
  c->aux = l.aux;
  c->sat = l.sat;
  c->means = l.means;
  c->wpart = l.wpart;
  c->wstat = l.wstat;
  const int g = grid1(c->plane, 4096);
  if (cfg->dtype == LBM_F64) {
    if (c->q == 27)
      hipLaunchKernelGGL((k3_init<double, 27>), dim3(g), dim3(256), 0, c->stream, static_cast<double*>(c->pop[0]),
                         rho0, ux0, uy0, uz0, cfg->nx, cfg->ny, cfg->nz);
    else
      hipLaunchKernelGGL((k3_init<double, 19>), dim3(g), dim3(256), 0, c->stream, static_cast<double*>(c->pop[0]),
                         rho0, ux0, uy0, uz0, cfg->nx, cfg->ny, cfg->nz);
  } else {
    if (c->q == 27)
      hipLaunchKernelGGL((k3_init<float, 27>), dim3(g), dim3(256), 0, c->stream, static_cast<float*>(c->pop[0]),
                         rho0, ux0, uy0, uz0, cfg->nx, cfg->ny, cfg->nz);
    else
      hipLaunchKernelGGL((k3_init<float, 19>), dim3(g), dim3(256), 0, c->stream, static_cast<float*>(c->pop[0]),
                         rho0, ux0, uy0, uz0, cfg->nx, cfg->ny, cfg->nz);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && cfg->has_force) {
    const double* src[3] = {fx, fy, fz};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
      if (cfg->dtype == LBM_F64)
        hipLaunchKernelGGL(k3_to_storage<double>, dim3(g), dim3(256), 0, c->stream, static_cast<double*>(c->f[k]),
                           src[k], c->plane);
      else
        hipLaunchKernelGGL(k3_to_storage<float>, dim3(g), dim3(256), 0, c->stream, static_cast<float*>(c->f[k]),
                           src[k], c->plane);
      e = hipGetLastError();
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->f64[k], src[k], c->plane * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    }
  }
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "lbm3_init");
  }
  *out = c;
  return LBM_OK;
}

int lbm3_step(lbm3_ctx c, int64_t n) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(LBM_E_INVALID, "n must be >= 0");
  const int64_t nhist = n < 2 ? n : 2;
  const int64_t plain = n - nhist;
  const int K = c->tile.fuse;
  const int64_t bulk = K > 1 ? plain / K : 0;
  for (int64_t k = 0; k < bulk; ++k)
    if (int rc = launch3_fused(c, c->tile)) return rc;
  for (int64_t k = bulk * (K > 1 ? K : 1); k < n; ++k)
    if (int rc = launch3_step(c, k >= n - nhist)) return rc;
  return LBM_OK;
}

int lbm3_set_tile(lbm3_ctx c, const lbm3_tile* tile) {
  if (!c || !tile) return fail(LBM_E_INVALID, "NULL argument");
  if (!tile3_ok(*tile, c->cfg.dtype, c->q))
    return fail(LBM_E_INVALID, "3D shape (fuse %d, %d x %d lanes, band %d) not valid", tile->fuse, tile->bx,
                tile->by, tile->bz);
  c->tile = *tile;
  if (c->tile.fuse == 1) c->tile.bx = c->tile.by = c->tile.bz = 0;
  return LBM_OK;
}

int lbm3_get_tile(lbm3_ctx c, lbm3_tile* tile) {
  if (!c || !tile) return fail(LBM_E_INVALID, "NULL argument");
  *tile = c->tile;
  return LBM_OK;
}

int lbm3_autotune(lbm3_ctx c, int32_t trial_launches, lbm3_tile* chosen) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (trial_launches < 1 || trial_launches > 1000) return fail(LBM_E_INVALID, "trial_launches in [1, 1000]");
  std::vector<lbm3_tile> cand{{1, 0, 0, 0}};
  const int shapes[6][2] = {{64, 4}, {64, 8}, {32, 8}, {32, 16}, {128, 4}, {16, 16}};
  const int bands[3] = {16, 32, 64};
  for (int K = 2; K <= 4; ++K)
    for (auto& sh : shapes)
      for (int bz : bands) {
        lbm3_tile t{K, sh[0], sh[1], bz};
        if (tile3_ok(t, c->cfg.dtype, c->q) && (bz <= c->cfg.nz || bz == 16)) cand.push_back(t);
      }
  hipEvent_t e0, e1;
  LBM_HIP(hipEventCreate(&e0));
  LBM_HIP(hipEventCreate(&e1));
  const lbm3_tile saved = c->tile;
  const int cur = c->cur;
  const int64_t t0 = c->t;
  float best = 1e30f;
  lbm3_tile best_t = saved;
  int rc = LBM_OK;
  for (const auto& t : cand) {
    // src -> dst repeatedly: the state (src) is never modified
    auto one = [&]() {
      c->cur = cur;
      return t.fuse == 1 ? launch3_step(c, false) : launch3_fused(c, t);
    };
    if ((rc = one())) break;
    if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = fail(LBM_E_HIP, "hipEventRecord"); break; }
    for (int k = 0; k < trial_launches && rc == LBM_OK; ++k) rc = one();
    if (rc) break;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(LBM_E_HIP, "hipEventRecord/Synchronize");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= static_cast<float>(trial_launches * t.fuse);
    if (ms < best) {
      best = ms;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->cur = cur;
  c->t = t0;
  c->tile = rc == LBM_OK ? best_t : saved;
  if (rc) return rc;
  if (chosen) *chosen = best_t;
  return LBM_OK;
}

int lbm3_moments(lbm3_ctx c, double* rho, double* ux, double* uy, double* uz, double* scalars9) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  return moments3(c, rho, ux, uy, uz, scalars9);
}

int lbm3_time(lbm3_ctx c, int64_t* t) {
  if (!c || !t) return fail(LBM_E_INVALID, "NULL argument");
  *t = c->t;
  return LBM_OK;
}

int lbm3_subvolume_balance(lbm3_ctx c, const int32_t* sizes, int32_t nsizes, lbm_balance_stats* out,
                           double* term_fields) {
  if (!c) return fail(LBM_E_INVALID, "ctx is NULL");
  if (!c->cfg.with_balance) return fail(LBM_E_STATE, "handle was created with with_balance = 0");
  if (nsizes < 0 || nsizes > kMaxSizes) return fail(LBM_E_INVALID, "nsizes must be in [0, %d]", kMaxSizes);
  if (nsizes > 0 && (!sizes || !out)) return fail(LBM_E_INVALID, "sizes/out must not be NULL");
  const int nx = c->cfg.nx, ny = c->cfg.ny, nz = c->cfg.nz;
  const int m = std::min(nx, std::min(ny, nz));
  for (int k = 0; k < nsizes; ++k)
    if (sizes[k] < 1 || sizes[k] > m) return fail(LBM_E_INVALID, "box size %d outside [1, %d]", sizes[k], m);
  const int64_t t = c->t;
  if (t < 2 || c->hist_t[(t - 1) & 1] != t - 1 || c->hist_t[(t - 2) & 1] != t - 2)
    return fail(LBM_E_STATE, "balance at t = %lld needs the moments of steps t-1 and t-2",
                static_cast<long long>(t));
  double sc[9];
  if (int rc = moments3(c, c->mom[0], c->mom[1], c->mom[2], c->mom[3], sc)) return rc;
  hipStream_t s = c->stream;
  const size_t plane = c->plane;
  Bal3 a{};
  const int s2 = static_cast<int>((t - 2) & 1), s1 = static_cast<int>((t - 1) & 1);
  a.rho[0] = c->hist[s2][0];
  a.rho[1] = c->hist[s1][0];
  a.rho[2] = c->mom[0];
  for (int k = 0; k < 3; ++k) {
    a.u[0][k] = c->hist[s2][k + 1];
    a.u[1][k] = c->hist[s1][k + 1];
    a.u[2][k] = c->mom[k + 1];
    a.F[k] = c->cfg.has_force ? c->f64[k] : nullptr;
  }
  a.nu = (c->cfg.tau - 0.5) / 3.0;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.terms = c->terms;
  a.aux = c->aux;
  // the pass kernels' row runs, in per-plane XCD bands (see site3)
  const int chunk = (((nx + 255) / 256) * ny + 7) / 8;
  const dim3 grid(8 * chunk * nz), block(256);
  hipLaunchKernelGGL(k3_bal_a, grid, block, 0, s, a);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k3_bal_b, grid, block, 0, s, a);
  LBM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k3_bal_c, grid, block, 0, s, a);
  LBM_HIP(hipGetLastError());
  if (term_fields)
    LBM_HIP(hipMemcpyAsync(term_fields, c->terms, NT3 * plane * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (int rc = field_means(c->terms, NT3, nx, ny * nz, c->wpart, c->means, s)) return rc;
  Vol v{c->sat, c->means, nx, ny, nz};
  if (nx <= 256 * kXYChunks) {
    // x scans and y sums in one pass per plane (the faces are zeroed on their own)
    hipLaunchKernelGGL(k3_sat_xy, dim3(nz, NT3), dim3(256), 0, s, c->terms, v);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k3_sat_faces, dim3(grid1(v.sy() * NT3, 4096)), dim3(256), 0, s, v, NT3);
    LBM_HIP(hipGetLastError());
  } else {
    hipLaunchKernelGGL(k3_sat_x, dim3(ny, nz, NT3), dim3(256), 0, s, c->terms, v);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k3_sat_faces, dim3(grid1(v.sy() * NT3, 4096)), dim3(256), 0, s, v, NT3);
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k3_sat_y, dim3((nx + 1 + 255) / 256, nz, NT3), dim3(256), 0, s, v);
    LBM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k3_sat_z, dim3((nx + 1 + 255) / 256, ny + 1, NT3), dim3(256), 0, s, v);
  LBM_HIP(hipGetLastError());
  for (int k = 0; k < nsizes; ++k) {
    const int L = sizes[k];
    const size_t count = (L == nx && L == ny && L == nz) ? 1 : plane;
    // walks along z over 64 x 4 corner tiles, the residues of z mod L split over jg
    // workgroups per tile so the partials fit; the one whole-grid cube, and grids with more
    // tiles than partial slots, take the corner-by-corner kernel
    const int tx = (nx + 63) / 64, ty = (ny + 3) / 4;
    int nb;
    if (count > 1 && tx * ty <= kW3MaxBlocks) {
      const int jg = std::max(1, std::min(L, kW3MaxBlocks / (tx * ty)));
      nb = tx * ty * jg;
      hipLaunchKernelGGL(k3_windows_walk, dim3(((nb + 7) / 8) * 8), dim3(64, 4), 0, s, v, L, tx, ty, jg,
                         c->wpart);
    } else {
      nb = grid1(count, kW3MaxBlocks);
      hipLaunchKernelGGL(k3_windows, dim3(nb), dim3(kW3Threads), 0, s, v, L, count, c->wpart);
    }
    LBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k3_windows_final, dim3(1), dim3(256), 0, s, c->wpart, nb, c->wstat + k * kW3Vals);
    LBM_HIP(hipGetLastError());
  }
  std::vector<double> st(static_cast<size_t>(nsizes) * kW3Vals);
  if (nsizes > 0)
    LBM_HIP(hipMemcpyAsync(st.data(), c->wstat, st.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  LBM_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < nsizes; ++k) {
    lbm_balance_stats& o = out[k];
    o = lbm_balance_stats{};
    o.L = sizes[k];
    auto fill = [&](int q, int64_t& cnt, int64_t* nan, double& mean, double& sd, double& mn, double& mx) {
      const double* r = st.data() + static_cast<size_t>(k) * kW3Vals + q * 6;
      cnt = static_cast<int64_t>(r[0]);
      if (nan) *nan = static_cast<int64_t>(r[5]);
      if (cnt > 0) {
        mean = r[1];
        sd = std::sqrt(r[2] / r[0]);
        mn = r[3];
        mx = r[4];
      } else {
        mean = sd = mn = mx = NAN;
      }
    };
    fill(0, o.count_dE, &o.nan_dE, o.mean_dE, o.std_dE, o.min_dE, o.max_dE);
    fill(1, o.count_dZ, &o.nan_dZ, o.mean_dZ, o.std_dZ, o.min_dZ, o.max_dZ);
    fill(2, o.count_Ma, nullptr, o.mean_Ma, o.std_Ma, o.min_Ma, o.max_Ma);
  }
  return LBM_OK;
}

int lbm3_destroy(lbm3_ctx c) {
  if (!c) return LBM_OK;
  (void)hipStreamSynchronize(c->stream);
  delete c;
  return LBM_OK;
}

}  // extern "C"
