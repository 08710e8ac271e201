// Shared device-side definitions of the EnVar HIP library (gfx950).
//
// Grid: the open-cavity MAC grid of Sec. 2 (channel over a square cavity),
// one bounding box of nx x ny cells per multigrid level. The fluid predicate,
// the face classes and every boundary rule below are derived from it
// arithmetically, so no geometry table is read by the hot kernels.
//
// Memory: every per-member field is a "plane" of `rows` x `pitch` elements,
// row-major with x fastest (pitch a multiple of 16 elements, so rows start
// 128-byte aligned); members are stacked plane after plane (ensemble-major).
// u faces use (i, j) for 0 <= i <= nx, 0 <= j < ny; v faces 0 <= i < nx,
// 0 <= j <= ny; cell fields 0 <= i < nx, 0 <= j < ny.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace envar {

// Tiles of the stencil kernels: 64 cells (one wave) wide.
constexpr int TILE_W = 64;
constexpr int COST_TH = 8;   // rows of a cost block: the S2 partial sums live on a fixed 64 x 8 grid
// Red-black sweeps before and after the coarse correction, by the V-cycle's element type:
// two for FP64 V-cycles, one for the FP32 V-cycles inside FP64 refinement (mixed precision).
// Measured at h = 1/128, 65 members, 20,000 steps: mixed 9.28e9 cell-steps/s with two sweeps
// (1.25 refinement passes per step) -> 1.05e10 with one (1.30 passes, each cheaper, and a
// wider tile); FP64 6.52e9 with two (2.09 V-cycles per step) -> 5.92e9 with one (3.11).
template <typename T>
__host__ __device__ constexpr int mg_ns() { return sizeof(T) == sizeof(float) ? 1 : 2; }
// window halo of the multigrid kernels: a sweep invalidates two rings, the residual one more
template <typename T>
__host__ __device__ constexpr int mg_h() { return 2 * mg_ns<T>() + 1; }
// multigrid tile width: the window is one wave wide
template <typename T>
__host__ __device__ constexpr int mg_tw() { return 64 - 2 * mg_h<T>(); }
// relaxation of the red-black sweeps on the tiled levels, by the V-cycle's element type, measured at
// h = 1/128 with 65 members (the LDS levels keep 1):
//  * FP64 V(2,2): V-cycles per step 3.04 (omega = 1) -> 2.06 (1.15) -> 3.05 (1.3);
//  * FP32 V(1,1) inside FP64 refinement, 6,000 steps: refinement passes per step 1.398 (0.9),
//    1.381 (0.95), 1.363 (1), 1.369 (1.05), 1.510 (1.15), 1.619 (1.25); cell-steps/s best at 1.
template <typename T>
__host__ __device__ constexpr double mg_omega() { return sizeof(T) == sizeof(float) ? 1.0 : 1.15; }
constexpr int COARSE_N = 16; // levels with inv_h <= 16 run inside one workgroup per member
constexpr int MAX_LEVELS = 12;
constexpr int MAX_COARSE_UNKNOWNS = 128;
constexpr int COARSE_INV_MAX = 8192;  // bound on the coarsest inverse (nc^2 doubles, read from global memory)

struct Geo {
  int nx, ny;    // bounding box in cells
  int jc;        // rows j >= jc are full channel rows
  int ic0, ic1;  // rows j < jc are fluid only for ic0 <= i < ic1
  int pitch;     // elements per row
  int rows;      // rows per plane
  int n;         // cells per unit length at this level
  double h;
  // momentum boundary kinds (finest level): slip top wall, slip lower channel wall for u faces
  // i <= slip_i0 or i >= slip_i1, convective outflow speed (the inflow's bulk speed)
  int slip_top, slip_i0, slip_i1;
  double uconv;

  __host__ __device__ __forceinline__ long plane() const { return (long)pitch * rows; }
  __host__ __device__ __forceinline__ long at(int i, int j) const { return (long)j * pitch + i; }
  __host__ __device__ __forceinline__ bool fluid(int i, int j) const {
    if (i < 0 || i >= nx || j < 0 || j >= ny) return false;
    return j >= jc || (i >= ic0 && i < ic1);
  }
  // u face (i, j) lies between cells (i-1, j) and (i, j)
  __host__ __device__ __forceinline__ bool u_solid(int i, int j) const {
    return !(fluid(i - 1, j) || fluid(i, j));
  }
  // v face (i, j) lies between cells (i, j-1) and (i, j)
  __host__ __device__ __forceinline__ bool v_solid(int i, int j) const {
    return !(fluid(i, j - 1) || fluid(i, j));
  }
  // sign of the mirrored u across the SOLID u face (i, jn) next to an active face: -1 no-slip
  // (u = 0 half a cell away), +1 slip (du/dy = 0)
  __host__ __device__ __forceinline__ double u_wall_sign(int i, int jn) const {
    if (jn >= ny) return slip_top ? 1.0 : -1.0;
    if (jn == jc - 1 && (i <= slip_i0 || i >= slip_i1)) return 1.0;
    return -1.0;
  }
  // number of Poisson neighbours (+2 for the Dirichlet outflow face)
  __host__ __device__ __forceinline__ int diag_count(int i, int j) const {
    return (int)fluid(i - 1, j) + (int)fluid(i + 1, j) + (int)fluid(i, j - 1) + (int)fluid(i, j + 1) +
           (i == nx - 1 ? 2 : 0);
  }
  __host__ __device__ Geo coarser() const {
    Geo c = *this;
    c.nx = nx / 2;
    c.ny = ny / 2;
    c.jc = jc / 2;
    c.ic0 = ic0 / 2;
    c.ic1 = ic1 / 2;
    c.n = n / 2;
    c.h = 2.0 * h;
    c.pitch = ((c.nx + 1 + 15) / 16) * 16;
    c.rows = c.ny + 1;
    return c;
  }
};

// Tiling of the fluid part of the box into TW x TH tiles: first the cavity tile
// rows (only the tile columns that meet the cavity), then full channel rows.
struct Tiling {
  int cav_c0, cav_cols, cav_rows, ch_cols, ch_rows, th, jc_tiles, tw;
  __host__ __device__ static Tiling make(const Geo& g, int th, int tw = TILE_W) {
    Tiling t;
    t.th = th;
    t.tw = tw;
    if (g.jc % th == 0 && g.ic1 > g.ic0) {
      t.cav_c0 = g.ic0 / tw;
      t.cav_cols = (g.ic1 - 1) / tw - t.cav_c0 + 1;
      t.cav_rows = g.jc / th;
      t.jc_tiles = g.jc;
    } else {
      t.cav_c0 = 0;
      t.cav_cols = 0;
      t.cav_rows = 0;
      t.jc_tiles = 0;
    }
    t.ch_cols = (g.nx + tw - 1) / tw;
    t.ch_rows = (g.ny - t.jc_tiles + th - 1) / th;
    return t;
  }
  __host__ __device__ int count() const { return cav_cols * cav_rows + ch_cols * ch_rows; }
  // index of the tile whose origin is (x0, y0) (the inverse of origin())
  __device__ __forceinline__ int index(int x0, int y0) const {
    if (y0 < jc_tiles) return (y0 / th) * cav_cols + (x0 / tw - cav_c0);
    return cav_cols * cav_rows + ((y0 - jc_tiles) / th) * ch_cols + x0 / tw;
  }
  __device__ __forceinline__ void origin(int t, int& x0, int& y0) const {
    int ncav = cav_cols * cav_rows;
    if (t < ncav) {
      y0 = (t / cav_cols) * th;
      x0 = (cav_c0 + t % cav_cols) * tw;
    } else {
      t -= ncav;
      y0 = jc_tiles + (t / ch_cols) * th;
      x0 = (t % ch_cols) * tw;
    }
  }
};

// Workgroups are dealt round-robin to the 8 XCDs; remap the flat workgroup id
// so that each XCD receives one contiguous range of (member, tile) items and
// neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int wg, int total) {
  const int q = total / 8;
  if (wg >= 8 * q) return wg;
  return (wg % 8) * q + wg / 8;
}

// Order-preserving bit pattern of a non-negative double for atomicMax.
__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = (w > v || w != w) ? w : v;  // NaN propagates
  }
  return v;
}

}  // namespace envar
