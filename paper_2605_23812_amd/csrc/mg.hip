// Batched masked geometric multigrid for the pressure Poisson equation
//   L_h phi = b,  L_h phi_c = (sum over fluid neighbours (phi_nb - phi_c) - 2 phi_c [outflow face]) / h^2
// on the channel-plus-cavity mask: homogeneous Neumann on walls and inflow,
// phi = 0 on the outflow face (mirror ghost -phi). The geometry is aligned on
// every level down to h = 1/4, so each coarse cell has four fluid children.
//
// Per fine level and V-cycle two launches, both over (member, 64 x 16 tile):
//   pre : load phi, b with a halo of 2 NS + 1 into LDS, NS red-black
//         Gauss-Seidel sweeps (temporal blocking: a sweep invalidates two
//         halo rings), residual r = b - L phi, restriction b_c = mean of the
//         four children; writes phi and b_c.
//   post: load phi, b with a halo of 2 NS (+1), add the bilinearly
//         prolongated coarse correction (Neumann mirror at walls, sign flip
//         across the outflow face), NS sweeps, optionally the per-member
//         max-norm of dt r (wave reductions + atomicMax); writes phi (or adds
//         it to the FP64 pressure in iterative refinement).
// Levels with inv_h <= 16 (at most 2048 box cells) run inside one workgroup
// per member with every level resident in LDS, ending in a dense FP64 solve
// of the h = 1/4 operator through its precomputed inverse.
// Members whose previous cycle met the tolerance exit at once (per-member
// convergence: a member's result never depends on the rest of the batch).
#include "common.h"
#include "kernels.h"

namespace envar {

template <typename T>
__device__ __forceinline__ T inv_diag(int d) {
  // d in 1..6
  return d == 4 ? (T)0.25 : d == 3 ? (T)(1.0 / 3.0) : d == 2 ? (T)0.5 : d == 5 ? (T)0.2 : d == 6 ? (T)(1.0 / 6.0) : (T)1;
}

// One red-black sweep on an LDS window (LW x LH) whose origin is (ox, oy) in
// level coordinates; the outermost ring is never updated. Non-fluid entries
// hold 0 and stay 0.
template <typename T, int LW, int LH>
__device__ __forceinline__ void rb_sweep(T* sp, const T* sb, const Geo& g, int ox, int oy, T h2) {
  for (int color = 0; color < 2; ++color) {
    for (int q = threadIdx.x; q < LH * (LW / 2); q += blockDim.x) {
      const int r = q / (LW / 2);
      const int c = 2 * (q % (LW / 2)) + ((color ^ r ^ ox ^ oy) & 1);
      if (r == 0 || r == LH - 1 || c == 0 || c == LW - 1) continue;
      const int i = ox + c, j = oy + r;
      if (!g.fluid(i, j)) continue;
      const int k = r * LW + c;
      const T s = (sp[k - 1] + sp[k + 1]) + (sp[k - LW] + sp[k + LW]);
      sp[k] = (s - h2 * sb[k]) * inv_diag<T>(g.diag_count(i, j));
    }
    __syncthreads();
  }
}

template <typename T, int LW>
__device__ __forceinline__ T resid_at(const T* sp, const T* sb, const Geo& g, int i, int j, int k, T inv_h2) {
  const T s = (sp[k - 1] + sp[k + 1]) + (sp[k - LW] + sp[k + LW]);
  return sb[k] - (s - (T)g.diag_count(i, j) * sp[k]) * inv_h2;
}

template <typename T>
__device__ __forceinline__ bool mg_skip(const MGArgs<T>& a, int mem, int tile) {
  if (a.k <= 0 || a.norms == nullptr) return false;
  const double prev = a.norms[(long)mem * a.norm_slots + a.k - 1];
  if (prev <= a.tol) {
    if (a.write_norm && tile == 0 && threadIdx.x == 0) a.norms[(long)mem * a.norm_slots + a.k] = prev;
    return true;
  }
  return false;
}

// ---------------------------------------------------------------------------- pre-smoothing + restriction
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_mg_pre(MGArgs<T> a) {
  constexpr int TW = TILE_W, TH = MG_TH, H = 2 * NS + 1;
  constexpr int LW = TW + 2 * H, LH = TH + 2 * H;
  __shared__ T sp[LH * LW];
  __shared__ T sb[LH * LW];
  const Geo& g = a.g;
  const int item = xcd_remap(blockIdx.x, a.ntiles * a.nmem);
  const int mem = item / a.ntiles, tile = item % a.ntiles;
  if (mg_skip(a, mem, tile)) return;
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const int ox = x0 - H, oy = y0 - H;
  const long off = (long)mem * a.plane;
  for (int k = threadIdx.x; k < LH * LW; k += 256) {
    const int i = ox + k % LW, j = oy + k / LW;
    const bool fl = g.fluid(i, j);
    sp[k] = (fl && !a.zero_guess) ? a.phi_in[off + g.at(i, j)] : (T)0;
    sb[k] = fl ? a.b[off + g.at(i, j)] : (T)0;
  }
  __syncthreads();
  const T h2 = (T)(g.h * g.h), inv_h2 = (T)(1.0 / (g.h * g.h));
  for (int s = 0; s < NS; ++s) rb_sweep<T, LW, LH>(sp, sb, g, ox, oy, h2);
  // restriction: one coarse cell per thread (32 x 8 per tile)
  {
    const Geo& gc = a.gc;
    const int ci = threadIdx.x % (TW / 2), cj = threadIdx.x / (TW / 2);
    const int I = x0 / 2 + ci, J = y0 / 2 + cj;
    if (gc.fluid(I, J)) {
      T rs = 0;
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
          const int c = H + 2 * ci + di, r = H + 2 * cj + dj;
          rs += resid_at<T, LW>(sp, sb, g, ox + c, oy + r, r * LW + c, inv_h2);
        }
      a.bc[(long)mem * a.cplane_c + gc.at(I, J)] = (T)0.25 * rs;
    }
  }
  for (int k = threadIdx.x; k < TW * TH; k += 256) {
    const int c = H + k % TW, r = H + k / TW;
    const int i = ox + c, j = oy + r;
    if (g.fluid(i, j)) a.phi_out[off + g.at(i, j)] = sp[r * LW + c];
  }
}

// ---------------------------------------------------------------------------- prolongation + post-smoothing
template <typename T, int NS, int NORM>
__global__ __launch_bounds__(256) void k_mg_post(MGArgs<T> a) {
  constexpr int TW = TILE_W, TH = MG_TH, H = 2 * NS + NORM;
  constexpr int LW = TW + 2 * H, LH = TH + 2 * H;
  __shared__ T sp[LH * LW];
  __shared__ T sb[LH * LW];
  __shared__ double red[4];
  const Geo& g = a.g;
  const Geo& gc = a.gc;
  const int item = xcd_remap(blockIdx.x, a.ntiles * a.nmem);
  const int mem = item / a.ntiles, tile = item % a.ntiles;
  if (mg_skip(a, mem, tile)) return;
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const int ox = x0 - H, oy = y0 - H;
  const long off = (long)mem * a.plane;
  const T* __restrict__ pc = a.phic + (long)mem * a.cplane_c;
  for (int k = threadIdx.x; k < LH * LW; k += 256) {
    const int i = ox + k % LW, j = oy + k / LW;
    T p = 0, bb = 0;
    if (g.fluid(i, j)) {
      const long at = g.at(i, j);
      bb = a.b[off + at];
      // bilinear prolongation of the coarse correction
      const int I = i >> 1, J = j >> 1;
      const int IX = I + ((i & 1) ? 1 : -1), JY = J + ((j & 1) ? 1 : -1);
      const T P = pc[gc.at(I, J)];
      const T X = gc.fluid(IX, J) ? pc[gc.at(IX, J)] : (IX == gc.nx ? -P : P);
      const T Y = gc.fluid(I, JY) ? pc[gc.at(I, JY)] : P;
      const T D = gc.fluid(IX, JY) ? pc[gc.at(IX, JY)] : X + Y - P;
      p = a.phi_in[off + at] + ((T)9 * P + (T)3 * (X + Y) + D) * (T)0.0625;
    }
    sp[k] = p;
    sb[k] = bb;
  }
  __syncthreads();
  const T h2 = (T)(g.h * g.h), inv_h2 = (T)(1.0 / (g.h * g.h));
  for (int s = 0; s < NS; ++s) rb_sweep<T, LW, LH>(sp, sb, g, ox, oy, h2);
  if (NORM && a.write_norm) {
    double m = 0.0;
    for (int k = threadIdx.x; k < TW * TH; k += 256) {
      const int c = H + k % TW, r = H + k / TW;
      const int i = ox + c, j = oy + r;
      if (g.fluid(i, j)) {
        const double rr = fabs((double)resid_at<T, LW>(sp, sb, g, i, j, r * LW + c, inv_h2)) * a.dt;
        m = (rr > m || rr != rr) ? rr : m;
      }
    }
    m = wave_max(m);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = red[0];
      for (int w = 1; w < 4; ++w) mm = (red[w] > mm || red[w] != red[w]) ? red[w] : mm;
      atomicMax((unsigned long long*)&a.norms[(long)mem * a.norm_slots + a.k], dbits(mm));
    }
  }
  for (int k = threadIdx.x; k < TW * TH; k += 256) {
    const int c = H + k % TW, r = H + k / TW;
    const int i = ox + c, j = oy + r;
    if (g.fluid(i, j)) {
      if (a.add_to)
        a.add_to[off + g.at(i, j)] += (double)sp[r * LW + c];
      else
        a.phi_out[off + g.at(i, j)] = sp[r * LW + c];
    }
  }
}

// ---------------------------------------------------------------------------- coarse levels in LDS
constexpr int COARSE_LDS = 2 * (64 * 32 + 32 * 16 + 16 * 8);

__device__ __forceinline__ void lds_sweep(double* p, const double* b, const Geo& g, double h2) {
  const int nx = g.nx, ncell = g.nx * g.ny;
  for (int color = 0; color < 2; ++color) {
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
      const int i = q % nx, j = q / nx;
      if (((i + j) & 1) != color || !g.fluid(i, j)) continue;
      double s = 0.0;
      if (g.fluid(i - 1, j)) s += p[q - 1];
      if (g.fluid(i + 1, j)) s += p[q + 1];
      if (g.fluid(i, j - 1)) s += p[q - nx];
      if (g.fluid(i, j + 1)) s += p[q + nx];
      p[q] = (s - h2 * b[q]) / (double)g.diag_count(i, j);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double lds_resid(const double* p, const double* b, const Geo& g, int i, int j, double inv_h2) {
  const int nx = g.nx, q = j * nx + i;
  double s = 0.0;
  if (g.fluid(i - 1, j)) s += p[q - 1];
  if (g.fluid(i + 1, j)) s += p[q + 1];
  if (g.fluid(i, j - 1)) s += p[q - nx];
  if (g.fluid(i, j + 1)) s += p[q + nx];
  return b[q] - (s - (double)g.diag_count(i, j) * p[q]) * inv_h2;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mg_coarse(CoarseArgs a) {
  __shared__ double lds[COARSE_LDS];
  __shared__ double red[4];
  const int mem = blockIdx.x;
  if (a.k > 0 && a.norms != nullptr) {
    const double prev = a.norms[(long)mem * a.norm_slots + a.k - 1];
    if (prev <= a.tol) {
      if (a.write_norm && threadIdx.x == 0) a.norms[(long)mem * a.norm_slots + a.k] = prev;
      return;
    }
  }
  Geo gl[6];
  double* P[6];
  double* B[6];
  gl[0] = a.g;
  int offs = 0;
  for (int l = 0; l < a.nlev; ++l) {
    if (l > 0) gl[l] = gl[l - 1].coarser();
    const int nc = gl[l].nx * gl[l].ny;
    P[l] = lds + offs;
    B[l] = lds + offs + nc;
    offs += 2 * nc;
  }
  const long off = (long)mem * a.plane;
  const T* gphi = (const T*)a.phi + off;
  const T* gb = (const T*)a.b + off;
  {
    const Geo& g = gl[0];
    for (int q = threadIdx.x; q < g.nx * g.ny; q += 256) {
      const int i = q % g.nx, j = q / g.nx;
      const bool fl = g.fluid(i, j);
      P[0][q] = (fl && a.warm) ? (double)gphi[g.at(i, j)] : 0.0;
      B[0][q] = fl ? (double)gb[g.at(i, j)] : 0.0;
    }
  }
  __syncthreads();
  const int L = a.nlev - 1;
  for (int l = 0; l < L; ++l) {
    const Geo& g = gl[l];
    const double h2 = g.h * g.h, inv_h2 = 1.0 / h2;
    for (int s = 0; s < a.nsweep_pre; ++s) lds_sweep(P[l], B[l], g, h2);
    const Geo& c = gl[l + 1];
    for (int q = threadIdx.x; q < c.nx * c.ny; q += 256) {
      const int I = q % c.nx, J = q / c.nx;
      double rs = 0.0;
      if (c.fluid(I, J))
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) rs += lds_resid(P[l], B[l], g, 2 * I + di, 2 * J + dj, inv_h2);
      B[l + 1][q] = 0.25 * rs;
      P[l + 1][q] = 0.0;
    }
    __syncthreads();
  }
  // dense solve on the coarsest level
  {
    const Geo& g = gl[L];
    for (int q = threadIdx.x; q < a.nc; q += 256) {
      double s = 0.0;
      for (int r = 0; r < a.nc; ++r) s += a.ainv[(long)q * a.nc + r] * B[L][a.aidx[r]];
      P[L][a.aidx[q]] = s;
    }
    (void)g;
    __syncthreads();
  }
  for (int l = L - 1; l >= 0; --l) {
    const Geo& g = gl[l];
    const Geo& c = gl[l + 1];
    for (int q = threadIdx.x; q < g.nx * g.ny; q += 256) {
      const int i = q % g.nx, j = q / g.nx;
      if (!g.fluid(i, j)) continue;
      const int I = i >> 1, J = j >> 1;
      const int IX = I + ((i & 1) ? 1 : -1), JY = J + ((j & 1) ? 1 : -1);
      const double* pc = P[l + 1];
      const double Pv = pc[J * c.nx + I];
      const double X = c.fluid(IX, J) ? pc[J * c.nx + IX] : (IX == c.nx ? -Pv : Pv);
      const double Y = c.fluid(I, JY) ? pc[JY * c.nx + I] : Pv;
      const double D = c.fluid(IX, JY) ? pc[JY * c.nx + IX] : X + Y - Pv;
      P[l][q] += (9.0 * Pv + 3.0 * (X + Y) + D) * 0.0625;
    }
    __syncthreads();
    const double h2 = g.h * g.h;
    for (int s = 0; s < a.nsweep_post; ++s) lds_sweep(P[l], B[l], g, h2);
  }
  const Geo& g = gl[0];
  if (a.write_norm) {
    const double inv_h2 = 1.0 / (g.h * g.h);
    double m = 0.0;
    for (int q = threadIdx.x; q < g.nx * g.ny; q += 256) {
      const int i = q % g.nx, j = q / g.nx;
      if (g.fluid(i, j)) {
        const double rr = fabs(lds_resid(P[0], B[0], g, i, j, inv_h2)) * a.dt;
        m = (rr > m || rr != rr) ? rr : m;
      }
    }
    m = wave_max(m);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = red[0];
      for (int w = 1; w < 4; ++w) mm = (red[w] > mm || red[w] != red[w]) ? red[w] : mm;
      a.norms[(long)mem * a.norm_slots + a.k] = mm;
    }
  }
  T* wphi = (T*)a.phi + off;
  for (int q = threadIdx.x; q < g.nx * g.ny; q += 256) {
    const int i = q % g.nx, j = q / g.nx;
    if (!g.fluid(i, j)) continue;
    if (a.add_to)
      a.add_to[off + g.at(i, j)] += P[0][q];
    else
      wphi[g.at(i, j)] = (T)P[0][q];
  }
}

// ---------------------------------------------------------------------------- FP64 residual (refinement)
__global__ __launch_bounds__(256) void k_resid64(ResidArgs a) {
  constexpr int TW = TILE_W, TH = STEP_TH;
  __shared__ double red[4];
  const Geo& g = a.g;
  const int item = xcd_remap(blockIdx.x, a.ntiles * a.nmem);
  const int mem = item / a.ntiles, tile = item % a.ntiles;
  if (a.k > 0) {
    const double prev = a.norms[(long)mem * a.norm_slots + a.k - 1];
    if (prev <= a.tol) {
      if (tile == 0 && threadIdx.x == 0) a.norms[(long)mem * a.norm_slots + a.k] = prev;
      return;
    }
  }
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const long off = (long)mem * a.plane;
  const double* __restrict__ phi = a.phi + off;
  const double inv_h2 = 1.0 / (g.h * g.h);
  const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
  double m = 0.0;
  for (int r = ty; r < TH; r += 4) {
    const int i = x0 + tx, j = y0 + r;
    if (!g.fluid(i, j)) continue;
    const long at = g.at(i, j);
    const double p = phi[at];
    double s = 0.0;
    if (g.fluid(i - 1, j)) s += phi[at - 1];
    if (g.fluid(i + 1, j)) s += phi[at + 1];
    if (g.fluid(i, j - 1)) s += phi[at - g.pitch];
    if (g.fluid(i, j + 1)) s += phi[at + g.pitch];
    const double rr = a.b[off + at] - (s - (double)g.diag_count(i, j) * p) * inv_h2;
    a.r[off + at] = (float)rr;
    const double ar = fabs(rr) * a.dt;
    m = (ar > m || ar != ar) ? ar : m;
  }
  m = wave_max(m);
  if (tx == 0) red[ty] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = red[0];
    for (int w = 1; w < 4; ++w) mm = (red[w] > mm || red[w] != red[w]) ? red[w] : mm;
    atomicMax((unsigned long long*)&a.norms[(long)mem * a.norm_slots + a.k], dbits(mm));
  }
}

// ---------------------------------------------------------------------------- launchers
template <typename T>
void launch_mg_pre(const MGArgs<T>& a, int nsweep, hipStream_t s) {
  const dim3 grid(a.ntiles * a.nmem), block(256);
  switch (nsweep) {
    case 1: hipLaunchKernelGGL((k_mg_pre<T, 1>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_mg_pre<T, 3>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_mg_pre<T, 2>), grid, block, 0, s, a); break;
  }
}
template <typename T>
void launch_mg_post(const MGArgs<T>& a, int nsweep, hipStream_t s) {
  const dim3 grid(a.ntiles * a.nmem), block(256);
  if (a.write_norm) {
    switch (nsweep) {
      case 1: hipLaunchKernelGGL((k_mg_post<T, 1, 1>), grid, block, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_mg_post<T, 3, 1>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_mg_post<T, 2, 1>), grid, block, 0, s, a); break;
    }
  } else {
    switch (nsweep) {
      case 1: hipLaunchKernelGGL((k_mg_post<T, 1, 0>), grid, block, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_mg_post<T, 3, 0>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_mg_post<T, 2, 0>), grid, block, 0, s, a); break;
    }
  }
}
template <typename T>
void launch_mg_coarse(const CoarseArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_coarse<T>, dim3(a.nmem), dim3(256), 0, s, a);
}
void launch_resid64(const ResidArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_resid64, dim3(a.ntiles * a.nmem), dim3(256), 0, s, a);
}

template void launch_mg_pre<double>(const MGArgs<double>&, int, hipStream_t);
template void launch_mg_pre<float>(const MGArgs<float>&, int, hipStream_t);
template void launch_mg_post<double>(const MGArgs<double>&, int, hipStream_t);
template void launch_mg_post<float>(const MGArgs<float>&, int, hipStream_t);
template void launch_mg_coarse<double>(const CoarseArgs&, hipStream_t);
template void launch_mg_coarse<float>(const CoarseArgs&, hipStream_t);

}  // namespace envar
