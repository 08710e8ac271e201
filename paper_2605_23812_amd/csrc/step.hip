// Time-step kernels: fused predictor (advection + diffusion + forcing + AB2 +
// convective outflow + Poisson right-hand side), projection fused with the
// on-the-fly cost accumulator, per-step convergence bookkeeping, and the
// final cost reduction.
//
// Discretisation of eq. (forced_NS) / eq. (discrete_NS) on the MAC grid:
//   T^n   = -div_h(u u) + nu lap_h u           (conservative central form, active faces)
//   u*    = u^n + dt (3/2 T^n - 1/2 T^{n-1} + F),  F = P f (face mean of the cell forcing)
//   u*_b  = u^n_b - dt U_c (u^n_b - u^n_{b-1}) / h   (outflow faces)
//   b     = div_h u* / dt                      (Poisson right-hand side)
//   u^{n+1} = u* - dt grad_h phi               (active and outflow faces; phi = 0 on the outflow face)
// Neighbour rules: a wall face holds 0, a face with no fluid cell on either
// side mirrors the own value (no-slip wall half a cell away; without the sign
// flip across a slip wall), the v value
// west of the inflow mirrors (v = 0 at the inlet) and east of the outflow
// copies (zero normal gradient of v at the outlet).
//
// Cost (eq. Envarcost with the fluctuation energy of eq. kinenergy): per cell
// S1_c += (u_c - s_c) and per tile S2 += sum |u_c - s_c|^2 with the shift s =
// the base-state cell velocity; at the end J_obs = dt h^2 (S2 - sum_c |S1_c|^2 / K).
#include "common.h"
#include "kernels.h"

namespace envar {

// ---------------------------------------------------------------------------- predictor
// FUSED: the projection of the previous step runs here first. The halo of
// u^n = u*^{n-1} - dt grad phi^{n-1} is rebuilt in LDS from u*, v* and phi
// (with the same expressions as k_project_cost, so every value is bitwise the
// same), and the tile cells take the previous step's cost sample, divergence
// and the warm start of this step's solve. u^n never goes to memory: the step
// carries u* and phi, which saves the u, v store and reload and a launch.
// CUBIC: the fused warm start extrapolates from a third history plane (FP64 jobs); the mixed
// instance is compiled without it, so it carries none of its registers
template <typename TT, bool ONE, int TH, bool FUSED, bool CUBIC>
__global__ __launch_bounds__(256) void k_predictor(Multi<PredArgs<TT>> ms) {
  constexpr int TW = TILE_W;
  constexpr int UW = TW + 3, UH = TH + 2;  // u halo: i in [x0-1, x0+TW+1], j in [y0-1, y0+TH]
  constexpr int VW = TW + 2, VH = TH + 3;  // v halo: i in [x0-1, x0+TW],   j in [y0-1, y0+TH+1]
  constexpr int PW = TW + 4, PH = TH + 4;  // phi halo (fused): i in [x0-2, x0+TW+1], j in [y0-2, y0+TH+1]
  constexpr int NB = TH / COST_TH;
  static_assert(TH % COST_TH == 0 && COST_TH == 8, "cost blocks are 64 x 8 (two rows per thread)");
  __shared__ double su[UH * UW];
  __shared__ double sv[VH * VW];
  __shared__ double sus[TH * (TW + 1)];
  __shared__ double svs[(TH + 1) * TW];
  __shared__ double sphi[FUSED ? PH * PW : 1];
  __shared__ double red_s[NB][4];
  __shared__ double red_m[4];

  int item;
  const PredArgs<TT>& a = ms.template pick<ONE>(xcd_remap(blockIdx.x, gridDim.x), item);
  const Geo& g = a.g;
  const int mem = item / a.ntiles;
  const int tile = item % a.ntiles;
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const long off = (long)mem * a.plane;
  const double* __restrict__ u = a.u + off;
  const double* __restrict__ v = a.v + off;
  const TT* __restrict__ tup = a.tu_prev + off;
  const TT* __restrict__ tvp = a.tv_prev + off;
  const double* __restrict__ f = a.ctrl ? a.ctrl + (long)mem * a.m : nullptr;
  const int tid = threadIdx.x;
  double* const phi_old2 = CUBIC ? a.phi_old2 : nullptr;

  if (tile == 0 && a.norms != nullptr)
    for (int k = tid; k < a.norm_slots; k += 256) a.norms[(long)mem * a.norm_slots + k] = 0.0;

  // Every global operand of the tile besides the halo is loaded into registers
  // right after the halo loads, so its latency overlaps the LDS phases.
  constexpr int KU = (TH * (TW + 1) + 255) / 256, KV = ((TH + 1) * TW + 255) / 256, KR = TH / 4;
  const bool cold = a.cold_flag != nullptr && *a.cold_flag != 0;
  const int tx = tid % TW, ty = tid / TW;
  const long coff = (long)mem * a.cplane;
  TT tpu[KU], tpv[KV];         // T^{n-1} of this thread's active faces
  int cmu[KU][2], cmv[KV][2];  // control index of the two cells of each face (-1: none)
  // fused: the per-member operands of the tile cells. The cost shift (base-state cell velocity) is
  // one plane shared by every member and stays in L2, so it is read where it is used: holding it
  // here took 8 more VGPRs, which cut the predictor to 4 waves per SIMD (5 without; 207 -> 189 us
  // per launch at h = 1/128 with 65 members)
  double pn[KR], po[KR], pr[KR], s1a[KR], s1b[KR];
  {
    // all global loads of the halo first, then the LDS stores
    constexpr int NU = (UH * UW + 255) / 256, NV = (VH * VW + 255) / 256;
    double lu[NU], lv[NV];
#pragma unroll
    for (int n = 0; n < NU; ++n) {
      const int k = tid + 256 * n;
      const int i = x0 - 1 + k % UW, j = y0 - 1 + k / UW;
      lu[n] = (k < UH * UW && i >= 0 && i <= g.nx && j >= 0 && j < g.ny) ? u[g.at(i, j)] : 0.0;
    }
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      const int k = tid + 256 * n;
      const int i = x0 - 1 + k % VW, j = y0 - 1 + k / VW;
      lv[n] = (k < VH * VW && i >= 0 && i < g.nx && j >= 0 && j <= g.ny) ? v[g.at(i, j)] : 0.0;
    }
    if (FUSED) {
      constexpr int NP = (PH * PW + 255) / 256;
      const double* __restrict__ ph = a.phi + off;
      double lp[NP];
#pragma unroll
      for (int n = 0; n < NP; ++n) {
        const int k = tid + 256 * n;
        const int i = x0 - 2 + k % PW, j = y0 - 2 + k / PW;
        lp[n] = (k < PH * PW && i >= 0 && i < g.nx && j >= 0 && j < g.ny) ? ph[g.at(i, j)] : 0.0;
      }
#pragma unroll
      for (int n = 0; n < NP; ++n)
        if (tid + 256 * n < PH * PW) sphi[tid + 256 * n] = lp[n];
    }
#pragma unroll
    for (int kk = 0; kk < KU; ++kk) {
      const int k = tid + 256 * kk;
      const int i = x0 + k % (TW + 1), j = y0 + k / (TW + 1);
      tpu[kk] = (TT)0;
      cmu[kk][0] = cmu[kk][1] = -1;
      if (k < TH * (TW + 1) && i <= g.nx && j < g.ny && g.fluid(i - 1, j) && g.fluid(i, j)) {
        if (!cold) tpu[kk] = __builtin_nontemporal_load(&tup[g.at(i, j)]);
        if (f) {
          cmu[kk][0] = a.cmap[g.at(i - 1, j)];
          cmu[kk][1] = a.cmap[g.at(i, j)];
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < KV; ++kk) {
      const int k = tid + 256 * kk;
      const int i = x0 + k % TW, j = y0 + k / TW;
      tpv[kk] = (TT)0;
      cmv[kk][0] = cmv[kk][1] = -1;
      if (k < (TH + 1) * TW && i < g.nx && j <= g.ny && g.fluid(i, j - 1) && g.fluid(i, j)) {
        if (!cold) tpv[kk] = __builtin_nontemporal_load(&tvp[g.at(i, j)]);
        if (f) {
          cmv[kk][0] = a.cmap[g.at(i, j - 1)];
          cmv[kk][1] = a.cmap[g.at(i, j)];
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < KR; ++rr) {
      pn[rr] = po[rr] = pr[rr] = s1a[rr] = s1b[rr] = 0.0;
      const int i = x0 + tx, j = y0 + ty + 4 * rr;
      if (FUSED && g.fluid(i, j)) {
        const long at = g.at(i, j), ac = (long)j * g.nx + i;
        if (a.phi_next) pn[rr] = a.phi_next[off + at];
        if (a.phi_old) po[rr] = __builtin_nontemporal_load(&a.phi_old[off + at]);
        if (phi_old2) pr[rr] = __builtin_nontemporal_load(&phi_old2[off + at]);
        if (a.s1u) {
          s1a[rr] = __builtin_nontemporal_load(&a.s1u[coff + ac]);
          s1b[rr] = __builtin_nontemporal_load(&a.s1v[coff + ac]);
        }
      }
    }
#pragma unroll
    for (int n = 0; n < NU; ++n)
      if (tid + 256 * n < UH * UW) su[tid + 256 * n] = lu[n];
#pragma unroll
    for (int n = 0; n < NV; ++n)
      if (tid + 256 * n < VH * VW) sv[tid + 256 * n] = lv[n];
  }
  __syncthreads();
#define SU(i, j) su[((j) - y0 + 1) * UW + ((i) - x0 + 1)]
#define SV(i, j) sv[((j) - y0 + 1) * VW + ((i) - x0 + 1)]
#define SP(i, j) sphi[((j) - y0 + 2) * PW + ((i) - x0 + 2)]
  // face forcing (operator P): the control values behind the prefetched indices
  double fu[KU], fv[KV];
#pragma unroll
  for (int kk = 0; kk < KU; ++kk)
    fu[kk] = 0.5 * ((cmu[kk][0] >= 0 ? f[cmu[kk][0]] : 0.0) + (cmu[kk][1] >= 0 ? f[cmu[kk][1]] : 0.0));
#pragma unroll
  for (int kk = 0; kk < KV; ++kk)
    fv[kk] = 0.5 * ((cmv[kk][0] >= 0 ? f[a.nctrl + cmv[kk][0]] : 0.0) +
                    (cmv[kk][1] >= 0 ? f[a.nctrl + cmv[kk][1]] : 0.0));
  double acc[NB], dmax = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = 0.0;
  if (FUSED) {
    const double dt = a.dt, inv_h = 1.0 / g.h;
    // u^n on the halo: active faces take the pressure gradient, the outflow face the
    // ghost -phi, walls and the inflow keep their boundary values (held by u*)
    for (int k = tid; k < UH * UW; k += 256) {
      const int i = x0 - 1 + k % UW, j = y0 - 1 + k / UW;
      if (i < 0 || i > g.nx || j < 0 || j >= g.ny) continue;
      const bool w = g.fluid(i - 1, j), e = g.fluid(i, j);
      if (w && e)
        su[k] = su[k] - dt * (SP(i, j) - SP(i - 1, j)) * inv_h;
      else if (w && i == g.nx)
        su[k] = su[k] + 2.0 * dt * SP(i - 1, j) * inv_h;
    }
    for (int k = tid; k < VH * VW; k += 256) {
      const int i = x0 - 1 + k % VW, j = y0 - 1 + k / VW;
      if (i < 0 || i >= g.nx || j < 0 || j > g.ny) continue;
      if (g.fluid(i, j - 1) && g.fluid(i, j)) sv[k] = sv[k] - dt * (SP(i, j) - SP(i, j - 1)) * inv_h;
    }
    __syncthreads();
    // the previous step's cost sample, divergence and this step's warm start on the tile cells
    // (thread layout and operand order of k_project_cost)
    const double done = a.stats ? a.stats[(long)mem * STATS_STRIDE + ST_STEPS] - 1.0 : 1.0;
    const int order = done < 0.5 ? 0 : done < 1.5 ? 1 : done < 2.5 ? 2 : 3;
#pragma unroll
    for (int rr = 0; rr < TH / 4; ++rr) {
      const int r = ty + 4 * rr;
      const int i = x0 + tx, j = y0 + r;
      if (!g.fluid(i, j)) continue;
      const long at = g.at(i, j);
      const double pc = SP(i, j);
      const double uw = SU(i, j), ue = SU(i + 1, j), vsv = SV(i, j), vn = SV(i, j + 1);
      if (a.phi_next) {
        const double p1 = pn[rr];
        double wn = order == 0 ? pc : 2.0 * pc - p1;
        if (a.phi_old) {
          if (order == 2 || (order == 3 && !phi_old2)) wn = 3.0 * (pc - p1) + po[rr];
          if (order == 3 && phi_old2) wn = (4.0 * (pc + po[rr]) - 6.0 * p1) - pr[rr];
          if (phi_old2) __builtin_nontemporal_store(po[rr], &phi_old2[off + at]);
          __builtin_nontemporal_store(p1, &a.phi_old[off + at]);
        }
        a.phi_next[off + at] = wn;
      }
      const double div = fabs((ue - uw + vn - vsv) * inv_h);
      dmax = (div > dmax || div != div) ? div : dmax;
      if (a.s1u) {
        const long ac = (long)j * g.nx + i;  // dense cell index
        const double du = 0.5 * (uw + ue) - a.shu[ac];
        const double dv = 0.5 * (vsv + vn) - a.shv[ac];
        __builtin_nontemporal_store(s1a[rr] + du, &a.s1u[coff + ac]);
        __builtin_nontemporal_store(s1b[rr] + dv, &a.s1v[coff + ac]);
        acc[rr >> 1] += du * du + dv * dv;  // row ty + 4 rr lies in cost block rr / 2
      }
    }
  }

  const TT h = (TT)g.h, inv4h = (TT)(0.25 / g.h), inv_h2 = (TT)(1.0 / (g.h * g.h)), nu = (TT)a.nu;
  const double dt = a.dt;

  // u faces i in [x0, x0+TW], j in [y0, y0+TH): the face i = x0+TW is the east
  // face of the tile, computed here for the divergence and owned by the next tile.
#pragma unroll
  for (int kk = 0; kk < (TH * (TW + 1) + 255) / 256; ++kk) {
    const int k = tid + 256 * kk;
    if (k >= TH * (TW + 1)) break;
    const int c = k % (TW + 1), r = k / (TW + 1);
    const int i = x0 + c, j = y0 + r;
    double us = 0.0;
    if (i <= g.nx && j < g.ny) {
      const bool w = g.fluid(i - 1, j), e = g.fluid(i, j);
      const double uo = SU(i, j);
      const bool owned = (c < TW) || (i == g.nx);
      if (w && e) {
        const TT uc = (TT)uo, uE = (TT)SU(i + 1, j), uW = (TT)SU(i - 1, j);
        const TT uN = g.u_solid(i, j + 1) ? (TT)g.u_wall_sign(i, j + 1) * uc : (TT)SU(i, j + 1);
        const TT uS = g.u_solid(i, j - 1) ? (TT)g.u_wall_sign(i, j - 1) * uc : (TT)SU(i, j - 1);
        const TT vSW = (TT)SV(i - 1, j), vSE = (TT)SV(i, j), vNW = (TT)SV(i - 1, j + 1), vNE = (TT)SV(i, j + 1);
        const TT adv = ((uc + uE) * (uc + uE) - (uW + uc) * (uW + uc)) * inv4h +
                       ((uc + uN) * (vNW + vNE) - (uS + uc) * (vSW + vSE)) * inv4h;
        const TT T = -adv + nu * (uE + uW + uN + uS - (TT)4 * uc) * inv_h2;
        const long at = g.at(i, j);
        const TT Tp = cold ? T : tpu[kk];
        us = uo + dt * ((double)((TT)1.5 * T - (TT)0.5 * Tp) + fu[kk]);
        if (owned) {
          __builtin_nontemporal_store(us, &a.us[off + at]);
          __builtin_nontemporal_store(T, &a.tu[off + at]);
        }
      } else if (w && i == g.nx) {
        us = uo - dt * g.uconv * (uo - SU(i - 1, j)) / g.h;
        if (owned) a.us[off + g.at(i, j)] = us;
      } else {
        us = uo;  // wall (0) or inflow profile
      }
    }
    sus[r * (TW + 1) + c] = us;
  }
  // v faces i in [x0, x0+TW), j in [y0, y0+TH]
#pragma unroll
  for (int kk = 0; kk < ((TH + 1) * TW + 255) / 256; ++kk) {
    const int k = tid + 256 * kk;
    if (k >= (TH + 1) * TW) break;
    const int c = k % TW, r = k / TW;
    const int i = x0 + c, j = y0 + r;
    double vs = 0.0;
    if (i < g.nx && j <= g.ny) {
      const bool s = g.fluid(i, j - 1), nn = g.fluid(i, j);
      const double vo = SV(i, j);
      const bool owned = (r < TH) || (j == g.ny);
      if (s && nn) {
        const TT vc = (TT)vo, vN = (TT)SV(i, j + 1), vS = (TT)SV(i, j - 1);
        const TT vW = (i == 0 || g.v_solid(i - 1, j)) ? -vc : (TT)SV(i - 1, j);
        const TT vE = (i == g.nx - 1) ? vc : (g.v_solid(i + 1, j) ? -vc : (TT)SV(i + 1, j));
        const TT uSW = (TT)SU(i, j - 1), uSE = (TT)SU(i + 1, j - 1), uNW = (TT)SU(i, j), uNE = (TT)SU(i + 1, j);
        const TT adv = ((uNE + uSE) * (vc + vE) - (uNW + uSW) * (vW + vc)) * inv4h +
                       ((vc + vN) * (vc + vN) - (vS + vc) * (vS + vc)) * inv4h;
        const TT T = -adv + nu * (vE + vW + vN + vS - (TT)4 * vc) * inv_h2;
        const long at = g.at(i, j);
        const TT Tp = cold ? T : tpv[kk];
        vs = vo + dt * ((double)((TT)1.5 * T - (TT)0.5 * Tp) + fv[kk]);
        if (owned) {
          __builtin_nontemporal_store(vs, &a.vs[off + at]);
          __builtin_nontemporal_store(T, &a.tv[off + at]);
        }
      } else {
        vs = vo;  // wall
      }
    }
    svs[r * TW + c] = vs;
  }
  (void)h;
  __syncthreads();
  // Poisson right-hand side on the tile cells
  const double inv_hdt = 1.0 / (g.h * dt);
  for (int k = tid; k < TH * TW; k += 256) {
    const int c = k % TW, r = k / TW;
    const int i = x0 + c, j = y0 + r;
    if (i < g.nx && j < g.ny) {
      double bb = 0.0;
      if (g.fluid(i, j))
        bb = ((sus[r * (TW + 1) + c + 1] - sus[r * (TW + 1) + c]) + (svs[(r + 1) * TW + c] - svs[r * TW + c])) *
             inv_hdt;
      a.b[off + g.at(i, j)] = bb;
    }
  }
  if (FUSED) {
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = wave_sum(acc[b]);
    dmax = wave_max(dmax);
    if (tx == 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) red_s[b][ty] = acc[b];
      red_m[ty] = dmax;
    }
    __syncthreads();
    if (tid == 0) {
      if (a.s2part)
        for (int b = 0; b < NB; ++b) {
          if (y0 + COST_TH * b >= g.ny) break;
          const double s = ((red_s[b][0] + red_s[b][1]) + red_s[b][2]) + red_s[b][3];
          a.s2part[(long)mem * a.cost_ntiles + a.cost_tiling.index(x0, y0 + COST_TH * b)] += s;
        }
      double m = red_m[0];
      for (int k = 1; k < 4; ++k) m = (red_m[k] > m || red_m[k] != red_m[k]) ? red_m[k] : m;
      atomicMax((unsigned long long*)&a.divmax[mem], dbits(m));
    }
  }
#undef SU
#undef SV
#undef SP
}

// ---------------------------------------------------------------------------- projection + cost
// The S2 partial of every 64 x 8 cost block is formed with the same operand
// order whatever the tile height, so J does not depend on the tile choice.
template <bool ONE, int TH>
__global__ __launch_bounds__(256) void k_project_cost(Multi<ProjArgs> ms) {
  constexpr int TW = TILE_W, NB = TH / COST_TH;
  static_assert(TH % COST_TH == 0 && COST_TH == 8, "cost blocks are 64 x 8 (two rows per thread)");
  __shared__ double red_s[NB][4];
  __shared__ double red_m[4];
  int item;
  const ProjArgs& a = ms.template pick<ONE>(xcd_remap(blockIdx.x, gridDim.x), item);
  const Geo& g = a.g;
  const int mem = item / a.ntiles;
  const int tile = item % a.ntiles;
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const long off = (long)mem * a.plane;
  double* __restrict__ u = a.u + off;
  double* __restrict__ v = a.v + off;
  const double* __restrict__ us = a.us + off;
  const double* __restrict__ vs = a.vs + off;
  const double* __restrict__ phi = a.phi + off;
  const long coff = (long)mem * a.cplane;
  const double dt = a.dt, inv_h = 1.0 / g.h;
  const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
  // extrapolation order of the warm start: constant after the first step (where the forcing
  // switches on), linear after the second, quadratic after the third, then cubic when a third
  // history plane is given (FP64: the solves are tight enough that truncation dominates; in
  // mixed precision the amplified convergence error of the previous solves does, and the
  // quadratic order converges in fewer passes)
  const double done = a.stats ? a.stats[(long)mem * STATS_STRIDE + ST_STEPS] : 1.0;
  const int order = done < 0.5 ? 0 : done < 1.5 ? 1 : done < 2.5 ? 2 : 3;
  double acc[NB], dmax = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = 0.0;
#pragma unroll
  for (int rr = 0; rr < TH / 4; ++rr) {
    const int r = ty + 4 * rr;
    const int i = x0 + tx, j = y0 + r;
    if (!g.fluid(i, j)) continue;
    const long at = g.at(i, j);
    const double pc = phi[at];
    double uw, ue, vsv, vn;
    if (g.fluid(i - 1, j)) {
      uw = us[at] - dt * (pc - phi[g.at(i - 1, j)]) * inv_h;
      u[at] = uw;
    } else {
      uw = u[at];
    }
    if (g.fluid(i + 1, j)) {
      ue = us[g.at(i + 1, j)] - dt * (phi[g.at(i + 1, j)] - pc) * inv_h;
    } else if (i + 1 == g.nx) {
      ue = us[g.at(i + 1, j)] + 2.0 * dt * pc * inv_h;
      u[g.at(i + 1, j)] = ue;
    } else {
      ue = u[g.at(i + 1, j)];
    }
    if (g.fluid(i, j - 1)) {
      vsv = vs[at] - dt * (pc - phi[g.at(i, j - 1)]) * inv_h;
      v[at] = vsv;
    } else {
      vsv = v[at];
    }
    if (g.fluid(i, j + 1)) {
      vn = vs[g.at(i, j + 1)] - dt * (phi[g.at(i, j + 1)] - pc) * inv_h;
    } else {
      vn = v[g.at(i, j + 1)];
    }
    if (a.phi_next) {
      const double p1 = a.phi_next[off + at];
      double wn = order == 0 ? pc : 2.0 * pc - p1;
      if (a.phi_old) {
        const double p2 = a.phi_old[off + at];
        if (order == 2 || (order == 3 && !a.phi_old2)) wn = 3.0 * (pc - p1) + p2;
        if (order == 3 && a.phi_old2) wn = (4.0 * (pc + p2) - 6.0 * p1) - a.phi_old2[off + at];
        if (a.phi_old2) a.phi_old2[off + at] = p2;
        a.phi_old[off + at] = p1;
      }
      a.phi_next[off + at] = wn;
    }
    const double div = fabs((ue - uw + vn - vsv) * inv_h);
    dmax = (div > dmax || div != div) ? div : dmax;
    if (a.s1u) {
      const long ac = (long)j * g.nx + i;  // dense cell index
      const double du = 0.5 * (uw + ue) - a.shu[ac];
      const double dv = 0.5 * (vsv + vn) - a.shv[ac];
      a.s1u[coff + ac] += du;
      a.s1v[coff + ac] += dv;
      acc[rr >> 1] += du * du + dv * dv;  // row ty + 4 rr lies in cost block rr / 2
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = wave_sum(acc[b]);
  dmax = wave_max(dmax);
  if (tx == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) red_s[b][ty] = acc[b];
    red_m[ty] = dmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (a.s2part)
      for (int b = 0; b < NB; ++b) {
        if (y0 + COST_TH * b >= g.ny) break;
        const double s = ((red_s[b][0] + red_s[b][1]) + red_s[b][2]) + red_s[b][3];
        a.s2part[(long)mem * a.cost_ntiles + a.cost_tiling.index(x0, y0 + COST_TH * b)] += s;
      }
    double m = red_m[0];
    for (int k = 1; k < 4; ++k) m = (red_m[k] > m || red_m[k] != red_m[k]) ? red_m[k] : m;
    atomicMax((unsigned long long*)&a.divmax[mem], dbits(m));
  }
}

// ---------------------------------------------------------------------------- velocity sensors
// After the pressure solve of a step: the projected velocity u = u* - dt grad phi at the
// sixteen active faces around the four sensors, combined bilinearly (the operand order is
// fixed by SensorArgs). Samples are taken at the end of steps every, 2 every, ...; the
// sample index comes from the member's step counter, so captured graphs stay valid.
__global__ void k_sensors(Multi<SensorArgs> ms) {
  int blk;
  const SensorArgs& a = ms.template pick<false>(blockIdx.x, blk);
  const int t = blk * blockDim.x + threadIdx.x;
  if (t >= a.nmem * OBS_CHANNELS) return;
  const int mem = t / OBS_CHANNELS, c = t % OBS_CHANNELS;
  const int n1 = (int)a.stats[(long)mem * STATS_STRIDE + ST_STEPS] + 1;  // this step's end state is u^{n1}
  if (n1 % a.every != 0) return;
  const int sidx = n1 / a.every - 1;
  if (sidx >= a.K) return;
  const Geo& g = a.g;
  const long off = (long)mem * a.plane;
  const double inv_h = 1.0 / g.h;
  double f[4];
  for (int q = 0; q < 4; ++q) {
    const int i = a.fi[c][q], j = a.fj[c][q];
    const long at = off + g.at(i, j);
    if ((c & 1) == 0)
      f[q] = a.us[at] - a.dt * (a.phi[at] - a.phi[off + g.at(i - 1, j)]) * inv_h;
    else
      f[q] = a.vs[at] - a.dt * (a.phi[at] - a.phi[off + g.at(i, j - 1)]) * inv_h;
  }
  const double tx = a.tx[c], ty = a.ty[c];
  a.obs[((long)mem * OBS_CHANNELS + c) * a.K + sidx] =
      (1 - ty) * ((1 - tx) * f[0] + tx * f[1]) + ty * ((1 - tx) * f[2] + tx * f[3]);
}

// ---------------------------------------------------------------------------- per-step bookkeeping
// One thread per member (step_book_member).
__global__ void k_step_book(Multi<BookArgs> ms) {
  int blk;
  const BookArgs& a = ms.template pick<false>(blockIdx.x, blk);
  const int mem = blk * blockDim.x + threadIdx.x;
  if (mem >= a.nmem) return;
  step_book_member(a, mem);
}

// ---------------------------------------------------------------------------- J finalisation
// J = dt h^2 (S2 - sum_c |S1_c|^2 / K) + lambda h^2 |f|^2, fixed-order reductions.
__global__ __launch_bounds__(256) void k_finalize_J(FinalArgs a) {
  __shared__ double red[3][4];
  const int mem = blockIdx.x;
  const Geo& g = a.g;
  const long coff = (long)mem * a.cplane;
  double q = 0.0, s2 = 0.0, ff = 0.0;
  const long ncell = (long)g.nx * g.ny;
  for (long c = threadIdx.x; c < ncell; c += 256) {
    const double x = a.s1u[coff + c], y = a.s1v[coff + c];
    q += x * x + y * y;
  }
  for (int t = threadIdx.x; t < a.ntiles; t += 256) s2 += a.s2part[(long)mem * a.ntiles + t];
  if (a.ctrl)
    for (long k = threadIdx.x; k < a.m; k += 256) {
      const double x = a.ctrl[(long)mem * a.m + k];
      ff += x * x;
    }
  q = wave_sum(q);
  s2 = wave_sum(s2);
  ff = wave_sum(ff);
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
    red[0][w] = q;
    red[1][w] = s2;
    red[2][w] = ff;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double Q = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    const double S2 = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    const double FF = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
    const double h2 = g.h * g.h;
    const double J = a.dt * h2 * (S2 - Q / (double)a.K) + a.penalty * h2 * FF;
    a.J[mem] = J;
    if (a.stats) a.stats[(long)mem * STATS_STRIDE + ST_J] = J;
  }
}

// ---------------------------------------------------------------------------- member initialisation
// Copies the base state into every member, zeroes the cost accumulators.
template <typename TT>
__global__ __launch_bounds__(256) void k_init_members(InitArgs<TT> a) {
  const int mem = blockIdx.y;
  const long off = (long)mem * a.plane;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < a.plane; k += (long)gridDim.x * 256L) {
    a.u[off + k] = a.bu[k];
    a.v[off + k] = a.bv[k];
    a.us[off + k] = a.bu[k];
    a.vs[off + k] = a.bv[k];
    a.us2[off + k] = a.bu[k];  // both u* buffers carry the boundary values of u
    a.vs2[off + k] = a.bv[k];
    a.tu[off + k] = (TT)a.btu[k];
    a.tv[off + k] = (TT)a.btv[k];
    a.phi[off + k] = a.bphi[k];
    a.phi2[off + k] = a.bphi[k];
  }
  const long coff = (long)mem * a.cplane;
  if (a.s1u)
    for (long k = blockIdx.x * 256L + threadIdx.x; k < a.cplane; k += (long)gridDim.x * 256L) {
      a.s1u[coff + k] = 0.0;
      a.s1v[coff + k] = 0.0;
    }
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < a.ntiles; t += 256)
      if (a.s2part) a.s2part[(long)mem * a.ntiles + t] = 0.0;
    for (int t = threadIdx.x; t < STATS_STRIDE; t += 256) a.stats[(long)mem * STATS_STRIDE + t] = 0.0;
    if (threadIdx.x == 0) a.divmax[mem] = 0.0;
  }
}

// Cell-centred base velocity (the cost shift s_c), dense (ny, nx).
__global__ void k_shift(Geo g, const double* u, const double* v, double* shu, double* shv) {
  const long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (c >= (long)g.nx * g.ny) return;
  const int i = (int)(c % g.nx), j = (int)(c / g.nx);
  if (g.fluid(i, j)) {
    shu[c] = 0.5 * (u[g.at(i, j)] + u[g.at(i + 1, j)]);
    shv[c] = 0.5 * (v[g.at(i, j)] + v[g.at(i, j + 1)]);
  } else {
    shu[c] = 0.0;
    shv[c] = 0.0;
  }
}

// Copy member 0's evolved fields back into a base state (spin-up).
template <typename TT>
__global__ void k_store_base(long plane, const double* u, const double* v, const TT* tu, const TT* tv,
                             const double* phi, double* bu, double* bv, double* btu, double* btv, double* bphi) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < plane; k += (long)gridDim.x * blockDim.x) {
    bu[k] = u[k];
    bv[k] = v[k];
    btu[k] = (double)tu[k];
    btv[k] = (double)tv[k];
    bphi[k] = phi[k];
  }
}

// Member fields to the dense oracle layout [mem][u (ny, nx+1) | v (ny+1, nx)].
__global__ void k_fields_out(Geo g, long plane, const double* u, const double* v, double* out) {
  const int mem = blockIdx.y;
  const long nu_ = (long)g.ny * (g.nx + 1), nv_ = (long)(g.ny + 1) * g.nx;
  double* o = out + (long)mem * (nu_ + nv_);
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < nu_ + nv_; k += (long)gridDim.x * blockDim.x) {
    if (k < nu_) {
      const int i = (int)(k % (g.nx + 1)), j = (int)(k / (g.nx + 1));
      o[k] = u[(long)mem * plane + g.at(i, j)];
    } else {
      const long q = k - nu_;
      const int i = (int)(q % g.nx), j = (int)(q / g.nx);
      o[k] = v[(long)mem * plane + g.at(i, j)];
    }
  }
}

__global__ void k_clear_flag(int* flag) { *flag = 0; }

// Plain streaming copy (16-byte vectors, grid-stride): the measured HBM ceiling
// and the reference that calibrates the memory-traffic counters.
// Streaming copy: each thread keeps COPY_U independent 16-byte nontemporal loads in flight before
// its stores (a one-load-per-iteration loop leaves the copy latency-bound); a workgroup covers
// 256 x COPY_U consecutive 16-byte chunks per iteration, so every load and store is coalesced.
typedef double copy_v2 __attribute__((ext_vector_type(2)));
constexpr int COPY_U = 4;
__global__ __launch_bounds__(256) void k_stream_copy(const copy_v2* __restrict__ src, copy_v2* __restrict__ dst,
                                                     long n) {
  const long stride = (long)gridDim.x * 256 * COPY_U;
  for (long base = (long)blockIdx.x * 256 * COPY_U + threadIdx.x; base < n; base += stride) {
    copy_v2 r[COPY_U];
#pragma unroll
    for (int u = 0; u < COPY_U; ++u) {
      const long k = base + (long)u * 256;
      if (k < n) r[u] = __builtin_nontemporal_load(src + k);
    }
#pragma unroll
    for (int u = 0; u < COPY_U; ++u) {
      const long k = base + (long)u * 256;
      if (k < n) __builtin_nontemporal_store(r[u], dst + k);
    }
  }
}
void launch_stream_copy(const void* src, void* dst, long n16, hipStream_t s) {
  long blocks = (n16 + 256L * COPY_U - 1) / (256L * COPY_U);
  if (blocks > 256L * 32) blocks = 256L * 32;  // 32 workgroups per CU, grid-stride beyond
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const copy_v2*)src, (copy_v2*)dst, n16);
}

// ---------------------------------------------------------------------------- launchers
template <typename TT, int TH, bool FUSED, bool CUBIC = false>
static void launch_predictor_(const Multi<PredArgs<TT>>& m, hipStream_t s) {
  if (m.nseg == 1)
    hipLaunchKernelGGL((k_predictor<TT, true, TH, FUSED, CUBIC>), dim3(m.total()), dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL((k_predictor<TT, false, TH, FUSED, CUBIC>), dim3(m.total()), dim3(256), 0, s, m);
}
// every segment of one launch shares the tile height and the fused flag (the host groups by them)
template <typename TT>
void launch_predictor(const Multi<PredArgs<TT>>& m, hipStream_t s) {
  const bool r8 = m.seg[0].trows == 8;
  if (m.seg[0].fused) {
    // one precision per batch, so every segment has the third history plane or none does
    const bool cubic = m.seg[0].phi_old2 != nullptr;
    if (r8)
      cubic ? launch_predictor_<TT, 8, true, true>(m, s) : launch_predictor_<TT, 8, true>(m, s);
    else
      cubic ? launch_predictor_<TT, 16, true, true>(m, s) : launch_predictor_<TT, 16, true>(m, s);
  } else {
    if (r8)
      launch_predictor_<TT, 8, false>(m, s);
    else
      launch_predictor_<TT, 16, false>(m, s);
  }
}
template void launch_predictor<double>(const Multi<PredArgs<double>>&, hipStream_t);

template <int TH>
static void launch_project_cost_(const Multi<ProjArgs>& m, hipStream_t s) {
  if (m.nseg == 1)
    hipLaunchKernelGGL((k_project_cost<true, TH>), dim3(m.total()), dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL((k_project_cost<false, TH>), dim3(m.total()), dim3(256), 0, s, m);
}
void launch_project_cost(const Multi<ProjArgs>& m, hipStream_t s) {
  if (m.seg[0].trows == 8)
    launch_project_cost_<8>(m, s);
  else
    launch_project_cost_<16>(m, s);
}
void launch_sensors(const Multi<SensorArgs>& m, hipStream_t s) {
  hipLaunchKernelGGL(k_sensors, dim3(m.total()), dim3(64), 0, s, m);
}
void launch_step_book(const Multi<BookArgs>& m, hipStream_t s) {
  hipLaunchKernelGGL(k_step_book, dim3(m.total()), dim3(64), 0, s, m);
}
void launch_finalize_J(const FinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_J, dim3(a.nmem), dim3(256), 0, s, a);
}
template <typename TT>
void launch_init_members(const InitArgs<TT>& a, hipStream_t s) {
  int bx = (int)((a.plane + 255) / 256);
  if (bx > 128) bx = 128;
  hipLaunchKernelGGL(k_init_members<TT>, dim3(bx, a.nmem), dim3(256), 0, s, a);
}
template void launch_init_members<double>(const InitArgs<double>&, hipStream_t);

void launch_shift(const Geo& g, const double* u, const double* v, double* shu, double* shv, hipStream_t s) {
  const long n = (long)g.nx * g.ny;
  hipLaunchKernelGGL(k_shift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, u, v, shu, shv);
}
template <typename TT>
void launch_store_base(long plane, const double* u, const double* v, const TT* tu, const TT* tv, const double* phi,
                       double* bu, double* bv, double* btu, double* btv, double* bphi, hipStream_t s) {
  hipLaunchKernelGGL(k_store_base<TT>, dim3(256), dim3(256), 0, s, plane, u, v, tu, tv, phi, bu, bv, btu, btv, bphi);
}
template void launch_store_base<double>(long, const double*, const double*, const double*, const double*,
                                        const double*, double*, double*, double*, double*, double*, hipStream_t);
void launch_fields_out(const Geo& g, long plane, int nmem, const double* u, const double* v, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_fields_out, dim3(64, nmem), dim3(256), 0, s, g, plane, u, v, out);
}
void launch_clear_flag(int* flag, hipStream_t s) { hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag); }

}  // namespace envar
