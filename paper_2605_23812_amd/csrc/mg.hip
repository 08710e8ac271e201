// Batched masked geometric multigrid for the pressure Poisson equation
//   L_h phi = b,  L_h phi_c = (sum over fluid neighbours (phi_nb - phi_c) - 2 phi_c [outflow face]) / h^2
// on the channel-plus-cavity mask: homogeneous Neumann on walls and inflow,
// phi = 0 on the outflow face (mirror ghost -phi). The geometry is aligned on
// every level down to h = 1/4, so each coarse cell has four fluid children.
//
// Per fine level and V-cycle two launches, both over (member, 64-wide tile of 8, 16 or 32 rows):
//   pre : load phi, b with a halo of 2 NS + 1 into LDS, NS red-black
//         Gauss-Seidel sweeps relaxed by mg_omega (temporal blocking: a sweep invalidates two
//         halo rings), residual r = b - L phi, restriction b_c = mean of the
//         four children; writes phi and b_c.
//   post: load phi, b with a halo of 2 NS (+1), add the bilinearly
//         prolongated coarse correction (Neumann mirror at walls, sign flip
//         across the outflow face), NS sweeps, optionally the per-member
//         max-norm of dt r (wave reductions + atomicMax); writes phi (or adds
//         it to the FP64 pressure in iterative refinement).
// In iterative refinement (FP32 V-cycles inside an FP64 solve) the finest
// pre kernel starts from the FP64 pressure instead of an FP32 right-hand side:
// it stages phi64 of its window in LDS, forms r = b64 - L phi64 there (the
// FP32 right-hand side of the correction), and records dt max|r| over its tile.
// phi64 is only read in that launch, so neighbouring tiles see one version.
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

// The multigrid tile kernels hold a 64 x (TR + 2H) window of one level in
// LDS around a (64 - 2H) x TR tile (TR = 8 or 16 rows, chosen per level by
// the tile tuner): a window row is one wave, lane = column,
// so no index needs a division. The two red-black colours live in separate
// padded planes; a cell's four neighbours are all of the other colour and sit
// at consecutive addresses for consecutive lanes. Each thread owns one column
// position q of each colour in every eighth window row; its 1/diag, diag and
// h^2 b stay in registers. Ring cells of the window and cells outside the
// fluid are frozen (1/diag = 0). The Poisson diagonal of every cell is read
// from a per-level byte plane shared by all members.
// (ox + oy) is even, so a cell's colour is (r + col) & 1 in window coordinates.
template <typename T, int TR>
struct Win {
  static constexpr int H = mg_h<T>(), LW = 64, TWI = mg_tw<T>(), TH = TR, LH = TH + 2 * H;
  static constexpr int QS = 34;                 // padded row stride of a colour plane (32 cells)
  static constexpr int CS = (LH + 2) * QS;      // padded colour plane
  static constexpr int NR = (LH + 3) / 4;       // window rows per wave
  static constexpr int NIT = (LH + 7) / 8;      // cells per thread and colour
  static __device__ __forceinline__ int idx(int r, int col) {
    return ((r + col) & 1) * CS + (r + 1) * QS + (col >> 1) + 1;
  }
};

template <typename T>
__device__ __forceinline__ T inv_of(int d) {
  return d == 4 ? (T)0.25 : d == 3 ? (T)(1.0 / 3.0) : d == 2 ? (T)0.5 : d == 5 ? (T)0.2 : d == 6 ? (T)(1.0 / 6.0)
                                                                                          : (T)1;
}

template <typename T, int TR>
struct Items {
  typedef Win<T, TR> W;
  int own0[2];        // LDS offset of the first item of each colour
  int left0[2];       // offset of its left neighbour (other colour)
  int r0, q;
  T hb[2][W::NIT];    // h^2 b
  T invd[2][W::NIT];  // 1/diag, 0 = frozen
  T d[2][W::NIT];     // diag

  __device__ __forceinline__ void init(const T* sb, const unsigned char* scode, T h2) {
    r0 = threadIdx.x >> 5;
    q = threadIdx.x & 31;
    for (int c = 0; c < 2; ++c) {
      const int p = (c ^ r0) & 1;  // column parity of this colour in rows r0 + 8n
      own0[c] = c * W::CS + (r0 + 1) * W::QS + q + 1;
      left0[c] = (1 - c) * W::CS + (r0 + 1) * W::QS + q + p;
#pragma unroll
      for (int n = 0; n < W::NIT; ++n) {
        const int r = r0 + 8 * n, col = 2 * q + p;
        const int o = own0[c] + 8 * n * W::QS;
        invd[c][n] = (T)0;
        d[c][n] = (T)1;
        hb[c][n] = (T)0;
        if (r < W::LH) {
          const int code = scode[o];
          const bool ring = r == 0 || r == W::LH - 1 || col == 0 || col == W::LW - 1;
          if (code && !ring) {
            invd[c][n] = inv_of<T>(code);
            d[c][n] = (T)code;
            hb[c][n] = h2 * sb[o];
          }
        }
      }
    }
  }
  __device__ __forceinline__ T nbsum(const T* sp, int c, int n) const {
    const int l = left0[c] + 8 * n * W::QS;
    const int m = l + 1 - ((c ^ r0) & 1);  // other colour, same column
    return (sp[l] + sp[l + 1]) + (sp[m - W::QS] + sp[m + W::QS]);
  }
  __device__ __forceinline__ void sweep(T* sp) const {
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int n = 0; n < W::NIT; ++n)
        if (invd[c][n] != (T)0) {
          T* const o = sp + own0[c] + 8 * n * W::QS;
          *o += (T)mg_omega<T>() * ((nbsum(sp, c, n) - hb[c][n]) * invd[c][n] - *o);
        }
      __syncthreads();
    }
  }
  // the same four neighbours summed in FP64
  __device__ __forceinline__ double nbsum64(const T* sp, int c, int n) const {
    const int l = left0[c] + 8 * n * W::QS;
    const int m = l + 1 - ((c ^ r0) & 1);
    return ((double)sp[l] + (double)sp[l + 1]) + ((double)sp[m - W::QS] + (double)sp[m + W::QS]);
  }
  // h^2 r = h^2 b - (sum nb - d phi)
  __device__ __forceinline__ T resid_h2(const T* sp, int c, int n) const {
    return hb[c][n] - (nbsum(sp, c, n) - d[c][n] * sp[own0[c] + 8 * n * W::QS]);
  }
  // window row and column of item (c, n)
  __device__ __forceinline__ int row(int n) const { return r0 + 8 * n; }
  __device__ __forceinline__ int col(int c) const { return 2 * q + ((c ^ r0) & 1); }
};

// window load shared by pre and post: phi (+ correction), b and the diagonal codes
template <typename T, int TR, typename E = T>
struct WinLoad {
  typedef Win<T, TR> W;
  E vp[W::NR], vb[W::NR];
  unsigned char vc[W::NR];
  __device__ __forceinline__ void fetch(const Geo& g, const unsigned char* code, const E* phi, const E* b, long off,
                                        int ox, int oy) {
    const int col = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = ox + col;
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m, j = oy + r;
      vp[m] = (E)0;
      vb[m] = (E)0;
      vc[m] = 0;
      if (r < W::LH && i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
        const long at = g.at(i, j);
        // independent loads (no wait on the code); non-fluid values are masked below
        vc[m] = code[at];
        vb[m] = b[off + at];
        if (phi) vp[m] = phi[off + at];
      }
    }
#pragma unroll
    for (int m = 0; m < W::NR; ++m)
      if (!vc[m]) {
        vp[m] = (E)0;
        vb[m] = (E)0;
      }
  }
};

// refinement pre: the previous pass's norm decides; a skipped member carries it forward
template <typename T>
__device__ __forceinline__ bool ref_skip(const MGArgs<T>& a, int mem, int tile) {
  if (a.rslot <= 0) return false;
  const double prev = a.norms[(long)mem * a.norm_slots + a.rslot - 1];
  if (prev <= a.tol) {
    if (tile == 0 && threadIdx.x == 0) a.norms[(long)mem * a.norm_slots + a.rslot] = prev;
    return true;
  }
  return false;
}

// ---------------------------------------------------------------------------- pre-smoothing + restriction
// REF: PRE_PLAIN; PRE_FIRST (mixed finest level, first pass: the FP64 residual r = b64 - L phi64 is
// formed on the window, stored rounded to T in r_out, its norm into norms[rslot]); PRE_LATER (mixed
// finest level, later passes: the right-hand side is the residual carried in `b` unless the
// member's previous norm exceeds `anchor`, in which case it is formed afresh as in PRE_FIRST and
// stored in r_out (the same plane), without a norm: a residual near the tolerance is carried, a
// large one re-anchored, so the carried residual's rounding stays below anchor x 6e-8)
// LDS of one pre tile: sp | sb (in refinement first the FP64 pressure window), diagonal codes
template <typename T, int TR>
struct PreLds {
  T spb[4 * Win<T, TR>::CS];
  unsigned char scode[2 * Win<T, TR>::CS];
  double red[4];
};

// One (member, tile) of the pre kernel; the tail kernel runs the same body over a member's tiles.
template <typename T, int NS, int REF, int TR>
__device__ __forceinline__ void mg_pre_tile(const MGArgs<T>& a, int mem, int tile, PreLds<T, TR>& S) {
  typedef Win<T, TR> W;
  static_assert(2 * NS + 1 <= W::H, "window halo too small for the sweep count");
  static_assert(W::TH * 64 <= 2 * W::CS, "residual staging does not fit");
  static_assert(REF == PRE_PLAIN || sizeof(double) * 64 * W::LH <= sizeof(T) * 4 * W::CS,
                "FP64 window does not fit");
  T* const spb = S.spb;
  unsigned char* const scode = S.scode;
  double* const red = S.red;
  T* const sp = spb;
  T* const sb = spb + 2 * W::CS;
  const Geo& g = a.g;
  if (REF == PRE_FIRST ? ref_skip(a, mem, tile) : mg_skip(a, mem, tile)) return;
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const int ox = x0 - W::H, oy = y0 - W::H;
  const long off = (long)mem * a.plane;
  const int col = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool form = REF == PRE_FIRST ||
                    (REF == PRE_LATER && a.norms[(long)mem * a.norm_slots + a.k - 1] > a.anchor);
  if (form) {
    // r = b64 - L phi64 on the window (ring excluded), same arithmetic order as k_resid64
    double* const P64 = (double*)spb;
    WinLoad<T, TR, double> L64;
    L64.fetch(g, a.code, a.phi64, a.b64, off, ox, oy);
    double (&vp)[W::NR] = L64.vp;
    double (&vb)[W::NR] = L64.vb;
    unsigned char (&vc)[W::NR] = L64.vc;
    const int i = ox + col;
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      if (!vc[m]) {
        vp[m] = 0.0;
        vb[m] = 0.0;
      }
      if (r < W::LH) {
        P64[r * 64 + col] = vp[m];
        scode[W::idx(r, col)] = vc[m];
      }
    }
    __syncthreads();
    const double inv_h2 = 1.0 / (g.h * g.h);
    const bool tcol = col >= W::H && col < W::H + W::TWI;
    double mx = 0.0;
    T rf[W::NR];
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      rf[m] = (T)0;
      if (vc[m] && r >= 1 && r < W::LH - 1 && col >= 1 && col < 63) {
        const double* q = P64 + r * 64 + col;
        double s = 0.0;
        s += q[-1];
        s += q[1];
        s += q[-64];
        s += q[64];
        const double rr = vb[m] - (s - (double)vc[m] * q[0]) * inv_h2;
        rf[m] = (T)rr;
        if (tcol && r >= W::H && r < W::H + W::TH) {
          a.r_out[off + g.at(i, oy + r)] = rf[m];
          const double ar = fabs(rr) * a.dt;
          mx = (ar > mx || ar != ar) ? ar : mx;
        }
      }
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) red[w] = mx;
    __syncthreads();  // every FP64 read is done before sp / sb overwrite the window
    if (REF == PRE_FIRST && threadIdx.x == 0) {
      double mm = red[0];
      for (int q = 1; q < 4; ++q) mm = (red[q] > mm || red[q] != red[q]) ? red[q] : mm;
      atomicMax((unsigned long long*)&a.norms[(long)mem * a.norm_slots + a.rslot], dbits(mm));
    }
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      if (r < W::LH) {
        const int x = W::idx(r, col);
        sp[x] = (T)0;
        sb[x] = rf[m];
      }
    }
  } else {
    WinLoad<T, TR> L;
    L.fetch(g, a.code, a.zero_guess ? nullptr : a.phi_in, a.b, off, ox, oy);
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      if (r < W::LH) {
        const int x = W::idx(r, col);
        sp[x] = L.vp[m];
        sb[x] = L.vb[m];
        scode[x] = L.vc[m];
      }
    }
  }
  __syncthreads();
  const T h2 = (T)(g.h * g.h);
  Items<T, TR> it;
  it.init(sb, scode, h2);
  for (int s = 0; s < NS; ++s) it.sweep(sp);
  // interior residuals staged in sb (dead by now) as a TR x 64 array
  T res[2][W::NIT];
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int n = 0; n < W::NIT; ++n) res[c][n] = it.invd[c][n] != (T)0 ? it.resid_h2(sp, c, n) : (T)0;
  __syncthreads();
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int n = 0; n < W::NIT; ++n) {
      const int r = it.row(n) - W::H;
      if (r >= 0 && r < W::TH) sb[r * 64 + it.col(c)] = res[c][n];
    }
  __syncthreads();
  {
    const Geo& gc = a.gc;
    const int ci = threadIdx.x & 31;
    for (int cj = 2 * w + (threadIdx.x >> 5 & 1); cj < W::TH / 2; cj += 8) {
      const int I = x0 / 2 + ci, J = y0 / 2 + cj;
      if (ci < W::TWI / 2 && gc.fluid(I, J)) {
        const T* rr = sb + (2 * cj) * 64 + W::H + 2 * ci;
        const T rs = (rr[0] + rr[1]) + (rr[64] + rr[65]);
        a.bc[(long)mem * a.cplane_c + gc.at(I, J)] = rs * (T)(0.25 / (g.h * g.h));
      }
    }
  }
  const int i = ox + col;
  if (col >= W::H && col < W::H + W::TWI && i < g.nx) {
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      const int j = oy + r;
      if (r >= W::H && r < W::H + W::TH && j < g.ny) {
        const int x = W::idx(r, col);
        if (scode[x]) a.phi_out[off + g.at(i, j)] = sp[x];
      }
    }
  }
}

template <typename T, int NS, int REF, bool ONE, int TR>
__global__ __launch_bounds__(256) void k_mg_pre(Multi<MGArgs<T>> ms) {
  __shared__ PreLds<T, TR> S;
  int item;
  const MGArgs<T>& a = ms.template pick<ONE>(xcd_remap(blockIdx.x, gridDim.x), item);
  mg_pre_tile<T, NS, REF, TR>(a, item / a.ntiles, item % a.ntiles, S);
}

// ---------------------------------------------------------------------------- prolongation + post-smoothing
// MODE: POST_PLAIN; POST_NORM (the residual norm of the V-cycle's own equation, FP64 cycles);
// POST_REFINE (mixed finest level: phi64 += e and the carried FP64 residual r - L e on the tile)
// LDS of one post tile: the window (phi, b, codes) and the coarse correction window
template <typename T, int TR>
struct PostLds {
  static constexpr int CW = 36, CH = Win<T, TR>::LH / 2 + 3;
  T sp[2 * Win<T, TR>::CS];
  T sb[2 * Win<T, TR>::CS];
  unsigned char scode[2 * Win<T, TR>::CS];
  T scw[CH * CW];
  unsigned char sccode[CH * CW];
  double red[4];
};

// One (member, tile) of the post kernel; the tail kernel runs the same body over a member's tiles.
template <typename T, int NS, int MODE, int TR>
__device__ __forceinline__ void mg_post_tile(const MGArgs<T>& a, int mem, int tile, PostLds<T, TR>& S) {
  typedef Win<T, TR> W;
  // the norm and the refinement update need the smoothed values on the tile and one ring around it
  static_assert(2 * NS + (MODE != POST_PLAIN ? 1 : 0) <= W::H, "window halo too small for the sweep count");
  constexpr int CW = PostLds<T, TR>::CW, CH = PostLds<T, TR>::CH;
  T* const sp = S.sp;
  T* const sb = S.sb;
  unsigned char* const scode = S.scode;
  T* const scw = S.scw;
  unsigned char* const sccode = S.sccode;
  double* const red = S.red;
  const Geo& g = a.g;
  const Geo& gc = a.gc;
  if (mg_skip(a, mem, tile)) return;
  int x0, y0;
  a.tiling.origin(tile, x0, y0);
  const int ox = x0 - W::H, oy = y0 - W::H;
  const long off = (long)mem * a.plane;
  const T* __restrict__ pc = a.phic + (long)mem * a.cplane_c;
  const int col = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cox = (ox >> 1) - 1, coy = (oy >> 1) - 1;
  WinLoad<T, TR> L;
  L.fetch(g, a.code, a.phi_in, a.b, off, ox, oy);
  // coarse correction window [cox, cox + 36) x [coy, coy + CH)
  {
    constexpr int NCR = (CH + 3) / 4;
    T vc[NCR];
    unsigned char cc[NCR];
    const int I = cox + col;
#pragma unroll
    for (int m = 0; m < NCR; ++m) {
      const int r = w + 4 * m, J = coy + r;
      vc[m] = (T)0;
      cc[m] = 0;
      if (col < CW && r < CH && I >= 0 && I < gc.nx && J >= 0 && J < gc.ny) {
        const long at = gc.at(I, J);
        cc[m] = a.codec[at];
        vc[m] = pc[at];
      }
    }
#pragma unroll
    for (int m = 0; m < NCR; ++m)
      if (!cc[m]) vc[m] = (T)0;
#pragma unroll
    for (int m = 0; m < NCR; ++m) {
      const int r = w + 4 * m;
      if (col < CW && r < CH) {
        scw[r * CW + col] = vc[m];
        sccode[r * CW + col] = cc[m];
      }
    }
  }
  __syncthreads();
  {
    const int i = ox + col;
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      if (r >= W::LH) continue;
      const int j = oy + r;
      T p = (T)0;
      if (L.vc[m]) {
        // bilinear prolongation: Neumann mirror at walls, sign flip across the outflow face
        const int I = i >> 1, J = j >> 1;
        const int IX = I + ((i & 1) ? 1 : -1), JY = J + ((j & 1) ? 1 : -1);
        const int cI = I - cox, cJ = J - coy, cX = IX - cox, cY = JY - coy;
        const T P = scw[cJ * CW + cI];
        const T X = sccode[cJ * CW + cX] ? scw[cJ * CW + cX] : (IX == gc.nx ? -P : P);
        const T Y = sccode[cY * CW + cI] ? scw[cY * CW + cI] : P;
        const T D = sccode[cY * CW + cX] ? scw[cY * CW + cX] : X + Y - P;
        p = L.vp[m] + ((T)9 * P + (T)3 * (X + Y) + D) * (T)0.0625;
      }
      const int x = W::idx(r, col);
      sp[x] = p;
      sb[x] = L.vb[m];
      scode[x] = L.vc[m];
    }
  }
  __syncthreads();
  const T h2 = (T)(g.h * g.h);
  Items<T, TR> it;
  it.init(sb, scode, h2);
  for (int s = 0; s < NS; ++s) it.sweep(sp);
  if (MODE == POST_REFINE) {
    // phi64 += e and r_out = r - L e (formed in FP64) on the tile's fluid cells; dt max|r - L e| -> norms[k].
    // Walked in the window layout (a wave's lanes on consecutive columns of one row), so that the FP32
    // residual and the FP64 pressure are read and written in whole rows; the sum of the four
    // neighbours runs in the same order as Items::nbsum64.
    const double inv_h2 = 1.0 / (g.h * g.h);
    double m = 0.0;
    const int i = ox + col;
    if (col >= W::H && col < W::H + W::TWI) {
#pragma unroll
      for (int q = 0; q < W::NR; ++q) {
        const int r = w + 4 * q;
        const int x = W::idx(r, col);
        if (r >= W::H && r < W::H + W::TH && scode[x]) {
          const long at = off + g.at(i, oy + r);
          const double e = (double)sp[x];
          const double nb = ((double)sp[W::idx(r, col - 1)] + (double)sp[W::idx(r, col + 1)]) +
                            ((double)sp[W::idx(r - 1, col)] + (double)sp[W::idx(r + 1, col)]);
          const double rn = (double)L.vb[q] - (nb - (double)scode[x] * e) * inv_h2;
          a.r_out[at] = (T)rn;
          a.add_to[at] += e;
          const double rr = fabs(rn) * a.dt;
          m = (rr > m || rr != rr) ? rr : m;
        }
      }
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = red[0];
      for (int q = 1; q < 4; ++q) mm = (red[q] > mm || red[q] != red[q]) ? red[q] : mm;
      atomicMax((unsigned long long*)&a.norms[(long)mem * a.norm_slots + a.k], dbits(mm));
    }
    return;
  }
  if (MODE == POST_NORM && a.write_norm) {
    double m = 0.0;
    const double sc = a.dt / (g.h * g.h);
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int n = 0; n < W::NIT; ++n) {
        const int r = it.row(n), cl = it.col(c);
        if (it.invd[c][n] != (T)0 && r >= W::H && r < W::H + W::TH && cl >= W::H && cl < W::H + W::TWI) {
          const double rr = fabs((double)it.resid_h2(sp, c, n)) * sc;
          m = (rr > m || rr != rr) ? rr : m;
        }
      }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = red[0];
      for (int q = 1; q < 4; ++q) mm = (red[q] > mm || red[q] != red[q]) ? red[q] : mm;
      atomicMax((unsigned long long*)&a.norms[(long)mem * a.norm_slots + a.k], dbits(mm));
    }
  }
  const int i = ox + col;
  if (col >= W::H && col < W::H + W::TWI && i < g.nx) {
#pragma unroll
    for (int m = 0; m < W::NR; ++m) {
      const int r = w + 4 * m;
      const int j = oy + r;
      if (r >= W::H && r < W::H + W::TH && j < g.ny) {
        const int x = W::idx(r, col);
        if (scode[x]) {
          if (a.add_to)
            a.add_to[off + g.at(i, j)] += (double)sp[x];
          else
            a.phi_out[off + g.at(i, j)] = sp[x];
        }
      }
    }
  }
}

template <typename T, int NS, int MODE, bool ONE, int TR>
__global__ __launch_bounds__(256) void k_mg_post(Multi<MGArgs<T>> ms) {
  __shared__ PostLds<T, TR> S;
  int item;
  const MGArgs<T>& a = ms.template pick<ONE>(xcd_remap(blockIdx.x, gridDim.x), item);
  mg_post_tile<T, NS, MODE, TR>(a, item / a.ntiles, item % a.ntiles, S);
}

// ---------------------------------------------------------------------------- coarse levels in LDS
// The levels inv_h = 16, 8, 4 of one member run in one workgroup, every level
// resident in LDS as a padded array: NX x ny cells plus a ring of ghost cells,
// row pitch NX + 2. Cells outside the fluid (and the ring) hold phi = 0 and a
// zero diagonal code, so a neighbour sum needs no geometry test; the code of a
// fluid cell is its Poisson diagonal count. NX is 64, 32, 16 (the channel is
// four units long); ny is the runtime height (cavity or plain channel).
constexpr int COARSE_THREADS = 1024;
constexpr int CNX0 = 64, CNX1 = 32, CNX2 = 16;
constexpr int CP0 = CNX0 + 2, CP1 = CNX1 + 2, CP2 = CNX2 + 2;
constexpr int CMAXNY0 = 32;
constexpr int CS0 = (CMAXNY0 + 2) * CP0, CS1 = (CMAXNY0 / 2 + 2) * CP1, CS2 = (CMAXNY0 / 4 + 2) * CP2;

template <int NX>
__device__ __forceinline__ int cx(int i, int j) {
  return (j + 1) * (NX + 2) + i + 1;
}

// diagonal codes of one level (ghost ring included)
template <int NX, int NTH>
__device__ __forceinline__ void lvl_codes(unsigned char* C, const Geo& g) {
  const int n = (g.ny + 2) * (NX + 2);
  for (int q = threadIdx.x; q < n; q += NTH) {
    const int jj = q / (NX + 2), i = q - jj * (NX + 2) - 1, j = jj - 1;
    C[q] = g.fluid(i, j) ? (unsigned char)g.diag_count(i, j) : (unsigned char)0;
  }
}

// one red-black Gauss-Seidel sweep (same operand order as the tiled kernels)
template <int NX, int NTH>
__device__ __forceinline__ void lvl_sweep(double* p, const double* b, const unsigned char* C, int ny, double h2) {
  constexpr int HX = NX / 2, P = NX + 2;
  constexpr int K = (HX * (CMAXNY0 * NX / CNX0) + NTH - 1) / NTH;
  const int n = HX * ny;
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = threadIdx.x + k * NTH;
      if (q >= n) break;
      const int j = q / HX, i = 2 * (q % HX) + ((c ^ j) & 1);
      const int x = cx<NX>(i, j);
      const int d = C[x];
      if (d) {
        double s = 0.0;
        s += p[x - 1];
        s += p[x + 1];
        s += p[x - P];
        s += p[x + P];
        p[x] = (s - h2 * b[x]) * inv_diag<double>(d);
      }
    }
    __syncthreads();
  }
}

template <int NX>
__device__ __forceinline__ double lvl_resid(const double* p, const double* b, const unsigned char* C, int x,
                                            double inv_h2) {
  constexpr int P = NX + 2;
  double s = 0.0;
  s += p[x - 1];
  s += p[x + 1];
  s += p[x - P];
  s += p[x + P];
  return b[x] - (s - (double)C[x] * p[x]) * inv_h2;
}

// residual of the fine level restricted (mean of the four children) into the
// coarse right-hand side; zero coarse guess
template <int NX, int NTH>
__device__ __forceinline__ void lvl_restrict(const double* p, const double* b, const unsigned char* C, double h,
                                             double* pc, double* bc, const unsigned char* Cc, int nyc) {
  constexpr int NXC = NX / 2;
  const double inv_h2 = 1.0 / (h * h);
  for (int q = threadIdx.x; q < NXC * nyc; q += NTH) {
    const int J = q / NXC, I = q % NXC;
    const int xc = cx<NXC>(I, J);
    double rs = 0.0;
    if (Cc[xc])
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) rs += lvl_resid<NX>(p, b, C, cx<NX>(2 * I + di, 2 * J + dj), inv_h2);
    bc[xc] = 0.25 * rs;
    pc[xc] = 0.0;
  }
  __syncthreads();
}

// bilinear prolongation of the coarse correction (Neumann mirror at walls,
// sign flip across the outflow face) added to the fine level
template <int NX, int NTH>
__device__ __forceinline__ void lvl_prolong(double* p, const unsigned char* C, int ny, const double* pc,
                                            const unsigned char* Cc) {
  constexpr int NXC = NX / 2;
  for (int q = threadIdx.x; q < NX * ny; q += NTH) {
    const int j = q / NX, i = q % NX;
    const int x = cx<NX>(i, j);
    if (!C[x]) continue;
    const int I = i >> 1, J = j >> 1;
    const int IX = I + ((i & 1) ? 1 : -1), JY = J + ((j & 1) ? 1 : -1);
    const int xP = cx<NXC>(I, J), xX = cx<NXC>(IX, J), xY = cx<NXC>(I, JY), xD = cx<NXC>(IX, JY);
    const double Pv = pc[xP];
    const double X = Cc[xX] ? pc[xX] : (IX == NXC ? -Pv : Pv);
    const double Y = Cc[xY] ? pc[xY] : Pv;
    const double D = Cc[xD] ? pc[xD] : X + Y - Pv;
    p[x] += (9.0 * Pv + 3.0 * (X + Y) + D) * 0.0625;
  }
  __syncthreads();
}

// V-cycle over the three LDS levels with NS red-black sweeps per level and a
// dense solve of the h = 1/4 operator through its inverse.
// The dense solve gives eight threads (consecutive lanes) to each coarsest unknown q, thread
// part = tid % 8 summing the terms r = part, part + 8, ... in order; with 1024 threads every
// unknown has its eight threads at once and their entries of the inverse are loaded into registers
// at the start, so that their latency hides behind the sweeps; with fewer threads (the tail kernel)
// the unknowns take several rounds with the same sums.
constexpr int COARSE_INV_PER_THREAD = (MAX_COARSE_UNKNOWNS + 7) / 8;

template <int NTH>
struct CoarseLds {
  double P0[CS0], B0[CS0], P1[CS1], B1[CS1], P2[CS2], B2[CS2];
  double sbc[MAX_COARSE_UNKNOWNS];
  double red[NTH / 64];
  unsigned char C0[CS0], C1[CS1], C2[CS2];
};

// The LDS levels of one member on NTH threads (the arithmetic does not depend on NTH).
template <typename T, int NTH>
__device__ __forceinline__ void mg_coarse_member(const CoarseArgs& a, int mem, CoarseLds<NTH>& S) {
  double* const P0 = S.P0;
  double* const B0 = S.B0;
  double* const P1 = S.P1;
  double* const B1 = S.B1;
  double* const P2 = S.P2;
  double* const B2 = S.B2;
  unsigned char* const C0 = S.C0;
  unsigned char* const C1 = S.C1;
  unsigned char* const C2 = S.C2;
  double* const sbc = S.sbc;
  double* const red = S.red;
  if (a.k > 0 && a.norms != nullptr) {
    const double prev = a.norms[(long)mem * a.norm_slots + a.k - 1];
    if (prev <= a.tol) {
      if (a.write_norm && threadIdx.x == 0) a.norms[(long)mem * a.norm_slots + a.k] = prev;
      return;
    }
  }
  const Geo g0 = a.g;
  const Geo g1 = g0.coarser();
  const Geo g2 = g1.coarser();
  const int ny0 = g0.ny, ny1 = g1.ny, ny2 = g2.ny;
  const long off = (long)mem * a.plane;
  const T* gphi = (const T*)a.phi + off;
  const T* gb = (const T*)a.b + off;
  // thread t owns the top-level cells (t & 63, (t >> 6) + RS k)
  constexpr int RS = NTH / 64;
  constexpr int NL = CMAXNY0 / RS;
  const int ti = threadIdx.x & 63, tj = threadIdx.x >> 6;
  static_assert((MAX_COARSE_UNKNOWNS * 8) % NTH == 0, "dense solve needs whole rounds of 8 threads per unknown");
  constexpr int DROUNDS = MAX_COARSE_UNKNOWNS * 8 / NTH;
  const int dpart = threadIdx.x & 7;
  // one round: this thread's entries of the transposed inverse, ainv[r * nc + q] for r = part + 8 k
  double inv_r[DROUNDS == 1 ? COARSE_INV_PER_THREAD : 1];
  if (DROUNDS == 1) {
    const int dq = threadIdx.x >> 3;
#pragma unroll
    for (int k = 0; k < COARSE_INV_PER_THREAD; ++k) {
      const int r = dpart + 8 * k;
      inv_r[k] = (dq < a.nc && r < a.nc) ? a.ainv[(long)r * a.nc + dq] : 0.0;
    }
  }
  {
    double vp[NL], vb[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int j = tj + RS * k;
      vp[k] = 0.0;
      vb[k] = 0.0;
      if (j < ny0 && g0.fluid(ti, j)) {
        vb[k] = (double)gb[g0.at(ti, j)];
        if (a.warm) vp[k] = (double)gphi[g0.at(ti, j)];
      }
    }
    for (int q = threadIdx.x; q < CS0; q += NTH) {
      P0[q] = 0.0;
      B0[q] = 0.0;
    }
    for (int q = threadIdx.x; q < CS1; q += NTH) {
      P1[q] = 0.0;
      B1[q] = 0.0;
    }
    for (int q = threadIdx.x; q < CS2; q += NTH) {
      P2[q] = 0.0;
      B2[q] = 0.0;
    }
    lvl_codes<CNX0, NTH>(C0, g0);
    lvl_codes<CNX1, NTH>(C1, g1);
    lvl_codes<CNX2, NTH>(C2, g2);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int j = tj + RS * k;
      if (j < ny0) {
        P0[cx<CNX0>(ti, j)] = vp[k];
        B0[cx<CNX0>(ti, j)] = vb[k];
      }
    }
  }
  __syncthreads();
  const double h20 = g0.h * g0.h, h21 = g1.h * g1.h;
  for (int s = 0; s < a.nsweep_pre; ++s) lvl_sweep<CNX0, NTH>(P0, B0, C0, ny0, h20);
  lvl_restrict<CNX0, NTH>(P0, B0, C0, g0.h, P1, B1, C1, ny1);
  for (int s = 0; s < a.nsweep_pre; ++s) lvl_sweep<CNX1, NTH>(P1, B1, C1, ny1, h21);
  lvl_restrict<CNX1, NTH>(P1, B1, C1, g1.h, P2, B2, C2, ny2);
  // dense solve on the coarsest level through the inverse
  for (int q = threadIdx.x; q < a.nc; q += NTH) {
    const int c = a.aidx[q];
    sbc[q] = B2[cx<CNX2>(c % g2.nx, c / g2.nx)];
  }
  __syncthreads();
#pragma unroll 1
  for (int rd = 0; rd < DROUNDS; ++rd) {
    // eight threads (consecutive lanes) per unknown, each summing every eighth term in order
    const int dq = (threadIdx.x >> 3) + rd * (NTH / 8);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < COARSE_INV_PER_THREAD; ++k) {
      const int r = dpart + 8 * k;
      if (dq < a.nc && r < a.nc) s += (DROUNDS == 1 ? inv_r[k] : a.ainv[(long)r * a.nc + dq]) * sbc[r];
    }
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    if (dq < a.nc && dpart == 0) {
      const int c = a.aidx[dq];
      P2[cx<CNX2>(c % g2.nx, c / g2.nx)] = s;
    }
  }
  __syncthreads();
  lvl_prolong<CNX1, NTH>(P1, C1, ny1, P2, C2);
  for (int s = 0; s < a.nsweep_post; ++s) lvl_sweep<CNX1, NTH>(P1, B1, C1, ny1, h21);
  lvl_prolong<CNX0, NTH>(P0, C0, ny0, P1, C1);
  for (int s = 0; s < a.nsweep_post; ++s) lvl_sweep<CNX0, NTH>(P0, B0, C0, ny0, h20);
  if (a.write_norm) {
    const double inv_h2 = 1.0 / h20;
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int j = tj + RS * k;
      if (j < ny0) {
        const int x = cx<CNX0>(ti, j);
        if (C0[x]) {
          const double rr = fabs(lvl_resid<CNX0>(P0, B0, C0, x, inv_h2)) * a.dt;
          m = (rr > m || rr != rr) ? rr : m;
        }
      }
    }
    m = wave_max(m);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = red[0];
      for (int w = 1; w < NTH / 64; ++w) mm = (red[w] > mm || red[w] != red[w]) ? red[w] : mm;
      a.norms[(long)mem * a.norm_slots + a.k] = mm;
    }
  }
  T* wphi = (T*)a.phi + off;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int j = tj + RS * k;
    if (j >= ny0) continue;
    const int x = cx<CNX0>(ti, j);
    if (!C0[x]) continue;
    if (a.add_to)
      a.add_to[off + g0.at(ti, j)] += P0[x];
    else
      wphi[g0.at(ti, j)] = (T)P0[x];
  }
}

template <typename T, bool ONE>
__global__ __launch_bounds__(COARSE_THREADS) void k_mg_coarse(Multi<CoarseArgs> ms) {
  __shared__ CoarseLds<COARSE_THREADS> S;
  int mem;
  const CoarseArgs& a = ms.template pick<ONE>(blockIdx.x, mem);
  mg_coarse_member<T, COARSE_THREADS>(a, mem, S);
}

// ---------------------------------------------------------------------------- tail passes
// Passes k0..k1 of one member per workgroup (256 threads): the level phases in the order of the
// level launches (pre on every tiled level, the LDS levels, post back up), each phase over the
// member's tiles in turn through the same tile bodies, with a barrier between tiles (the LDS is
// reused) and between phases (the next phase reads what this one wrote; a phase never reads what
// it writes, so the order of its tiles does not matter). The norm of the previous pass decides,
// as in the level kernels: a converged member carries it into the remaining slots and stops. With
// `book_member` the workgroup then writes its member's step record (the bookkeeping launch's work).
template <typename T>
__global__ __launch_bounds__(256) void k_mg_tail(TailArgs<T> ta) {
  constexpr int NS = mg_ns<T>();
  constexpr bool MIXED = sizeof(T) == sizeof(float);
  __shared__ union {
    PreLds<T, TAIL_ROWS> pre;
    PostLds<T, TAIL_ROWS> post;
    CoarseLds<256> coarse;
  } S;
  const int mem = blockIdx.x;
  const int L = ta.nlev;
  double* const nr = ta.pre[0].norms + (long)mem * ta.pre[0].norm_slots;
  const double tol = ta.pre[0].tol;
  for (int k = ta.k0; k <= ta.k1; ++k) {
    const double prev = __hip_atomic_load(nr + k - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // a converged member, or one whose residual is not a number (no pass can change that; its
    // record is the same: no slot at or below the tolerance)
    if (prev <= tol || prev != prev) {
      for (int q = k + (int)threadIdx.x; q <= ta.k1; q += 256) nr[q] = prev;
      break;
    }
    for (int l = 0; l < L; ++l) {
      MGArgs<T> a = ta.pre[l];
      a.k = k;
      if (MIXED && l == 0) {
        a.b = ta.rpl[(k - 1) & 1];
        a.r_out = ta.rpl[(k - 1) & 1];
      }
      for (int t = 0; t < a.ntiles; ++t) {
        if (MIXED && l == 0)
          mg_pre_tile<T, NS, PRE_LATER, TAIL_ROWS>(a, mem, t, S.pre);
        else
          mg_pre_tile<T, NS, PRE_PLAIN, TAIL_ROWS>(a, mem, t, S.pre);
        __syncthreads();
      }
    }
    {
      CoarseArgs c = ta.coarse;
      c.k = k;
      mg_coarse_member<T, 256>(c, mem, S.coarse);
      __syncthreads();
    }
    for (int l = L - 1; l >= 0; --l) {
      MGArgs<T> a = ta.post[l];
      a.k = k;
      if (MIXED && l == 0) {
        a.b = ta.rpl[(k - 1) & 1];
        a.r_out = ta.rpl[k & 1];
      }
      for (int t = 0; t < a.ntiles; ++t) {
        if (l > 0)
          mg_post_tile<T, NS, POST_PLAIN, TAIL_ROWS>(a, mem, t, S.post);
        else if (MIXED)
          mg_post_tile<T, NS, POST_REFINE, TAIL_ROWS>(a, mem, t, S.post);
        else
          mg_post_tile<T, NS, POST_NORM, TAIL_ROWS>(a, mem, t, S.post);
        __syncthreads();
      }
    }
  }
  if (ta.book_member) {
    __syncthreads();  // every norm slot of the step is written
    if (threadIdx.x == 0) step_book_member(ta.book, mem);
  }
}

static_assert(sizeof(TailArgs<double>) <= 4096, "tail arguments exceed the kernel argument space");
template <typename T>
void launch_mg_tail(const TailArgs<T>& a, int nmem, hipStream_t s) {
  hipLaunchKernelGGL((k_mg_tail<T>), dim3(nmem), dim3(256), 0, s, a);
}
template void launch_mg_tail<float>(const TailArgs<float>&, int, hipStream_t);
template void launch_mg_tail<double>(const TailArgs<double>&, int, hipStream_t);

// ---------------------------------------------------------------------------- FP64 residual (refinement)
template <bool ONE>
__global__ __launch_bounds__(256) void k_resid64(Multi<ResidArgs> ms) {
  constexpr int TW = TILE_W, TH = COST_TH;
  __shared__ double red[4];
  int item;
  const ResidArgs& a = ms.template pick<ONE>(xcd_remap(blockIdx.x, gridDim.x), item);
  const Geo& g = a.g;
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
template <typename T, int REF, int TR>
static void launch_mg_pre_(const Multi<MGArgs<T>>& m, hipStream_t s) {
  if (m.nseg == 1)
    hipLaunchKernelGGL((k_mg_pre<T, mg_ns<T>(), REF, true, TR>), dim3(m.total()), dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL((k_mg_pre<T, mg_ns<T>(), REF, false, TR>), dim3(m.total()), dim3(256), 0, s, m);
}
// every segment of one launch shares the tile height (the host groups segments by it)
template <typename T, int REF>
static void launch_mg_pre_rows(const Multi<MGArgs<T>>& m, hipStream_t s) {
  if (m.seg[0].trows == 8)
    launch_mg_pre_<T, REF, 8>(m, s);
  else if (m.seg[0].trows == 16)
    launch_mg_pre_<T, REF, 16>(m, s);
  else
    launch_mg_pre_<T, REF, 32>(m, s);
}
template <>
void launch_mg_pre<double>(const Multi<MGArgs<double>>& m, hipStream_t s) {
  launch_mg_pre_rows<double, PRE_PLAIN>(m, s);
}
template <>
void launch_mg_pre<float>(const Multi<MGArgs<float>>& m, hipStream_t s) {
  // every segment of a finest-level launch in mixed precision refines (one precision per batch),
  // and all of them are in the same pass
  if (m.seg[0].pre_mode == PRE_FIRST)
    launch_mg_pre_rows<float, PRE_FIRST>(m, s);
  else if (m.seg[0].pre_mode == PRE_LATER)
    launch_mg_pre_rows<float, PRE_LATER>(m, s);
  else
    launch_mg_pre_rows<float, PRE_PLAIN>(m, s);
}
template <typename T, int MODE, int TR>
static void launch_mg_post_(const Multi<MGArgs<T>>& m, hipStream_t s) {
  if (m.nseg == 1)
    hipLaunchKernelGGL((k_mg_post<T, mg_ns<T>(), MODE, true, TR>), dim3(m.total()), dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL((k_mg_post<T, mg_ns<T>(), MODE, false, TR>), dim3(m.total()), dim3(256), 0, s, m);
}
template <typename T, int MODE>
static void launch_mg_post_rows(const Multi<MGArgs<T>>& m, hipStream_t s) {
  const int tr = m.seg[0].trows;
  if (tr == 8)
    launch_mg_post_<T, MODE, 8>(m, s);
  else if (tr == 16)
    launch_mg_post_<T, MODE, 16>(m, s);
  else
    launch_mg_post_<T, MODE, 32>(m, s);
}
template <>
void launch_mg_post<double>(const Multi<MGArgs<double>>& m, int mode, hipStream_t s) {
  if (mode == POST_NORM)
    launch_mg_post_rows<double, POST_NORM>(m, s);
  else
    launch_mg_post_rows<double, POST_PLAIN>(m, s);
}
template <>
void launch_mg_post<float>(const Multi<MGArgs<float>>& m, int mode, hipStream_t s) {
  if (mode == POST_REFINE)
    launch_mg_post_rows<float, POST_REFINE>(m, s);
  else
    launch_mg_post_rows<float, POST_PLAIN>(m, s);
}
template <typename T>
void launch_mg_coarse(const Multi<CoarseArgs>& m, hipStream_t s) {
  if (m.nseg == 1)
    hipLaunchKernelGGL((k_mg_coarse<T, true>), dim3(m.total()), dim3(COARSE_THREADS), 0, s, m);
  else
    hipLaunchKernelGGL((k_mg_coarse<T, false>), dim3(m.total()), dim3(COARSE_THREADS), 0, s, m);
}
void launch_resid64(const Multi<ResidArgs>& m, hipStream_t s) {
  if (m.nseg == 1)
    hipLaunchKernelGGL(k_resid64<true>, dim3(m.total()), dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL(k_resid64<false>, dim3(m.total()), dim3(256), 0, s, m);
}

template void launch_mg_coarse<double>(const Multi<CoarseArgs>&, hipStream_t);
template void launch_mg_coarse<float>(const Multi<CoarseArgs>&, hipStream_t);

}  // namespace envar
