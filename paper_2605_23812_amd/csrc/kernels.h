// Kernel argument blocks and host launchers of the EnVar HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace envar {

// A launch carries up to MAX_SEG ensembles ("segments"): segment s owns the
// workgroups [start[s], start[s+1]) of the grid. Workgroup ids are first
// remapped for XCD locality, then looked up here.
constexpr int MAX_SEG = 8;
template <typename A>
struct Multi {
  int nseg;
  int start[MAX_SEG + 1];
  A seg[MAX_SEG];
  // ONE: the launch carries a single segment (known at compile time)
  template <bool ONE>
  __device__ __forceinline__ const A& pick(int wg, int& local) const {
    if (ONE) {
      local = wg;
      return seg[0];
    }
    int s = 0;
#pragma unroll
    for (int q = 1; q < MAX_SEG; ++q) s += (q < nseg && wg >= start[q]) ? 1 : 0;
    local = wg - start[s];
    return seg[s];
  }
  int total() const { return start[nseg]; }
};

// per-member statistics slots (FP64)
// ST_RECENT: a maximum of the cycles used that decays by 1/16 per step (drives the cycle cap)
enum { ST_CYCLES = 0, ST_MAXCYC, ST_UNCONV, ST_MAXRES, ST_STEPS, ST_J, ST_RECENT, STATS_STRIDE = 8 };

template <typename TT>
struct PredArgs {
  Geo g;
  Tiling tiling;
  int trows;                  // tile height of `tiling` (8 or 16)
  int ntiles, nmem;
  long plane;
  double nu, dt;
  const int* cold_flag;       // device flag: first step of a cold start (T^{-1} = T^0)
  const double* u;            // u^n, v^n
  const double* v;
  double* us;                 // u*, v*
  double* vs;
  const TT* tu_prev;          // T^{n-1}
  const TT* tv_prev;
  TT* tu;                     // T^n
  TT* tv;
  double* b;                  // div_h u* / dt
  const double* ctrl;         // [nmem][m] control rows, NULL = unforced
  long m;
  int nctrl;
  const int* cmap;            // control index of every cell (plane layout), -1 outside
  double* norms;              // [nmem][norm_slots], cleared here
  int norm_slots;
  // fused with the projection of the previous step: u, v above then hold u*^{n-1}, v*^{n-1};
  // u^n = u* - dt grad phi^{n-1} is rebuilt on the halo, and the previous step's cost sample,
  // divergence and warm start of this step's solve are produced here (see ProjArgs)
  int fused;
  const double* phi;          // phi^{n-1}
  double* phi_next;           // phi^{n-2} on entry -> warm start of this step's solve
  double* phi_old;            // phi^{n-3} on entry -> phi^{n-2}
  double* phi_old2;           // phi^{n-4} on entry -> phi^{n-3} (cubic warm start; NULL: quadratic)
  const double* stats;
  const double* shu;
  const double* shv;
  double* s1u;
  double* s1v;
  double* s2part;
  double* divmax;
  Tiling cost_tiling;
  int cost_ntiles;
  long cplane;
};

struct ProjArgs {
  Geo g;
  Tiling tiling;
  int trows;          // tile height of `tiling` (8 or 16)
  int ntiles, nmem;
  Tiling cost_tiling; // 64 x 8 cost blocks: s2part[mem][cost_ntiles]
  int cost_ntiles;
  long plane, cplane;
  double dt;
  double* u;
  double* v;
  const double* us;
  const double* vs;
  const double* phi;
  // optional warm start of the next solve, extrapolated from the pressures of the last steps:
  // phi_next holds phi^{n-1} on entry and receives the guess for phi^{n+1};
  // phi_old holds phi^{n-2} on entry and receives phi^{n-1}
  double* phi_next;
  double* phi_old;
  // phi^{n-3} on entry, receives phi^{n-2}: the cubic warm start (NULL: quadratic)
  double* phi_old2;
  const double* stats;  // [nmem][STATS_STRIDE]: steps done so far select the extrapolation order
  const double* shu;  // cost shift (dense cells, shared by members)
  const double* shv;
  double* s1u;        // [nmem][cplane] running sums of (u_c - s_c); NULL = no cost
  double* s1v;
  double* s2part;     // [nmem][cost_ntiles]
  double* divmax;     // [nmem] max |div u^{n+1}| (atomicMax on the bit pattern)
};

struct BookArgs {
  int nmem;
  int norm_slots;
  int cap;        // slots filled this step: cap + slot_base
  int slot_base;  // 0 (FP64: slot k = after V-cycle k) or 1 (mixed: slot 0 = initial residual)
  double tol;     // on dt * max|r|, in the units stored in norms
  const double* norms;
  double* stats;
};

// One member's step record: norms[mem][k] holds dt*max|r| after cycle k and a skipped cycle
// carries the previous value, so the first slot at or below tol ends the solve. Records the
// cycles run, the final residual and whether the tolerance was met.
__device__ __forceinline__ void step_book_member(const BookArgs& a, int mem) {
  const double* nr = a.norms + (long)mem * a.norm_slots;
  const int filled = a.cap + a.slot_base;
  int used = filled;
  for (int k = 0; k < filled; ++k)
    if (nr[k] <= a.tol) {
      used = k + 1;
      break;
    }
  const double last = nr[used - 1];
  const int cycles = used - a.slot_base;
  double* st = a.stats + (long)mem * STATS_STRIDE;
  st[ST_CYCLES] += (double)cycles;
  st[ST_MAXCYC] = fmax(st[ST_MAXCYC], (double)cycles);
  if (!(last <= a.tol)) st[ST_UNCONV] += 1.0;
  st[ST_MAXRES] = (last > st[ST_MAXRES] || last != last) ? last : st[ST_MAXRES];
  st[ST_STEPS] += 1.0;
  st[ST_RECENT] = fmax((double)cycles, st[ST_RECENT] - 1.0 / 16.0);
}

struct FinalArgs {
  Geo g;
  int nmem, ntiles;
  long cplane;
  long K;
  double dt, penalty;
  const double* s1u;
  const double* s1v;
  const double* s2part;
  const double* ctrl;
  long m;
  double* J;
  double* stats;
};

template <typename TT>
struct InitArgs {
  int nmem, ntiles;
  long plane, cplane;
  const double *bu, *bv, *btu, *btv, *bphi;
  double *u, *v, *us, *vs, *us2, *vs2, *phi, *phi2;
  TT *tu, *tv;
  double *s1u, *s1v, *s2part, *stats, *divmax;
};

// pre kernel at the finest level in mixed precision: the first pass forms the residual, later
// passes carry it (re-forming it while it is large)
enum { PRE_PLAIN = 0, PRE_FIRST = 1, PRE_LATER = 2 };

// multigrid level arguments (T = arithmetic / storage type of the level)
template <typename T>
struct MGArgs {
  Geo g, gc;          // this level and the next coarser one
  const unsigned char* code;   // this level: Poisson diagonal count of every cell (0 = not fluid), plane layout
  const unsigned char* codec;  // the coarser level
  Tiling tiling;
  int trows;          // tile height of `tiling` (8, 16 or 32): selects the kernel instance
  int ntiles, nmem;
  long plane, cplane_c;  // plane of this level and of the coarse level
  const T* phi_in;    // [nmem][plane] read (halo included); never written by this launch
  T* phi_out;         // [nmem][plane] written (tile interiors) -- ping-pong avoids inter-tile races
  const T* b;
  T* phic;            // coarse correction
  T* bc;              // coarse right-hand side
  double* add_to;     // post, mixed: phi64 += phi instead of storing phi (NULL = store)
  int zero_guess;     // pre: start from phi = 0
  // Mixed precision, finest level (iterative refinement of the FP64 pressure). The residual
  // r = b64 - L phi64 is carried across the passes of a step in two T planes (pass k reads one
  // as its right-hand side `b` and writes the other):
  //  * the first pass's pre kernel forms r in FP64 on its window from phi64 and b64, stores it
  //    (rounded to T) on its tile in r_out and puts dt*max|r| of the tile into norms[rslot] (slot 0);
  //  * the post kernel adds its correction e to phi64 and stores r - L e, formed in FP64 (e is
  //    exact on the tile and one ring around it), in r_out, with dt*max|r - L e| of the tile into
  //    norms[k]. The rounding of the stored residual (relative 6e-8 of a residual near the
  //    tolerance) stays far below the tolerance; the next step forms r afresh.
  const double* phi64;
  const double* b64;
  T* r_out;
  int rslot;
  double anchor;      // later passes: re-form the residual when the previous norm exceeds this
  int pre_mode;       // PRE_PLAIN | PRE_FIRST | PRE_LATER (selects the kernel instance)
  // convergence control: skip members whose previous cycle met tol
  double* norms;      // [nmem][norm_slots]
  int norm_slots;
  int k;              // this cycle's slot (skip when k > 0 and norms[k-1] <= tol)
  int write_norm;     // post at the finest level: write dt*max|r| into norms[k]
  double tol;         // on dt*max|r|
  double dt;          // residual scale for the stored norm
};

struct CoarseArgs {
  Geo g;              // top level handled in LDS (inv_h <= 16)
  int nlev;           // levels from the top down to inv_h = 4 (inclusive)
  int nmem;
  long plane;
  void* phi;          // [nmem][plane] of type T
  const void* b;
  int warm;           // start from the stored phi (top = finest level)
  double* add_to;     // mixed with no tiled level: phi64 += phi instead of storing phi
  const double* ainv; // dense inverse of the coarsest operator, transposed: ainv[r * nc + q] = A^{-1}[q][r]
  const int* aidx;    // cell (i + j * nx) of each coarsest unknown
  int nc;
  double* norms;
  int norm_slots;
  int k;
  int write_norm;
  double tol, dt;
  int nsweep_pre, nsweep_post;
};

struct ResidArgs {
  Geo g;
  Tiling tiling;
  int ntiles, nmem;
  long plane;
  const double* phi;  // FP64 pressure
  const double* b;    // FP64 right-hand side
  float* r;           // FP32 residual (right-hand side of the next correction)
  double* norms;
  int norm_slots;
  int k;
  double tol, dt;
};

template <typename TT>
void launch_predictor(const Multi<PredArgs<TT>>& m, hipStream_t s);
void launch_project_cost(const Multi<ProjArgs>& m, hipStream_t s);
void launch_step_book(const Multi<BookArgs>& m, hipStream_t s);
void launch_finalize_J(const FinalArgs& a, hipStream_t s);
template <typename TT>
void launch_init_members(const InitArgs<TT>& a, hipStream_t s);
void launch_shift(const Geo& g, const double* u, const double* v, double* shu, double* shv, hipStream_t s);
template <typename TT>
void launch_store_base(long plane, const double* u, const double* v, const TT* tu, const TT* tv, const double* phi,
                       double* bu, double* bv, double* btu, double* btv, double* bphi, hipStream_t s);
void launch_fields_out(const Geo& g, long plane, int nmem, const double* u, const double* v, double* out,
                       hipStream_t s);
void launch_clear_flag(int* flag, hipStream_t s);
void launch_stream_copy(const void* src, void* dst, long n16, hipStream_t s);

// velocity sensors (the vector observation): channel c = 2 s + component of sensor s;
// each sample is the bilinear combination of four active faces of its component,
// ((1 - ty) ((1 - tx) f00 + tx f01) + ty ((1 - tx) f10 + tx f11)), of the projected velocity
constexpr int OBS_CHANNELS = 8;
struct SensorArgs {
  Geo g;
  int nmem;
  long plane;
  double dt;
  const double* us;     // u*, v* of the step
  const double* vs;
  const double* phi;    // its solved pressure
  const double* stats;  // steps done (the sample index)
  double* obs;          // [nmem][OBS_CHANNELS][K]
  int K, every;
  int fi[OBS_CHANNELS][4], fj[OBS_CHANNELS][4];  // face (i, j) of f00, f01, f10, f11
  double tx[OBS_CHANNELS], ty[OBS_CHANNELS];
};
void launch_sensors(const Multi<SensorArgs>& m, hipStream_t s);

template <typename T>
void launch_mg_pre(const Multi<MGArgs<T>>& m, hipStream_t s);
// post kernel at the finest level: 0 plain, 1 the V-cycle's residual norm (FP64 cycles), 2 the
// refinement update of phi64 and of the carried residual (mixed precision)
enum { POST_PLAIN = 0, POST_NORM = 1, POST_REFINE = 2 };

template <typename T>
void launch_mg_post(const Multi<MGArgs<T>>& m, int mode, hipStream_t s);
template <typename T>
void launch_mg_coarse(const Multi<CoarseArgs>& m, hipStream_t s);
void launch_resid64(const Multi<ResidArgs>& m, hipStream_t s);

// The passes of a step beyond those launched level by level (the "tail"): one workgroup per
// member runs passes k0..k1 in order while the member's previous norm exceeds the tolerance, each
// phase over the member's tiles in turn with the tile bodies of the level kernels (16-row tiles)
// and the LDS levels on 256 threads, so a pass gives bitwise the result of its level launches.
// A member that has converged carries its norm through slots k..k1 and leaves at once, so the
// tail costs one launch when no member needs it. Jobs with 1 to TAIL_MAX_LEV tiled levels.
constexpr int TAIL_MAX_LEV = 4;
constexpr int TAIL_ROWS = 16;
template <typename T>
struct TailArgs {
  MGArgs<T> pre[TAIL_MAX_LEV];   // pass-independent fields; `k` (and, mixed, the finest level's
  MGArgs<T> post[TAIL_MAX_LEV];  // residual planes) are set per pass
  CoarseArgs coarse;
  T* rpl[2];  // mixed: the finest level's residual planes by pass parity (pass k reads k - 1, writes k)
  int nlev, k0, k1, mixed;
  BookArgs book;  // the step record of each member, written at the end (book_member), when set
  int book_member;
};
template <typename T>
void launch_mg_tail(const TailArgs<T>& a, int nmem, hipStream_t s);

// anomaly reduction
struct GramPlan {
  int n;          // rows of X (Gram is n x n)
  long m;         // contraction length
  int nsplit;     // split-K partials
  long kchunk;    // columns per split (a whole number of the Gram kernel's LDS chunks)
};
template <typename TX>
void launch_anomaly(const double* ctrl, const double* J, int n, long m, TX* X, double* dJ, hipStream_t s);
template <typename TX>
void launch_gram(const TX* X, int n, long m, long ldx, double* partial, int nsplit, long kchunk, hipStream_t s);
// the Gram's block rows (64 or 128) and the split of its contraction of length klen (elements of
// elem_bytes) that every caller sizes its partials by (nsplit x n x n doubles)
int gram_block_rows(int n);
void gram_split(int n, long klen, int elem_bytes, int& nsplit, long& kchunk);
int gram_reduce_groups(int nsplit);
void launch_gram_reduce(const double* partial, int n, int nsplit, double* tmp, double* G, hipStream_t s);
// (G + ridge_rel tr(G)/n I) x = rhs; G may be overwritten (n > 64). work[0] (int) <- 0, the first
// pivot that is not positive (1-based), or -1 when the pivots are fine but x is not finite.
// Returns 0, or -1 for n > 1024 and -2 when the launch could not be configured.
int launch_chol_solve(double* G, const double* rhs, int n, double* x, double* work, hipStream_t s,
                      double ridge_rel = 1e-12);
// vector-observation EnVar step and posterior variance
void launch_obs_fluct(const double* series, int rows, int channels, long K, double* D, hipStream_t s);
void launch_yrows(const double* D, int n, long n_obs, double eps, double* Y, hipStream_t s);
// out[i] = scale * A_i . B_i + add_coef * add[i], with B_i = B (shared) or row i of B (per_row_b)
void launch_rowdot(const double* A, const double* B, int rows, long len, double scale, const double* add,
                   double add_coef, double* out, hipStream_t s, bool per_row_b = false);
void launch_shift_diag(const double* G, int n, double shift, double* H, const double* grad, double* neg, hipStream_t s);
int launch_spd_inverse(const double* H, int n, double* C, double* work, hipStream_t s);
int launch_post_var(const double* ctrl, int n, long m, double eps, const double* C, double* var, hipStream_t s);
// rows[0] = fe + sum_i w_i E_i, rows[1 + i] = rows[0] + eps E_i for i < nrows - 1
// eigen-ensemble of the tapered Gaussian covariance (csrc/eigen.hip)
void launch_eig_sigma(const int* bidx, int ncc, int nxb, int nyb, double h, double sig2max, int taper, double* sig,
                      hipStream_t s);
void launch_kernel1d(int n, double h, double a, double* K, hipStream_t s);
void launch_eig_random(double* Q, int b, long M, const double* sig, unsigned long long seed, hipStream_t s);
void launch_scale_rows(const double* Q, const double* sig, int rows, long M, double* W, hipStream_t s);
void launch_dgemm(int M, int N, int K, const double* A, long lda, long sA, const double* B, long ldb, long sB,
                  double* C, long ldc, long sC, int batch, const double* S, long lds, hipStream_t s);
size_t jacobi_scratch_doubles(int n);
int launch_jacobi(const double* A, int lda, int n, double* evals, double* W, double* Wt, double* scratch,
                  hipStream_t s, int max_sweeps = 40);
int launch_chol_inv(const double* G, int n, double* Linv, double* scratch, hipStream_t s);
void launch_small_gemm(int n, const double* A, int ta, const double* B, int tb, const double* d, double* C,
                       hipStream_t s);
void launch_eig_blocks(const double* G, int b, double* T, double* ZZ, double* QQ, hipStream_t s);
void launch_eig_unit_gram(const double* P, int n, double* Gy, double* ninv, hipStream_t s);
void launch_eig_rsqrt(const double* lam, int n, double* d, hipStream_t s);
void launch_eig_resid(const double* U, const double* V, const double* theta, int N, long M, double* out,
                      hipStream_t s);
int eig_resid_split();  // slices per residual (partial sums of squares [N][slices])
void launch_eig_extract(const double* U, const double* theta, int N, long M, const int* bidx, int ncc, int comp,
                        double* E, double* mu, hipStream_t s);
long recon_blocks(long m);
void launch_recon(const double* E, int N, long m, const double* f, const double* ef, const double* ee, double* coef,
                  double* part, double* out, hipStream_t s);
// rows[t] = fe + sum_i W[t][i] E_i for t < nw
void launch_combine_rows(const double* fe, const double* E, int n, long m, const double* W, int nw, double* rows,
                         hipStream_t s);
void launch_build_rows(const double* fe, const double* E, int n, long m, const double* w, double eps, int nrows,
                       double* rows, hipStream_t s);
template <typename TX>
void launch_gemv_t(const TX* X, int n, long m, long ldx, const double* c, double* g, hipStream_t s);
// FP64 Gram partials and g = X^T c with the anomalies X_i = ctrl[i + 1] - ctrl[0] formed on the
// fly from the n + 1 control rows (no stored copy of X)
void launch_gram_anom(const double* ctrl, int n, long m, double* partial, int nsplit, long kchunk, hipStream_t s);
void launch_cost_anomaly(const double* J, int n, double* dJ, hipStream_t s);
void launch_gemv_anom(const double* ctrl, int n, long m, const double* c, double* g, hipStream_t s);
// out = pinv(A) rhs from A's eigenpairs (launch_jacobi's evals and W), eigenvalues at or below
// rcond times the largest dropped; n <= 512 (else -1); *info = 0, or -1 for a non-finite result
int launch_pinv_apply(const double* W, const double* ev, int n, const double* rhs, double* out, double rcond,
                      int* info, hipStream_t s);
template <typename TX>
void launch_transpose(const TX* X, int n, long m, TX* Xt, hipStream_t s);

}  // namespace envar
