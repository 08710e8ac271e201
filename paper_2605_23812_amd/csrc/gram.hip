// Anomaly reduction {delta f_i, J_i} -> g on the matrix cores.
//
// The ensemble gradient of eq. (gradient_EnVar), in its scalar-cost form,
// needs the minimum-norm least-squares solution of X g = dJ with
// X_i = f_i - f_0 (n x m, tall-skinny as m^T) and dJ_i = J_i - J_0:
//     G = X X^T (n x n),  G c = dJ,  g = X^T c.
// G is the only dense contraction of the hot path: 2 n^2 m flops over n m
// operands, so it runs on MFMA (v_mfma_f64_16x16x4f64, or
// v_mfma_f32_16x16x4f32 for FP32 operands) with a split over m and FP64
// partials reduced in a fixed order (two levels). The n x n solve is an FP64
// Cholesky in one workgroup (in the registers of four waves up to n = 64, in
// 32-column panels with MFMA trailing updates up to n = 256); the projection g = X^T c is a
// bandwidth-bound GEMV with FP64 accumulation.
#include "common.h"
#include "kernels.h"

namespace envar {

// ---------------------------------------------------------------------------- anomalies
template <typename TX>
__global__ void k_anomaly(const double* ctrl, const double* J, int n, long m, TX* X, double* dJ) {
  const int i = blockIdx.y;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < m; k += (long)gridDim.x * blockDim.x)
    X[(long)i * m + k] = (TX)(ctrl[(long)(i + 1) * m + k] - ctrl[k]);
  if (blockIdx.x == 0 && threadIdx.x == 0) dJ[i] = J[i + 1] - J[0];
}

// the cost anomalies dJ_i = J_{i+1} - J_0 alone, for a solve whose Gram and final product form the
// control anomalies where they read them
__global__ void k_cost_anomaly(const double* J, int n, double* dJ) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dJ[i] = J[i + 1] - J[0];
}

// ---------------------------------------------------------------------------- Gram on MFMA
// One workgroup (4 waves) computes a 64 x 64 block G[I0:I0+64, J0:J0+64] of
// one split's partial sum over columns [kbeg, kend). X rows are staged through
// LDS in KC-column chunks (rows padded by one element against bank
// conflicts); wave w owns rows I0 + 16w .. +16 and the four 16 x 16 tiles
// across J. MFMA operand layout (16x16x4): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the r-th result register of lane l holds D[row][l%16] with
// row = l/16 + 4 r for the FP64 instruction and 4 (l/16) + r for the FP32 one
// (measured on gfx950).
template <typename TX>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef double __attribute__((ext_vector_type(4))) V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return lane / 16 + 4 * r; }
};
template <>
struct MfmaAcc<float> {
  typedef float __attribute__((ext_vector_type(4))) V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

constexpr int GRAM_KC = 64;  // contraction columns per LDS chunk
constexpr int GRAM_REDUCE_GROUP = 32;  // splits summed per group in the first reduction level

template <typename TX>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float __attribute__((ext_vector_type(4))) T;
};
template <>
struct Vec16<double> {
  typedef double __attribute__((ext_vector_type(2))) T;
};

// Only the block pairs bi <= bj are computed; an off-diagonal block is written twice (as G[I][J] and
// transposed as G[J][I]), so G is exactly symmetric. The X rows are fetched as 16-byte vectors into
// registers one chunk ahead of the MFMA work on the chunk in LDS (a diagonal block fetches its rows
// once and uses them for both operands).
// BS: rows of a block, 64 or 128. Wave w owns the BS / 4 rows from I0 + w BS / 4 (BS / 64 row tiles
// of 16) against the BS / 16 column tiles of the J block; at each step of 4 along the contraction it
// reads its A fragments and the B fragments once and issues every tile's MFMA. 128-row blocks read
// each X row for fewer block pairs (at n = 256: two row blocks, three pairs, against four and ten).
// ANOM: row r of X is formed on the fly as X[r] - X0 (the anomaly of a control row about the
// centre row X0, the values k_anomaly would store), so that no copy of the anomalies is needed.
template <typename TX, bool ANOM = false, int BS = 64>
__global__ __launch_bounds__(256) void k_gram(const TX* __restrict__ X, int n, long m, long ldx,
                                              double* __restrict__ partial, int nsplit, long kchunk, int nbt,
                                              const TX* __restrict__ X0 = nullptr) {
  typedef typename MfmaAcc<TX>::V V;
  typedef typename Vec16<TX>::T VT;
  static_assert(BS == 64 || BS == 128, "64- or 128-row blocks");
  constexpr int KC = GRAM_KC, LDR = KC + 1;
  constexpr int VW = 16 / sizeof(TX);      // elements per vector
  constexpr int VPR = KC / VW;             // vectors per row and chunk
  constexpr int NV = BS * VPR / 256;       // vectors per thread and operand
  constexpr int RT = BS / 64;              // 16-row tiles per wave
  constexpr int CT = BS / 16;              // 16-column tiles
  __shared__ TX sa[BS * LDR];
  __shared__ TX sb[BS * LDR];
  const int split = blockIdx.x % nsplit;
  int pair = blockIdx.x / nsplit;
  int bi = 0;
  while (pair >= nbt - bi) {
    pair -= nbt - bi;
    ++bi;
  }
  const int bj = bi + pair;
  const bool diag = bi == bj;
  const int I0 = bi * BS, J0 = bj * BS;
  const long kbeg = (long)split * kchunk;
  long kend = kbeg + kchunk;
  if (kend > m) kend = m;
  // 16-byte vector loads need 16-byte aligned rows (control rows passed by the caller may not be)
  const bool vec = ldx % VW == 0 && (((uintptr_t)X | (uintptr_t)(ANOM ? X0 : X)) % 16) == 0;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  VT ra[NV], rb[NV];
  // the raw row values (0 outside the rows and the chunk); ANOM subtracts the centre row when the
  // chunk goes to LDS, so that the loads stay in flight during the MFMA work on the previous chunk
  auto load = [&](int row, long k) -> VT {
    if (row < n && vec && k + VW <= kend) return *(const VT*)(X + (long)row * ldx + k);
    VT v;
    for (int e = 0; e < VW; ++e) v[e] = row < n && k + e < kend ? X[(long)row * ldx + k + e] : (TX)0;
    return v;
  };
  // every vector of a thread covers the same columns of the chunk (256 is a multiple of VPR), so
  // one vector of the centre row serves all of them
  static_assert(256 % VPR == 0, "a thread's vectors share their columns");
  const int cth = (threadIdx.x % VPR) * VW;
  VT z{};
  auto fetch = [&](long k0) {
    if constexpr (ANOM) {
      const long k = k0 + cth;
      if (vec && k + VW <= kend)
        z = *(const VT*)(X0 + k);
      else
        for (int e = 0; e < VW; ++e) z[e] = k + e < kend ? X0[k + e] : (TX)0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int r = (threadIdx.x + 256 * v) / VPR;
      ra[v] = load(I0 + r, k0 + cth);
      if (!diag) rb[v] = load(J0 + r, k0 + cth);
    }
  };
  V acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = V{0, 0, 0, 0};
  if (kbeg < kend) fetch(kbeg);
  for (long k0 = kbeg; k0 < kend; k0 += KC) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int r = (threadIdx.x + 256 * v) / VPR;
      VT xa = ra[v], xb = rb[v];
      if constexpr (ANOM) {
        if (I0 + r < n) xa -= z;
        if (!diag && J0 + r < n) xb -= z;
      }
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        sa[r * LDR + cth + e] = xa[e];
        if (!diag) sb[r * LDR + cth + e] = xb[e];
      }
    }
    __syncthreads();
    if (k0 + KC < kend) fetch(k0 + KC);  // the next chunk's loads overlap this chunk's MFMA work
    const TX* sB = diag ? sa : sb;
    for (int kk = 0; kk < KC; kk += 4) {
      TX a[RT], b[CT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt] = sa[(16 * (wave * RT + rt) + lane % 16) * LDR + kk + lane / 16];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) b[ct] = sB[(16 * ct + lane % 16) * LDR + kk + lane / 16];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = MfmaAcc<TX>::mma(a[rt], b[ct], acc[rt][ct]);
    }
    __syncthreads();
  }
  double* P = partial + (long)split * n * n;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int j = J0 + 16 * ct + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I0 + 16 * (wave * RT + rt) + MfmaAcc<TX>::row(lane, r);
        if (i < n && j < n) {
          P[(long)i * n + j] = (double)acc[rt][ct][r];
          if (!diag) P[(long)j * n + i] = (double)acc[rt][ct][r];
        }
      }
    }
}

// Rows of a Gram block: 128 above n = 64 (three block pairs at n = 256 instead of ten, and each
// pair's MFMA work per loaded row doubles), else 64.
int gram_block_rows(int n) { return n > 64 ? 128 : 64; }

// Split of the contraction (at least one LDS chunk of columns). 64-row blocks: about
// 512 / nbt^2 splits. 128-row blocks: the registers of the FP64 kernel hold one workgroup per CU,
// those of the FP32 kernel two, so the grid stays at or below 256 or 512 workgroups (one more would
// run alone after the rest). A split is a whole number of LDS chunks, so that no MFMA work runs on
// zero padding inside the contraction.
void gram_split(int n, long klen, int elem_bytes, int& nsplit, long& kchunk) {
  const int bs = gram_block_rows(n);
  const long nbt = (n + bs - 1) / bs;
  const long slots = elem_bytes == 8 ? 256L : 512L;
  const long want = bs == 128 ? std::max(1L, slots / (nbt * (nbt + 1) / 2)) : std::max(1L, 512L / (nbt * nbt));
  long chunk = (klen + want - 1) / want;
  chunk = std::max((long)GRAM_KC, ((chunk + GRAM_KC - 1) / GRAM_KC) * GRAM_KC);  // whole LDS chunks
  kchunk = chunk;
  nsplit = (int)((klen + chunk - 1) / chunk);
}

// Fixed-order reduction of the split-K partials in two levels: groups of
// consecutive splits summed in order, then the group sums in order.
__global__ void k_gram_reduce_groups(const double* partial, long nn, int nsplit, int rg, double* tmp) {
  const int grp = blockIdx.y;
  const int p0 = grp * rg, p1 = min(nsplit, p0 + rg);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = p0; p < p1; ++p) s += partial[(long)p * nn + e];
    tmp[(long)grp * nn + e] = s;
  }
}

// Both levels in one launch when there are at most 16 groups (the split count stays below
// 512 for every layout here): a workgroup takes 16 consecutive entries, thread t sums group
// t / 16 of entry t % 16 with its 32 loads unrolled (clamped addresses, masked by a factor
// 0 or 1, so that no branch separates them), and 16 threads add the group sums from LDS.
// The order of the additions is the two-level order above, so the result is bitwise the same.
__global__ __launch_bounds__(256) void k_gram_reduce_fused(const double* partial, long nn, int nsplit,
                                                           double* G) {
  __shared__ double gs[16][16];
  const int t = threadIdx.x, el = t & 15, g = t >> 4;
  const long e = (long)blockIdx.x * 16 + el;
  const long ec = e < nn ? e : nn - 1;
  double sum = 0.0;
  if (g * GRAM_REDUCE_GROUP < nsplit) {
    double v[GRAM_REDUCE_GROUP];  // all loads first, then the additions in order
#pragma unroll
    for (int q = 0; q < GRAM_REDUCE_GROUP; ++q)
      v[q] = __builtin_nontemporal_load(&partial[(long)min(g * GRAM_REDUCE_GROUP + q, nsplit - 1) * nn + ec]);
#pragma unroll
    for (int q = 0; q < GRAM_REDUCE_GROUP; ++q) sum += v[q] * (g * GRAM_REDUCE_GROUP + q < nsplit ? 1.0 : 0.0);
  }
  gs[g][el] = sum;
  __syncthreads();
  if (t < 16 && e < nn) {
    const int ng = (nsplit + GRAM_REDUCE_GROUP - 1) / GRAM_REDUCE_GROUP;
    double s = 0.0;
    for (int q = 0; q < ng; ++q) s += gs[q][t];
    G[e] = s;
  }
}

__global__ void k_gram_reduce(const double* partial, int n, int nsplit, double* G) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += partial[(long)p * nn + e];
    G[e] = s;
  }
}

// ---------------------------------------------------------------------------- FP64 Cholesky solve
// Solves (G + ridge I) x = rhs, ridge = ridge_rel tr(G) / n, in one workgroup with
// one barrier per column (the fallback for n > CHOL_BLK_MAX). At step k every thread
// updates its entries of the trailing block with a_ik a_jk / a_kk from the still
// unscaled column k, so the factor is kept as A~ (column k as it stood at step k,
// pivot d_k = A~_kk) and G = A~ D^-1 A~^T, D = diag(d). The solves run right-looking
// on that form: A~ z = rhs, then A~^T x = D z. Threads form a 32-wide grid over the
// trailing block; thread j owns entry j of the vectors. The matrix is updated in place
// in global memory (L2 resident for the sizes allowed) as a full symmetric block, so
// that column k is read as row k.
constexpr int CHOL_VEC_MAX = 1024;

template <int NT>
__global__ __launch_bounds__(NT) void k_chol_solve(double* A, const double* rhs, int n, double* x, int* info,
                                                   double ridge_rel) {
  constexpr int RS = NT / 32;
  __shared__ double sv[CHOL_VEC_MAX];  // right-hand side, then z, then x
  __shared__ double sz[CHOL_VEC_MAX];
  __shared__ double sdi[CHOL_VEC_MAX];  // 1 / d_k
  __shared__ double ridge;
  const long ld = n;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  for (int i = tid; i < n; i += NT) sv[i] = rhs[i];
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += A[i * ld + i];
    ridge = ridge_rel * tr / (double)n;
    *info = 0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) A[i * ld + i] += ridge;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double akk = A[k * ld + k];
    if (tid == 0 && !(akk > 0.0)) *info = k + 1;
    const double inv = 1.0 / (akk > 0.0 ? akk : 1e-300);
    for (int i = k + 1 + ty; i < n; i += RS) {
      const double aik = A[k * ld + i] * inv;
      for (int j = k + 1 + tx; j < n; j += 32) A[i * ld + j] -= aik * A[k * ld + j];
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) {
    const double d = A[i * ld + i];
    sdi[i] = 1.0 / (d > 0.0 ? d : 1e-300);
  }
  __syncthreads();
  // A~ z = rhs (column k of A~ read as row k of the symmetric form)
  for (int k = 0; k < n; ++k) {
    const double zk = sv[k] * sdi[k];
    if (tid == 0) sz[k] = zk;
    for (int i = k + 1 + tid; i < n; i += NT) sv[i] -= A[k * ld + i] * zk;
    __syncthreads();
  }
  // A~^T x = D z: x_j = z_j - sum_{k>j} A~_kj x_k / d_j, right-looking over the rows of A~
  for (int i = tid; i < n; i += NT) sv[i] = sz[i];
  __syncthreads();
  for (int k = n - 1; k >= 0; --k) {
    const double xk = sv[k];
    for (int j = tid; j < k; j += NT) sv[j] -= A[k * ld + j] * xk * sdi[j];
    __syncthreads();
  }
  bool nonfinite = false;
  for (int i = tid; i < n; i += NT) {
    x[i] = sv[i];
    nonfinite = nonfinite || !isfinite(sv[i]);
  }
  if (__syncthreads_or(nonfinite) && tid == 0 && *info == 0) *info = -1;
}

// Blocked variant (n <= CHOL_BLK_MAX), same system: right-looking Cholesky G = L L^T in
// 32-column panels with the matrix in global memory (L2 resident) and the current panel in
// LDS. Per panel: all threads take the panel's 32 columns one barrier each (unscaled
// column steps over the diagonal block and the rows below it, then one scaling pass), the
// panel goes back to memory, and the trailing lower triangle takes the rank-32 update. The triangular solves are blocked the same way (the diagonal block by one wave,
// the off-diagonal blocks as GEMVs by all threads), so a panel costs a handful of barriers
// instead of one per column.
// orders one wave's LDS accesses across lanes (the diagonal-block solves run in wave 0 only)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr int CHOL_BS = 32;
constexpr int CHOL_BLK_MAX = 448;
constexpr int CHOL_PS = CHOL_BS + 1;  // panel row stride (odd: conflict-free row reads)
constexpr int CHOL_BLK_NT = 512;     // threads (the diagonal block keeps a 32-double row per lane in registers)

__global__ __launch_bounds__(CHOL_BLK_NT) void k_chol_blocked(double* A, const double* rhs, int n, double* x, int* info,
                                                       double ridge_rel) {
  __shared__ double P[CHOL_BLK_MAX * CHOL_PS];
  __shared__ double sv[CHOL_BLK_MAX];
  __shared__ double sq[CHOL_BS];
  __shared__ double ridge;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tid & 31, ty = tid >> 5;  // 32 x (CHOL_BLK_NT / 32) thread grid
  constexpr int RS = CHOL_BLK_NT / 32;
  const long ld = n;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += A[i * ld + i];
    ridge = ridge_rel * tr / (double)n;
    *info = 0;
  }
  for (int i = tid; i < n; i += CHOL_BLK_NT) sv[i] = rhs[i];
  __syncthreads();
  for (int i = tid; i < n; i += CHOL_BLK_NT) A[i * ld + i] += ridge;
  __threadfence_block();
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += CHOL_BS) {
    const int kw = min(CHOL_BS, n - k0), rows = n - k0;
    for (int r = ty; r < rows; r += RS)
      if (tx < kw) P[r * CHOL_PS + tx] = A[(k0 + r) * ld + k0 + tx];
    __syncthreads();
    // the panel's columns one barrier each, all threads, unscaled:
    // a_rj -= a_rc a_jc / a_cc for c < j <= r, j < kw; then column c scaled by 1 / sqrt(a_cc)
    for (int c = 0; c < kw; ++c) {
      const double d = P[c * CHOL_PS + c];
      if (tid == 0 && !(d > 0.0)) *info = k0 + c + 1;
      const double dinv = 1.0 / (d > 0.0 ? d : 1e-300);
      const int j = c + 1 + tx;
      if (j < kw)
        for (int r = c + 1 + ty; r < rows; r += RS)
          if (j <= r) P[r * CHOL_PS + j] -= P[r * CHOL_PS + c] * dinv * P[j * CHOL_PS + c];
      __syncthreads();
    }
    if (tid < kw) {
      const double d = P[tid * CHOL_PS + tid];
      sq[tid] = sqrt(d > 0.0 ? d : 1e-300);
    }
    __syncthreads();
    for (int r = ty; r < rows; r += RS)
      if (tx < kw && tx <= r) P[r * CHOL_PS + tx] = r == tx ? sq[tx] : P[r * CHOL_PS + tx] / sq[tx];
    __syncthreads();
    for (int r = ty; r < rows; r += RS)
      if (tx < kw && tx <= r) A[(k0 + r) * ld + k0 + tx] = P[r * CHOL_PS + tx];
    // rank-kw update of the trailing lower triangle
    for (int i = kw + ty; i < rows; i += RS)
      for (int j = kw + tx; j <= i; j += 32) {
        double t = 0.0;
        for (int c = 0; c < kw; ++c) t += P[i * CHOL_PS + c] * P[j * CHOL_PS + c];
        A[(k0 + i) * ld + k0 + j] -= t;
      }
    __threadfence_block();
    __syncthreads();
  }
  // L y = rhs (the diagonal block staged in P)
  for (int k0 = 0; k0 < n; k0 += CHOL_BS) {
    const int kw = min(CHOL_BS, n - k0);
    for (int r = ty; r < kw; r += RS)
      if (tx <= r) P[r * CHOL_PS + tx] = A[(k0 + r) * ld + k0 + tx];
    __syncthreads();
    if (wave == 0) {
      for (int c = 0; c < kw; ++c) {
        if (lane == c) sv[k0 + c] /= P[c * CHOL_PS + c];
        wave_sync();
        if (lane > c && lane < kw) sv[k0 + lane] -= P[lane * CHOL_PS + c] * sv[k0 + c];
        wave_sync();
      }
    }
    __syncthreads();
    for (int i = k0 + kw + tid; i < n; i += CHOL_BLK_NT) {
      double t = sv[i];
      for (int c = 0; c < kw; ++c) t -= A[i * ld + k0 + c] * sv[k0 + c];
      sv[i] = t;
    }
    __syncthreads();
  }
  // L^T x = y
  for (int k0 = ((n - 1) / CHOL_BS) * CHOL_BS; k0 >= 0; k0 -= CHOL_BS) {
    const int kw = min(CHOL_BS, n - k0);
    for (int r = ty; r < kw; r += RS)
      if (tx <= r) P[r * CHOL_PS + tx] = A[(k0 + r) * ld + k0 + tx];
    __syncthreads();
    if (wave == 0) {
      for (int c = kw - 1; c >= 0; --c) {
        if (lane == c) sv[k0 + c] /= P[c * CHOL_PS + c];
        wave_sync();
        if (lane < c) sv[k0 + lane] -= P[c * CHOL_PS + lane] * sv[k0 + c];
        wave_sync();
      }
    }
    __syncthreads();
    for (int i = tid; i < k0; i += CHOL_BLK_NT) {
      double t = sv[i];
      for (int c = 0; c < kw; ++c) t -= A[(k0 + c) * ld + i] * sv[k0 + c];
      sv[i] = t;
    }
    __syncthreads();
  }
  bool nonfinite = false;
  for (int i = tid; i < n; i += CHOL_BLK_NT) {
    x[i] = sv[i];
    nonfinite = nonfinite || !isfinite(sv[i]);
  }
  if (__syncthreads_or(nonfinite) && tid == 0 && *info == 0) *info = -1;
}

// ---------------------------------------------------------------------------- register Cholesky (n <= 64) and 32-column panels
// Same system, (G + ridge I) x = rhs, as the kernels above, through the plain
// factor G + ridge I = L L^T.
//
// lane l's value of v (l wave-uniform), as a scalar
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// lane src's value of v, for every lane (src may differ per lane)
__device__ __forceinline__ double bperm_d(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// wave_chol32 factors a symmetric 32 x 32 block in one wave, with no barrier and no LDS: lane
// (p, q) = (lane / 8, lane % 8) holds the entries (p + 8a, q + 8b) of the lower triangle in slot
// e[a][b], b <= a (in the diagonal slots, the entries with p < q are upper and never used). Step
// k: the lanes of column class k % 8 scale column k by r = 1 / sqrt(pivot) (the rows below k;
// the pivot's own entry becomes pivot * r = sqrt(pivot)), every lane fetches the multipliers of
// its four rows and four columns from those lanes (ds_bpermute, zero at rows <= k) and updates
// the slots that can still hold trailing entries (both indices >= 8 (k / 8)). The next pivot is
// formed from scalars read across lanes as soon as r is known, E(k+1, k+1) - (E(k+1, k) r)^2,
// bit for bit the value the update leaves, so that the pivot chain does not wait for the
// permutes: a step costs about one FP64 reciprocal square root and a few dependent operations.
// The eight steps of a block of columns share their code (a rolled loop, the last one apart):
// the kernel runs once per solve, and code that does not stay in the instruction cache is
// fetched again for every panel. On return the slots hold L (lower entries); rsv[k] =
// 1 / L[k][k] (written by lane 0). Returns (wave-uniform) the first step whose pivot is not
// positive, plus one, or 0.
// one step k = 8 KB + kq of wave_chol32; LAST: kq = 7, the next pivot lies in the next block
template <int KB, bool LAST>
__device__ __forceinline__ void wave_chol32_step(double (&e)[4][4], double* rsv, int kq, double& piv, int& bad) {
  const int lane = threadIdx.x & 63, p = lane >> 3, q = lane & 7;
  const int k = 8 * KB + kq;
  if (!(piv > 0.0) && bad == 0) bad = k + 1;
  const double pv = piv > 0.0 ? piv : 1e-300;
  const double r = rsqrt(pv);
  if (lane == 0) rsv[k] = r;
  if constexpr (!LAST) {  // the next pivot, (k + 1, k + 1), in this block
    const double l1 = readlane_d(e[KB][KB], (kq + 1) * 8 + kq) * r;
    piv = fma(-l1, l1, readlane_d(e[KB][KB], (kq + 1) * 9));
  } else if constexpr (KB < 3) {  // (8 KB + 8, 8 KB + 8): row class 0 of the next block
    const double l1 = readlane_d(e[KB + 1][KB], 7) * r;
    piv = fma(-l1, l1, readlane_d(e[KB + 1][KB + 1], 0));
  }
  double lval[4];
#pragma unroll
  for (int a = KB; a < 4; ++a) {
    const int i = p + 8 * a;
    const double l = e[a][KB] * r;
    lval[a] = (q == kq && i > k) ? l : 0.0;
    e[a][KB] = q == kq ? (i > k ? l : (i == k ? pv * r : e[a][KB])) : e[a][KB];
  }
  double lr[4], lc[4];
#pragma unroll
  for (int a = KB; a < 4; ++a) {
    lr[a] = bperm_d(lval[a], p * 8 + kq);
    lc[a] = bperm_d(lval[a], q * 8 + kq);
  }
#pragma unroll
  for (int a = KB; a < 4; ++a)
#pragma unroll
    for (int b = KB; b <= a; ++b) e[a][b] = fma(-lr[a], lc[b], e[a][b]);
}
template <int KB>
__device__ __forceinline__ void wave_chol32_block(double (&e)[4][4], double* rsv, double& piv, int& bad) {
#pragma unroll 1
  for (int kq = 0; kq < 7; ++kq) wave_chol32_step<KB, false>(e, rsv, kq, piv, bad);
  wave_chol32_step<KB, true>(e, rsv, 7, piv, bad);
}
__device__ __forceinline__ int wave_chol32(double (&e)[4][4], double* rsv) {
  int bad = 0;
  double piv = readlane_d(e[0][0], 0);
  wave_chol32_block<0>(e, rsv, piv, bad);
  wave_chol32_block<1>(e, rsv, piv, bad);
  wave_chol32_block<2>(e, rsv, piv, bad);
  wave_chol32_block<3>(e, rsv, piv, bad);
  return bad;
}

// n <= 64: four waves, wave w holding rows 16w..16w+15 of every column (lane j: column j).
// Step k: the wave that holds row k reads the pivot from lane k (its own register, updated in
// its previous step), scales row k by rsqrt(a_kk) (l_j = a_kj / sqrt(a_kk) for lanes j > k)
// and broadcasts it through LDS with zeros for j <= k; after one workgroup barrier every wave
// subtracts l_i l_j from its rows, where the zeros leave finished rows and finished columns as
// they are. The product is the same for (i, j) and (j, i), so the trailing block stays exactly
// symmetric. Against the one-wave form (one lane holding a whole column, 64 updates per lane per
// step) each step costs 16 updates per lane and one barrier: 27 against 37 us at n = 64 for the
// factor and both solves. Afterwards row k holds, for lane j,
// L[j][k] (j > k), the pivot (j = k) or the trailing entry A^(j)[k][j] (j < k), so that
// L[k][j] = row_k[j] / L[j][j]; wave 0 then runs both solves with the rows in LDS, the pivots'
// reciprocals and the running right-hand side read across lanes.
__global__ __launch_bounds__(256) void k_chol_wave(const double* G, const double* rhs, int n, double* x, int* info,
                                                   double ridge_rel) {
  __shared__ double cb[2][64];
  __shared__ double sT[64 * 64];
  __shared__ double srs[64];
  __shared__ int sbad[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double dg = lane < n ? G[(long)lane * n + lane] : 0.0;
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += readlane_d(dg, i);
  const double ridge = ridge_rel * tr / (double)n;
  // lower triangle only, mirrored: the factored matrix is symmetric by construction. Every
  // load is unconditional (clamped address) and masked arithmetically, fma(g, 1, ridge or 0)
  // or fma(g, 0, 1 or 0): a select on the loaded value is turned into a branch around each
  // load, and the loads then run one after another.
  const int lc = min(lane, n - 1);
  double a[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 16 * w + r;
    const int ic = min(i, n - 1);
    const double g = G[(long)max(ic, lc) * n + min(ic, lc)];
    const bool in = i < n && lane < n;
    a[r] = fma(g, in ? 1.0 : 0.0, i == lane ? (in ? ridge : 1.0) : 0.0);
  }
  int bad = 0;
  const double* const crow = &cb[0][16 * w];
  // steps k = 16 blk + st: wave blk holds row k in a[st] (a static register index)
  const int nblk = (n + 15) >> 4;
  for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int k = 16 * blk + st;
      if (k < n) {  // workgroup-uniform
        if (w == blk) {
          const double piv = readlane_d(a[st], k);
          if (!(piv > 0.0) && bad == 0) bad = k + 1;
          const double pv = piv > 0.0 ? piv : 1e-300;
          const double r = rsqrt(pv);
          const double t = a[st] * r;
          cb[st & 1][lane] = lane > k ? t : 0.0;
          if (lane == k) srs[k] = r;
          a[st] = lane > k ? t : a[st];
        }
        __syncthreads();  // two broadcast buffers: a wave still reading step k - 1's is past this barrier
        // every wave updates all its rows: the zero multipliers of rows i <= k leave them as they
        // are, and a test per row or per wave costs more than the updates it saves (27 against
        // 30 to 40 us at n = 64)
        const double tt = cb[st & 1][lane];
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = fma(-crow[(st & 1) * 64 + r], tt, a[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) sT[(16 * w + r) * 64 + lane] = a[r];
  if (lane == 0) sbad[w] = bad;
  __syncthreads();
  if (w != 0) return;
  int first = 0;  // the first failing step over the waves (each tests only its own rows)
  for (int q = 0; q < 4; ++q)
    if (sbad[q] != 0 && (first == 0 || sbad[q] < first)) first = sbad[q];
  const double rs = lane < n ? srs[lane] : 1.0;
  const double b = rhs[lc];
  double v = lane < n ? b : 0.0;
  for (int k = 0; k < n; ++k) {
    const double yk = readlane_d(v * rs, k);
    const double l = sT[k * 64 + lane];
    v = lane == k ? yk : lane > k ? fma(-l, yk, v) : v;
  }
  for (int k = n - 1; k >= 0; --k) {
    const double xk = readlane_d(v * rs, k);
    const double l = sT[k * 64 + lane] * rs;
    v = lane == k ? xk : lane < k ? fma(-l, xk, v) : v;
  }
  if (lane < n) x[lane] = v;
  const bool nonfinite = __any(lane < n && !isfinite(v));
  if (lane == 0) *info = first != 0 ? first : nonfinite ? -1 : 0;
}

// 64 < n <= CHOL_M32_MAX: right-looking in 32-column panels in one workgroup of four waves (one
// per SIMD, so that each has the whole register file: 256 VGPRs and 256 AGPRs), with the
// trailing matrix held, negated, in registers as MFMA accumulators. The system is padded to
// n_p = 32 ceil(n / 32) with an identity block (its factor is the identity, its part of y and x
// is zero), so every panel is full and every tile whole. G is read once, through a buffer
// resource of n^2 doubles whose range check returns zero for a padded row of the lower triangle
// (row >= n puts the offset row n + col past the end). The 16 x 16 tiles (ti, tj) of the lower
// triangle below the first panel (2 <= tj <= ti < n_p / 16) are dealt in (tj, ti) order, tile q
// to wave q mod 4 as its register slot q div 4; the tiles still trailing at panel p are those
// with tj >= 2p + 2, a suffix q >= q0(p) of that order, so each panel's update is balanced over
// the waves to within one tile. Each panel's 32 columns (all rows from its diagonal down) live
// in an LDS buffer, two of them used in turn. Per panel p, three barriers (LDS only: the stores
// of L to G are waited for once, before the backward solve):
//   1. wave 0 factors the diagonal block L11 in registers (wave_chol32, the block spread over
//      all 64 lanes) from the buffer, keeps it (column-major) in LDS with the pivots'
//      reciprocals and stores it to G;
//   2. one thread per row below solves L11 l^T = a^T right-looking with L11 broadcast from LDS
//      (32 doubles in registers) and writes the row of L21 over its input in the buffer and to
//      G; one more thread solves the right-hand side's block the same way (y's block: the
//      forward solve L y = rhs rides along as one more row);
//   3. the rows below take rhs_i -= l_i . y, and every wave adds L21 L21^T to its (negated)
//      trailing tiles with v_mfma_f64_16x16x4f64 (A operand: L21 rows of tile row ti; B
//      operand: L21 rows of tile row tj), then stores the tiles of the next panel's two tile
//      columns, negated back, into the other buffer. Lane l supplies A[l%16][kk] and
//      B[kk][l%16], kk = l/16; instruction s gives it the panel column c = 8 kk + s, so each
//      lane reads eight consecutive doubles of one buffer row (four 16-byte LDS reads per
//      operand); any assignment of the 32 columns to (kk, s) gives the same sum of products.
// The backward solve L^T x = y runs block by block from the last, each block's rows of L staged
// in LDS while the block before is solved: wave 0 the diagonal block (its columns in registers,
// the running right-hand side read across lanes), then the rows above as a GEMV.
// Scheduling notes, measured: the kernel runs once per solve, mostly straight-line code, and
// code that does not stay in the instruction cache is fetched again for every panel, so it is
// kept compact (one short block per register slot, the tile coordinates in an LDS table, the
// diagonal factor's steps rolled within blocks of eight). Left to itself the scheduler issues
// each LDS read at its first use and waits for it there (about 120 cycles a read); the reads of
// a panel row's column, of the backward block and of the first panel are therefore issued
// together ahead of their uses (scheduling barriers keep them there). At n = 256 the kernel
// takes about 175 us (the 64-column kernel it replaced: 425 us), of which about 60 us are the
// eight diagonal factors, each a chain of 32 FP64 reciprocal square roots.
constexpr int CHOL_M32_MAX = 256;
constexpr int CHOL_M32_NT = 256;
constexpr int CHOL_M32_NW = CHOL_M32_NT / 64;
constexpr int CHOL_M32_SLOTS = 27;  // ceil(105 / 4): the tiles below the first panel at n_p = 256
constexpr int CHOL_M32_PS = 34;     // buffer row stride, doubles: 16-byte rows, 16 rows span all banks
constexpr int CHOL_M32_R0 = CHOL_M32_MAX;       // rows of buffer 0 (the first panel: all rows)
constexpr int CHOL_M32_R1 = CHOL_M32_MAX - 32;  // rows of buffer 1 (odd panels)
constexpr int CHOL_M32_LDS = (CHOL_M32_R0 + CHOL_M32_R1) * CHOL_M32_PS * (int)sizeof(double);
static_assert((CHOL_M32_MAX / 16 - 2) * (CHOL_M32_MAX / 16 - 1) / 2 <= CHOL_M32_SLOTS * CHOL_M32_NW, "slots");
static_assert(CHOL_M32_NT > CHOL_M32_MAX - 32, "one thread per panel row and one for the right-hand side");

__device__ __forceinline__ double buf_load_d(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// workgroup barrier that orders LDS only (global stores stay in flight)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__global__ __launch_bounds__(CHOL_M32_NT) void k_chol_m32(double* A, const double* rhs, int n, double* x, int* info,
                                                      double ridge_rel) {
  __shared__ __align__(16) double sLc[32 * 32];  // sLc[c * 32 + k] = L11[k][c]
  __shared__ double sR[32];        // 1 / L11[c][c]
  __shared__ double sridge;
  __shared__ double sv[CHOL_M32_MAX];                    // rhs -> y -> x (zero in the padding)
  __shared__ int stab[CHOL_M32_NW * CHOL_M32_SLOTS];     // tile q: ti | tj << 8
  extern __shared__ __align__(16) double Pbuf[];         // two panel buffers, row r = the panel's row k0 + r
  constexpr int PS = CHOL_M32_PS;
  typedef double __attribute__((ext_vector_type(4))) acc4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, kk = lane >> 4;
  const long ld = n;
  const int np = (n + 31) & ~31, T = np >> 4, ntile = (T - 2) * (T - 1) / 2;
  const __amdgpu_buffer_rsrc_t gr = __builtin_amdgcn_make_buffer_rsrc(A, 0, n * n * (int)sizeof(double), 0x00020000);
  if (tid < CHOL_M32_NW * CHOL_M32_SLOTS) {  // the tile order: column tj = 2, 3, ... of the tile grid
    int q = tid, c = 2;
    while (c < T && q >= T - c) {
      q -= T - c;
      ++c;
    }
    stab[tid] = (c + q) | (c << 8);
  }
  if (wave == 0) {  // trace: four clamped loads per lane, then a fixed shuffle tree
    double tr = 0.0;
#pragma unroll
    for (int q = 0; q < CHOL_M32_MAX / 64; ++q) {
      const int i = lane + 64 * q, ic = min(i, n - 1);
      const double d = buf_load_d(gr, ic * (n + 1) * (int)sizeof(double), 0);
      tr += i < n ? d : 0.0;
    }
    tr = wave_sum(tr);
    if (lane == 0) {
      sridge = ridge_rel * tr / (double)n;
      *info = 0;
    }
  }
  // the first panel into buffer 0 (lower triangle mirrored; padded rows load as zero), without
  // the ridge (wave 0 adds it to the first diagonal block)
  double* const B0 = Pbuf;
  {
    constexpr int Q = CHOL_M32_MAX * 32 / CHOL_M32_NT;
    double g[Q];  // all loads in flight at once (an offset past n^2 reads zero)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + CHOL_M32_NT * q, i = e >> 5, j = e & 31;
      g[q] = buf_load_d(gr, (max(i, j) * n + min(i, j)) * (int)sizeof(double), 0);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + CHOL_M32_NT * q, i = e >> 5, j = e & 31;
      if (i < np) B0[i * PS + j] = g[q];
    }
  }
  for (int i = tid; i < np; i += CHOL_M32_NT) sv[i] = i < n ? rhs[i] : 0.0;
  lds_barrier();
  // the trailing tiles, negated, into their registers, a group of slots at a time (all loads of a
  // group in flight together; a slot without a tile reads past the end, zeros); the diagonal
  // takes the ridge, and the padding's identity (its entries load as zero)
  int loff[4];  // byte offset of this lane's entries within a tile
#pragma unroll
  for (int r = 0; r < 4; ++r) loff[r] = ((kk + 4 * r) * n + li) * (int)sizeof(double);
  acc4 acc[CHOL_M32_SLOTS];
  constexpr int GRP = 9;
#pragma unroll
  for (int g0 = 0; g0 < CHOL_M32_SLOTS; g0 += GRP) {
#pragma unroll
    for (int s = g0; s < g0 + GRP && s < CHOL_M32_SLOTS; ++s) {
      const int q = CHOL_M32_NW * s + wave;
      const int t = __builtin_amdgcn_readfirstlane(stab[q]), ti = t & 255, tj = t >> 8;
      const int tb = q < ntile ? (16 * ti * n + 16 * tj) * (int)sizeof(double) : n * n * (int)sizeof(double);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[s][r] = buf_load_d(gr, tb + loff[r], 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    const double ridge = sridge;
#pragma unroll
    for (int s = g0; s < g0 + GRP && s < CHOL_M32_SLOTS; ++s) {
      const int q = CHOL_M32_NW * s + wave;
      const int t = __builtin_amdgcn_readfirstlane(stab[q]), ti = t & 255, tj = t >> 8;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti + kk + 4 * r;
        const bool dg = q < ntile && ti == tj && row == 16 * tj + li;
        acc[s][r] = dg ? (row < n ? -(acc[s][r] + ridge) : -1.0) : -acc[s][r];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  int q0 = 0;  // the first tile of the order still trailing
  for (int p = 0; 32 * p < np; ++p) {
    const int k0 = 32 * p, R = np - k0;  // rows of this panel, its diagonal block included
    double* const Bp = Pbuf + (p & 1) * CHOL_M32_R0 * PS;
    double* const Bn = Pbuf + ((p + 1) & 1) * CHOL_M32_R0 * PS;
    // 1. the diagonal block
    if (wave == 0) {
      // opaque per panel: otherwise the offsets below are hoisted out of the panel loop, and
      // spilled
      int pq = lane;
      asm volatile("" : "+v"(pq));
      const int pp = pq >> 3, qq = pq & 7;
      double e[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          const int i = pp + 8 * a, j = qq + 8 * b;
          e[a][b] = Bp[max(i, j) * PS + min(i, j)] + (p == 0 && i == j ? sridge : 0.0);
        }
      const int bad = wave_chol32(e, sR);
      if (lane == 0 && bad != 0 && *info == 0) *info = k0 + bad;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          const int i = pp + 8 * a, j = qq + 8 * b;
          if (i >= j) {
            sLc[j * 32 + i] = e[a][b];
            if (k0 + i < n) A[(k0 + i) * ld + k0 + j] = e[a][b];
          }
        }
    }
    lds_barrier();
    // 2. the rows below and the right-hand side's block. Column c's multipliers L11[k][c]
    // (k > c, 16-byte reads) are all read before its updates, which then wait for each read in
    // turn (LDS returns in order); left to itself the scheduler issues each read at its first use
    // and waits for it there.
    const int nrow = R - 32;
    if (tid <= nrow) {
      const bool isrhs = tid == nrow;
      double ar[32];
      const double* const src = Bp + (32 + min(tid, nrow - 1)) * PS;
#pragma unroll
      for (int c = 0; c < 32; c += 2) {
        const double2 g = nrow > 0 ? *(const double2*)(src + c) : make_double2(0.0, 0.0);
        ar[c] = isrhs ? sv[k0 + c] : g.x;
        ar[c + 1] = isrhs ? sv[k0 + c + 1] : g.y;
      }
#pragma unroll
      for (int c = 0; c < 32; ++c) {
        // column c's multipliers, all reads issued before the updates that wait for them
        double lv[32];
        const double rc = sR[c];
#pragma unroll
        for (int k = (c + 1) & ~1; k < 32; k += 2) {
          const double2 v = *(const double2*)(sLc + c * 32 + k);
          lv[k] = v.x;
          lv[k + 1] = v.y;
        }
        __builtin_amdgcn_sched_barrier(0);
        ar[c] *= rc;
#pragma unroll
        for (int k = c + 1; k < 32; ++k) ar[k] = fma(-lv[k], ar[c], ar[k]);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (isrhs) {
#pragma unroll
        for (int c = 0; c < 32; ++c) sv[k0 + c] = ar[c];
      } else {
        double* const dst = Bp + (32 + tid) * PS;
#pragma unroll
        for (int c = 0; c < 32; c += 2) *(double2*)(dst + c) = make_double2(ar[c], ar[c + 1]);
        if (k0 + 32 + tid < n) {
          double* const g = A + (long)(k0 + 32 + tid) * ld + k0;
#pragma unroll
          for (int c = 0; c < 32; ++c) g[c] = ar[c];
        }
      }
    }
    lds_barrier();
    // 3. the right-hand side below, then the trailing tiles
    if (tid < nrow) {
      double t = sv[k0 + 32 + tid];
      const double* const row = Bp + (32 + tid) * PS;
#pragma unroll
      for (int c = 0; c < 32; c += 2) {
        const double2 l = *(const double2*)(row + c);
        t = fma(-l.x, sv[k0 + c], t);
        t = fma(-l.y, sv[k0 + c + 1], t);
      }
      sv[k0 + 32 + tid] = t;
    }
#pragma unroll
    for (int s = 0; s < CHOL_M32_SLOTS; ++s) {
      const int q = CHOL_M32_NW * s + wave;
      if (q >= q0 && q < ntile) {  // wave-uniform
        const int t = __builtin_amdgcn_readfirstlane(stab[q]), ti = t & 255, tj = t >> 8;
        const double* const pa = Bp + (16 * (ti - 2 * p) + li) * PS + 8 * kk;
        const double* const pb = Bp + (16 * (tj - 2 * p) + li) * PS + 8 * kk;
        double2 va[4], vb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          va[c] = *(const double2*)(pa + 2 * c);
          vb[c] = *(const double2*)(pb + 2 * c);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[c].x, vb[c].x, acc[s], 0, 0, 0);
          acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[c].y, vb[c].y, acc[s], 0, 0, 0);
        }
        if (tj <= 2 * p + 3) {  // a tile of the next panel: into the other buffer
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Bn[(16 * (ti - 2 * p - 2) + kk + 4 * r) * PS + 16 * (tj - 2 * p - 2) + li] = -acc[s][r];
        }
      }
    }
    q0 += 2 * (T - 2 * p) - 5;  // the tiles of columns 2p + 2 and 2p + 3 leave the trailing matrix
    lds_barrier();
  }
  __threadfence_block();  // L in G, visible to the whole workgroup
  __syncthreads();
  // L^T x = y, block by block from the last; each block's 32 rows of L are staged in LDS (one
  // row per CHOL_M32_MAX doubles, thread t taking column t of every row) from registers that were
  // loaded while the block before was being solved
  double* const Lb = Pbuf;
  constexpr int LS = CHOL_M32_MAX;
  const int kl = ((n - 1) / 32) * 32, tc = min(tid, n - 1);
  double lv[32];
#pragma unroll
  for (int c = 0; c < 32; ++c)
    lv[c] = buf_load_d(gr, tc * (int)sizeof(double), (kl + min(c, n - 1 - kl)) * n * (int)sizeof(double));
  for (int k0 = kl; k0 >= 0; k0 -= 32) {
    const int kw = min(32, n - k0);
#pragma unroll
    for (int c = 0; c < 32; ++c) Lb[c * LS + tid] = lv[c];
    lds_barrier();
    if (k0 >= 32) {  // the next block's rows, in flight while this one is solved
#pragma unroll
      for (int c = 0; c < 32; ++c)
        lv[c] = buf_load_d(gr, tc * (int)sizeof(double), (k0 - 32 + c) * n * (int)sizeof(double));
    }
    if (wave == 0) {
      const int lc = min(lane, kw - 1);
      double a[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) a[k] = Lb[min(k, kw - 1) * LS + k0 + lc];
      const double dg = Lb[lc * LS + k0 + lc], b = sv[k0 + lc];
      __builtin_amdgcn_sched_barrier(0);
      // unmasked: a padding lane k >= kw keeps v = 0 (its updates are finite entries times
      // zero), so x_k = 0 and the clamped entries it meets change nothing
      const double rs = lane < kw ? 1.0 / dg : 1.0;
      double v = lane < kw ? b : 0.0;
#pragma unroll
      for (int k = 31; k >= 0; --k) {
        const double xk = readlane_d(v * rs, k);
        v = lane == k ? xk : lane < k ? fma(-a[k], xk, v) : v;
      }
      if (lane < kw) sv[k0 + lane] = v;
    }
    lds_barrier();
    if (tid < k0) {  // k0 < CHOL_M32_NT: one row of the system per thread
      double l[32], xs[32];
#pragma unroll
      for (int c = 0; c < 32; ++c) {
        l[c] = Lb[c * LS + tid];
        xs[c] = sv[k0 + c];
      }
      __builtin_amdgcn_sched_barrier(0);
      double t = sv[tid];
#pragma unroll
      for (int c = 0; c < 32; ++c) t = fma(c < kw ? -l[c] : 0.0, xs[c], t);
      sv[tid] = t;
    }
    lds_barrier();
  }
  bool nonfinite = false;
  for (int i = tid; i < n; i += CHOL_M32_NT) {
    x[i] = sv[i];
    nonfinite = nonfinite || !isfinite(sv[i]);
  }
  if (__syncthreads_or(nonfinite) && tid == 0 && *info == 0) *info = -1;
}

// ---------------------------------------------------------------------------- GEMVs
// g[k] = sum_i X[i][k] c[i]: 64 columns per block, four row groups summed in order
// ANOM: X[i] - X0 on the fly, as in k_gram
template <typename TX, bool ANOM = false>
__global__ __launch_bounds__(256) void k_gemv_t(const TX* __restrict__ X, int n, long m, long ldx,
                                                const double* __restrict__ c, double* __restrict__ g,
                                                const TX* __restrict__ X0 = nullptr) {
  __shared__ double part[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (long k0 = blockIdx.x * 64L; k0 < m; k0 += (long)gridDim.x * 64L) {
    const long k = k0 + tx;
    double s = 0.0;
    if (k < m) {
      const TX x0 = ANOM ? X0[k] : (TX)0;
#pragma unroll 4
      for (int i = ty; i < n; i += 4) s += (double)(ANOM ? X[(long)i * ldx + k] - x0 : X[(long)i * ldx + k]) * c[i];
    }
    part[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && k < m) g[k] = ((part[0][tx] + part[1][tx]) + part[2][tx]) + part[3][tx];
    __syncthreads();
  }
}

template <typename TX>
__global__ void k_transpose(const TX* X, int n, long m, TX* Xt) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)n * m; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / m);
    const long k = e % m;
    Xt[k * n + i] = X[e];
  }
}

// ---------------------------------------------------------------------------- pseudo-inverse solve
// out = W diag(1 / lambda_k, lambda_k > rcond lambda_0; else 0) W^T rhs for the eigenpairs of a
// symmetric n x n matrix (W[i][k]: component i of eigenvector k, eigenvalues in decreasing order,
// so lambda_0 is the largest), n <= 512, one workgroup: the eigenvalue cut of a pseudo-inverse.
// Each sum runs in index order. *info: 0, or -1 for a non-finite result or a largest eigenvalue
// that is not positive and finite.
__global__ __launch_bounds__(512) void k_pinv_apply(const double* __restrict__ W, const double* __restrict__ ev,
                                                    int n, const double* __restrict__ rhs, double* __restrict__ out,
                                                    double rcond, int* __restrict__ info) {
  __shared__ double t[512];
  const int tid = threadIdx.x;
  const double l0 = ev[0];
  const bool ok0 = l0 > 0.0 && isfinite(l0);
  if (tid < n) {
    const double lk = ev[tid];
    double sum = 0.0;
    for (int i = 0; i < n; ++i) sum = fma(W[(long)i * n + tid], rhs[i], sum);
    t[tid] = (ok0 && lk > rcond * l0) ? sum / lk : 0.0;
  }
  __syncthreads();
  bool bad = !ok0;
  if (tid < n) {
    double sum = 0.0;
    for (int k = 0; k < n; ++k) sum = fma(W[(long)tid * n + k], t[k], sum);
    out[tid] = sum;
    bad = bad || !isfinite(sum);
  }
  const int anybad = __syncthreads_or(bad);
  if (tid == 0) *info = anybad ? -1 : 0;
}

// ---------------------------------------------------------------------------- launchers
template <typename TX>
void launch_anomaly(const double* ctrl, const double* J, int n, long m, TX* X, double* dJ, hipStream_t s) {
  int bx = (int)((m + 255) / 256);
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_anomaly<TX>, dim3(bx, n), dim3(256), 0, s, ctrl, J, n, m, X, dJ);
}
void launch_cost_anomaly(const double* J, int n, double* dJ, hipStream_t s) {
  hipLaunchKernelGGL(k_cost_anomaly, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, J, n, dJ);
}
template <typename TX>
void launch_gram(const TX* X, int n, long m, long ldx, double* partial, int nsplit, long kchunk, hipStream_t s) {
  const int bs = gram_block_rows(n), nbt = (n + bs - 1) / bs;
  const dim3 grid(nsplit * nbt * (nbt + 1) / 2);
  if (bs == 128)
    hipLaunchKernelGGL((k_gram<TX, false, 128>), grid, dim3(256), 0, s, X, n, m, ldx, partial, nsplit, kchunk, nbt,
                       nullptr);
  else
    hipLaunchKernelGGL((k_gram<TX, false, 64>), grid, dim3(256), 0, s, X, n, m, ldx, partial, nsplit, kchunk, nbt,
                       nullptr);
}
void launch_gram_anom(const double* ctrl, int n, long m, double* partial, int nsplit, long kchunk, hipStream_t s) {
  const int bs = gram_block_rows(n), nbt = (n + bs - 1) / bs;
  const dim3 grid(nsplit * nbt * (nbt + 1) / 2);
  if (bs == 128)
    hipLaunchKernelGGL((k_gram<double, true, 128>), grid, dim3(256), 0, s, ctrl + m, n, m, m, partial, nsplit, kchunk,
                       nbt, ctrl);
  else
    hipLaunchKernelGGL((k_gram<double, true, 64>), grid, dim3(256), 0, s, ctrl + m, n, m, m, partial, nsplit, kchunk,
                       nbt, ctrl);
}
void launch_gemv_anom(const double* ctrl, int n, long m, const double* c, double* g, hipStream_t s) {
  long bx = (m + 63) / 64;
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL((k_gemv_t<double, true>), dim3((unsigned)bx), dim3(256), 0, s, ctrl + m, n, m, m, c, g, ctrl);
}
int launch_pinv_apply(const double* W, const double* ev, int n, const double* rhs, double* out, double rcond,
                      int* info, hipStream_t s) {
  if (n > 512) return -1;
  hipLaunchKernelGGL(k_pinv_apply, dim3(1), dim3(512), 0, s, W, ev, n, rhs, out, rcond, info);
  return 0;
}
int gram_reduce_groups(int nsplit) { return (nsplit + GRAM_REDUCE_GROUP - 1) / GRAM_REDUCE_GROUP; }
void launch_gram_reduce(const double* partial, int n, int nsplit, double* tmp, double* G, hipStream_t s) {
  const long nn = (long)n * n;
  int bx = (int)((nn + 255) / 256);
  if (bx > 1024) bx = 1024;
  const int ng = gram_reduce_groups(nsplit);
  if (ng <= 16) {
    hipLaunchKernelGGL(k_gram_reduce_fused, dim3((unsigned)((nn + 15) / 16)), dim3(256), 0, s, partial, nn, nsplit,
                       G);
    return;
  }
  hipLaunchKernelGGL(k_gram_reduce_groups, dim3(bx, ng), dim3(256), 0, s, partial, nn, nsplit, GRAM_REDUCE_GROUP,
                     tmp);
  hipLaunchKernelGGL(k_gram_reduce, dim3(bx), dim3(256), 0, s, tmp, n, ng, G);
}
int launch_chol_solve(double* G, const double* rhs, int n, double* x, double* work, hipStream_t s, double ridge_rel) {
  if (n > CHOL_VEC_MAX) return -1;
  if (n <= 64) {
    hipLaunchKernelGGL(k_chol_wave, dim3(1), dim3(256), 0, s, G, rhs, n, x, (int*)work, ridge_rel);
  } else if (n <= CHOL_M32_MAX) {
    static bool attr = false;
    if (!attr) {
      if (hipFuncSetAttribute((const void*)k_chol_m32, hipFuncAttributeMaxDynamicSharedMemorySize, CHOL_M32_LDS) !=
          hipSuccess)
        return -2;
      attr = true;
    }
    hipLaunchKernelGGL(k_chol_m32, dim3(1), dim3(CHOL_M32_NT), CHOL_M32_LDS, s, G, rhs, n, x, (int*)work, ridge_rel);
  } else if (n <= CHOL_BLK_MAX)
    hipLaunchKernelGGL(k_chol_blocked, dim3(1), dim3(CHOL_BLK_NT), 0, s, G, rhs, n, x, (int*)work, ridge_rel);
  else
    hipLaunchKernelGGL(k_chol_solve<1024>, dim3(1), dim3(1024), 0, s, G, rhs, n, x, (int*)work, ridge_rel);
  return 0;
}

// ---------------------------------------------------------------------------- vector-observation EnVar step
// Fluctuations about each channel's time mean: one workgroup per (row, channel), the
// mean summed in a fixed order (per-thread strided sums, then waves, then workgroup).
__global__ __launch_bounds__(256) void k_obs_fluct(const double* series, long K, double* D) {
  __shared__ double red[4];
  const long base = (long)blockIdx.x * K;  // row r, channel c: blockIdx.x = r * channels + c
  double s = 0.0;
  for (long t = threadIdx.x; t < K; t += 256) s += series[base + t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double mean = (((red[0] + red[1]) + red[2]) + red[3]) / (double)K;
  for (long t = threadIdx.x; t < K; t += 256) D[base + t] = series[base + t] - mean;
}

// Y rows (n x n_obs): Y_i = (d_i - d_0) / eps, i = 1 .. n
__global__ void k_yrows(const double* D, int n, long n_obs, double inv_eps, double* Y) {
  const int i = blockIdx.y;
  for (long o = blockIdx.x * (long)blockDim.x + threadIdx.x; o < n_obs; o += (long)gridDim.x * blockDim.x)
    Y[(long)i * n_obs + o] = (D[(long)(i + 1) * n_obs + o] - D[o]) * inv_eps;
}

// out[i] = scale * sum_o A[i][o] B[o] + add_coef * add[i] (one workgroup per row, fixed order)
__global__ __launch_bounds__(256) void k_rowdot(const double* A, const double* B, long bstride, long len,
                                                double scale, const double* add, double add_coef, double* out) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const double* b = B + (long)i * bstride;
  double s = 0.0;
  for (long o = threadIdx.x; o < len; o += 256) s += A[(long)i * len + o] * b[o];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[i] = scale * (((red[0] + red[1]) + red[2]) + red[3]) + (add ? add_coef * add[i] : 0.0);
}

// H = G + shift I (n x n), and rhs = -grad
__global__ void k_shift_diag(const double* G, int n, double shift, double* H, const double* grad, double* neg) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    H[e] = G[e] + (i == j ? shift : 0.0);
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < n; i += blockDim.x) neg[i] = -grad[i];
}

// ---------------------------------------------------------------------------- posterior variance
// Inverse of an SPD matrix by in-place Gauss-Jordan sweeps in LDS (no pivoting: the
// pivots of an SPD matrix stay positive): for each k, with d = a_kk, the other entries
// take a_ij - a_ik a_kj / d, then row k is divided by d, column k by -d and a_kk = 1 / d.
// (A variant keeping each thread's entries in registers and passing only row and column k
// through LDS measured slower at n = 64: 94 against 68 us.)
constexpr int SPD_INV_MAX = 128;
__global__ __launch_bounds__(1024) void k_spd_inverse(const double* H, int n, double* C, int* info) {
  __shared__ double sA[SPD_INV_MAX * (SPD_INV_MAX + 1)];
  const long ld = n + 1;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  for (int i = ty; i < n; i += 32)
    for (int j = tx; j < n; j += 32) sA[i * ld + j] = H[(long)i * n + j];
  if (tid == 0) *info = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double d = sA[k * ld + k];
    if (tid == 0 && !(d > 0.0)) *info = k + 1;
    const double inv = 1.0 / d;
    for (int i = ty; i < n; i += 32) {
      if (i == k) continue;
      const double aik = sA[i * ld + k] * inv;
      for (int j = tx; j < n; j += 32)
        if (j != k) sA[i * ld + j] -= aik * sA[k * ld + j];
    }
    __syncthreads();
    for (int j = tid; j < n; j += 1024)
      if (j != k) {
        sA[k * ld + j] *= inv;
        sA[j * ld + k] *= -inv;
      }
    if (tid == 0) sA[k * ld + k] = inv;
    __syncthreads();
  }
  for (int i = ty; i < n; i += 32)
    for (int j = tx; j < n; j += 32) C[(long)i * n + j] = sA[i * ld + j];
}

// var[k] = e_k^T C e_k with e_k[a] = (ctrl[a + 1][k] - ctrl[0][k]) / eps: one workgroup per 64
// columns, the E block (rows padded to a multiple of 16 with zeros) staged in LDS; wave w forms
// V = C E for columns 16w .. 16w + 15 on the FP64 matrix cores (16 x 16 tiles over all row
// blocks, v_mfma_f64_16x16x4f64), then each lane sums E o V over its rows (l/16 + 4r of every row
// block) and the four lanes of a column are added in a fixed order. Every load is unconditional
// and masked arithmetically, so the loads of a loop overlap.
constexpr int POST_COLS = 64;
__global__ __launch_bounds__(256) void k_post_var(const double* __restrict__ ctrl, int n, long m, double inv_eps,
                                                  const double* __restrict__ C, double* __restrict__ var) {
  extern __shared__ double sE[];  // [np][POST_COLS]
  const int np = (n + 15) & ~15;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long c0 = (long)blockIdx.x * POST_COLS;
  {
    const long col = c0 + lane, colc = col < m ? col : m - 1;
    const double base = ctrl[colc];
#pragma unroll 4
    for (int a = w; a < np; a += 4) {
      const int ac = a < n ? a : n - 1;
      const double x = (ctrl[(long)(ac + 1) * m + colc] - base) * inv_eps;
      sE[a * POST_COLS + lane] = x * ((a < n && col < m) ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  const int lr = lane & 15, lq = lane >> 4, cw = 16 * w + lr;
  double part = 0.0;
  for (int R = 0; R < np; R += 16) {
    MfmaAcc<double>::V acc = {0.0, 0.0, 0.0, 0.0};
    const int row = R + lr, rowc = row < n ? row : n - 1;
    // np is a multiple of 16: four MFMA steps per trip, their operands loaded first (the
    // instruction is convergent, so the compiler does not unroll a loop that might leave a remainder)
    for (int k0 = 0; k0 < np; k0 += 16) {
      double a_op[4], b_op[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k0 + 4 * u + lq, kc = kk < n ? kk : n - 1;
        a_op[u] = C[(long)rowc * n + kc] * ((row < n && kk < n) ? 1.0 : 0.0);
        b_op[u] = sE[kk * POST_COLS + cw];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = MfmaAcc<double>::mma(a_op[u], b_op[u], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part = fma(sE[(R + lq + 4 * r) * POST_COLS + cw], acc[r], part);
  }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  if (lq == 0 && c0 + cw < m) var[c0 + cw] = part;
}

// one column k per thread: the centre sums the members in index order, then each member row
// adds its own scaled direction to that centre
__global__ __launch_bounds__(256) void k_build_rows(const double* __restrict__ fe, const double* __restrict__ E,
                                                   int n, long m, const double* __restrict__ w, double eps,
                                                   int nrows, double* __restrict__ rows) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < m; k += (long)gridDim.x * 256) {
    double f = fe[k];
    for (int i = 0; i < n; ++i) f = fma(w[i], E[(long)i * m + k], f);
    rows[k] = f;
    for (int i = 0; i + 1 < nrows; ++i) rows[(long)(i + 1) * m + k] = fma(eps, E[(long)i * m + k], f);
  }
}

// rows[t] = fe + sum_i W[t][i] E_i for t < nw (the same summation order as the centre above)
__global__ __launch_bounds__(256) void k_combine_rows(const double* __restrict__ fe, const double* __restrict__ E,
                                                     int n, long m, const double* __restrict__ W, int nw,
                                                     double* __restrict__ rows) {
  for (long k = blockIdx.x * 256L + threadIdx.x; k < m; k += (long)gridDim.x * 256)
    for (int t = 0; t < nw; ++t) {
      double f = fe[k];
      for (int i = 0; i < n; ++i) f = fma(W[(long)t * n + i], E[(long)i * m + k], f);
      rows[(long)t * m + k] = f;
    }
}

void launch_combine_rows(const double* fe, const double* E, int n, long m, const double* W, int nw, double* rows,
                         hipStream_t s) {
  long bx = (m + 255) / 256;
  if (bx > 2048) bx = 2048;
  hipLaunchKernelGGL(k_combine_rows, dim3((unsigned)bx), dim3(256), 0, s, fe, E, n, m, W, nw, rows);
}

void launch_build_rows(const double* fe, const double* E, int n, long m, const double* w, double eps, int nrows,
                       double* rows, hipStream_t s) {
  long bx = (m + 255) / 256;
  if (bx > 2048) bx = 2048;
  hipLaunchKernelGGL(k_build_rows, dim3((unsigned)bx), dim3(256), 0, s, fe, E, n, m, w, eps, nrows, rows);
}

void launch_obs_fluct(const double* series, int rows, int channels, long K, double* D, hipStream_t s) {
  hipLaunchKernelGGL(k_obs_fluct, dim3(rows * channels), dim3(256), 0, s, series, K, D);
}
void launch_yrows(const double* D, int n, long n_obs, double eps, double* Y, hipStream_t s) {
  long bx = (n_obs + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_yrows, dim3((unsigned)bx, n), dim3(256), 0, s, D, n, n_obs, 1.0 / eps, Y);
}
void launch_rowdot(const double* A, const double* B, int rows, long len, double scale, const double* add,
                   double add_coef, double* out, hipStream_t s, bool per_row_b) {
  hipLaunchKernelGGL(k_rowdot, dim3(rows), dim3(256), 0, s, A, B, per_row_b ? len : 0L, len, scale, add, add_coef,
                     out);
}
void launch_shift_diag(const double* G, int n, double shift, double* H, const double* grad, double* neg, hipStream_t s) {
  long bx = ((long)n * n + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_shift_diag, dim3((unsigned)bx), dim3(256), 0, s, G, n, shift, H, grad, neg);
}
int launch_spd_inverse(const double* H, int n, double* C, double* work, hipStream_t s) {
  if (n < 1 || n > SPD_INV_MAX) return -1;
  hipLaunchKernelGGL(k_spd_inverse, dim3(1), dim3(1024), 0, s, H, n, C, (int*)work);
  return 0;
}
int launch_post_var(const double* ctrl, int n, long m, double eps, const double* C, double* var, hipStream_t s) {
  if (n < 1 || n > SPD_INV_MAX) return -1;
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_post_var, hipFuncAttributeMaxDynamicSharedMemorySize,
                            SPD_INV_MAX * POST_COLS * (int)sizeof(double)) != hipSuccess)
      return -2;
    attr = true;
  }
  const size_t dyn = (size_t)((n + 15) & ~15) * POST_COLS * sizeof(double);
  hipLaunchKernelGGL(k_post_var, dim3((unsigned)((m + POST_COLS - 1) / POST_COLS)), dim3(256), dyn, s, ctrl, n, m,
                     1.0 / eps, C, var);
  return 0;
}
template <typename TX>
void launch_gemv_t(const TX* X, int n, long m, long ldx, const double* c, double* g, hipStream_t s) {
  long bx = (m + 63) / 64;
  if (bx > 8192) bx = 8192;
  hipLaunchKernelGGL(k_gemv_t<TX>, dim3((unsigned)bx), dim3(256), 0, s, X, n, m, ldx, c, g);
}
template <typename TX>
void launch_transpose(const TX* X, int n, long m, TX* Xt, hipStream_t s) {
  long e = (long)n * m;
  int bx = (int)((e + 255) / 256);
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_transpose<TX>, dim3(bx), dim3(256), 0, s, X, n, m, Xt);
}

template void launch_anomaly<double>(const double*, const double*, int, long, double*, double*, hipStream_t);
template void launch_anomaly<float>(const double*, const double*, int, long, float*, double*, hipStream_t);
template void launch_gram<double>(const double*, int, long, long, double*, int, long, hipStream_t);
template void launch_gram<float>(const float*, int, long, long, double*, int, long, hipStream_t);
template void launch_gemv_t<double>(const double*, int, long, long, const double*, double*, hipStream_t);
template void launch_gemv_t<float>(const float*, int, long, long, const double*, double*, hipStream_t);
template void launch_transpose<double>(const double*, int, long, double*, hipStream_t);
template void launch_transpose<float>(const float*, int, long, float*, hipStream_t);

}  // namespace envar
