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
// 64-column panels up to n = 256); the projection g = X^T c is a
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

constexpr int GRAM_KC = 32;
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

// Only the tile pairs bi <= bj are computed; an off-diagonal tile is written twice (as G[I][J] and
// transposed as G[J][I]), so G is exactly symmetric. The X rows are fetched as 16-byte vectors into
// registers one chunk ahead of the MFMA work on the chunk in LDS (a diagonal tile fetches its rows
// once and uses them for both operands).
template <typename TX>
__global__ __launch_bounds__(256) void k_gram(const TX* __restrict__ X, int n, long m, long ldx,
                                              double* __restrict__ partial, int nsplit, long kchunk, int nbt) {
  typedef typename MfmaAcc<TX>::V V;
  typedef typename Vec16<TX>::T VT;
  constexpr int KC = GRAM_KC, LDR = KC + 1;
  constexpr int VW = 16 / sizeof(TX);      // elements per vector
  constexpr int VPR = KC / VW;             // vectors per row and chunk
  constexpr int NV = 64 * VPR / 256;       // vectors per thread and operand
  __shared__ TX sa[64 * LDR];
  __shared__ TX sb[64 * LDR];
  const int split = blockIdx.x % nsplit;
  int pair = blockIdx.x / nsplit;
  int bi = 0;
  while (pair >= nbt - bi) {
    pair -= nbt - bi;
    ++bi;
  }
  const int bj = bi + pair;
  const bool diag = bi == bj;
  const int I0 = bi * 64, J0 = bj * 64;
  const long kbeg = (long)split * kchunk;
  long kend = kbeg + kchunk;
  if (kend > m) kend = m;
  const bool vec = ldx % VW == 0;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  VT ra[NV], rb[NV];
  auto load = [&](int row, long k) -> VT {
    VT v;
    if (row < n && vec && k + VW <= kend) return *(const VT*)(X + (long)row * ldx + k);
    for (int e = 0; e < VW; ++e) v[e] = (row < n && k + e < kend) ? X[(long)row * ldx + k + e] : (TX)0;
    return v;
  };
  auto fetch = [&](long k0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int q = threadIdx.x + 256 * v, r = q / VPR, c = (q % VPR) * VW;
      ra[v] = load(I0 + r, k0 + c);
      if (!diag) rb[v] = load(J0 + r, k0 + c);
    }
  };
  V acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = V{0, 0, 0, 0};
  if (kbeg < kend) fetch(kbeg);
  for (long k0 = kbeg; k0 < kend; k0 += KC) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int q = threadIdx.x + 256 * v, r = q / VPR, c = (q % VPR) * VW;
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        sa[r * LDR + c + e] = ra[v][e];
        if (!diag) sb[r * LDR + c + e] = rb[v][e];
      }
    }
    __syncthreads();
    if (k0 + KC < kend) fetch(k0 + KC);  // the next chunk's loads overlap this chunk's MFMA work
    const TX* sB = diag ? sa : sb;
    const int row = 16 * wave + lane % 16;
    for (int kk = 0; kk < KC; kk += 4) {
      const TX a = sa[row * LDR + kk + lane / 16];
      for (int t = 0; t < 4; ++t) {
        const TX b = sB[(16 * t + lane % 16) * LDR + kk + lane / 16];
        acc[t] = MfmaAcc<TX>::mma(a, b, acc[t]);
      }
    }
    __syncthreads();
  }
  double* P = partial + (long)split * n * n;
  for (int t = 0; t < 4; ++t) {
    const int j = J0 + 16 * t + lane % 16;
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + 16 * wave + MfmaAcc<TX>::row(lane, r);
      if (i < n && j < n) {
        P[(long)i * n + j] = (double)acc[t][r];
        if (!diag) P[(long)j * n + i] = (double)acc[t][r];
      }
    }
  }
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

// ---------------------------------------------------------------------------- register Cholesky (n <= 64) and 64-column panels
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

// wave_chol64 factors a symmetric 64 x 64 block held one column per lane of one wave,
// a[i] = A[i][lane], with no workgroup barrier, for the 64-column blocks of k_chol_p64. Step k
// scales row k by 1 / sqrt(a_kk) (l_j = a_kj / sqrt(a_kk), lanes j > k), broadcasts it through
// LDS, and every lane j > k subtracts l_i l_j from its entries i > k; lanes j <= k multiply by
// zero instead of branching, so that a step is one basic block and the next pivot's chain
// overlaps the updates. All 64 steps are unrolled (measured with the other phases of that
// kernel: 415 us at n = 256 against 530 us for a loop over panels of eight). On return lane j
// holds L[j][k] in a[k] for k < j, its pivot in a[j] and the trailing entries A^(j)[i][j] below
// (i > j); rs = 1 / L[j][j] (rsqrt of the pivot) and sq = L[j][j] (pivot * rs). Returns
// (wave-uniform) the first step whose pivot is not positive, plus one, or 0.
__device__ __forceinline__ int wave_chol64(double (&a)[64], double& sq, double& rs, double* colk) {
  const int lane = threadIdx.x & 63;
  int bad = 0;
  sq = 1.0;
  rs = 1.0;
  double piv = readlane_d(a[0], 0);
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    if (!(piv > 0.0) && bad == 0) bad = k + 1;
    const double p = piv > 0.0 ? piv : 1e-300;
    const double r = rsqrt(p);
    double* const c = colk + (k & 1) * 64;  // two buffers: one wave sync per step
    const double t = a[k] * r;
    c[lane] = t;
    wave_sync();
    // lanes <= k multiply by zero instead of branching, so that a step is one basic block and
    // the next pivot's chain overlaps this step's updates. That pivot is lane k + 1's own
    // diagonal update (c[k + 1] is its t), bit for bit the value the loop below leaves.
    const double tt = lane > k ? t : 0.0;
    if (k + 1 < 64) piv = readlane_d(fma(-t, tt, a[k + 1]), k + 1);
    sq = lane == k ? p * r : sq;
    rs = lane == k ? r : rs;
    a[k] = lane > k ? t : a[k];
#pragma unroll
    for (int i = k + 1; i < 64; ++i) a[i] = fma(-c[i], tt, a[i]);
  }
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

// 64 < n <= CHOL_P64_MAX: right-looking in 64-column panels, the matrix in
// global memory (L2 resident; lower triangle kept) and one workgroup. Per panel:
// wave 0 factors the diagonal block (wave_chol64) and stores L11; every thread
// takes one row of the panel below and solves L11 l^T = a^T right-looking (column
// c final once scaled, then 63 - c independent updates) with L11 broadcast from
// LDS; the panel, transposed in LDS, then takes the trailing lower triangle
// A22 -= L21 L21^T in 4 x 4 register tiles. The solves are blocked the same way:
// the diagonal blocks by wave 0 with the block in registers and the pivots and
// running right-hand side read across lanes, the off-diagonal blocks as GEMVs by
// all threads.
constexpr int CHOL_P64_MAX = 256;
constexpr int CHOL_P64_NT = 512;                 // eight waves: 256 VGPRs for wave 0's 64-double column
constexpr int CHOL_P64_PR = CHOL_P64_MAX - 64;   // rows of the transposed panel
constexpr int CHOL_P64_LDS = 64 * CHOL_P64_PR * (int)sizeof(double);  // dynamic part: the transposed panel

__global__ __launch_bounds__(CHOL_P64_NT) void k_chol_p64(double* A, const double* rhs, int n, double* x, int* info,
                                                      double ridge_rel) {
  // the small buffers are static so that their constant offsets fold into the LDS
  // instructions (offsets into the dynamic block are materialised one register each)
  __shared__ double sL[64 * 65];  // L11, row stride 65
  __shared__ double sR[64];       // 1 / L11[c][c]
  __shared__ double colk[128];
  __shared__ double sv[CHOL_P64_MAX];  // rhs -> y -> x
  extern __shared__ double Pt[];       // Pt[c * PR + r] = L21[r][c]
  constexpr int PR = CHOL_P64_PR;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long ld = n;
  if (wave == 0) {  // trace: strided partial sums, then a fixed shuffle tree
    double tr = 0.0;
    for (int i = lane; i < n; i += 64) tr += A[i * ld + i];
    tr = wave_sum(tr);
    if (lane == 0) {
      colk[0] = ridge_rel * tr / (double)n;
      *info = 0;
    }
  }
  __syncthreads();
  const double ridge = colk[0];
  for (int i = tid; i < n; i += CHOL_P64_NT) A[i * ld + i] += ridge;
  __threadfence_block();
  __syncthreads();
  for (int i = tid; i < n; i += CHOL_P64_NT) sv[i] = rhs[i];
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int kw = min(64, n - k0), rows = n - k0 - kw;
    double* const Ak = A + (long)k0 * ld + k0;
    if (wave == 0) {
      double a[64];
      const int lc = min(lane, kw - 1);
#pragma unroll
      for (int i = 0; i < 64; ++i) {  // unconditional loads, masked arithmetically (as in k_chol_wave)
        const int ic = min(i, kw - 1);
        const double g = Ak[max(ic, lc) * ld + min(ic, lc)];
        const bool in = i < kw && lane < kw;
        a[i] = fma(g, in ? 1.0 : 0.0, (i == lane && !in) ? 1.0 : 0.0);
      }
      double sq, rs;
      const int bad = wave_chol64(a, sq, rs, colk);
      if (lane == 0 && bad != 0 && bad <= kw && *info == 0) *info = k0 + bad;
#pragma unroll
      for (int k = 0; k < 64; ++k) sL[lane * 65 + k] = k < lane ? a[k] : k == lane ? sq : 0.0;
      sR[lane] = rs;
      // row lane of L11 back to memory (lower triangle) from LDS, without per-element branches
      // on the register array
      wave_sync();
      for (int e = lane; e < kw * kw; e += 64) {
        const int i = e / kw, k = e - i * kw;
        if (k <= i) Ak[i * ld + k] = sL[i * 65 + k];
      }
    }
    __syncthreads();
    const int rows4 = (rows + 3) & ~3;
    // a panel with rows below it is full (kw = 64); rows4 <= PR < CHOL_P64_NT: one row per thread
    if (tid < rows4) {
      const int r = tid;
      double* const src = Ak + (long)(kw + r) * ld;
      const double* const srow = Ak + (long)(kw + min(r, rows - 1)) * ld;
      double ar[64];
      const double keep = r < rows ? 1.0 : 0.0;
#pragma unroll
      for (int c = 0; c < 64; ++c) ar[c] = srow[c] * keep;
      // right-looking: column c is final once scaled, then leaves the 63 - c independent updates
#pragma unroll
      for (int c = 0; c < 64; ++c) {
        ar[c] *= sR[c];
#pragma unroll
        for (int k = c + 1; k < 64; ++k) ar[k] = fma(-sL[k * 65 + c], ar[c], ar[k]);
      }
      if (r < rows) {
#pragma unroll
        for (int c = 0; c < 64; ++c) src[c] = ar[c];
      }
#pragma unroll
      for (int c = 0; c < 64; ++c) Pt[c * PR + r] = ar[c];
    }
    __syncthreads();
    const int T = rows4 >> 2, ntile = T * (T + 1) / 2;
    double* const A22 = Ak + (long)kw * ld + kw;
    for (int idx = tid; idx < ntile; idx += CHOL_P64_NT) {
      int ti = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
      while (ti * (ti + 1) / 2 > idx) --ti;
      while ((ti + 1) * (ti + 2) / 2 <= idx) ++ti;
      const int tj = idx - ti * (ti + 1) / 2;
      double acc[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
      const double* const pi = Pt + 4 * ti;
      const double* const pj = Pt + 4 * tj;
#pragma unroll 4
      for (int c = 0; c < kw; ++c) {
        const double2 i01 = *(const double2*)(pi + c * PR), i23 = *(const double2*)(pi + c * PR + 2);
        const double2 j01 = *(const double2*)(pj + c * PR), j23 = *(const double2*)(pj + c * PR + 2);
        const double li[4] = {i01.x, i01.y, i23.x, i23.y}, lj[4] = {j01.x, j01.y, j23.x, j23.y};
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] = fma(li[p], lj[q], acc[p][q]);
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int i = 4 * ti + p;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = 4 * tj + q;
          if (i < rows && j <= i) A22[i * ld + j] -= acc[p][q];
        }
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  // L y = rhs
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int kw = min(64, n - k0);
    const double* const Ak = A + (long)k0 * ld + k0;
    if (wave == 0) {
      double a[64];
      const int lc = min(lane, kw - 1);
      // unmasked: only k < lane is used by a lane below kw; padding lanes start at zero and
      // their broadcasts reach padding lanes only
#pragma unroll
      for (int k = 0; k < 64; ++k) a[k] = Ak[lc * ld + min(k, kw - 1)];
      const double dg = Ak[lc * ld + lc], b = sv[k0 + lc];
      const double rs = lane < kw ? 1.0 / dg : 1.0;
      double v = lane < kw ? b : 0.0;
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        const double yk = readlane_d(v * rs, k);
        if (lane == k)
          v = yk;
        else if (lane > k)
          v = fma(-a[k], yk, v);
      }
      if (lane < kw) sv[k0 + lane] = v;
    }
    __syncthreads();
    for (int i = k0 + kw + tid; i < n; i += CHOL_P64_NT) {
      const double* const Li = A + (long)i * ld + k0;
      double t = sv[i];
      for (int c = 0; c < kw; ++c) t = fma(-Li[c], sv[k0 + c], t);
      sv[i] = t;
    }
    __syncthreads();
  }
  // L^T x = y
  for (int k0 = ((n - 1) / 64) * 64; k0 >= 0; k0 -= 64) {
    const int kw = min(64, n - k0);
    const double* const Ak = A + (long)k0 * ld + k0;
    if (wave == 0) {
      double a[64];
      const int lc = min(lane, kw - 1);
      // unmasked: a padding lane k >= kw keeps v = 0 (its updates are finite entries times
      // zero), so x_k = 0 and the clamped entries it meets change nothing
#pragma unroll
      for (int k = 0; k < 64; ++k) a[k] = Ak[min(k, kw - 1) * ld + lc];
      const double dg = Ak[lc * ld + lc], b = sv[k0 + lc];
      const double rs = lane < kw ? 1.0 / dg : 1.0;
      double v = lane < kw ? b : 0.0;
#pragma unroll
      for (int k = 63; k >= 0; --k) {
        const double xk = readlane_d(v * rs, k);
        if (lane == k)
          v = xk;
        else if (lane < k)
          v = fma(-a[k], xk, v);
      }
      if (lane < kw) sv[k0 + lane] = v;
    }
    __syncthreads();
    for (int i = tid; i < k0; i += CHOL_P64_NT) {
      double t = sv[i];
      for (int c = 0; c < kw; ++c) t = fma(-A[(long)(k0 + c) * ld + i], sv[k0 + c], t);
      sv[i] = t;
    }
    __syncthreads();
  }
  bool nonfinite = false;
  for (int i = tid; i < n; i += CHOL_P64_NT) {
    x[i] = sv[i];
    nonfinite = nonfinite || !isfinite(sv[i]);
  }
  if (__syncthreads_or(nonfinite) && tid == 0 && *info == 0) *info = -1;
}

// ---------------------------------------------------------------------------- GEMVs
// g[k] = sum_i X[i][k] c[i]: 64 columns per block, four row groups summed in order
template <typename TX>
__global__ __launch_bounds__(256) void k_gemv_t(const TX* __restrict__ X, int n, long m, long ldx,
                                                const double* __restrict__ c, double* __restrict__ g) {
  __shared__ double part[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (long k0 = blockIdx.x * 64L; k0 < m; k0 += (long)gridDim.x * 64L) {
    const long k = k0 + tx;
    double s = 0.0;
    if (k < m) {
#pragma unroll 4
      for (int i = ty; i < n; i += 4) s += (double)X[(long)i * ldx + k] * c[i];
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

// ---------------------------------------------------------------------------- launchers
template <typename TX>
void launch_anomaly(const double* ctrl, const double* J, int n, long m, TX* X, double* dJ, hipStream_t s) {
  int bx = (int)((m + 255) / 256);
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_anomaly<TX>, dim3(bx, n), dim3(256), 0, s, ctrl, J, n, m, X, dJ);
}
template <typename TX>
void launch_gram(const TX* X, int n, long m, long ldx, double* partial, int nsplit, long kchunk, hipStream_t s) {
  const int nbt = (n + 63) / 64;
  hipLaunchKernelGGL(k_gram<TX>, dim3(nsplit * nbt * (nbt + 1) / 2), dim3(256), 0, s, X, n, m, ldx, partial, nsplit,
                     kchunk, nbt);
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
  } else if (n <= CHOL_P64_MAX) {
    static bool attr = false;
    if (!attr) {
      if (hipFuncSetAttribute((const void*)k_chol_p64, hipFuncAttributeMaxDynamicSharedMemorySize, CHOL_P64_LDS) !=
          hipSuccess)
        return -2;
      attr = true;
    }
    hipLaunchKernelGGL(k_chol_p64, dim3(1), dim3(CHOL_P64_NT), CHOL_P64_LDS, s, G, rhs, n, x, (int*)work, ridge_rel);
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
