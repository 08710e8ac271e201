// Deterministic eigen-ensemble of the tapered Gaussian covariance (Sec. 3.3.2).
//
// B = D K D over the control cells (eq. covarianceB with c_xy = infinity): D = diag(sigma_i) and
// K_ij = exp(-(x_i - x_j)^2 / a_x^2 - (y_i - y_j)^2 / a_y^2). The control cells are embedded in their
// bounding rectangle of nx x ny cells (sigma = 0 at rectangle cells outside the region), where the
// kernel factors as K = Ky (x) Kx. B applied to a block of b vectors is then two dense contractions,
// along x (rows of nx) and along y (columns of ny), on the FP64 matrix cores: 2 b M (nx + ny) flops
// for M = nx ny instead of 2 b M^2.
//
// The N leading eigenpairs come from block subspace iteration with a Rayleigh-Ritz step every
// iteration. Per iteration, with Q [b][M] orthonormal rows:
//   Z = B Q;  G = [Q; Z][Q; Z]^T (MFMA Gram);  T = sym(Q Z^T) = W diag(theta) W^T (Jacobi);
//   U = W^T Q, V = W^T Z (Ritz vectors and their images), residuals |V_k - theta_k U_k|;
//   next Q = the Cholesky orthonormalisation of V with rows scaled to unit norm (rows in decreasing
//   Ritz value), formed from the b x b blocks of G without another pass over M.
// The b x b symmetric eigenproblem is solved by cyclic Jacobi in one workgroup (parallel round-robin
// ordering, the matrix and the rotations in LDS up to b = 96); the Cholesky factor and its inverse
// also in one workgroup.
#include "common.h"
#include "kernels.h"

namespace envar {

// ---------------------------------------------------------------------------- set-up
// sigma of every rectangle cell (zero outside the region): sigma_max^2 (1 - r^2)^2 inside the
// ellipse inscribed in the rectangle, r the elliptic radius (taper = 1), or sigma_max^2 (taper = 0)
__global__ void k_eig_sigma(const int* __restrict__ bidx, int ncc, int nxb, int nyb, double h, double sig2max,
                            int taper, double* __restrict__ sig) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncc; c += gridDim.x * blockDim.x) {
    const int b = bidx[c];
    const int ii = b % nxb, jj = b / nxb;
    double s2 = sig2max;
    if (taper) {
      // offsets from the rectangle's centre in units of its half-widths
      const double ex = ((ii + 0.5) * h - 0.5 * nxb * h) / (0.5 * nxb * h);
      const double ey = ((jj + 0.5) * h - 0.5 * nyb * h) / (0.5 * nyb * h);
      const double r2 = ex * ex + ey * ey;
      s2 = r2 < 1.0 ? sig2max * (1.0 - r2) * (1.0 - r2) : 0.0;
    }
    sig[b] = sqrt(s2);
  }
}

// K[i][j] = exp(-((i - j) h)^2 / a^2) on n cells of spacing h
__global__ void k_kernel1d(int n, double h, double a, double* __restrict__ K) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const double d = (double)((int)(e / n) - (int)(e % n)) * h;
    K[e] = exp(-(d * d) / (a * a));
  }
}

// counter-based start block: uniform in [-1, 1) on the cells with sigma > 0 (splitmix64 of the index)
__global__ void k_eig_random(double* __restrict__ Q, int b, long M, const double* __restrict__ sig,
                             unsigned long long seed) {
  const long n = (long)b * M;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
    Q[e] = sig[e % M] > 0.0 ? 2.0 * u - 1.0 : 0.0;
  }
}

// W[r][i] = sig[i] Q[r][i]
__global__ void k_scale_rows(const double* __restrict__ Q, const double* __restrict__ sig, long n, long M,
                             double* __restrict__ W) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    W[e] = sig[e % M] * Q[e];
}

// ---------------------------------------------------------------------------- batched FP64 GEMM on MFMA
// C[z] = A[z] B[z] (row-major, M x K times K x N), optionally scaled elementwise by S (C_ij = S_ij (AB)_ij,
// S shared by the batch). One workgroup (4 waves) per 64 x 64 block of C; K in chunks of 32 through
// LDS; wave w owns rows 16 w .. 16 w + 15 and four 16 x 16 tiles (v_mfma_f64_16x16x4f64: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16], result register r holds row l / 16 + 4 r).
constexpr int DG_KC = 32, DG_LDA = DG_KC + 1, DG_LDB = 80;

__global__ __launch_bounds__(256) void k_dgemm(int M, int N, int K, const double* __restrict__ A, long lda, long sA,
                                               const double* __restrict__ B, long ldb, long sB, double* __restrict__ C,
                                               long ldc, long sC, const double* __restrict__ S, long lds) {
  typedef double __attribute__((ext_vector_type(4))) V4;
  __shared__ double sa[64 * DG_LDA];
  __shared__ double sb[DG_KC * DG_LDB];
  const int I0 = blockIdx.y * 64, J0 = blockIdx.x * 64;
  const long z = blockIdx.z;
  A += z * sA;
  B += z * sB;
  C += z * sC;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V4 acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = V4{0, 0, 0, 0};
  // A 64 x 32 and B 32 x 64 chunk: eight values of each per thread, loaded into registers one
  // chunk ahead of the MFMA work; every load is unconditional (clamped address, arithmetic mask):
  // a select on the loaded value becomes a branch around each load, and the loads then run one
  // after another
  constexpr int NQ = 64 * DG_KC / 256;
  double va[NQ], vb[NQ];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = threadIdx.x + 256 * i, r = q / DG_KC, c = q % DG_KC;
      const int rr = min(I0 + r, M - 1), cc = min(k0 + c, K - 1);
      va[i] = A[(long)rr * lda + cc] * ((I0 + r < M && k0 + c < K) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = threadIdx.x + 256 * i, r = q >> 6, c = q & 63;
      const int rr = min(k0 + r, K - 1), cc = min(J0 + c, N - 1);
      vb[i] = B[(long)rr * ldb + cc] * ((k0 + r < K && J0 + c < N) ? 1.0 : 0.0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += DG_KC) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = threadIdx.x + 256 * i;
      sa[(q / DG_KC) * DG_LDA + q % DG_KC] = va[i];
      sb[(q >> 6) * DG_LDB + (q & 63)] = vb[i];
    }
    __syncthreads();
    if (k0 + DG_KC < K) fetch(k0 + DG_KC);
    const int row = 16 * wave + (lane & 15);
    for (int kk = 0; kk < DG_KC; kk += 4) {
      const double a = sa[row * DG_LDA + kk + (lane >> 4)];
      for (int t = 0; t < 4; ++t) {
        const double bv = sb[(kk + (lane >> 4)) * DG_LDB + 16 * t + (lane & 15)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  for (int t = 0; t < 4; ++t) {
    const int j = J0 + 16 * t + (lane & 15);
    for (int r = 0; r < 4; ++r) {
      const int i = I0 + 16 * wave + (lane >> 4) + 4 * r;
      if (i < M && j < N) C[(long)i * ldc + j] = S ? S[(long)i * lds + j] * acc[t][r] : acc[t][r];
    }
  }
}

// ---------------------------------------------------------------------------- b x b work
// Cyclic Jacobi for a symmetric n x n matrix in one workgroup: n (padded to even) indices in n - 1
// rounds of n / 2 disjoint pairs (round-robin), each round a rotation angle per pair, then J^T A J
// in one pass over the 2 x 2 blocks of pair pairs (and the eigenvector columns). A pair is rotated unless |a_pq| is below
// n ulp of sqrt(|a_pp a_qq|) or of the largest diagonal entry; the iteration ends before a sweep in
// which no pair would rotate. Outputs the eigenvalues in decreasing order, W with eigenvector k in column k, and its
// transpose Wt.
constexpr int JAC_LDS_MAX = 96;
constexpr int JAC_MAX = 512;

__device__ __forceinline__ void jac_pair(int t, int k, int ne, int& p, int& q) {
  if (k == 0) {
    p = ne - 1;
    q = t;
  } else {
    p = (t + k) % (ne - 1);
    q = (t - k + ne - 1) % (ne - 1);
  }
}

__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ Ain, int lda, int n, int max_sweeps,
                                                 double* __restrict__ evals, double* __restrict__ W,
                                                 double* __restrict__ Wt, double* __restrict__ gscratch) {
  extern __shared__ double dyn[];
  __shared__ double cs[JAC_MAX];  // (c, s) per pair; the sorted diagonal at the end
  __shared__ int pq[JAC_MAX];     // (p, q) per pair
  __shared__ int rk[JAC_MAX];
  __shared__ double red[16];
  __shared__ int rotated;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ne = n + (n & 1);
  const int ld = ne + 1;  // odd row stride: a column walk touches every LDS bank
  double* A = ne <= JAC_LDS_MAX ? dyn : gscratch;
  double* V = A + (long)ne * ld;
  for (int i = wave; i < ne; i += 16)
    for (int j = lane; j < ne; j += 64) {
      A[i * ld + j] = (i < n && j < n) ? Ain[(long)i * lda + j] : 0.0;
      V[i * ld + j] = i == j ? 1.0 : 0.0;
    }
  if (tid == 0) rotated = 0;
  __syncthreads();
  const int half = ne / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // largest |diagonal| of this sweep: the absolute floor of the rotation test
    double dmax = 0.0;
    for (int k = tid; k < ne; k += 1024) dmax = fmax(dmax, fabs(A[k * ld + k]));
    dmax = wave_max(dmax);
    if (lane == 0) red[wave] = dmax;
    __syncthreads();
    dmax = 0.0;
    for (int w = 0; w < 16; ++w) dmax = fmax(dmax, red[w]);
    // skip the sweep when no pair would rotate (a converged matrix costs one scan, not a sweep)
    const double tol = ne * 1.1102230246251565e-16;
    for (int e = tid; e < ne * ne; e += 1024) {
      const int i = e / ne, j = e % ne;
      const double a = fabs(A[i * ld + j]);
      if (i != j && a > tol * dmax && a > tol * sqrt(fabs(A[i * ld + i] * A[j * ld + j]))) rotated = 1;
    }
    __syncthreads();
    const int need = rotated;
    __syncthreads();
    if (tid == 0) rotated = 0;
    if (!need) break;
    for (int t = 0; t < ne - 1; ++t) {
      if (tid < half) {
        int p, q;
        jac_pair(t, tid, ne, p, q);
        const double apq = A[p * ld + q];
        double c = 1.0, s = 0.0;
        // rotate unless a_pq is at the rounding level (n ulp) of sqrt(|a_pp a_qq|) or of the largest
        // diagonal entry (the floor for pairs of near-zero eigenvalues)
        if (fabs(apq) > tol * dmax && fabs(apq) > tol * sqrt(fabs(A[p * ld + p] * A[q * ld + q]))) {
          const double th = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
          const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
      }
      __syncthreads();
      // A <- J^T A J block by block: the 2 x 2 block of rows (p, q) of pair a and columns (p', q') of
      // pair b only needs its own four old entries, so rows and columns rotate in one pass
      for (int e = tid; e < half * half; e += 1024) {
        const int a = e / half, bb = e % half;
        const int p = pq[2 * a], q = pq[2 * a + 1], r = pq[2 * bb], u = pq[2 * bb + 1];
        const double c1 = cs[2 * a], s1 = cs[2 * a + 1], c2 = cs[2 * bb], s2 = cs[2 * bb + 1];
        const double apr = A[p * ld + r], apu = A[p * ld + u], aqr = A[q * ld + r], aqu = A[q * ld + u];
        // rows: (p, q) <- (c1 p - s1 q, s1 p + c1 q)
        const double bpr = c1 * apr - s1 * aqr, bpu = c1 * apu - s1 * aqu;
        const double bqr = s1 * apr + c1 * aqr, bqu = s1 * apu + c1 * aqu;
        // columns: (r, u) <- (c2 r - s2 u, s2 r + c2 u)
        A[p * ld + r] = c2 * bpr - s2 * bpu;
        A[p * ld + u] = s2 * bpr + c2 * bpu;
        A[q * ld + r] = c2 * bqr - s2 * bqu;
        A[q * ld + u] = s2 * bqr + c2 * bqu;
      }
      for (int k = wave; k < half; k += 16) {  // eigenvector columns p, q <- V J
        const int p = pq[2 * k], q = pq[2 * k + 1];
        const double c = cs[2 * k], s = cs[2 * k + 1];
        if (s == 0.0) continue;
        for (int i = lane; i < ne; i += 64) {
          const double vp = V[i * ld + p], vq = V[i * ld + q];
          V[i * ld + p] = c * vp - s * vq;
          V[i * ld + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  double* dg = cs;
  for (int k = tid; k < n; k += 1024) dg[k] = A[k * ld + k];
  __syncthreads();
  for (int k = tid; k < n; k += 1024) {
    const double lk = dg[k];
    int r = 0;
    for (int j = 0; j < n; ++j) r += (dg[j] > lk) || (dg[j] == lk && j < k);
    rk[k] = r;
    evals[r] = lk;
  }
  __syncthreads();
  for (int i = wave; i < n; i += 16)
    for (int k = lane; k < n; k += 64) {
      const double v = V[i * ld + k];
      W[(long)i * n + rk[k]] = v;
      Wt[(long)rk[k] * n + i] = v;
    }
}

// Cholesky G = L L^T and Linv = L^-1 for an n x n SPD matrix in one workgroup (in LDS up to
// n = 96). Factor: one barrier per column, the trailing update from the unscaled column
// (a_ij -= a_ik a_jk / a_kk), the columns scaled at the end. Inverse: forward substitution on the
// identity, one barrier per row, rows scaled at the end. A pivot below 1e-20 of the largest diagonal
// entry drops its direction (that row of Linv is 0).
__global__ __launch_bounds__(1024) void k_chol_inv(const double* __restrict__ G, int n, double* __restrict__ Linv,
                                                   double* __restrict__ gscratch) {
  extern __shared__ double dyn[];
  __shared__ double piv[JAC_MAX];
  __shared__ double red[16];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ld = n + 1;
  double* A = n <= JAC_LDS_MAX ? dyn : gscratch;
  double* X = A + (long)n * ld;
  double dm = 0.0;
  for (int i = wave; i < n; i += 16)
    for (int j = lane; j < n; j += 64) {
      const double g = G[(long)i * n + j];
      A[i * ld + j] = g;
      X[i * ld + j] = i == j ? 1.0 : 0.0;
      if (i == j) dm = fmax(dm, fabs(g));
    }
  dm = wave_max(dm);
  if (lane == 0) red[wave] = dm;
  __syncthreads();
  dm = 0.0;
  for (int w = 0; w < 16; ++w) dm = fmax(dm, red[w]);
  const double floor_ = 1e-20 * dm;
  for (int k = 0; k < n; ++k) {
    const double akk = A[k * ld + k];
    const bool ok = akk > floor_;
    if (tid == 0) piv[k] = ok ? akk : 0.0;
    if (ok) {
      const double inv = 1.0 / akk;
      const int m = n - k - 1;
      for (int e = tid; e < m * m; e += 1024) {  // lower triangle of the trailing block
        const int i = k + 1 + e / m, j = k + 1 + e % m;
        if (j <= i) A[i * ld + j] -= A[i * ld + k] * A[j * ld + k] * inv;
      }
    }
    __syncthreads();
  }
  // L = lower(A) with column k scaled by 1 / sqrt(piv_k); rows of dropped pivots are zero
  for (int i = wave; i < n; i += 16)
    for (int j = lane; j <= i; j += 64) {
      const double pj = piv[j];
      A[i * ld + j] = pj > 0.0 ? A[i * ld + j] / sqrt(pj) : 0.0;
    }
  __syncthreads();
  for (int k = 0; k < n; ++k) {  // rows i > k of X -= L_ik / L_kk * X_k (X_k not yet scaled)
    const double lkk = A[k * ld + k];
    if (lkk > 0.0) {
      const double inv = 1.0 / lkk;
      const int m = n - k - 1;
      for (int e = tid; e < m * (k + 1); e += 1024) {
        const int i = k + 1 + e / (k + 1), c = e % (k + 1);
        X[i * ld + c] -= A[i * ld + k] * inv * X[k * ld + c];
      }
    }
    __syncthreads();
  }
  for (int i = wave; i < n; i += 16) {
    const double lii = A[i * ld + i];
    for (int c = lane; c < n; c += 64)
      Linv[(long)i * n + c] = (lii > 0.0 && c <= i) ? X[i * ld + c] / lii : 0.0;
  }
}

// C = op(A) diag(d) op(B) for n x n matrices (op = transpose when the flag is set; d may be NULL)
__global__ void k_small_gemm(int n, const double* __restrict__ A, int ta, const double* __restrict__ B, int tb,
                             const double* __restrict__ d, double* __restrict__ C) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
      const double a = ta ? A[(long)k * n + i] : A[(long)i * n + k];
      const double bv = tb ? B[(long)j * n + k] : B[(long)k * n + j];
      s = fma(d ? a * d[k] : a, bv, s);
    }
    C[e] = s;
  }
}

// from the Gram of [Q; Z] (2b x 2b): T = sym(Q Z^T), ZZ = Z Z^T and QQ = Q Q^T
__global__ void k_eig_blocks(const double* __restrict__ G, int b, double* __restrict__ T, double* __restrict__ ZZ,
                             double* __restrict__ QQ) {
  const long nn = (long)b * b;
  const long ld = 2L * b;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / b), j = (int)(e % b);
    T[e] = 0.5 * (G[i * ld + b + j] + G[j * ld + b + i]);
    ZZ[e] = G[(long)(b + i) * ld + b + j];
    QQ[e] = G[i * ld + j];
  }
}

// Gy = Dn^-1 P Dn^-1 with Dn = diag(sqrt(P_kk)) (the Gram of the unit-norm rows); ninv = 1 / sqrt(P_kk)
__global__ void k_eig_unit_gram(const double* __restrict__ P, int n, double* __restrict__ Gy,
                                double* __restrict__ ninv) {
  const long nn = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double di = 1.0 / sqrt(fmax(P[(long)i * n + i], 1e-300));
    const double dj = 1.0 / sqrt(fmax(P[(long)j * n + j], 1e-300));
    Gy[e] = P[e] * di * dj;
    if (i == j) ninv[i] = di;
  }
}

// d_k = lambda_k^-1/2, or 0 below 1e-14 of the largest (lambda sorted decreasing)
__global__ void k_eig_rsqrt(const double* __restrict__ lam, int n, double* __restrict__ d) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    d[k] = lam[k] > 1e-14 * lam[0] ? 1.0 / sqrt(lam[k]) : 0.0;
}

// partial sums of |V_k - theta_k U_k|^2 for k < N over EIG_RSPLIT slices of M (workgroup (k, slice));
// the host adds the slices in order
constexpr int EIG_RSPLIT = 16;
__global__ __launch_bounds__(256) void k_eig_resid(const double* __restrict__ U, const double* __restrict__ V,
                                                   const double* __restrict__ theta, long M,
                                                   double* __restrict__ out) {
  __shared__ double red[4];
  const int k = blockIdx.x / EIG_RSPLIT, sl = blockIdx.x % EIG_RSPLIT;
  const double th = theta[k];
  const long chunk = (M + EIG_RSPLIT - 1) / EIG_RSPLIT;
  const long i0 = sl * chunk, i1 = i0 + chunk < M ? i0 + chunk : M;
  double s = 0.0;
  for (long i = i0 + threadIdx.x; i < i1; i += 256) {
    const double r = V[(long)k * M + i] - th * U[(long)k * M + i];
    s += r * r;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// control rows E[k] (component `comp` = U_k sqrt(theta_k (N - 1)) on the region's cells, other
// component 0) and mu = theta
__global__ void k_eig_extract(const double* __restrict__ U, const double* __restrict__ theta, int N, long M,
                              const int* __restrict__ bidx, int ncc, int comp, double* __restrict__ E,
                              double* __restrict__ mu) {
  const long m = 2L * ncc;
  const long n = (long)N * ncc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ncc), c = (int)(e % ncc);
    const double sc = sqrt(fmax(theta[k], 0.0) * (double)(N - 1));
    E[k * m + (long)comp * ncc + c] = U[(long)k * M + bidx[c]] * sc;
    E[k * m + (long)(1 - comp) * ncc + c] = 0.0;
    if (c == 0) mu[k] = theta[k];
  }
}

// ---------------------------------------------------------------------------- reconstruction error
// partial sums over 256-entry blocks of |f - sum_k coef_k E_k|^2 and |f|^2 (fixed order), then one
// workgroup sums the partials in order
__global__ __launch_bounds__(256) void k_recon_partial(const double* __restrict__ E, int N, long m,
                                                       const double* __restrict__ f, const double* __restrict__ coef,
                                                       double* __restrict__ part) {
  __shared__ double red[2][4];
  const long i = blockIdx.x * 256L + threadIdx.x;
  double r2 = 0.0, f2 = 0.0;
  if (i < m) {
    const double fi = f[i];
    double r = fi;
    for (int k = 0; k < N; ++k) r -= coef[k] * E[(long)k * m + i];
    r2 = r * r;
    f2 = fi * fi;
  }
  r2 = wave_sum(r2);
  f2 = wave_sum(f2);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = r2;
    red[1][threadIdx.x >> 6] = f2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    part[2 * blockIdx.x + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

// coef_k = (E_k . f) / |E_k|^2 from the two row dots
__global__ void k_recon_coef(const double* __restrict__ ef, const double* __restrict__ ee, int N,
                             double* __restrict__ coef) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x)
    coef[k] = ee[k] > 0.0 ? ef[k] / ee[k] : 0.0;
}

__global__ __launch_bounds__(256) void k_recon_final(const double* __restrict__ part, long nb,
                                                     double* __restrict__ out) {
  __shared__ double red[2][256];
  double r2 = 0.0, f2 = 0.0;
  for (long b = threadIdx.x; b < nb; b += 256) {
    r2 += part[2 * b];
    f2 += part[2 * b + 1];
  }
  red[0][threadIdx.x] = r2;
  red[1][threadIdx.x] = f2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int t = 0; t < 256; ++t) {
      a += red[0][t];
      c += red[1][t];
    }
    out[0] = c > 0.0 ? a / c : 0.0;
  }
}

// ---------------------------------------------------------------------------- launchers
static unsigned grid_for(long n, long cap = 4096) {
  long b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

void launch_eig_sigma(const int* bidx, int ncc, int nxb, int nyb, double h, double sig2max, int taper, double* sig,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_eig_sigma, dim3(grid_for(ncc)), dim3(256), 0, s, bidx, ncc, nxb, nyb, h, sig2max, taper, sig);
}
void launch_kernel1d(int n, double h, double a, double* K, hipStream_t s) {
  hipLaunchKernelGGL(k_kernel1d, dim3(grid_for((long)n * n)), dim3(256), 0, s, n, h, a, K);
}
void launch_eig_random(double* Q, int b, long M, const double* sig, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_random, dim3(grid_for((long)b * M)), dim3(256), 0, s, Q, b, M, sig, seed);
}
void launch_scale_rows(const double* Q, const double* sig, int rows, long M, double* W, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rows, dim3(grid_for((long)rows * M)), dim3(256), 0, s, Q, sig, (long)rows * M, M, W);
}
void launch_dgemm(int M, int N, int K, const double* A, long lda, long sA, const double* B, long ldb, long sB,
                  double* C, long ldc, long sC, int batch, const double* S, long lds, hipStream_t s) {
  hipLaunchKernelGGL(k_dgemm, dim3((N + 63) / 64, (M + 63) / 64, batch), dim3(256), 0, s, M, N, K, A, lda, sA, B, ldb,
                     sB, C, ldc, sC, S, lds);
}
size_t jacobi_scratch_doubles(int n) {
  const int ne = n + (n & 1);
  return ne <= JAC_LDS_MAX ? 0 : 2 * (size_t)ne * (ne + 1);
}
int launch_jacobi(const double* A, int lda, int n, double* evals, double* W, double* Wt, double* scratch,
                  hipStream_t s, int max_sweeps) {
  if (n < 1 || n > JAC_MAX) return -1;
  const int ne = n + (n & 1);
  const size_t dyn = ne <= JAC_LDS_MAX ? 2 * (size_t)ne * (ne + 1) * sizeof(double) : 0;
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * JAC_LDS_MAX * (JAC_LDS_MAX + 1) * (int)sizeof(double)) != hipSuccess)
      return -2;
    attr = true;
  }
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), dyn, s, A, lda, n, max_sweeps, evals, W, Wt, scratch);
  return 0;
}
int launch_chol_inv(const double* G, int n, double* Linv, double* scratch, hipStream_t s) {
  if (n < 1 || n > JAC_MAX) return -1;
  const size_t dyn = n <= JAC_LDS_MAX ? 2 * (size_t)n * (n + 1) * sizeof(double) : 0;
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * JAC_LDS_MAX * (JAC_LDS_MAX + 1) * (int)sizeof(double)) != hipSuccess)
      return -2;
    attr = true;
  }
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), dyn, s, G, n, Linv, scratch);
  return 0;
}
void launch_small_gemm(int n, const double* A, int ta, const double* B, int tb, const double* d, double* C,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_small_gemm, dim3(grid_for((long)n * n, 1024)), dim3(256), 0, s, n, A, ta, B, tb, d, C);
}
void launch_eig_blocks(const double* G, int b, double* T, double* ZZ, double* QQ, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_blocks, dim3(grid_for((long)b * b)), dim3(256), 0, s, G, b, T, ZZ, QQ);
}
void launch_eig_unit_gram(const double* P, int n, double* Gy, double* ninv, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_unit_gram, dim3(grid_for((long)n * n)), dim3(256), 0, s, P, n, Gy, ninv);
}
void launch_eig_rsqrt(const double* lam, int n, double* d, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_rsqrt, dim3(grid_for(n)), dim3(256), 0, s, lam, n, d);
}
void launch_eig_resid(const double* U, const double* V, const double* theta, int N, long M, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_eig_resid, dim3(N * EIG_RSPLIT), dim3(256), 0, s, U, V, theta, M, out);
}
int eig_resid_split() { return EIG_RSPLIT; }
void launch_eig_extract(const double* U, const double* theta, int N, long M, const int* bidx, int ncc, int comp,
                        double* E, double* mu, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_extract, dim3(grid_for((long)N * ncc)), dim3(256), 0, s, U, theta, N, M, bidx, ncc, comp,
                     E, mu);
}
long recon_blocks(long m) { return (m + 255) / 256; }
void launch_recon(const double* E, int N, long m, const double* f, const double* ef, const double* ee, double* coef,
                  double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_recon_coef, dim3(1), dim3(256), 0, s, ef, ee, N, coef);
  hipLaunchKernelGGL(k_recon_partial, dim3((unsigned)recon_blocks(m)), dim3(256), 0, s, E, N, m, f, coef, part);
  hipLaunchKernelGGL(k_recon_final, dim3(1), dim3(256), 0, s, part, recon_blocks(m), out);
}

}  // namespace envar
