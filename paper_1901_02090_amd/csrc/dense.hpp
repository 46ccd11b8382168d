// Dense FP64 linear algebra executed by one 256-thread workgroup.
//
// Every routine is called by all threads of the workgroup (uniform control
// flow) and ends with a barrier, so results are visible to the whole group.
// Matrices are column major: A(i, j) = A[i + j * lda].  Work arrays live in
// global memory (L2 resident for the sizes used here); `lds` is a scratch area
// of at least LDS_DOUBLES doubles in shared memory.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace bddc {

constexpr int WG = 256;
constexpr int TILE = 64;    // C tile edge of the workgroup GEMM
constexpr int KT = 16;      // k depth staged per LDS round
constexpr int NB = 32;      // block size of the blocked factorizations
constexpr int LDS_DOUBLES = 2 * KT * TILE + NB * NB + 2 * NB + 2;

// One TILE x TILE tile of C at (i0, j0); see wg_gemm.  No trailing barrier.
template <bool TA, bool TB, bool LOWER = false>
__device__ __forceinline__ void wg_gemm_tile(int i0, int j0, int m, int n, int k, double alpha,
                                             const double *__restrict__ A, int lda, const double *__restrict__ B,
                                             int ldb, double beta, double *C, int ldc, double *lds,
                                             const double *kscale) {
  double *As = lds;              // As[kk * TILE + i] = op(A)(i0 + i, k0 + kk)
  double *Bs = lds + KT * TILE;  // Bs[kk * TILE + j] = op(B)(k0 + kk, j0 + j)
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  {
    {
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      for (int k0 = 0; k0 < k; k0 += KT) {
        for (int e = tid; e < KT * TILE; e += WG) {
          int i, kk;
          if (!TA) { i = e & (TILE - 1); kk = e / TILE; }
          else { kk = e & (KT - 1); i = e / KT; }
          const int gi = i0 + i, gk = k0 + kk;
          double v = 0.0;
          if (gi < m && gk < k) {
            v = TA ? A[gk + (size_t)gi * lda] : A[gi + (size_t)gk * lda];
            if (kscale) v *= kscale[gk];
          }
          As[kk * TILE + i] = v;
        }
        for (int e = tid; e < KT * TILE; e += WG) {
          int j, kk;
          if (!TB) { kk = e & (KT - 1); j = e / KT; }
          else { j = e & (TILE - 1); kk = e / TILE; }
          const int gj = j0 + j, gk = k0 + kk;
          double v = 0.0;
          if (gj < n && gk < k) v = TB ? B[gj + (size_t)gk * ldb] : B[gk + (size_t)gj * ldb];
          Bs[kk * TILE + j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KT; ++kk) {
          double a[4], b[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = As[kk * TILE + ty + 16 * r];
#pragma unroll
          for (int c = 0; c < 4; ++c) b[c] = Bs[kk * TILE + tx + 16 * c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + ty + 16 * r;
        if (gi >= m) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int gj = j0 + tx + 16 * c;
          if (gj >= n) continue;
          if (LOWER && gj > gi) continue;
          double *dst = C + gi + (size_t)gj * ldc;
          *dst = (beta == 0.0) ? alpha * acc[r][c] : fma(alpha, acc[r][c], beta * (*dst));
        }
      }
    }
  }
}

// C = alpha * op(A) * op(B) * [diag(kscale)] + beta * C, op = transpose if TA/TB.
// op(A) is m x k, op(B) is k x n.  kscale (length k, may be null) multiplies
// column kk of op(A).  If LOWER, only tiles touching the lower triangle are
// computed and only entries with row >= column are written.
template <bool TA, bool TB, bool LOWER = false>
__device__ __forceinline__ void wg_gemm(int m, int n, int k, double alpha, const double *__restrict__ A, int lda,
                                        const double *__restrict__ B, int ldb, double beta, double *C, int ldc,
                                        double *lds, const double *kscale = nullptr) {
  for (int i0 = 0; i0 < m; i0 += TILE) {
    for (int j0 = 0; j0 < n; j0 += TILE) {
      if (LOWER && j0 > i0 + TILE - 1) continue;
      wg_gemm_tile<TA, TB, LOWER>(i0, j0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lds, kscale);
    }
  }
  __syncthreads();
}

// Unblocked signed Cholesky of an nb x nb block held in LDS (ld NB):
// K = L diag(s) L^T, s = +-1 (s == nullptr: all +1).  `flag` is one LDS word
// owned by the caller.  Returns the number of the first failing pivot + 1, or 0.
__device__ __forceinline__ int lds_sign_chol(double *L, int nb, const double *s, int *flag) {
  int &fail = *flag;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double sj = s ? s[j] : 1.0;
      const double d = sj * L[j + j * NB];
      if (!(d > 0.0) || !isfinite(d)) {
        if (!fail) fail = j + 1;
        L[j + j * NB] = 1.0;
      } else {
        L[j + j * NB] = sqrt(d);
      }
    }
    __syncthreads();
    const double sj = s ? s[j] : 1.0;
    const double inv = 1.0 / (sj * L[j + j * NB]);
    for (int i = j + 1 + tid; i < nb; i += WG) L[i + j * NB] *= inv;
    __syncthreads();
    // trailing update of the block: K(i,l) -= L(i,j) s_j L(l,j), i >= l > j
    const int m = nb - j - 1;
    for (int e = tid; e < m * m; e += WG) {
      const int i = j + 1 + e % m, l = j + 1 + e / m;
      if (i >= l) L[i + l * NB] -= L[i + j * NB] * sj * L[l + j * NB];
    }
    __syncthreads();
  }
  const int f = fail;
  __syncthreads();
  return f;
}

// In-place blocked signed Cholesky of the n x n lower triangle of A:
// A = L diag(s) L^T with s = +-1 per column (s == nullptr: ordinary Cholesky).
// Returns 0, or (index + 1) of the first pivot whose sign disagrees with s.
// With nrows > n only the first n pivots are taken over the nrows x nrows
// lower triangle: rows n.. receive the panel A_{2,1} L_11^{-T} diag(s) and the
// trailing block the update A_22 - L_21 diag(s) L_21^T.
__device__ __forceinline__ int wg_potrf(int n, double *A, int lda, double *lds, const double *s = nullptr,
                                        int nrows = -1) {
  const int nr = nrows < 0 ? n : nrows;
  double *Lk = lds + 2 * KT * TILE;  // NB x NB
  double *sk = Lk + NB * NB;         // NB signs
  int *flag = (int *)(sk + NB);      // pivot-failure word
  int fail = 0;
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = min(NB, n - k0);
    for (int e = tid; e < nb * nb; e += WG) {
      const int i = e % nb, j = e / nb;
      Lk[i + j * NB] = (i >= j) ? A[(k0 + i) + (size_t)(k0 + j) * lda] : 0.0;
    }
    if (tid < nb) sk[tid] = s ? s[k0 + tid] : 1.0;
    __syncthreads();
    const int f = lds_sign_chol(Lk, nb, sk, flag);
    if (f && !fail) fail = k0 + f;
    for (int e = tid; e < nb * nb; e += WG) {
      const int i = e % nb, j = e / nb;
      if (i >= j) A[(k0 + i) + (size_t)(k0 + j) * lda] = Lk[i + j * NB];
    }
    // panel: X with X diag(s_k) L_kk^T = A_panel  (row-wise forward substitution)
    const int r0 = k0 + nb;
    for (int r = r0 + tid; r < nr; r += WG) {
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          double v = A[r + (size_t)(k0 + j) * lda];
#pragma unroll
          for (int l = 0; l < j; ++l) v -= x[l] * Lk[j + l * NB];
          x[j] = v / Lk[j + j * NB];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < nb) A[r + (size_t)(k0 + j) * lda] = x[j] * sk[j];
    }
    __syncthreads();
    // trailing: A22 -= X diag(s_k) X^T  (lower triangle only)
    if (r0 < nr) {
      double *X = A + r0 + (size_t)k0 * lda;
      wg_gemm<false, true, true>(nr - r0, nr - r0, nb, -1.0, X, lda, X, lda, 1.0,
                                 A + r0 + (size_t)r0 * lda, lda, lds, sk);
    }
  }
  return fail;
}

// B <- L^{-1} B  (L lower triangular n x n, B n x nrhs).
__device__ __forceinline__ void wg_trsm_lower(int n, int nrhs, const double *L, int ldl, double *B, int ldb,
                                     double *lds) {
  double *Lk = lds + 2 * KT * TILE;
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = min(NB, n - k0);
    for (int e = tid; e < nb * nb; e += WG) {
      const int i = e % nb, j = e / nb;
      Lk[i + j * NB] = (i >= j) ? L[(k0 + i) + (size_t)(k0 + j) * ldl] : 0.0;
    }
    __syncthreads();
    for (int c = tid; c < nrhs; c += WG) {
      double *b = B + k0 + (size_t)c * ldb;
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          double v = b[j];
#pragma unroll
          for (int l = 0; l < j; ++l) v -= Lk[j + l * NB] * x[l];
          x[j] = v / Lk[j + j * NB];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < nb) b[j] = x[j];
    }
    __syncthreads();
    const int r0 = k0 + nb;
    if (r0 < n)
      wg_gemm<false, false>(n - r0, nrhs, nb, -1.0, L + r0 + (size_t)k0 * ldl, ldl, B + k0, ldb, 1.0,
                            B + r0, ldb, lds);
  }
}

// B <- L^{-T} B  (L lower triangular n x n, B n x nrhs).
__device__ __forceinline__ void wg_trsm_lower_t(int n, int nrhs, const double *L, int ldl, double *B, int ldb,
                                       double *lds) {
  double *Lk = lds + 2 * KT * TILE;
  const int tid = threadIdx.x;
  const int nblk = (n + NB - 1) / NB;
  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int k0 = kb * NB;
    const int nb = min(NB, n - k0);
    for (int e = tid; e < nb * nb; e += WG) {
      const int i = e % nb, j = e / nb;
      Lk[i + j * NB] = (i >= j) ? L[(k0 + i) + (size_t)(k0 + j) * ldl] : 0.0;
    }
    __syncthreads();
    // solve L_kk^T x = b_k (backward substitution)
    for (int c = tid; c < nrhs; c += WG) {
      double *b = B + k0 + (size_t)c * ldb;
      double x[NB];
#pragma unroll
      for (int jj = NB - 1; jj >= 0; --jj) {
        if (jj < nb) {
          double v = b[jj];
#pragma unroll
          for (int l = jj + 1; l < NB; ++l)
            if (l < nb) v -= Lk[l + jj * NB] * x[l];
          x[jj] = v / Lk[jj + jj * NB];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < nb) b[j] = x[j];
    }
    __syncthreads();
    // B[0:k0] -= L[k0:k0+nb, 0:k0]^T B[k0:k0+nb]
    if (k0 > 0)
      wg_gemm<true, false>(k0, nrhs, nb, -1.0, L + k0, ldl, B + k0, ldb, 1.0, B, ldb, lds);
  }
}

// Copy / fill helpers.
__device__ __forceinline__ void wg_set_identity(int n, double *A, int lda) {
  for (int e = threadIdx.x; e < n * n; e += WG) {
    const int i = e % n, j = e / n;
    A[i + (size_t)j * lda] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
}

// Zero the strict upper triangle (after an in-place factorization).
__device__ __forceinline__ void wg_zero_upper(int n, double *A, int lda) {
  for (int e = threadIdx.x; e < n * n; e += WG) {
    const int i = e % n, j = e / n;
    if (j > i) A[i + (size_t)j * lda] = 0.0;
  }
  __syncthreads();
}

// Symmetrise from the lower triangle.
__device__ __forceinline__ void wg_symmetrize_lower(int n, double *A, int lda) {
  for (int e = threadIdx.x; e < n * n; e += WG) {
    const int i = e % n, j = e / n;
    if (j > i) A[i + (size_t)j * lda] = A[j + (size_t)i * lda];
  }
  __syncthreads();
}

// Workgroup sum reduction (all threads receive the result).
__device__ __forceinline__ double wg_sum(double v, double *red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < WG / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Cyclic Jacobi eigensolver for a symmetric n x n matrix A (n <= 256) with a
// parallel round-robin pair ordering.  On exit A is diagonal (eigenvalues on
// the diagonal) and V holds the eigenvectors as columns.  `pairs` is a shared
// buffer of at least 3 * 128 doubles + 256 ints.
__device__ __forceinline__ void wg_jacobi(int n, double *A, int lda, double *V, int ldv, double *shared,
                                 int *perm, int max_sweeps = 40) {
  const int tid = threadIdx.x;
  double *cs = shared;          // cos per pair
  double *sn = shared + 128;    // sin per pair
  double *red = shared + 256;   // reduction scratch (4)
  wg_set_identity(n, V, ldv);
  const int m = (n + 1) & ~1;   // even number of players (n odd: one bye)
  const int npair = m / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal mass vs diagonal mass
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += WG) {
      const int i = e % n, j = e / n;
      const double a = A[i + (size_t)j * lda];
      if (i == j) dia += a * a; else off += a * a;
    }
    off = wg_sum(off, red);
    dia = wg_sum(dia, red);
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int round = 0; round < m - 1; ++round) {
      // round-robin schedule: player 0 fixed, others rotate
      if (tid < m) {
        int p;
        if (tid == 0) p = 0;
        else p = 1 + ((tid - 1 + round) % (m - 1));
        perm[tid] = p;
      }
      __syncthreads();
      if (tid < npair) {
        int p = perm[tid], q = perm[m - 1 - tid];
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p + (size_t)q * lda];
          if (apq != 0.0) {
            const double app = A[p + (size_t)p * lda], aqq = A[q + (size_t)q * lda];
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < npair * n; e += WG) {
        const int t = e % npair, k = e / npair;
        int p = perm[t], q = perm[m - 1 - t];
        if (p > q) { const int x = p; p = q; q = x; }
        if (q >= n) continue;
        const double c = cs[t], s = sn[t];
        const double ap = A[p + (size_t)k * lda], aq = A[q + (size_t)k * lda];
        A[p + (size_t)k * lda] = c * ap - s * aq;
        A[q + (size_t)k * lda] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < npair * n; e += WG) {
        const int t = e % npair, k = e / npair;
        int p = perm[t], q = perm[m - 1 - t];
        if (p > q) { const int x = p; p = q; q = x; }
        if (q >= n) continue;
        const double c = cs[t], s = sn[t];
        const double ap = A[k + (size_t)p * lda], aq = A[k + (size_t)q * lda];
        A[k + (size_t)p * lda] = c * ap - s * aq;
        A[k + (size_t)q * lda] = s * ap + c * aq;
        const double vp = V[k + (size_t)p * ldv], vq = V[k + (size_t)q * ldv];
        V[k + (size_t)p * ldv] = c * vp - s * vq;
        V[k + (size_t)q * ldv] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

}  // namespace bddc
