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
constexpr int KB = 4 * NB;  // super-block: updates below it are delayed to its end
constexpr int LDS_DOUBLES = 2 * KT * TILE + NB * NB + 2 * NB + 2;

// One TILE x TILE tile of C at (i0, j0); see wg_gemm.  No trailing barrier.
// The k panels are staged in LDS (zero padded past m, n, k); the product runs
// on the FP64 matrix cores: wave w owns the 32 x 32 quarter at rows 32 (w & 1),
// columns 32 (w >> 1), as 2 x 2 blocks of 16 x 16.  One
// v_mfma_f64_16x16x4f64 takes A(i, k) from lane i + 16 k, B(k, j) from lane
// j + 16 k, and leaves C(4 r + lane / 16, lane % 16) in result register r.
typedef double f64x4 __attribute__((ext_vector_type(4)));

// r1 (may be null): a rank-one term subtracted from the result,
// C(i, j) = ... - r1[i] r1[j].
template <bool TA, bool TB, bool LOWER = false>
__device__ __forceinline__ void wg_gemm_tile(int i0, int j0, int m, int n, int k, double alpha,
                                             const double *__restrict__ A, int lda, const double *__restrict__ B,
                                             int ldb, double beta, double *C, int ldc, double *lds,
                                             const double *kscale, const double *r1 = nullptr) {
  double *As = lds;              // As[kk * TILE + i] = op(A)(i0 + i, k0 + kk)
  double *Bs = lds + KT * TILE;  // Bs[kk * TILE + j] = op(B)(k0 + kk, j0 + j)
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int rb = 32 * (wv & 1), cb = 32 * (wv >> 1);
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f64x4{0.0, 0.0, 0.0, 0.0};
  // The next k panel is loaded into registers while the matrix cores work on
  // the current one.
  constexpr int PER = KT * TILE / WG;
  double pa[PER], pb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + r * WG;
      int i, kk;
      if (!TA) { i = e & (TILE - 1); kk = e / TILE; }
      else { kk = e & (KT - 1); i = e / KT; }
      const int gi = i0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < k) {
        v = TA ? A[gk + (size_t)gi * lda] : A[gi + (size_t)gk * lda];
        if (kscale) v *= kscale[gk];
      }
      pa[r] = v;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + r * WG;
      int j, kk;
      if (!TB) { kk = e & (KT - 1); j = e / KT; }
      else { j = e & (TILE - 1); kk = e / TILE; }
      const int gj = j0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < n && gk < k) v = TB ? B[gj + (size_t)gk * ldb] : B[gk + (size_t)gj * ldb];
      pb[r] = v;
    }
  };
  load(0);
  for (int k0 = 0; k0 < k; k0 += KT) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + r * WG;
      if (!TA) As[(e / TILE) * TILE + (e & (TILE - 1))] = pa[r];
      else As[(e & (KT - 1)) * TILE + e / KT] = pa[r];
      if (!TB) Bs[(e & (KT - 1)) * TILE + e / KT] = pb[r];
      else Bs[(e / TILE) * TILE + (e & (TILE - 1))] = pb[r];
    }
    __syncthreads();
    if (k0 + KT < k) load(k0 + KT);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const double *Ak = As + (kk + lk) * TILE, *Bk = Bs + (kk + lk) * TILE;
      const double a0 = Ak[rb + li], a1 = Ak[rb + 16 + li];
      const double b0 = Bk[cb + li], b1 = Bk[cb + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + rb + 16 * bi + 4 * r + lk;
        const int gj = j0 + cb + 16 * bj + li;
        if (gi >= m || gj >= n) continue;
        if (LOWER && gj > gi) continue;
        double *dst = C + gi + (size_t)gj * ldc;
        const double v = acc[bi][bj][r];
        const double o = (beta == 0.0) ? alpha * v : fma(alpha, v, beta * (*dst));
        *dst = r1 ? fma(-r1[gi], r1[gj], o) : o;
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

// Diagonal block of a lower triangular matrix into LDS (ld NB), padded to
// NB x NB with the identity so that the substitutions below need no bounds:
// padded unknowns stay zero and never touch the real ones.
__device__ __forceinline__ void lds_load_lower_block(double *Lk, const double *L, int ldl, int k0, int nb) {
  for (int e = threadIdx.x; e < NB * NB; e += WG) {
    const int i = e % NB, j = e / NB;
    double v = (i == j) ? 1.0 : 0.0;
    if (i < nb && j < nb) v = (i >= j) ? L[(k0 + i) + (size_t)(k0 + j) * ldl] : 0.0;
    Lk[e] = v;
  }
}

// x <- Lk^{-1} x for one right-hand side held in registers (Lk padded as
// above).  Column oriented: x_i receives its updates in increasing order of
// the eliminated unknown, as in a row-wise forward substitution.  Padded
// entries x_j, j >= nb, may hold any value: no x_i with i < nb reads them.
__device__ __forceinline__ void lds_lower_solve(const double *Lk, double (&x)[NB]) {
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    // One column of Lk in flight at a time.  Without these empty asm
    // statements the compiler sinks each update to the step that next needs
    // x_i and keeps every block element read before it in registers (up to
    // NB (NB + 1) / 2 of them), which spills.
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = j; i < NB; ++i) asm volatile("" : "+v"(x[i]));
    x[j] = x[j] / Lk[j + j * NB];
#pragma unroll
    for (int i = j + 1; i < NB; ++i) x[i] = fma(-Lk[i + j * NB], x[j], x[i]);
  }
}

// x <- Lk^{-T} x for one right-hand side held in registers (Lk padded).
// Padded entries must be zero: they are eliminated first.
__device__ __forceinline__ void lds_lower_t_solve(const double *Lk, double (&x)[NB]) {
#pragma unroll
  for (int j = NB - 1; j >= 0; --j) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i <= j; ++i) asm volatile("" : "+v"(x[i]));
    x[j] = x[j] / Lk[j + j * NB];
#pragma unroll
    for (int i = 0; i < j; ++i) x[i] = fma(-Lk[j + i * NB], x[j], x[i]);
  }
}

// In-place blocked signed Cholesky of the n x n lower triangle of A:
// A = L diag(s) L^T with s = +-1 per column (s == nullptr: ordinary Cholesky).
// Returns 0, or (index + 1) of the first pivot whose sign disagrees with s.
// With nrows > n only the first n pivots are taken over the nrows x nrows
// lower triangle: rows n.. receive the panel A_{2,1} L_11^{-T} diag(s) and the
// trailing block the update A_22 - L_21 diag(s) L_21^T.
// defer_bb (with nrows > n): the trailing block A[n:, n:] is left untouched;
// the caller applies A[n:, n:] -= L_21 diag(s) L_21^T itself.
__device__ __forceinline__ int wg_potrf(int n, double *A, int lda, double *lds, const double *s = nullptr,
                                        int nrows = -1, bool defer_bb = false) {
  const int nr = nrows < 0 ? n : nrows;
  const int ncu = defer_bb ? n : nr;   // trailing updates reach columns < ncu
  double *Lk = lds + 2 * KT * TILE;  // NB x NB
  double *sk = Lk + NB * NB;         // NB signs
  int *flag = (int *)(sk + NB);      // pivot-failure word
  int fail = 0;
  const int tid = threadIdx.x;
  for (int kb0 = 0; kb0 < n; kb0 += KB) {
    const int kb1 = min(kb0 + KB, n);
    for (int k0 = kb0; k0 < kb1; k0 += NB) {
      const int nb = min(NB, n - k0);
      lds_load_lower_block(Lk, A, lda, k0, nb);
      if (tid < NB) sk[tid] = (tid < nb && s) ? s[k0 + tid] : 1.0;
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
        for (int j = 0; j < NB; ++j) x[j] = A[r + (size_t)(k0 + min(j, nb - 1)) * lda];
        lds_lower_solve(Lk, x);
        // recompute the row addresses and re-read the signs here rather than
        // keep NB of each live across the substitution
        int ld = lda;
        asm volatile("" : "+s"(ld) : : "memory");
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nb) A[r + (size_t)(k0 + j) * ld] = x[j] * sk[j];
      }
      __syncthreads();
      // the super-block's remaining columns: A[r0:, r0:kb1] -= X diag(s_k) X[r0:kb1]^T
      if (r0 < kb1) {
        double *X = A + r0 + (size_t)k0 * lda;
        wg_gemm<false, true, true>(nr - r0, kb1 - r0, nb, -1.0, X, lda, X, lda, 1.0,
                                   A + r0 + (size_t)r0 * lda, lda, lds, sk);
      }
    }
    // delayed trailing update by the whole super-block (lower triangle only)
    if (kb1 < nr && kb1 < ncu) {
      double *X = A + kb1 + (size_t)kb0 * lda;
      wg_gemm<false, true, true>(nr - kb1, ncu - kb1, kb1 - kb0, -1.0, X, lda, X, lda, 1.0,
                                 A + kb1 + (size_t)kb1 * lda, lda, lds, s ? s + kb0 : nullptr);
    }
  }
  return fail;
}

// B <- L^{-1} B  (L lower triangular n x n, B n x nrhs).
// lower_rhs: column c of B vanishes above row c (B = I, say), and so does the
// same column of L^{-1} B; block k0 then only involves columns < k0 + NB.
// Rows [ra, rb) (all >= n) of a partial signed factor whose leading n x n
// block wg_potrf(n, A, lda, lds, s, n, true) has factored: the panel solves
// and trailing updates that wg_potrf(n, A, lda, lds, s, nr, true) applies to
// those rows, in the same blocks and order, so the rows receive the same
// values.  Rows of different calls are independent (each update of a row
// reads only that row and the factored leading columns).
__device__ __forceinline__ void wg_potrf_rows(int n, double *A, int lda, double *lds, const double *s, int ra,
                                              int rb) {
  double *Lk = lds + 2 * KT * TILE;  // NB x NB
  double *sk = Lk + NB * NB;         // NB signs
  const int tid = threadIdx.x;
  for (int kb0 = 0; kb0 < n; kb0 += KB) {
    const int kb1 = min(kb0 + KB, n);
    for (int k0 = kb0; k0 < kb1; k0 += NB) {
      const int nb = min(NB, n - k0);
      lds_load_lower_block(Lk, A, lda, k0, nb);
      if (tid < NB) sk[tid] = (tid < nb && s) ? s[k0 + tid] : 1.0;
      __syncthreads();
      for (int r = ra + tid; r < rb; r += WG) {
        double x[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) x[j] = A[r + (size_t)(k0 + min(j, nb - 1)) * lda];
        lds_lower_solve(Lk, x);
        int ld = lda;
        asm volatile("" : "+s"(ld) : : "memory");
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nb) A[r + (size_t)(k0 + j) * ld] = x[j] * sk[j];
      }
      __syncthreads();
      const int r0 = k0 + nb;
      if (r0 < kb1)
        wg_gemm<false, true>(rb - ra, kb1 - r0, nb, -1.0, A + ra + (size_t)k0 * lda, lda, A + r0 + (size_t)k0 * lda,
                             lda, 1.0, A + ra + (size_t)r0 * lda, lda, lds, sk);
    }
    if (kb1 < n)
      wg_gemm<false, true>(rb - ra, n - kb1, kb1 - kb0, -1.0, A + ra + (size_t)kb0 * lda, lda,
                           A + kb1 + (size_t)kb0 * lda, lda, 1.0, A + ra + (size_t)kb1 * lda, lda, lds,
                           s ? s + kb0 : nullptr);
  }
}

__device__ __forceinline__ void wg_trsm_lower(int n, int nrhs, const double *L, int ldl, double *B, int ldb,
                                     double *lds, bool lower_rhs = false) {
  double *Lk = lds + 2 * KT * TILE;
  const int tid = threadIdx.x;
  for (int kb0 = 0; kb0 < n; kb0 += KB) {
    const int kb1 = min(kb0 + KB, n);
    for (int k0 = kb0; k0 < kb1; k0 += NB) {
      const int nb = min(NB, n - k0);
      const int ncol = lower_rhs ? min(nrhs, k0 + nb) : nrhs;
      lds_load_lower_block(Lk, L, ldl, k0, nb);
      __syncthreads();
      for (int c = tid; c < ncol; c += WG) {
        double *b = B + k0 + (size_t)c * ldb;
        double x[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) x[j] = (j < nb) ? b[j] : 0.0;
        lds_lower_solve(Lk, x);
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nb) b[j] = x[j];
      }
      __syncthreads();
      // the rest of the super-block's rows
      const int r0 = k0 + nb;
      if (r0 < kb1)
        wg_gemm<false, false>(kb1 - r0, ncol, nb, -1.0, L + r0 + (size_t)k0 * ldl, ldl, B + k0, ldb, 1.0,
                              B + r0, ldb, lds);
    }
    // delayed update of the rows below by the whole super-block
    if (kb1 < n) {
      const int ncol = lower_rhs ? min(nrhs, kb1) : nrhs;
      wg_gemm<false, false>(n - kb1, ncol, kb1 - kb0, -1.0, L + kb1 + (size_t)kb0 * ldl, ldl, B + kb0, ldb, 1.0,
                            B + kb1, ldb, lds);
    }
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
    lds_load_lower_block(Lk, L, ldl, k0, nb);
    __syncthreads();
    // solve L_kk^T x = b_k (backward substitution)
    for (int c = tid; c < nrhs; c += WG) {
      double *b = B + k0 + (size_t)c * ldb;
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) x[j] = (j < nb) ? b[j] : 0.0;
      lds_lower_t_solve(Lk, x);
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

// B[:, c] <- B[:, c] - (z . B[:, c]) z for the ncols columns of B (n rows,
// z of unit length).  Wave w takes columns w, w + 4, ... two at a time; its
// lanes split the rows and a butterfly sums the dot product.
__device__ __forceinline__ void wg_project_out(int n, const double *z, int ncols, double *B, int ldb) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int NW = WG / 64;
  for (int c = wv; c < ncols; c += 2 * NW) {
    const int c2 = min(c + NW, ncols - 1);
    const bool two = c + NW < ncols;
    double *b1 = B + (size_t)c * ldb, *b2 = B + (size_t)c2 * ldb;
    double d1 = 0.0, d2 = 0.0;
#pragma unroll 4
    for (int a = lane; a < n; a += 64) {
      const double za = z[a];
      d1 += za * b1[a];
      d2 += za * b2[a];
    }
    for (int o = 32; o > 0; o >>= 1) {
      d1 += __shfl_xor(d1, o, 64);
      d2 += __shfl_xor(d2, o, 64);
    }
#pragma unroll 4
    for (int a = lane; a < n; a += 64) {
      const double za = z[a];
      b1[a] -= d1 * za;
      if (two) b2[a] -= d2 * za;
    }
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

}  // namespace bddc
