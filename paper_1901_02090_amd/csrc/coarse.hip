// Coarse saddle point of Algorithm "BDDC preconditioner" (step 1 of the
// preconditioner and step 1 of Algorithm "BDDC method").
//
// The coarse unknowns are ordered slab by slab along the axis with the most
// subdomains: block j holds the coarse dofs of the faces inside super-slab j,
// then those of the faces between super-slabs j and j+1, then the rescaled
// pressures of the subdomains of super-slab j (the last subdomain's pressure is
// pinned).  A face touches at most two adjacent super-slabs, so the matrix is
// block tridiagonal; the faces between j and j+1 and the pressures of j form the
// "tail" of block j, the only columns through which block j couples forward.
// In this order the signed block Cholesky K = L diag(+-1) L^T (+1 on fluxes,
// -1 on pressures) needs no pivoting: every leading principal submatrix is a
// saddle point whose divergence rows have full rank.
//
// Setup: D_j -= L_{j,j-1} S L_{j,j-1}^T, D_j = L_jj S_j L_jj^T, Linv_j = L_jj^{-1},
// L_{j+1,j} = K_{j+1,j} Linv_j^T S_j.  Per solve, a forward sweep
// y_j = Linv_j b_j - M_j y_{j-1}[tail] (M_j = Linv_j L_{j,j-1}) and a backward
// sweep x_j = Linv_j^T (S_j y_j - [0; L_{j+1,j}^T x_{j+1}]): streamed GEMVs.
#include "common.hpp"
#include "dense.hpp"

namespace bddc {

// Device-wide GEMM: one TILE x TILE tile of C per workgroup (2D grid).
template <bool TA, bool TB, bool LOWER>
__global__ __launch_bounds__(256) void k_gemm_tiles(int m, int n, int k, double alpha, const double *__restrict__ A,
                                                    int lda, const double *__restrict__ B, int ldb, double beta,
                                                    double *C, int ldc, const double *kscale) {
  __shared__ double lds[LDS_DOUBLES];
  const int i0 = blockIdx.x * TILE, j0 = blockIdx.y * TILE;
  if (LOWER && j0 > i0 + TILE - 1) return;
  wg_gemm_tile<TA, TB, LOWER>(i0, j0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lds, kscale);
}

// Whole signed Cholesky in one workgroup (small blocks).
__global__ __launch_bounds__(256) void k_potrf_one(int b, double *D, const double *sgn, int *err) {
  __shared__ double lds[LDS_DOUBLES];
  if (wg_potrf(b, D, b, lds, sgn)) {
    if (threadIdx.x == 0) atomicOr(err, 64);
  }
}

// Diagonal nb x nb block at k0 of a device-wide blocked factorization.
__global__ __launch_bounds__(256) void k_potrf_diag(int b, double *D, int k0, int nb, const double *sgn, int *err) {
  __shared__ double lds[LDS_DOUBLES];
  if (wg_potrf(nb, D + k0 + (size_t)k0 * b, b, lds, sgn + k0)) {
    if (threadIdx.x == 0) atomicOr(err, 64);
  }
}

// Panel below the diagonal block: rows r >= k0 + nb, X = A_panel L_kk^{-T} diag(s).
__global__ __launch_bounds__(256) void k_potrf_panel(int b, double *D, int k0, int nb, const double *sgn) {
  __shared__ double Lk[NB * NB];
  __shared__ double sk[NB];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    Lk[i + j * NB] = (i >= j) ? D[(k0 + i) + (size_t)(k0 + j) * b] : 0.0;
  }
  if (threadIdx.x < nb) sk[threadIdx.x] = sgn[k0 + threadIdx.x];
  __syncthreads();
  const int r = k0 + nb + blockIdx.x * 256 + threadIdx.x;
  if (r >= b) return;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {
      double v = D[r + (size_t)(k0 + j) * b];
#pragma unroll
      for (int l = 0; l < j; ++l) v -= x[l] * Lk[j + l * NB];
      x[j] = v / Lk[j + j * NB];
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < nb) D[r + (size_t)(k0 + j) * b] = x[j] * sk[j];
}

// W[:, c0:c0+w] = L^{-1}[:, c0:c0+w] for lower-triangular L (b x b); one
// workgroup per column block of width w (the inverse's columns are independent).
__global__ __launch_bounds__(256) void k_trtri_cols(int b, const double *__restrict__ L, double *W, int w) {
  __shared__ double lds[LDS_DOUBLES];
  const int c0 = blockIdx.x * w;
  const int nc = min(w, b - c0);
  for (int e = threadIdx.x; e < b * nc; e += 256) {
    const int r = e % b, c = c0 + e / b;
    W[r + (size_t)c * b] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_trsm_lower(b - c0, nc, L + c0 + (size_t)c0 * b, b, W + c0 + (size_t)c0 * b, b, lds);
}

// Row-packed and column-packed copies of the lower triangle of W (b x b).
__global__ void k_pack_lower(int b, const double *__restrict__ W, double *rowp, double *colp) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)b * b) return;
  const int r = (int)(e % b), c = (int)(e / b);
  if (r < c) return;
  const double v = W[e];
  rowp[(int64_t)r * (r + 1) / 2 + c] = v;
  colp[(int64_t)c * b - (int64_t)c * (c - 1) / 2 + (r - c)] = v;
}

// Column-major (m x n) to row-major copy.
__global__ void k_to_rowmajor(int m, int n, const double *__restrict__ A, double *out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int r = (int)(e % m), c = (int)(e / m);
  out[(int64_t)r * n + c] = A[e];
}

__global__ void k_scale_cols(int m, int n, double *A, int lda, const double *__restrict__ s) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int r = (int)(e % m), c = (int)(e / m);
  A[r + (size_t)c * lda] *= s[c];
}

// Scatter the local coarse matrices A_c^i and the divergence rows B_c into the
// diagonal blocks D_j (dense, column major) and the sub-diagonal tail blocks
// E_j = K_{j+1,j}[:, tail_j] (b_{j+1} x t_j, column major).  An entry receives at
// most two contributions (a face has two subdomains), so the atomic sums are
// order independent.
struct BlockMap {
  int J;
  const int *blk;          // [nk] block of every coarse index
  const int *boff, *toff;  // [J+1], [J]
  double *D;               // diagonal blocks
  const int64_t *d_off;
  double *E;               // tail blocks
  const int64_t *e_off;
};

__device__ __forceinline__ void blk_add(const BlockMap &bm, int ga, int gb, double v, bool atomic) {
  const int ja = bm.blk[ga], jb = bm.blk[gb];
  if (ja == jb) {
    const int bsz = bm.boff[ja + 1] - bm.boff[ja];
    double *p = bm.D + bm.d_off[ja] + (ga - bm.boff[ja]) + (size_t)(gb - bm.boff[ja]) * bsz;
    if (atomic) atomicAdd(p, v); else *p = v;
  } else if (ja == jb + 1) {
    const int bsz = bm.boff[ja + 1] - bm.boff[ja];
    double *p = bm.E + bm.e_off[jb] + (ga - bm.boff[ja]) + (size_t)(gb - bm.toff[jb]) * bsz;
    if (atomic) atomicAdd(p, v); else *p = v;
  }
}

__global__ __launch_bounds__(256) void k_block_assemble(DevGeom g, DevCoarse cs, BlockMap bm, const double *Ac,
                                                        const int64_t *ac_off, const double *dscale) {
  const int i = blockIdx.x;
  const int c0 = cs.sub_coff[i];
  const int nci = cs.sub_coff[i + 1] - c0;
  const double *A = Ac + ac_off[i];
  for (int e = threadIdx.x; e < nci * nci; e += WG) {
    const int a = e % nci, b = e / nci;
    blk_add(bm, cs.sub_cmap[c0 + a], cs.sub_cmap[c0 + b], A[e], true);
  }
  const int pi = cs.pidx[i];
  if (pi >= 0) {
    for (int t = g.sub_face_off[i] + threadIdx.x; t < g.sub_face_off[i + 1]; t += WG) {
      const int f = g.sub_faces[t];
      const double s = (g.f_minus[f] == i) ? 1.0 : -1.0;   // +1: face orientation leaves Omega^i
      const double val = -dscale[i] * s;
      const int jf = cs.face_cofs[f];
      blk_add(bm, pi, jf, val, false);
      blk_add(bm, jf, pi, val, false);
    }
  }
}

// ---- per-iteration sweep -----------------------------------------------------
struct CgState;
__device__ __forceinline__ double wave_sum_c(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum over 256 threads (four waves); every thread gets the result.
__device__ __forceinline__ double block_sum256(double v, double *red) {
  v = wave_sum_c(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Each of the sweep GEMVs gives one workgroup per output entry: a row (or
// column) of a few thousand entries is covered by 256 lanes with four
// independent loads in flight each, so one entry costs about one memory round
// trip instead of a chain of them.

// y[r] = sum_{c<=r} Linv[r,c] b[c] - sum_t M[r,t] yprev[t].  Workgroup k
// computes rows k and b-1-k, which together hold b+1 triangle entries, so
// every workgroup streams the same amount.
__device__ __forceinline__ double cfwd_row(int r, const double *__restrict__ rowp, const double *__restrict__ bvec,
                                           const double *__restrict__ M, int tprev, const double *__restrict__ yprev,
                                           double *red) {
  const int tid = threadIdx.x;
  const double *row = rowp + (int64_t)r * (r + 1) / 2;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = tid; c0 <= r; c0 += 1024) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + 256 * u;
      if (c <= r) a[u] = fma(row[c], bvec[c], a[u]);
    }
  }
  if (M) {
    const double *mr = M + (int64_t)r * tprev;
    for (int t0 = tid; t0 < tprev; t0 += 1024) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + 256 * u;
        if (t < tprev) a[u] = fma(-mr[t], yprev[t], a[u]);
      }
    }
  }
  return block_sum256((a[0] + a[1]) + (a[2] + a[3]), red);
}

__global__ __launch_bounds__(256) void k_cfwd(int bsz, const double *__restrict__ rowp, const double *__restrict__ bvec,
                                              const double *__restrict__ M, int tprev,
                                              const double *__restrict__ yprev, double *__restrict__ y,
                                              const int *done) {
  __shared__ double red[8];
  if (done && *done) return;
  const int r1 = blockIdx.x, r2 = bsz - 1 - blockIdx.x;
  const double s1 = cfwd_row(r1, rowp, bvec, M, tprev, yprev, red);
  if (r2 > r1) {
    const double s2 = cfwd_row(r2, rowp, bvec, M, tprev, yprev, red + 4);
    if (threadIdx.x == 0) y[r2] = s2;
  }
  if (threadIdx.x == 0) y[r1] = s1;
}

// u[t] = sum_r Lc[r,t] x[r]  (Lc: bnext x t, column major)
__global__ __launch_bounds__(256) void k_cbwd_u(int bnext, int tcur, const double *__restrict__ Lc,
                                                const double *__restrict__ x, double *__restrict__ u, const int *done) {
  __shared__ double red[4];
  if (done && *done) return;
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const double *col = Lc + (int64_t)t * bnext;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = tid; r0 < bnext; r0 += 1024) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 256 * q;
      if (r < bnext) a[q] = fma(col[r], x[r], a[q]);
    }
  }
  const double s = block_sum256((a[0] + a[1]) + (a[2] + a[3]), red);
  if (tid == 0) u[t] = s;
}

// x[c] = sum_{r>=c} Linv[r,c] (s_r y[r] - u[r - ts]); workgroup k computes
// columns k and b-1-k.
__device__ __forceinline__ double cbwd_col(int c, int bsz, const double *__restrict__ colp,
                                           const double *__restrict__ y, const double *__restrict__ sg,
                                           const double *__restrict__ u, int ts, double *red) {
  const int tid = threadIdx.x;
  const double *col = colp + (int64_t)c * bsz - (int64_t)c * (c - 1) / 2;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = c + tid; r0 < bsz; r0 += 1024) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + 256 * q;
      if (r < bsz) {
        double v = sg[r] * y[r];
        if (u && r >= ts) v -= u[r - ts];
        a[q] = fma(col[r - c], v, a[q]);
      }
    }
  }
  return block_sum256((a[0] + a[1]) + (a[2] + a[3]), red);
}

__global__ __launch_bounds__(256) void k_cbwd_x(int bsz, const double *__restrict__ colp, const double *__restrict__ y,
                                                const double *__restrict__ sg, const double *__restrict__ u, int ts,
                                                double *__restrict__ x, const int *done) {
  __shared__ double red[8];
  if (done && *done) return;
  const int c1 = blockIdx.x, c2 = bsz - 1 - blockIdx.x;
  const double s1 = cbwd_col(c1, bsz, colp, y, sg, u, ts, red);
  if (c2 > c1) {
    const double s2 = cbwd_col(c2, bsz, colp, y, sg, u, ts, red + 4);
    if (threadIdx.x == 0) x[c2] = s2;
  }
  if (threadIdx.x == 0) x[c1] = s1;
}

}  // namespace bddc
