// Setup kernels: everything the CG loop of step 3 consumes.
//
// Per subdomain (one 256-thread workgroup each):
//   * the RT0 coefficients m_d = h_d / (k_d prod_{e != d} h_e) of every cell and
//     direction (the exact mass matrix of a rectangle with diagonal k decouples
//     by direction, Section 2 eq. a) and the rescaling d_i (Section 5);
//   * the interface Schur complement S^i of the Stokes-harmonic extension
//     (Section 3, mapping P; Section 4, S^{ij}) by structured elimination: the
//     interior mass matrix is tridiagonal along every grid line, so
//     G = A_II^{-1} is applied line by line; the cell-pressure system
//     P = B_I G B_I^T is dense per subdomain and has the constants as kernel,
//     which the zero-mean condition C_Q^i p = 0 (eq. Qi-def) removes;
//     S^i = (A_GG - A_GI G A_IG) + H^T X H with H = B_G - B_I G A_IG and X the
//     generalized inverse of P on the zero-mean subspace;
//   * the pair eigenproblems of every face (eq. eigenvalue-problem-local-matrix)
//     in reduced form (see k_face_reduce) and the adaptive rows (eq. constraints,
//     Algorithm "Adaptive BDDC");
//   * the coarse basis Psi^i, the coarse matrix block A_c^i and the substructure
//     operator T^i of Algorithm "BDDC preconditioner" from one Cholesky factor
//     of S^i;
//   * the coarse saddle point and its inverse.
#include "common.hpp"
#include "dense.hpp"

namespace bddc {

// ---------------------------------------------------------------------------
// line helpers
// ---------------------------------------------------------------------------

// Local cells of line `l` along direction d: start + t * st[d], t in [0, ext[d]).
__device__ __forceinline__ int line_start(int d, int l, const int *ext, const int *st) {
  int a0 = -1, a1 = -1;
  for (int e = 0; e < 3; ++e)
    if (e != d) { if (a0 < 0) a0 = e; else a1 = e; }
  const int v0 = l % ext[a0], v1 = l / ext[a0];
  return v0 * st[a0] + v1 * st[a1];
}

// Solve the interior-face system of one line of n cells: faces j = 1..n-1,
// diagonal (m[j-1] + m[j]) / 3, coupling of faces j and j+1 through cell j:
// m[j] / 6.  y[1..n-1] holds the right-hand side on entry, the solution on exit.
template <int CAP>
__device__ __forceinline__ void line_solve(int n, const double *m, double *y) {
  double cp[CAP];
  if (n < 2) return;
  double den = (m[0] + m[1]) / 3.0;
  cp[1] = (n > 2) ? (m[1] / 6.0) / den : 0.0;
  y[1] = y[1] / den;
  for (int j = 2; j <= n - 1; ++j) {
    const double e = m[j - 1] / 6.0;
    den = (m[j - 1] + m[j]) / 3.0 - e * cp[j - 1];
    cp[j] = (j <= n - 2) ? (m[j] / 6.0) / den : 0.0;
    y[j] = (y[j] - e * y[j - 1]) / den;
  }
  for (int j = n - 2; j >= 1; --j) y[j] -= cp[j] * y[j + 1];
}

// (B_l y)[c] for the line's cells: cell c has -d face c (B = +1) and +d face
// c+1 (B = -1); only interior faces 1..n-1 carry y.
__device__ __forceinline__ double line_B(int n, const double *y, int c) {
  double v = 0.0;
  if (c >= 1) v += y[c];
  if (c + 1 <= n - 1) v -= y[c + 1];
  return v;
}

__global__ void k_cell_coef(DevGeom g, const double *__restrict__ perm, int64_t ncells,
                            double *__restrict__ mcoef, int *err) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  for (int d = 0; d < 3; ++d) {
    double m = 0.0;
    if (d < g.dim) {
      const double k = perm[c * g.dim + d];
      if (!(k > 0.0) || !isfinite(k)) atomicOr(err, 1);
      double other = 1.0;
      for (int e = 0; e < g.dim; ++e)
        if (e != d) other *= g.h[e];
      m = g.h[d] / (k * other);
    }
    mcoef[c * 3 + d] = m;
  }
}

// Weights of the averaging operator E for stiffness scaling (Section 6; for
// RT0 the same as rho-scaling).  On the face between i and j, a_s is the mean
// over the face's dofs of the diagonal entry of A^s there (m / 3 of the cell of
// Omega^s next to the face); the two copies are weighted a_i / (a_i + a_j) and
// a_j / (a_i + a_j), constant along the face as the Remark on the starting
// flux constraints requires.  One wave per face.
__global__ __launch_bounds__(64) void k_face_weights(DevGeom g, const double *__restrict__ mcoef, double *fwm,
                                                     double *fwp, double *lw) {
  const int f = blockIdx.x, lane = threadIdx.x;
  const int i = g.f_minus[f], j = g.f_plus[f], n = g.f_n[f];
  const int64_t bi = g.g_off[i] + g.f_loffm[f], bj = g.g_off[j] + g.f_loffp[f];
  auto diag = [&](int sd, int64_t fl) {
    const int gc = g.lcell_global[g.cell_off[sd] + g.lg_cell[fl]];
    return mcoef[(int64_t)gc * 3 + g.lg_dir[fl]] / 3.0;
  };
  double si = 0.0, sj = 0.0;
  for (int a = lane; a < n; a += 64) {
    si += diag(i, bi + a);
    sj += diag(j, bj + a);
  }
  for (int o = 32; o > 0; o >>= 1) {
    si += __shfl_xor(si, o, 64);
    sj += __shfl_xor(sj, o, 64);
  }
  const double ai = si / n, aj = sj / n;
  const double wi = ai / (ai + aj), wj = aj / (ai + aj);
  if (lane == 0) {
    fwm[f] = wi;
    fwp[f] = wj;
  }
  for (int a = lane; a < n; a += 64) {
    lw[bi + a] = wi;
    lw[bj + a] = wj;
  }
}

// ---------------------------------------------------------------------------
// per-subdomain: d_i, P, H, S_A, L_P, S^i, X^i
// ---------------------------------------------------------------------------
// Subdomains of split .. split_max cells (split = 0: none) stop before the
// Cholesky of P~ (step 4): k_pchol_diag / _panel / _update factor P~ by
// blocks over many workgroups, then k_ls_solve, k_ls_project, k_ls_gemm and
// k_ls_sym finish steps 5-7 (the same quantities, summed in another order:
// X^i through the rank-one form below).
template <int CAP>
__global__ __launch_bounds__(256, 2) void k_local_setup(DevGeom g, const double *__restrict__ mcoef,
                                                     SetupWs ws, double *dscale, int *err, int split,
                                                     int split_max) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ double red[8];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  int ext[3], lo[3], st[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = g.ext[3 * i + d];
    lo[d] = g.lo[3 * i + d];
  }
  st[0] = 1;
  st[1] = ext[0];
  st[2] = ext[0] * ext[1];
  const int nc = g.nc[i], nG = g.nG[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double *P = ws.base + ws.P[i];
  double *V = ws.base + ws.V[i];
  double *H = ws.base + ws.H[i];
  double *S = ws.base + ws.S[i];
  double *X = ws.Xmat + ws.X[i];
  const int64_t goff = g.g_off[i];
  auto mloc = [&](int lc, int d) { return mcoef[(int64_t)lcg[lc] * 3 + d]; };

  // (1) rescaling: mean of the subdomain's assembled diag(A) over its flux dofs
  double acc = 0.0;
  int nI = 0;
  for (int d = 0; d < g.dim; ++d) {
    const int n = ext[d], lines = nc / n;
    nI += lines * (n - 1);
    for (int l = tid; l < lines; l += WG) {
      const int s0 = line_start(d, l, ext, st);
      for (int j = 1; j <= n - 1; ++j)
        acc += (mloc(s0 + (j - 1) * st[d], d) + mloc(s0 + j * st[d], d)) / 3.0;
      if (lo[d] > 0) acc += mloc(s0, d) / 3.0;
      if (lo[d] + n < g.n[d]) acc += mloc(s0 + (n - 1) * st[d], d) / 3.0;
    }
  }
  const double tot = wg_sum(acc, red);
  if (tid == 0) dscale[i] = tot / (double)(nI + nG);

  // (2) P = sum over lines of B_l G_l B_l^T
  for (int e = tid; e < nc * nc; e += WG) P[e] = 0.0;
  __syncthreads();
  for (int d = 0; d < g.dim; ++d) {
    const int n = ext[d], lines = nc / n;
    if (n >= 2) {
      for (int it = tid; it < lines * n; it += WG) {
        const int l = it / n, c = it % n;
        const int s0 = line_start(d, l, ext, st);
        double m[CAP], y[CAP + 1];
        for (int t = 0; t < n; ++t) m[t] = mloc(s0 + t * st[d], d);
        for (int j = 0; j <= n; ++j) y[j] = 0.0;
        if (c >= 1) y[c] += 1.0;
        if (c + 1 <= n - 1) y[c + 1] -= 1.0;
        line_solve<CAP>(n, m, y);
        const int colc = s0 + c * st[d];
        for (int cp = 0; cp < n; ++cp) P[(s0 + cp * st[d]) + (size_t)colc * nc] += line_B(n, y, cp);
      }
    }
    __syncthreads();
  }

  // (3) H = B_G - B_I G A_IG (line supported columns), S_A into S, c into H[:, nG]
  const int ldh = nc;
  for (int e = tid; e < nc * (nG + 1); e += WG) H[e] = (e >= nc * nG) ? g.vol : 0.0;
  for (int e = tid; e < nG * nG; e += WG) S[e] = 0.0;
  __syncthreads();
  for (int t = tid; t < nG; t += WG) {
    const int64_t fl = goff + t;
    const int d = g.lg_dir[fl], lc = g.lg_cell[fl], end = g.lg_end[fl];
    const int n = ext[d];
    const int cd = (lc / st[d]) % n;
    const int s0 = lc - cd * st[d];
    double m[CAP], y[CAP + 1];
    for (int u = 0; u < n; ++u) m[u] = mloc(s0 + u * st[d], d);
    const int eidx = end ? n - 1 : 0;
    const double mend = m[eidx];
    H[(s0 + eidx * st[d]) + (size_t)t * ldh] += end ? -1.0 : 1.0;
    const int p = g.lg_partner[fl];
    if (n >= 2) {
      const int adj = end ? n - 1 : 1, oadj = end ? 1 : n - 1;
      for (int j = 0; j <= n; ++j) y[j] = 0.0;
      y[adj] = 1.0;
      line_solve<CAP>(n, m, y);
      for (int cp = 0; cp < n; ++cp)
        H[(s0 + cp * st[d]) + (size_t)t * ldh] -= (mend / 6.0) * line_B(n, y, cp);
      S[t + (size_t)t * nG] += mend / 3.0 - (mend / 6.0) * (mend / 6.0) * y[adj];
      if (p >= 0) {
        const double moth = m[end ? 0 : n - 1];
        S[t + (size_t)p * nG] += -(mend / 6.0) * (moth / 6.0) * y[oadj];
      }
    } else {
      S[t + (size_t)t * nG] += mend / 3.0;
      if (p >= 0) S[t + (size_t)p * nG] += mend / 6.0;
    }
  }
  __syncthreads();

  // (4) P~ = P + (tr P / nc^2) 1 1^T is positive definite (kernel of P = constants)
  double tr = 0.0;
  for (int a = tid; a < nc; a += WG) tr += P[a + (size_t)a * nc];
  tr = wg_sum(tr, red);
  const double shift = (tr > 0.0) ? tr / ((double)nc * nc) : 1.0;
  for (int e = tid; e < nc * nc; e += WG) P[e] += shift;
  __syncthreads();
  if (split > 0 && nc >= split && nc <= split_max) return;   // factored by k_pchol_*
  if (wg_potrf(nc, P, nc, lds)) {
    if (tid == 0) atomicOr(err, 2);
  }
  // (5) Y = L_P^{-1} [H c]
  wg_trsm_lower(nc, nG + 1, P, nc, H, ldh, lds);
  double *zc = H + (size_t)nG * ldh;
  double zz = 0.0;
  for (int a = tid; a < nc; a += WG) zz += zc[a] * zc[a];
  zz = wg_sum(zz, red);
  const double zinv = 1.0 / sqrt(zz);
  for (int a = tid; a < nc; a += WG) zc[a] *= zinv;
  __syncthreads();
  // Y' = (I - z z^T) Y  (the projection realises the zero-mean constraint)
  wg_project_out(nc, zc, nG, H, ldh);
  // (6) S = S_A + Y'^T Y'
  wg_gemm<true, false, true>(nG, nG, nc, 1.0, H, ldh, H, ldh, 1.0, S, nG, lds);
  wg_symmetrize_lower(nG, S, nG);
  // (7) X = V'^T V' with V' = (I - z z^T) V, V = L_P^{-1}: as |z| = 1,
  // X = V^T V - w w^T with w = V^T z, and V is lower triangular, so the
  // lower tile (i0, j0) sums over k >= i0 only.  w goes into the first column
  // of P, whose factor is not read again.
  wg_set_identity(nc, V, nc);
  wg_trsm_lower(nc, nc, P, nc, V, nc, lds, true);
  {
    const int lane = tid & 63, wv = tid >> 6;
    for (int c = wv; c < nc; c += WG / 64) {
      double d = 0.0;
      for (int k = c + lane; k < nc; k += 64) d = fma(V[k + (size_t)c * nc], zc[k], d);
      for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
      if (lane == 0) P[c] = d;
    }
    __syncthreads();
  }
  for (int i0 = 0; i0 < nc; i0 += TILE)
    for (int j0 = 0; j0 <= i0; j0 += TILE)
      wg_gemm_tile<true, false, true>(i0, j0, nc, nc, nc - i0, 1.0, V + i0, nc, V + i0, nc, 0.0, X, nc, lds,
                                      nullptr, P);
  __syncthreads();
  wg_symmetrize_lower(nc, X, nc);
}

// Steps 5-7 of k_local_setup for the large subdomains, over many workgroups.
// Items are (subdomain, first column or tile row, kind, tile column):
//   k_ls_solve   kind 0: columns [c0, c0 + LS_COLS) of Y = L_P^{-1} [H c];
//                kind 1: columns [c0, c0 + LS_COLS) of V = L_P^{-1} (identity
//                right-hand side: the rows above c0 stay zero);
//   k_ls_project the same column blocks, Y' = (I - z z^T) Y (columns < nG),
//                z = c / |c| from the last column of Y; or w = V^T z (kind 1);
//   k_ls_gemm    lower 64 x 64 tiles of S += Y'^T Y' (kind 0) and of
//                X = V'^T V' = V^T V - w w^T (kind 1, V' = (I - z z^T) V and
//                |z| = 1): V is lower triangular, so tile (i0, j0 <= i0)
//                sums over k >= i0 only;
//   k_ls_sym     columns [c0, c0 + 64) of S (kind 0) or X (kind 1) mirrored.
// Right-looking blocked Cholesky of P~ for the large subdomains, one step per
// super-block [k0, k1 = k0 + KB) (all large subdomains at once; `big` lists
// them): k_pchol_diag factors the diagonal block, k_pchol_panel the rows
// below it in blocks of 64 (wg_potrf_rows), k_pchol_update the lower 64 x 64
// tiles of the trailing matrix.  These are the operations wg_potrf applies
// per super-block (panel solves and the super-block's own updates, then its
// delayed trailing update), so every entry gets the same values.  Item
// offsets per large subdomain: off[b] .. off[b + 1] (prefix sums).
__device__ __forceinline__ int find_item(const int *__restrict__ off, int nb, int x) {
  int lo = 0, hi = nb;   // largest b with off[b] <= x
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256, 2) void k_pchol_diag(DevGeom g, SetupWs ws, const int *__restrict__ big, int k0,
                                                       int *err) {
  __shared__ double lds[LDS_DOUBLES];
  const int i = big[blockIdx.x];
  const int nc = g.nc[i];
  if (nc <= k0) return;
  double *P = ws.base + ws.P[i];
  const int nb = min(KB, nc - k0);
  if (wg_potrf(nb, P + k0 + (size_t)k0 * nc, nc, lds)) {
    if (threadIdx.x == 0) atomicOr(err, 2);
  }
}

__global__ __launch_bounds__(256, 2) void k_pchol_panel(DevGeom g, SetupWs ws, const int *__restrict__ big, int nbig,
                                                        const int *__restrict__ off, int k0) {
  __shared__ double lds[LDS_DOUBLES];
  const int b = find_item(off, nbig, blockIdx.x);
  const int i = big[b];
  const int nc = g.nc[i], k1 = k0 + KB;
  const int ra = k1 + 64 * (blockIdx.x - off[b]), rb = min(ra + 64, nc);
  wg_potrf_rows(KB, ws.base + ws.P[i] + k0 + (size_t)k0 * nc, nc, lds, nullptr, ra - k0, rb - k0);
}

__global__ __launch_bounds__(256) void k_pchol_update(DevGeom g, SetupWs ws, const int *__restrict__ big, int nbig,
                                                      const int *__restrict__ off, int k0) {
  __shared__ double lds[2 * KT * TILE];
  const int b = find_item(off, nbig, blockIdx.x);
  const int i = big[b];
  const int nc = g.nc[i], k1 = k0 + KB, M = nc - k1;
  // lower tile t -> (ti, tj), tj <= ti, t = ti (ti + 1) / 2 + tj
  const int t = blockIdx.x - off[b];
  int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  double *P = ws.base + ws.P[i];
  const double *X = P + k1 + (size_t)k0 * nc;
  wg_gemm_tile<false, true, true>(64 * ti, 64 * tj, M, M, KB, -1.0, X, nc, X, nc, 1.0, P + k1 + (size_t)k1 * nc, nc,
                                  lds, nullptr);
}

constexpr int LS_COLS = 64;   // columns per item of k_ls_solve / k_ls_project

__global__ __launch_bounds__(256, 2) void k_ls_solve(DevGeom g, SetupWs ws, const int4 *__restrict__ items) {
  __shared__ double lds[LDS_DOUBLES];
  const int4 it = items[blockIdx.x];
  const int i = it.x, c0 = it.y, kind = it.z;
  const int nc = g.nc[i], nG = g.nG[i];
  const double *P = ws.base + ws.P[i];
  if (kind == 0) {
    double *H = ws.base + ws.H[i];
    wg_trsm_lower(nc, min(LS_COLS, nG + 1 - c0), P, nc, H + (size_t)c0 * nc, nc, lds);
  } else {
    double *V = ws.base + ws.V[i];
    const int ncol = min(LS_COLS, nc - c0);
    for (int e = threadIdx.x; e < nc * ncol; e += WG) {
      const int r = e % nc, c = c0 + e / nc;
      V[r + (size_t)c * nc] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    wg_trsm_lower(nc - c0, ncol, P + c0 + (size_t)c0 * nc, nc, V + c0 + (size_t)c0 * nc, nc, lds, true);
  }
}

// dynamic LDS: nc doubles (z); w at woff[i] in wbuf
__global__ __launch_bounds__(256) void k_ls_project(DevGeom g, SetupWs ws, const int4 *__restrict__ items,
                                                    const int64_t *__restrict__ woff, double *wbuf) {
  extern __shared__ double zl[];
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const int i = it.x, c0 = it.y, kind = it.z;
  const int nc = g.nc[i], nG = g.nG[i];
  double *H = ws.base + ws.H[i];
  const double *zc = H + (size_t)nG * nc;
  double zz = 0.0;
  for (int a = threadIdx.x; a < nc; a += WG) zz += zc[a] * zc[a];
  zz = wg_sum(zz, red);
  const double zinv = 1.0 / sqrt(zz);
  for (int a = threadIdx.x; a < nc; a += WG) zl[a] = zc[a] * zinv;
  __syncthreads();
  if (kind == 0) {
    if (c0 < nG) wg_project_out(nc, zl, min(LS_COLS, nG - c0), H + (size_t)c0 * nc, nc);
  } else {
    // w[c] = sum over k >= c of V(k, c) z[k], a wave per column
    const double *V = ws.base + ws.V[i];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = c0 + wv; c < min(c0 + LS_COLS, nc); c += WG / 64) {
      double d = 0.0;
      for (int k = c + lane; k < nc; k += 64) d = fma(V[k + (size_t)c * nc], zl[k], d);
      for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
      if (lane == 0) wbuf[woff[i] + c] = d;
    }
  }
}

__global__ __launch_bounds__(256) void k_ls_gemm(DevGeom g, SetupWs ws, const int4 *__restrict__ items,
                                                 const int64_t *__restrict__ woff, const double *__restrict__ wbuf) {
  __shared__ double lds[2 * KT * TILE];
  const int4 it = items[blockIdx.x];
  const int i = it.x, i0 = it.y, kind = it.z, j0 = it.w;
  const int nc = g.nc[i], nG = g.nG[i];
  if (kind == 0) {
    const double *H = ws.base + ws.H[i];
    wg_gemm_tile<true, false, true>(i0, j0, nG, nG, nc, 1.0, H, nc, H, nc, 1.0, ws.base + ws.S[i], nG, lds, nullptr);
  } else {
    // rows k >= i0 of V: V + i0 shifts the summation index
    const double *V = ws.base + ws.V[i] + i0;
    wg_gemm_tile<true, false, true>(i0, j0, nc, nc, nc - i0, 1.0, V, nc, V, nc, 0.0, ws.Xmat + ws.X[i], nc, lds,
                                    nullptr, wbuf + woff[i]);
  }
}

__global__ __launch_bounds__(256) void k_ls_sym(DevGeom g, SetupWs ws, const int4 *__restrict__ items) {
  const int4 it = items[blockIdx.x];
  const int i = it.x, c0 = it.y, kind = it.z;
  const int n = kind == 0 ? g.nG[i] : g.nc[i];
  double *A = kind == 0 ? ws.base + ws.S[i] : ws.Xmat + ws.X[i];
  const int c1 = min(c0 + 64, n);
  for (int e = threadIdx.x; e < n * (c1 - c0); e += WG) {
    const int r = e % n, c = c0 + e / n;
    if (c > r) A[r + (size_t)c * n] = A[c + (size_t)r * n];
  }
}

// Cholesky of S^i and W_S = L_S^{-1}; packed copy of S^i for the CG operator.
__global__ __launch_bounds__(256, 2) void k_schur_factor(DevGeom g, SetupWs ws, int *err) {
  __shared__ double lds[LDS_DOUBLES];
  const int i = blockIdx.x;
  const int nG = g.nG[i];
  double *S = ws.base + ws.S[i];
  double *L = ws.base + ws.L[i];
  double *W = ws.base + ws.W[i];
  for (int e = threadIdx.x; e < nG * nG; e += WG) L[e] = S[e];
  double *pk = ws.Spk + ws.pk[i];
  for (int64_t e = threadIdx.x; e < gp_size(nG); e += WG) pk[e] = 0.0;
  __syncthreads();
  for (int e = threadIdx.x; e < nG * nG; e += WG) {
    const int r = e % nG, c = e / nG;
    if (r >= c) pk[gp_index(nG, r, c)] = S[e];
  }
  __syncthreads();
  if (wg_potrf(nG, L, nG, lds)) {
    if (threadIdx.x == 0) atomicOr(err, 4);
  }
  wg_zero_upper(nG, L, nG);
  wg_set_identity(nG, W, nG);
  wg_trsm_lower(nG, nG, L, nG, W, nG, lds, true);
}

// ---------------------------------------------------------------------------
// face eigenproblems
// ---------------------------------------------------------------------------
// For the face F shared by subdomains i and j the pair problem of eq.
// eigenvalue-problem-local-matrix has, besides zeros, the eigenvalues of the
// reduced problem on the jump d = w^i_F - w^j_F restricted to 1^T d = 0:
//     1/4 Z^T (S^i_FF + S^j_FF) Z y = lambda Z^T ((S^i)^{-1}_FF + (S^j)^{-1}_FF)^{-1} Z y,
// since (I - E^{ij}) only sees the jump on F and minimising the pair energy for
// a fixed jump yields the parallel sum of the two face Schur complements.  Z is
// an orthonormal basis of 1^perp (a Householder reflector).  The row of eq.
// constraints for eigenvector y is, up to scale and within span{1}, X_F Z y.
//
// The work is split in three launches that pass everything through the face's
// workspace: k_face_reduce forms the reduced m x m matrix C = L^{-1} Xr L^{-T}
// (into U; L, the Cholesky factor of Yr, stays in T1), k_face_eig finds its
// eigenvalues (onto the diagonal of U) and the eigenvectors of those above tau
// (into T2), and k_face_rows selects them and builds the rows.
__global__ __launch_bounds__(256, 2) void k_face_reduce(DevGeom g, SetupWs ws, double *fbase,
                                                     const int64_t *foff, int all_constrained,
                                                     double *eig_out, const int64_t *eig_off, int *kout,
                                                     double *omega_out, double *rows_out,
                                                     const int64_t *rows_off, int *err) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ double red[8];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int i = g.f_minus[f], j = g.f_plus[f], n = g.f_n[f];
  const int oi = g.f_loffm[f], oj = g.f_loffp[f];
  const int ni = g.nG[i], nj = g.nG[j];
  const int m = n - 1;
  double *w = fbase + foff[f];
  double *XF = w, *XH = w + n * n, *YF = w + 2 * n * n, *T1 = w + 3 * n * n, *T2 = w + 4 * n * n,
         *U = w + 5 * n * n, *v = w + 6 * n * n;
  double *rows = rows_out + rows_off[f];
  double *eig = eig_out + eig_off[f];
  const double beta = 2.0 / ((1.0 + sqrt((double)n)) * (1.0 + sqrt((double)n)) + (double)(n - 1));
  for (int a = tid; a < n; a += WG) v[a] = (a == 0) ? 1.0 + sqrt((double)n) : 1.0;
  __syncthreads();
  if (m == 0) {
    if (tid == 0) { kout[f] = 0; omega_out[f] = 0.0; }
    return;
  }
  if (all_constrained) {
    // every interface dof constrained: rows = the reflector basis of 1^perp
    for (int e = tid; e < m * n; e += WG) {
      const int l = e / n, a = e % n;
      rows[e] = ((a == l + 1) ? 1.0 : 0.0) - beta * v[a] * v[l + 1];
    }
    for (int a = tid; a < m; a += WG) eig[a] = 0.0;
    if (tid == 0) { kout[f] = m; omega_out[f] = 0.0; }
    return;
  }
  const double *Si = ws.base + ws.S[i], *Sj = ws.base + ws.S[j];
  const double *Wi = ws.base + ws.W[i], *Wj = ws.base + ws.W[j];
  // X_F = S^i_FF + S^j_FF
  for (int e = tid; e < n * n; e += WG) {
    const int a = e % n, b = e / n;
    XF[e] = Si[(oi + a) + (size_t)(oi + b) * ni] + Sj[(oj + a) + (size_t)(oj + b) * nj];
  }
  // (S^{-1})_FF = W[:,F]^T W[:,F], summed over the two sides
  wg_gemm<true, false>(n, n, ni, 1.0, Wi + (size_t)oi * ni, ni, Wi + (size_t)oi * ni, ni, 0.0, T1, n, lds);
  wg_gemm<true, false>(n, n, nj, 1.0, Wj + (size_t)oj * nj, nj, Wj + (size_t)oj * nj, nj, 1.0, T1, n, lds);
  // Y_F = T1^{-1} via Cholesky
  if (wg_potrf(n, T1, n, lds)) {
    if (tid == 0) atomicOr(err, 8);
  }
  wg_zero_upper(n, T1, n);
  wg_set_identity(n, T2, n);
  wg_trsm_lower(n, n, T1, n, T2, n, lds, true);
  wg_gemm<true, false>(n, n, n, 1.0, T2, n, T2, n, 0.0, YF, n, lds);
  // two-sided reflector on copies: M <- H M H
  for (int e = tid; e < n * n; e += WG) XH[e] = XF[e];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    double *M = pass ? YF : XH;
    // p = beta M v (into U[:,0]), Kc = beta v.p / 2, wv = p - Kc v (into U[:,1])
    for (int r = tid; r < n; r += WG) {
      double s = 0.0;
      for (int c = 0; c < n; ++c) s += M[r + (size_t)c * n] * v[c];
      U[r] = beta * s;
    }
    __syncthreads();
    double vp = 0.0;
    for (int r = tid; r < n; r += WG) vp += v[r] * U[r];
    vp = wg_sum(vp, red);
    const double Kc = beta * vp / 2.0;
    for (int r = tid; r < n; r += WG) U[n + r] = U[r] - Kc * v[r];
    __syncthreads();
    for (int e = tid; e < n * n; e += WG) {
      const int r = e % n, c = e / n;
      M[e] -= v[r] * U[n + c] + U[n + r] * v[c];
    }
    __syncthreads();
  }
  // reduced m x m problems: T1 = Yr, T2 = Xr / 4
  for (int e = tid; e < m * m; e += WG) {
    const int r = e % m, c = e / m;
    T1[e] = YF[(r + 1) + (size_t)(c + 1) * n];
    T2[e] = 0.25 * XH[(r + 1) + (size_t)(c + 1) * n];
  }
  __syncthreads();
  if (wg_potrf(m, T1, m, lds)) {
    if (tid == 0) atomicOr(err, 16);
  }
  wg_zero_upper(m, T1, m);
  wg_trsm_lower(m, m, T1, m, T2, m, lds);           // B1 = L^{-1} Xr
  for (int e = tid; e < m * m; e += WG) {
    const int r = e % m, c = e / m;
    U[e] = T2[c + (size_t)r * m];                    // U = B1^T
  }
  __syncthreads();
  wg_trsm_lower(m, m, T1, m, U, m, lds);             // C = L^{-1} Xr L^{-T}
  for (int e = tid; e < m * m; e += WG) {
    const int r = e % m, c = e / m;
    if (r > c) {
      const double s = 0.5 * (U[e] + U[c + (size_t)r * m]);
      U[e] = s;
      U[c + (size_t)r * m] = s;
    }
  }
  __syncthreads();
}

// Multiscale constraint of a face (Section 6, in place of the eigenproblem):
// the face fluxes of the Darcy problem on the two neighbours with source w_i
// in Omega^i, the matching sink -w_j in Omega^j and no flow through their
// other faces; w_s is uniform, or f / int f in a subdomain holding a well.
// With those other fluxes zero the problem reduces to the face: the flux u
// minimises 1/2 u^T (S^i_FF + S^j_FF) u + u^T g at unit net flux, g the face
// load that the non-uniform part of the sources puts on the two local
// Dirichlet problems (the uniform part lies in the constants the local
// pressure operators leave out).  hs holds -H^{sT} X^s w_s per local interface
// dof (null: no wells), so g = hs^j_F - hs^i_F and u = mu y + z with
// y = (S^i_FF + S^j_FF)^{-1} 1, z = (S^i_FF + S^j_FF)^{-1} (hs^i_F - hs^j_F),
// mu fixing 1^T u = 1.  The row is u projected off the zero-net-flux row and
// normalised; a uniform u adds none.
__global__ __launch_bounds__(256, 2) void k_face_ms(DevGeom g, SetupWs ws, const double *__restrict__ hs,
                                                 double *fbase, const int64_t *foff,
                                                 double *eig_out, const int64_t *eig_off, int *kout,
                                                 double *omega_out, double *rows_out, const int64_t *rows_off,
                                                 int *err) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ double red[8];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int i = g.f_minus[f], j = g.f_plus[f], n = g.f_n[f];
  const int oi = g.f_loffm[f], oj = g.f_loffp[f];
  const int ni = g.nG[i], nj = g.nG[j];
  const int m = n - 1;
  double *w = fbase + foff[f];
  double *XF = w, *y = w + n * n, *z = y + n;   // y and z: two right-hand sides, leading dimension n
  double *eig = eig_out + eig_off[f];
  for (int a = tid; a < m; a += WG) eig[a] = 0.0;
  if (m == 0) {
    if (tid == 0) { kout[f] = 0; omega_out[f] = 0.0; }
    return;
  }
  const double *Si = ws.base + ws.S[i], *Sj = ws.base + ws.S[j];
  for (int e = tid; e < n * n; e += WG) {
    const int a = e % n, b = e / n;
    XF[e] = Si[(oi + a) + (size_t)(oi + b) * ni] + Sj[(oj + a) + (size_t)(oj + b) * nj];
  }
  const int64_t hi = g.g_off[i] + oi, hj = g.g_off[j] + oj;
  for (int a = tid; a < n; a += WG) {
    y[a] = 1.0;
    z[a] = hs ? hs[hi + a] - hs[hj + a] : 0.0;
  }
  __syncthreads();
  if (wg_potrf(n, XF, n, lds)) {
    if (tid == 0) atomicOr(err, 8);
  }
  wg_trsm_lower(n, 2, XF, n, y, n, lds);
  wg_trsm_lower_t(n, 2, XF, n, y, n, lds);
  double sy = 0.0, sz = 0.0;
  for (int a = tid; a < n; a += WG) {
    sy += y[a];
    sz += z[a];
  }
  sy = wg_sum(sy, red);
  sz = wg_sum(sz, red);
  const double mu = (1.0 - sz) / sy;
  double su = 0.0, suu = 0.0;
  for (int a = tid; a < n; a += WG) {
    const double u = fma(mu, y[a], z[a]);
    su += u;
    suu += u * u;
  }
  su = wg_sum(su, red);
  suu = wg_sum(suu, red);
  const double mean = su / n;
  double rr = 0.0;
  for (int a = tid; a < n; a += WG) {
    const double d = fma(mu, y[a], z[a]) - mean;
    rr += d * d;
  }
  const double nrm = sqrt(wg_sum(rr, red));
  const int k = (nrm > 1e-12 * sqrt(suu)) ? 1 : 0;
  if (k) {
    double *rows = rows_out + rows_off[f];
    for (int a = tid; a < n; a += WG) rows[a] = (fma(mu, y[a], z[a]) - mean) / nrm;
  }
  if (tid == 0) {
    kout[f] = k;
    omega_out[f] = 0.0;
  }
}

// Source distribution w_s of the multiscale constraints (Section 6), cell
// integrated: f / (the sum of f over Omega^s) in a subdomain holding a well
// (a source not zero there), zero elsewhere, where w_s is uniform and its load
// vanishes.  A subdomain whose wells cancel keeps the uniform w_s.
__global__ __launch_bounds__(256) void k_ms_weight(DevGeom g, const double *__restrict__ src,
                                                   double *__restrict__ wsrc) {
  __shared__ double red[8];
  const int i = blockIdx.x;
  const int nc = g.nc[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double s = 0.0, a = 0.0;
  for (int c = threadIdx.x; c < nc; c += WG) {
    const double v = src[lcg[c]];
    s += v;
    a += fabs(v);
  }
  s = wg_sum(s, red);
  a = wg_sum(a, red);
  const bool well = a > 0.0 && fabs(s) > 1e-12 * a;
  for (int c = threadIdx.x; c < nc; c += WG) wsrc[lcg[c]] = well ? src[lcg[c]] / s : 0.0;
}

// Symmetric eigenproblem of a face's reduced matrix C (m x m, m <= 255, in U
// with leading dimension m, full storage): Householder reduction to a
// tridiagonal T = Q^T C Q (reflector k: v stored below the diagonal of column
// k, beta_k in LDS), every eigenvalue of T by bisection on its Sturm sequence
// (thread t finds the t-th smallest), the eigenvectors of those above tau by
// inverse iteration on T (three steps from distinct starting vectors, a
// partially pivoted tridiagonal LU each), orthogonalised within clusters of
// close eigenvalues, and carried back through the reflectors.  Out: the
// eigenvalues on the diagonal of U, the eigenvectors of those above tau in
// the matching columns of T2 (leading dimension m); XH and YF of the face
// workspace are scratch.  One workgroup per face.
constexpr int EIG_MAX = 256;

// Sturm count: eigenvalues of the tridiagonal (d, e) below x.
__device__ __forceinline__ int sturm_below(int m, const double *d, const double *e, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < m; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

__global__ __launch_bounds__(256) void k_face_eig(DevGeom g, double *fbase, const int64_t *foff, double tau) {
  __shared__ double d[EIG_MAX], e[EIG_MAX], bet[EIG_MAX], lam[EIG_MAX], vs[EIG_MAX], ws[EIG_MAX];
  __shared__ double red[8];
  const int f = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = g.f_n[f], m = n - 1;
  if (m <= 0) return;
  double *w = fbase + foff[f];
  double *XH = w + (size_t)n * n, *T2 = w + 4 * (size_t)n * n, *U = w + 5 * (size_t)n * n;
  double *A = U;
  // the two triangles of C, formed separately, are averaged
  for (int64_t q = tid; q < (int64_t)m * m; q += 256) {
    const int i = (int)(q % m), j = (int)(q / m);
    if (i > j) {
      const double a = 0.5 * (A[i + (size_t)j * m] + A[j + (size_t)i * m]);
      A[i + (size_t)j * m] = a;
      A[j + (size_t)i * m] = a;
    }
  }
  __syncthreads();
  // --- Householder reduction (lower): column k below the diagonal -> beta, v
  for (int k = 0; k + 2 < m; ++k) {
    const int L = m - k - 1;
    double *col = A + (size_t)k * m + (k + 1);
    double s2 = 0.0;
    for (int i = tid; i < L; i += 256) {
      const double x = col[i];
      vs[i] = x;
      if (i > 0) s2 += x * x;
    }
    s2 = wg_sum(s2, red);   // (barrier inside: vs visible)
    const double x0 = col[0];   // (vs[0] becomes v0 below, in thread 0)
    double beta = 0.0, alpha = x0;
    if (s2 > 0.0) {
      const double mu = sqrt(x0 * x0 + s2);
      alpha = x0 <= 0.0 ? mu : -mu;
      const double v0 = x0 - alpha;
      beta = 2.0 / (v0 * v0 + s2);
      if (tid == 0) vs[0] = v0;
    }
    if (tid == 0) {
      d[k] = A[(size_t)k * m + k];
      e[k] = alpha;
      bet[k] = beta;
    }
    __syncthreads();
    if (beta == 0.0) continue;
    for (int i = tid; i < L; i += 256) col[i] = vs[i];   // the reflector, for the back transformation
    // p = beta A22 v (A22 symmetric: column i of A22 against v), a wave per column
    double *A22 = A + (size_t)(k + 1) * m + (k + 1);
    for (int i = wv; i < L; i += 4) {
      const double *ci = A22 + (size_t)i * m;
      double a = 0.0;
      for (int j = lane; j < L; j += 64) a = fma(ci[j], vs[j], a);
      for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
      if (lane == 0) ws[i] = beta * a;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < L; i += 256) pv += ws[i] * vs[i];
    const double K = 0.5 * beta * wg_sum(pv, red);
    for (int i = tid; i < L; i += 256) ws[i] -= K * vs[i];
    __syncthreads();
    // A22 -= v w^T + w v^T
    for (int64_t q = tid; q < (int64_t)L * L; q += 256) {
      const int i = (int)(q % L), j = (int)(q / L);
      A22[i + (size_t)j * m] -= vs[i] * ws[j] + ws[i] * vs[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int k0 = m >= 2 ? m - 2 : 0;
    if (m >= 2) {
      d[k0] = A[(size_t)k0 * m + k0];
      e[k0] = A[(size_t)k0 * m + k0 + 1];
      bet[k0] = 0.0;
    }
    d[m - 1] = A[(size_t)(m - 1) * m + (m - 1)];
    e[m - 1] = 0.0;
  }
  __syncthreads();
  // --- eigenvalues: bisection, thread t the t-th smallest (ascending)
  double lo = 0.0, hi = 0.0, tnorm = 0.0;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo = i == 0 ? d[i] - r : fmin(lo, d[i] - r);
    hi = i == 0 ? d[i] + r : fmax(hi, d[i] + r);
  }
  tnorm = fmax(fabs(lo), fabs(hi));
  const double eps = 2.220446049250313e-16;
  // smallest pivot allowed in the Sturm counts: the safe minimum times max(1, e_i^2)
  double emax2 = 1.0;
  for (int i = 0; i + 1 < m; ++i) emax2 = fmax(emax2, e[i] * e[i]);
  const double pivmin = 2.2250738585072014e-308 * emax2;
  for (int t = tid; t < m; t += 256) {
    double a = lo - eps * tnorm - pivmin, b = hi + eps * tnorm + pivmin;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b || (b - a) <= 2.0 * eps * fmax(fabs(a), fabs(b)) + pivmin) break;
      if (sturm_below(m, d, e, mid, pivmin) > t) b = mid;
      else a = mid;
    }
    lam[t] = 0.5 * (a + b);
  }
  __syncthreads();
  // --- eigenvectors of the eigenvalues above tau: lam[t0 .. m)
  int t0 = m;
  for (int t = 0; t < m; ++t)
    if (lam[t] > tau) { t0 = t; break; }
  const int k = m - t0;
  if (k > 0) {
    // per vector: the upper factor (u0, u1, u2) of the pivoted LU, 3m doubles of scratch
    const int per = (int)std::min<int64_t>(k, (2 * (int64_t)n * n) / (3 * (int64_t)m));
    for (int b0 = 0; b0 < k; b0 += per) {
      for (int jj = tid; jj < per && b0 + jj < k; jj += 256) {
        const int t = t0 + b0 + jj;
        double *y = T2 + (size_t)t * m;
        double *u0 = XH + (size_t)jj * 3 * m, *u1 = u0 + m, *u2 = u1 + m;
        // distinct starting vectors (their components in a cluster differ)
        for (int i = 0; i < m; ++i) y[i] = 1.0 + 0.5 * sin(0.7 * (double)(i + 1) * (double)(t + 1));
        const double shift = lam[t] + eps * tnorm;
        for (int step = 0; step < 3; ++step) {
          // LU of T - shift I with row interchanges, applied to y on the fly
          double a = d[0] - shift, bb = m > 1 ? e[0] : 0.0, cc = 0.0;
          double rhs = y[0];
          for (int i = 0; i + 1 < m; ++i) {
            // rows i (a, bb, cc) and i + 1 (e[i], d[i+1] - shift, e[i+1])
            const double l0 = e[i], l1 = d[i + 1] - shift, l2 = i + 2 < m ? e[i + 1] : 0.0;
            double r1 = y[i + 1];
            if (fabs(l0) > fabs(a)) {
              // swap rows i and i + 1
              const double mlt = a / l0;
              u0[i] = l0;
              u1[i] = l1;
              u2[i] = l2;
              const double nb = bb - mlt * l1, nc = cc - mlt * l2;
              const double ry = rhs - mlt * r1;
              y[i] = r1;
              a = nb;
              bb = nc;
              cc = 0.0;
              rhs = ry;
            } else {
              const double mlt = a != 0.0 ? l0 / a : 0.0;
              u0[i] = a;
              u1[i] = bb;
              u2[i] = cc;
              y[i] = rhs;
              a = l1 - mlt * bb;
              bb = l2 - mlt * cc;
              cc = 0.0;
              rhs = r1 - mlt * rhs;
            }
          }
          u0[m - 1] = a;
          y[m - 1] = rhs;
          // back substitution with tiny pivots replaced
          const double tiny = eps * tnorm + pivmin;
          double s = 0.0;
          for (int i = m - 1; i >= 0; --i) {
            double piv = u0[i];
            if (fabs(piv) < tiny) piv = piv < 0.0 ? -tiny : tiny;
            double v = y[i];
            if (i + 1 < m) v -= u1[i] * y[i + 1];
            if (i + 2 < m) v -= u2[i] * y[i + 2];
            v /= piv;
            y[i] = v;
            s = fmax(s, fabs(v));
          }
          const double sc = s > 0.0 ? 1.0 / s : 1.0;
          for (int i = 0; i < m; ++i) y[i] *= sc;
        }
      }
      __syncthreads();
    }
    // orthonormalise within clusters of close eigenvalues (twice), normalise the rest
    const double gap = 1e-3 * tnorm;
    int c0 = t0;
    for (int t = t0; t < m; ++t) {
      if (t > t0 && lam[t] - lam[t - 1] > gap) c0 = t;
      double *yt = T2 + (size_t)t * m;
      for (int pass = 0; pass < 2; ++pass)
        for (int q = c0; q < t; ++q) {
          const double *yq = T2 + (size_t)q * m;
          double dot = 0.0;
          for (int i = tid; i < m; i += 256) dot += yq[i] * yt[i];
          dot = wg_sum(dot, red);
          for (int i = tid; i < m; i += 256) yt[i] -= dot * yq[i];
          __syncthreads();
        }
      double nr = 0.0;
      for (int i = tid; i < m; i += 256) nr += yt[i] * yt[i];
      nr = sqrt(wg_sum(nr, red));
      for (int i = tid; i < m; i += 256) yt[i] /= nr;
      __syncthreads();
    }
    // back transformation y <- H_0 ... H_{m-3} y, a wave per vector
    for (int t = t0 + wv; t < m; t += 4) {
      double *y = T2 + (size_t)t * m;
      for (int r = m - 3; r >= 0; --r) {
        const double br = bet[r];
        if (br == 0.0) continue;
        const double *v = A + (size_t)r * m + (r + 1);
        const int L = m - r - 1;
        double a = 0.0;
        for (int i = lane; i < L; i += 64) a = fma(v[i], y[r + 1 + i], a);
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        a *= br;
        for (int i = lane; i < L; i += 64) y[r + 1 + i] -= a * v[i];
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < m; t += 256) U[(size_t)t * m + t] = lam[t];
}

__global__ __launch_bounds__(256) void k_face_rows(DevGeom g, double *fbase, const int64_t *foff, double tau,
                                                   double *eig_out, const int64_t *eig_off, int *kout,
                                                   double *omega_out, double *rows_out,
                                                   const int64_t *rows_off) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ int perm[256];
  __shared__ double red[8];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int n = g.f_n[f];
  const int m = n - 1;
  if (m <= 0) return;
  double *w = fbase + foff[f];
  double *XF = w, *XH = w + n * n, *YF = w + 2 * n * n, *T1 = w + 3 * n * n, *T2 = w + 4 * n * n,
         *U = w + 5 * n * n, *v = w + 6 * n * n;
  double *rows = rows_out + rows_off[f];
  double *eig = eig_out + eig_off[f];
  const double beta = 2.0 / ((1.0 + sqrt((double)n)) * (1.0 + sqrt((double)n)) + (double)(n - 1));
  // sort eigenvalues descending (rank by count, ties by index)
  for (int t = tid; t < m; t += WG) {
    const double lt = U[t + (size_t)t * m];
    int rank = 0;
    for (int s = 0; s < m; ++s) {
      const double ls = U[s + (size_t)s * m];
      if (ls > lt || (ls == lt && s < t)) ++rank;
    }
    eig[rank] = lt;
    perm[rank] = t;
  }
  __syncthreads();
  int k = 0;
  if (tau > 0.0 && isfinite(tau)) {
    for (int t = 0; t < m; ++t)
      if (eig[t] > tau) ++k;
  }
  if (tid == 0) {
    kout[f] = k;
    omega_out[f] = (k < m) ? eig[k] : 0.0;
  }
  if (k == 0) return;
  // eigenvectors of the generalized problem: y = L^{-T} u  (gathered into YF, ld m)
  for (int e = tid; e < m * k; e += WG) {
    const int r = e % m, l = e / m;
    YF[r + (size_t)l * m] = T2[r + (size_t)perm[l] * m];
  }
  __syncthreads();
  wg_trsm_lower_t(m, k, T1, m, YF, m, lds);
  // delta = H [0; y]  (into XH, ld n)
  for (int l = 0; l < k; ++l) {
    double s = 0.0;
    for (int r = tid; r < m; r += WG) s += v[r + 1] * YF[r + (size_t)l * m];
    s = wg_sum(s, red);
    for (int a = tid; a < n; a += WG)
      XH[a + (size_t)l * n] = ((a > 0) ? YF[(a - 1) + (size_t)l * m] : 0.0) - beta * v[a] * s;
    __syncthreads();
  }
  // rows = X_F delta, projected onto 1^perp and orthonormalised (two Gram-Schmidt passes)
  wg_gemm<false, false>(n, k, n, 1.0, XF, n, XH, n, 0.0, T2, n, lds);
  for (int l = 0; l < k; ++l) {
    double *r = T2 + (size_t)l * n;
    double mean = 0.0;
    for (int a = tid; a < n; a += WG) mean += r[a];
    mean = wg_sum(mean, red) / n;
    for (int a = tid; a < n; a += WG) r[a] -= mean;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < l; ++q) {
        const double *rq = T2 + (size_t)q * n;
        double dot = 0.0;
        for (int a = tid; a < n; a += WG) dot += rq[a] * r[a];
        dot = wg_sum(dot, red);
        for (int a = tid; a < n; a += WG) r[a] -= dot * rq[a];
        __syncthreads();
      }
    }
    double nrm = 0.0;
    for (int a = tid; a < n; a += WG) nrm += r[a] * r[a];
    nrm = sqrt(wg_sum(nrm, red));
    for (int a = tid; a < n; a += WG) {
      r[a] /= nrm;
      rows[(size_t)l * n + a] = r[a];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// local coarse space: Psi^i, A_c^i, T^i
// ---------------------------------------------------------------------------
// With S = L L^T, W = L^{-1} and the constraint rows C of the subdomain:
// V = W C^T = Q R,  Psi = S^{-1} C^T (C S^{-1} C^T)^{-1} = W^T Q R^{-T},
// A_c^i = (C S^{-1} C^T)^{-1} = R^{-1} R^{-T},
// T = S^{-1} - Psi C S^{-1} = W'^T W' with W' = (I - Q Q^T) W, formed as
// W^T W - (Q^T W)^T (Q^T W).
struct CoarseLocalWs {
  double *base;
  const int64_t *off;     // per subdomain workspace offset
  double *Ac;             // A_c^i blocks
  const int64_t *ac_off;
  double *psi64;
  float *psi32;
  const int64_t *psi_off;
  double *t64;
  float *t32;
  const int64_t *pk;      // packed offsets (same as S)
};

__global__ __launch_bounds__(256) void k_coarse_local(DevGeom g, SetupWs ws, DevCoarse cs,
                                                      CoarseLocalWs cw, int *err) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ double red[8];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int nG = g.nG[i];
  const int c0 = cs.sub_coff[i];
  const int nci = cs.sub_coff[i + 1] - c0;
  double *W = ws.base + ws.W[i];
  double *Tfull = ws.base + ws.L[i];
  double *base = cw.base + cw.off[i];
  double *C = base;                         // nci x nG
  double *Q = C + (size_t)nci * nG;         // nG x nci
  double *R = Q + (size_t)nG * nci;         // nci x nci
  double *U = R + (size_t)nci * nci;        // nG x nci
  double *M1 = U + (size_t)nG * nci;        // nci x nG
  double *Rinv = M1 + (size_t)nci * nG;     // nci x nci
  double *Ac = cw.Ac + cw.ac_off[i];
  double *Psi = cw.psi64 + cw.psi_off[i];

  for (int e = tid; e < nci * nG; e += WG) C[e] = 0.0;
  for (int e = tid; e < nci * nci; e += WG) R[e] = 0.0;
  __syncthreads();
  {
    int r0 = 0;
    for (int t = g.sub_face_off[i]; t < g.sub_face_off[i + 1]; ++t) {
      const int f = g.sub_faces[t];
      const int n = g.f_n[f];
      const int off = (g.f_minus[f] == i) ? g.f_loffm[f] : g.f_loffp[f];
      const int k = cs.face_k[f];
      const double *rows = cs.face_rows + cs.face_rows_off[f];
      for (int e = tid; e < (k + 1) * n; e += WG) {
        const int l = e / n, a = e % n;
        C[(r0 + l) + (size_t)(off + a) * nci] = (l == 0) ? 1.0 : rows[(size_t)(l - 1) * n + a];
      }
      r0 += k + 1;
    }
    __syncthreads();
  }
  // V = W C^T into Q
  wg_gemm<false, true>(nG, nci, nG, 1.0, W, nG, C, nci, 0.0, Q, nG, lds);
  // classical Gram-Schmidt, two passes per column
  for (int jc = 0; jc < nci; ++jc) {
    double *qj = Q + (size_t)jc * nG;
    for (int pass = 0; pass < 2; ++pass) {
      // d_k = q_k . q_j for k < j: wave w takes k = w, w + 4, ... (two at a
      // time), its lanes split the rows and a butterfly sums them
      {
        const int lane = tid & 63, wv = tid >> 6;
        constexpr int NW = WG / 64;
        for (int kk = wv; kk < jc; kk += 2 * NW) {
          const int k2 = kk + NW;
          const double *qa = Q + (size_t)kk * nG;
          const double *qb = Q + (size_t)min(k2, jc - 1) * nG;
          double sa = 0.0, sb = 0.0;
#pragma unroll 4
          for (int r = lane; r < nG; r += 64) {
            const double x = qj[r];
            sa += qa[r] * x;
            sb += qb[r] * x;
          }
          for (int o = 32; o > 0; o >>= 1) {
            sa += __shfl_xor(sa, o, 64);
            sb += __shfl_xor(sb, o, 64);
          }
          if (lane == 0) {
            lds[kk] = sa;
            if (k2 < jc) lds[k2] = sb;
          }
        }
      }
      __syncthreads();
      for (int kk = tid; kk < jc; kk += WG) R[kk + (size_t)jc * nci] += lds[kk];
      for (int r = tid; r < nG; r += WG) {
        double s = qj[r];
#pragma unroll 8
        for (int kk = 0; kk < jc; ++kk) s -= Q[r + (size_t)kk * nG] * lds[kk];
        qj[r] = s;
      }
      __syncthreads();
    }
    double nrm = 0.0;
    for (int r = tid; r < nG; r += WG) nrm += qj[r] * qj[r];
    nrm = sqrt(wg_sum(nrm, red));
    if (!(nrm > 0.0)) {
      if (tid == 0) atomicOr(err, 32);
      nrm = 1.0;
    }
    if (tid == 0) R[jc + (size_t)jc * nci] = nrm;
    for (int r = tid; r < nG; r += WG) qj[r] /= nrm;
    __syncthreads();
  }
  // U = Q R^{-T} (row-wise backward substitution)
  for (int r = tid; r < nG; r += WG) {
    for (int jj = nci - 1; jj >= 0; --jj) {
      double s = Q[r + (size_t)jj * nG];
#pragma unroll 8
      for (int l = jj + 1; l < nci; ++l) s -= U[r + (size_t)l * nG] * R[jj + (size_t)l * nci];
      U[r + (size_t)jj * nG] = s / R[jj + (size_t)jj * nci];
    }
  }
  __syncthreads();
  // Psi = W^T U  (leading dimension ld4(nG), padding rows zero)
  const int ldp = ld4(nG);
  for (int e = tid; e < ldp * nci; e += WG) Psi[e] = 0.0;
  __syncthreads();
  wg_gemm<true, false>(nG, nci, nG, 1.0, W, nG, U, nG, 0.0, Psi, ldp, lds);
  for (int e = tid; e < ldp * nci; e += WG) cw.psi32[cw.psi_off[i] + e] = (float)Psi[e];
  // R^{-1} (column-wise backward substitution), A_c^i = R^{-1} R^{-T}
  for (int c = tid; c < nci; c += WG) {
    for (int r = nci - 1; r >= 0; --r) {
      double s = (r == c) ? 1.0 : 0.0;
      if (r > c) { Rinv[r + (size_t)c * nci] = 0.0; continue; }
      for (int l = r + 1; l <= c; ++l) s -= R[r + (size_t)l * nci] * Rinv[l + (size_t)c * nci];
      Rinv[r + (size_t)c * nci] = s / R[r + (size_t)r * nci];
    }
  }
  __syncthreads();
  wg_gemm<false, true>(nci, nci, nci, 1.0, Rinv, nci, Rinv, nci, 0.0, Ac, nci, lds);
  // T = W'^T W' with W' = (I - Q Q^T) W = W^T W - M1^T M1, M1 = Q^T W (Q has
  // orthonormal columns).  W = L_S^{-1} is lower triangular, so the lower
  // tile (i0, j0) of W^T W sums over k >= i0 only.
  wg_gemm<true, false>(nci, nG, nG, 1.0, Q, nG, W, nG, 0.0, M1, nci, lds);
  for (int i0 = 0; i0 < nG; i0 += TILE)
    for (int j0 = 0; j0 <= i0; j0 += TILE)
      wg_gemm_tile<true, false, true>(i0, j0, nG, nG, nG - i0, 1.0, W + i0, nG, W + i0, nG, 0.0, Tfull, nG, lds,
                                      nullptr);
  __syncthreads();
  wg_gemm<true, false, true>(nG, nG, nci, -1.0, M1, nci, M1, nci, 1.0, Tfull, nG, lds);
  const int64_t po = cw.pk[i];
  for (int64_t e = tid; e < gp_size(nG); e += WG) {
    cw.t64[po + e] = 0.0;
    cw.t32[po + e] = 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < nG * nG; e += WG) {
    const int r = e % nG, c = e / nG;
    if (r >= c) {
      const int64_t k = po + gp_index(nG, r, c);
      const double t = Tfull[e];
      cw.t64[k] = t;
      cw.t32[k] = (float)t;
    }
  }
}

}  // namespace bddc
