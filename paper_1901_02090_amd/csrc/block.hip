// Block form of step 3 (Algorithm "BDDC method"): the CG of eqs.
// corr-reduced-1/2 for BK right-hand sides at once.  Every column keeps its
// own CG scalars and stopping test, so each column runs the iteration of a
// single solve (to rounding: the block kernels add in another order), while
// one pass over the local operators S^i and T^i, the bases Psi^i, the swept
// coarse factor and S_t^{-1} serves all BK columns.  The local operators and
// bases are applied as 16 x 16 tiles on the FP64 matrix cores (a tile against
// the block's 16 columns), the coarse sweeps by the column tasks of front.hip.
//
// Layout: every vector (interface, local, coarse, the coarse sweeps' work
// vectors) keeps the BK values of an entry together ([n][BK]).
//
// Reductions are deterministic: a block writes one partial per column, a
// consumer adds the partials of a column in a fixed order.
#include <vector>

#include "common.hpp"
#include "dense.hpp"

namespace bddc {

constexpr int BK = 16;   // right-hand sides per block (the N of a 16 x 16 x 4 MFMA)

// Device arrays of the block CG (allocated at the first block solve).
struct BlockWs {
  bool ready = false;
  int4 *task = nullptr;                      // coarse sweep tasks (k_blk_nd_fwd / k_blk_nd_bwd)
  std::vector<int> tf_off, tb_lo, tb_hi;     // forward tasks of level h, backward tasks of level h
  double *ru = nullptr, *zu = nullptr, *pu = nullptr, *xu = nullptr, *qu = nullptr, *u0 = nullptr;  // [nGamma][BK]
  double *yloc = nullptr, *wloc = nullptr;   // [sum nG][BK]
  double *pp = nullptr, *xp = nullptr;       // [N][BK]
  double *bc = nullptr, *cy = nullptr, *csol = nullptr;   // [nk][BK]
  double *S0 = nullptr, *S1 = nullptr;       // [v_off[nfr]][BK]
  double *XB = nullptr;                      // [b_off[nfr]][BK]
  double *tt = nullptr;                      // [nt][BK]
  double *cA = nullptr, *cB = nullptr;       // [sum nc][BK]: local cell loads, their X^i products
  double *part_g = nullptr, *part_r = nullptr, *part_z = nullptr;   // [PART_BLOCKS][BK]
  double *alpha_h = nullptr, *beta_h = nullptr;                     // [max_it + 2][BK]
  struct CgBlockState *st = nullptr;
  size_t psi_shm = 0, corr_shm = 0;
};

struct CgBlockState {
  double rho[BK];        // r.z of the current iteration
  double alpha[BK], beta[BK];
  double r0sq[BK], relres[BK];
  double rtol2;
  int it;                // block iterations completed
  int maxit;
  int done;              // every column has stopped
  int nupd[BK];          // x / r updates applied to each column
  int cdone[BK];         // the column has stopped
  int converged[BK], fail[BK];
};

// ---- per-column reductions ----------------------------------------------------
// Thread t of a 256-thread block holds v for column t % BK; the block's BK
// column sums go to part[blockIdx.x * BK + j].
__device__ __forceinline__ void col_partial(double v, double *part, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  if (t < BK) {
    double s = 0.0;
    for (int q = 0; q < 256 / BK; ++q) s += red[q * BK + t];
    part[(int64_t)blockIdx.x * BK + t] = s;
  }
  __syncthreads();
}

// Column totals of np partials part[p * BK + j] into tot[j] (LDS); called by
// one whole 256-thread block.
__device__ __forceinline__ void col_sums(const double *__restrict__ part, int np, double *red, double *tot) {
  const int t = threadIdx.x, j = t & (BK - 1);
  double s = 0.0;
  for (int p = t / BK; p < np; p += 256 / BK) s += part[(int64_t)p * BK + j];
  red[t] = s;
  __syncthreads();
  if (t < BK) {
    double v = 0.0;
    for (int q = 0; q < 256 / BK; ++q) v += red[q * BK + t];
    tot[t] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ bool blk_done(const CgBlockState *st) { return st && st->done; }

// ---- CG scalars (one block of 256 threads each) ----------------------------------
// Start: ||r_0||^2 per column; zero columns (padding of a partial block) stop at once.
__global__ __launch_bounds__(256) void k_blk_init(CgBlockState *st, const double *__restrict__ rpart, int np,
                                                  double rtol, int maxit) {
  __shared__ double red[256], tot[BK];
  col_sums(rpart, np, red, tot);
  const int t = threadIdx.x;
  if (t < BK) {
    const double r0 = tot[t];
    st->r0sq[t] = r0;
    st->relres[t] = r0 > 0.0 ? 1.0 : 0.0;
    st->nupd[t] = 0;
    st->alpha[t] = st->beta[t] = 0.0;
    st->fail[t] = isfinite(r0) ? 0 : 1;
    st->converged[t] = (r0 == 0.0) ? 1 : 0;
    st->cdone[t] = (r0 > 0.0 && isfinite(r0)) ? 0 : 1;
  }
  __syncthreads();
  if (t == 0) {
    st->rtol2 = rtol * rtol;
    st->it = 0;
    st->maxit = maxit;
    int all = 1;
    for (int j = 0; j < BK; ++j) all &= st->cdone[j];
    st->done = all;
  }
}

// First r.z: rho, and beta = 0 so that the p update gives p = z.
__global__ __launch_bounds__(256) void k_blk_rho(CgBlockState *st, const double *__restrict__ zpart, int np) {
  __shared__ double red[256], tot[BK];
  col_sums(zpart, np, red, tot);
  if (threadIdx.x < BK) {
    st->rho[threadIdx.x] = tot[threadIdx.x];
    st->beta[threadIdx.x] = 0.0;
  }
}

// alpha = rho / (p.q) per running column; a column whose p.q is not positive
// and finite stops (breakdown).
__global__ __launch_bounds__(256) void k_blk_alpha(CgBlockState *st, const double *__restrict__ gpart, int np,
                                                   double *__restrict__ alpha_h) {
  __shared__ double red[256], tot[BK];
  if (st->done) return;
  col_sums(gpart, np, red, tot);
  const int t = threadIdx.x;
  if (t < BK) {
    double a = 0.0;
    if (!st->cdone[t]) {
      const double gam = tot[t];
      if (gam > 0.0 && isfinite(gam)) {
        a = st->rho[t] / gam;
      } else {
        st->fail[t] = 1;
        st->cdone[t] = 1;
      }
    }
    st->alpha[t] = a;
    alpha_h[(int64_t)st->it * BK + t] = a;
  }
  __syncthreads();
  if (t == 0) {
    int all = 1;
    for (int j = 0; j < BK; ++j) all &= st->cdone[j];
    st->done = all;
  }
}

// Stopping test after the x / r update, per running column.
__global__ __launch_bounds__(256) void k_blk_test(CgBlockState *st, const double *__restrict__ rpart, int np) {
  __shared__ double red[256], tot[BK];
  if (st->done) return;
  col_sums(rpart, np, red, tot);
  const int t = threadIdx.x;
  if (t < BK && !st->cdone[t]) {
    const double rn2 = tot[t];
    const bool conv = rn2 <= st->rtol2 * st->r0sq[t];
    const bool cap = st->nupd[t] >= st->maxit;
    st->relres[t] = st->r0sq[t] > 0.0 ? sqrt(rn2 / st->r0sq[t]) : 0.0;
    if (conv || cap || !isfinite(rn2)) {
      st->cdone[t] = 1;
      st->converged[t] = conv ? 1 : 0;
      if (!isfinite(rn2)) st->fail[t] = 1;
    }
  }
  __syncthreads();
  if (t == 0) {
    int all = 1;
    for (int j = 0; j < BK; ++j) all &= st->cdone[j];
    st->done = all;
  }
}

// beta = rho' / rho per running column (0 for stopped ones, whose p is then
// just z and is not used again); the block iteration is complete.
__global__ __launch_bounds__(256) void k_blk_beta(CgBlockState *st, const double *__restrict__ zpart, int np,
                                                  double *__restrict__ beta_h) {
  __shared__ double red[256], tot[BK];
  if (st->done) return;
  col_sums(zpart, np, red, tot);
  const int t = threadIdx.x;
  if (t < BK) {
    double b = 0.0;
    if (!st->cdone[t]) {
      b = tot[t] / st->rho[t];
      st->rho[t] = tot[t];
    }
    st->beta[t] = b;
    beta_h[(int64_t)st->it * BK + t] = b;
  }
  __syncthreads();
  if (t == 0) st->it += 1;
}

// ---- CG vector kernels (grid-stride over the n * BK entries: a thread keeps
// the column threadIdx.x % BK) ------------------------------------------------------
__global__ __launch_bounds__(256) void k_blk_fill(int64_t n, double *x, double v, const CgBlockState *st) {
  if (blk_done(st)) return;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) x[e] = v;
}

__global__ __launch_bounds__(256) void k_blk_norm2(int64_t n, const double *__restrict__ x, double *part) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * BK; e += (int64_t)gridDim.x * 256)
    v = fma(x[e], x[e], v);
  col_partial(v, part, red);
}

// q = assembled local products + B_0^T x_p; partials of p.q
__global__ __launch_bounds__(256) void k_blk_assemble(DevGeom g, const double *__restrict__ yloc,
                                                      const double *__restrict__ xp,
                                                      const double *__restrict__ dscale,
                                                      const double *__restrict__ pu, double *__restrict__ q,
                                                      double *part, const CgBlockState *st) {
  __shared__ double red[256];
  if (blk_done(st)) return;
  const int j = threadIdx.x & (BK - 1);
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)g.nGamma * BK;
       e += (int64_t)gridDim.x * 256) {
    const int gi = (int)(e / BK);
    const int sm = g.sub_minus[gi], sp = g.sub_plus[gi];
    const double b0 = -dscale[sm] * xp[(int64_t)sm * BK + j] + dscale[sp] * xp[(int64_t)sp * BK + j];
    const double qq = yloc[(int64_t)g.own_minus[gi] * BK + j] + yloc[(int64_t)g.own_plus[gi] * BK + j] + b0;
    q[e] = qq;
    v = fma(pu[e], qq, v);
  }
  col_partial(v, part, red);
}

// x += alpha p, r -= alpha q (running columns); partials of r.r
__global__ __launch_bounds__(256) void k_blk_update_xr(int nGamma, int N, const double *__restrict__ pu,
                                                       const double *__restrict__ q, const double *__restrict__ pp,
                                                       double *xu, double *ru, double *xp, double *rpart,
                                                       CgBlockState *st) {
  __shared__ double red[256];
  if (st->done) return;
  const int j = threadIdx.x & (BK - 1);
  const bool run = !st->cdone[j];
  const double a = st->alpha[j];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)nGamma * BK; e += (int64_t)gridDim.x * 256) {
    double r = ru[e];
    if (run) {
      xu[e] = fma(a, pu[e], xu[e]);
      r = fma(-a, q[e], r);
      ru[e] = r;
    }
    v = fma(r, r, v);
  }
  if (blockIdx.x == 0 && run) {
    for (int64_t e = threadIdx.x; e < (int64_t)N * BK; e += 256) xp[e] = fma(a, pp[e], xp[e]);
  }
  col_partial(v, rpart, red);   // ends with a barrier: every thread has read cdone
  if (blockIdx.x == 0 && threadIdx.x < BK && !st->cdone[threadIdx.x]) st->nupd[threadIdx.x] += 1;
}

// p = z + beta p (flux and coarse pressure, z_p from the coarse solution)
__global__ __launch_bounds__(256) void k_blk_update_p(int nGamma, int N, const int *__restrict__ pidx,
                                                      const double *__restrict__ zu, const double *__restrict__ csolb,
                                                      double *pu, double *pp, const CgBlockState *st) {
  if (st->done) return;
  const int j = threadIdx.x & (BK - 1);
  const double b = st->beta[j];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)nGamma * BK; e += (int64_t)gridDim.x * 256)
    pu[e] = fma(b, pu[e], zu[e]);
  if (blockIdx.x == 0) {
    for (int64_t e = threadIdx.x; e < (int64_t)N * BK; e += 256) {
      const int k = (int)(e / BK);
      const double zp = pidx[k] >= 0 ? csolb[(int64_t)pidx[k] * BK + j] : 0.0;
      pp[e] = fma(b, pp[e], zp);
    }
  }
}

// column j of a block vector <-> a single vector
__global__ void k_blk_put(int64_t n, int j, const double *__restrict__ x, double *__restrict__ xb) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) xb[k * BK + j] = x[k];
}
__global__ void k_blk_get(int64_t n, int j, const double *__restrict__ xb, double *__restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) x[k] = xb[k * BK + j];
}

// ---- the local interior problems of the block's sources --------------------------
// Column j of the block's local cell loads: F[e][j] = -f[cell of local cell e]
// (the sign of the single-source kernel's F^i), e over all subdomains' local
// cells (the subdomains' local cell order).
__global__ void k_blk_src_put(int64_t ncells, int j, const int *__restrict__ lcell_global,
                              const double *__restrict__ src, double *__restrict__ F) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < ncells) F[e * BK + j] = -src[lcell_global[e]];
}

// P^i = X^i Y^i for the BK columns of a block, X^i = V'^T V' the symmetric
// pressure operator of subdomain i's interior problem in full column-major
// storage (nc x nc), Y and P in [local cell][BK].  The serial kernels read X^i once per
// source; here one pass over X^i serves all BK sources, as a 16-column product
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64, the lane layout of
// k_blk_symv).  Workgroup (i, y) owns the 256 rows 256 y .. 256 y + 255 of
// subdomain i, wave w the 64 rows R0 = 256 y + 64 w ..; accumulator u holds
// the rows R0 + 16 u + (lane % 16), so that each load instruction reads 128
// contiguous bytes of four columns.  Y^i is staged in LDS XG_CK rows at a
// time (zero padded to whole 16-row tiles), and each wave issues the loads
// of its next tile before the MFMAs of the current one.
constexpr int XG_CK = 256;

__global__ __launch_bounds__(256) void k_blk_xgemm(DevGeom g, const double *__restrict__ Xmat,
                                                   const int64_t *__restrict__ Xoff, const double *__restrict__ Y,
                                                   double *__restrict__ P) {
  __shared__ double ys[XG_CK * BK];
  const int i = blockIdx.x, nc = g.nc[i];
  const int rb = (int)blockIdx.y * 256;
  if (rb >= nc) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t co = g.cell_off[i];
  const double *Xi = Xmat + Xoff[i];
  const double *Yi = Y + co * BK;
  const int R0 = rb + 64 * wv;
  f64x4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  // tile J of the chunk at column c0: this lane's columns c0 + 16 J + 4 lk + k
  // (step k).  Every lane loads, past the edge from a clamped address: a row
  // past the edge is never stored, and a column past it meets the zero
  // padding of Y^i (the entries of X^i are finite).  No load sits in a
  // branch, so the wait before a tile's MFMAs need not cover the next tile's
  // loads, which are issued first (after a chunk's last tile: the next
  // chunk's first).
  auto load_tile = [&](int c0, int J, double (&a)[4][4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = c0 + 16 * J + 4 * lk + k;
      const int64_t cb = (int64_t)(c < nc ? c : 0) * nc;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = R0 + 16 * u + li;
        a[k][u] = __builtin_nontemporal_load(Xi + cb + (r < nc ? r : 0));
      }
    }
  };
  double a[4][4], an[4][4];
  if (R0 < nc) load_tile(0, 0, a);
  static_assert(XG_CK % 32 == 0, "tiles are taken in pairs");
  for (int c0 = 0; c0 < nc; c0 += XG_CK) {
    const int ck = min(XG_CK, nc - c0);
    __syncthreads();   // the previous chunk has been used
    for (int e = tid; e < XG_CK * BK; e += 256) ys[e] = (e < ck * BK) ? Yi[(int64_t)c0 * BK + e] : 0.0;
    __syncthreads();
    if (R0 >= nc) continue;   // the wave still takes part in the barriers
    // tile J from cur, the loads of tile J + 1 into nxt first
    auto step = [&](int J, const double (&cur)[4][4], double (&nxt)[4][4]) {
      load_tile(c0, J + 1, nxt);
      const int cl = 16 * J + 4 * lk;
      double b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) b[k] = ys[(cl + k) * BK + li];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[k][u], b[k], acc[u], 0, 0, 0);
    };
    // tiles in pairs (a, then an), so that no copy waits on loads in flight;
    // an odd count ends with a tile past the edge (its staged Y rows are zero)
    const int nt = (((ck + 15) >> 4) + 1) & ~1;
    for (int J = 0; J < nt; J += 2) {
      step(J, a, an);
      step(J + 1, an, a);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = R0 + 16 * u + 4 * q + lk;
      if (row < nc) P[(co + row) * BK + li] = acc[u][q];
    }
}

// h^i = H^{iT} X^i F^i for the BK columns (the line part of k_source_term,
// from XF = X^i F^i of k_blk_xgemm): thread pairs (interface dof t, column j),
// j fastest, so that 16 neighbouring threads solve the same line for the 16
// columns and read XF coalesced.  h in [sum nG][BK].
template <int CAP, bool STAGED>
__global__ __launch_bounds__(256) void k_blk_source_lines(DevGeom g, const double *__restrict__ mcoef,
                                                          const double *__restrict__ XF, double *__restrict__ hloc) {
  extern __shared__ double mc[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = g.nc[i], nG = g.nG[i];
  const int64_t go = g.g_off[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  const double *ys = XF + g.cell_off[i] * BK;
  if (STAGED) {
    stage_mcoef(nc, lcg, mcoef, mc);
    __syncthreads();
  }
  int ext[3], st[3];
  for (int d = 0; d < 3; ++d) ext[d] = g.ext[3 * i + d];
  st[0] = 1; st[1] = ext[0]; st[2] = ext[0] * ext[1];
  for (int e = tid; e < nG * BK; e += 256) {
    const int t = e / BK, j = e % BK;
    const int64_t fl = go + t;
    const int d = g.lg_dir[fl], lc = g.lg_cell[fl], end = g.lg_end[fl];
    const int n = ext[d];
    const int cd = (lc / st[d]) % n;
    const int s0 = lc - cd * st[d];
    int ms;
    const double *m = line_coef<STAGED>(g, mc, mcoef, lcg, s0, d, st, ms);
    double y[CAP + 1];
    const int eidx = end ? n - 1 : 0;
    double v = (end ? -1.0 : 1.0) * ys[(s0 + eidx * st[d]) * BK + j];
    if (n >= 2) {
      y[0] = 0.0;
      for (int q = 1; q <= n - 1; ++q) y[q] = ys[(s0 + q * st[d]) * BK + j] - ys[(s0 + (q - 1) * st[d]) * BK + j];
      line_solve_s<CAP>(n, m, ms, y);
      const int adj = end ? n - 1 : 1;
      v -= (m[eidx * ms] / 6.0) * y[adj];
    }
    hloc[fl * BK + j] = v;
  }
}

// f* of eq. (reduced right-hand side) for the BK columns: -assembled S u0 +
// assembled h (+ the boundary-flux load sb, shared by all sources; may be null).
__global__ void k_blk_fstar(DevGeom g, const double *__restrict__ yloc, const double *__restrict__ hloc,
                            const double *__restrict__ sb, double *__restrict__ r) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)g.nGamma * BK) return;
  const int64_t gi = e / BK;
  const int j = (int)(e % BK);
  const int64_t a = g.own_minus[gi], b = g.own_plus[gi];
  double v = -(yloc[a * BK + j] + yloc[b * BK + j]) + hloc[a * BK + j] + hloc[b * BK + j];
  if (sb) v += sb[a] + sb[b];
  r[e] = v;
}

// ---- local operators on the matrix cores ---------------------------------------
// Four consecutive entries of a packed column (16-byte aligned: column
// segments start at multiples of four entries), widened to FP64.
__device__ __forceinline__ void load4(const float *p, double *o) {
  const f32x4 v = *reinterpret_cast<const f32x4 *>(p);
  o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ __forceinline__ void load4(const double *p, double *o) {
  const f64x2 v0 = *reinterpret_cast<const f64x2 *>(p), v1 = *reinterpret_cast<const f64x2 *>(p + 2);
  o[0] = v0[0]; o[1] = v0[1]; o[2] = v1[0]; o[3] = v1[1];
}

// Y^i = M^i (w * R_i X) for the BK columns, M^i in packed storage (S^i, or T^i
// of the preconditioner; FP32 entries are widened).  Workgroup (i, y) of
// BLK_SYMV_WAVES waves covers the rows 64 W y .. of subdomain i, one 64-row
// block I per wave, so a large interface is spread over several workgroups
// and CUs; w * R_i X is staged in LDS SYMV_CJ 16-row tiles at a time (32 KB
// whatever the interface size, so that several workgroups share a CU).  Wave
// I forms its rows of Y^i from the whole block row of the symmetric M^i, 16
// columns at a time, on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A(i, k)
// from lane i + 16 k, B(k, j) from lane j + 16 k, C(4 q + lane / 16, lane %
// 16) in register q).  Four accumulators u = 0..3 hold the rows 64 I + 4 i +
// u, and step k of a 16-column tile J takes the columns cl + k, cl = 16 J + 4
// (lane / 16): a lane needs the 4 x 4 block M(r0 + u, cl + k), r0 = 64 I + 4
// i.  Every lane reads four consecutive stored entries per k: at or below the
// diagonal (r0 >= cl) the rows r0 .. r0 + 3 of the columns cl + k, above it the
// rows cl .. cl + 3 of the mirror columns r0 + k, which hold the transpose of
// the block; the 4 x 4 diagonal blocks (r0 = cl) take their upper half from
// their own lower half.  So every tile, left of, across or right of the
// diagonal, issues the same loads, and each wave issues the loads of its next
// tile before the MFMAs of the current one.  M^i is read twice (as rows and
// as mirror columns), both times once per block of BK columns.
constexpr int BLK_SYMV_WAVES = 4;
constexpr int SYMV_CJ = 16;

template <typename TS>
__global__ __launch_bounds__(64 * BLK_SYMV_WAVES) void k_blk_symv(DevGeom g, const TS *__restrict__ M,
                                                                  const int64_t *__restrict__ pk,
                                                                  const double *__restrict__ X, double xscale,
                                                                  const double *__restrict__ xw,
                                                                  double *__restrict__ yloc, const CgBlockState *st) {
  __shared__ double xs[SYMV_CJ * 16 * BK];
  if (blk_done(st)) return;
  // subdomains i = blockIdx.x, + gridDim.x, ... (a grid narrower than N
  // leaves CUs to the work beside it)
  for (int i = blockIdx.x; i < g.N; i += gridDim.x) {
  const int n = g.nG[i], nb = (n + 15) >> 4, np = 4 * ((n + 3) / 4);
  if (64 * BLK_SYMV_WAVES * (int)blockIdx.y >= n) continue;   // whole workgroup past the interface
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int I = BLK_SYMV_WAVES * (int)blockIdx.y + wv;   // this wave's 64-row block
  const bool live = 64 * I < n;
  const int64_t go = g.g_off[i];
  const TS *Mi = M + pk[i];
  f64x4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int r0 = 64 * I + 4 * li;   // this lane's rows r0 + u (accumulator u)
  // t[k][s]: the stored entries of tile J.  Past the edge (also in the tile
  // past the last, J = nb) a lane reads the matrix's first entries instead: a
  // row past the edge is never stored, and a column past it meets the zero
  // padding of the staged X (the stored entries are finite).  No load sits in
  // a branch, so the wait before a tile's MFMAs need not cover the next
  // tile's loads.
  auto load_tile = [&](int J, double (&t)[4][4]) {
    const int cl = 16 * J + 4 * lk;
    const bool ok = r0 < np && cl < np, low = r0 >= cl;
    const int rr = ok ? (low ? r0 : cl) : 0, cb = ok ? (low ? cl : r0) : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) load4(Mi + gp_index(n, rr, cb + k), t[k]);
  };
  double t[4][4], tn[4][4];
  if (live) load_tile(0, t);
  static_assert(SYMV_CJ % 2 == 0, "tiles are taken in pairs");
  for (int J0 = 0; J0 < nb; J0 += SYMV_CJ) {
    __syncthreads();   // the previous chunk has been used
    for (int e = tid; e < SYMV_CJ * 16 * BK; e += 64 * BLK_SYMV_WAVES) {
      const int r = 16 * J0 + e / BK, j = e % BK;
      xs[e] = (r < n) ? (xw ? xw[go + r] : xscale) * X[(int64_t)g.Rmap[go + r] * BK + j] : 0.0;
    }
    __syncthreads();
    if (!live) continue;   // the wave still takes part in the barriers
    // tile J from cur, the loads of tile J + 1 into nxt first
    auto step = [&](int J, const double (&cur)[4][4], double (&nxt)[4][4]) {
      load_tile(J + 1, nxt);
      const int cl = 16 * J + 4 * lk;
      double b[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) b[k] = xs[(cl - 16 * J0 + k) * BK + li];
      // M(r0 + u, cl + k): cur[k][u] at or below the diagonal, cur[u][k] above
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool lower = r0 > cl || (r0 == cl && u >= k);
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(lower ? cur[k][u] : cur[u][k], b[k], acc[u], 0, 0, 0);
        }
    };
    // tiles in pairs (t, then tn), so that no copy waits on loads in flight;
    // an odd count ends with the tile past the last (J = nb, inside the
    // chunk's LDS: its staged X rows are zero)
    const int J1 = J0 + ((min(nb, J0 + SYMV_CJ) - J0 + 1) & ~1);
    for (int J = J0; J < J1; J += 2) {
      step(J, t, tn);
      step(J + 1, tn, t);
    }
  }
  if (live) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 64 * I + 16 * q + 4 * lk + u;
        if (row < n) yloc[(go + row) * BK + li] = acc[u][q];
      }
  }
  }
}

// g^i = Psi^{iT} (w * R_i X) for the BK columns, added into the coarse
// right-hand sides b at the coarse dofs: as in the
// single-column kernel, a face's coarse dof gets the pieces of its two
// subdomains onto zero, the same sum in either order.  The waves split the
// 16-row blocks of Psi^i, C(i, j) = sum_k Psi(k, 16 K + i) X(k, j) on the
// matrix cores (A(i, k) from lane i + 16 k: four consecutive rows of one column
// per lane quad), and their four partial tiles are added in LDS, wave after
// wave (a fixed order in 2 KB, so that X of interfaces up to 1,232 dofs fits).
template <typename TS>
__global__ __launch_bounds__(256) void k_blk_psi_apply(DevGeom g, const TS *__restrict__ Psi,
                                                       const int64_t *__restrict__ psi_off,
                                                       const int *__restrict__ sub_coff,
                                                       const int *__restrict__ sub_cmap, const double *__restrict__ X,
                                                       double xscale, const double *__restrict__ xw,
                                                       double *__restrict__ b, const CgBlockState *st) {
  extern __shared__ double sh[];
  if (blk_done(st)) return;
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // (wave-uniform loop bounds)
  const int li = lane & 15, lk = lane >> 4;
  const int n = g.nG[i], nb = (n + 15) >> 4, ldp = ld4(n);
  const int64_t go = g.g_off[i];
  double *xs = sh, *red = sh + nb * 16 * BK;   // red: one 16 x 16 tile
  for (int e = tid; e < nb * 16 * BK; e += 256) {
    const int r = e / BK, j = e % BK;
    xs[e] = (r < n) ? (xw ? xw[go + r] : xscale) * X[(int64_t)g.Rmap[go + r] * BK + j] : 0.0;
  }
  __syncthreads();
  const int c0 = sub_coff[i], nci = sub_coff[i + 1] - c0;
  const TS *P = Psi + psi_off[i];
  for (int K = 0; 16 * K < nci; ++K) {
    // Two independent MFMA chains, eight loads issued at once.  No load sits
    // in a branch (the compiler would wait on each one): an entry past the
    // edge is read from the basis's first entry instead; a row past the
    // interface meets the zero padding of xs, a column past the subdomain's
    // coarse dofs is never stored.
    f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int c = 16 * K + li;
    const int64_t cb = (int64_t)(c < nci ? c : 0) * ldp;
    auto ld = [&](int R, int s) {
      const int r = 16 * R + 4 * s + lk;
      return (double)P[(c < nci && r < n) ? cb + r : 0];
    };
    int R = wv;
    for (; R + 4 < nb; R += 8) {
      double a[8];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a[s] = ld(R, s);
        a[4 + s] = ld(R + 4, s);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], xs[(16 * R + 4 * s + lk) * BK + li], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[4 + s], xs[(16 * (R + 4) + 4 * s + lk) * BK + li], acc1, 0, 0,
                                                    0);
      }
    }
    for (; R < nb; R += 4) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ld(R, s), xs[(16 * R + 4 * s + lk) * BK + li], acc0, 0, 0, 0);
    }
    const f64x4 acc = acc0 + acc1;
    for (int w = 0; w < 4; ++w) {
      if (wv == w) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[q * 64 + lane] = (w == 0 ? 0.0 : red[q * 64 + lane]) + acc[q];
      }
      __syncthreads();
    }
    {
      const int q = tid >> 6, l = tid & 63;
      const int cc = 16 * K + 4 * q + (l >> 4), j = l & 15;
      if (cc < nci) atomicAdd(b + (int64_t)sub_cmap[c0 + cc] * BK + j, red[q * 64 + l]);
    }
    __syncthreads();
  }
}

// W^i = Psi^i alpha^(i) for the BK columns (alpha gathered from the coarse
// solutions into LDS, [nc^i][BK]); wave w forms the 16-row blocks w, w + 4, ...
// (A(i, k) = Psi(16 R + i, 16 K + 4 s + k): 16 consecutive rows of a column
// per 16 lanes).
template <typename TS>
__global__ __launch_bounds__(256) void k_blk_psi_correct(DevGeom g, DevCoarse cs, const TS *__restrict__ Psi,
                                                         const int64_t *__restrict__ psi_off,
                                                         const double *__restrict__ csolb,
                                                         double *__restrict__ wloc, const CgBlockState *st) {
  extern __shared__ double al[];
  if (blk_done(st)) return;
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int n = g.nG[i], nb = (n + 15) >> 4, ldp = ld4(n);
  const int64_t go = g.g_off[i];
  const int c0 = cs.sub_coff[i], nci = cs.sub_coff[i + 1] - c0, ncb = (nci + 15) >> 4;
  for (int e = tid; e < ncb * 16 * BK; e += 256) {
    const int c = e / BK, j = e % BK;
    al[e] = (c < nci) ? csolb[(int64_t)cs.sub_cmap[c0 + c] * BK + j] : 0.0;
  }
  __syncthreads();
  const TS *P = Psi + psi_off[i];
  for (int R = wv; R < nb; R += 4) {
    // Two independent MFMA chains, eight loads issued at once.  No load sits
    // in a branch (the compiler would wait on each one): an entry past the
    // edge is read from the basis's first entry instead; a column past the
    // subdomain's coarse dofs meets the zero padding of al, a row past the
    // interface is never stored.
    f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int r = 16 * R + li;
    auto ld = [&](int K, int s) {
      const int c = 16 * K + 4 * s + lk;
      return (double)P[(r < n && c < nci) ? (int64_t)c * ldp + r : 0];
    };
    int K = 0;
    for (; K + 1 < ncb; K += 2) {
      double a[8];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a[s] = ld(K, s);
        a[4 + s] = ld(K + 1, s);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], al[(16 * K + 4 * s + lk) * BK + li], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[4 + s], al[(16 * (K + 1) + 4 * s + lk) * BK + li], acc1, 0, 0,
                                                    0);
      }
    }
    for (; K < ncb; ++K) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ld(K, s), al[(16 * K + 4 * s + lk) * BK + li], acc0, 0, 0, 0);
    }
    const f64x4 acc = acc0 + acc1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * R + 4 * q + lk;
      if (row < n) wloc[(go + row) * BK + li] = acc[q];
    }
  }
}

// z = E (y + w) per column (multiplicity or stiffness weights), then each
// face's total set to its zero-net-flux coarse dof; partials of r.z.  One
// face per wave (lanes: column lane % 16, every fourth dof from lane / 16).
__global__ __launch_bounds__(256) void k_blk_average(DevGeom g, DevCoarse cs, const double *__restrict__ wloc,
                                                     const double *__restrict__ yloc,
                                                     const double *__restrict__ csolb,
                                                     double *__restrict__ z, const double *__restrict__ r,
                                                     double *part, const CgBlockState *st) {
  __shared__ double red[256];
  if (blk_done(st)) return;
  const int lane = threadIdx.x & 63, j = lane & 15, lk = lane >> 4;
  double v = 0.0;
  for (int f = blockIdx.x * 4 + (threadIdx.x >> 6); f < g.nF; f += gridDim.x * 4) {
    const int n = g.f_n[f];
    const int64_t base = g.g_off[g.f_minus[f]] + g.f_loffm[f];
    const bool sw = g.fw_minus != nullptr;
    const double wm = sw ? g.fw_minus[f] : 0.5, wp = sw ? g.fw_plus[f] : 0.5;
    // four steps' loads (each a chain Rmap -> own_plus -> values) issued
    // together, added in the order of one step at a time
    double tsum = 0.0;
    int a = lk;
    for (; a + 12 < n; a += 16) {
      double vm[4], vp[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t km = (base + a + 4 * u) * BK + j, kp = (int64_t)g.own_plus[g.Rmap[base + a + 4 * u]] * BK + j;
        vm[u] = yloc[km] + wloc[km];
        vp[u] = yloc[kp] + wloc[kp];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) tsum += wm * vm[u] + wp * vp[u];
    }
    for (; a < n; a += 4) {
      const int64_t km = (base + a) * BK + j, kp = (int64_t)g.own_plus[g.Rmap[base + a]] * BK + j;
      tsum += wm * (yloc[km] + wloc[km]) + wp * (yloc[kp] + wloc[kp]);
    }
    tsum += __shfl_xor(tsum, 16, 64);
    tsum += __shfl_xor(tsum, 32, 64);
    const double corr = (csolb[(int64_t)cs.face_cofs[f] * BK + j] - tsum) / n;
    auto put = [&](int gi, double wsm, double wsp, double rr) {
      const double zz = (sw ? wm * wsm + wp * wsp : 0.5 * (wsm + wsp)) + corr;
      z[(int64_t)gi * BK + j] = zz;
      v = fma(rr, zz, v);
    };
    a = lk;
    for (; a + 12 < n; a += 16) {
      int gi[4];
      double sm[4], sp[4], rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        gi[u] = g.Rmap[base + a + 4 * u];
        const int64_t km = (base + a + 4 * u) * BK + j, kp = (int64_t)g.own_plus[gi[u]] * BK + j;
        sm[u] = yloc[km] + wloc[km];
        sp[u] = yloc[kp] + wloc[kp];
        rv[u] = r[(int64_t)gi[u] * BK + j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) put(gi[u], sm[u], sp[u], rv[u]);
    }
    for (; a < n; a += 4) {
      const int gi = g.Rmap[base + a];
      const int64_t km = (base + a) * BK + j, kp = (int64_t)g.own_plus[gi] * BK + j;
      put(gi, yloc[km] + wloc[km], yloc[kp] + wloc[kp], r[(int64_t)gi * BK + j]);
    }
  }
  col_partial(v, part, red);
}

// ---- coarse sweeps ---------------------------------------------------------------
// The sweeps of coarse.hip for the BK columns, with the coarse vectors
// interleaved ([dof][BK], like the interface vectors).  A task is 64 rows
// (forward) or 64 columns (backward) of one front, a 16-row (16-column) block
// per wave, on the matrix cores: each entry of R is read once per block of BK
// columns.  Task descriptor, three int4: {first row / column, n, m, first
// dof}, {v_off, b_off, child slot, 0}, {r_off low, r_off high, 0, 0}.
constexpr int BLK_SWEEP_ROWS = 64;

// Forward: t_p = b_P + S0_p[P] + S1_p[P]; rows r < n of R = [L_PP^{-1};
// L_BP L_PP^{-1}] (packed lower triangle, then m full rows) give z_P[r], rows
// n + k push w_p[k] = S0_p[B] + S1_p[B] - row . t_p into the parent's slot
// array.  t_p is staged in LDS FWD_KC entries at a time (32 KB whatever the
// front size: a level holding one large front among many small ones keeps
// several workgroups per CU), and the four waves split each chunk's k range:
// wave w forms the partial products of all 64 rows of the task over its
// quarter, four 16-row blocks as independent MFMA chains, and the partials
// are added in LDS in wave order (in the chunk's space).
constexpr int FWD_KC = 256;
constexpr int FWD_SHM_DOUBLES = FWD_KC * BK;   // = 4 waves x 64 rows x BK partials

__global__ __launch_bounds__(256) void k_blk_nd_fwd(int t0, const int4 *__restrict__ task,
                                                    const double *__restrict__ FR, const int *__restrict__ wdst,
                                                    const double *__restrict__ b, double *S0, double *S1,
                                                    double *__restrict__ z, const CgBlockState *st) {
  __shared__ double tl[FWD_SHM_DOUBLES];
  const int4 *td = task + 3 * (int64_t)(t0 + blockIdx.x);
  const int4 d0 = td[0], d1 = td[1], d2 = td[2];
  if (blk_done(st)) return;
  const int j0 = d0.x, n = d0.y, m = d0.z, fst = d0.w, vo = d1.x, bo = d1.y, slot = d1.z;
  const int64_t ro = (int64_t)(((uint64_t)(uint32_t)d2.y << 32) | (uint32_t)d2.x);
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // (wave-uniform loop bounds)
  const int n4 = (n + 3) & ~3;
  // the task's rows j0 + 16 u + li (u = 0..3); rows below n stop at their
  // diagonal, rows past the front have none.  No load sits in a branch (the
  // compiler would wait on each one): past a row's end a lane reads a
  // clamped entry and multiplies it by 0 (the factor's entries are finite).
  const double *row[4];
  int len[4], lmax[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = j0 + 16 * u + li;
    if (r < n) {
      row[u] = FR + ro + (int64_t)r * (r + 1) / 2;
      len[u] = r + 1;
    } else if (r < n + m) {
      row[u] = FR + ro + (int64_t)n * (n + 1) / 2 + (int64_t)(r - n) * n;
      len[u] = n;
    } else {
      row[u] = FR + ro;
      len[u] = 0;
    }
    lmax[u] = len[u] > 0 ? len[u] - 1 : 0;
  }
  const int kmax = (j0 + 64 < n) ? min(n4, (j0 + 64 + 3) & ~3) : n4;
  f64x4 ac[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) ac[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < kmax; c0 += FWD_KC) {
    const int ck = min(FWD_KC, kmax - c0);
    __syncthreads();   // the previous chunk has been used
    // (padding rows c >= n read row n - 1 and are multiplied by 0)
#pragma unroll 8
    for (int e = tid; e < ck * BK; e += 256) {
      const int c = c0 + e / BK, j = e % BK, cc = min(c, n - 1);
      tl[e] = ((b[(int64_t)(fst + cc) * BK + j] + S0[(int64_t)(vo + cc) * BK + j]) + S1[(int64_t)(vo + cc) * BK + j]) *
              (c < n ? 1.0 : 0.0);
    }
    __syncthreads();
    // wave w: chunk entries 64 w .. 64 w + 63, 32 loads per lane in flight
    const int kw0 = min(ck, 64 * wv), kw1 = min(ck, kw0 + 64);
    int k0 = kw0;
    for (; k0 + 32 <= kw1; k0 += 32) {
      double a[8][4], bv[8];
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int kl = k0 + 4 * h + lk, k = c0 + kl;
        bv[h] = tl[kl * BK + li];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[h][u] = row[u][min(k, lmax[u])] * (k < len[u] ? 1.0 : 0.0);
      }
#pragma unroll
      for (int h = 0; h < 8; ++h)
#pragma unroll
        for (int u = 0; u < 4; ++u) ac[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][u], bv[h], ac[u], 0, 0, 0);
    }
    for (; k0 < kw1; k0 += 4) {
      const int kl = k0 + lk, k = c0 + kl;
      const double bk = tl[kl * BK + li];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        ac[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[u][min(k, lmax[u])] * (k < len[u] ? 1.0 : 0.0), bk, ac[u],
                                                     0, 0, 0);
    }
  }
  __syncthreads();   // the last chunk has been used: its space takes the partials
  double *red = tl;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[(wv * 64 + 16 * u + 4 * q + lk) * BK + li] = ac[u][q];
  __syncthreads();
  for (int e = tid; e < 64 * BK; e += 256) {
    const int rl = e / BK, j = e % BK, rr = j0 + rl;
    const double v = ((red[rl * BK + j] + red[(64 + rl) * BK + j]) + red[(128 + rl) * BK + j]) + red[(192 + rl) * BK + j];
    if (rr < n) {
      z[(int64_t)(fst + rr) * BK + j] = v;
    } else if (rr < n + m) {
      const double base = S0[(int64_t)(vo + rr) * BK + j] + S1[(int64_t)(vo + rr) * BK + j];
      (slot ? S1 : S0)[(int64_t)wdst[bo + (rr - n)] * BK + j] = base - v;
    }
  }
}

// Backward: columns c of the packed lower trapezoid BC (column c holds rows
// c .. n + m - 1): x_c = sum_rho BC(rho, c) in(rho), in = s z on the own dofs
// and -x_B on the B part; each x[d] is also stored into every B vector that
// holds d.  The four waves split the task's rho range (the top levels hold
// few, large fronts): wave w forms the partial sums of all 64 columns of the
// task over its quarter, four 16-column blocks as independent MFMA chains
// sharing each step's in(rho), and the partials are added in LDS in wave
// order.  in is read from the (L2 resident) vectors.
__global__ __launch_bounds__(256) void k_blk_nd_bwd(int t0, const int4 *__restrict__ task,
                                                    const double *__restrict__ BC, const double *__restrict__ z,
                                                    const double *__restrict__ sg, const int *__restrict__ xsc_off,
                                                    const int *__restrict__ xsc, double *XB, double *__restrict__ x,
                                                    const CgBlockState *st) {
  __shared__ double red[4 * 64 * BK];
  const int4 *td = task + 3 * (int64_t)(t0 + blockIdx.x);
  const int4 d0 = td[0], d1 = td[1], d2 = td[2];
  if (blk_done(st)) return;
  const int c0 = d0.x, n = d0.y, m = d0.z, fst = d0.w, bo = d1.y;
  const int64_t ro = (int64_t)(((uint64_t)(uint32_t)d2.y << 32) | (uint32_t)d2.x);
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // (wave-uniform loop bounds)
  const int f = n + m;
  // this lane's columns c0 + 16 u + li; col[u][rho], rho >= c (a column past
  // the front: the front's first entry).  No load sits in a branch (the
  // compiler would wait on each one): outside its range a lane reads a clamped
  // entry and multiplies it by 0 (the factor's entries and the vectors are
  // finite).
  const double *col[4];
  int cu[4], rlo[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = c0 + 16 * u + li;
    cu[u] = c < n ? c : f;   // a column past the front takes no rows
    col[u] = c < n ? BC + ro + (int64_t)c * f - (int64_t)c * (c - 1) / 2 - c : BC + ro;
    rlo[u] = c < n ? c : 0;
  }
  const int rho0 = c0 & ~3;
  const int qr = 4 * ((f - rho0 + 15) / 16);   // per wave, a multiple of 4
  const int rw0 = min(f, rho0 + wv * qr), rw1 = min(f, rw0 + qr);
  auto in_of = [&](int rho) {
    const int rz = min(rho, n - 1);
    const int64_t rx = m > 0 ? bo + min(max(rho - n, 0), m - 1) : 0;
    return sg[fst + rz] * z[(int64_t)(fst + rz) * BK + li] * (rho < n ? 1.0 : 0.0) -
           XB[rx * BK + li] * ((rho >= n && rho < f) ? 1.0 : 0.0);
  };
  f64x4 ac[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) ac[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  int k0 = rw0;
  for (; k0 + 16 <= rw1; k0 += 16) {
    double a[4][4], in[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int rho = k0 + 4 * h + lk;
      in[h] = in_of(rho);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool ia = rho >= cu[u] && rho < f;
        a[h][u] = col[u][ia ? rho : rlo[u]] * (ia ? 1.0 : 0.0);
      }
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int u = 0; u < 4; ++u) ac[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][u], in[h], ac[u], 0, 0, 0);
  }
  for (; k0 < rw1; k0 += 4) {
    const int rho = k0 + lk;
    const double inr = in_of(rho);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ia = rho >= cu[u] && rho < f;
      ac[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(col[u][ia ? rho : rlo[u]] * (ia ? 1.0 : 0.0), inr, ac[u], 0, 0,
                                                   0);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[(wv * 64 + 16 * u + 4 * q + lk) * BK + li] = ac[u][q];
  __syncthreads();
  for (int e = tid; e < 64 * BK; e += 256) {
    const int cl = e / BK, j = e % BK, cc = c0 + cl;
    if (cc >= n) continue;
    const double v = ((red[cl * BK + j] + red[(64 + cl) * BK + j]) + red[(128 + cl) * BK + j]) + red[(192 + cl) * BK + j];
    const int d = fst + cc;
    x[(int64_t)d * BK + j] = v;
    for (int p = xsc_off[d]; p < xsc_off[d + 1]; ++p) XB[(int64_t)xsc[p] * BK + j] = v;
  }
}

// ---- dense top block of the coarse solve ------------------------------------------
// t_t[t][j] = b_j[d0 + t] + the updates the swept fronts pushed for that dof
__global__ __launch_bounds__(256) void k_blk_top_gather(int nt, int d0, const int *__restrict__ tg_off,
                                                        const int *__restrict__ tg, const double *__restrict__ b,
                                                        const double *__restrict__ S0, const double *__restrict__ S1,
                                                        double *__restrict__ tt, const CgBlockState *st) {
  if (blk_done(st)) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nt * BK) return;
  const int t = (int)(e / BK), j = (int)(e % BK);
  double v = b[(int64_t)(d0 + t) * BK + j];
  for (int q = tg_off[t]; q < tg_off[t + 1]; ++q) v += S0[(int64_t)tg[q] * BK + j] + S1[(int64_t)tg[q] * BK + j];
  tt[e] = v;
}

// x_t = S_t^{-1} t_t for the rows [16 blockIdx.x, 16 blockIdx.x + 16) and the
// BK columns: eight waves split the columns of S_t^{-1} (row major, ld),
// A(i, k) = S_t^{-1}(16 I + i, k0 + 4 s + k) (four consecutive entries of a row
// per lane quad), B(k, j) = t_t(k0 + 4 s + k, j), eight steps of loads in
// flight per lane; the partial tiles meet in LDS in a fixed order.  Each x[d]
// is also stored into every B vector holding d (for the backward sweeps of
// the levels below).
constexpr int TOP_GEMM_WAVES = 8;

__global__ __launch_bounds__(64 * TOP_GEMM_WAVES) void k_blk_top_gemm(int nt, int ld, const double *__restrict__ Kt,
                                                                      const double *__restrict__ tt, int d0,
                                                                      const int *__restrict__ xsc_off,
                                                                      const int *__restrict__ xsc,
                                                                      double *__restrict__ XB,
                                                                      double *__restrict__ x,
                                                                      const CgBlockState *st) {
  __shared__ double red[TOP_GEMM_WAVES * 256];
  if (blk_done(st)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int r = 16 * blockIdx.x + li;
  const int nk4 = (nt + 3) / 4, per = (nk4 + TOP_GEMM_WAVES - 1) / TOP_GEMM_WAVES;
  const int s0 = wv * per, s1 = min(nk4, s0 + per);
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  const double *row = Kt + (int64_t)min(r, nt - 1) * ld;
  for (int s = s0; s < s1; s += 8) {
    double a[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = 4 * (s + u) + lk;
      const bool ok = s + u < s1 && k < nt;
      a[u] = (ok && r < nt) ? row[k] : 0.0;
      bv[u] = ok ? tt[(int64_t)k * BK + li] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bv[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[wv * 256 + q * 64 + lane] = acc[q];
  __syncthreads();
  if (tid >= 256) return;
  const int q = tid >> 6, l = tid & 63;
  double v = 0.0;
#pragma unroll
  for (int w = 0; w < TOP_GEMM_WAVES; ++w) v += red[w * 256 + q * 64 + l];
  const int rr = 16 * blockIdx.x + 4 * q + (l >> 4), j = l & 15;
  if (rr < nt) {
    const int d = d0 + rr;
    x[(int64_t)d * BK + j] = v;
    for (int p = xsc_off[d]; p < xsc_off[d + 1]; ++p) XB[(int64_t)xsc[p] * BK + j] = v;
  }
}

template __global__ void k_blk_symv<double>(DevGeom, const double *, const int64_t *, const double *, double,
                                            const double *, double *, const CgBlockState *);
template __global__ void k_blk_symv<float>(DevGeom, const float *, const int64_t *, const double *, double,
                                           const double *, double *, const CgBlockState *);
template __global__ void k_blk_psi_apply<double>(DevGeom, const double *, const int64_t *, const int *, const int *,
                                                 const double *, double, const double *, double *,
                                                 const CgBlockState *);
template __global__ void k_blk_psi_apply<float>(DevGeom, const float *, const int64_t *, const int *, const int *,
                                                const double *, double, const double *, double *,
                                                const CgBlockState *);
template __global__ void k_blk_psi_correct<double>(DevGeom, DevCoarse, const double *, const int64_t *,
                                                   const double *, double *, const CgBlockState *);
template __global__ void k_blk_psi_correct<float>(DevGeom, DevCoarse, const float *, const int64_t *, const double *,
                                                  double *, const CgBlockState *);

}  // namespace bddc
