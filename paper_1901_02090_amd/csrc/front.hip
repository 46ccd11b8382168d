// Setup of the coarse saddle point's multifrontal signed Cholesky
// K = L diag(s) L^T (step 1 of Algorithm "BDDC preconditioner"; coarse.hip
// applies the result), one launch per nested-dissection level, one workgroup
// per front p (own dofs P, n of them, later dofs B, m of them):
//   F = [K_PP K_PB; K_BP K_BB]-part assembled from the local coarse matrices
//       A_c^i and divergence rows, plus the children's update matrices;
//   partial factor: L_PP, L_BP = K_BP L_PP^{-T} s_P, U = F_BB - L_BP s_P L_BP^T
//       (U stays in F for the parent's extend-add);
//   stored per front: R = [L_PP^{-1}; L_BP L_PP^{-1}] ((n+m) x n, the first
//       block lower triangular), row-packed for the forward sweep and
//       column-packed for the backward sweep.
#include "common.hpp"
#include "dense.hpp"

namespace bddc {

struct DevFronts {
  const int *first, *n, *m, *ch, *b_off, *bidx, *ext, *touch_off, *touch;
  const int64_t *F_off, *w_off, *q_off, *r_off, *v_off;
};

// Assemble, partially factor and invert the fronts [f0, f0 + gridDim.x) of one
// level.  F, W (n x n), Q (m x n) are workspaces; FR / BC receive R.
// Fronts with at least `split` own dofs (0: none) factor only their own block
// here: L_BP, the inverse, Q and the packing are spread over many workgroups
// by k_front_rows, k_front_inv, k_front_q and k_front_pack.
__global__ __launch_bounds__(256, 2) void k_front_factor(DevGeom g, DevCoarse cs, DevFronts fd, int f0,
                                                      const double *__restrict__ Ac, const int64_t *__restrict__ ac_off,
                                                      const double *__restrict__ dscale,
                                                      const double *__restrict__ sgn, double *F, double *W,
                                                      double *Q, double *FR, double *BC, int *err, int split) {
  __shared__ double lds[LDS_DOUBLES];
  const int p = f0 + blockIdx.x, tid = threadIdx.x;
  const int first = fd.first[p], n = fd.n[p], m = fd.m[p], f = n + m;
  const int *Bp = fd.bidx + fd.b_off[p];
  double *Fp = F + fd.F_off[p];
  for (int64_t e = tid; e < (int64_t)f * f; e += WG) Fp[e] = 0.0;
  __syncthreads();
  // position of coarse dof u >= first in [P, B]; -1 if absent
  auto pos = [&](int u) -> int {
    if (u < first + n) return u - first;
    int lo = 0, hi = m;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Bp[mid] < u) lo = mid + 1; else hi = mid;
    }
    return (lo < m && Bp[lo] == u) ? n + lo : -1;
  };
  // original entries K(u, v), u >= v, v in P: subdomain by subdomain, so a
  // face entry shared by two subdomains is summed in a fixed order
  for (int t = fd.touch_off[p]; t < fd.touch_off[p + 1]; ++t) {
    const int i = fd.touch[t];
    const int c0 = cs.sub_coff[i], nci = cs.sub_coff[i + 1] - c0;
    const double *A = Ac + ac_off[i];
    for (int e = tid; e < nci * nci; e += WG) {
      const int a = e % nci, b = e / nci;
      const int u = cs.sub_cmap[c0 + a], v = cs.sub_cmap[c0 + b];
      if (u < v || v < first || v >= first + n) continue;
      const int pu = pos(u);
      if (pu < 0) { atomicOr(err, 128); continue; }
      Fp[pu + (size_t)(v - first) * f] += A[e];
    }
    const int pi = cs.pidx[i];
    if (pi >= 0) {
      // divergence row of subdomain i: -d_i * (+1 if the face normal leaves Omega^i)
      for (int t2 = g.sub_face_off[i] + tid; t2 < g.sub_face_off[i + 1]; t2 += WG) {
        const int fc = g.sub_faces[t2];
        const int jf = cs.face_cofs[fc];
        if (jf < first || jf >= first + n) continue;
        const double so = (g.f_minus[fc] == i) ? 1.0 : -1.0;
        const int pp = pos(pi);
        if (pp < 0 || pi < jf) { atomicOr(err, 128); continue; }
        Fp[pp + (size_t)(jf - first) * f] += -dscale[i] * so;
      }
    }
    __syncthreads();
  }
  // extend-add of the children's update matrices (lower triangles): wave w
  // takes columns w, w + 4, ...; its lanes run down the column four rows at a
  // time (ex is one-to-one, so the four targets are distinct)
  const int lane = tid & 63, wv = tid >> 6;
  constexpr int NW = WG / 64;
  for (int k = 0; k < 2; ++k) {
    const int c = fd.ch[2 * p + k];
    if (c < 0) continue;
    const int nc = fd.n[c], mc = fd.m[c], fc = nc + mc;
    const double *Uc = F + fd.F_off[c] + nc + (size_t)nc * fc;
    const int *ex = fd.ext + fd.b_off[c];
    for (int k2 = wv; k2 < mc; k2 += NW) {
      double *Fcol = Fp + (size_t)ex[k2] * f;
      const double *Ucol = Uc + (size_t)k2 * fc;
      int k1 = k2 + lane;
      for (; k1 + 192 < mc; k1 += 256) {
        const int e0 = ex[k1], e1 = ex[k1 + 64], e2 = ex[k1 + 128], e3 = ex[k1 + 192];
        const double u0 = Ucol[k1], u1 = Ucol[k1 + 64], u2 = Ucol[k1 + 128], u3 = Ucol[k1 + 192];
        const double v0 = Fcol[e0], v1 = Fcol[e1], v2 = Fcol[e2], v3 = Fcol[e3];
        Fcol[e0] = v0 + u0;
        Fcol[e1] = v1 + u1;
        Fcol[e2] = v2 + u2;
        Fcol[e3] = v3 + u3;
      }
      for (; k1 < mc; k1 += 64) Fcol[ex[k1]] += Ucol[k1];
    }
    __syncthreads();
  }
  // U = F_BB - L_BP s_P L_BP^T is left to k_front_schur (many workgroups)
  // a large front factors its own block here; k_front_rows forms L_BP
  const bool big = split > 0 && n >= split;
  if (wg_potrf(n, Fp, f, lds, sgn + first, big ? n : f, true)) {
    if (tid == 0) atomicOr(err, 64);
  }
  if (big) return;
  double *Wp = W + fd.w_off[p];
  wg_set_identity(n, Wp, n);
  wg_trsm_lower(n, n, Fp, f, Wp, n, lds, true);
  double *Qp = Q + fd.q_off[p];
  if (m > 0) wg_gemm<false, false>(m, n, n, 1.0, Fp + n, f, Wp, n, 0.0, Qp, m, lds);
  double *R = FR + fd.r_off[p];
  double *C = BC + fd.r_off[p];
  const int64_t tri = (int64_t)n * (n + 1) / 2;
  // packing: wave per column c, lanes down the rows r >= c (then the m rows of Q)
  for (int c = wv; c < n; c += NW) {
    double *Cc = C + (int64_t)c * f - (int64_t)c * (c - 1) / 2;
    for (int r = c + lane; r < n; r += 64) {
      const double v = Wp[r + (size_t)c * n];
      R[(int64_t)r * (r + 1) / 2 + c] = v;
      Cc[r - c] = v;
    }
    for (int k = lane; k < m; k += 64) {
      const double v = Qp[k + (size_t)c * m];
      R[tri + (int64_t)k * n + c] = v;
      Cc[(n - c) + k] = v;
    }
  }
}

// The rest of k_front_factor for the large fronts, over many workgroups.
// k_front_inv: columns [c0, c0 + KB) of W = L_PP^{-1} (item (front, c0)):
// the rows above c0 are zero, the rest solve the trailing triangle against
// the identity columns; with c0 a multiple of KB the blocks line up with those
// of the single-workgroup solve, so every column sees the same operations.
__global__ __launch_bounds__(256, 2) void k_front_inv(DevFronts fd, const int4 *__restrict__ items,
                                                      const double *__restrict__ F, double *W) {
  __shared__ double lds[LDS_DOUBLES];
  const int4 it = items[blockIdx.x];
  const int p = it.x, c0 = it.y;
  const int n = fd.n[p], m = fd.m[p], f = n + m;
  const int nc = min(KB, n - c0);
  const double *Fp = F + fd.F_off[p];
  double *Wp = W + fd.w_off[p];
  for (int e = threadIdx.x; e < n * nc; e += WG) {
    const int r = e % n, c = c0 + e / n;
    Wp[r + (size_t)c * n] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_trsm_lower(n - c0, nc, Fp + c0 + (size_t)c0 * f, f, Wp + c0 + (size_t)c0 * n, n, lds, true);
}

// k_front_rows: the B rows [n + r0, n + r0 + 64) of L_BP (item (front, r0)).
__global__ __launch_bounds__(256, 2) void k_front_rows(DevFronts fd, const int4 *__restrict__ items,
                                                       const double *__restrict__ sgn, double *F) {
  __shared__ double lds[LDS_DOUBLES];
  const int4 it = items[blockIdx.x];
  const int p = it.x;
  const int n = fd.n[p], m = fd.m[p], f = n + m;
  const int ra = n + it.y, rb = min(ra + 64, f);
  wg_potrf_rows(n, F + fd.F_off[p], f, lds, sgn + fd.first[p], ra, rb);
}

// k_front_q: one 64 x 64 tile (front, i0, j0) of Q = L_BP W (m x n).
__global__ __launch_bounds__(256) void k_front_q(DevFronts fd, const int4 *__restrict__ tiles,
                                                 const double *__restrict__ F, const double *__restrict__ W,
                                                 double *Q) {
  __shared__ double lds[2 * KT * TILE];
  const int4 t = tiles[blockIdx.x];
  const int p = t.x;
  const int n = fd.n[p], m = fd.m[p], f = n + m;
  const double *Fp = F + fd.F_off[p];
  wg_gemm_tile<false, false>(t.y, t.z, m, n, n, 1.0, Fp + n, f, W + fd.w_off[p], n, 0.0, Q + fd.q_off[p], m, lds,
                             nullptr);
}

// k_front_pack: columns [c0, c0 + 64) of R (item (front, c0)), packed as in
// k_front_factor: a wave per column, lanes down the rows.
__global__ __launch_bounds__(256) void k_front_pack(DevFronts fd, const int4 *__restrict__ items,
                                                    const double *__restrict__ W, const double *__restrict__ Q,
                                                    double *FR, double *BC) {
  const int4 it = items[blockIdx.x];
  const int p = it.x;
  const int n = fd.n[p], m = fd.m[p], f = n + m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double *Wp = W + fd.w_off[p], *Qp = Q + fd.q_off[p];
  double *R = FR + fd.r_off[p], *C = BC + fd.r_off[p];
  const int64_t tri = (int64_t)n * (n + 1) / 2;
  for (int c = it.y + wv; c < min(it.y + 64, n); c += 4) {
    double *Cc = C + (int64_t)c * f - (int64_t)c * (c - 1) / 2;
    for (int r = c + lane; r < n; r += 64) {
      const double v = Wp[r + (size_t)c * n];
      R[(int64_t)r * (r + 1) / 2 + c] = v;
      Cc[r - c] = v;
    }
    for (int k = lane; k < m; k += 64) {
      const double v = Qp[k + (size_t)c * m];
      R[tri + (int64_t)k * n + c] = v;
      Cc[(n - c) + k] = v;
    }
  }
}

// The update matrices of one level's fronts, U = F_BB - L_BP diag(s_P) L_BP^T,
// one 64 x 64 tile of a lower triangle per workgroup; tiles[b] = (front,
// first row, first column).  Large fronts near the root get as many
// workgroups as they have tiles instead of one.
__global__ __launch_bounds__(256) void k_front_schur(DevFronts fd, const int4 *__restrict__ tiles,
                                                     const double *__restrict__ sgn, double *F) {
  __shared__ double lds[2 * KT * TILE];
  const int4 t = tiles[blockIdx.x];
  const int p = t.x;
  const int n = fd.n[p], m = fd.m[p], f = n + m;
  double *Fp = F + fd.F_off[p];
  const double *X = Fp + n;                 // L_BP, m x n, ld f
  wg_gemm_tile<false, true, true>(t.y, t.z, m, m, n, -1.0, X, f, X, f, 1.0, Fp + n + (size_t)n * f, f, lds,
                                  sgn + fd.first[p]);
}

// Several right-hand sides of the coarse solve at once (the columns of
// S_t^{-1} at setup, the block CG's coarse solves): the forward and backward
// sweep tasks of coarse.hip for TOP_NC columns per workgroup, so that each
// entry of R is read once per TOP_NC columns.  Every column's sums run in the
// order of the single-column tasks (same results).  Columns are stored one
// after the other (strides sk, sv, sb); done: optional stop flag.  With stage
// set, each task first stages its columns' inputs in LDS (dynamic: TOP_NC
// times the level's largest n_p forward, n_p + m_p backward), so that the
// lane groups do not reload them row after row (the same values).
constexpr int TOP_NC = 4;

__global__ __launch_bounds__(256) void k_top_fwd_cols(int t0, DevSweep sw, const double *__restrict__ FR,
                                                      const double *__restrict__ b, double *S0, double *S1,
                                                      double *__restrict__ z, int64_t sk, int64_t sv, int ncols,
                                                      const int *done, int stage) {
  extern __shared__ double tl[];   // with stage: t_p of the task's columns, [TOP_NC][nt]
  const int4 *td = sw.task + 4 * (int64_t)(t0 + blockIdx.x);
  const int4 d0 = td[0], d1 = td[1], d2 = td[2];
  if (done && *done) return;
  const int c0 = blockIdx.y * TOP_NC, nq = min(TOP_NC, ncols - c0);
  const int g = d0.z, n = d0.w, m = d1.x, fst = d1.y, vo = d1.z, bo = d1.w;
  const int64_t ro = (int64_t)(((uint64_t)(uint32_t)d2.y << 32) | (uint32_t)d2.x);
  // the task's rows read t_p up to its last own row (all n with a B row)
  const int nt = min(n, d0.y + 256 / g);
  if (stage) {
    for (int e = threadIdx.x; e < nq * nt; e += 256) {
      const int q = e / nt, c = e - q * nt;
      const int64_t o = c0 + q;
      tl[e] = (b[o * sk + fst + c] + S0[o * sv + vo + c]) + S1[o * sv + vo + c];
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & (g - 1), r = d0.y + threadIdx.x / g;
  if (r >= n + m) return;            // whole lane groups leave together
  const double *row;
  int len;
  if (r < n) {
    row = FR + ro + (int64_t)r * (r + 1) / 2;
    len = r + 1;
  } else {
    row = FR + ro + (int64_t)n * (n + 1) / 2 + (int64_t)(r - n) * n;
    len = n;
  }
  double base[TOP_NC] = {};
  int dst = 0;
  if (r >= n && lane == 0) {
    for (int q = 0; q < nq; ++q) {
      const int64_t o = c0 + q;
      base[q] = S0[o * sv + vo + r] + S1[o * sv + vo + r];
    }
    dst = sw.wdst[bo + (r - n)];
  }
  double a[TOP_NC][4] = {};
  for (int e0 = lane; e0 < len; e0 += 4 * g) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = e0 + u * g;
      if (c < len) {
        const double rv = row[c];
#pragma unroll
        for (int q = 0; q < TOP_NC; ++q)
          if (q < nq) {
            const int64_t o = c0 + q;
            const double t = stage ? tl[q * nt + c] : (b[o * sk + fst + c] + S0[o * sv + vo + c]) + S1[o * sv + vo + c];
            a[q][u] = fma(rv, t, a[q][u]);
          }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < TOP_NC; ++q) {
    const double s = group_reduce((a[q][0] + a[q][1]) + (a[q][2] + a[q][3]), g);
    if (q < nq && lane == 0) {
      const int64_t o = c0 + q;
      if (r < n) z[o * sk + fst + r] = s;
      else (d2.z ? S1 : S0)[o * sv + dst] = base[q] - s;
    }
  }
}

__global__ __launch_bounds__(256) void k_top_bwd_cols(int t0, DevSweep sw, const double *__restrict__ BC,
                                                      const double *__restrict__ z, const double *__restrict__ sg,
                                                      double *XB, double *__restrict__ x, int64_t sk, int64_t sb,
                                                      int ncols, const int *done, int stage) {
  extern __shared__ double vl[];   // with stage: the task's inputs, [TOP_NC][n + m - first column]
  const int4 *td = sw.task + 4 * (int64_t)(t0 + blockIdx.x);
  const int4 d0 = td[0], d1 = td[1], d2 = td[2];
  if (done && *done) return;
  const int c0 = blockIdx.y * TOP_NC, nq = min(TOP_NC, ncols - c0);
  const int g = d0.z, n = d0.w, m = d1.x, fst = d1.y, bo = d1.w;
  const int64_t ro = (int64_t)(((uint64_t)(uint32_t)d2.y << 32) | (uint32_t)d2.x);
  // columns c >= cl read s z from own dof c on, then -x_B
  const int cl = d0.y, W = n + m - cl;
  if (stage) {
    for (int e = threadIdx.x; e < nq * W; e += 256) {
      const int k = e / W, q = cl + (e - k * W);
      const int64_t o = c0 + k;
      vl[e] = q < n ? sg[fst + q] * z[o * sk + fst + q] : -XB[o * sb + bo + (q - n)];
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & (g - 1), c = cl + threadIdx.x / g;
  if (c >= n) return;
  const int f = n + m, d = fst + c;
  const int s0 = sw.xsc_off[d], s1 = sw.xsc_off[d + 1];
  const double *col = BC + ro + (int64_t)c * f - (int64_t)c * (c - 1) / 2;
  const int nl = n - c, len = nl + m;
  double a[TOP_NC][4] = {};
  for (int e0 = lane; e0 < len; e0 += 4 * g) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = e0 + u * g;
      if (q < len) {
        const double cv = col[q];
#pragma unroll
        for (int k = 0; k < TOP_NC; ++k)
          if (k < nq) {
            const int64_t o = c0 + k;
            const double in = stage ? vl[k * W + (c - cl) + q]
                                    : (q < nl ? sg[d + q] * z[o * sk + d + q] : -XB[o * sb + bo + (q - nl)]);
            a[k][u] = fma(cv, in, a[k][u]);
          }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < TOP_NC; ++k) {
    const double s = group_reduce((a[k][0] + a[k][1]) + (a[k][2] + a[k][3]), g);
    if (k < nq) {
      const int64_t o = c0 + k;
      if (lane == 0) x[o * sk + d] = s;
      for (int j = s0 + lane; j < s1; j += g) XB[o * sb + sw.xsc[j]] = s;
    }
  }
}

}  // namespace bddc
