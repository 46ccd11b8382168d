// Coarse saddle point of Algorithm "BDDC preconditioner" (step 1 of the
// preconditioner and step 1 of Algorithm "BDDC method"), factored by a
// multifrontal signed Cholesky K = L diag(s) L^T over the nested-dissection
// fronts of nd.hpp (s = +1 on face dofs, -1 on pressures).
//
// The fronts are assembled and factored at setup (front.hip); the stored
// per-front R = [L_PP^{-1}; L_BP L_PP^{-1}] is applied here.
//
// Solve (a front's results go straight into contiguous vectors of the fronts
// that read them next; one launch per level and direction):
//   forward, from the leaves: t_p = b_P + S0_p[P] + S1_p[P], where S0 / S1 hold
//     the updates pushed by children 0 / 1 at their positions in [P, B(p)];
//     z_P = L_PP^{-1} t_p and w_p = S0_p[B] + S1_p[B] - L_BP L_PP^{-1} t_p,
//     pushed into the parent's slot array of this child.
//   backward, from the root: x_P = L_PP^{-T} s_P z_P - (L_BP L_PP^{-1})^T x_B,
//     where x_B (the front's B vector) was filled by the ancestors: every x[d]
//     is stored into all B vectors that hold d as soon as it is computed.
// A row (column) of R is handled by a group of g = 4, 16 or 64 lanes chosen
// from its length, so short rows do not leave lanes idle.
#include "common.hpp"
#include "dense.hpp"

namespace bddc {

struct DevSweep {
  const int *wdst;                 // forward push target of every B row
  const int *xsc_off, *xsc;        // backward: B-vector positions holding x[d]
  const int4 *task;                // four int4 per task (nd.hpp)
  int nfr;                         // fronts
};

// ---- per-solve sweeps --------------------------------------------------------
template <int W>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

__device__ __forceinline__ double group_reduce(double v, int g) {
  if (g == 64) return group_sum<64>(v);
  if (g == 16) return group_sum<16>(v);
  if (g == 4) return group_sum<4>(v);
  return v;
}

// Rows [d0.y, d0.y + 256/g) of one front, forward: each lane group of g
// lanes forms one row of R against t_p; rows r < n give z_P[r], rows n + k
// push w_p[k] into the parent's slot array of this front.  Called by 256
// lanes (tid = 0 .. 255, whole wavefronts).
// tl: t_p staged in LDS by the caller (the whole task's workgroup), or null:
// each lane group forms the t_p entries it needs from b, S0 and S1 (the same
// sums, so the same bits).  A single lane (g = 1) takes a row with eight
// independent loads in flight.
__device__ __forceinline__ void fwd_task(const int4 d0, const int4 d1, const int4 d2, const DevSweep &sw,
                                         const double *__restrict__ FR, const double *__restrict__ b, double *S0,
                                         double *S1, double *z, int tid, const double *tl = nullptr) {
  const int g = d0.z, n = d0.w, m = d1.x, fst = d1.y, vo = d1.z, bo = d1.w;
  const int64_t ro = (int64_t)(((uint64_t)(uint32_t)d2.y << 32) | (uint32_t)d2.x);
  const int lane = tid & (g - 1), r = d0.y + tid / g;
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
  double base = 0.0;
  int dst = 0;
  if (r >= n && lane == 0) {
    base = S0[vo + r] + S1[vo + r];
    dst = sw.wdst[bo + (r - n)];
  }
  double s;
  if (g == 1) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < len; c0 += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u;
        if (c < len) a[u] = fma(row[c], tl ? tl[c] : (b[fst + c] + S0[vo + c]) + S1[vo + c], a[u]);
      }
    }
    s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  } else {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = lane; c0 < len; c0 += 4 * g) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * g;
        if (c < len) {
          const double t = tl ? tl[c] : (b[fst + c] + S0[vo + c]) + S1[vo + c];
          a[u] = fma(row[c], t, a[u]);
        }
      }
    }
    s = group_reduce((a[0] + a[1]) + (a[2] + a[3]), g);
  }
  if (lane == 0) {
    if (r < n) z[fst + r] = s;
    else (d2.z ? S1 : S0)[dst] = base - s;
  }
}

// Columns [d0.y, d0.y + 256/g) of one front, backward; each x[d] is also
// stored into every B vector that holds d (those of the fronts below), and
// the right-hand side b[d], consumed by the forward sweep, is cleared for the
// next solve.  Called by 256 lanes (tid = 0 .. 255, whole wavefronts).
// vl: the task's input staged in LDS by the caller (sg z over the front's own
// dofs, then -x_B), or null: read from z, sg and XB as needed.
__device__ __forceinline__ void bwd_task(const int4 d0, const int4 d1, const int4 d2, const DevSweep &sw,
                                         const double *__restrict__ BC, const double *z,
                                         const double *__restrict__ sg, double *XB, double *__restrict__ x,
                                         double *__restrict__ b, int tid, const double *vl = nullptr) {
  const int g = d0.z, n = d0.w, m = d1.x, fst = d1.y, bo = d1.w;
  const int64_t ro = (int64_t)(((uint64_t)(uint32_t)d2.y << 32) | (uint32_t)d2.x);
  const int lane = tid & (g - 1), c = d0.y + tid / g;
  const double *xb = XB + bo;
  if (c >= n) return;
  const int f = n + m, d = fst + c;
  const int s0 = sw.xsc_off[d], s1 = sw.xsc_off[d + 1];
  const double *col = BC + ro + (int64_t)c * f - (int64_t)c * (c - 1) / 2;
  const int nl = n - c, len = nl + m;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q0 = lane; q0 < len; q0 += 4 * g) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u * g;
      if (q < len) {
        const double in = vl ? vl[c + q] : (q < nl ? sg[d + q] * z[d + q] : -xb[q - nl]);
        a[u] = fma(col[q], in, a[u]);
      }
    }
  }
  const double s = group_reduce((a[0] + a[1]) + (a[2] + a[3]), g);
  if (lane == 0) {
    x[d] = s;
    b[d] = 0.0;
  }
  for (int k = s0 + lane; k < s1; k += g) XB[sw.xsc[k]] = s;
}

// Level-synchronous sweeps: the tasks [t0, t0 + gridDim.x) of one level, one
// per workgroup; kernel boundaries order the levels.  The task descriptor is
// read before the CG stop flag, so that the two loads are in flight together
// (a level is a few dependent memory round trips long).
// With stage set, the level kernels stage the task's input vector in LDS
// (dynamic, at least the largest n_p (forward) or n_p + m_p (backward) of the
// level's fronts), so that each entry is loaded once per task rather than once
// per row; the same sums and products, so the same bits.
__global__ __launch_bounds__(256) void k_nd_fwd(int t0, DevSweep sw, const double *__restrict__ FR,
                                                const double *__restrict__ b, double *S0, double *S1,
                                                double *__restrict__ z, const int *done, int stage) {
  __builtin_amdgcn_s_setprio(3);   // the coarse chain is the apply's critical path
  extern __shared__ double tl[];
  const int4 *td = sw.task + 4 * (int64_t)(t0 + blockIdx.x);
  const int4 d0 = td[0], d1 = td[1], d2 = td[2];
  if (done && *done) return;
  if (!stage) {
    fwd_task(d0, d1, d2, sw, FR, b, S0, S1, z, threadIdx.x);
    return;
  }
  const int n = d0.w, fst = d1.y, vo = d1.z;
  // rows [d0.y, d0.y + 256 / g) read t_p up to the last own row of the task
  const int nt = min(n, d0.y + 256 / d0.z);
  for (int c = threadIdx.x; c < nt; c += 256) tl[c] = (b[fst + c] + S0[vo + c]) + S1[vo + c];
  __syncthreads();
  fwd_task(d0, d1, d2, sw, FR, b, S0, S1, z, threadIdx.x, tl);
}

__global__ __launch_bounds__(256) void k_nd_bwd(int t0, DevSweep sw, const double *__restrict__ BC,
                                                const double *__restrict__ z, const double *__restrict__ sg,
                                                double *XB, double *__restrict__ x, double *__restrict__ b,
                                                const int *done, int stage) {
  __builtin_amdgcn_s_setprio(3);   // the coarse chain is the apply's critical path
  extern __shared__ double vl[];
  const int4 *td = sw.task + 4 * (int64_t)(t0 + blockIdx.x);
  const int4 d0 = td[0], d1 = td[1], d2 = td[2];
  if (done && *done) return;
  if (!stage) {
    bwd_task(d0, d1, d2, sw, BC, z, sg, XB, x, b, threadIdx.x);
    return;
  }
  // columns c >= d0.y read sg z from dof c on, then -x_B
  const int n = d0.w, m = d1.x, fst = d1.y, bo = d1.w, cl = d0.y;
  for (int q = cl + threadIdx.x; q < n + m; q += 256)
    vl[q] = q < n ? sg[fst + q] * z[fst + q] : -XB[bo + (q - n)];
  __syncthreads();
  bwd_task(d0, d1, d2, sw, BC, z, sg, XB, x, b, threadIdx.x, vl);
}

// Bottom subtrees (nd_subtrees), one per workgroup of SUB_Q x 256 lanes: the
// subtree's phases (levels) in order, each phase's tasks dealt to the SUB_Q
// groups of 256 lanes, with a workgroup barrier between phases.  What one
// phase writes (the pushes into the parents' slot arrays forward, the x values
// in the descendants' B vectors backward) is read by a later phase of the same
// workgroup, so the barrier orders it; no level launch boundary is paid inside
// the subtree.  ph: this subtree's nph + 1 phase offsets into the task copies.
constexpr int SUB_Q = 4;
constexpr int SUB_THREADS = 256 * SUB_Q;

__global__ __launch_bounds__(SUB_THREADS) void k_nd_fwd_sub(int nph, const int *__restrict__ sph,
                                                            const int4 *__restrict__ stask, DevSweep sw,
                                                            const double *__restrict__ FR,
                                                            const double *__restrict__ b, double *S0, double *S1,
                                                            double *__restrict__ z, const int *done) {
  if (done && *done) return;
  const int *ph = sph + (int64_t)blockIdx.x * (nph + 1);
  const int q = threadIdx.x >> 8, tid = threadIdx.x & 255;
  for (int k = 0; k < nph; ++k) {
    const int e = ph[k + 1];
    for (int t = ph[k] + q; t < e; t += SUB_Q) {
      const int4 *td = stask + 4 * (int64_t)t;
      fwd_task(td[0], td[1], td[2], sw, FR, b, S0, S1, z, tid);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(SUB_THREADS) void k_nd_bwd_sub(int nph, const int *__restrict__ sph,
                                                            const int4 *__restrict__ stask, DevSweep sw,
                                                            const double *__restrict__ BC,
                                                            const double *__restrict__ z,
                                                            const double *__restrict__ sg, double *XB,
                                                            double *__restrict__ x, double *__restrict__ b,
                                                            const int *done) {
  if (done && *done) return;
  const int *ph = sph + (int64_t)blockIdx.x * (nph + 1);
  const int q = threadIdx.x >> 8, tid = threadIdx.x & 255;
  for (int k = 0; k < nph; ++k) {
    const int e = ph[k + 1];
    for (int t = ph[k] + q; t < e; t += SUB_Q) {
      const int4 *td = stask + 4 * (int64_t)t;
      bwd_task(td[0], td[1], td[2], sw, BC, z, sg, XB, x, b, tid);
    }
    __syncthreads();
  }
}

// ---- dense top block (nd_dense_top) ---------------------------------------------
// t_t[j] = b[d0 + j] plus the updates the lower fronts pushed into the top
// fronts' vectors for that dof.
__global__ __launch_bounds__(256) void k_top_gather(int nt, int d0, const int *__restrict__ tg_off,
                                                    const int *__restrict__ tg, const double *__restrict__ b,
                                                    const double *__restrict__ S0, const double *__restrict__ S1,
                                                    double *__restrict__ tt, const int *done) {
  __builtin_amdgcn_s_setprio(3);   // the coarse chain is the apply's critical path
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nt) return;
  double v = b[d0 + j];
  const int q0 = tg_off[j], q1 = tg_off[j + 1];
  if (done && *done) return;
  for (int q = q0; q < q1; ++q) {
    const int p = tg[q];
    v += S0[p] + S1[p];
  }
  tt[j] = v;
}

// x_t = S_t^{-1} t_t for the rows [8 blockIdx.x, 8 blockIdx.x + 8): t_t is
// staged in LDS (ld doubles, zero padded), each wave forms two rows of the
// row-major inverse (leading dimension ld, even, so rows are 16-byte aligned)
// with 16-byte loads.  Each x[d] is also stored into every B vector holding d,
// for the backward sweep of the levels below, and b[d] (read by the gather
// before this launch) is cleared for the next solve.
constexpr int TOP_THREADS = 256;
constexpr int TOP_ROWS_PER_WG = 8;
constexpr int TOP_DEFAULT_DOFS = 4096;   // 128 MB of FP64 inverse at most
constexpr int TOP_MAX_DOFS = 8192;       // t_t in 64 KB of LDS

__global__ __launch_bounds__(TOP_THREADS) void k_top_gemv(int nt, int ld, const double *__restrict__ Kt,
                                                          const double *__restrict__ tt, int d0,
                                                          const int *__restrict__ xsc_off,
                                                          const int *__restrict__ xsc, double *__restrict__ XB,
                                                          double *__restrict__ x, double *__restrict__ b,
                                                          const int *done) {
  __builtin_amdgcn_s_setprio(3);   // the coarse chain is the apply's critical path
  extern __shared__ double tl[];
  for (int j = threadIdx.x; j < ld; j += TOP_THREADS) tl[j] = j < nt ? tt[j] : 0.0;
  __syncthreads();
  if (done && *done) return;
  const int lane = threadIdx.x & 63;
  const int r0 = blockIdx.x * TOP_ROWS_PER_WG + 2 * (threadIdx.x >> 6);
  if (r0 >= nt) return;
  const bool two = r0 + 1 < nt;
  const int ld2 = ld >> 1;
  const double2 *A0 = reinterpret_cast<const double2 *>(Kt + (int64_t)r0 * ld);
  const double2 *A1 = two ? A0 + ld2 : A0;
  const double2 *T = reinterpret_cast<const double2 *>(tl);
  double a0 = 0.0, c0 = 0.0, a1 = 0.0, c1 = 0.0;
  int k = lane;
  for (; k + 192 < ld2; k += 256) {
    double2 u[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u[q] = A0[k + 64 * q];
      v[q] = A1[k + 64 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 t = T[k + 64 * q];
      a0 = fma(u[q].x, t.x, a0);
      c0 = fma(u[q].y, t.y, c0);
      a1 = fma(v[q].x, t.x, a1);
      c1 = fma(v[q].y, t.y, c1);
    }
  }
  for (; k < ld2; k += 64) {
    const double2 u = A0[k], v = A1[k], t = T[k];
    a0 = fma(u.x, t.x, a0);
    c0 = fma(u.y, t.y, c0);
    a1 = fma(v.x, t.x, a1);
    c1 = fma(v.y, t.y, c1);
  }
  const double s0 = group_sum<64>(a0 + c0), s1 = group_sum<64>(a1 + c1);
  const int d = d0 + r0;
  if (lane == 0) {
    x[d] = s0;
    b[d] = 0.0;
    if (two) {
      x[d + 1] = s1;
      b[d + 1] = 0.0;
    }
  }
  for (int q = xsc_off[d] + lane; q < xsc_off[d + 1]; q += 64) XB[xsc[q]] = s0;
  if (two)
    for (int q = xsc_off[d + 1] + lane; q < xsc_off[d + 2]; q += 64) XB[xsc[q]] = s1;
}

// Setup of S_t^{-1}, gridDim.y columns [j0, j0 + gridDim.y) at a time: each
// column c has its own copies of the sweep vectors (strides sk for dof
// vectors, sv for front vectors, sb for B vectors), its top right-hand side
// is the unit vector of dof j0 + c and the top fronts' vectors [v0, v1) start
// cleared; the sweeps of the top levels then leave column j0 + c of S_t^{-1}
// in the top part of x.
__global__ __launch_bounds__(256) void k_top_unit(int j0, int nt, int d0, int64_t sk, int64_t v0, int64_t v1,
                                                  int64_t sv, double *__restrict__ b, double *__restrict__ S0,
                                                  double *__restrict__ S1) {
  const int64_t c = blockIdx.y;
  const int64_t len = std::max<int64_t>(nt, v1 - v0);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
    if (i < nt) b[c * sk + d0 + i] = (i == j0 + c) ? 1.0 : 0.0;
    if (i < v1 - v0) {
      S0[c * sv + v0 + i] = 0.0;
      S1[c * sv + v0 + i] = 0.0;
    }
  }
}

__global__ __launch_bounds__(256) void k_top_store(int j0, int nt, int d0, int ld, const double *__restrict__ x,
                                                   int64_t sk, double *__restrict__ Kt) {
  const int64_t c = blockIdx.y;
  const double *xc = x + c * sk + d0;
  double *row = Kt + (int64_t)(j0 + c) * ld;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < ld; i += gridDim.x * 256) row[i] = i < nt ? xc[i] : 0.0;
}

}  // namespace bddc
