// Solve kernels: Algorithm "BDDC method" steps 1-3 on the device.
//
// Step 3 is conjugate gradients on the interface saddle point of eqs.
// corr-reduced-1/2 in the balanced subspace: the operator is
// (S x_u + B_0^T x_p, B_0 x_u), the preconditioner is Algorithm "BDDC
// preconditioner" (restriction with multiplicity weights 1/2, local
// substructure correction T^i, coarse correction through Psi^i and the coarse
// saddle point, averaging E).  The flux iterates stay balanced, so the
// pressure component of the residual stays zero and is not stored.
//
// Reductions are deterministic: every producer writes one partial per block,
// every consumer block re-adds the partials in the same fixed order.
#include "common.hpp"
#include "dense.hpp"

namespace bddc {

struct CgState {
  double rho, rho_next, r0sq, rtol2, relres;
  int it;        // iterations whose updates are complete and advanced
  int nupd;      // x/r updates performed
  int done;      // stop flag read by every kernel of the loop
  int converged;
  int fail;      // 1: breakdown
  int maxit;
  int pending;   // 1: rho = rho_next and it += 1 still to do (left by the p update)
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum four per-lane values over the 64 lanes at once: after the exchange
// with lane^32 and lane^16 each 16-lane group holds one of the four partial
// sums, which four more steps finish.  Lane 16*q returns the total of d[q].
__device__ __forceinline__ double transpose_reduce4(const double *d, int lane) {
  const bool hi32 = (lane & 32) != 0;
  double v0 = hi32 ? d[2] : d[0], v1 = hi32 ? d[3] : d[1];
  const double w0 = hi32 ? d[0] : d[2], w1 = hi32 ? d[1] : d[3];
  v0 += __shfl_xor(w0, 32, 64);
  v1 += __shfl_xor(w1, 32, 64);
  const bool hi16 = (lane & 16) != 0;
  double u = hi16 ? v1 : v0;
  const double o = hi16 ? v0 : v1;
  u += __shfl_xor(o, 16, 64);
  for (int off = 8; off > 0; off >>= 1) u += __shfl_xor(u, off, 64);
  return u;
}

__device__ __forceinline__ double block_sum_partials(const double *__restrict__ part, int n, double *red) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) s += part[k];
  s = wave_sum(s);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = s;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
  __syncthreads();
  return t;
}

// Kernels that leave one partial per block for a dot product run on at most
// PART_BLOCKS blocks (grid-stride loops), so that every block of the kernel
// that needs the total can add the partials up cheaply.
constexpr int PART_BLOCKS = 512;

__device__ __forceinline__ void block_write_partial(double v, double *part, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    part[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Local symmetric operators y^i = M^i (xscale R^i x) with M^i in the
// group-aligned packed lower storage of common.hpp.  Each wave streams column
// groups (coalesced 16-byte loads), accumulating the strictly-lower product in
// its own LDS row buffer and the transposed product by a wave reduction.  With
// residual partials given, the first kernel of the preconditioner evaluates the
// stopping test before any work.
// ---------------------------------------------------------------------------
// 16-byte vector load of 16/sizeof(TS) consecutive entries, widened to FP64.
// The local operators and bases are read once per application and are far
// larger than the caches: their loads are marked non-temporal, so that they do
// not push out of the L2s and the Infinity Cache the data that is read again
// (the coarse factor, the sweep descriptors and the interface vectors).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load16(const float *p, double *o) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
  o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ __forceinline__ void load16(const double *p, double *o) {
  const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
  o[0] = v[0]; o[1] = v[1];
}

// The same 16 bytes kept in their storage type (widened at use), for kernels
// that hold many loads in flight.
template <typename TS> struct Raw16;
template <> struct Raw16<float> {
  f32x4 v;
  __device__ __forceinline__ double operator[](int i) const { return v[i]; }
};
template <> struct Raw16<double> {
  f64x2 v;
  __device__ __forceinline__ double operator[](int i) const { return v[i]; }
};
template <typename TS>
__device__ __forceinline__ Raw16<TS> load_raw16(const TS *p) {
  Raw16<TS> r;
  r.v = __builtin_nontemporal_load(reinterpret_cast<const decltype(r.v) *>(p));
  return r;
}

// Convergence test at the head of the first kernel of the preconditioner:
// ||r||^2 from the partials of the residual update decides whether the CG
// stops here.  Returns true when the calling kernel must leave.
__device__ __forceinline__ bool cg_exit(CgState *st, const double *__restrict__ rpart, int nrpart, double *red) {
  if (!st) return false;
  if (st->done) return true;
  if (!rpart) return false;
  const double rn2 = block_sum_partials(rpart, nrpart, red);
  const bool conv = rn2 <= st->rtol2 * st->r0sq;
  const bool cap = st->nupd >= st->maxit;
  if (conv || cap || !isfinite(rn2)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->done = 1;
      st->converged = conv ? 1 : 0;
      st->relres = st->r0sq > 0.0 ? sqrt(rn2 / st->r0sq) : 0.0;
      if (!isfinite(rn2)) st->fail = 1;
    }
    return true;
  }
  return false;
}

// y^i = M^i (w * R_i x), w = xw (per local dof) or xscale, for every subdomain (one workgroup of SYMV_WAVES
// wavefronts each), M^i in group-aligned packed storage (S^i, or T^i of the
// preconditioner).  Eight waves per workgroup: with one subdomain per
// workgroup the launch is about three rounds of resident workgroups on 256
// CUs for the 2,244 subdomains of the reservoir, so the last round is nearly
// full (four waves left it half empty).
constexpr int SYMV_WAVES = 8;
constexpr int SYMV_THREADS = 64 * SYMV_WAVES;

template <typename TS>
__global__ __launch_bounds__(SYMV_THREADS) void k_symv(DevGeom g, const TS *__restrict__ M,
                                                       const int64_t *__restrict__ pk,
                                                       const double *__restrict__ x, double xscale,
                                                       const double *__restrict__ xw,
                                                       double *__restrict__ yloc, CgState *st,
                                                       const double *__restrict__ rpart, int nrpart) {
  extern __shared__ double sh[];
  __shared__ double red[SYMV_WAVES];
  if (cg_exit(st, rpart, nrpart, red)) return;
  constexpr int VW = 16 / sizeof(TS);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // subdomains blockIdx.x, blockIdx.x + gridDim.x, ... (one each with a full grid)
  for (int i = blockIdx.x; i < g.N; i += gridDim.x) {
    const int n = g.nG[i];
    const int G4 = (n + 3) / 4, np = 4 * G4;
    const int64_t go = g.g_off[i];
    double *xs = sh;
    double *yw = sh + np;
    for (int r = tid; r < np; r += SYMV_THREADS) xs[r] = (r < n) ? (xw ? xw[go + r] : xscale) * x[g.Rmap[go + r]] : 0.0;
    for (int e = tid; e < SYMV_WAVES * np; e += SYMV_THREADS) yw[e] = 0.0;
    __syncthreads();
    const TS *Mi = M + pk[i];
    double *yme = yw + wv * np;
    // A wave takes one column group (four columns, common first row rs) at a
    // time: each lane loads VW consecutive rows of all four columns with 16-byte
    // loads, folds the strictly-lower products into one LDS update per row, and
    // the four transposed dot products are reduced together.
    for (int gi = wv; gi < G4; gi += SYMV_WAVES) {
      const int rs = 4 * gi;
      const int L = 4 * (G4 - gi);
      const TS *base = Mi + gp_group(n, gi);
      double xj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xj[q] = xs[rs + q];
      double d[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = lane * VW; t < L; t += 64 * VW) {
        double a[4][VW];
#pragma unroll
        for (int q = 0; q < 4; ++q) load16(base + (int64_t)q * L + t, a[q]);
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          const int r = rs + t + v;
          const double xr = xs[r];
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            d[q] = fma(a[q][v], xr, d[q]);
            if (r > rs + q) acc = fma(a[q][v], xj[q], acc);
          }
          yme[r] += acc;
        }
      }
      const double tot = transpose_reduce4(d, lane);
      if ((lane & 15) == 0) yme[rs + (lane >> 4)] += tot;
    }
    __syncthreads();
    for (int r = tid; r < n; r += SYMV_THREADS) {
      double y = 0.0;
#pragma unroll
      for (int w = 0; w < SYMV_WAVES; ++w) y += yw[w * np + r];
      yloc[go + r] = y;
    }
    __syncthreads();   // LDS is reused by the next subdomain
  }
}


// g^i = Psi^{iT} (w * R_i x), w = xw or xscale: the coarse right-hand side pieces of the
// preconditioner (one workgroup per subdomain; four columns per wave, 16-byte
// loads over the ld4-padded columns), added straight into the coarse
// right-hand side b at the coarse dofs (sub_cmap).  A face's coarse dof gets
// the pieces of its two subdomains, b must be zero there on entry (the coarse
// solve clears b as it consumes it), and the sum of two values onto zero is
// the same in either order; the pressure rows of b stay zero.
template <typename TS>
__global__ __launch_bounds__(256) void k_psi_apply(DevGeom g, const TS *__restrict__ Psi,
                                                   const int64_t *__restrict__ psi_off,
                                                   const int *__restrict__ sub_coff, const int *__restrict__ sub_cmap,
                                                   const double *__restrict__ x, double xscale,
                                                   const double *__restrict__ xw, double *__restrict__ b, CgState *st,
                                                   const double *__restrict__ rpart, int nrpart) {
  extern __shared__ double sh[];
  __shared__ double red[8];
  if (cg_exit(st, rpart, nrpart, red)) return;
  constexpr int VW = 16 / sizeof(TS);
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = g.nG[i], np = ld4(n);
  const int64_t go = g.g_off[i];
  double *xs = sh;
  for (int r = tid; r < np; r += 256) xs[r] = (r < n) ? (xw ? xw[go + r] : xscale) * x[g.Rmap[go + r]] : 0.0;
  __syncthreads();
  const int c0 = sub_coff[i], nci = sub_coff[i + 1] - c0;
  const TS *P = Psi + psi_off[i];
  // eight columns per wave and round: sixteen 16-byte loads per lane in flight
  // for two row steps, then two four-column transposed reductions
  for (int cb = 8 * wv; cb < nci; cb += 32) {
    double d[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = lane * VW; t < np; t += 64 * VW) {
      Raw16<TS> a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (cb + q < nci) a[q] = load_raw16(P + (int64_t)(cb + q) * np + t);
        else a[q].v = {};
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) d[q] = fma(a[q][v], xs[t + v], d[q]);
    }
    const double tot0 = transpose_reduce4(d, lane);
    const double tot1 = transpose_reduce4(d + 4, lane);
    if ((lane & 15) == 0) {
      const int c = cb + (lane >> 4);
      if (c < nci) atomicAdd(b + sub_cmap[c0 + c], tot0);
      if (c + 4 < nci) atomicAdd(b + sub_cmap[c0 + c + 4], tot1);
    }
  }
}

// q = assembled local products + B_0^T x_p;  partial of p_u . q
__global__ __launch_bounds__(256) void k_sys_assemble(DevGeom g, const double *__restrict__ yloc,
                                                      const double *__restrict__ xp,
                                                      const double *__restrict__ dscale,
                                                      const double *__restrict__ pu, double *__restrict__ q,
                                                      double *part, CgState *st) {
  __shared__ double red[8];
  if (st && st->done) return;
  // the state advance of the previous p update: no block of this kernel or of
  // the S^i products before it reads rho or the iteration count
  if (st && blockIdx.x == 0 && threadIdx.x == 0 && st->pending) {
    st->rho = st->rho_next;
    st->it += 1;
    st->pending = 0;
  }
  double v = 0.0;
  for (int gi = blockIdx.x * 256 + threadIdx.x; gi < g.nGamma; gi += gridDim.x * 256) {
    const int sm = g.sub_minus[gi], sp = g.sub_plus[gi];
    double b0 = 0.0;
    if (xp) b0 = -dscale[sm] * xp[sm] + dscale[sp] * xp[sp];
    const double qq = yloc[g.own_minus[gi]] + yloc[g.own_plus[gi]] + b0;
    q[gi] = qq;
    if (pu) v = fma(pu[gi], qq, v);
  }
  if (part) block_write_partial(v, part, red);
}

// alpha = rho / (p.q); x += alpha p; r -= alpha q; partial of r.r
__global__ __launch_bounds__(256) void k_update_xr(int nGamma, int N, const double *__restrict__ gpart,
                                                   int ngpart, const double *__restrict__ pu,
                                                   const double *__restrict__ q, const double *__restrict__ pp,
                                                   double *xu, double *ru, double *xp, double *rpart,
                                                   CgState *st, double *alpha_hist) {
  __shared__ double red[8];
  if (st->done) return;
  const double gam = block_sum_partials(gpart, ngpart, red);
  if (!(gam > 0.0) || !isfinite(gam)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->fail = 1;
      st->done = 1;
    }
    return;
  }
  const double alpha = st->rho / gam;
  double v = 0.0;
  for (int gi = blockIdx.x * 256 + threadIdx.x; gi < nGamma; gi += gridDim.x * 256) {
    xu[gi] = fma(alpha, pu[gi], xu[gi]);
    const double r = fma(-alpha, q[gi], ru[gi]);
    ru[gi] = r;
    v = fma(r, r, v);
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < N; k += 256) xp[k] = fma(alpha, pp[k], xp[k]);
    if (threadIdx.x == 0) {
      alpha_hist[st->it] = alpha;
      st->nupd = st->it + 1;
    }
  }
  block_write_partial(v, rpart, red);
}

// w^i = y^i + Psi^i alpha^(i)  (y may be null: w^i = Psi^i alpha^(i)).  Each lane owns 16-byte row
// chunks of the ld4-padded columns (VW rows), the four waves split the
// columns, and the partial sums meet in LDS; a lane keeps a dozen independent
// 16-byte loads in flight.
template <typename TS>
__global__ __launch_bounds__(256) void k_psi_correct(DevGeom g, DevCoarse cs, const TS *__restrict__ Psi,
                                                     const int64_t *__restrict__ psi_off,
                                                     const double *__restrict__ yloc,
                                                     const double *__restrict__ csol, double *__restrict__ wloc,
                                                     const CgState *st) {
  constexpr int VW = 16 / sizeof(TS);
  constexpr int RB = 64 * VW;        // rows per block
  __shared__ double al[1024];
  __shared__ double part[4 * RB];
  const int i = blockIdx.x;
  const int n = g.nG[i];
  const int64_t go = g.g_off[i];
  const int c0 = cs.sub_coff[i], nci = cs.sub_coff[i + 1] - c0;
  if (st && st->done) return;   // read beside the subdomain's sizes
  for (int c = threadIdx.x; c < nci; c += 256) al[c] = csol[cs.sub_cmap[c0 + c]];
  __syncthreads();
  const TS *P = Psi + psi_off[i];
  const int ldp = ld4(n);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int rb = 0; rb < n; rb += RB) {
    const int r0 = rb + lane * VW;
    double acc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = 0.0;
    if (r0 < ldp) {
#pragma unroll 4
      for (int c = wv; c < nci; c += 4) {
        double a[VW];
        load16(P + (int64_t)c * ldp + r0, a);
        const double ac = al[c];
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] = fma(a[v], ac, acc[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < VW; ++v) part[wv * RB + lane * VW + v] = acc[v];
    __syncthreads();
    for (int r = threadIdx.x; r < RB && rb + r < n; r += 256) {
      const double s = (part[r] + part[RB + r]) + (part[2 * RB + r] + part[3 * RB + r]);
      wloc[go + rb + r] = (yloc ? yloc[go + rb + r] : 0.0) + s;
    }
    __syncthreads();
  }
}

// z = E w (weights 1/2) with w = y + wloc (y may be null: w = wloc), then
// each face total is set to the face's zero-net-flux coarse dof (a no-op in
// exact arithmetic, since C^i T^i = 0 and C^i Psi^i = I; it keeps the output
// balanced to rounding).  One block per face; optional partial of r . z.
__device__ __forceinline__ double wsum(const double *__restrict__ y, const double *__restrict__ wloc, int64_t k) {
  return y ? y[k] + wloc[k] : wloc[k];
}

__global__ __launch_bounds__(256) void k_average_balance(DevGeom g, DevCoarse cs,
                                                         const double *__restrict__ wloc,
                                                         const double *__restrict__ yloc,
                                                         const double *__restrict__ csol, double *__restrict__ z,
                                                         const double *__restrict__ r, double *part,
                                                         const CgState *st) {
  __shared__ double red[8];
  if (st && st->done) return;
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  // one face per wave: faces 4 blockIdx.x + wave, then strided by the grid
  for (int f = blockIdx.x * 4 + (threadIdx.x >> 6); f < g.nF; f += gridDim.x * 4) {
    const int n = g.f_n[f];
    const int64_t base = g.g_off[g.f_minus[f]] + g.f_loffm[f];
    double tsum = 0.0;
    const double wm = g.fw_minus ? g.fw_minus[f] : 0.5, wp = g.fw_minus ? g.fw_plus[f] : 0.5;
    for (int a = lane; a < n; a += 64) {
      const int gi = g.Rmap[base + a];
      tsum += wm * wsum(yloc, wloc, base + a) + wp * wsum(yloc, wloc, g.own_plus[gi]);
    }
    const double corr = (csol[cs.face_cofs[f]] - wave_sum(tsum)) / n;
    for (int a = lane; a < n; a += 64) {
      const int gi = g.Rmap[base + a];
      const double zz = (g.fw_minus ? wm * wsum(yloc, wloc, base + a) + wp * wsum(yloc, wloc, g.own_plus[gi])
                                    : 0.5 * (wsum(yloc, wloc, base + a) + wsum(yloc, wloc, g.own_plus[gi]))) +
                        corr;
      z[gi] = zz;
      if (r) v = fma(r[gi], zz, v);
    }
  }
  if (part) block_write_partial(v, part, red);
}

// beta = rho' / rho; p = z + beta p (flux and coarse pressure)
__global__ __launch_bounds__(256) void k_update_p(int nGamma, int N, const int *__restrict__ pidx,
                                                  const double *__restrict__ zpart, int nzpart,
                                                  const double *__restrict__ zu, const double *__restrict__ csol,
                                                  double *pu, double *pp, CgState *st, double *beta_hist) {
  __shared__ double red[8];
  if (st->done) return;
  const double rn = block_sum_partials(zpart, nzpart, red);
  const double beta = rn / st->rho;
  for (int gi = blockIdx.x * 256 + threadIdx.x; gi < nGamma; gi += gridDim.x * 256)
    pu[gi] = fma(beta, pu[gi], zu[gi]);
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < N; k += 256) {
      const double zp = (pidx[k] >= 0) ? csol[pidx[k]] : 0.0;
      pp[k] = fma(beta, pp[k], zp);
    }
    if (threadIdx.x == 0) {
      beta_hist[st->it] = beta;
      st->rho_next = rn;
      st->pending = 1;     // applied by the next assembly kernel
    }
  }
}

// initial direction p = z, rho = r.z, ||r_0||^2
__global__ __launch_bounds__(256) void k_init_p(int nGamma, int N, const int *__restrict__ pidx,
                                                const double *__restrict__ zpart,
                                                int nzpart, const double *__restrict__ rpart, int nrpart,
                                                const double *__restrict__ zu, const double *__restrict__ csol,
                                                double *pu, double *pp, CgState *st, double rtol, int maxit) {
  __shared__ double red[8];
  const double rn = block_sum_partials(zpart, nzpart, red);
  const double r0 = block_sum_partials(rpart, nrpart, red);
  const int gi = blockIdx.x * 256 + threadIdx.x;
  if (gi < nGamma) pu[gi] = zu[gi];
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < N; k += 256) pp[k] = (pidx[k] >= 0) ? csol[pidx[k]] : 0.0;
    if (threadIdx.x == 0) {
      st->rho = rn;
      st->rho_next = rn;
      st->r0sq = r0;
      st->rtol2 = rtol * rtol;
      st->relres = 1.0;
      st->it = 0;
      st->nupd = 0;
      st->converged = (r0 == 0.0) ? 1 : 0;
      st->done = (r0 == 0.0) ? 1 : 0;
      st->fail = 0;
      st->maxit = maxit;
      st->pending = 0;
    }
  }
}

// partial of x.x over a vector
__global__ __launch_bounds__(256) void k_norm2_partial(int n, const double *__restrict__ x, double *part) {
  __shared__ double red[8];
  double v = 0.0;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) v = fma(x[k], x[k], v);
  block_write_partial(v, part, red);
}

__global__ void k_fill(int64_t n, double *x, double v) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) x[k] = v;
}

__global__ void k_axpby(int n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                        double *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = a * x[k] + b * y[k];
}

// ---------------------------------------------------------------------------
// steps 1-2 and the reduced right-hand side
// ---------------------------------------------------------------------------
// Coarse right-hand side of step 1: (0, D F_0), F = -source, F_0^i = sum over
// Omega^i.  The flux rows of b must be zero on entry.
__global__ __launch_bounds__(256) void k_step1_rhs(DevGeom g, const int *__restrict__ pidx,
                                                   const double *__restrict__ src,
                                                   const double *__restrict__ dscale, double *b) {
  __shared__ double red[8];
  const int i = blockIdx.x;
  const int nc = g.nc[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double s = 0.0;
  for (int c = threadIdx.x; c < nc; c += 256) s -= src[lcg[c]];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    if (pidx[i] >= 0) b[pidx[i]] = dscale[i] * t;
  }
}

__device__ __forceinline__ int line_start_s(int d, int l, const int *ext, const int *st) {
  int a0 = -1, a1 = -1;
  for (int e = 0; e < 3; ++e)
    if (e != d) { if (a0 < 0) a0 = e; else a1 = e; }
  return (l % ext[a0]) * st[a0] + (l / ext[a0]) * st[a1];
}

// Flux at an end of a line of subdomain cells that is not an interface dof:
// a face of the domain boundary, whose flux is prescribed (zero without
// boundary data).  lc: the line's end cell (local index), d: direction, e: 0
// for the minus end, 1 for the plus end.
__device__ __forceinline__ double boundary_end_flux(const DevGeom &g, int d, int lc, int e, const int *lo,
                                                    const int *ext) {
  if (!g.bflux) return 0.0;
  int c[3] = {lo[0] + lc % ext[0], lo[1] + (lc / ext[0]) % ext[1], lo[2] + lc / (ext[0] * ext[1])};
  c[d] += e;
  return g.bflux[g.face_off[d] + c[0] + (int64_t)g.fshape[d][0] * (c[1] + (int64_t)g.fshape[d][1] * c[2])];
}

// The line's cell coefficients are m[0], m[ms], ..., m[(n-1) ms] (staged in
// LDS by the caller, or read in place; see line_coef).
template <int CAP>
__device__ __forceinline__ void line_solve_s(int n, const double *m, int ms, double *y) {
  double cp[CAP];
  if (n < 2) return;
  double den = (m[0] + m[ms]) / 3.0;
  cp[1] = (n > 2) ? (m[ms] / 6.0) / den : 0.0;
  y[1] = y[1] / den;
  for (int j = 2; j <= n - 1; ++j) {
    const double mj1 = m[(j - 1) * ms], mj = m[j * ms];
    const double e = mj1 / 6.0;
    den = (mj1 + mj) / 3.0 - e * cp[j - 1];
    cp[j] = (j <= n - 2) ? (mj / 6.0) / den : 0.0;
    y[j] = (y[j] - e * y[j - 1]) / den;
  }
  for (int j = n - 2; j >= 1; --j) y[j] -= cp[j] * y[j + 1];
}

// Cell coefficients of the subdomain's local cells, mc[3c + d], gathered once
// per block so that the line solves read them from LDS.
__device__ __forceinline__ void stage_mcoef(int nc, const int *__restrict__ lcg, const double *__restrict__ mcoef,
                                            double *mc) {
  for (int k = threadIdx.x; k < 3 * nc; k += blockDim.x) {
    const int c = k / 3;
    mc[k] = mcoef[(int64_t)lcg[c] * 3 + (k - 3 * c)];
  }
}

// Coefficients of the line of cells that starts at local cell s0 along d:
// from the staged copy mc (local strides), or, in the kernels' unstaged form
// for subdomains whose staged copy does not fit in LDS, in place in the
// global array (strides of the lexicographic global cell numbering).
template <bool STAGED>
__device__ __forceinline__ const double *line_coef(const DevGeom &g, const double *mc, const double *mcoef,
                                                   const int *lcg, int s0, int d, const int *st, int &ms) {
  if (STAGED) {
    ms = 3 * st[d];
    return mc + 3 * s0 + d;
  }
  ms = 3 * (d == 0 ? 1 : (d == 1 ? g.n[0] : g.n[0] * g.n[1]));
  return mcoef + 3 * (int64_t)lcg[s0] + d;
}

// Block GEMV y = X v, X n x n column major, v and y in LDS.  A thread owns two
// rows (r, r + 256) and walks the columns four at a time with eight
// independent accumulators, so eight loads are in flight per thread and every
// column is read coalesced across the rows (non-temporal: X is read once).  (One wave per row with a strided
// inner loop waits on one load after another and ran at a third of this.)
__device__ __forceinline__ void block_gemv(int n, const double *__restrict__ X, const double *v, double *y) {
  for (int r0 = threadIdx.x; r0 < n; r0 += 512) {
    const int r1 = r0 + 256;
    const bool two = r1 < n;
    const double *x0 = X + r0, *x1 = X + (two ? r1 : r0);
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int c = 0;
    for (; c + 4 <= n; c += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t o = (int64_t)(c + q) * n;
        const double vc = v[c + q];
        a[q] = fma(__builtin_nontemporal_load(x0 + o), vc, a[q]);
        a[4 + q] = fma(__builtin_nontemporal_load(x1 + o), vc, a[4 + q]);
      }
    }
    for (; c < n; ++c) {
      const int64_t o = (int64_t)c * n;
      a[0] = fma(__builtin_nontemporal_load(x0 + o), v[c], a[0]);
      a[4] = fma(__builtin_nontemporal_load(x1 + o), v[c], a[4]);
    }
    y[r0] = (a[0] + a[1]) + (a[2] + a[3]);
    if (two) y[r1] = (a[4] + a[5]) + (a[6] + a[7]);
  }
  __syncthreads();
}

// h^i = H^{iT} X^i F^i: the source-dependent part of the reduced right-hand
// side f* (zero in subdomains without source).
// LDS: ys = X F (nc), then F (nc), whose space the staged coefficients (3 nc)
// take over once the product is formed.
template <int CAP, bool STAGED>
__global__ __launch_bounds__(256) void k_source_term(DevGeom g, const double *__restrict__ mcoef,
                                                     const double *__restrict__ Xmat, const int64_t *__restrict__ Xoff,
                                                     const double *__restrict__ src, double *__restrict__ hloc) {
  extern __shared__ double sh[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = g.nc[i], nG = g.nG[i];
  const int64_t go = g.g_off[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double *ys = sh, *Fs = sh + nc, *mc = sh + nc;
  int any = 0;
  for (int c = tid; c < nc; c += 256) {
    const double v = -src[lcg[c]];
    Fs[c] = v;
    any |= v != 0.0;
  }
  if (!__syncthreads_or(any)) {
    for (int t = tid; t < nG; t += 256) hloc[go + t] = 0.0;
    return;
  }
  block_gemv(nc, Xmat + Xoff[i], Fs, ys);   // ends with a barrier
  if (STAGED) {
    stage_mcoef(nc, lcg, mcoef, mc);
    __syncthreads();
  }
  int ext[3], st[3];
  for (int d = 0; d < 3; ++d) ext[d] = g.ext[3 * i + d];
  st[0] = 1; st[1] = ext[0]; st[2] = ext[0] * ext[1];
  for (int t = tid; t < nG; t += 256) {
    const int64_t fl = go + t;
    const int d = g.lg_dir[fl], lc = g.lg_cell[fl], end = g.lg_end[fl];
    const int n = ext[d];
    const int cd = (lc / st[d]) % n;
    const int s0 = lc - cd * st[d];
    int ms;
    const double *m = line_coef<STAGED>(g, mc, mcoef, lcg, s0, d, st, ms);
    double y[CAP + 1];
    const int eidx = end ? n - 1 : 0;
    double v = (end ? -1.0 : 1.0) * ys[s0 + eidx * st[d]];
    if (n >= 2) {
      // (G B_l^T y)[adj]: (B_l^T y)_j = y[c_j] - y[c_{j-1}]
      y[0] = 0.0;
      for (int j = 1; j <= n - 1; ++j) y[j] = ys[s0 + j * st[d]] - ys[s0 + (j - 1) * st[d]];
      line_solve_s<CAP>(n, m, ms, y);
      const int adj = end ? n - 1 : 1;
      v -= (m[eidx * ms] / 6.0) * y[adj];
    }
    hloc[go + t] = v;
  }
}

// f* = -assembled S u0 + assembled h (+ assembled sb, the interface load of
// the boundary fluxes; may be null)  (step-3 reduced right-hand side)
__global__ void k_fstar(DevGeom g, const double *__restrict__ yloc, const double *__restrict__ hloc,
                        const double *__restrict__ sb, double *__restrict__ r) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= g.nGamma) return;
  const int a = g.own_minus[gi], b = g.own_plus[gi];
  double v = -(yloc[a] + yloc[b]) + hloc[a] + hloc[b];
  if (sb) v += sb[a] + sb[b];
  r[gi] = v;
}

// Boundary flux data (prescribed normal fluxes g on the boundary faces) for the
// reduced problem.  With u = u_b + u_0, u_b carrying g on the boundary faces,
// each local problem gains the cell load H_b g = B_b g - B_I A_II^{-1} A_Ib g
// (its flux-row load -A_Ib g eliminated along the lines of cells) and each
// interface dof t the load -(A_tb - A_tI A_II^{-1} A_Ib) g of the line through
// it whose other end is on the boundary.  hb: per cell (global order), the
// first; sb: per local interface dof, the second.  One block per subdomain.
template <int CAP, bool STAGED>
__global__ __launch_bounds__(256) void k_bflux_load(DevGeom g, const double *__restrict__ mcoef,
                                                    double *__restrict__ hb, double *__restrict__ sb) {
  extern __shared__ double sh[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = g.nc[i], nG = g.nG[i];
  const int64_t go = g.g_off[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double *ys = sh, *mc = sh + nc;
  int ext[3], lo[3], st[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = g.ext[3 * i + d];
    lo[d] = g.lo[3 * i + d];
  }
  st[0] = 1; st[1] = ext[0]; st[2] = ext[0] * ext[1];
  for (int c = tid; c < nc; c += 256) ys[c] = 0.0;
  if (STAGED) stage_mcoef(nc, lcg, mcoef, mc);
  __syncthreads();
  const int *lg = g.line_g + g.line_off[i];
  int64_t lbase = 0;
  for (int d = 0; d < g.dim; ++d) {
    const int n = ext[d], lines = nc / n;
    for (int l = tid; l < lines; l += 256) {
      const int s0 = line_start_s(d, l, ext, st), s1 = s0 + (n - 1) * st[d];
      const double gm = lg[lbase + 2 * l] < 0 ? boundary_end_flux(g, d, s0, 0, lo, ext) : 0.0;
      const double gp = lg[lbase + 2 * l + 1] < 0 ? boundary_end_flux(g, d, s1, 1, lo, ext) : 0.0;
      ys[s0] += gm;
      ys[s1] -= gp;
      if (n >= 2 && (gm != 0.0 || gp != 0.0)) {
        int ms;
        const double *m = line_coef<STAGED>(g, mc, mcoef, lcg, s0, d, st, ms);
        double y[CAP + 1];
        for (int j = 0; j <= n; ++j) y[j] = 0.0;
        y[1] += (m[0] / 6.0) * gm;
        y[n - 1] += (m[(n - 1) * ms] / 6.0) * gp;
        line_solve_s<CAP>(n, m, ms, y);
        for (int c = 0; c < n; ++c) {
          double v = 0.0;
          if (c >= 1) v += y[c];
          if (c + 1 <= n - 1) v -= y[c + 1];
          ys[s0 + c * st[d]] -= v;
        }
      }
    }
    lbase += 2 * lines;
    __syncthreads();
  }
  for (int c = tid; c < nc; c += 256) hb[lcg[c]] = ys[c];
  // interface dofs whose line ends on the boundary at its other end
  for (int t = tid; t < nG; t += 256) {
    const int64_t fl = go + t;
    const int d = g.lg_dir[fl], lc = g.lg_cell[fl], end = g.lg_end[fl];
    const int n = ext[d];
    const int cd = (lc / st[d]) % n;
    const int s0 = lc - cd * st[d], s1 = s0 + (n - 1) * st[d];
    const bool other_on_boundary = end ? (lo[d] == 0) : (lo[d] + n == g.n[d]);
    double v = 0.0;
    if (other_on_boundary) {
      const double gb = end ? boundary_end_flux(g, d, s0, 0, lo, ext) : boundary_end_flux(g, d, s1, 1, lo, ext);
      int ms;
      const double *m = line_coef<STAGED>(g, mc, mcoef, lcg, s0, d, st, ms);
      if (gb != 0.0) {
        if (n == 1) {
          v = -(m[0] / 6.0) * gb;                  // -A_tb g: both faces of one cell
        } else {
          double y[CAP + 1];
          for (int j = 0; j <= n; ++j) y[j] = 0.0;
          if (end) y[1] = (m[0] / 6.0) * gb;       // A_Ib g next to the minus (boundary) end
          else y[n - 1] = (m[(n - 1) * ms] / 6.0) * gb;
          line_solve_s<CAP>(n, m, ms, y);
          v = end ? (m[(n - 1) * ms] / 6.0) * y[n - 1] : (m[0] / 6.0) * y[1];   // A_tI A_II^{-1} A_Ib g
        }
      }
    }
    sb[fl] = v;
  }
}

// B_0 x per subdomain (diagnostic operator)
__global__ __launch_bounds__(256) void k_b0(DevGeom g, const double *__restrict__ x, const double *__restrict__ dscale,
                                            double *__restrict__ y) {
  __shared__ double red[8];
  const int i = blockIdx.x;
  const int64_t go = g.g_off[i];
  double s = 0.0;
  for (int t = threadIdx.x; t < g.nG[i]; t += 256) {
    const double sign = g.lg_end[go + t] ? -1.0 : 1.0;
    s += sign * x[g.Rmap[go + t]];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) y[i] = dscale[i] * (red[0] + red[1] + red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// post-correction: interior fluxes and pressures of every subdomain from the
// final interface flux u_G and the source (local Dirichlet problems), in three
// launches: the pressure right-hand side (one block per subdomain), the
// product with X^i (a pure stream over X^i in row chunks, so the 4.5 GB of the
// reservoir are read at the copy rate with no latency-bound line solves and no
// partial last round of whole subdomains in the way), and the interior fluxes
// and pressures (one block per subdomain).  ybuf and pbuf hold one value per
// local cell, in the subdomains' local cell order.
// ---------------------------------------------------------------------------
// y = H w - F = H w + source, with w = R_i u_G
template <int CAP, bool STAGED>
__global__ __launch_bounds__(256) void k_recover_rhs(DevGeom g, const double *__restrict__ mcoef,
                                                     const double *__restrict__ src, const double *__restrict__ uG,
                                                     double *__restrict__ ybuf) {
  extern __shared__ double sh[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = g.nc[i], nG = g.nG[i];
  const int64_t go = g.g_off[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double *ws = sh, *ys = sh + nG, *mc = sh + nG + nc;
  int ext[3], lo[3], st[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = g.ext[3 * i + d];
    lo[d] = g.lo[3 * i + d];
  }
  st[0] = 1; st[1] = ext[0]; st[2] = ext[0] * ext[1];
  for (int t = tid; t < nG; t += 256) ws[t] = uG ? uG[g.Rmap[go + t]] : 0.0;
  for (int c = tid; c < nc; c += 256) ys[c] = src ? src[lcg[c]] : 0.0;
  if (STAGED) stage_mcoef(nc, lcg, mcoef, mc);
  __syncthreads();
  const int *lg = g.line_g + g.line_off[i];
  int64_t lbase = 0;
  for (int d = 0; d < g.dim; ++d) {
    const int n = ext[d], lines = nc / n;
    for (int l = tid; l < lines; l += 256) {
      const int s0 = line_start_s(d, l, ext, st);
      const int tm = lg[lbase + 2 * l], tp = lg[lbase + 2 * l + 1];
      const int s1 = s0 + (n - 1) * st[d];
      const double wm = tm >= 0 ? ws[tm] : boundary_end_flux(g, d, s0, 0, lo, ext);
      const double wp = tp >= 0 ? ws[tp] : boundary_end_flux(g, d, s1, 1, lo, ext);
      ys[s0] += wm;
      ys[s1] -= wp;
      if (n >= 2 && (wm != 0.0 || wp != 0.0)) {
        int ms;
        const double *m = line_coef<STAGED>(g, mc, mcoef, lcg, s0, d, st, ms);
        double y[CAP + 1];
        for (int j = 0; j <= n; ++j) y[j] = 0.0;
        y[1] += (m[0] / 6.0) * wm;
        y[n - 1] += (m[(n - 1) * ms] / 6.0) * wp;
        line_solve_s<CAP>(n, m, ms, y);
        for (int c = 0; c < n; ++c) {
          double v = 0.0;
          if (c >= 1) v += y[c];
          if (c + 1 <= n - 1) v -= y[c + 1];
          ys[s0 + c * st[d]] -= v;
        }
      }
    }
    lbase += 2 * lines;
    __syncthreads();
  }
  double *yo = ybuf + g.cell_off[i];
  for (int c = tid; c < nc; c += 256) yo[c] = ys[c];
}

// p = X^i y: block (i, k) forms rows 256k .. 256k + 255 of subdomain i, one row
// per thread, eight columns per step with eight independent accumulators (eight
// loads in flight, each column read coalesced across the rows, non-temporal:
// X^i is read once).
__global__ __launch_bounds__(256) void k_recover_xgemv(DevGeom g, const double *__restrict__ Xmat,
                                                       const int64_t *__restrict__ Xoff,
                                                       const double *__restrict__ ybuf, double *__restrict__ pbuf) {
  extern __shared__ double vs[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = g.nc[i];
  const int r0 = (int)blockIdx.y * 256, r = r0 + tid;
  if (r0 >= nc) return;   // the whole block leaves
  const double *yi = ybuf + g.cell_off[i];
  for (int c = tid; c < nc; c += 256) vs[c] = yi[c];
  __syncthreads();
  if (r >= nc) return;
  const double *xr = Xmat + Xoff[i] + r;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c = 0;
  for (; c + 8 <= nc; c += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = fma(__builtin_nontemporal_load(xr + (int64_t)(c + q) * nc), vs[c + q], a[q]);
  }
  for (; c < nc; ++c) a[0] = fma(__builtin_nontemporal_load(xr + (int64_t)c * nc), vs[c], a[0]);
  pbuf[g.cell_off[i] + r] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// interior fluxes u_I = G(-A_IG w - B_I^T p), line by line, and the pressures
// p + D p_0
template <int CAP, bool STAGED>
__global__ __launch_bounds__(256) void k_recover_flux(DevGeom g, const double *__restrict__ mcoef,
                                                      const double *__restrict__ uG, const double *__restrict__ pbuf,
                                                      const double *__restrict__ xp,
                                                      const double *__restrict__ dscale, double *__restrict__ flux,
                                                      double *__restrict__ pressure) {
  extern __shared__ double sh[];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = g.nc[i], nG = g.nG[i];
  const int64_t go = g.g_off[i];
  const int *lcg = g.lcell_global + g.cell_off[i];
  double *ws = sh, *ps = sh + nG, *mc = sh + nG + nc;
  int ext[3], lo[3], st[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = g.ext[3 * i + d];
    lo[d] = g.lo[3 * i + d];
  }
  st[0] = 1; st[1] = ext[0]; st[2] = ext[0] * ext[1];
  const double *pi = pbuf + g.cell_off[i];
  for (int t = tid; t < nG; t += 256) ws[t] = uG[g.Rmap[go + t]];
  for (int c = tid; c < nc; c += 256) ps[c] = pi[c];
  if (STAGED) stage_mcoef(nc, lcg, mcoef, mc);
  __syncthreads();
  const int *lg = g.line_g + g.line_off[i];
  int64_t lbase = 0;
  for (int d = 0; d < g.dim; ++d) {
    const int n = ext[d], lines = nc / n;
    if (n >= 2) {
      for (int l = tid; l < lines; l += 256) {
        const int s0 = line_start_s(d, l, ext, st);
        const int tm = lg[lbase + 2 * l], tp = lg[lbase + 2 * l + 1];
        const double wm = tm >= 0 ? ws[tm] : boundary_end_flux(g, d, s0, 0, lo, ext);
        const double wp = tp >= 0 ? ws[tp] : boundary_end_flux(g, d, s0 + (n - 1) * st[d], 1, lo, ext);
        int ms;
        const double *m = line_coef<STAGED>(g, mc, mcoef, lcg, s0, d, st, ms);
        double y[CAP + 1];
        y[0] = 0.0;
        for (int j = 1; j <= n - 1; ++j) y[j] = -(ps[s0 + j * st[d]] - ps[s0 + (j - 1) * st[d]]);
        y[1] -= (m[0] / 6.0) * wm;
        y[n - 1] -= (m[(n - 1) * ms] / 6.0) * wp;
        line_solve_s<CAP>(n, m, ms, y);
        for (int j = 1; j <= n - 1; ++j) {
          const int lc = s0 + j * st[d];
          int c[3] = {lo[0] + lc % ext[0], lo[1] + (lc / ext[0]) % ext[1], lo[2] + lc / (ext[0] * ext[1])};
          const int64_t fid = g.face_off[d] + c[0] + (int64_t)g.fshape[d][0] * (c[1] + (int64_t)g.fshape[d][1] * c[2]);
          flux[fid] = y[j];
        }
      }
    }
    lbase += 2 * lines;
  }
  const double p0 = (i < g.N - 1) ? dscale[i] * xp[i] : 0.0;
  for (int c = tid; c < nc; c += 256) pressure[lcg[c]] = ps[c] + p0;
}

__global__ void k_scatter_iface(int nGamma, const int64_t *__restrict__ gamma_face, const double *__restrict__ uG,
                                double *__restrict__ flux) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi < nGamma) flux[gamma_face[gi]] = uG[gi];
}

__global__ __launch_bounds__(256) void k_sum_partial(int64_t n, const double *__restrict__ x, double *part) {
  __shared__ double red[8];
  double s = 0.0;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) s += x[k];
  block_write_partial(s, part, red);
}

__global__ __launch_bounds__(256) void k_sub_mean(int64_t n, double *x, const double *__restrict__ part, int npart) {
  __shared__ double red[8];
  const double tot = block_sum_partials(part, npart, red);
  const double mean = tot / (double)n;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) x[k] -= mean;
}

// explicit instantiations used by the host code
template __global__ void k_symv<double>(DevGeom, const double *, const int64_t *, const double *, double,
                                        const double *, double *, CgState *, const double *, int);
template __global__ void k_symv<float>(DevGeom, const float *, const int64_t *, const double *, double, const double *,
                                       double *, CgState *, const double *, int);
template __global__ void k_psi_apply<double>(DevGeom, const double *, const int64_t *, const int *, const int *,
                                             const double *, double, const double *, double *, CgState *,
                                             const double *, int);
template __global__ void k_psi_apply<float>(DevGeom, const float *, const int64_t *, const int *, const int *,
                                            const double *, double, const double *, double *, CgState *,
                                            const double *, int);

template __global__ void k_psi_correct<double>(DevGeom, DevCoarse, const double *, const int64_t *, const double *,
                                               const double *, double *, const CgState *);
template __global__ void k_psi_correct<float>(DevGeom, DevCoarse, const float *, const int64_t *, const double *,
                                              const double *, double *, const CgState *);

}  // namespace bddc
