// C ABI of the BDDC library: handle, setup orchestration, CG driver,
// diagnostics.  All numerical work runs in the kernels of setup.hip and
// solve.hip (compiled into this translation unit).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <shared_mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bddc.h"
#include "common.hpp"
#include "layout.hpp"
#include "nd.hpp"
#include "gate.hpp"
#include "setup.hip"
#include "solve.hip"
#include "coarse.hip"
#include "block.hip"
#include "front.hip"

using namespace bddc;

namespace {

thread_local std::string g_last_error;

// Device allocator for the arrays of every handle created afterwards
// (bddc_set_allocator); null: hipMalloc / hipFree.  Each allocation keeps the
// free routine it came with.
struct Allocator {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*free)(void *, void *) = nullptr;
  void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

struct Error {
  int code;
  std::string msg;
};

// Scratch of one solve's CG: the dot-product partials of the producing
// kernels (at most PART_BLOCKS each), the device CG state and the alpha / beta
// history the Lanczos estimate reads.
struct CgScratch {
  CgState *st = nullptr;
  double *part_g = nullptr, *part_r = nullptr, *part_z = nullptr, *part_p = nullptr;
  double *alpha_h = nullptr, *beta_h = nullptr;
};

// Static scratch of bddc_solve_noalloc (512 KiB, one copy per device, held
// until the process ends).  In host code `scratch` names a host-side stand-in:
// its device address comes from hipGetSymbolAddress, once per device, and
// only that address is passed on.  Layout in doubles: the CG state (32), the
// partials of the operator dot product, the residual norm and the
// preconditioned dot product (PART_BLOCKS each), those of the pressure mean
// (256), then the alpha and the beta history (NOALLOC_HIST each).
constexpr int64_t NOALLOC_DOUBLES = 65536;
constexpr int64_t NOALLOC_HEAD = 32 + 3 * PART_BLOCKS + 256;
constexpr int64_t NOALLOC_HIST = (NOALLOC_DOUBLES - NOALLOC_HEAD) / 2;
static_assert(sizeof(CgState) <= 32 * sizeof(double), "CG state exceeds its scratch slot");
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
constexpr size_t SWEEP_STAGE_BYTES = 32768;   // level sweeps stage their task's input in LDS up to this size
constexpr size_t TOP_STAGE_BYTES = 65536;     // ... and the setup's column sweeps of the top block
constexpr int LS_SPLIT = 1024;     // subdomains with this many cells finish their local setup over many workgroups
constexpr int LS_SPLIT_MAX = 8192; // (up to this many: the projection keeps z in 64 KB of LDS)
constexpr int FRONT_SPLIT = 192;   // fronts with this many own dofs finish their factor over many workgroups
constexpr int SUB_CANDS = 7;   // autotuner: bottom-subtree depths -1 (none) .. 5
constexpr int SUB_DEFAULT_LEVELS = -1;   // levels swept by bottom subtrees without the autotuner (< 0: none)
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      throw Error{e_ == hipErrorOutOfMemory ? BDDC_ENOMEM : BDDC_EDEVICE,                 \
                  std::string(#x) + ": " + hipGetErrorString(e_)};                        \
  } while (0)

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Launch the instance of a line kernel whose private line arrays hold the
// longest subdomain extent of the problem (SHORTLINE or MAXLINE cells).
#define LINE_LAUNCH(longl, K, grid, block, shm, stream, ...)                   \
  do {                                                                          \
    if (longl) K<MAXLINE><<<(grid), (block), (shm), (stream)>>>(__VA_ARGS__);   \
    else K<SHORTLINE><<<(grid), (block), (shm), (stream)>>>(__VA_ARGS__);       \
  } while (0)
// the line kernels that read the cell coefficients from an LDS copy (staged)
// or in place
#define LINE_LAUNCH_S(longl, staged, K, grid, block, shm, stream, ...)                                  \
  do {                                                                                                 \
    if (longl && staged) K<MAXLINE, true><<<(grid), (block), (shm), (stream)>>>(__VA_ARGS__);          \
    else if (longl) K<MAXLINE, false><<<(grid), (block), (shm), (stream)>>>(__VA_ARGS__);              \
    else if (staged) K<SHORTLINE, true><<<(grid), (block), (shm), (stream)>>>(__VA_ARGS__);            \
    else K<SHORTLINE, false><<<(grid), (block), (shm), (stream)>>>(__VA_ARGS__);                       \
  } while (0)
// blocks of the kernels that leave dot-product partials: interface vectors
// (256 entries per block and round) and faces (four per block and round)
inline int vec_blocks(int64_t n) { return (int)std::min<int64_t>(nblk(n), PART_BLOCKS); }
inline int face_blocks(int64_t nF) { return (int)std::min<int64_t>(nblk(nF, 4), PART_BLOCKS); }

}  // namespace

struct bddc_problem {
  Layout L;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  int precision = BDDC_FP64;
  int max_it = 10000;
  uint32_t flags = 0;
  int coarse_leaf = 0;
  int coarse_top = 0;
  int coarse_sub = 0;                             // bottom-subtree levels (0: default, < 0: none)
  int sweep_single = 0;                           // single-lane sweep rows up to this length (0: none)
  int t_grid = 0;                                 // workgroups of the T^i launch beside the coarse solve
  int n_cu = 0;                                   // compute units of the device
  double tau = 0.0;
  const double *ms_src = nullptr;                 // caller's source for the multiscale rows (setup only)
  const double *bflux_in = nullptr;               // caller's boundary fluxes (setup only)
  double *d_bflux = nullptr;                      // [n_faces_all] boundary fluxes, interior entries zero
  double *d_hb = nullptr, *d_sb = nullptr;        // their cell load H_b g [n_cells], interface load [sum nG]
  double *d_srcb = nullptr;                       // [n_cells] source plus H_b g (per solve)
  double b_outflow = 0.0, b_abs = 0.0;            // net outflow through the boundary and sum |g|
  std::vector<void *> allocs;
  std::vector<double> alloc_bytes;
  std::vector<Allocator> alloc_by;
  double device_bytes = 0;

  DevGeom g{};
  DevCoarse cs{};
  int ncu = 0, nk = 0, n_adaptive = 0;
  double omega_tilde = 0.0;
  std::vector<int> face_k;
  std::vector<double> face_omega, face_eig;
  std::vector<int64_t> eig_off_h;
  std::vector<int64_t> pk_h, psi_off_h;
  std::vector<int> sub_coff_h;

  double *mcoef = nullptr, *dscale = nullptr;
  double *Spk = nullptr, *T64 = nullptr, *Psi64 = nullptr, *Xmat = nullptr;
  float *T32 = nullptr, *Psi32 = nullptr;
  // coarse factorization (nested-dissection fronts)
  NdPlan nd;
  DevFronts fd{};
  DevSweep sw{};
  std::vector<int> pidx_h;
  double *FR = nullptr, *BC = nullptr, *csgn = nullptr, *cy = nullptr, *cS0 = nullptr, *cS1 = nullptr,
         *cXB = nullptr;
  double *Kt = nullptr, *ctt = nullptr;           // dense top block: S_t^{-1} (nt x top_ld), t_t
  int *tg_off = nullptr, *tg = nullptr;           // gather map of t_t
  int top_ld = 0;
  int *d_sph = nullptr;                           // bottom-subtree sweeps (nd_subtrees): phase offsets,
  const int4 *d_stask = nullptr;                  // task copies
  bool longl = false;                             // a subdomain extent exceeds SHORTLINE cells
  bool mc_staged = true;                          // the line kernels' coefficient copies fit in LDS
  double tune_coarse_ms[4] = {0, 0, 0, 0};        // autotuner: coarse solve per sweep width candidate
  double tune_sub_ms[SUB_CANDS] = {};              // autotuner: coarse solve per bottom-subtree depth
  double tune_w1_ms[4] = {};                       // autotuner: coarse solve per single-lane row limit
  double tune_precond_ms[4] = {0, 0, 0, 0};       // autotuner: preconditioner per T^i grid candidate
  double coarse_bytes = 0.0;
  int64_t *d_pk = nullptr, *d_psi_off = nullptr, *d_Xoff = nullptr, *d_gamma_face = nullptr;

  double *xu = nullptr, *ru = nullptr, *pu = nullptr, *zu = nullptr, *qu = nullptr, *u0 = nullptr, *uG = nullptr;
  double *xp = nullptr, *pp = nullptr, *yloc = nullptr, *wloc = nullptr, *bc = nullptr,
         *csol = nullptr;
  double *d_src = nullptr, *d_flux = nullptr, *d_pres = nullptr;
  double *d_zero_src = nullptr;                   // zero source of the step-1-only mode
  double *rec_y = nullptr, *rec_p = nullptr;      // [n_cells] post-correction: pressure rhs, X^i product
  double *lw = nullptr;                           // [sum nG] weights of E^T per local interface dof (null: 1/2)
  // dot-product partials, CG state and coefficient history of a solve: the
  // handle's own arrays (cgw_own), or the library's static scratch while
  // bddc_solve_noalloc runs
  CgScratch cgw{}, cgw_own{};
  int device = 0;                                 // device the handle lives on
  CgState *st_host = nullptr;                     // [2] pinned: state after chunk k lands in [k & 1]
  double *ab_host = nullptr;                      // pinned: CG alpha / beta history of the last solve
  hipEvent_t ev_state[2] = {nullptr, nullptr};    // recorded after each chunk's state copy
  // the solve in progress (solve_begin ... solve_finish)
  struct Run {
    bool dev = false, eager = false;
    const double *src = nullptr;
    const double *lsrc = nullptr;                 // source of the local problems (src, plus H_b g)
    double *fl = nullptr, *pr = nullptr;          // device outputs
    double *flux = nullptr, *pressure = nullptr;  // caller's outputs (host unless dev)
    int chunks = 0, checked = 0;                  // chunks launched / whose state was read
    bool stop = false;                            // a chunk reported completion
    int upto = 0;                                 // 1 / 2: stop after step 1 / steps 1-2
    std::chrono::steady_clock::time_point t0;
  } run;
  double peak_bytes = 0;                          // high-water mark of device_bytes
  int *d_err = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t side = nullptr;                     // coarse solve of the preconditioner
  hipGraphExec_t cg_graph = nullptr;              // CG_CHUNK iterations, captured once
  BlockWs blk{};                                  // block CG (several sources at once)
  hipGraphExec_t blk_graph = nullptr;             // CG_CHUNK block iterations, captured once
  CgBlockState *blk_st_host = nullptr;            // pinned: block CG state after a chunk
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  bddc_stats_t stats{};

  template <typename T>
  T *alloc(int64_t count) {
    if (count <= 0) count = 1;
    const size_t bytes = (size_t)count * sizeof(T);
    Allocator a;
    {
      std::lock_guard<std::mutex> lk(g_alloc_mu);
      a = g_alloc;
    }
    void *p = nullptr;
    if (a.alloc) {
      p = a.alloc(bytes, a.ctx);
      if (!p) throw Error{BDDC_ENOMEM, "the caller's allocator returned no memory"};
    } else {
      HIPCHK(hipMalloc(&p, bytes));
    }
    allocs.push_back(p);
    alloc_bytes.push_back((double)bytes);
    alloc_by.push_back(a);
    device_bytes += (double)bytes;
    peak_bytes = std::max(peak_bytes, device_bytes);
    return (T *)p;
  }
  void free_at(size_t k) {
    if (!allocs[k]) return;
    if (alloc_by[k].free)
      alloc_by[k].free(allocs[k], alloc_by[k].ctx);
    else if (!alloc_by[k].alloc)
      (void)hipFree(allocs[k]);
    allocs[k] = nullptr;
  }
  void release(void *p) {
    for (size_t k = 0; k < allocs.size(); ++k)
      if (allocs[k] == p) {
        free_at(k);
        device_bytes -= alloc_bytes[k];
        alloc_bytes[k] = 0.0;
      }
  }
  template <typename T>
  T *upload(const std::vector<T> &v) {
    T *d = alloc<T>((int64_t)v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
  }
  // The graph goes first (its nodes name the events and streams below), the
  // streams are drained before anything they use is released.
  ~bddc_problem() {
    if (cg_graph) (void)hipGraphExecDestroy(cg_graph);
    if (blk_graph) (void)hipGraphExecDestroy(blk_graph);
    if (side) (void)hipStreamSynchronize(side);
    if (own_stream) (void)hipStreamSynchronize(own_stream);
    for (hipEvent_t e : ev_state)
      if (e) (void)hipEventDestroy(e);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    if (own_stream) (void)hipStreamDestroy(own_stream);
    if (st_host) (void)hipHostFree(st_host);
    if (ab_host) (void)hipHostFree(ab_host);
    if (blk_st_host) (void)hipHostFree(blk_st_host);
    for (size_t k = 0; k < allocs.size(); ++k) free_at(k);
  }
};

namespace {

void check_err(bddc_problem *h, const char *stage) {
  int e = 0;
  HIPCHK(hipMemcpy(&e, h->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (e & 1) throw Error{BDDC_EINVAL, "permeability must be finite and > 0"};
  if (e) throw Error{BDDC_EFACTOR, std::string("factorization lost definiteness in ") + stage +
                                       " (code " + std::to_string(e) + ")"};
}

// LDS of k_symv: the gathered x and one row buffer per wavefront.
inline size_t symv_shm(const Layout &L) { return (size_t)(1 + SYMV_WAVES) * ld4(L.maxG) * sizeof(double); }
// LDS of the line kernels: k_source_term (X F, then F or the staged cell
// coefficients in its place), the post-correction's (w, one cell vector,
// staged coefficients) and k_bflux_load (one cell vector, staged
// coefficients).  Unstaged, they read the coefficients in place.
inline size_t source_shm(const Layout &L, bool staged) { return (size_t)(staged ? 4 : 2) * L.maxC * sizeof(double); }
inline size_t recover_shm(const Layout &L, bool staged) {
  return (size_t)(L.maxG + (staged ? 4 : 1) * L.maxC) * sizeof(double);
}
inline size_t bflux_shm(const Layout &L, bool staged) { return (size_t)(staged ? 4 : 1) * L.maxC * sizeof(double); }

// Every device array the coarse kernels dereference must exist before a launch.
void check_coarse_ptrs(const bddc_problem *h) {
  const DevFronts &f = h->fd;
  const DevSweep &w = h->sw;
  const void *p[] = {f.first, f.n, f.m, f.ch, f.b_off, f.bidx, f.ext, f.touch_off, f.touch, f.F_off, f.w_off,
                     f.q_off, f.r_off, f.v_off, w.wdst, w.xsc_off, w.xsc, w.task, h->FR, h->BC, h->csgn,
                     h->cy, h->cS0, h->cS1, h->cXB, h->bc, h->csol};
  for (const void *q : p)
    if (!q) throw Error{BDDC_EDEVICE, "coarse solver arrays not initialised"};
  if (h->nd.nt > 0 && (!h->Kt || !h->ctt || !h->tg_off || !h->tg || h->top_ld < h->nd.nt))
    throw Error{BDDC_EDEVICE, "dense top block not initialised"};
}

void fill(bddc_problem *h, double *x, int64_t n, double v) {
  if (n > 0) k_fill<<<nblk(n), 256, 0, h->stream>>>(n, x, v);
}

// Bottom-subtree sweeps of levels [0, lv] (lv < 0: none; nd_subtrees caps lv
// below the dense top block): host lists and their device copies.  The
// stream must be idle (the lists are replaced).
void set_subtrees(bddc_problem *h, int lv) {
  NdPlan &P = h->nd;
  nd_subtrees(P, lv);
  if (h->d_sph) h->release(h->d_sph);
  if (h->d_stask) h->release((void *)h->d_stask);
  h->d_sph = nullptr;
  h->d_stask = nullptr;
  if (P.sub_lv < 0) return;
  h->d_sph = h->upload(P.sph);
  h->d_stask = (const int4 *)h->upload(P.stask);
}

// Dense top block of the coarse solve (nd_dense_top): S_t^{-1} column by
// column, each column the top part of the sweeps of the top levels applied to
// a unit right-hand side (the factor of the top levels is that of S_t), for
// TOP_BATCH columns per pass.  Rounding aside, the dense product then gives
// what those sweeps give.
constexpr int TOP_BATCH = 128;

void setup_dense_top(bddc_problem *h, hipStream_t s) {
  NdPlan &P = h->nd;
  const int cap = h->coarse_top == 0 ? TOP_DEFAULT_DOFS : h->coarse_top;
  nd_dense_top(P, cap);
  if (P.nt == 0) return;
  const int nt = P.nt, d0 = P.lvl_dof[P.top], nfr = P.nfr;
  if (nt > TOP_MAX_DOFS) throw Error{BDDC_EINVAL, "dense top block too large"};
  int dev = 0, max_lds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  h->top_ld = (nt + 1) & ~1;
  if ((size_t)h->top_ld * sizeof(double) > (size_t)max_lds)
    throw Error{BDDC_EINVAL, "dense top block exceeds the LDS of one workgroup"};
  h->Kt = h->alloc<double>((int64_t)nt * h->top_ld);
  h->ctt = h->alloc<double>(nt);
  h->tg_off = h->upload(P.tg_off);
  h->tg = h->upload(P.tg);
  const int nb = std::min(nt, TOP_BATCH);
  const int64_t sk = h->nk, sv = P.v_off[nfr], sb = std::max<int64_t>(P.b_off[nfr], 1);
  const int64_t v0 = P.v_off[P.lvl_off[P.top]], v1 = P.v_off[nfr];
  double *bb = h->alloc<double>(nb * sk), *zb = h->alloc<double>(nb * sk), *xb = h->alloc<double>(nb * sk);
  double *S0b = h->alloc<double>(nb * sv), *S1b = h->alloc<double>(nb * sv), *XBb = h->alloc<double>(nb * sb);
  const unsigned ub = std::min(64u, nblk(std::max<int64_t>(nt, v1 - v0)));
  for (int j0 = 0; j0 < nt; j0 += nb) {
    const unsigned nc = (unsigned)std::min(nb, nt - j0);
    k_top_unit<<<dim3(ub, nc), 256, 0, s>>>(j0, nt, d0, sk, v0, v1, sv, bb, S0b, S1b);
    for (int lv = P.top; lv < P.H; ++lv) {
      const int t0 = P.ftask_off[lv], ntk = P.ftask_off[lv + 1] - t0;
      const size_t shm = (size_t)TOP_NC * P.lvl_maxn[lv] * sizeof(double);
      const int stage = shm <= TOP_STAGE_BYTES;
      k_top_fwd_cols<<<dim3(ntk, (nc + TOP_NC - 1) / TOP_NC), 256, stage ? shm : 0, s>>>(
          t0, h->sw, h->FR, bb, S0b, S1b, zb, sk, sv, (int)nc, nullptr, stage);
    }
    for (int lv = P.H - 1; lv >= P.top; --lv) {
      const int t0 = P.btask_lo[lv], ntk = P.btask_hi[lv] - t0;
      const size_t shm = (size_t)TOP_NC * P.lvl_maxnm[lv] * sizeof(double);
      const int stage = shm <= TOP_STAGE_BYTES;
      k_top_bwd_cols<<<dim3(ntk, (nc + TOP_NC - 1) / TOP_NC), 256, stage ? shm : 0, s>>>(
          t0, h->sw, h->BC, zb, h->csgn, XBb, xb, sk, sb, (int)nc, nullptr, stage);
    }
    k_top_store<<<dim3(nblk(h->top_ld), nc), 256, 0, s>>>(j0, nt, d0, h->top_ld, xb, sk, h->Kt);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(s));
  for (double *q : {bb, zb, xb, S0b, S1b, XBb}) h->release(q);
  // streamed per coarse solve: R of the swept fronts twice, S_t^{-1} once, the gather
  h->coarse_bytes = 2.0 * 8.0 * (double)P.r_off[P.lvl_off[P.top]] + 8.0 * (double)nt * h->top_ld +
                    (4.0 + 16.0) * (double)P.tg.size() + 16.0 * nt;
}

void do_setup(bddc_problem *h, const bddc_grid *gr, const double *perm, const bddc_partition *part) {
  Layout &L = h->L;
  {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  if ((h->flags & BDDC_STIFFNESS_SCALING) && !(h->flags & (BDDC_MULTISCALE | BDDC_ALL_CONSTRAINED)) &&
      h->tau > 0.0 && isfinite(h->tau))
    throw Error{BDDC_EINVAL, "stiffness scaling needs tau off or the multiscale constraints: the face "
                             "eigenproblems assume the weights 1/2"};
  int n[3] = {gr->n[0], gr->n[1], gr->n[2]};
  double hh[3] = {gr->h[0], gr->h[1], gr->h[2]};
  const int *cuts[3] = {part->cuts[0], part->cuts[1], part->cuts[2]};
  for (int d = 0; d < gr->dim; ++d)
    if (!cuts[d]) throw Error{BDDC_EINVAL, "partition cuts missing"};
  try {
    L.build(gr->dim, n, hh, part->nsub, cuts);
  } catch (const std::exception &e) {
    throw Error{BDDC_EINVAL, e.what()};
  }
  for (int i = 0; i < L.N; ++i)
    for (int d = 0; d < L.dim; ++d)
      if (L.ext[d][i] > MAXLINE) throw Error{BDDC_EINVAL, "subdomain extent exceeds 128 cells"};
      else if (L.ext[d][i] > SHORTLINE) h->longl = true;
  const int dim = L.dim;
  for (int64_t c = 0; c < L.ncells * dim; ++c)
    if (!(perm[c] > 0.0) || !isfinite(perm[c])) throw Error{BDDC_EINVAL, "permeability must be finite and > 0"};
  const int N = L.N;
  hipStream_t s = h->stream;

  // index data
  DevGeom &g = h->g;
  g.dim = dim;
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = L.n[d];
    g.h[d] = L.h[d];
    if (d < dim) vol *= L.h[d];
    for (int e = 0; e < 3; ++e) g.fshape[d][e] = L.fshape[d][e];
  }
  for (int d = 0; d < 4; ++d) g.face_off[d] = L.face_off[d];
  g.vol = vol;
  g.N = N;
  g.nGamma = L.nGamma;
  g.nF = L.nF;
  std::vector<int> lo3(3 * N), ext3(3 * N);
  for (int i = 0; i < N; ++i)
    for (int d = 0; d < 3; ++d) {
      lo3[3 * i + d] = L.lo[d][i];
      ext3[3 * i + d] = L.ext[d][i];
    }
  g.lo = h->upload(lo3);
  g.ext = h->upload(ext3);
  g.nc = h->upload(L.nc);
  g.nG = h->upload(L.nG);
  g.cell_off = h->upload(L.cell_off);
  g.g_off = h->upload(L.g_off);
  g.lcell_global = h->upload(L.lcell_global);
  g.lg_dir = h->upload(L.lg_dir);
  g.lg_cell = h->upload(L.lg_cell);
  g.lg_end = h->upload(L.lg_end);
  g.lg_partner = h->upload(L.lg_partner);
  g.Rmap = h->upload(L.Rmap);
  g.own_minus = h->upload(L.own_minus);
  g.own_plus = h->upload(L.own_plus);
  g.sub_minus = h->upload(L.sub_minus);
  g.sub_plus = h->upload(L.sub_plus);
  g.f_minus = h->upload(L.f_minus);
  g.f_plus = h->upload(L.f_plus);
  g.f_n = h->upload(L.f_n);
  g.f_loffm = h->upload(L.f_loff_minus);
  g.f_loffp = h->upload(L.f_loff_plus);
  g.sub_face_off = h->upload(L.sub_face_off);
  g.sub_faces = h->upload(L.sub_faces);
  g.line_off = h->upload(L.line_off);
  g.line_g = h->upload(L.line_g);
  h->d_gamma_face = h->upload(L.gamma_face);
  h->d_err = h->alloc<int>(1);
  {
    const int zero = 0;
    HIPCHK(hipMemcpy(h->d_err, &zero, sizeof(int), hipMemcpyHostToDevice));
  }

  // cell coefficients (Section 5 rescaling)
  std::vector<double> permv(perm, perm + L.ncells * dim);
  double *d_perm = h->upload(permv);
  h->mcoef = h->alloc<double>(L.ncells * 3);
  k_cell_coef<<<nblk(L.ncells), 256, 0, s>>>(g, d_perm, L.ncells, h->mcoef, h->d_err);
  HIPCHK(hipGetLastError());
  if (h->flags & BDDC_STIFFNESS_SCALING) {
    // weights of E, constant along each face (stiffness scaling)
    double *fwm = h->alloc<double>(std::max(L.nF, 1)), *fwp = h->alloc<double>(std::max(L.nF, 1));
    h->lw = h->alloc<double>(std::max<int64_t>(L.g_off[N], 1));
    if (L.nF > 0) {
      k_face_weights<<<L.nF, 64, 0, s>>>(g, h->mcoef, fwm, fwp, h->lw);
      HIPCHK(hipGetLastError());
    }
    g.fw_minus = fwm;
    g.fw_plus = fwp;
  }
  h->dscale = h->alloc<double>(N);

  // local dense setup: Schur complements S^i and the pressure operators
  std::vector<int64_t> oP(N), oV(N), oH(N), oS(N), oL(N), oW(N), oX(N), opk(N);
  int64_t ws = 0, xs = 0, pks = 0;
  for (int i = 0; i < N; ++i) {
    const int64_t nc = L.nc[i], nG = L.nG[i];
    oP[i] = ws; ws += nc * nc;
    oV[i] = ws; ws += nc * nc;
    oH[i] = ws; ws += nc * (nG + 1);
    oS[i] = ws; ws += nG * nG;
    oL[i] = ws; ws += nG * nG;
    oW[i] = ws; ws += nG * nG;
    oX[i] = xs; xs += nc * nc;
    opk[i] = pks; pks += gp_size((int)nG);
  }
  double *wsb = h->alloc<double>(ws);
  SetupWs sw;
  sw.base = wsb;
  sw.P = h->upload(oP);
  sw.V = h->upload(oV);
  sw.H = h->upload(oH);
  sw.S = h->upload(oS);
  sw.L = h->upload(oL);
  sw.W = h->upload(oW);
  sw.X = h->d_Xoff = h->upload(oX);
  sw.Xmat = h->Xmat = h->alloc<double>(xs);
  sw.pk = h->d_pk = h->upload(opk);
  sw.Spk = h->Spk = h->alloc<double>(pks);
  h->pk_h = opk;
  LINE_LAUNCH(h->longl, k_local_setup, N, 256, 0, s, g, h->mcoef, sw, h->dscale, h->d_err, LS_SPLIT, LS_SPLIT_MAX);
  HIPCHK(hipGetLastError());
  {
    // subdomains of at least LS_SPLIT cells: steps 5-7 over many workgroups
    std::vector<int> it_cols, it_tiles, it_sym;
    std::vector<int64_t> woff(N, 0);
    int64_t wsz = 0;
    int maxnc = 0;
    for (int i = 0; i < N; ++i) {
      const int nc = L.nc[i], nG = L.nG[i];
      if (nc < LS_SPLIT || nc > LS_SPLIT_MAX) continue;
      maxnc = std::max(maxnc, nc);
      woff[i] = wsz;
      wsz += nc;
      for (int c0 = 0; c0 < nG + 1; c0 += LS_COLS) it_cols.insert(it_cols.end(), {i, c0, 0, 0});
      for (int c0 = 0; c0 < nc; c0 += LS_COLS) it_cols.insert(it_cols.end(), {i, c0, 1, 0});
      for (int i0 = 0; i0 < nG; i0 += TILE)
        for (int j0 = 0; j0 <= i0; j0 += TILE) it_tiles.insert(it_tiles.end(), {i, i0, 0, j0});
      for (int i0 = 0; i0 < nc; i0 += TILE)
        for (int j0 = 0; j0 <= i0; j0 += TILE) it_tiles.insert(it_tiles.end(), {i, i0, 1, j0});
      for (int c0 = 0; c0 < nG; c0 += 64) it_sym.insert(it_sym.end(), {i, c0, 0, 0});
      for (int c0 = 0; c0 < nc; c0 += 64) it_sym.insert(it_sym.end(), {i, c0, 1, 0});
    }
    if (!it_cols.empty()) {
      // blocked Cholesky of P~, super-block by super-block (TILE = 64-row panels and tiles)
      std::vector<int> big;
      for (int i = 0; i < N; ++i)
        if (L.nc[i] >= LS_SPLIT && L.nc[i] <= LS_SPLIT_MAX) big.push_back(i);
      const int nbig = (int)big.size();
      const int *d_big = h->upload(big);
      std::vector<int> poff, uoff;   // per step: nbig + 1 prefix sums each
      std::vector<int> npan, nupd;
      const int nsteps = (maxnc + KB - 1) / KB;
      for (int st = 0; st < nsteps; ++st) {
        const int k1 = st * KB + KB;
        int pa = 0, up = 0;
        for (int b = 0; b < nbig; ++b) {
          poff.push_back(pa);
          uoff.push_back(up);
          const int M = L.nc[big[b]] - k1;
          if (M > 0) {
            const int q = (M + TILE - 1) / TILE;
            pa += q;
            up += q * (q + 1) / 2;
          }
        }
        poff.push_back(pa);
        uoff.push_back(up);
        npan.push_back(pa);
        nupd.push_back(up);
      }
      const int *d_poff = h->upload(poff), *d_uoff = h->upload(uoff);
      for (int st = 0; st < nsteps; ++st) {
        const int k0 = st * KB;
        k_pchol_diag<<<nbig, 256, 0, s>>>(g, sw, d_big, k0, h->d_err);
        if (npan[st] > 0)
          k_pchol_panel<<<npan[st], 256, 0, s>>>(g, sw, d_big, nbig, d_poff + (size_t)st * (nbig + 1), k0);
        if (nupd[st] > 0)
          k_pchol_update<<<nupd[st], 256, 0, s>>>(g, sw, d_big, nbig, d_uoff + (size_t)st * (nbig + 1), k0);
      }
      HIPCHK(hipGetLastError());
      const int4 *d_c = (const int4 *)h->upload(it_cols), *d_t = (const int4 *)h->upload(it_tiles),
                 *d_y = (const int4 *)h->upload(it_sym);
      const int64_t *d_woff = h->upload(woff);
      double *d_w = h->alloc<double>(wsz);
      const int nci = (int)it_cols.size() / 4;
      k_ls_solve<<<nci, 256, 0, s>>>(g, sw, d_c);
      // the projection needs each subdomain's whole last column of Y: a separate launch
      k_ls_project<<<nci, 256, (size_t)maxnc * sizeof(double), s>>>(g, sw, d_c, d_woff, d_w);
      k_ls_gemm<<<(int)it_tiles.size() / 4, 256, 0, s>>>(g, sw, d_t, d_woff, d_w);
      k_ls_sym<<<(int)it_sym.size() / 4, 256, 0, s>>>(g, sw, d_y);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      for (const int4 *q : {d_c, d_t, d_y}) h->release((void *)q);
      for (const int *q : {d_big, d_poff, d_uoff}) h->release((void *)q);
      h->release((void *)d_woff);
      h->release(d_w);
    }
  }
  k_schur_factor<<<N, 256, 0, s>>>(g, sw, h->d_err);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  check_err(h, "the subdomain setup");

  {
    int dev = 0, lds_max = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (symv_shm(L) > (size_t)lds_max)
      throw Error{BDDC_EINVAL, "subdomain interface too large for the local operator kernels' LDS"};
    // source term, boundary loads and post-correction: their vectors, with
    // the cell coefficients staged beside them where that fits (these
    // kernels have no static LDS)
    h->mc_staged = std::max({source_shm(L, true), recover_shm(L, true), bflux_shm(L, true)}) <= (size_t)lds_max;
    if (std::max({source_shm(L, false), recover_shm(L, false), (size_t)L.maxC * sizeof(double)}) > (size_t)lds_max)
      throw Error{BDDC_EINVAL, "subdomain too large for the LDS of the source-term and post-correction kernels"};
  }
  // face eigenproblems of Algorithm "Adaptive BDDC"
  const int nF = L.nF;
  h->face_k.assign(nF, 0);
  h->face_omega.assign(nF, 0.0);
  std::vector<int64_t> foff(nF), eoff(nF), roff(nF);
  int64_t fws = 0, es = 0, rs = 0;
  for (int f = 0; f < nF; ++f) {
    const int64_t fn = L.f_n[f];
    foff[f] = fws; fws += 6 * fn * fn + fn;
    eoff[f] = es; es += fn - 1;
    roff[f] = rs; rs += fn * fn;
  }
  h->eig_off_h = eoff;
  h->face_eig.assign(es, 0.0);
  const bool allc = (h->flags & BDDC_ALL_CONSTRAINED) != 0;
  const bool ms = !allc && (h->flags & BDDC_MULTISCALE) != 0;
  const bool adaptive = !ms && (h->tau > 0.0 && isfinite(h->tau));
  if ((adaptive || allc || ms) && L.maxFn > 256)
    throw Error{BDDC_EINVAL, "adaptive constraints need faces of at most 256 dofs"};
  double *d_rows = h->alloc<double>(rs);
  double *d_fws = nullptr;
  if (nF > 0 && (adaptive || allc || ms)) {
    d_fws = h->alloc<double>(fws);
    double *d_eig = h->alloc<double>(es);
    int *d_k = h->alloc<int>(nF);
    double *d_om = h->alloc<double>(nF);
    int64_t *d_foff = h->upload(foff), *d_eoff = h->upload(eoff), *d_roff = h->upload(roff);
    if (ms) {
      // the load of the well-shaped sources w_s on the local Dirichlet
      // problems, -H^{sT} X^s w_s (none without a source: every w_s uniform)
      double *hs = nullptr, *d_ms = nullptr, *d_w = nullptr;
      if (h->ms_src) {
        std::vector<double> msv(h->ms_src, h->ms_src + L.ncells);
        for (double v : msv)
          if (!isfinite(v)) throw Error{BDDC_EINVAL, "multiscale source must be finite"};
        d_ms = h->upload(msv);
        d_w = h->alloc<double>(L.ncells);
        hs = h->alloc<double>(std::max<int64_t>(L.g_off[N], 1));
        k_ms_weight<<<N, 256, 0, s>>>(g, d_ms, d_w);
        LINE_LAUNCH_S(h->longl, h->mc_staged, k_source_term, N, 256, source_shm(L, h->mc_staged), s, g, h->mcoef,
                      h->Xmat, h->d_Xoff, d_w, hs);
        HIPCHK(hipGetLastError());
      }
      k_face_ms<<<nF, 256, 0, s>>>(g, sw, hs, d_fws, d_foff, d_eig, d_eoff, d_k, d_om, d_rows, d_roff, h->d_err);
      if (hs) {
        HIPCHK(hipStreamSynchronize(s));
        for (double *q : {hs, d_ms, d_w}) h->release(q);
      }
    } else {
      k_face_reduce<<<nF, 256, 0, s>>>(g, sw, d_fws, d_foff, allc ? 1 : 0, d_eig, d_eoff, d_k, d_om, d_rows,
                                       d_roff, h->d_err);
    }
    HIPCHK(hipGetLastError());
    if (!allc && !ms) {
      k_face_eig<<<nF, 256, 0, s>>>(g, d_fws, d_foff, h->tau);
      k_face_rows<<<nF, 256, 0, s>>>(g, d_fws, d_foff, h->tau, d_eig, d_eoff, d_k, d_om, d_rows, d_roff);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    check_err(h, "the face eigenproblems");
    HIPCHK(hipMemcpy(h->face_k.data(), d_k, nF * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(h->face_omega.data(), d_om, nF * sizeof(double), hipMemcpyDeviceToHost));
    if (es > 0) HIPCHK(hipMemcpy(h->face_eig.data(), d_eig, es * sizeof(double), hipMemcpyDeviceToHost));
    h->release(d_fws);
  }
  h->n_adaptive = 0;
  h->omega_tilde = 0.0;
  for (int f = 0; f < nF; ++f) {
    h->n_adaptive += h->face_k[f];
    h->omega_tilde = std::max(h->omega_tilde, h->face_omega[f]);
  }

  // coarse numbering: nested-dissection fronts, level by level (see nd.hpp)
  NdPlan &P = h->nd;
  try {
    nd_plan(L, h->face_k, h->coarse_leaf, P);
    if (h->sweep_single > 0) nd_tasks(P, P.wide4, P.wide16, h->sweep_single);
  } catch (const std::logic_error &e) {
    throw Error{BDDC_EINVAL, std::string("coarse plan: ") + e.what()};
  }
  const std::vector<int> &face_cofs = P.face_cofs, &pidx = P.pidx;
  std::vector<int> sub_coff(N + 1, 0), sub_cmap;
  int ncu = 0;
  for (int f = 0; f < nF; ++f) ncu += 1 + h->face_k[f];
  const int nkc = P.nk;
  std::vector<int> co_minus(nkc, -1), co_plus(nkc, -1);
  for (int i = 0; i < N; ++i) {
    for (int t = L.sub_face_off[i]; t < L.sub_face_off[i + 1]; ++t) {
      const int f = L.sub_faces[t];
      for (int l = 0; l <= h->face_k[f]; ++l) {
        const int gdof = face_cofs[f] + l;
        const int flat = (int)sub_cmap.size();
        sub_cmap.push_back(gdof);
        if (L.f_minus[f] == i) co_minus[gdof] = flat;
        else co_plus[gdof] = flat;
      }
    }
    sub_coff[i + 1] = (int)sub_cmap.size();
    if (sub_coff[i + 1] - sub_coff[i] > 1024)
      throw Error{BDDC_EINVAL, "more than 1024 coarse dofs on one subdomain"};
  }
  h->ncu = ncu;
  h->nk = nkc;
  h->sub_coff_h = sub_coff;
  h->pidx_h = pidx;
  if ((int)h->pidx_h.size() != N || (int)h->sub_coff_h.size() != N + 1)
    throw Error{BDDC_EDEVICE, "coarse bookkeeping of the subdomains incomplete"};
  DevCoarse &cs = h->cs;
  cs.ncu = ncu;
  cs.nk = h->nk;
  cs.face_cofs = h->upload(face_cofs);
  cs.face_k = h->upload(h->face_k);
  cs.face_rows_off = h->upload(roff);
  cs.face_rows = d_rows;
  cs.sub_coff = h->upload(sub_coff);
  cs.sub_cmap = h->upload(sub_cmap);
  cs.co_minus = h->upload(co_minus);
  cs.co_plus = h->upload(co_plus);
  cs.pidx = h->upload(pidx);

  // local coarse spaces Psi^i, coarse matrices and substructure operators T^i
  std::vector<int64_t> cwoff(N), acoff(N), psioff(N);
  int64_t cws = 0, acs = 0, pss = 0;
  for (int i = 0; i < N; ++i) {
    const int64_t nci = sub_coff[i + 1] - sub_coff[i], nG = L.nG[i];
    cwoff[i] = cws; cws += 4 * nci * nG + 2 * nci * nci;
    acoff[i] = acs; acs += nci * nci;
    psioff[i] = pss; pss += ld4((int)nG) * nci;
  }
  h->psi_off_h = psioff;
  CoarseLocalWs cw;
  cw.base = h->alloc<double>(cws);
  cw.off = h->upload(cwoff);
  cw.Ac = h->alloc<double>(acs);
  cw.ac_off = h->upload(acoff);
  cw.psi64 = h->Psi64 = h->alloc<double>(pss);
  cw.psi32 = h->Psi32 = h->alloc<float>(pss);
  cw.psi_off = h->d_psi_off = h->upload(psioff);
  cw.t64 = h->T64 = h->alloc<double>(pks);
  cw.t32 = h->T32 = h->alloc<float>(pks);
  cw.pk = h->d_pk;
  k_coarse_local<<<N, 256, 0, s>>>(g, sw, cs, cw, h->d_err);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  check_err(h, "the local coarse spaces");

  // coarse saddle point: multifrontal signed Cholesky, level by level
  const int nk = h->nk;
  h->coarse_bytes = 0.0;
  h->bc = h->alloc<double>(nk + 1);
  fill(h, h->bc, nk + 1, 0.0);   // the preconditioner adds into b; the coarse solve clears what it read
  h->csol = h->alloc<double>(nk + 1);
  if (nk > 0) {
    DevFronts &fd = h->fd;
    fd.first = h->upload(P.first);
    fd.n = h->upload(P.n);
    fd.m = h->upload(P.m);
    fd.ch = h->upload(P.ch);
    fd.b_off = h->upload(P.b_off);
    fd.bidx = h->upload(P.bidx);
    fd.ext = h->upload(P.ext);
    fd.touch_off = h->upload(P.touch_off);
    fd.touch = h->upload(P.touch);
    fd.F_off = h->upload(P.F_off);
    fd.w_off = h->upload(P.w_off);
    fd.q_off = h->upload(P.q_off);
    fd.r_off = h->upload(P.r_off);
    fd.v_off = h->upload(P.v_off);
    const int nfr = P.nfr;
    double *Fall = h->alloc<double>(P.F_off[nfr]);
    double *Wall = h->alloc<double>(P.w_off[nfr]);
    double *Qall = h->alloc<double>(P.q_off[nfr]);
    h->FR = h->alloc<double>(P.r_off[nfr]);
    h->BC = h->alloc<double>(P.r_off[nfr]);
    h->cy = h->alloc<double>(nk);
    h->cS0 = h->alloc<double>(P.v_off[nfr]);
    h->cS1 = h->alloc<double>(P.v_off[nfr]);
    h->cXB = h->alloc<double>(P.b_off[nfr]);
    fill(h, h->cS0, P.v_off[nfr], 0.0);   // slots no child writes stay zero
    fill(h, h->cS1, P.v_off[nfr], 0.0);
    DevSweep &sv = h->sw;
    sv.wdst = h->upload(P.wdst);
    sv.xsc_off = h->upload(P.xsc_off);
    sv.xsc = h->upload(P.xsc);
    sv.task = (const int4 *)h->upload(P.task);
    sv.nfr = P.nfr;
    std::vector<double> sg(nk, 1.0);
    for (int i = 0; i < N; ++i)
      if (pidx[i] >= 0) sg[pidx[i]] = -1.0;
    h->csgn = h->upload(sg);
    check_coarse_ptrs(h);
    // tiles of the update matrices, level by level
    std::vector<int> tl_off(P.H + 1, 0);
    std::vector<int> tl;
    for (int lv = 0; lv < P.H; ++lv) {
      for (int r = P.lvl_off[lv]; r < P.lvl_off[lv + 1]; ++r)
        for (int i0 = 0; i0 < P.m[r]; i0 += TILE)
          for (int j0 = 0; j0 <= i0; j0 += TILE) {
            tl.push_back(r);
            tl.push_back(i0);
            tl.push_back(j0);
            tl.push_back(0);
          }
      tl_off[lv + 1] = (int)(tl.size() / 4);
    }
    const int4 *d_tl = (const int4 *)h->upload(tl);
    // fronts of at least FRONT_SPLIT own dofs: rows of L_BP (64 per item),
    // inverse columns (KB per item), tiles of Q and packed columns (64 per
    // item) over many workgroups
    std::vector<int> si_off(P.H + 1, 0), sq_off(P.H + 1, 0), sp_off(P.H + 1, 0), sr_off(P.H + 1, 0);
    std::vector<int> si, sq, sp, sr;
    for (int lv = 0; lv < P.H; ++lv) {
      for (int r = P.lvl_off[lv]; r < P.lvl_off[lv + 1]; ++r) {
        if (P.n[r] < FRONT_SPLIT) continue;
        for (int r0 = 0; r0 < P.m[r]; r0 += 64) sr.insert(sr.end(), {r, r0, 0, 0});
        for (int c0 = 0; c0 < P.n[r]; c0 += KB) si.insert(si.end(), {r, c0, 0, 0});
        for (int i0 = 0; i0 < P.m[r]; i0 += TILE)
          for (int j0 = 0; j0 < P.n[r]; j0 += TILE) sq.insert(sq.end(), {r, i0, j0, 0});
        for (int c0 = 0; c0 < P.n[r]; c0 += 64) sp.insert(sp.end(), {r, c0, 0, 0});
      }
      si_off[lv + 1] = (int)(si.size() / 4);
      sq_off[lv + 1] = (int)(sq.size() / 4);
      sp_off[lv + 1] = (int)(sp.size() / 4);
      sr_off[lv + 1] = (int)(sr.size() / 4);
    }
    const int4 *d_si = (const int4 *)h->upload(si), *d_sq = (const int4 *)h->upload(sq),
               *d_sp = (const int4 *)h->upload(sp), *d_sr = (const int4 *)h->upload(sr);
    for (int lv = 0; lv < P.H; ++lv) {
      const int f0 = P.lvl_off[lv], nf = P.lvl_off[lv + 1] - f0;
      k_front_factor<<<nf, 256, 0, s>>>(g, cs, fd, f0, cw.Ac, cw.ac_off, h->dscale, h->csgn, Fall, Wall, Qall,
                                        h->FR, h->BC, h->d_err, FRONT_SPLIT);
      HIPCHK(hipGetLastError());
      const int nr = sr_off[lv + 1] - sr_off[lv];
      if (nr > 0) k_front_rows<<<nr, 256, 0, s>>>(fd, d_sr + sr_off[lv], h->csgn, Fall);
      const int nt = tl_off[lv + 1] - tl_off[lv];
      if (nt > 0) {
        k_front_schur<<<nt, 256, 0, s>>>(fd, d_tl + tl_off[lv], h->csgn, Fall);
        HIPCHK(hipGetLastError());
      }
      const int ni = si_off[lv + 1] - si_off[lv], nq = sq_off[lv + 1] - sq_off[lv], np = sp_off[lv + 1] - sp_off[lv];
      if (ni > 0) k_front_inv<<<ni, 256, 0, s>>>(fd, d_si + si_off[lv], Fall, Wall);
      if (nq > 0) k_front_q<<<nq, 256, 0, s>>>(fd, d_sq + sq_off[lv], Fall, Wall, Qall);
      if (np > 0) k_front_pack<<<np, 256, 0, s>>>(fd, d_sp + sp_off[lv], Wall, Qall, h->FR, h->BC);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    check_err(h, "the coarse problem");
    h->release((void *)d_tl);
    for (const int4 *q : {d_si, d_sq, d_sp, d_sr}) h->release((void *)q);
    h->release(Fall);
    h->release(Wall);
    h->release(Qall);
    // streamed per coarse solve: R twice (rows forward, columns backward)
    h->coarse_bytes = 2.0 * 8.0 * (double)P.r_off[nfr];
    setup_dense_top(h, s);
    set_subtrees(h, (h->coarse_sub == 0 ? SUB_DEFAULT_LEVELS : h->coarse_sub) - 1);
  }

  const int nGm = L.nGamma;
  const int64_t totG = L.g_off[N];
  h->xu = h->alloc<double>(nGm);
  h->ru = h->alloc<double>(nGm);
  h->pu = h->alloc<double>(nGm);
  h->zu = h->alloc<double>(nGm);
  h->qu = h->alloc<double>(nGm);
  h->u0 = h->alloc<double>(nGm);
  h->uG = h->alloc<double>(nGm);
  h->xp = h->alloc<double>(N);
  h->pp = h->alloc<double>(N);
  h->yloc = h->alloc<double>(totG);
  h->wloc = h->alloc<double>(totG);
  h->cgw.part_g = h->alloc<double>(nblk(nGm) + 1);
  h->cgw.part_r = h->alloc<double>(nblk(nGm) + 1);
  h->cgw.part_z = h->alloc<double>(nF + 1);
  h->cgw.part_p = h->alloc<double>(1024);
  h->d_src = h->alloc<double>(L.ncells);
  h->d_zero_src = h->alloc<double>(L.ncells);
  h->rec_y = h->alloc<double>(L.ncells);
  h->rec_p = h->alloc<double>(L.ncells);
  h->d_flux = h->alloc<double>(L.nfaces_all);
  h->d_pres = h->alloc<double>(L.ncells);
  h->cgw.alpha_h = h->alloc<double>(h->max_it + 2);
  h->cgw.beta_h = h->alloc<double>(h->max_it + 2);
  h->cgw.st = h->alloc<CgState>(1);
  h->cgw_own = h->cgw;
  HIPCHK(hipHostMalloc((void **)&h->st_host, 2 * sizeof(CgState), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void **)&h->ab_host, 2 * (size_t)(h->max_it + 2) * sizeof(double), hipHostMallocDefault));
  for (hipEvent_t &e : h->ev_state) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipEventCreate(&h->ev0));
  HIPCHK(hipEventCreate(&h->ev1));
  HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  if (h->bflux_in) {
    // prescribed boundary fluxes (eq. problem-4): the boundary entries of the
    // caller's array, their net outflow for the compatibility check, and
    // their loads on the local problems
    std::vector<double> bf(L.nfaces_all, 0.0);
    for (int d = 0; d < dim; ++d) {
      const int *fs = L.fshape[d];
      for (int k = 0; k < fs[0] * fs[1] * fs[2]; ++k) {
        int c[3] = {k % fs[0], (k / fs[0]) % fs[1], k / (fs[0] * fs[1])};
        if (c[d] != 0 && c[d] != L.n[d]) continue;
        const int64_t fid = L.face_off[d] + k;
        const double v = h->bflux_in[fid];
        if (!isfinite(v)) throw Error{BDDC_EINVAL, "boundary fluxes must be finite"};
        bf[fid] = v;
        h->b_outflow += c[d] == 0 ? -v : v;
        h->b_abs += fabs(v);
      }
    }
    h->d_bflux = h->upload(bf);
    g.bflux = h->d_bflux;
    h->d_hb = h->alloc<double>(L.ncells);
    h->d_sb = h->alloc<double>(std::max<int64_t>(totG, 1));
    h->d_srcb = h->alloc<double>(L.ncells);
    LINE_LAUNCH_S(h->longl, h->mc_staged, k_bflux_load, N, 256, bflux_shm(L, h->mc_staged), s, g, h->mcoef,
                  h->d_hb, h->d_sb);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(s));

  // statistics of the operators streamed per iteration
  // entries of the operators as the method defines them: lower triangles of
  // T^i and S^i, the n_Gamma^i x n_c^i bases Psi^i (storage padding excluded)
  double sumpk = 0.0, sumpsi = 0.0, sumsq = 0.0;
  for (int i = 0; i < N; ++i) {
    const double nG = L.nG[i];
    sumpk += nG * (nG + 1) / 2;
    sumsq += nG * nG;
    sumpsi += nG * (double)(sub_coff[i + 1] - sub_coff[i]);
  }
  const double sT = h->precision == BDDC_MIXED ? 4.0 : 8.0;
  h->stats.bytes_prec = sumpk * sT + 2.0 * sumpsi * sT + h->coarse_bytes + 6.0 * totG * 8.0 + 4.0 * nGm * 8.0;
  // the block preconditioner (FP64 operators in both forms), 16 columns of the vectors
  h->stats.bytes_prec_block =
      sumpk * 8.0 + 2.0 * sumpsi * 8.0 + h->coarse_bytes + BK * (6.0 * totG * 8.0 + 4.0 * nGm * 8.0);
  h->stats.flops_block_local = 2.0 * BK * sumsq;
  h->stats.bytes_per_iter = h->stats.bytes_prec + sumpk * 8.0 + 2.0 * totG * 8.0 + 8.0 * nGm * 8.0;
}

// Coarse solve csol = K^{-1} bc by the multifrontal forward / backward sweeps:
// the levels below the dense top block (all of them without one) sweep one
// launch per level and direction; the top block is one gather and one dense
// product with S_t^{-1}.  bc is left zero (each entry is cleared once read),
// ready for the next right-hand side to be added into it.
void launch_coarse_solve(bddc_problem *h, hipStream_t s, const int *done) {
  const NdPlan &P = h->nd;
  if (h->nk == 0) return;
  check_coarse_ptrs(h);
  // levels [0, sl] by bottom subtrees, one launch per direction
  const int sl = P.sub_lv;
  if (sl >= 0 && (!h->d_sph || !h->d_stask)) throw Error{BDDC_EDEVICE, "subtree sweep lists not uploaded"};
  if (sl >= 0)
    k_nd_fwd_sub<<<P.nsubt, SUB_THREADS, 0, s>>>(sl + 1, h->d_sph, h->d_stask, h->sw, h->FR, h->bc, h->cS0, h->cS1,
                                                 h->cy, done);
  for (int lv = sl + 1; lv < P.top; ++lv) {
    const int t0 = P.ftask_off[lv], nt = P.ftask_off[lv + 1] - t0;
    const size_t shm = (size_t)P.lvl_maxn[lv] * sizeof(double);
    const int stage = shm <= SWEEP_STAGE_BYTES;
    k_nd_fwd<<<nt, 256, stage ? shm : 0, s>>>(t0, h->sw, h->FR, h->bc, h->cS0, h->cS1, h->cy, done, stage);
  }
  if (P.nt > 0) {
    const int d0 = P.lvl_dof[P.top];
    k_top_gather<<<nblk(P.nt), 256, 0, s>>>(P.nt, d0, h->tg_off, h->tg, h->bc, h->cS0, h->cS1, h->ctt, done);
    k_top_gemv<<<nblk(P.nt, TOP_ROWS_PER_WG), TOP_THREADS, (size_t)h->top_ld * sizeof(double), s>>>(
        P.nt, h->top_ld, h->Kt, h->ctt, d0, h->sw.xsc_off, h->sw.xsc, h->cXB, h->csol, h->bc, done);
  }
  for (int lv = P.top - 1; lv > sl; --lv) {
    const int t0 = P.btask_lo[lv], nt = P.btask_hi[lv] - t0;
    const size_t shm = (size_t)P.lvl_maxnm[lv] * sizeof(double);
    const int stage = shm <= SWEEP_STAGE_BYTES;
    k_nd_bwd<<<nt, 256, stage ? shm : 0, s>>>(t0, h->sw, h->BC, h->cy, h->csgn, h->cXB, h->csol, h->bc, done, stage);
  }
  if (sl >= 0)
    k_nd_bwd_sub<<<P.nsubt, SUB_THREADS, 0, s>>>(sl + 1, h->d_sph + (int64_t)P.nsubt * (sl + 2), h->d_stask, h->sw,
                                                 h->BC, h->cy, h->csgn, h->cXB, h->csol, h->bc, done);
}


void launch_precond(bddc_problem *h, const double *r, double *z, double *zpart, bool check) {
  const Layout &L = h->L;
  hipStream_t s = h->stream;
  const int N = L.N, nF = L.nF;
  const size_t shm = (size_t)5 * ld4(L.maxG) * sizeof(double);
  CgState *st = check ? h->cgw.st : nullptr;
  const double *rp = check ? h->cgw.part_r : nullptr;
  const int nrp = vec_blocks(L.nGamma);
  const bool mixed = h->precision == BDDC_MIXED;
  // The coarse chain (right-hand side pieces Psi^{iT} r^i with the stopping
  // test, the coarse solve, the correction Psi^i alpha) is the longest path
  // and stays on the main stream; the substructure corrections T^i r^i run
  // beside it on the side stream (t_grid workgroups, which sets how much of
  // the memory bandwidth they take from the latency-bound coarse sweeps) and
  // join before the averaging, which adds the two parts.
  if (mixed)
    k_psi_apply<float><<<N, 256, shm, s>>>(h->g, h->Psi32, h->d_psi_off, h->cs.sub_coff, h->cs.sub_cmap, r, 0.5,
                                           h->lw, h->bc, st, rp, nrp);
  else
    k_psi_apply<double><<<N, 256, shm, s>>>(h->g, h->Psi64, h->d_psi_off, h->cs.sub_coff, h->cs.sub_cmap, r, 0.5,
                                            h->lw, h->bc, st, rp, nrp);
  HIPCHK(hipEventRecord(h->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  // By default the FP32 T^i gets one workgroup of SYMV_THREADS per CU (a
  // grid-stride loop over the subdomains): with two per CU it finishes sooner
  // but takes enough bandwidth from the coarse sweeps to lengthen the apply.
  const int tg = h->t_grid > 0 ? std::min(h->t_grid, N) : (mixed && h->n_cu > 0 ? std::min(h->n_cu, N) : N);
  if (mixed)
    k_symv<float><<<tg, SYMV_THREADS, symv_shm(L), h->side>>>(h->g, h->T32, h->d_pk, r, 0.5, h->lw, h->yloc, st, nullptr, 0);
  else
    k_symv<double><<<tg, SYMV_THREADS, symv_shm(L), h->side>>>(h->g, h->T64, h->d_pk, r, 0.5, h->lw, h->yloc, st, nullptr,
                                                               0);
  HIPCHK(hipEventRecord(h->ev_join, h->side));
  // The coarse solve stays FP64 in both forms: the CG runs in the balanced
  // subspace, so the face-average coarse fluxes must satisfy B_c alpha = 0 to
  // FP64 accuracy (the FP32 local operators are corrected by the balance step).
  if (h->nk > 0) {
    launch_coarse_solve(h, s, st ? &st->done : nullptr);
  }
  if (mixed)
    k_psi_correct<float><<<N, 256, 0, s>>>(h->g, h->cs, h->Psi32, h->d_psi_off, nullptr, h->csol, h->wloc, st);
  else
    k_psi_correct<double><<<N, 256, 0, s>>>(h->g, h->cs, h->Psi64, h->d_psi_off, nullptr, h->csol, h->wloc, st);
  HIPCHK(hipStreamWaitEvent(s, h->ev_join, 0));
  if (nF > 0)
    k_average_balance<<<face_blocks(nF), 256, 0, s>>>(h->g, h->cs, h->wloc, h->yloc, h->csol, z, r, zpart, st);
}
void launch_iteration(bddc_problem *h) {
  const Layout &L = h->L;
  hipStream_t s = h->stream;
  const int N = L.N, nGm = L.nGamma;
  const int nb = vec_blocks(nGm);
  k_symv<double><<<N, SYMV_THREADS, symv_shm(L), s>>>(h->g, h->Spk, h->d_pk, h->pu, 1.0, nullptr, h->yloc, h->cgw.st, nullptr, 0);
  k_sys_assemble<<<nb, 256, 0, s>>>(h->g, h->yloc, h->pp, h->dscale, h->pu, h->qu, h->cgw.part_g, h->cgw.st);
  k_update_xr<<<nb, 256, 0, s>>>(nGm, N, h->cgw.part_g, nb, h->pu, h->qu, h->pp, h->xu, h->ru, h->xp, h->cgw.part_r,
                                 h->cgw.st, h->cgw.alpha_h);
  launch_precond(h, h->ru, h->zu, h->cgw.part_z, true);
  k_update_p<<<nb, 256, 0, s>>>(nGm, N, h->cs.pidx, h->cgw.part_z, face_blocks(L.nF), h->zu, h->csol, h->pu, h->pp,
                                h->cgw.st, h->cgw.beta_h);
}

double lanczos_kappa(const std::vector<double> &a, const std::vector<double> &b, double *lmin, double *lmax) {
  int k = (int)a.size();
  for (int j = 0; j + 1 < k && j < (int)b.size(); ++j)
    if (!(b[j] > 0.0)) { k = j + 1; break; }
  if (k == 0) { *lmin = *lmax = 1.0; return 1.0; }
  // symmetric tridiagonal: bisection on the Sturm sequence for the extremes
  std::vector<double> d(k), e(k, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / a[j] + (j > 0 ? b[j - 1] / a[j - 1] : 0.0);
    if (j + 1 < k) e[j] = sqrt(b[j]) / a[j];
  }
  double lo = d[0], hi = d[0];
  for (int j = 0; j < k; ++j) {
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j + 1 < k ? fabs(e[j]) : 0.0);
    lo = std::min(lo, d[j] - r);
    hi = std::max(hi, d[j] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int j = 1; j < k; ++j) {
      if (q == 0.0) q = 1e-300;
      q = d[j] - x - e[j - 1] * e[j - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  auto kth = [&](int idx) {
    double a0 = lo, b0 = hi;
    for (int it = 0; it < 200; ++it) {
      const double m = 0.5 * (a0 + b0);
      if (count_below(m) > idx) b0 = m; else a0 = m;
      if (b0 - a0 <= 1e-15 * std::max(fabs(a0), fabs(b0))) break;
    }
    return 0.5 * (a0 + b0);
  };
  *lmin = kth(0);
  *lmax = kth(k - 1);
  return *lmax / *lmin;
}

constexpr int CG_CHUNK = 8;   // CG iterations between host convergence checks

// Capture `count` calls of fn (launches on the main and side stream) into a
// graph.  The capture runs on the handle's own stream; the graph is replayed
// on whatever stream the handle uses.  The capturing thread only launches
// kernels and records / waits on events; the capture is relaxed so that other
// threads (the server's driver) may keep synchronising, copying and freeing
// meanwhile; the HIP gate keeps such calls out of the capture.  Called without
// the gate held.
template <typename F>
hipGraphExec_t capture_graph(bddc_problem *h, int count, F &&fn, const char *what) {
  GateExclusive capture_lock(g_gate);
  hipStream_t keep = h->stream;
  h->stream = h->own_stream;
  hipGraph_t gr = nullptr;
  hipGraphExec_t ex = nullptr;
  std::string where = "begin";
  hipError_t e = hipStreamBeginCapture(h->own_stream, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    for (int k = 0; k < count && e == hipSuccess; ++k) {
      try {
        fn();
      } catch (const Error &err) {
        e = hipErrorUnknown;
        where = "call " + std::to_string(k) + ": " + err.msg;
      }
      if (e == hipSuccess) {
        e = hipGetLastError();
        if (e != hipSuccess) where = "launch in call " + std::to_string(k);
      }
    }
    const hipError_t e2 = hipStreamEndCapture(h->own_stream, &gr);
    if (e == hipSuccess) {
      e = e2;
      where = "end";
    }
  }
  h->stream = keep;
  if (e == hipSuccess) {
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    where = "instantiate";
  }
  if (gr) (void)hipGraphDestroy(gr);
  if (e != hipSuccess)
    throw Error{BDDC_EDEVICE, std::string("capturing ") + what + " (" + where + "): " + hipGetErrorString(e)};
  return ex;
}

// CG_CHUNK iterations in one graph: every kernel reads its scalars from the
// device CG state, so one graph serves every chunk of every solve.
void build_cg_graph(bddc_problem *h) {
  h->cg_graph = nullptr;
  h->cg_graph = capture_graph(h, CG_CHUNK, [&] { launch_iteration(h); }, "the CG iteration graph");
}

// Mean duration (ms) of fn as a solve runs it: GRAPH_REPS calls captured into
// one graph, replayed ceil(reps / GRAPH_REPS) times after one warm-up replay,
// timed with HIP events on the handle's stream.  (Launched one by one, the
// short kernels of the coarse chain wait on the host's launch rate.)  Called
// without the gate held.
constexpr int GRAPH_REPS = 8;

template <typename F>
double time_graph_ms(bddc_problem *h, int reps, F &&fn, const char *what) {
  hipGraphExec_t ex = capture_graph(h, GRAPH_REPS, fn, what);
  GateShared g(g_gate);
  const int launches = std::max(1, (reps + GRAPH_REPS - 1) / GRAPH_REPS);
  float ms = 0.f;
  hipError_t e = hipGraphLaunch(ex, h->stream);
  if (e == hipSuccess) e = hipEventRecord(h->ev0, h->stream);
  for (int k = 0; k < launches && e == hipSuccess; ++k) e = hipGraphLaunch(ex, h->stream);
  if (e == hipSuccess) e = hipEventRecord(h->ev1, h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->ev0, h->ev1);
  (void)hipGraphExecDestroy(ex);
  HIPCHK(e);
  return ms / (launches * GRAPH_REPS);
}

// Autotuner of the launch shapes of the per-iteration kernels (BDDC_AUTOTUNE),
// run at the end of the setup on the problem's own operators:
//  * the lane-group widths of the coarse sweeps (rows or columns up to wide4
//    entries take 4 lanes, up to wide16 16, longer ones 64; a workgroup takes
//    256 / g of them): fewer, fuller workgroups per level against more
//    parallelism.  Each candidate task list is timed on the coarse solve;
//  * the workgroups of the substructure corrections T^i, which run beside the
//    coarse solve and share the memory bandwidth with it: timed on the whole
//    preconditioner.
// Each candidate is timed as the solve runs it, from a graph replay.  Both
// only change how the work is laid out on the device: a sweep row is
// summed by a different number of lanes (rounding order only), and the T^i
// grid changes which workgroup takes which subdomain (same bits).
void autotune(bddc_problem *h) {
  const auto t0 = std::chrono::steady_clock::now();
  NdPlan &P = h->nd;
  const Layout &L = h->L;
  constexpr int REPS = 16;   // two timed replays of eight calls after a warm one
  auto set_tasks = [&](int c4, int c16, int w1) {
    GateShared g(g_gate);
    nd_tasks(P, c4, c16, w1);
    HIPCHK(hipStreamSynchronize(h->stream));
    h->release((void *)h->sw.task);
    h->sw.task = (const int4 *)h->upload(P.task);
    set_subtrees(h, P.sub_lv);   // nd_tasks rebuilt the subtree copies of the tasks
  };
  auto set_sub = [&](int lv) {
    GateShared g(g_gate);
    HIPCHK(hipStreamSynchronize(h->stream));
    set_subtrees(h, lv);
  };
  if (h->nk > 0 && P.top > 0) {
    {
      GateShared g(g_gate);
      fill(h, h->bc, h->nk, 1.0);
    }
    static const int cand[][2] = {{8, 32}, {12, 48}, {24, 96}, {48, 192}};
    double best = 1e300;
    int bi = 0;
    for (int c = 0; c < 4; ++c) {
      set_tasks(cand[c][0], cand[c][1], -1);
      const double ms =
          time_graph_ms(h, REPS, [&] { launch_coarse_solve(h, h->stream, nullptr); }, "the coarse solve");
      h->tune_coarse_ms[c] = ms;
      if (ms < best) { best = ms; bi = c; }
    }
    if (bi != 3) set_tasks(cand[bi][0], cand[bi][1], -1);   // else the last candidate's tasks are in place
    // single-lane rows (and columns) up to w1 entries
    {
      static const int w1c[4] = {0, 8, 16, 32};
      const int c4 = P.wide4, c16 = P.wide16;
      best = 1e300;
      int bw = 0;
      for (int c = 0; c < 4; ++c) {
        set_tasks(c4, c16, w1c[c]);
        const double ms =
            time_graph_ms(h, REPS, [&] { launch_coarse_solve(h, h->stream, nullptr); }, "the coarse solve");
        h->tune_w1_ms[c] = ms;
        if (ms < best) { best = ms; bw = c; }
      }
      if (bw != 3) set_tasks(c4, c16, w1c[bw]);
    }
    // bottom subtrees: levels [0, lv] in one launch per direction
    const int lv0 = P.sub_lv;
    best = 1e300;
    int blv = lv0;
    for (int c = 0; c < SUB_CANDS; ++c) {
      const int lv = c - 1;
      if (lv >= P.top) break;
      set_sub(lv);
      const double ms =
          time_graph_ms(h, REPS, [&] { launch_coarse_solve(h, h->stream, nullptr); }, "the coarse solve");
      h->tune_sub_ms[c] = ms;
      if (ms < best) { best = ms; blv = lv; }
      if (ms > 1.25 * best) break;   // deeper subtrees only serialise more of the wide fronts
    }
    set_sub(blv);
    GateShared g(g_gate);
    fill(h, h->bc, h->nk, 0.0);
  }
  if (L.N > 1 && L.nGamma > 0) {
    {
      GateShared g(g_gate);
      fill(h, h->ru, L.nGamma, 1.0);
    }
    const int cand[] = {3 * h->n_cu / 4, h->n_cu, 2 * h->n_cu, L.N};
    double best = 1e300;
    int bg = L.N;
    for (int c = 0; c < 4; ++c) {
      const int tg = std::max(1, std::min(cand[c], L.N));
      h->t_grid = tg;
      const double ms = time_graph_ms(h, REPS, [&] { launch_precond(h, h->ru, h->zu, nullptr, false); },
                                      "the preconditioner");
      h->tune_precond_ms[c] = ms;
      if (ms < best) { best = ms; bg = tg; }
    }
    h->t_grid = bg;
  }
  GateShared g(g_gate);
  HIPCHK(hipStreamSynchronize(h->stream));
  h->stats.t_tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}


// One solve in phases, so that a scheduler can interleave several handles
// without blocking on any of them:
//   solve_begin   validates and uploads the source and enqueues steps 1-2, the
//                 reduced right-hand side, the first preconditioner apply and p_0;
//   solve_chunk   enqueues CG_CHUNK iterations and an asynchronous copy of the
//                 CG state (several chunks may be in flight: iterations after
//                 convergence leave at once);
//   solve_poll    tells, without blocking, whether the oldest chunk in flight
//                 has landed and whether the CG has stopped;
//   solve_finish  waits for the chunks in flight, enqueues the final interface
//                 flux, the post-correction and the output copies, and waits.
// bddc_solve runs them back to back with one chunk in flight.
bool solve_needs_cg(const bddc_problem *h) { return h->L.N > 1 && h->run.upto == 0; }

// upto_u0 stops after step 1 (u0, and R.lsrc set), for the block CG, which
// forms the reduced right-hand sides f* of several sources at once and starts
// its iterations from them.
void solve_begin_launch(bddc_problem *h, const double *rhs, double rtol, double *flux, double *pressure,
                        uint32_t flags, bool upto_u0 = false) {
  const Layout &L = h->L;
  hipStream_t s = h->stream;
  const int N = L.N, nF = L.nF, nGm = L.nGamma;
  auto &R = h->run;
  R = bddc_problem::Run();
  R.t0 = std::chrono::steady_clock::now();
  R.dev = (flags & BDDC_DEVICE_PTRS) != 0;
  R.eager = (flags & BDDC_EAGER) != 0;
  if ((flags & BDDC_STEP1_ONLY) && (flags & BDDC_STEP12_ONLY))
    throw Error{BDDC_EINVAL, "BDDC_STEP1_ONLY and BDDC_STEP12_ONLY exclude each other"};
  R.upto = (flags & BDDC_STEP1_ONLY) ? 1 : (flags & BDDC_STEP12_ONLY) ? 2 : 0;
  if (!(rtol > 0.0)) throw Error{BDDC_EINVAL, "rtol must be > 0"};
  R.src = rhs;
  if (!R.dev) {
    double sum = 0.0, asum = 0.0;
    for (int64_t c = 0; c < L.ncells; ++c) {
      if (!isfinite(rhs[c])) throw Error{BDDC_EINVAL, "source must be finite"};
      sum += rhs[c];
      asum += fabs(rhs[c]);
    }
    if (fabs(sum - h->b_outflow) > 1e-12 * (asum + h->b_abs))
      throw Error{BDDC_EINVAL, h->d_bflux ? "source must equal the net boundary outflow (compatibility)"
                                          : "source must sum to zero (no-flow compatibility)"};
    HIPCHK(hipMemcpyAsync(h->d_src, rhs, L.ncells * sizeof(double), hipMemcpyHostToDevice, s));
    R.src = h->d_src;
  }
  R.flux = flux;
  R.pressure = pressure;
  R.fl = R.dev ? flux : h->d_flux;
  R.pr = R.dev ? pressure : h->d_pres;
  if (N <= 1) return;
  const int nb = (int)nblk(nGm);
  const double *src = R.src;
  if (h->d_bflux) {
    // with boundary fluxes the local problems see the source plus H_b g
    k_axpby<<<nblk(L.ncells), 256, 0, s>>>((int)L.ncells, 1.0, R.src, 1.0, h->d_hb, h->d_srcb);
    src = h->d_srcb;
  }
  R.lsrc = src;
  // step 1: coarse solve with (0, D F_0), u0 = E Psi alpha
  fill(h, h->bc, h->nk, 0.0);
  k_step1_rhs<<<N, 256, 0, s>>>(h->g, h->cs.pidx, src, h->dscale, h->bc);
  launch_coarse_solve(h, h->stream, nullptr);
  k_psi_correct<double><<<N, 256, 0, s>>>(h->g, h->cs, h->Psi64, h->d_psi_off, nullptr, h->csol, h->wloc,
                                          nullptr);
  k_average_balance<<<face_blocks(nF), 256, 0, s>>>(h->g, h->cs, h->wloc, nullptr, h->csol, h->u0, nullptr, nullptr,
                                                    nullptr);
  if (R.upto || upto_u0) {
    // u_0 or u^*: the post-correction with x = 0 continues u_0 into the interiors
    if (R.upto) fill(h, h->xp, N, 0.0);
    HIPCHK(hipGetLastError());
    return;
  }
  // steps 2-3 right-hand side: f* = -S u0 + H^T X F
  k_symv<double><<<N, SYMV_THREADS, symv_shm(L), s>>>(h->g, h->Spk, h->d_pk, h->u0, 1.0, nullptr, h->yloc, nullptr, nullptr, 0);
  LINE_LAUNCH_S(h->longl, h->mc_staged, k_source_term, N, 256, source_shm(L, h->mc_staged), s, h->g, h->mcoef,
                h->Xmat, h->d_Xoff, src, h->wloc);
  k_fstar<<<nblk(nGm), 256, 0, s>>>(h->g, h->yloc, h->wloc, h->d_sb, h->ru);
  fill(h, h->xu, nGm, 0.0);
  fill(h, h->xp, N, 0.0);
  k_norm2_partial<<<vec_blocks(nGm), 256, 0, s>>>(nGm, h->ru, h->cgw.part_r);
  launch_precond(h, h->ru, h->zu, h->cgw.part_z, false);
  k_init_p<<<nb, 256, 0, s>>>(nGm, N, h->cs.pidx, h->cgw.part_z, face_blocks(nF), h->cgw.part_r, vec_blocks(nGm), h->zu,
                              h->csol, h->pu, h->pp,
                              h->cgw.st, rtol, h->max_it);
  HIPCHK(hipGetLastError());
}

void solve_begin(bddc_problem *h, const double *rhs, double rtol, double *flux, double *pressure, uint32_t flags) {
  {
    GateShared g(g_gate);
    solve_begin_launch(h, rhs, rtol, flux, pressure, flags);
  }
  if (!solve_needs_cg(h)) return;
  if (!h->run.eager && !h->cg_graph) build_cg_graph(h);
  GateShared g(g_gate);
  HIPCHK(hipEventRecord(h->ev0, h->stream));
}

void solve_chunk(bddc_problem *h) {
  GateShared g(g_gate);
  auto &R = h->run;
  hipStream_t s = h->stream;
  if (R.chunks > h->max_it / CG_CHUNK + 2) throw Error{BDDC_EDEVICE, "CG loop did not report completion"};
  if (R.chunks - R.checked >= 2) throw Error{BDDC_EINVAL, "at most two CG chunks in flight"};
  if (R.eager) {
    for (int k = 0; k < CG_CHUNK; ++k) launch_iteration(h);
  } else {
    HIPCHK(hipGraphLaunch(h->cg_graph, s));
  }
  HIPCHK(hipGetLastError());
  const int slot = R.chunks & 1;
  HIPCHK(hipMemcpyAsync(h->st_host + slot, h->cgw.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(h->ev_state[slot], s));
  ++R.chunks;
}

// 1: the oldest chunk in flight has landed (R.stop tells whether the CG has
// stopped); 0: not yet; throws on a device error.
int solve_poll(bddc_problem *h, bool wait) {
  GateShared g(g_gate);
  auto &R = h->run;
  if (R.checked >= R.chunks) return 0;
  const int slot = R.checked & 1;
  if (wait) {
    HIPCHK(hipEventSynchronize(h->ev_state[slot]));
  } else {
    const hipError_t e = hipEventQuery(h->ev_state[slot]);
    if (e == hipErrorNotReady) return 0;
    HIPCHK(e);
  }
  if (h->st_host[slot].done) R.stop = true;
  ++R.checked;
  return 1;
}

// Post-correction of Algorithm "BDDC method": the interior fluxes and
// pressures of every subdomain from the final interface flux uG and the
// source (local Dirichlet problems), into the run's outputs (enqueued only).
// In three parts, so that the block solve can multiply the right-hand sides of
// all its sources by X^i at once: the pressure right-hand side (rec_y), its
// product with X^i (rec_p), and the fluxes, pressures and output copies.
void post_correct_rhs(bddc_problem *h) {
  const Layout &L = h->L;
  auto &R = h->run;
  // step 1 alone continues u_0 with zero source
  const double *rsrc = R.src;
  if (R.upto == 1) {
    fill(h, h->d_zero_src, L.ncells, 0.0);
    rsrc = h->d_zero_src;
  }
  LINE_LAUNCH_S(h->longl, h->mc_staged, k_recover_rhs, L.N, 256, recover_shm(L, h->mc_staged), h->stream, h->g,
                h->mcoef, rsrc, h->uG, h->rec_y);
}

void post_correct_out(bddc_problem *h) {
  const Layout &L = h->L;
  hipStream_t s = h->stream;
  const int N = L.N, nGm = L.nGamma;
  auto &R = h->run;
  double *fl = R.fl, *pr = R.pr;
  if (h->d_bflux)
    HIPCHK(hipMemcpyAsync(fl, h->d_bflux, L.nfaces_all * sizeof(double), hipMemcpyDeviceToDevice, s));
  else
    fill(h, fl, L.nfaces_all, 0.0);
  if (nGm > 0) k_scatter_iface<<<nblk(nGm), 256, 0, s>>>(nGm, h->d_gamma_face, h->uG, fl);
  if (N == 1) fill(h, h->xp, 1, 0.0);
  LINE_LAUNCH_S(h->longl, h->mc_staged, k_recover_flux, N, 256, recover_shm(L, h->mc_staged), s, h->g, h->mcoef,
                h->uG, h->rec_p, h->xp, h->dscale, fl, pr);
  k_sum_partial<<<256, 256, 0, s>>>(L.ncells, pr, h->cgw.part_p);
  k_sub_mean<<<256, 256, 0, s>>>(L.ncells, pr, h->cgw.part_p, 256);
  HIPCHK(hipGetLastError());
  if (!R.dev) {
    HIPCHK(hipMemcpyAsync(R.flux, fl, L.nfaces_all * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(R.pressure, pr, L.ncells * sizeof(double), hipMemcpyDeviceToHost, s));
  }
}

void post_correct(bddc_problem *h) {
  const Layout &L = h->L;
  post_correct_rhs(h);
  k_recover_xgemv<<<dim3(L.N, nblk(L.maxC)), 256, (size_t)L.maxC * sizeof(double), h->stream>>>(
      h->g, h->Xmat, h->d_Xoff, h->rec_y, h->rec_p);
  post_correct_out(h);
}

int solve_finish_locked(bddc_problem *h);

int solve_finish(bddc_problem *h) {
  auto &R = h->run;
  while (R.checked < R.chunks) solve_poll(h, true);
  GateShared g(g_gate);
  return solve_finish_locked(h);
}

int solve_finish_locked(bddc_problem *h) {
  const Layout &L = h->L;
  hipStream_t s = h->stream;
  const int N = L.N, nGm = L.nGamma;
  auto &R = h->run;
  int iters = 0, converged = 1, fail = 0;
  double relres = 0.0;
  float pcg_ms = 0.f;
  // Everything below is enqueued behind the CG and the host waits once, at the
  // end: the CG coefficients for the condition estimate come back through
  // pinned memory (at most CG_CHUNK iterations per chunk were run).
  const bool cg = solve_needs_cg(h);
  const int it_bound = std::min(h->max_it + 1, R.chunks * CG_CHUNK + 1);
  if (cg) {
    HIPCHK(hipEventRecord(h->ev1, s));
    if (it_bound > 0) {
      double *ah = h->ab_host, *bh = h->ab_host + (h->max_it + 2);
      HIPCHK(hipMemcpyAsync(ah, h->cgw.alpha_h, it_bound * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(bh, h->cgw.beta_h, it_bound * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    // final interface flux
    k_axpby<<<nblk(nGm), 256, 0, s>>>(nGm, 1.0, h->u0, 1.0, h->xu, h->uG);
  } else if (R.upto && nGm > 0) {
    k_axpby<<<nblk(nGm), 256, 0, s>>>(nGm, 1.0, h->u0, 0.0, h->u0, h->uG);
  }
  post_correct(h);
  HIPCHK(hipStreamSynchronize(s));
  if (cg) {
    const CgState &fs = h->st_host[(R.chunks - 1) & 1];
    HIPCHK(hipEventElapsedTime(&pcg_ms, h->ev0, h->ev1));
    iters = std::min(fs.nupd, it_bound);
    converged = fs.converged;
    fail = fs.fail;
    relres = fs.relres;
    // Lanczos estimate from the CG coefficients
    std::vector<double> a(h->ab_host, h->ab_host + iters),
        b(h->ab_host + (h->max_it + 2), h->ab_host + (h->max_it + 2) + (iters > 0 ? iters - 1 : 0));
    double lmin = 1, lmax = 1;
    h->stats.kappa = lanczos_kappa(a, b, &lmin, &lmax);
    h->stats.lambda_min = lmin;
    h->stats.lambda_max = lmax;
  }
  h->stats.it = iters;
  h->stats.converged = converged;
  h->stats.relres = relres;
  h->stats.t_pcg_ms = pcg_ms;
  h->stats.t_solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - R.t0).count();
  if (fail) throw Error{BDDC_EBREAKDOWN, "CG breakdown (p^T S p <= 0 or not finite)"};
  if (!converged) return BDDC_ENOCONV;
  return BDDC_OK;
}

int do_solve(bddc_problem *h, const double *rhs, double rtol, double *flux, double *pressure, uint32_t flags) {
  solve_begin(h, rhs, rtol, flux, pressure, flags);
  if (solve_needs_cg(h)) {
    do {
      solve_chunk(h);
      solve_poll(h, true);
    } while (!h->run.stop);
  }
  return solve_finish(h);
}

// ---- block CG: several sources at once ---------------------------------------
// Workspace of the block CG, allocated at the first block solve.
void block_setup(bddc_problem *h) {
  BlockWs &B = h->blk;
  if (B.ready) return;
  const Layout &L = h->L;
  const NdPlan &P = h->nd;
  const int N = L.N;
  if ((int)h->sub_coff_h.size() != N + 1) throw Error{BDDC_EDEVICE, "coarse basis offsets missing"};
  int dev = 0, lds_max = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  int maxnc = 0;
  for (int i = 0; i < N; ++i) maxnc = std::max(maxnc, h->sub_coff_h[i + 1] - h->sub_coff_h[i]);
  const size_t nbmax = (size_t)(L.maxG + 15) / 16;
  B.psi_shm = nbmax * 16 * BK * sizeof(double) + 256 * sizeof(double);
  B.corr_shm = (size_t)((maxnc + 15) / 16) * 16 * BK * sizeof(double);
  // coarse sweep tasks of the swept levels: 64 rows / columns of a front each
  std::vector<int> tk;
  auto push = [&](int r, int j0) {
    const int64_t ro = P.r_off[r];
    const int d[12] = {j0, P.n[r], P.m[r], P.first[r], (int)P.v_off[r], P.b_off[r], P.cslot[r], 0,
                       (int)(uint32_t)(ro & 0xffffffff), (int)(uint32_t)(ro >> 32), 0, 0};
    tk.insert(tk.end(), d, d + 12);
  };
  B.tf_off.assign(P.top + 1, 0);
  B.tb_lo.assign(P.top, 0);
  B.tb_hi.assign(P.top, 0);
  for (int lv = 0; lv < P.top; ++lv) {
    for (int r = P.lvl_off[lv]; r < P.lvl_off[lv + 1]; ++r) {
      for (int j0 = 0; j0 < P.n[r] + P.m[r]; j0 += BLK_SWEEP_ROWS) push(r, j0);
    }
    B.tf_off[lv + 1] = (int)tk.size() / 12;
  }
  for (int lv = P.top - 1; lv >= 0; --lv) {
    B.tb_lo[lv] = (int)tk.size() / 12;
    for (int r = P.lvl_off[lv]; r < P.lvl_off[lv + 1]; ++r)
      for (int c0 = 0; c0 < P.n[r]; c0 += BLK_SWEEP_ROWS) push(r, c0);
    B.tb_hi[lv] = (int)tk.size() / 12;
  }
  if (std::max(B.psi_shm, B.corr_shm) > (size_t)lds_max)
    throw Error{BDDC_EINVAL, "a subdomain interface or coarse basis is too large for the block "
                             "kernels' LDS"};
  const int64_t nG = L.nGamma, totG = L.g_off[N];
  const int64_t nk = std::max(h->nk, 1), nv = std::max<int64_t>(P.v_off[P.nfr], 1),
                nbv = std::max<int64_t>(P.b_off[P.nfr], 1);
  B.task = (int4 *)h->upload(tk);
  for (double **v : {&B.ru, &B.zu, &B.pu, &B.xu, &B.qu, &B.u0}) *v = h->alloc<double>(nG * BK);
  B.yloc = h->alloc<double>(totG * BK);
  B.wloc = h->alloc<double>(totG * BK);
  B.pp = h->alloc<double>((int64_t)N * BK);
  B.xp = h->alloc<double>((int64_t)N * BK);
  B.bc = h->alloc<double>(nk * BK);
  B.cy = h->alloc<double>(nk * BK);
  B.csol = h->alloc<double>(nk * BK);
  B.S0 = h->alloc<double>(nv * BK);
  B.S1 = h->alloc<double>(nv * BK);
  B.XB = h->alloc<double>(nbv * BK);
  B.tt = h->alloc<double>((int64_t)std::max(P.nt, 1) * BK);
  B.cA = h->alloc<double>(L.ncells * BK);
  B.cB = h->alloc<double>(L.ncells * BK);
  B.part_g = h->alloc<double>((int64_t)PART_BLOCKS * BK);
  B.part_r = h->alloc<double>((int64_t)PART_BLOCKS * BK);
  B.part_z = h->alloc<double>((int64_t)PART_BLOCKS * BK);
  B.alpha_h = h->alloc<double>((int64_t)(h->max_it + 2) * BK);
  B.beta_h = h->alloc<double>((int64_t)(h->max_it + 2) * BK);
  B.st = h->alloc<CgBlockState>(1);
  fill(h, B.S0, nv * BK, 0.0);   // slots no child writes stay zero
  fill(h, B.S1, nv * BK, 0.0);
  fill(h, B.csol, nk * BK, 0.0);
  if (!h->blk_st_host) HIPCHK(hipHostMalloc((void **)&h->blk_st_host, sizeof(CgBlockState), hipHostMallocDefault));
  HIPCHK(hipStreamSynchronize(h->stream));
  B.ready = true;
}

// k_blk_symv's grid: one wave per 64-row block of the largest interface
inline dim3 blk_symv_grid(const Layout &L) { return dim3(L.N, nblk(L.maxG, 64 * BLK_SYMV_WAVES)); }

// grid of the block vector kernels (they leave one partial per block)
inline int blk_vec_blocks(int64_t n) { return (int)std::min<int64_t>(nblk(n * BK), PART_BLOCKS); }

// Z = M R for the block's columns: the steps of launch_precond, each over all
// BK columns (T^i on the side stream beside the coarse chain).
// st: the block CG state (every kernel leaves once all columns have stopped),
// or null (timing).
void launch_precond_blk(bddc_problem *h, CgBlockState *st) {
  const Layout &L = h->L;
  const NdPlan &P = h->nd;
  BlockWs &B = h->blk;
  hipStream_t s = h->stream;
  const int N = L.N;
  k_blk_fill<<<256, 256, 0, s>>>((int64_t)std::max(h->nk, 1) * BK, B.bc, 0.0, st);
  // Both forms stream the FP64 copies of T^i and Psi^i here (both copies are
  // resident): on the matrix cores the FP32 tiles, widened, loaded slower.
  k_blk_psi_apply<double><<<N, 256, B.psi_shm, s>>>(h->g, h->Psi64, h->d_psi_off, h->cs.sub_coff, h->cs.sub_cmap,
                                                   B.ru, 0.5, h->lw, B.bc, st);
  HIPCHK(hipEventRecord(h->ev_fork, s));
  // the coarse chain before T^i, as in launch_precond (it keeps the queue of
  // the node it depends on in a captured graph)
  if (h->nk > 0) {
    check_coarse_ptrs(h);
    for (int lv = 0; lv < P.top; ++lv) {
      const int t0 = B.tf_off[lv], nt = B.tf_off[lv + 1] - t0;
      if (nt > 0)
        k_blk_nd_fwd<<<nt, 256, 0, s>>>(t0, B.task, h->FR, h->sw.wdst, B.bc, B.S0, B.S1, B.cy, st);
    }
    if (P.nt > 0) {
      const int d0 = P.lvl_dof[P.top];
      k_blk_top_gather<<<nblk((int64_t)P.nt * BK), 256, 0, s>>>(P.nt, d0, h->tg_off, h->tg, B.bc, B.S0, B.S1, B.tt,
                                                                 st);
      k_blk_top_gemm<<<nblk(P.nt, 16), 64 * TOP_GEMM_WAVES, 0, s>>>(P.nt, h->top_ld, h->Kt, B.tt, d0,
                                                                     h->sw.xsc_off, h->sw.xsc, B.XB, B.csol, st);
    }
    for (int lv = P.top - 1; lv >= 0; --lv) {
      const int t0 = B.tb_lo[lv], nt = B.tb_hi[lv] - t0;
      if (nt > 0)
        k_blk_nd_bwd<<<nt, 256, 0, s>>>(t0, B.task, h->BC, B.cy, h->csgn, h->sw.xsc_off, h->sw.xsc, B.XB, B.csol,
                                        st);
    }
  }
  HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  // T^i beside the coarse chain on about two workgroups per CU (the kernel
  // loops over the subdomains), leaving room for the chain's small launches
  const int tgy = (int)nblk(L.maxG, 64 * BLK_SYMV_WAVES);
  const dim3 tgrid(std::min(L.N, std::max(2 * h->n_cu / tgy, 1)), tgy);
  k_blk_symv<double><<<tgrid, 64 * BLK_SYMV_WAVES, 0, h->side>>>(h->g, h->T64, h->d_pk, B.ru, 0.5, h->lw, B.yloc, st);
  HIPCHK(hipEventRecord(h->ev_join, h->side));
  k_blk_psi_correct<double><<<N, 256, B.corr_shm, s>>>(h->g, h->cs, h->Psi64, h->d_psi_off, B.csol, B.wloc, st);
  HIPCHK(hipStreamWaitEvent(s, h->ev_join, 0));
  k_blk_average<<<face_blocks(L.nF), 256, 0, s>>>(h->g, h->cs, B.wloc, B.yloc, B.csol, B.zu, B.ru, B.part_z, st);
}

// One block CG iteration: q = A p, alpha, x / r update, stopping test, z = M r, beta, p update.
void launch_iteration_blk(bddc_problem *h) {
  const Layout &L = h->L;
  BlockWs &B = h->blk;
  hipStream_t s = h->stream;
  const int N = L.N, nGm = L.nGamma;
  const int gv = blk_vec_blocks(nGm);
  CgBlockState *st = B.st;
  k_blk_symv<double><<<blk_symv_grid(L), 64 * BLK_SYMV_WAVES, 0, s>>>(h->g, h->Spk, h->d_pk, B.pu, 1.0, nullptr, B.yloc, st);
  k_blk_assemble<<<gv, 256, 0, s>>>(h->g, B.yloc, B.pp, h->dscale, B.pu, B.qu, B.part_g, st);
  k_blk_alpha<<<1, 256, 0, s>>>(st, B.part_g, gv, B.alpha_h);
  k_blk_update_xr<<<gv, 256, 0, s>>>(nGm, N, B.pu, B.qu, B.pp, B.xu, B.ru, B.xp, B.part_r, st);
  k_blk_test<<<1, 256, 0, s>>>(st, B.part_r, gv);
  launch_precond_blk(h, st);
  k_blk_beta<<<1, 256, 0, s>>>(st, B.part_z, face_blocks(L.nF), B.beta_h);
  k_blk_update_p<<<gv, 256, 0, s>>>(nGm, N, h->cs.pidx, B.zu, B.csol, B.pu, B.pp, st);
}

// Sources [0, k) of one block: step 1 of each (the single-source kernels),
// the reduced right-hand sides f* of all k at once (one pass over S^i and one
// over X^i), the block CG, and the post-correction (one pass over X^i for the
// k pressure right-hand sides, then the fluxes of each).  its[j], conv[j], relres[j] (each may be null) receive each source's
// CG iterations, convergence flag and final relative residual.  Returns the
// worst status of the block.
int solve_block_of(bddc_problem *h, int k, const double *rhs, double rtol, double *flux, double *pressure,
                   uint32_t flags, int32_t *its, int32_t *conv = nullptr, double *relres = nullptr) {
  const Layout &L = h->L;
  BlockWs &B = h->blk;
  const int N = L.N, nGm = L.nGamma;
  const int64_t nc = L.ncells, nf = L.nfaces_all;
  const bool dev = (flags & BDDC_DEVICE_PTRS) != 0, eager = (flags & BDDC_EAGER) != 0;
  const int gv = blk_vec_blocks(nGm);
  const auto t0 = std::chrono::steady_clock::now();
  {
    GateShared g(g_gate);
    hipStream_t s = h->stream;
    // columns k .. BK-1 (a partial block) stay zero: their f* is zero and
    // the block CG stops them at once
    fill(h, B.u0, nGm * BK, 0.0);
    if (k < BK) fill(h, B.cA, nc * BK, 0.0);
    for (int j = 0; j < k; ++j) {
      solve_begin_launch(h, rhs + j * nc, rtol, flux + j * nf, pressure + j * nc, flags, true);
      k_blk_put<<<nblk(nGm), 256, 0, s>>>(nGm, j, h->u0, B.u0);
      k_blk_src_put<<<nblk(nc), 256, 0, s>>>(nc, j, h->g.lcell_global, h->run.lsrc, B.cA);
    }
    // f* = -S u0 + H^T X F for the block's columns
    k_blk_symv<double><<<blk_symv_grid(L), 64 * BLK_SYMV_WAVES, 0, s>>>(h->g, h->Spk, h->d_pk, B.u0, 1.0, nullptr, B.yloc,
                                                             nullptr);
    k_blk_xgemm<<<dim3(N, nblk(L.maxC)), 256, 0, s>>>(h->g, h->Xmat, h->d_Xoff, B.cA, B.cB);
    LINE_LAUNCH_S(h->longl, h->mc_staged, k_blk_source_lines, N, 256, source_shm(L, h->mc_staged), s, h->g,
                  h->mcoef, B.cB, B.wloc);
    k_blk_fstar<<<nblk(nGm * BK), 256, 0, s>>>(h->g, B.yloc, B.wloc, h->d_sb, B.ru);
    for (double *v : {B.xu, B.pu}) fill(h, v, nGm * BK, 0.0);
    for (double *v : {B.xp, B.pp}) fill(h, v, (int64_t)N * BK, 0.0);
    k_blk_norm2<<<gv, 256, 0, s>>>(nGm, B.ru, B.part_r);
    k_blk_init<<<1, 256, 0, s>>>(B.st, B.part_r, gv, rtol, h->max_it);
    launch_precond_blk(h, B.st);
    k_blk_rho<<<1, 256, 0, s>>>(B.st, B.part_z, face_blocks(L.nF));
    k_blk_update_p<<<gv, 256, 0, s>>>(nGm, N, h->cs.pidx, B.zu, B.csol, B.pu, B.pp, B.st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(h->ev0, s));
  }
  if (!eager && !h->blk_graph)
    h->blk_graph = capture_graph(h, CG_CHUNK, [&] { launch_iteration_blk(h); }, "the block CG iteration graph");
  CgBlockState &fs = *h->blk_st_host;
  int chunks = 0;
  {
    GateShared g(g_gate);
    hipStream_t s = h->stream;
    for (;;) {
      if (chunks > h->max_it / CG_CHUNK + 2) throw Error{BDDC_EDEVICE, "block CG did not report completion"};
      if (eager) {
        for (int c = 0; c < CG_CHUNK; ++c) launch_iteration_blk(h);
      } else {
        HIPCHK(hipGraphLaunch(h->blk_graph, s));
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&fs, B.st, sizeof(CgBlockState), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      ++chunks;
      if (fs.done) break;
    }
    HIPCHK(hipEventRecord(h->ev1, s));
    // post-correction: the pressure right-hand sides of all sources, one
    // X^i pass for all of them, then each source's fluxes and pressures
    auto &R = h->run;
    auto set_source = [&](int j) {
      R = bddc_problem::Run();
      R.t0 = t0;
      R.dev = dev;
      R.src = rhs + j * nc;
      R.flux = flux + j * nf;
      R.pressure = pressure + j * nc;
      R.fl = dev ? R.flux : h->d_flux;
      R.pr = dev ? R.pressure : h->d_pres;
      k_blk_get<<<nblk(nGm), 256, 0, s>>>(nGm, j, B.xu, h->xu);
      k_blk_get<<<nblk(nGm), 256, 0, s>>>(nGm, j, B.u0, h->u0);
      k_axpby<<<nblk(nGm), 256, 0, s>>>(nGm, 1.0, h->u0, 1.0, h->xu, h->uG);
    };
    for (int j = 0; j < k; ++j) {   // (columns k .. BK-1 of the products are not read)
      set_source(j);
      if (!dev) {
        HIPCHK(hipMemcpyAsync(h->d_src, rhs + j * nc, nc * sizeof(double), hipMemcpyHostToDevice, s));
        R.src = h->d_src;
      }
      post_correct_rhs(h);
      k_blk_put<<<nblk(nc), 256, 0, s>>>(nc, j, h->rec_y, B.cA);
    }
    k_blk_xgemm<<<dim3(N, nblk(L.maxC)), 256, 0, s>>>(h->g, h->Xmat, h->d_Xoff, B.cA, B.cB);
    for (int j = 0; j < k; ++j) {
      set_source(j);
      k_blk_get<<<nblk(N), 256, 0, s>>>(N, j, B.xp, h->xp);
      k_blk_get<<<nblk(nc), 256, 0, s>>>(nc, j, B.cB, h->rec_p);
      post_correct_out(h);
    }
    HIPCHK(hipStreamSynchronize(s));
  }
  // statistics of the block's last source
  const int jl = k - 1;
  const int iters = fs.nupd[jl];
  std::vector<double> ah((size_t)(iters + 1) * BK), bh((size_t)(iters + 1) * BK);
  if (iters > 0) {
    GateShared g(g_gate);
    HIPCHK(hipMemcpy(ah.data(), B.alpha_h, (size_t)iters * BK * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(bh.data(), B.beta_h, (size_t)iters * BK * sizeof(double), hipMemcpyDeviceToHost));
  }
  std::vector<double> a(iters), b(iters > 0 ? iters - 1 : 0);
  for (int t = 0; t < iters; ++t) a[t] = ah[(size_t)t * BK + jl];
  for (int t = 0; t + 1 < iters; ++t) b[t] = bh[(size_t)t * BK + jl];
  double lmin = 1, lmax = 1;
  h->stats.kappa = lanczos_kappa(a, b, &lmin, &lmax);
  h->stats.lambda_min = lmin;
  h->stats.lambda_max = lmax;
  float pcg_ms = 0.f;
  HIPCHK(hipEventElapsedTime(&pcg_ms, h->ev0, h->ev1));
  h->stats.it = iters;
  h->stats.converged = fs.converged[jl];
  h->stats.relres = fs.relres[jl];
  h->stats.t_pcg_ms = pcg_ms;
  h->stats.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int rc = BDDC_OK;
  for (int j = 0; j < k; ++j) {
    if (its) its[j] = fs.nupd[j];
    if (conv) conv[j] = fs.converged[j];
    if (relres) relres[j] = fs.relres[j];
    if (fs.fail[j]) rc = BDDC_EBREAKDOWN;
    else if (!fs.converged[j] && rc == BDDC_OK) rc = BDDC_ENOCONV;
  }
  return rc;
}

// Up to BK sources on one handle (host buffers), for the request server: the
// block CG, or single solves where there is no interface to iterate on.
int block_solve_host(bddc_problem *h, int k, const double *rhs, double rtol, double *flux, double *pressure,
                     int32_t *its, int32_t *conv, double *relres) {
  if (k <= 0) return BDDC_OK;
  if (k > BK) throw Error{BDDC_EINVAL, "at most 16 sources per block"};
  const int64_t nc = h->L.ncells, nf = h->L.nfaces_all;
  if (h->L.N <= 1 || h->L.nGamma == 0) {
    int rc_all = BDDC_OK;
    for (int j = 0; j < k; ++j) {
      const int rc = do_solve(h, rhs + j * nc, rtol, flux + j * nf, pressure + j * nc, 0);
      its[j] = h->stats.it;
      conv[j] = h->stats.converged;
      relres[j] = h->stats.relres;
      if (rc != BDDC_OK) rc_all = rc;
    }
    return rc_all;
  }
  {
    GateShared g(g_gate);
    block_setup(h);
  }
  return solve_block_of(h, k, rhs, rtol, flux, pressure, 0, its, conv, relres);
}

void apply_options(bddc_problem *h, const bddc_options *opt) {
  if (opt) {
    h->precision = opt->precision;
    if (opt->max_it > 0) h->max_it = opt->max_it;
    h->flags = opt->flags;
    h->coarse_leaf = opt->coarse_leaf;
    h->coarse_top = opt->coarse_top;
    h->coarse_sub = opt->coarse_subtree;
    h->sweep_single = opt->sweep_single;
    h->t_grid = opt->t_workgroups;
    h->ms_src = opt->ms_source;
    h->bflux_in = opt->bflux;
  }
  if (h->coarse_top > TOP_MAX_DOFS) throw Error{BDDC_EINVAL, "coarse_top above 8192"};
  if (h->sweep_single < 0) throw Error{BDDC_EINVAL, "sweep_single must be >= 0"};
  if (h->precision != BDDC_FP64 && h->precision != BDDC_MIXED) throw Error{BDDC_EINVAL, "bad precision"};
}

// Device address of `scratch` on device `dev` (the current device), looked up
// once per device at the first setup on it.
void resolve_scratch(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) throw Error{BDDC_EDEVICE, "device index beyond the static scratch table"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void *p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error{BDDC_EDEVICE, "no device address for the static scratch"};
  g_scratch_ptr[dev] = p;
}

// The CG scratch of bddc_solve_noalloc, carved out of device `dev`'s copy of
// `scratch` (layout at its declaration).
CgScratch noalloc_scratch(int dev) {
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < MAX_DEVICES) base = g_scratch_ptr[dev];
  }
  if (!base) throw Error{BDDC_EDEVICE, "static scratch not resolved on the handle's device"};
  double *b = (double *)base;
  CgScratch w;
  w.st = (CgState *)b;
  w.part_g = b + 32;
  w.part_r = w.part_g + PART_BLOCKS;
  w.part_z = w.part_r + PART_BLOCKS;
  w.part_p = w.part_z + PART_BLOCKS;
  w.alpha_h = b + NOALLOC_HEAD;
  w.beta_h = w.alpha_h + NOALLOC_HIST;
  return w;
}

bddc_problem *make_problem(const bddc_grid *g, const double *perm, const bddc_partition *part, double tau,
                           const bddc_options *opt) {
  GateShared gate(g_gate);
  auto t0 = std::chrono::steady_clock::now();
  bddc_problem *h = new bddc_problem();
  try {
    apply_options(h, opt);
    h->tau = tau;
    HIPCHK(hipGetDevice(&h->device));
    resolve_scratch(h->device);
    HIPCHK(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
    h->stream = h->own_stream;
    do_setup(h, g, perm, part);
    gate.unlock();   // the autotuner captures graphs, which takes the gate exclusively
    if (h->flags & BDDC_AUTOTUNE) autotune(h);
  } catch (...) {
    if (!gate.owns_lock()) gate.lock();
    delete h;
    throw;
  }
  h->stats.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return h;
}

template <typename F>
int guarded(F &&fn) {
  try {
    return fn();
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host out of memory";
    return BDDC_ENOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return BDDC_EDEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return BDDC_EDEVICE;
  }
}

}  // namespace

extern "C" {

int bddc_setup(const bddc_grid *g, const double *perm, const bddc_partition *part, double tau,
               const bddc_options *opt, bddc_handle *out) {
  return guarded([&]() -> int {
    if (!g || !perm || !part || !out) throw Error{BDDC_EINVAL, "null argument"};
    *out = nullptr;
    *out = make_problem(g, perm, part, tau, opt);
    return BDDC_OK;
  });
}

int bddc_solve(bddc_handle h, const double *rhs, double rtol, double *flux, double *pressure, uint32_t flags) {
  return guarded([&]() -> int {
    if (!h || !rhs || !flux || !pressure) throw Error{BDDC_EINVAL, "null argument"};
    const int rc = do_solve(h, rhs, rtol, flux, pressure, flags);
    if (rc == BDDC_ENOCONV) g_last_error = "maximum number of CG iterations reached";
    return rc;
  });
}

int bddc_solve_noalloc(bddc_handle h, const double *rhs, double rtol, double *flux, double *pressure) {
  return guarded([&]() -> int {
    if (!h || !rhs || !flux || !pressure) throw Error{BDDC_EINVAL, "null argument"};
    if ((int64_t)h->max_it + 2 > NOALLOC_HIST)
      throw Error{BDDC_EINVAL, "max_it above " + std::to_string(NOALLOC_HIST - 2) +
                                   ", the CG history the static scratch holds"};
    // the handle's CG scratch is swapped for the static one for this call only
    struct Restore {
      bddc_problem *h;
      ~Restore() { h->cgw = h->cgw_own; }
    } restore{h};
    h->cgw = noalloc_scratch(h->device);
    const int rc = do_solve(h, rhs, rtol, flux, pressure, BDDC_DEVICE_PTRS | BDDC_EAGER);
    if (rc == BDDC_ENOCONV) g_last_error = "maximum number of CG iterations reached";
    return rc;
  });
}

int bddc_solve_batch(bddc_handle h, int32_t nrhs, const double *rhs, double rtol, double *flux, double *pressure,
                     uint32_t flags, int32_t *iterations) {
  return guarded([&]() -> int {
    if (!h || !rhs || !flux || !pressure || nrhs < 0) throw Error{BDDC_EINVAL, "bad argument"};
    const int64_t nc = h->L.ncells, nf = h->L.nfaces_all;
    int rc_all = BDDC_OK;
    for (int32_t k = 0; k < nrhs; ++k) {
      const int rc = do_solve(h, rhs + k * nc, rtol, flux + k * nf, pressure + k * nc, flags);
      if (iterations) iterations[k] = h->stats.it;
      if (rc == BDDC_ENOCONV) rc_all = BDDC_ENOCONV;
    }
    if (rc_all == BDDC_ENOCONV) g_last_error = "maximum number of CG iterations reached for a right-hand side";
    return rc_all;
  });
}

int bddc_solve_block(bddc_handle h, int32_t nrhs, const double *rhs, double rtol, double *flux, double *pressure,
                     uint32_t flags, int32_t *iterations) {
  return guarded([&]() -> int {
    if (!h || nrhs < 0 || (nrhs > 0 && (!rhs || !flux || !pressure))) throw Error{BDDC_EINVAL, "bad argument"};
    if (flags & (BDDC_STEP1_ONLY | BDDC_STEP12_ONLY))
      throw Error{BDDC_EINVAL, "the block solve runs whole solves (no step flags)"};
    if (!(rtol > 0.0)) throw Error{BDDC_EINVAL, "rtol must be > 0"};
    const int64_t nc = h->L.ncells, nf = h->L.nfaces_all;
    int rc_all = BDDC_OK;
    if (h->L.N <= 1 || h->L.nGamma == 0) {
      // no interface: nothing to iterate on, the solves are direct
      for (int32_t k = 0; k < nrhs; ++k) {
        const int rc = do_solve(h, rhs + k * nc, rtol, flux + k * nf, pressure + k * nc, flags);
        if (iterations) iterations[k] = h->stats.it;
        if (rc != BDDC_OK) rc_all = rc;
      }
      return rc_all;
    }
    {
      GateShared g(g_gate);
      block_setup(h);
    }
    for (int32_t b0 = 0; b0 < nrhs; b0 += BK) {
      const int k = std::min<int32_t>(BK, nrhs - b0);
      const int rc = solve_block_of(h, k, rhs + b0 * nc, rtol, flux + b0 * nf, pressure + b0 * nc, flags,
                                    iterations ? iterations + b0 : nullptr);
      if (rc == BDDC_EBREAKDOWN || (rc == BDDC_ENOCONV && rc_all == BDDC_OK)) rc_all = rc;
    }
    if (rc_all == BDDC_EBREAKDOWN) g_last_error = "CG breakdown (p^T S p <= 0 or not finite) for a right-hand side";
    if (rc_all == BDDC_ENOCONV) g_last_error = "maximum number of CG iterations reached for a right-hand side";
    return rc_all;
  });
}

int bddc_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx) {
  return guarded([&]() -> int {
    if ((alloc == nullptr) != (free_fn == nullptr)) throw Error{BDDC_EINVAL, "give both routines or neither"};
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = Allocator{alloc, free_fn, ctx};
    return BDDC_OK;
  });
}

int bddc_stats(bddc_handle h, bddc_stats_t *out) {
  return guarded([&]() -> int {
    if (!h || !out) throw Error{BDDC_EINVAL, "null argument"};
    bddc_stats_t s = h->stats;
    s.omega_tilde = h->omega_tilde;
    s.n_adaptive = h->n_adaptive;
    s.n_coarse_flux = h->ncu;
    s.n_coarse = h->ncu + h->L.N;
    s.n_sub = h->L.N;
    s.n_gamma = h->L.nGamma;
    s.n_faces = h->L.nF;
    s.precision = h->precision;
    s.coarse_levels = h->nd.H;
    s.coarse_fronts = h->nd.nfr;
    s.coarse_dense = h->nd.nt;
    s.device_bytes = h->device_bytes;
    s.sweep_wide4 = h->nd.wide4;
    s.sweep_wide16 = h->nd.wide16;
    s.t_workgroups = h->t_grid > 0 ? std::min(h->t_grid, h->L.N)
                                   : (h->precision == BDDC_MIXED && h->n_cu > 0 ? std::min(h->n_cu, h->L.N) : h->L.N);
    for (int c = 0; c < 4; ++c) {
      s.tune_coarse_ms[c] = h->tune_coarse_ms[c];
      s.tune_precond_ms[c] = h->tune_precond_ms[c];
    }
    s.sweep_subtree_levels = h->nd.sub_lv + 1;
    s.sweep_wide1 = h->nd.wide1;
    for (int c = 0; c < 4; ++c) s.tune_wide1_ms[c] = h->tune_w1_ms[c];
    static_assert(SUB_CANDS == sizeof(s.tune_subtree_ms) / sizeof(double), "subtree candidates");
    for (int c = 0; c < SUB_CANDS; ++c) s.tune_subtree_ms[c] = h->tune_sub_ms[c];
    *out = s;
    return BDDC_OK;
  });
}

int bddc_set_stream(bddc_handle h, void *stream) {
  return guarded([&]() -> int {
    if (!h) throw Error{BDDC_EINVAL, "null handle"};
    GateShared g(g_gate);
    HIPCHK(hipStreamSynchronize(h->stream));
    h->stream = stream ? (hipStream_t)stream : h->own_stream;
    return BDDC_OK;
  });
}

int bddc_destroy(bddc_handle h) {
  return guarded([&]() -> int {
    if (h) {
      GateShared g(g_gate);
      (void)hipStreamSynchronize(h->stream);
      delete h;
    }
    return BDDC_OK;
  });
}

const char *bddc_last_error(void) { return g_last_error.c_str(); }

int bddc_sizes(bddc_handle h, int64_t *out) {
  return guarded([&]() -> int {
    if (!h || !out) throw Error{BDDC_EINVAL, "null argument"};
    out[0] = h->L.N;
    out[1] = h->L.nGamma;
    out[2] = h->L.nF;
    out[3] = h->ncu;
    out[4] = h->L.ncells;
    out[5] = h->L.nfaces_all;
    out[6] = h->n_adaptive;
    out[7] = h->L.maxG;
    return BDDC_OK;
  });
}

int64_t bddc_export(bddc_handle h, int32_t what, int32_t index, void *dst, int64_t cap) {
  int64_t count = 0;
  const int rc = guarded([&]() -> int {
    if (!h || !dst) throw Error{BDDC_EINVAL, "null argument"};
    GateShared g(g_gate);
    const Layout &L = h->L;
    switch (what) {
      case BDDC_X_SCHUR: {
        if (index < 0 || index >= L.N) throw Error{BDDC_EINVAL, "bad subdomain index"};
        const int n = L.nG[index];
        count = (int64_t)n * n;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        std::vector<double> pk(gp_size(n));
        if (n > 0)
          HIPCHK(hipMemcpy(pk.data(), h->Spk + h->pk_h[index], pk.size() * sizeof(double), hipMemcpyDeviceToHost));
        double *o = (double *)dst;
        for (int c = 0; c < n; ++c)
          for (int r = c; r < n; ++r) {
            const double v = pk[gp_index(n, r, c)];
            o[r + (size_t)c * n] = v;
            o[c + (size_t)r * n] = v;
          }
        break;
      }
      case BDDC_X_T: {
        if (index < 0 || index >= L.N) throw Error{BDDC_EINVAL, "bad subdomain index"};
        const int n = L.nG[index];
        count = (int64_t)n * n;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        std::vector<double> pk(gp_size(n));
        if (n > 0)
          HIPCHK(hipMemcpy(pk.data(), h->T64 + h->pk_h[index], pk.size() * sizeof(double), hipMemcpyDeviceToHost));
        double *o = (double *)dst;
        for (int c = 0; c < n; ++c)
          for (int r = c; r < n; ++r) {
            const double v = pk[gp_index(n, r, c)];
            o[r + (size_t)c * n] = v;
            o[c + (size_t)r * n] = v;
          }
        break;
      }
      case BDDC_X_PSI: {
        if (index < 0 || index >= L.N) throw Error{BDDC_EINVAL, "bad subdomain index"};
        const int64_t nci = h->sub_coff_h[index + 1] - h->sub_coff_h[index];
        const int n = L.nG[index], ldp = ld4(n);
        count = (int64_t)n * nci;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        std::vector<double> full((size_t)ldp * nci);
        if (count > 0)
          HIPCHK(hipMemcpy(full.data(), h->Psi64 + h->psi_off_h[index], full.size() * sizeof(double),
                           hipMemcpyDeviceToHost));
        double *o = (double *)dst;
        for (int64_t c = 0; c < nci; ++c)
          for (int r = 0; r < n; ++r) o[r + c * n] = full[r + c * ldp];
        break;
      }
      case BDDC_X_COARSE_INV: {
        // columns of the flux-flux block of K^{-1}, in face-major flux order
        const int nk = h->nk, ncu = h->ncu;
        if (ncu > 4096) throw Error{BDDC_EINVAL, "coarse inverse export limited to 4096 flux dofs"};
        count = (int64_t)ncu * ncu;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        std::vector<int> fl;   // coarse indices of the flux dofs, face by face
        for (int f = 0; f < L.nF; ++f)
          for (int l = 0; l <= h->face_k[f]; ++l) fl.push_back(0);
        {
          std::vector<int> fc(L.nF);
          HIPCHK(hipMemcpy(fc.data(), h->cs.face_cofs, L.nF * sizeof(int), hipMemcpyDeviceToHost));
          int t = 0;
          for (int f = 0; f < L.nF; ++f)
            for (int l = 0; l <= h->face_k[f]; ++l) fl[t++] = fc[f] + l;
        }
        std::vector<double> e(nk), x(nk);
        double *o = (double *)dst;
        for (int c = 0; c < ncu; ++c) {
          std::fill(e.begin(), e.end(), 0.0);
          e[fl[c]] = 1.0;
          HIPCHK(hipMemcpy(h->bc, e.data(), nk * sizeof(double), hipMemcpyHostToDevice));
          launch_coarse_solve(h, h->stream, nullptr);
          HIPCHK(hipStreamSynchronize(h->stream));
          HIPCHK(hipMemcpy(x.data(), h->csol, nk * sizeof(double), hipMemcpyDeviceToHost));
          for (int r = 0; r < ncu; ++r) o[r + (size_t)c * ncu] = x[fl[r]];
        }
        break;
      }
      case BDDC_X_FACE_EIG: {
        if (index < 0 || index >= L.nF) throw Error{BDDC_EINVAL, "bad face index"};
        count = L.f_n[index] - 1;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        memcpy(dst, h->face_eig.data() + h->eig_off_h[index], count * sizeof(double));
        break;
      }
      case BDDC_X_FACE_K:
        count = L.nF;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        memcpy(dst, h->face_k.data(), count * sizeof(int));
        break;
      case BDDC_X_OMEGA:
        count = L.nF;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        memcpy(dst, h->face_omega.data(), count * sizeof(double));
        break;
      case BDDC_X_DSCALE:
        count = L.N;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        HIPCHK(hipMemcpy(dst, h->dscale, count * sizeof(double), hipMemcpyDeviceToHost));
        break;
      case BDDC_X_GAMMA: {
        count = L.nGamma;
        if (cap < count) throw Error{BDDC_EINVAL, "capacity too small"};
        int *o = (int *)dst;
        for (int g = 0; g < L.nGamma; ++g) o[g] = (int)L.gamma_face[g];
        break;
      }
      default:
        throw Error{BDDC_EINVAL, "unknown export"};
    }
    return BDDC_OK;
  });
  return rc == BDDC_OK ? count : rc;
}

int bddc_apply(bddc_handle h, int32_t which, const double *x_u, const double *x_p, double *y_u, double *y_p) {
  return guarded([&]() -> int {
    if (!h || !x_u || !y_u || !y_p) throw Error{BDDC_EINVAL, "null argument"};
    GateShared g(g_gate);
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    const int N = L.N, nGm = L.nGamma;
    if (nGm == 0) throw Error{BDDC_EINVAL, "no interface"};
    HIPCHK(hipMemcpyAsync(h->ru, x_u, nGm * sizeof(double), hipMemcpyHostToDevice, s));
    if (which == BDDC_OP_SYSTEM) {
      if (!x_p) throw Error{BDDC_EINVAL, "x_p required"};
      HIPCHK(hipMemcpyAsync(h->pp, x_p, N * sizeof(double), hipMemcpyHostToDevice, s));
      k_symv<double><<<N, SYMV_THREADS, symv_shm(L), s>>>(h->g, h->Spk, h->d_pk, h->ru, 1.0, nullptr, h->yloc, nullptr, nullptr, 0);
      k_sys_assemble<<<nblk(nGm), 256, 0, s>>>(h->g, h->yloc, h->pp, h->dscale, nullptr, h->qu, nullptr, nullptr);
      k_b0<<<N, 256, 0, s>>>(h->g, h->ru, h->dscale, h->xp);
      HIPCHK(hipMemcpyAsync(y_u, h->qu, nGm * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(y_p, h->xp, N * sizeof(double), hipMemcpyDeviceToHost, s));
    } else if (which == BDDC_OP_PRECOND) {
      launch_precond(h, h->ru, h->zu, nullptr, false);
      HIPCHK(hipMemcpyAsync(y_u, h->zu, nGm * sizeof(double), hipMemcpyDeviceToHost, s));
      std::vector<double> c(h->nk + 1, 0.0);
      if (h->nk > 0) HIPCHK(hipMemcpyAsync(c.data(), h->csol, h->nk * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int i = 0; i < N; ++i) y_p[i] = (h->pidx_h[i] >= 0) ? c[h->pidx_h[i]] : 0.0;
    } else {
      throw Error{BDDC_EINVAL, "unknown operator"};
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return BDDC_OK;
  });
}

int bddc_time_kernel(bddc_handle h, int32_t which, int32_t reps, double *avg_ms, double *bytes) {
  return guarded([&]() -> int {
    if (!h || !avg_ms || !bytes || reps <= 0) throw Error{BDDC_EINVAL, "bad argument"};
    if (which == BDDC_K_PRECOND_FULL) {
      // as the solve runs it: applies replayed from a graph
      *avg_ms = time_graph_ms(h, reps, [&] { launch_precond(h, h->ru, h->zu, nullptr, false); },
                              "the preconditioner");
      *bytes = h->stats.bytes_prec;
      return BDDC_OK;
    }
    if (which >= BDDC_K_BLOCK_SCHUR && which <= BDDC_K_BLOCK_PRECOND_FULL && !h->blk.ready)
      throw Error{BDDC_EINVAL, "no block solve has run on this handle"};
    if (which == BDDC_K_BLOCK_PRECOND_FULL) {
      *avg_ms = time_graph_ms(h, reps, [&] { launch_precond_blk(h, nullptr); }, "the block preconditioner");
      *bytes = h->stats.bytes_prec_block;
      return BDDC_OK;
    }
    GateShared g(g_gate);
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    const int N = L.N;
    if (L.nGamma == 0) throw Error{BDDC_EINVAL, "no interface"};
    double pk = 0.0;
    for (int i = 0; i < N; ++i) pk += (double)L.nG[i] * (L.nG[i] + 1) / 2;
    const double totG = (double)L.g_off[N];
    const double sT = h->precision == BDDC_MIXED ? 4.0 : 8.0;
    double b = 0.0;
    const BlockWs &B = h->blk;
    auto launch = [&]() {
      if (which == BDDC_K_BLOCK_SCHUR)
        k_blk_symv<double><<<blk_symv_grid(L), 64 * BLK_SYMV_WAVES, 0, s>>>(h->g, h->Spk, h->d_pk, B.pu, 1.0, nullptr, B.yloc, nullptr);
      else if (which == BDDC_K_BLOCK_PRECOND_APPLY)
        k_blk_symv<double><<<blk_symv_grid(L), 64 * BLK_SYMV_WAVES, 0, s>>>(h->g, h->T64, h->d_pk, B.ru, 0.5, h->lw, B.yloc, nullptr);
      else if (which == BDDC_K_SCHUR_APPLY)
        k_symv<double><<<N, SYMV_THREADS, symv_shm(L), s>>>(h->g, h->Spk, h->d_pk, h->pu, 1.0, nullptr, h->yloc, nullptr, nullptr, 0);
      else if (h->precision == BDDC_MIXED)
        k_symv<float><<<N, SYMV_THREADS, symv_shm(L), s>>>(h->g, h->T32, h->d_pk, h->ru, 0.5, h->lw, h->yloc, nullptr, nullptr, 0);
      else
        k_symv<double><<<N, SYMV_THREADS, symv_shm(L), s>>>(h->g, h->T64, h->d_pk, h->ru, 0.5, h->lw, h->yloc, nullptr, nullptr, 0);
    };
    // algorithmic bytes: the lower triangles, the gather map and gathered x, y
    if (which == BDDC_K_SCHUR_APPLY)
      b = pk * 8.0 + totG * (4.0 + 8.0) + totG * 8.0;
    else if (which == BDDC_K_PRECOND_APPLY)
      b = pk * sT + totG * (4.0 + 8.0) + totG * 8.0;
    else if (which == BDDC_K_BLOCK_SCHUR)
      b = pk * 8.0 + totG * (4.0 + 8.0 * BK) + totG * 8.0 * BK;
    else if (which == BDDC_K_BLOCK_PRECOND_APPLY)
      b = pk * 8.0 + totG * (4.0 + 8.0 * BK) + totG * 8.0 * BK;
    else
      throw Error{BDDC_EINVAL, "unknown kernel"};
    launch();
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(h->ev0, s));
    for (int r = 0; r < reps; ++r) launch();
    HIPCHK(hipEventRecord(h->ev1, s));
    HIPCHK(hipEventSynchronize(h->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    *avg_ms = ms / reps;
    *bytes = b;
    return BDDC_OK;
  });
}

}  // extern "C"

#include "server.hpp"
