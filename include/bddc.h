/*
 * bddc.h -- C ABI of the MI355X (gfx950) adaptive BDDC solver for the mixed
 * RT0/P0 Darcy problem.
 *
 * Method: B. Sousedik, "On adaptive BDDC for the flow in heterogeneous porous
 * media".  The library solves the saddle-point system of Section 2
 * (eqs. variational-1/2; matrix form eq. system, rescaled as eq. system-scaled)
 * by Algorithm "BDDC method": a coarse solve (step 1), independent subdomain
 * solves (step 2) and conjugate gradients on the divergence-free correction
 * (step 3) preconditioned by Algorithm "BDDC preconditioner", with the flux
 * coarse space enriched by Algorithm "Adaptive BDDC" (Section 4, eqs.
 * eigenvalue-problem-local-matrix and constraints).
 *
 * Data conventions (all entry points):
 *   - cells are numbered x-fastest: c = ix + nx*(iy + ny*iz);
 *   - a flux unknown is the total normal flux through one grid face, oriented
 *     along +x/+y/+z.  Faces are numbered direction by direction (all x-faces,
 *     then y-faces, then z-faces); inside direction d the face with integer
 *     position (i0,i1,i2), i_d in [0, n_d], has index i0 + s0*(i1 + s1*i2)
 *     with s_e = n_e + (e == d).  Boundary faces are included; they carry
 *     zero flux (no-flow boundary, Section 2) unless bddc_options.bflux
 *     prescribes their fluxes (eq. problem-4);
 *   - the source is cell integrated (injection > 0) and must sum to zero
 *     (eq. compatibility with g_E = 0), or to the net boundary outflow.
 *
 * Ownership: input arrays are read during the call only.  The handle owns all
 * device memory it allocates; it is released by bddc_destroy.  A handle is not
 * thread safe; distinct handles are independent.
 *
 * Errors: every entry point returns BDDC_OK (0) or a negative code; the
 * message of the last failure on the calling thread is bddc_last_error().
 * No C++ exception crosses this interface.
 */
#ifndef BDDC_H
#define BDDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BDDC_OK          0
#define BDDC_EINVAL     -1   /* bad shape, partition, permeability or source   */
#define BDDC_ENOMEM     -2   /* device memory could not be obtained            */
#define BDDC_ENOCONV    -3   /* max_it reached; outputs hold the last iterate  */
#define BDDC_EBREAKDOWN -4   /* CG breakdown: p^T S p <= 0 or not finite       */
#define BDDC_EFACTOR    -5   /* a local or coarse factorization lost definiteness */
#define BDDC_EDEVICE    -6   /* HIP runtime error                              */
#define BDDC_EBUSY      -7   /* server request still pending                   */

/* precision of the preconditioner (the CG recurrences and S are always FP64) */
#define BDDC_FP64  0
#define BDDC_MIXED 1         /* T^i and Psi^i stored and streamed in FP32      */

/* bddc_options.flags */
#define BDDC_ALL_CONSTRAINED 1u  /* diagnostic: every interface dof is a coarse dof */
#define BDDC_MULTISCALE 4u       /* multiscale constraints (Section 6) in place of
                                    the face eigenproblems, tau unused: each face
                                    gets one row, its fluxes in the Darcy problem
                                    on the two neighbours with a unit source /
                                    sink (uniform, or shaped by the well source
                                    bddc_options.ms_source) and no flow on their
                                    other faces, projected off the zero-net-flux
                                    row (none when that flux is uniform)         */
#define BDDC_AUTOTUNE 16u        /* at the end of bddc_setup, time candidate launch
                                    shapes of the per-iteration kernels on the
                                    problem's own operators and keep the fastest:
                                    the lane-group widths of the coarse sweeps
                                    (coarse solve timed) and the workgroups of
                                    the T^i corrections beside it (whole
                                    preconditioner timed); see bddc_stats_t    */
#define BDDC_STIFFNESS_SCALING 8u /* averaging weights a_i / (a_i + a_j) per face,
                                    a_s the mean diagonal of A^s over the face
                                    (rho-scaling for RT0; the paper's choice when
                                    coefficient jumps follow the interfaces) in
                                    place of 1/2; needs tau off (or multiscale):
                                    BDDC_EINVAL otherwise                        */

/* bddc_solve flags */
#define BDDC_DEVICE_PTRS 1u      /* rhs, flux and pressure are device pointers   */
#define BDDC_EAGER       2u      /* launch the CG iterations kernel by kernel
                                    instead of replaying the captured graph     */
#define BDDC_STEP1_ONLY  4u      /* return u_0 of step 1 (see bddc_solve)        */
#define BDDC_STEP12_ONLY 8u      /* return u^* of steps 1-2 (see bddc_solve)     */

typedef struct bddc_problem *bddc_handle;

/* Cartesian grid: dim 2 or 3, cells per axis n[0..dim), cell size h[0..dim). */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double h[3];
} bddc_grid;

/* Box partition by axis cut planes: cuts[d] has nsub[d]+1 increasing entries,
 * cuts[d][0] = 0 and cuts[d][nsub[d]] = n[d] (Section 6, regular partitions). */
typedef struct {
  int32_t nsub[3];
  const int32_t *cuts[3];
} bddc_partition;

typedef struct {
  int32_t precision;     /* BDDC_FP64 or BDDC_MIXED                          */
  int32_t max_it;        /* CG iteration cap (<= 0: 10000)                    */
  uint32_t flags;        /* BDDC_ALL_CONSTRAINED (diagnostic)                 */
  int32_t coarse_leaf;   /* nested dissection of the coarse problem stops at
                            boxes of at most this many subdomains (<= 0: 1) */
  int32_t coarse_top;    /* the top levels of the coarse tree holding at most
                            this many coarse dofs are solved with the explicit
                            inverse of their Schur complement, formed at setup
                            (0: 4096; < 0: none; at most 8192)             */
  int32_t t_workgroups;  /* workgroups of the substructure corrections T^i,
                            which run beside the coarse solve; fewer leave
                            more memory bandwidth to its latency-bound
                            sweeps (<= 0 or > N: one per subdomain)        */
  const double *ms_source; /* with BDDC_MULTISCALE: host array [n_cells], the
                            cell-integrated well source that shapes the
                            multiscale sources (Section 6): a subdomain whose
                            source is not zero uses w = f / (its sum of f),
                            the others 1/|Omega^i| (as does a subdomain whose
                            wells cancel); NULL: uniform everywhere.  Read
                            during bddc_setup only                         */
  const double *bflux;    /* host array [n_faces_all] (global face numbering and
                            orientation): the prescribed normal fluxes of the
                            boundary faces (eq. problem-4; interior entries
                            are ignored); NULL: no flow.  Every solve on the
                            handle uses them; its source must then sum to
                            the net outflow through the boundary instead of
                            zero, and the boundary entries of the flux
                            output carry them.  Read during bddc_setup only */
  int32_t coarse_subtree; /* the bottom levels 0 .. coarse_subtree - 1 of the
                            coarse tree (below the dense top block) are swept
                            by one launch per direction, one workgroup per
                            subtree (0: the library's default; < 0: one
                            launch per level).  BDDC_AUTOTUNE times 0 .. 6
                            levels and keeps the fastest                   */
  int32_t sweep_single;   /* coarse sweeps: rows and columns of at most this
                            many entries are taken by one lane each (0:
                            none).  BDDC_AUTOTUNE times 0, 8, 16, 32        */
} bddc_options;

typedef struct {
  int32_t it;               /* CG iterations of the last solve                  */
  int32_t converged;        /* 1 if ||r|| <= rtol ||r_0||                        */
  double relres;            /* final ||r|| / ||r_0||                             */
  double kappa;             /* Lanczos condition estimate (Section 6)            */
  double lambda_min, lambda_max;
  double omega_tilde;       /* eq. indicator (0 without adaptivity)              */
  int32_t n_adaptive;       /* adaptive flux constraints added                   */
  int32_t n_coarse_flux;    /* flux coarse dofs                                  */
  int32_t n_coarse;         /* n_c = flux coarse dofs + N (Table 1 column n_c)   */
  int32_t n_sub;            /* N                                                 */
  int32_t n_gamma;          /* interface flux dofs                               */
  int32_t n_faces;          /* subdomain faces                                   */
  int32_t precision;
  int32_t coarse_levels;    /* levels of the coarse multifrontal factorization   */
  int32_t coarse_fronts;    /* fronts (separators and leaf boxes) of it          */
  int32_t coarse_dense;     /* coarse dofs of the dense top block (0: none)      */
  double t_setup_ms;        /* wall time of bddc_setup                           */
  double t_solve_ms;        /* wall time of the last bddc_solve                  */
  double t_pcg_ms;          /* device time of the CG loop of the last solve      */
  double bytes_per_iter;    /* algorithmic HBM bytes of one CG iteration         */
  double bytes_prec;        /* ... of which the BDDC preconditioner              */
  double device_bytes;      /* device memory held by the handle                  */
  int32_t sweep_wide4;      /* coarse sweeps: rows / columns up to this long take
                               4 lanes, up to sweep_wide16 16, longer 64       */
  int32_t sweep_wide16;
  int32_t t_workgroups;     /* workgroups of the T^i launch                      */
  double t_tune_ms;         /* wall time of the autotuner (0: not run)           */
  double tune_coarse_ms[4]; /* coarse solve with widths (8,32) (12,48) (24,96)
                               (48,192)                                         */
  double tune_precond_ms[4];/* preconditioner with T^i on 3 n_cu/4, n_cu, 2 n_cu, N
                               workgroups (n_cu: compute units)                 */
  double bytes_prec_block;  /* algorithmic bytes of one block preconditioner
                               apply (16 columns; 0 before a block solve)      */
  double flops_block_local; /* 2 * 16 * sum n_Gamma^i^2: the flops of one block
                               product with S^i or T^i (16 columns)             */
  int32_t sweep_subtree_levels; /* coarse sweeps: levels 0 .. this - 1 are swept
                               by one launch per direction, one workgroup per
                               bottom subtree (0: one launch per level)        */
  int32_t sweep_wide1;      /* coarse sweeps: rows / columns up to this long take
                               one lane (0: none)                               */
  double tune_subtree_ms[7];/* coarse solve with bottom subtrees of 0 .. 6
                               levels (0 where not timed)                       */
  double tune_wide1_ms[4];  /* coarse solve with single-lane rows up to 0, 8,
                               16, 32 entries (0 where not timed)               */
} bddc_stats_t;

/*
 * Build everything the solve needs, on the device: local RT0 coefficients and
 * the rescaling D (Section 5), the interface Schur complements S^i and the
 * pressure operators of every subdomain, the pair eigenproblems and adaptive
 * constraints of every face (Section 4, threshold tau; tau <= 0 or infinite
 * disables adaptivity), the local coarse bases Psi^i, the substructure
 * operators T^i and the coarse saddle point (Section 3, Algorithm "BDDC
 * preconditioner").
 *   g     : grid (dim 2|3, n[d] >= 1, h[d] > 0)
 *   perm  : host array [n_cells][dim], diagonal permeability, finite and > 0
 *   part  : box partition; every axis interval must be non-empty
 *   opt   : NULL for defaults (FP64, max_it 10000)
 *   out   : receives the handle on success
 * Returns BDDC_EINVAL on bad input, BDDC_ENOMEM, BDDC_EFACTOR, BDDC_EDEVICE.
 */
int bddc_setup(const bddc_grid *g, const double *perm, const bddc_partition *part,
               double tau, const bddc_options *opt, bddc_handle *out);

/*
 * Solve with the given source (Algorithm "BDDC method", steps 1-3 and the
 * post-correction of interiors).  CG stops when ||r||_2 <= rtol ||r_0||_2.
 *   rhs      : [n_cells] cell-integrated source, sum within 1e-12 sum|rhs| of 0
 *   flux     : [n_faces_all] output, global orientation, boundary faces = 0
 *   pressure : [n_cells] output, zero volume-weighted mean
 *   flags    : BDDC_DEVICE_PTRS if the three arrays live in device memory
 *              (then the call is asynchronous on the handle's stream except for
 *              the convergence checks of the CG loop); BDDC_EAGER to launch the
 *              CG iterations one kernel at a time.  By default the first solve
 *              captures a chunk of eight CG iterations (both streams) into a
 *              HIP graph that later chunks and solves replay; both ways run
 *              the same kernels on the same data and give identical results.
 *              BDDC_STEP1_ONLY / BDDC_STEP12_ONLY (at most one of the two) stop
 *              before the CG and return the approximations whose errors the
 *              paper reports as epsilon_0 and epsilon^* (eq. epsilon, Section 6):
 *              u_0 = E Psi alpha_0 on the interface, continued into every
 *              subdomain by the local saddle point with zero source (the
 *              coarse solution of step 1), or u^* = u_0 plus the substructure
 *              components of step 2 (the local saddle points with the source
 *              and interface flux u_0).  The pressure output is that of the
 *              same local problems.  Statistics report 0 iterations.
 * Returns BDDC_OK, BDDC_ENOCONV (outputs hold the last iterate),
 * BDDC_EBREAKDOWN, BDDC_EINVAL, BDDC_EDEVICE.
 */
int bddc_solve(bddc_handle h, const double *rhs, double rtol, double *flux, double *pressure,
               uint32_t flags);

/* Statistics of the setup and of the last solve. */
int bddc_stats(bddc_handle h, bddc_stats_t *out);

/* Run all later work of this handle on the given hipStream_t (NULL: the
 * handle's own stream).  The stream must outlive its use by the handle. */
int bddc_set_stream(bddc_handle h, void *hip_stream);

/* Release all device memory of the handle.  NULL is accepted. */
int bddc_destroy(bddc_handle h);

/* Thread-local message describing the last non-zero return on this thread. */
const char *bddc_last_error(void);

/* ---- diagnostics used by the parity tests ----------------------------------
 * Sizes of the problem: out[0..8) = {N, n_gamma, n_faces, n_coarse_flux,
 * n_cells, n_faces_all, n_adaptive, max n_gamma^i}. */
int bddc_sizes(bddc_handle h, int64_t *out);

/* Copy an internal array to host memory (FP64 unless stated).
 *   what = BDDC_X_SCHUR     : S^i of subdomain `index`, dense n x n column major
 *          BDDC_X_FACE_EIG  : eigenvalues (descending) of face `index`'s
 *                             reduced pair problem, n_F - 1 values
 *          BDDC_X_FACE_K    : int32 adaptive row count of every face
 *          BDDC_X_DSCALE    : rescaling d_i of every subdomain
 *          BDDC_X_GAMMA     : int32 global face index of every interface dof
 *          BDDC_X_OMEGA     : omega^F of every face
 *          BDDC_X_T         : T^i of subdomain `index` (FP64 form), dense n x n
 *          BDDC_X_PSI       : Psi^i of subdomain `index`, n_gamma^i x n_c^i column major
 *          BDDC_X_COARSE_INV: flux-flux block of the coarse saddle-point
 *                             inverse, n_coarse_flux^2 column major
 * `cap` is the capacity of dst in elements; returns the element count or a
 * negative code. */
#define BDDC_X_SCHUR    1
#define BDDC_X_FACE_EIG 2
#define BDDC_X_FACE_K   3
#define BDDC_X_DSCALE   4
#define BDDC_X_GAMMA    5
#define BDDC_X_OMEGA    6
#define BDDC_X_T        7
#define BDDC_X_PSI      8
#define BDDC_X_COARSE_INV 9
int64_t bddc_export(bddc_handle h, int32_t what, int32_t index, void *dst, int64_t cap);

/* Apply one operator of the CG iteration to host vectors of the interface
 * problem (eqs. corr-reduced-1/2):
 *   which = BDDC_OP_SYSTEM : (y_u, y_p) = (S x_u + B_0^T x_p, B_0 x_u)
 *           BDDC_OP_PRECOND: (y_u, y_p) = BDDC preconditioner applied to (x_u, 0)
 * x_u, y_u: [n_gamma]; x_p, y_p: [N] (pressures in the rescaled variable). */
#define BDDC_OP_SYSTEM  1
#define BDDC_OP_PRECOND 2
int bddc_apply(bddc_handle h, int32_t which, const double *x_u, const double *x_p, double *y_u,
               double *y_p);

/* Solve nrhs sources on the resident problem, one after the other with the
 * captured CG iterations (each result equals that of bddc_solve on the same
 * source, bit for bit).  rhs [nrhs][n_cells], flux [nrhs][n_faces_all],
 * pressure [nrhs][n_cells], host or (BDDC_DEVICE_PTRS) device pointers;
 * iterations [nrhs] receives each CG count (may be NULL).  Returns BDDC_OK,
 * BDDC_ENOCONV if some source reached max_it (all are still solved), or the
 * first error, which stops the batch.  Statistics are those of the last
 * source. */
int bddc_solve_batch(bddc_handle h, int32_t nrhs, const double *rhs, double rtol, double *flux, double *pressure,
                     uint32_t flags, int32_t *iterations);

/* Several sources solved together (Algorithm "BDDC method" for each): steps
 * 1-2, the reduced right-hand side and the post-correction run source by
 * source, and step 3's CG runs for blocks of up to 16 sources at once.  Each
 * source keeps its own CG scalars and stopping test, so it takes the
 * iterations of its single solve, while every block iteration streams S^i,
 * T^i, Psi^i, the swept coarse factor and S_t^{-1} once for all 16 columns:
 * the local operators and bases as 16 x 16 tiles on the FP64 matrix cores
 * against the block's columns (a partial block is padded with zero sources,
 * which stop at once).  Both forms stream the FP64 copies of T^i and Psi^i
 * (resident in both): widened FP32 tiles loaded slower on the matrix cores.
 * The results equal those of bddc_solve to rounding (the block kernels add in
 * another order; in the mixed form, also the FP64 operators).  Arguments as bddc_solve_batch
 * (BDDC_DEVICE_PTRS and BDDC_EAGER apply; the step flags are refused with
 * BDDC_EINVAL).  The first call allocates the block's vectors (16 copies of
 * the interface, local and coarse vectors, about 2 GB on the 60x220x85
 * reservoir).  BDDC_EINVAL too if a subdomain's interface (over 1,232 dofs)
 * or coarse basis does not fit the block kernels' LDS.  Returns BDDC_OK,
 * BDDC_ENOCONV if a source reached max_it, BDDC_EBREAKDOWN if a source's CG
 * broke down (all sources are still solved), or the first error.  Statistics
 * are those of the last source. */
int bddc_solve_block(bddc_handle h, int32_t nrhs, const double *rhs, double rtol, double *flux, double *pressure,
                     uint32_t flags, int32_t *iterations);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): bddc_solve with
 * BDDC_DEVICE_PTRS | BDDC_EAGER semantics that calls no hipMalloc, hipFree or
 * allocating routine.  rhs [n_cells], flux [n_faces_all] and pressure
 * [n_cells] are device pointers owned by the caller; the result equals that of
 * bddc_solve on the same source.  The CG scratch (dot-product partials, the
 * device CG state, the alpha / beta history of the condition estimate) lives
 * in a static 512 KiB device array of the library, one per device, instead of
 * the handle's own arrays; every other array the solve uses was allocated by
 * bddc_setup.  The array is shared by every call on the device and keeps the
 * last call's contents (each call initialises what it reads): calls that
 * overlap on one device race, also across handles.  The handle's max_it must
 * be at most 31,854 (the history the array holds): BDDC_EINVAL otherwise.
 * Returns as bddc_solve; statistics are those of this solve. */
int bddc_solve_noalloc(bddc_handle h, const double *rhs, double rtol, double *flux, double *pressure);

/* Device memory of every handle set up afterwards comes from alloc(bytes,
 * ctx) and goes back through free(ptr, ctx) (for instance a framework's
 * caching allocator); both NULL restore hipMalloc / hipFree.  The routines
 * must be thread-safe when a server runs (its setup workers allocate).  An
 * allocation is released through the routine it came from, whatever is set
 * later.  Host-only; BDDC_EINVAL if only one routine is given. */
int bddc_set_allocator(void *(*alloc)(size_t, void *), void (*free)(void *, void *), void *ctx);

/* Time one kernel of the CG iteration on the handle's stream with HIP events:
 * `reps` back-to-back launches on the vectors of the last solve, bracketed by
 * two events.  which = BDDC_K_SCHUR_APPLY (local Schur products S^i of the
 * CG operator), BDDC_K_PRECOND_APPLY (local substructure corrections T^i of
 * the preconditioner) or BDDC_K_PRECOND_FULL (the whole preconditioner of
 * Algorithm "BDDC preconditioner" as one CG iteration applies it: coarse
 * right-hand sides Psi^{iT} r^i, the corrections T^i r^i beside the coarse
 * solve, the coarse correction Psi^i alpha and the weighted averaging; one
 * "launch" is that sequence of kernels on two streams, timed as the solve
 * runs it: eight applies captured into a HIP graph on the handle's own
 * stream, the graph replayed ceil(reps / 8) times on the handle's stream).
 * avg_ms receives the mean duration of one launch, bytes the algorithmic HBM
 * bytes of one launch (operator entries read once, vectors gathered and
 * written once).  Call after a bddc_solve. */
#define BDDC_K_SCHUR_APPLY   1
#define BDDC_K_PRECOND_APPLY 2
#define BDDC_K_PRECOND_FULL  3
/* The block CG's kernels (after a bddc_solve_block; BDDC_EINVAL before), on
 * the last block's vectors: the local Schur products S^i for 16 columns
 * (BDDC_K_BLOCK_SCHUR), the local corrections T^i for 16 columns
 * (BDDC_K_BLOCK_PRECOND_APPLY), and the whole block preconditioner as a
 * graph replay (BDDC_K_BLOCK_PRECOND_FULL).  bytes: each operator entry once,
 * the gather map, 16 gathered and 16 written values per local dof; the
 * matrix-core flops of the first two are in bddc_stats_t.flops_block_local. */
#define BDDC_K_BLOCK_SCHUR         4
#define BDDC_K_BLOCK_PRECOND_APPLY 5
#define BDDC_K_BLOCK_PRECOND_FULL  6
int bddc_time_kernel(bddc_handle h, int32_t which, int32_t reps, double *avg_ms, double *bytes);

/* Device bytes a problem may hold at the peak of its setup (the figure the
 * server admits requests by).  Every array fixed by the grid and partition is
 * counted exactly; the adaptive rows of a face are unknown before its
 * eigenproblem and are taken as min(n_F - 1, 8) when tau is finite (none
 * otherwise), which also fixes the coarse plan the estimate is built on.
 * Host-only; opt may be NULL.  Returns BDDC_OK or BDDC_EINVAL. */
int bddc_estimate_bytes(const bddc_grid *g, const bddc_partition *part, double tau, const bddc_options *opt,
                        double *bytes);

/* ------------------------------------------------------------------------
 * Serving: a request loop over independent problems (own grid, permeability,
 * partition, tau and source each), with continuous batching.  Requests are
 * admitted in arrival order while fewer than max_active are set up or
 * solving and their estimated bytes (bddc_estimate_bytes) fit under mem_cap
 * next to what the admitted ones hold (after its setup a problem counts with
 * the bytes it actually holds).  Setup runs on worker threads, beside the CG
 * iterations of the requests already solving; a driver thread advances every
 * solving request by captured chunks of CG iterations on its own streams, so
 * the requests' kernels overlap on the device, and a request that finishes
 * frees its memory and slot for the next.  Every request's arithmetic is that
 * of bddc_solve on its own handle: its result does not depend on the mix.
 *
 * Resident problems and batched solves: requests that carry the same nonzero
 * problem_key name one problem (the caller promises equal permeability; the
 * server checks grid, partition and tau, and the source's compatibility at
 * submission, BDDC_EINVAL otherwise).  The first
 * one is admitted and set up like any request; its problem then stays
 * resident (its bytes count against mem_cap) and later requests of the key
 * skip the setup.  The requests of a key that are waiting together (up to 16,
 * equal rtol) are solved as one block of bddc_solve_block: one pass over the
 * problem's operators per CG iteration serves all of them, and each result
 * equals its own single solve to rounding.  An idle resident problem is
 * released when a queued request needs its memory, or at
 * bddc_server_destroy.
 * ------------------------------------------------------------------------ */
typedef struct bddc_server *bddc_server_handle;

typedef struct {
  double mem_cap;         /* device bytes the admitted problems may hold
                             (<= 0: 90% of the free device memory at create) */
  int32_t max_active;     /* problems set up or solving at once (<= 0: 4)   */
  int32_t setup_workers;  /* host threads running setups (<= 0: 1)          */
  int32_t precision;      /* BDDC_FP64 or BDDC_MIXED, for every request     */
  uint32_t flags;         /* bddc_options flags for every request           */
} bddc_server_options;

typedef struct {
  bddc_grid grid;
  const double *perm;     /* [n_cells][dim], as for bddc_setup; copied       */
  bddc_partition part;    /* cuts copied                                    */
  double tau;             /* as for bddc_setup                              */
  const double *rhs;      /* [n_cells] cell sources summing to 0; copied     */
  double rtol;            /* > 0                                            */
  int32_t max_it;         /* <= 0: 10000 (a keyed problem keeps its first)  */
  uint64_t problem_key;   /* 0: an independent problem; else see above      */
} bddc_request;

typedef struct {
  int32_t status;         /* BDDC_OK, BDDC_ENOCONV or the error code        */
  int32_t it, converged;
  double relres, kappa;
  int32_t n_sub, n_coarse;
  double queue_ms;        /* submit to admission                            */
  double setup_ms;        /* setup and the solve's start                    */
  double solve_ms;        /* CG and post-correction, after the setup        */
  double latency_ms;      /* submit to completion                           */
  double est_bytes;       /* admission estimate                             */
  double device_bytes;    /* bytes the problem held while solving           */
  double peak_bytes;      /* high-water mark during its setup               */
  int32_t batch;          /* sources solved together with it (1: alone)     */
  int32_t reused;         /* 1: its problem was resident (no setup)         */
} bddc_request_stats;

typedef struct {
  int64_t submitted, completed, failed, queued, active;
  int32_t peak_active;    /* most problems set up or solving at once        */
  double p50_ms, p99_ms;  /* latency percentiles of the completed requests  */
  double solves_per_s;    /* completed / (last completion - first submit)   */
  double peak_bytes;      /* most bytes counted against mem_cap at once     */
  double mem_cap;
} bddc_server_stats_t;

/* Start the scheduler threads on the current device. */
int bddc_server_create(const bddc_server_options *opt, bddc_server_handle *out);
/* Queue a request (its arrays are copied; the call does not wait for the GPU).
 * BDDC_EINVAL for a bad request, BDDC_ENOMEM if its estimate exceeds mem_cap. */
int bddc_server_submit(bddc_server_handle s, const bddc_request *req, uint64_t *ticket);
/* Wait up to wait_ms (< 0: no limit) for a request.  While it is pending:
 * BDDC_EBUSY.  Once done: copies flux [n_faces_all] and pressure [n_cells]
 * (host arrays, either may be NULL) and its statistics (may be NULL), releases
 * the ticket and returns the request's status. */
int bddc_server_poll(bddc_server_handle s, uint64_t ticket, double wait_ms, double *flux, double *pressure,
                     bddc_request_stats *st);
int bddc_server_stats(bddc_server_handle s, bddc_server_stats_t *out);
/* Drop the queued requests, finish the admitted ones, stop the threads. */
int bddc_server_destroy(bddc_server_handle s);

#ifdef __cplusplus
}
#endif
#endif /* BDDC_H */
