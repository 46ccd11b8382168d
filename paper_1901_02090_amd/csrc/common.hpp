// Device-visible descriptions shared by the setup and solve kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bddc {

// Kernels that solve along lines of subdomain cells keep a line in private
// arrays; they come in two instances, for extents up to SHORTLINE cells (all
// boxes of the benchmarks) and up to MAXLINE, the longest subdomain extent
// along one axis that the library accepts.
constexpr int SHORTLINE = 32;
constexpr int MAXLINE = 128;

// Group-aligned packed storage of a symmetric n x n matrix (lower triangle).
// Columns come in groups of four; group g holds its four columns over rows
// 4g .. 4G-1 (G = ceil(n/4)), each column contiguous with length 4(G-g).
// Entries above the diagonal inside a group and rows >= n are zero.  Every
// column of a group starts at the same row and on a 16-byte boundary, so a
// wavefront reads four columns with 16-byte vector loads, contiguous across
// lanes.  Size 8 G (G+1) (n(n+1)/2 plus O(n) padding).
__host__ __device__ inline int64_t gp_size(int n) {
  const int64_t G = (n + 3) / 4;
  return 8 * G * (G + 1);
}
__host__ __device__ inline int64_t gp_group(int n, int g) {
  const int64_t G = (n + 3) / 4;
  return 16 * ((int64_t)g * G - (int64_t)g * (g - 1) / 2);
}
__host__ __device__ inline int64_t gp_index(int n, int r, int c) {
  const int64_t G = (n + 3) / 4;
  const int g = c / 4, q = c % 4;
  return gp_group(n, g) + (int64_t)q * 4 * (G - g) + (r - 4 * g);
}
// Leading dimension of the coarse bases Psi^i: rows padded to a multiple of 4.
__host__ __device__ inline int ld4(int n) { return (n + 3) & ~3; }

// Read-only index data of the partition (device pointers).
struct DevGeom {
  int dim;
  int n[3];
  double h[3];
  double vol;                 // cell volume (C_Q^i entries)
  int N, nGamma, nF;
  int fshape[3][3];
  int64_t face_off[4];
  const int *lo, *ext;        // [N][3]
  const int *nc, *nG;         // [N]
  const int64_t *cell_off, *g_off;  // [N+1]
  const int *lcell_global;    // [sum nc]
  const int *lg_dir, *lg_cell, *lg_end, *lg_partner;  // [sum nG]
  const int *Rmap;            // [sum nG] -> interface index
  const int *own_minus, *own_plus, *sub_minus, *sub_plus;  // [nGamma]
  const int *f_minus, *f_plus, *f_n, *f_loffm, *f_loffp;   // [nF]
  const int *sub_face_off, *sub_faces;
  const int64_t *line_off;    // [N+1] offsets into line_g
  const int *line_g;          // per subdomain, direction d, line l, end e: local interface index or -1
  // weights of the averaging operator E on the minus / plus copy of each
  // face's dofs (stiffness scaling); null: 1/2 each (multiplicity)
  const double *fw_minus = nullptr, *fw_plus = nullptr;   // [nF]
  // prescribed normal fluxes of the boundary faces (global face numbering,
  // interior entries zero); null: no flow through the boundary
  const double *bflux = nullptr;
};

// Per-subdomain dense setup workspace (FP64, column major).
struct SetupWs {
  double *base;
  const int64_t *P, *V, *H, *S, *L, *W;   // offsets per subdomain
  const int64_t *X;                        // offsets into Xmat
  double *Xmat;                            // persistent pressure operators X^i
  const int64_t *pk;                       // packed offsets (S, T)
  double *Spk;                             // persistent packed S^i (FP64)
};

// Coarse-space description built after the eigenproblems.  Coarse indices
// run over [0, nk): flux coarse dofs and rescaled subdomain pressures, in the
// slab-block order of the coarse factorization.
struct DevCoarse {
  int ncu;                     // flux coarse dofs
  int nk;                      // size of the coarse saddle point (ncu + N - 1)
  const int *face_cofs;        // [nF] coarse index of each face's zero-net-flux row
  const int *face_k;           // [nF] adaptive rows per face
  const int64_t *face_rows_off;  // [nF] offset of the adaptive rows (k x n_F, row major)
  const double *face_rows;
  const int *sub_coff;         // [N+1] offsets of local coarse dofs
  const int *sub_cmap;         // [sum nc_i] -> coarse index
  const int *co_minus, *co_plus;  // [nk] flat local index in the two subdomains (-1: pressure)
  const int *pidx;             // [N] coarse index of each subdomain pressure (-1: pinned)
};

}  // namespace bddc
