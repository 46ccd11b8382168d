"""RT0/P0 discretisation of the mixed Darcy problem on Cartesian grids (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Follows Section 2 of the paper: a(u,v) = int k^-1 u.v (eq. a),
b(u,q) = -int (div u) q (eq. b), <f,q> = -int f q (eq. rhs), U = RT0 with zero
normal flux on the boundary, Q = P0 with zero mean (eqs. variational-1/2).

Degrees of freedom: one total normal flux per grid face in the global +x/+y/+z
direction (boundary faces are held at zero, or at prescribed values when a
boundary flux is given), one pressure per cell.  On a rectangular cell with a
diagonal permeability the lowest-order Raviart-Thomas velocity component along
axis d is linear in that coordinate only, so the exact element mass matrix
decouples by direction:  for the two faces (-d, +d) of the cell,

    m_d * [[1/3, 1/6], [1/6, 1/3]],   m_d = h_d / (k_d * prod_{e != d} h_e),

and the divergence integral over the cell is (flux out of +d) - (flux into -d).

Pins (tests/test_oracle_rt0.py): a linear pressure at constant k is reproduced
exactly (closed form), the dof counts 39,880 and 110,700 printed in Section 6,
and the kernel of B^T is the constants.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class Grid:
    """Cartesian grid with x-fastest cells and per-direction face blocks."""

    def __init__(self, n, h):
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.dim = len(self.n)
        self.ncells = int(np.prod(self.n))
        self.face_shape = []
        for d in range(self.dim):
            self.face_shape.append(tuple(self.n[e] + (1 if e == d else 0) for e in range(self.dim)))
        self.nfaces_dir = [int(np.prod(s)) for s in self.face_shape]
        self.face_offset = np.concatenate([[0], np.cumsum(self.nfaces_dir)]).astype(np.int64)
        self.nfaces = int(self.face_offset[-1])
        self.cell_volume = float(np.prod(self.h))

    # -- numbering ---------------------------------------------------------
    def cell_id(self, idx):
        return np.ravel_multi_index(tuple(idx), self.n, order="F")

    def cell_coords(self):
        """Integer coordinates (dim arrays) of all cells in cell order."""
        return np.unravel_index(np.arange(self.ncells), self.n, order="F")

    def face_id(self, d, idx):
        return self.face_offset[d] + np.ravel_multi_index(tuple(idx), self.face_shape[d], order="F")

    def face_dir_coords(self):
        """For every global face: its direction and integer coordinates."""
        dirs = np.empty(self.nfaces, dtype=np.int64)
        coords = np.empty((self.nfaces, self.dim), dtype=np.int64)
        for d in range(self.dim):
            s, e = self.face_offset[d], self.face_offset[d + 1]
            dirs[s:e] = d
            cc = np.unravel_index(np.arange(e - s), self.face_shape[d], order="F")
            for a in range(self.dim):
                coords[s:e, a] = cc[a]
        return dirs, coords

    def boundary_faces(self):
        dirs, coords = self.face_dir_coords()
        nd = np.asarray(self.n)[dirs]
        pos = coords[np.arange(self.nfaces), dirs]
        return (pos == 0) | (pos == nd)

    def cell_faces(self, d):
        """(-d face, +d face) global ids of every cell, in cell order."""
        cc = self.cell_coords()
        lo = self.face_id(d, cc)
        hi_idx = list(cc)
        hi_idx[d] = hi_idx[d] + 1
        hi = self.face_id(d, hi_idx)
        return lo, hi


def element_coefficients(grid, perm):
    """m_d for every cell and direction: [ncells, dim]."""
    perm = np.asarray(perm, dtype=np.float64).reshape(grid.ncells, grid.dim)
    m = np.empty_like(perm)
    for d in range(grid.dim):
        other = np.prod([grid.h[e] for e in range(grid.dim) if e != d])
        m[:, d] = grid.h[d] / (perm[:, d] * other)
    return m


def assemble(grid, perm, cells=None):
    """Assemble the mass matrix A and divergence matrix B over ``cells``.

    Returns COO-style triplets (global face ids / cell ids) so callers can
    build either the global matrices or the unassembled subdomain matrices.
    A: nfaces x nfaces, B: ncells x nfaces with B[c, +d face] = -1,
    B[c, -d face] = +1 (b(u,q) = -int div u q).
    """
    m = element_coefficients(grid, perm)
    if cells is None:
        cells = np.arange(grid.ncells)
    cells = np.asarray(cells, dtype=np.int64)
    ar, ac, av = [], [], []
    br, bc, bv = [], [], []
    for d in range(grid.dim):
        lo, hi = grid.cell_faces(d)
        lo, hi, md = lo[cells], hi[cells], m[cells, d]
        ar += [lo, hi, lo, hi]
        ac += [lo, hi, hi, lo]
        av += [md / 3.0, md / 3.0, md / 6.0, md / 6.0]
        br += [cells, cells]
        bc += [hi, lo]
        bv += [-np.ones(len(cells)), np.ones(len(cells))]
    A = (np.concatenate(ar), np.concatenate(ac), np.concatenate(av))
    B = (np.concatenate(br), np.concatenate(bc), np.concatenate(bv))
    return A, B


def global_matrices(grid, perm):
    (ar, ac, av), (br, bc, bv) = assemble(grid, perm)
    A = sp.csr_matrix((av, (ar, ac)), shape=(grid.nfaces, grid.nfaces))
    B = sp.csr_matrix((bv, (br, bc)), shape=(grid.ncells, grid.nfaces))
    return A, B


def cell_volumes(grid):
    return np.full(grid.ncells, grid.cell_volume)


def direct_solve(grid, perm, source, bflux=None):
    """Monolithic sparse direct solve of the saddle-point system (eq. system).

    ``source`` is the cell-integrated f (so F = -source, eq. rhs).  Boundary
    faces carry ``bflux`` (zero = no flow).  The pressure is fixed by a zero
    volume-weighted mean via a bordered system with the volume vector.
    Returns (u over all faces, p over cells).
    """
    A, B = global_matrices(grid, perm)
    bnd = grid.boundary_faces()
    inner = np.flatnonzero(~bnd)
    outer = np.flatnonzero(bnd)
    ub = np.zeros(grid.nfaces)
    if bflux is not None:
        ub[:] = np.where(bnd, bflux, 0.0)
    F = -np.asarray(source, dtype=np.float64)
    Aii = A[inner][:, inner]
    Bi = B[:, inner]
    vol = cell_volumes(grid)[:, None]
    K = sp.bmat([[Aii, Bi.T, None],
                 [Bi, None, sp.csr_matrix(vol)],
                 [None, sp.csr_matrix(vol.T), None]], format="csc")
    rhs = np.concatenate([-(A[inner][:, outer] @ ub[outer]),
                          F - B[:, outer] @ ub[outer],
                          [0.0]])
    sol = spla.spsolve(K, rhs)
    u = ub.copy()
    u[inner] = sol[:len(inner)]
    p = sol[len(inner):len(inner) + grid.ncells]
    return u, p


def remove_mean(grid, p):
    vol = cell_volumes(grid)
    return p - (vol @ p) / vol.sum()
