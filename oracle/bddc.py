"""Adaptive BDDC for the RT0/P0 saddle-point problem (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Literal CPU FP64 statement of the paper's method:

* substructuring into box subdomains, interface, faces (Section 3);
* pressure rescaling D, one scalar per subdomain (Section 5, eq. system-scaled);
* Stokes-harmonic extension and the interface Schur complement S^i through the
  un-reduced local Dirichlet saddle point (Section 3, mapping P; eq.
  discrete-harm; Section 4, S^{ij});
* the pair generalized eigenproblems eq. eigenvalue-problem-local-matrix with the
  projection onto null(C_U^{ij}(I - E^{ij})), rows eq. constraints and the
  threshold rule of Algorithm "Adaptive BDDC", indicator eq. indicator;
* coarse basis and the substructure correction from the un-reduced constrained
  local saddle point (Algorithm "BDDC preconditioner", steps 1-2; eq. C^i);
* Algorithm "BDDC method" steps 1-3, step 3 by conjugate gradients on the
  interface problem eqs. corr-reduced-1/2 in the balanced subspace, and the
  post-correction of interiors;
* the Lanczos condition-number estimate from the CG coefficients (Section 6).

Readings of points the paper leaves open (tie at tau, pair space, stopping norm,
gauge, row basis) are listed in the design notes and marked ``READING`` below.

Pins: tests/test_oracle_bddc.py (steps 1-2 reproduce the source exactly, the
correction is divergence free, all-interface constraints give one iteration,
outputs balanced, E is a projection, lambda_min >= 1, the decoupled symmetric
pair has eigenvalues {0, 1}, the minimax lemma, brute-force agreement with the
direct solve, Table 1 counts and the k = 1 rows of Tables 2 and 5).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import rt0


# ----------------------------------------------------------------------------
# substructuring (Section 3)
# ----------------------------------------------------------------------------

class Substructuring:
    """Box subdomains from per-axis cut planes; interface, faces, local dofs."""

    def __init__(self, grid, cuts):
        self.grid = grid
        self.cuts = [np.asarray(c, dtype=np.int64) for c in cuts]
        self.nsub_axis = [len(c) - 1 for c in self.cuts]
        self.N = int(np.prod(self.nsub_axis))
        cc = grid.cell_coords()
        sub_ax = [np.searchsorted(self.cuts[d], cc[d], side="right") - 1 for d in range(grid.dim)]
        self.cell_sub = np.ravel_multi_index(tuple(sub_ax), tuple(self.nsub_axis), order="F")

        # the cell on the minus / plus side of every face (-1 outside the grid)
        minus = -np.ones(grid.nfaces, dtype=np.int64)
        plus = -np.ones(grid.nfaces, dtype=np.int64)
        cells = np.arange(grid.ncells)
        for d in range(grid.dim):
            lo, hi = grid.cell_faces(d)
            minus[hi] = cells
            plus[lo] = cells
        self.face_minus, self.face_plus = minus, plus
        inner = (minus >= 0) & (plus >= 0)
        sm = np.where(minus >= 0, self.cell_sub[np.maximum(minus, 0)], -1)
        spl = np.where(plus >= 0, self.cell_sub[np.maximum(plus, 0)], -1)
        is_iface = inner & (sm != spl)
        self.gamma = np.flatnonzero(is_iface)
        self.n_gamma = len(self.gamma)
        self.gamma_pos = -np.ones(grid.nfaces, dtype=np.int64)
        self.gamma_pos[self.gamma] = np.arange(self.n_gamma)

        # faces = pairs of adjacent subdomains and their shared grid faces
        pairs = {}
        for f in self.gamma:
            key = (min(sm[f], spl[f]), max(sm[f], spl[f]))
            pairs.setdefault(key, []).append(f)
        self.face_pairs = sorted(pairs.keys())
        self.face_dofs = [np.asarray(sorted(pairs[k]), dtype=np.int64) for k in self.face_pairs]
        self.n_faces = len(self.face_pairs)

        # per-subdomain dofs
        self.sub_cells, self.sub_interior, self.sub_iface, self.sub_faces = [], [], [], []
        bnd = grid.boundary_faces()
        for i in range(self.N):
            ci = np.flatnonzero(self.cell_sub == i)
            fl = []
            for d in range(grid.dim):
                lo, hi = grid.cell_faces(d)
                fl += [lo[ci], hi[ci]]
            fl = np.unique(np.concatenate(fl))
            fl = fl[~bnd[fl]]
            interior = fl[~is_iface[fl]]
            my_faces = [k for k, pr in enumerate(self.face_pairs) if i in pr]
            # face-major local interface ordering, grid order inside each face
            iface = np.concatenate([self.face_dofs[k] for k in my_faces]) if my_faces else np.zeros(0, np.int64)
            self.sub_cells.append(ci)
            self.sub_interior.append(np.sort(interior))
            self.sub_iface.append(iface)
            self.sub_faces.append(my_faces)

    def table1(self):
        """N, n_Gamma, n_f and the initial n_c = n_f + N (Table 1)."""
        return self.N, self.n_gamma, self.n_faces, self.n_faces + self.N


# ----------------------------------------------------------------------------
# local saddle-point systems
# ----------------------------------------------------------------------------

class LocalProblem:
    """Unassembled matrices of one subdomain and its two local saddle points."""

    def __init__(self, grid, perm, subs, i):
        self.i = i
        self.cells = subs.sub_cells[i]
        self.I = subs.sub_interior[i]
        self.G = subs.sub_iface[i]
        self.nI, self.nG, self.nc = len(self.I), len(self.G), len(self.cells)
        flux = np.concatenate([self.I, self.G])
        loc = -np.ones(grid.nfaces, dtype=np.int64)
        loc[flux] = np.arange(len(flux))
        cloc = -np.ones(grid.ncells, dtype=np.int64)
        cloc[self.cells] = np.arange(self.nc)
        (ar, ac, av), (br, bc, bv) = rt0.assemble(grid, perm, self.cells)
        keep = (loc[ar] >= 0) & (loc[ac] >= 0)
        nf = len(flux)
        self.A = sp.csr_matrix((av[keep], (loc[ar[keep]], loc[ac[keep]])), shape=(nf, nf))
        keep = loc[bc] >= 0
        Bloc = sp.csr_matrix((bv[keep], (cloc[br[keep]], loc[bc[keep]])), shape=(self.nc, nf))
        # rescaling D: average of the diagonal of A over this subdomain's flux dofs
        self.d = float(self.A.diagonal().mean())
        self.B = self.d * Bloc                      # D B
        self.vol = np.full(self.nc, grid.cell_volume)   # C_Q^i (eq. Qi-def)
        sI, sG = slice(0, self.nI), slice(self.nI, nf)
        self.AII, self.AIG = self.A[sI, sI], self.A[sI, sG]
        self.AGI, self.AGG = self.A[sG, sI], self.A[sG, sG]
        self.BI, self.BG = self.B[:, sI], self.B[:, sG]
        c = sp.csr_matrix(self.vol[:, None])
        KD = sp.bmat([[self.AII, self.BI.T, None],
                      [self.BI, None, c],
                      [None, c.T, None]], format="csc")
        self.KD = spla.splu(KD)

    # Dirichlet problem: given interface flux w and right-hand sides on the
    # interior flux rows (gI) and pressure rows (hP), the Stokes-harmonic
    # interior with p in Q^i (zero volume-weighted mean).
    def dirichlet(self, w, gI=None, hP=None):
        w = np.atleast_2d(np.asarray(w, dtype=np.float64).T).T if np.ndim(w) == 1 else w
        k = w.shape[1]
        rhs = np.zeros((self.nI + self.nc + 1, k))
        rhs[:self.nI] = -(self.AIG @ w)
        rhs[self.nI:self.nI + self.nc] = -(self.BG @ w)
        if gI is not None:
            rhs[:self.nI] += gI.reshape(self.nI, -1)
        if hP is not None:
            rhs[self.nI:self.nI + self.nc] += hP.reshape(self.nc, -1)
        sol = self.KD.solve(rhs)
        return sol[:self.nI], sol[self.nI:self.nI + self.nc]

    def schur(self):
        """S^i, column by column from the Dirichlet saddle point."""
        E = np.eye(self.nG)
        uI, p = self.dirichlet(E)
        S = (self.AGG @ E) + self.AGI @ uI + self.BG.T @ p
        return 0.5 * (S + S.T)

    def set_constraints(self, C):
        """Factor the constrained (Neumann) saddle point with rows C on Gamma^i."""
        self.C = C
        nC = C.shape[0]
        nf = self.nI + self.nG
        Cbar = sp.hstack([sp.csr_matrix((nC, self.nI)), sp.csr_matrix(C)])
        c = sp.csr_matrix(self.vol[:, None])
        K = sp.bmat([[self.A, self.B.T, Cbar.T, None],
                     [self.B, None, None, c],
                     [Cbar, None, None, None],
                     [None, c.T, None, None]], format="csc")
        self.KN = spla.splu(K)
        self.nC = nC
        # coarse basis: coarse dofs e_j, zero flux load
        rhs = np.zeros((nf + self.nc + nC + 1, nC))
        rhs[nf + self.nc:nf + self.nc + nC] = np.eye(nC)
        sol = self.KN.solve(rhs)
        self.Phi = sol[:nf]                       # full local coarse basis
        self.Psi = sol[self.nI:nf]                # interface part
        self.Ac = -sol[nf + self.nc:nf + self.nc + nC]
        self.Ac = 0.5 * (self.Ac + self.Ac.T)
        # net (scaled) divergence of each coarse basis function: 1^T (D B) Phi
        self.Bc = np.ones(self.nc) @ (self.B @ self.Phi)

    def delta_solve(self, r):
        """Substructure correction: min energy with zero coarse dofs, load r on Gamma^i."""
        nf = self.nI + self.nG
        rhs = np.zeros(nf + self.nc + self.nC + 1)
        rhs[self.nI:nf] = r
        sol = self.KN.solve(rhs)
        return sol[self.nI:nf]


# ----------------------------------------------------------------------------
# adaptive constraints (Section 4)
# ----------------------------------------------------------------------------

def pair_eigenproblem(Si, Sj, pos_i, pos_j, extra_rows=None):
    """Generalized eigenproblem eq. eigenvalue-problem-local-matrix for one face.

    ``Si``, ``Sj``: Schur complements of the two subdomains; ``pos_i``,
    ``pos_j``: positions of the face dofs (same grid order) inside Gamma^i and
    Gamma^j.  READING: E^{ij} averages only the shared face and C_U^{ij} holds
    only that face's initial zero-net-flux constraint, plus ``extra_rows``
    (k x n_F, applied to both copies of the face) when given.

    Returns eigenvalues (descending), eigenvectors (pair space), and the
    constraint rows eq. constraints split into the i-half on the face.
    """
    ni, nj = Si.shape[0], Sj.shape[0]
    n = ni + nj
    S = sla.block_diag(Si, Sj)
    E = np.eye(n)
    a = np.asarray(pos_i)
    b = ni + np.asarray(pos_j)
    E[a, a] = 0.5
    E[b, b] = 0.5
    E[a, b] = 0.5
    E[b, a] = 0.5
    IE = np.eye(n) - E
    face_rows_ = [np.ones(len(a))] + ([] if extra_rows is None else list(extra_rows))
    CU = np.zeros((2 * len(face_rows_), n))
    for t, row in enumerate(face_rows_):
        CU[2 * t, a] = row
        CU[2 * t + 1, b] = row
    Cc = CU @ IE
    Z = sla.null_space(Cc)               # basis of null(C)
    Q = sla.orth(Cc.T)
    Pi = np.eye(n) - Q @ Q.T             # orthogonal projection onto null(C)
    M = IE.T @ S @ IE
    lam, Y = sla.eigh(Z.T @ M @ Z, Z.T @ S @ Z)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    W = Z @ Y[:, order]
    rows = (W.T @ Pi @ M @ Pi)           # c_l^{ij}
    return lam, W, rows[:, a], rows[:, b]


def face_rows(lam, ci, tau, n_f):
    """Rows of C_U on one face: zero-net-flux row plus adaptive rows.

    Algorithm "Adaptive BDDC": the smallest k with lambda_{k+1} <= tau, i.e.
    k = #{lambda > tau} (READING at ties).  The adaptive rows are orthonormalised
    (span preserving).  Returns (rows, k, omega_F).
    """
    k = int(np.sum(lam > tau)) if math.isfinite(tau) else 0
    omega = float(lam[k]) if k < len(lam) else 0.0
    rows = [np.ones(n_f)]
    if k > 0:
        Cad = ci[:k]
        Cad = Cad - np.outer(Cad @ np.ones(n_f) / n_f, np.ones(n_f))
        q, _ = np.linalg.qr(Cad.T)
        rows += list(q.T)
    return np.array(rows), k, omega


def multiscale_weight(source, cells):
    """Source distribution w of the multiscale constraints on one subdomain (Section 6).

    Cell-integrated values over ``cells``, summing to 1: w = 1/|Omega^s| in a
    subdomain without a well, w = f / int_{Omega^s} f in a subdomain that
    contains one (the source f is not zero there), so that the local flow is
    conservative on the fine grid.  ``source`` None: no wells anywhere.
    READING: a subdomain whose wells cancel (zero net source) keeps the
    uniform w, since the normalisation is undefined there.
    """
    n = len(cells)
    if source is not None:
        f = np.asarray(source, dtype=np.float64)[cells]
        tot = f.sum()
        if np.any(f != 0.0) and abs(tot) > 1e-12 * np.abs(f).sum():
            return f / tot
    return np.full(n, 1.0 / n)


def multiscale_face_flux(grid, perm, subs, i, j, dofs, source=None):
    """Face flux of the local Darcy problem behind the multiscale constraints (Section 6).

    On the union of the neighbours i and j (i on the minus side of the face):
    source w_i in Omega^i and -w_j in Omega^j (``multiscale_weight``: uniform,
    or shaped by the well source ``source`` in a subdomain that contains a
    well), no flow on the union's boundary, the pressure fixed by a zero mean.
    Returns the fluxes on the face dofs ``dofs`` (global orientation; they sum
    to the unit net flux from i to j).
    """
    perm = np.asarray(perm, dtype=np.float64).reshape(grid.ncells, grid.dim)
    ci, cj = subs.sub_cells[i], subs.sub_cells[j]
    cells = np.concatenate([ci, cj])
    (ar, ac, av), (br, bc, bv) = rt0.assemble(grid, perm, cells)
    # flux dofs: faces shared by two cells of the union (the rest carry no flow)
    cnt = np.zeros(grid.nfaces, dtype=np.int64)
    np.add.at(cnt, bc, 1)
    inner = np.flatnonzero(cnt == 2)
    loc = -np.ones(grid.nfaces, dtype=np.int64)
    loc[inner] = np.arange(len(inner))
    cloc = -np.ones(grid.ncells, dtype=np.int64)
    cloc[cells] = np.arange(len(cells))
    keep = (loc[ar] >= 0) & (loc[ac] >= 0)
    A = sp.csr_matrix((av[keep], (loc[ar[keep]], loc[ac[keep]])), shape=(len(inner), len(inner)))
    keep = loc[bc] >= 0
    B = sp.csr_matrix((bv[keep], (cloc[br[keep]], loc[bc[keep]])), shape=(len(cells), len(inner)))
    vol = np.full(len(cells), grid.cell_volume)
    # cell-integrated source: +w_i over Omega^i, -w_j over Omega^j
    f = np.concatenate([multiscale_weight(source, ci), -multiscale_weight(source, cj)])
    K = sp.bmat([[A, B.T, None],
                 [B, None, sp.csr_matrix(vol[:, None])],
                 [None, sp.csr_matrix(vol[None, :]), None]], format="csc")
    rhs = np.concatenate([np.zeros(len(inner)), -f, [0.0]])     # b(u, q) = -int div u q = -<f, q>
    sol = spla.spsolve(K, rhs)
    return sol[loc[np.asarray(dofs)]]


def multiscale_rows(u_face, n_f):
    """Rows of C_U on one face with the multiscale constraint: the zero-net-flux
    row plus the face flux of the local problem, projected off the first row and
    normalised (dropped when the flux is uniform).  Returns (rows, k)."""
    rows = [np.ones(n_f)]
    r = u_face - u_face.mean()
    if n_f > 1 and np.linalg.norm(r) > 1e-12 * np.linalg.norm(u_face):
        rows.append(r / np.linalg.norm(r))
    return np.array(rows), len(rows) - 1


# ----------------------------------------------------------------------------
# the BDDC method
# ----------------------------------------------------------------------------

class BDDC:
    """Setup of Algorithm "BDDC method" for a given grid, field and partition."""

    def __init__(self, grid, perm, cuts, tau=math.inf, all_constrained=False, multiscale=False,
                 scaling="multiplicity", ms_source=None):
        self.grid = grid
        self.perm = np.asarray(perm, dtype=np.float64).reshape(grid.ncells, grid.dim)
        self.tau = tau
        self.subs = subs = Substructuring(grid, cuts)
        self.loc = [LocalProblem(grid, self.perm, subs, i) for i in range(subs.N)]
        self.S = [lp.schur() for lp in self.loc]
        self.d = np.array([lp.d for lp in self.loc])

        # local positions of each face's dofs inside Gamma^i
        self.face_pos = []
        for k, (i, j) in enumerate(subs.face_pairs):
            dofs = subs.face_dofs[k]
            mi = {g: t for t, g in enumerate(subs.sub_iface[i])}
            mj = {g: t for t, g in enumerate(subs.sub_iface[j])}
            self.face_pos.append((np.array([mi[g] for g in dofs]), np.array([mj[g] for g in dofs])))

        # pair eigenproblems and face constraint rows
        self.face_lam, self.face_k, self.face_omega, self.face_C = [], [], [], []
        for k, (i, j) in enumerate(subs.face_pairs):
            nF = len(subs.face_dofs[k])
            if multiscale:
                # Section 6: the local Darcy problem in place of the eigenproblem (tau unused)
                uF = multiscale_face_flux(grid, self.perm, subs, i, j, subs.face_dofs[k], ms_source)
                rows, kk = multiscale_rows(uF, nF)
                self.face_lam.append(np.zeros(0))
                self.face_k.append(kk)
                self.face_omega.append(0.0)
                self.face_C.append(rows)
                continue
            if all_constrained:
                Z = sla.null_space(np.ones((1, nF)))
                rows = np.vstack([np.ones(nF), Z.T])
                self.face_lam.append(np.zeros(0))
                self.face_k.append(nF - 1)
                self.face_omega.append(0.0)
                self.face_C.append(rows)
                continue
            if math.isfinite(tau):
                lam, _, ci, _ = pair_eigenproblem(self.S[i], self.S[j], *self.face_pos[k])
            else:
                lam, ci = np.zeros(0), np.zeros((0, nF))
            rows, kk, om = face_rows(lam, ci, tau, nF)
            self.face_lam.append(lam)
            self.face_k.append(kk)
            self.face_omega.append(om)
            self.face_C.append(rows)
        self.omega_tilde = max(self.face_omega) if self.face_omega else 0.0

        # weights of the averaging operator E on the two copies of every interface
        # dof: multiplicity (1/2 each), or stiffness scaling (the paper's choice
        # when coefficient jumps follow the interfaces; for RT0 it is rho-scaling
        # with rho = 1/k), kept constant along each face as the Remark on the
        # starting flux constraints requires: delta_i = a_i / (a_i + a_j), a_i
        # the mean of diag(A^i) over the face's dofs
        if scaling not in ("multiplicity", "stiffness"):
            raise ValueError("scaling must be 'multiplicity' or 'stiffness'")
        if scaling == "stiffness" and math.isfinite(tau) and not (multiscale or all_constrained):
            raise ValueError("the pair eigenproblems assume the multiplicity weights")
        self.weight = [np.full(lp.nG, 0.5) for lp in self.loc]
        if scaling == "stiffness":
            for k, (i, j) in enumerate(subs.face_pairs):
                pi, pj = self.face_pos[k]
                ai = self.loc[i].AGG.diagonal()[pi].mean()
                aj = self.loc[j].AGG.diagonal()[pj].mean()
                self.weight[i][pi] = ai / (ai + aj)
                self.weight[j][pj] = aj / (ai + aj)

        # global coarse dof numbering: face by face
        self.cofs = np.concatenate([[0], np.cumsum([c.shape[0] for c in self.face_C])]).astype(np.int64)
        self.n_cu = int(self.cofs[-1])
        self.n_c = self.n_cu + subs.N
        self.sub_cdofs = []
        for i in range(subs.N):
            rows, gidx, col0 = [], [], 0
            blocks = []
            for k in subs.sub_faces[i]:
                nF = len(subs.face_dofs[k])
                blocks.append((k, col0, nF))
                col0 += nF
            C = np.zeros((sum(self.face_C[k].shape[0] for k, _, _ in blocks), col0))
            r0 = 0
            for k, c0, nF in blocks:
                nr = self.face_C[k].shape[0]
                C[r0:r0 + nr, c0:c0 + nF] = self.face_C[k]
                gidx += list(range(self.cofs[k], self.cofs[k] + nr))
                r0 += nr
            self.loc[i].set_constraints(C)
            self.sub_cdofs.append(np.array(gidx, dtype=np.int64))

        # coarse saddle point [A_c B_c^T 0; B_c 0 g; 0 g^T 0] (gauge g: zero mean of D p0)
        # (sparse storage: A_c = sum of the local blocks, an entry shared by two
        # subdomains is the sum of their two values; exact zeros are dropped)
        N, ncu = subs.N, self.n_cu
        ar, ac, av, br, bcol, bv = [], [], [], [], [], []
        for i, lp in enumerate(self.loc):
            idx = self.sub_cdofs[i]
            rr, cc = np.meshgrid(idx, idx, indexing="ij")
            ar.append(rr.ravel())
            ac.append(cc.ravel())
            av.append(np.asarray(lp.Ac).ravel())
            br.append(np.full(len(idx), i))
            bcol.append(idx)
            bv.append(lp.Bc)
        cat = lambda v, dt=np.float64: np.concatenate(v).astype(dt) if v else np.zeros(0, dt)
        Ac = sp.csr_matrix((cat(av), (cat(ar, np.int64), cat(ac, np.int64))), shape=(ncu, ncu))
        Bc = sp.csr_matrix((cat(bv), (cat(br, np.int64), cat(bcol, np.int64))), shape=(N, ncu))
        Ac.sum_duplicates()
        Bc.sum_duplicates()
        Ac.eliminate_zeros()
        Bc.eliminate_zeros()
        self.Ac, self.Bc = Ac, Bc
        gvec = np.array([len(lp.cells) * grid.cell_volume * lp.d for lp in self.loc])
        self.gauge = gvec
        K = sp.bmat([[Ac, sp.csr_matrix(Bc.T), None],
                     [Bc, None, sp.csr_matrix(gvec[:, None])],
                     [None, sp.csr_matrix(gvec[None, :]), None]], format="csc")
        self.Kc = spla.splu(K)

        # B_0: interface flux -> scaled net divergence per subdomain (sparse)
        rows, cols, vals = [], [], []
        for i, lp in enumerate(self.loc):
            rows.append(np.full(lp.nG, i))
            cols.append(subs.gamma_pos[lp.G])
            vals.append(np.asarray(np.ones(lp.nc) @ lp.BG).ravel())
        self.B0 = sp.csr_matrix((cat(vals), (cat(rows, np.int64), cat(cols, np.int64))), shape=(N, subs.n_gamma))

    # -- pieces --------------------------------------------------------------
    def coarse_solve(self, gu, hp):
        rhs = np.concatenate([gu, hp, [0.0]])
        sol = self.Kc.solve(rhs)
        return sol[:self.n_cu], sol[self.n_cu:self.n_cu + self.subs.N]

    def restrict(self, i, x):
        return x[self.subs.gamma_pos[self.loc[i].G]]

    def apply_S(self, xu):
        """Assembled interface Schur complement sum_i R^iT S^i R^i."""
        y = np.zeros(self.subs.n_gamma)
        for i, lp in enumerate(self.loc):
            pos = self.subs.gamma_pos[lp.G]
            y[pos] += self.S[i] @ xu[pos]
        return y

    def operator(self, xu, xp):
        """The interface saddle point of eqs. corr-reduced-1/2."""
        return self.apply_S(xu) + self.B0.T @ xp, self.B0 @ xu

    def average(self, locals_):
        """E: weighted sum of the subdomain copies (weights 1/2, or the stiffness weights)."""
        y = np.zeros(self.subs.n_gamma)
        for i, lp in enumerate(self.loc):
            y[self.subs.gamma_pos[lp.G]] += self.weight[i] * locals_[i]
        return y

    def precondition(self, ru):
        """Algorithm "BDDC preconditioner": (r_B, 0) -> (w_hat, p_0)."""
        N = self.subs.N
        rloc = [self.weight[i] * self.restrict(i, ru) for i in range(N)]   # E^T r: <r_B, E z> pairing
        gu = np.zeros(self.n_cu)
        for i, lp in enumerate(self.loc):
            gu[self.sub_cdofs[i]] += lp.Psi.T @ rloc[i]
        alpha, p0 = self.coarse_solve(gu, np.zeros(N))
        w = []
        for i, lp in enumerate(self.loc):
            wpi = lp.Psi @ alpha[self.sub_cdofs[i]]
            wdelta = lp.delta_solve(rloc[i])
            w.append(wpi + wdelta)
        return self.average(w), p0

    # -- Algorithm "BDDC method" ----------------------------------------------
    def solve(self, source, rtol=1e-6, maxit=5000, record=False):
        g, subs = self.grid, self.subs
        N = subs.N
        F = -np.asarray(source, dtype=np.float64)       # <f, q> = -int f q
        out = {}

        # step 1: coarse component
        hp = np.array([lp.d * F[lp.cells].sum() for lp in self.loc])
        alpha0, _ = self.coarse_solve(np.zeros(self.n_cu), hp)
        w0 = [lp.Psi @ alpha0[self.sub_cdofs[i]] for i, lp in enumerate(self.loc)]
        u0G = self.average(w0)
        u0 = np.zeros(g.nfaces)
        u0[subs.gamma] = u0G
        for i, lp in enumerate(self.loc):
            uI, _ = lp.dirichlet(self.restrict(i, u0G))
            u0[lp.I] = uI[:, 0]

        # step 2: substructure components with zero interface flux
        ustar = u0.copy()
        for i, lp in enumerate(self.loc):
            ul = u0[np.concatenate([lp.I, lp.G])]
            Au = lp.A @ ul
            Bu = lp.B @ ul
            uI, _ = lp.dirichlet(np.zeros(lp.nG), gI=-Au[:lp.nI], hP=lp.d * F[lp.cells] - Bu)
            ustar[lp.I] += uI[:, 0]

        # reduced right-hand side of step 3
        fstar = np.zeros(subs.n_gamma)
        for i, lp in enumerate(self.loc):
            x = -(lp.A @ ustar[np.concatenate([lp.I, lp.G])])
            # K_D^{-1} [x_I; 0; 0] is the Dirichlet solve with zero interface flux
            # and load x_I on the interior flux rows
            yI, yP = lp.dirichlet(np.zeros(lp.nG), gI=x[:lp.nI])
            fi = x[lp.nI:] - (lp.AGI @ yI[:, 0] + lp.BG.T @ yP[:, 0])
            fstar[subs.gamma_pos[lp.G]] += fi

        # step 3: CG on the balanced interface saddle point
        xu = np.zeros(subs.n_gamma)
        xp = np.zeros(N)
        ru, rp = fstar.copy(), np.zeros(N)
        r0 = math.sqrt(ru @ ru + rp @ rp)
        zu, zp = self.precondition(ru)
        pu, pp = zu.copy(), zp.copy()
        rho = ru @ zu + rp @ zp
        alphas, betas, hist = [], [], [1.0]
        it = 0
        converged = r0 == 0.0
        while not converged and it < maxit:
            qu, qp = self.operator(pu, pp)
            gam = pu @ qu + pp @ qp
            a = rho / gam
            xu += a * pu
            xp += a * pp
            ru -= a * qu
            rp -= a * qp
            it += 1
            alphas.append(a)
            rn = math.sqrt(ru @ ru + rp @ rp)
            hist.append(rn / r0)
            if rn <= rtol * r0:
                converged = True
                break
            zu, zp = self.precondition(ru)
            rho_new = ru @ zu + rp @ zp
            b = rho_new / rho
            betas.append(b)
            rho = rho_new
            pu = zu + b * pu
            pp = zp + b * pp

        # post-correction: interiors of the correction and the pressure
        ucorr = np.zeros(g.nfaces)
        ucorr[subs.gamma] = xu
        pbar = np.zeros(g.ncells)
        for i, lp in enumerate(self.loc):
            ul = ustar[np.concatenate([lp.I, lp.G])]
            Au = lp.A @ ul
            uI, pI = lp.dirichlet(self.restrict(i, xu), gI=-Au[:lp.nI])
            ucorr[lp.I] = uI[:, 0]
            pbar[lp.cells] = pI[:, 0] + xp[i]
        u = ustar + ucorr
        dcell = np.empty(g.ncells)
        for lp in self.loc:
            dcell[lp.cells] = lp.d
        p = rt0.remove_mean(g, dcell * pbar)

        out.update(u=u, p=p, u0=u0, ustar=ustar, ucorr=ucorr, fstar=fstar, xu=xu, xp=xp,
                   it=it, converged=converged, relres=hist[-1], history=np.array(hist),
                   alphas=np.array(alphas), betas=np.array(betas),
                   kappa=lanczos_kappa(alphas, betas)[2])
        return out


def lanczos_kappa(alphas, betas):
    """Extreme eigenvalues of the CG Lanczos tridiagonal and their ratio.

    T_kk = 1/a_k + b_{k-1}/a_{k-1},  T_{k,k+1} = sqrt(b_k)/a_k  (Section 6: the
    condition number estimate from the Lanczos sequence of CG).
    """
    k = len(alphas)
    # r^T z can only turn non-positive at the rounding floor; the sequence is
    # cut there (later coefficients carry no spectral information)
    for j, b in enumerate(betas[:max(k - 1, 0)]):
        if not b > 0.0:
            k = j + 1
            break
    if k == 0:
        return 1.0, 1.0, 1.0
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1], ev[-1] / ev[0]
