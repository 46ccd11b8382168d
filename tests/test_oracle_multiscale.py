"""Oracle pins for the multiscale constraints (Section 6, MsMFEM-inspired rows).

For the face between neighbours i and j the oracle solves the Darcy problem on
the union of the two subdomains with source +1/|Omega^i| and -1/|Omega^j| and
no flow on the union's boundary, and takes the face fluxes as one more
constraint row.  Pinned by:
* conservation: the face fluxes carry the whole source, so they sum to 1;
* the reduced form: with no flow through the other faces, the face flux is
  the unit-net-flux minimiser of u^T (S^i_FF + S^j_FF) u, i.e. proportional to
  (S^i_FF + S^j_FF)^{-1} 1 (Schur complements from the local Dirichlet
  problems, an independent route through the same equations);
* closed forms and symmetry: two equal homogeneous boxes give a uniform face
  flux (the flow is one-dimensional), a mirror-symmetric field a
  mirror-symmetric face flux;
* the method: BDDC with these rows reproduces the direct solution and its
  preconditioned spectrum stays above 1.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bddc as ob
from oracle import rt0


def _reduced(o, k):
    i, j = o.subs.face_pairs[k]
    pi, pj = o.face_pos[k]
    X = o.S[i][np.ix_(pi, pi)] + o.S[j][np.ix_(pj, pj)]
    y = np.linalg.solve(X, np.ones(len(pi)))
    return y / y.sum()


@pytest.mark.parametrize("seed", [0, 3])
def test_face_flux_conserves_and_matches_reduced_form(seed):
    pr = W.unit_square_16(seed)
    g = rt0.Grid(pr.n, pr.h)
    o = ob.BDDC(g, pr.perm, pr.cuts, tau=math.inf)
    for k in range(o.subs.n_faces):
        i, j = o.subs.face_pairs[k]
        uF = ob.multiscale_face_flux(g, pr.perm, o.subs, i, j, o.subs.face_dofs[k])
        assert abs(uF.sum() - 1.0) <= 1e-12
        assert np.linalg.norm(uF - _reduced(o, k)) <= 1e-12 * np.linalg.norm(uF)


def test_face_flux_3d_reduced_form():
    rng = np.random.default_rng(5)
    n = (4, 4, 4)
    pr = W.Problem("cube4", n, (1.0, 2.0, 0.5), np.exp(rng.normal(0, 1.5, (64, 3))), W.corner_pair(n),
                   W.regular_cuts(n, (2, 2, 2)))
    g = rt0.Grid(pr.n, pr.h)
    o = ob.BDDC(g, pr.perm, pr.cuts, tau=math.inf)
    for k in range(o.subs.n_faces):
        i, j = o.subs.face_pairs[k]
        uF = ob.multiscale_face_flux(g, pr.perm, o.subs, i, j, o.subs.face_dofs[k])
        assert abs(uF.sum() - 1.0) <= 1e-12
        assert np.linalg.norm(uF - _reduced(o, k)) <= 1e-12 * np.linalg.norm(uF)


def test_homogeneous_face_flux_is_one_dimensional():
    # two equal homogeneous boxes side by side: uniform source, uniform sink and
    # no flow elsewhere make the flow one-dimensional, so the face flux is
    # uniform (1 / n_F per face dof) and the multiscale row adds nothing
    n = (8, 6)
    pr = W.homogeneous(n, (1.0, 1.0), W.regular_cuts(n, (4, 6)))   # two 4 x 6 boxes
    g = rt0.Grid(pr.n, pr.h)
    subs = ob.Substructuring(g, pr.cuts)
    assert subs.n_faces == 1
    uF = ob.multiscale_face_flux(g, pr.perm, subs, 0, 1, subs.face_dofs[0])
    assert len(uF) == 6
    assert np.allclose(uF, 1.0 / 6.0, rtol=0, atol=1e-14)
    rows, k = ob.multiscale_rows(uF, 6)
    assert k == 0 and rows.shape == (1, 6)


def test_face_flux_symmetric_under_mirrored_field():
    # a field symmetric about the box's mid-line in y gives a mirror-symmetric face flux
    n = (8, 6)
    rng = np.random.default_rng(2)
    half = np.exp(rng.normal(0, 1.0, (8, 3)))
    k = np.concatenate([half, half[:, ::-1]], axis=1)          # k(x, y) = k(x, 5 - y)
    kc = k.reshape(-1, order="F")
    pr = W.Problem("mirror", n, (1.0, 1.0), np.stack([kc, kc], 1), W.corner_pair(n), W.regular_cuts(n, (4, 6)))
    g = rt0.Grid(pr.n, pr.h)
    subs = ob.Substructuring(g, pr.cuts)
    uF = ob.multiscale_face_flux(g, pr.perm, subs, 0, 1, subs.face_dofs[0])
    assert np.allclose(uF, uF[::-1], rtol=0, atol=1e-13)
    assert not np.allclose(uF, uF.mean(), rtol=0, atol=1e-6)    # the heterogeneity shows
    assert abs(uF.sum() - 1.0) <= 1e-12


@pytest.mark.parametrize("seed", [0, 3])
def test_multiscale_bddc_solves(seed):
    pr = W.unit_square_16(seed)
    g = rt0.Grid(pr.n, pr.h)
    ue, _ = rt0.direct_solve(g, pr.perm, pr.source)
    o = ob.BDDC(g, pr.perm, pr.cuts, multiscale=True)
    assert all(k == 1 for k in o.face_k)
    out = o.solve(pr.source, rtol=1e-12)
    assert np.linalg.norm(out["u"] - ue) <= 1e-9 * np.linalg.norm(ue)
    lmin, _, _ = ob.lanczos_kappa(out["alphas"], out["betas"])
    assert lmin >= 1 - 1e-8


# ---- the well-shaped source w_i = f / int f (Section 6, MsMFEM paragraph) ------

def _face_load(o, s, f_s, pos):
    """Face rows of the interface load that the source f_s (cell integrated, on
    Omega^s) puts on the Dirichlet problem of subdomain s with zero interface
    flux: the un-reduced local saddle point, scaled pressure rows D B u = -D f."""
    lp = o.loc[s]
    uI, p = lp.dirichlet(np.zeros(lp.nG), hP=-lp.d * f_s)
    return (lp.AGI @ uI[:, 0] + lp.BG.T @ p[:, 0])[pos]


def _reduced_with_source(o, k, source):
    """Unit-net-flux minimiser of 1/2 u^T (S^i_FF + S^j_FF) u + u^T (g^i + g^j):
    the union problem eliminated onto the face, g^s the face load of w_s."""
    i, j = o.subs.face_pairs[k]
    pi, pj = o.face_pos[k]
    K = o.S[i][np.ix_(pi, pi)] + o.S[j][np.ix_(pj, pj)]
    wi = ob.multiscale_weight(source, o.subs.sub_cells[i])
    wj = ob.multiscale_weight(source, o.subs.sub_cells[j])
    g = _face_load(o, i, wi, pi) + _face_load(o, j, -wj, pj)
    y = np.linalg.solve(K, np.ones(len(pi)))
    z = np.linalg.solve(K, g)
    mu = (1.0 + z.sum()) / y.sum()
    return mu * y - z


def _well_square(seed):
    pr = W.unit_square_16(seed)
    src = pr.source.copy()
    src[5 + 16 * 6] = 0.7          # an extra injector inside an interior subdomain, sink beside it
    src[6 + 16 * 6] = -0.2
    src[0] -= 0.5
    return pr, src


@pytest.mark.parametrize("seed", [0, 3])
def test_well_face_flux_conserves_and_matches_reduced_form(seed):
    pr, src = _well_square(seed)
    g = rt0.Grid(pr.n, pr.h)
    o = ob.BDDC(g, pr.perm, pr.cuts, tau=math.inf)
    wells = {i for i in range(o.subs.N) if np.any(src[o.subs.sub_cells[i]] != 0.0)}
    assert len(wells) == 3
    checked = 0
    for k in range(o.subs.n_faces):
        i, j = o.subs.face_pairs[k]
        if not ({i, j} & wells):
            continue
        uF = ob.multiscale_face_flux(g, pr.perm, o.subs, i, j, o.subs.face_dofs[k], src)
        assert abs(uF.sum() - 1.0) <= 1e-12
        assert np.linalg.norm(uF - _reduced_with_source(o, k, src)) <= 1e-11 * np.linalg.norm(uF)
        # the well shapes the flux: it differs from the uniform w's
        u0 = ob.multiscale_face_flux(g, pr.perm, o.subs, i, j, o.subs.face_dofs[k])
        assert np.linalg.norm(uF - u0) > 1e-6 * np.linalg.norm(u0)
        checked += 1
    assert checked >= 6


def test_faces_without_wells_keep_the_uniform_weight_bit_for_bit():
    pr, src = _well_square(0)
    g = rt0.Grid(pr.n, pr.h)
    subs = ob.Substructuring(g, pr.cuts)
    wells = {i for i in range(subs.N) if np.any(src[subs.sub_cells[i]] != 0.0)}
    n = 0
    for k, (i, j) in enumerate(subs.face_pairs):
        if {i, j} & wells:
            continue
        a = ob.multiscale_face_flux(g, pr.perm, subs, i, j, subs.face_dofs[k], src)
        b = ob.multiscale_face_flux(g, pr.perm, subs, i, j, subs.face_dofs[k])
        assert np.array_equal(a, b)
        n += 1
    assert n > 10


def test_uniformly_spread_well_is_the_uniform_weight():
    """A well spread evenly over its subdomain gives w = 1/|Omega^i| again, for an
    injector and a producer alike (w = f / int f is positive and sums to 1)."""
    pr = W.unit_square_16(1)
    g = rt0.Grid(pr.n, pr.h)
    subs = ob.Substructuring(g, pr.cuts)
    i = 5                                   # an interior 4 x 4 subdomain
    for rate in (3.7, -0.4):
        src = np.zeros(g.ncells)
        src[subs.sub_cells[i]] = rate / 16
        src[subs.sub_cells[15][0]] = -rate  # compensating well far away
        w = ob.multiscale_weight(src, subs.sub_cells[i])
        assert np.allclose(w, 1.0 / 16, rtol=0, atol=1e-16) and abs(w.sum() - 1.0) <= 1e-15
        for k, pair in enumerate(subs.face_pairs):
            if i not in pair:
                continue
            a = ob.multiscale_face_flux(g, pr.perm, subs, *pair, subs.face_dofs[k], src)
            b = ob.multiscale_face_flux(g, pr.perm, subs, *pair, subs.face_dofs[k])
            assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


def test_cancelling_wells_keep_the_uniform_weight():
    cells = np.arange(4)
    src = np.array([1.0, -1.0, 0.0, 0.0])
    assert np.array_equal(ob.multiscale_weight(src, cells), np.full(4, 0.25))
    assert np.array_equal(ob.multiscale_weight(None, cells), np.full(4, 0.25))


def test_well_multiscale_bddc_solves():
    pr, src = _well_square(3)
    g = rt0.Grid(pr.n, pr.h)
    ue, _ = rt0.direct_solve(g, pr.perm, src)
    o = ob.BDDC(g, pr.perm, pr.cuts, multiscale=True, ms_source=src)
    out = o.solve(src, rtol=1e-12)
    assert np.linalg.norm(out["u"] - ue) <= 1e-9 * np.linalg.norm(ue)
    lmin, _, _ = ob.lanczos_kappa(out["alphas"], out["betas"])
    assert lmin >= 1 - 1e-8
