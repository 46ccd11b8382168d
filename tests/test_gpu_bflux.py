"""Prescribed boundary fluxes (eq. problem-4) on the GPU: bddc_options.bflux.

* Section 2's closed form: at constant k a linear pressure p = a.x lies in
  RT0 x P0, so with the boundary fluxes of u = -k grad p (total flux through
  each boundary face) and no source the discrete solution is the flux
  interpolant and the cell-centre pressures, in 2D and 3D, through the whole
  BDDC path (steps 1-3 and the post-correction) with several subdomains
  along each axis, including boxes one cell thick;
* against the oracle's monolithic direct solve with boundary fluxes on a
  heterogeneous field with wells, both forms (1e-8 / 1e-6);
* the compatibility check: a source that does not sum to the net boundary
  outflow is refused.
"""
import numpy as np
import pytest

import workloads as W
from oracle import rt0

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_02090_amd import Solver
    return Solver


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _linear(n, h, k, a):
    g = rt0.Grid(n, h)
    dim = len(n)
    dirs, _ = g.face_dir_coords()
    area = np.array([np.prod([h[e] for e in range(dim) if e != d]) for d in range(dim)])
    uex = -np.asarray(k)[dirs] * np.asarray(a)[dirs] * area[dirs]
    cc = g.cell_coords()
    pex = sum(a[d] * (cc[d] + 0.5) * h[d] for d in range(dim))
    perm = np.tile(np.asarray(k, dtype=float), (g.ncells, 1))
    return g, perm, uex, rt0.remove_mean(g, pex)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", [
    ((12, 10), (0.5, 1.3), (2.0, 0.5), (0.7, -1.3), ([0, 4, 8, 12], [0, 1, 6, 10])),
    ((60, 220), (20.0, 10.0), (3.0, 3.0), (1e-3, 2e-3), None),
    ((6, 8, 5), (20.0, 10.0, 2.0), (1.5, 1.5, 0.15), (0.7, -1.3, 0.4), ([0, 3, 6], [0, 4, 8], [0, 1, 5])),
], ids=["2d_thin_boxes", "layer", "3d"])
def test_linear_pressure_is_reproduced(case, prec):
    Solver = _gpu()
    n, h, k, a, cuts = case
    if cuts is None:
        cuts = W.regular_cuts(n, (10, 10))
    g, perm, uex, pex = _linear(n, h, k, a)
    bnd = g.boundary_faces()
    s = Solver(n, h, perm, cuts, precision=prec, bflux=np.where(bnd, uex, 0.0))
    try:
        u, p = s.solve(np.zeros(g.ncells), rtol=1e-13)
        st = s.stats()
    finally:
        s.close()
    eu = np.abs(u - uex).max() / np.abs(uex).max()
    ep = np.abs(p - pex).max() / np.abs(pex).max()
    print(f"linear {n} {prec}: it {st['it']}, flux {eu:.1e}, pressure {ep:.1e}", flush=True)
    assert np.array_equal(u[bnd], uex[bnd])
    assert eu <= 1e-11 and ep <= 1e-11


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("dim", [2, 3])
def test_matches_direct_solve_with_boundary_fluxes(dim, prec, tol):
    Solver = _gpu()
    rng = np.random.default_rng(40 + dim)
    if dim == 2:
        pr = W.layer_60x220(0, tau=10.0)
        n, h, perm, cuts, tau = pr.n, pr.h, pr.perm, pr.cuts, 10.0
    else:
        full = W.reservoir_3d(nz=85, seed=0, tau=10.0)
        n, h = (20, 20, 10), full.h
        idx = np.arange(np.prod(full.n)).reshape(full.n, order="F")[20:40, 100:120, 30:40].reshape(-1, order="F")
        perm, cuts, tau = full.perm[idx], W.regular_cuts(n, (10, 10, 5)), 10.0
    g = rt0.Grid(n, h)
    bnd = g.boundary_faces()
    bf = np.where(bnd, rng.standard_normal(g.nfaces), 0.0)
    dirs, coords = g.face_dir_coords()
    hi = coords[np.arange(g.nfaces), dirs] > 0
    outflow = np.sum(np.where(bnd & hi, bf, 0.0)) - np.sum(np.where(bnd & ~hi, bf, 0.0))
    src = W.seeded_wells(n, rng)
    src[0] += outflow                      # the source carries the net outflow
    ue, pe = rt0.direct_solve(g, perm, src, bflux=bf)
    pe = rt0.remove_mean(g, pe)
    s = Solver(n, h, perm, cuts, tau=tau, precision=prec, bflux=bf)
    try:
        u, p = s.solve(src, rtol=1e-11)
        st = s.stats()
        bad = src.copy()
        bad[0] += 1.0
        with pytest.raises(Exception):
            s.solve(bad, rtol=1e-8)
    finally:
        s.close()
    print(f"bflux {dim}D {prec}: it {st['it']}, flux {_relerr(u, ue):.1e}, pressure {_relerr(p, pe):.1e}",
          flush=True)
    assert _relerr(u, ue) <= tol and _relerr(p, pe) <= tol
