"""Uneven partitions (GPU): boxes of 4 to 16 cells per axis from seeded cut planes.

The SPE10-shaped field of the reservoir with cut-plane widths drawn from
[4, 16] gives subdomains from 4^3 to 16^3 cells (interfaces of up to 1,224
flux dofs, faces of up to 256) in one batch, tau = 5.

* A 30 x 30 x 16 cutout of the field (24 subdomains, boxes up to 14 x 14 x 11)
  is compared with the oracle: the preconditioner, S^i of the largest box, and
  whole solves (FP64 1e-8 with equal iterations, mixed 1e-6 within +-1).
* At full size (60 x 220 x 85, 1,260 subdomains) 32 seeded well placements are
  solved as one batch in both forms; checked are the divergence and flux rows
  of the global RT0 system (oracle matrices) for three of them, mixed against
  FP64 for all 32, and S^i of the largest box against the oracle on a cutout
  holding the box and its neighbours.
* Boxes at the LDS limits of the line kernels (source term, boundary loads,
  post-correction): 16^3-cell boxes, whose cell coefficients are still staged
  in LDS beside the kernels' vectors, and 20^3-cell boxes, where they no longer
  fit and are read in place; with wells and prescribed boundary fluxes, against
  the oracle's monolithic direct solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bddc as ob
from oracle import rt0

pytestmark = pytest.mark.gpu

TAU = 5.0


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_02090_amd import Solver
    return Solver


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _say(*a):
    print(*a, flush=True)


def _field():
    return W.reservoir_3d(nz=85, seed=0, tau=TAU)


def _sub_field(full, lo, ext):
    idx = np.arange(np.prod(full.n)).reshape(full.n, order="F")[
        lo[0]:lo[0] + ext[0], lo[1]:lo[1] + ext[1], lo[2]:lo[2] + ext[2]].reshape(-1, order="F")
    return full.perm[idx]


def _largest_box(cuts):
    w = [np.diff(c) for c in cuts]
    nsub = [len(x) for x in w]
    best, key = None, -1
    for k in range(int(np.prod(nsub))):
        s = (k % nsub[0], (k // nsub[0]) % nsub[1], k // (nsub[0] * nsub[1]))
        cells = w[0][s[0]] * w[1][s[1]] * w[2][s[2]]
        if cells > key:
            best, key = k, cells
    return best, nsub


def test_uneven_cutout_matches_oracle():
    Solver = _gpu()
    full = _field()
    n, lo = (30, 30, 16), (10, 90, 40)
    perm = _sub_field(full, lo, n)
    cuts = W.seeded_cuts(n, 4, 16, 2)
    src = W.five_spot(n, (15, 15))
    o = ob.BDDC(rt0.Grid(n, full.h), perm, cuts, tau=TAU)
    ref = o.solve(src, rtol=1e-8, maxit=3000)
    i, _ = _largest_box(cuts)
    for prec, tol, dit in (("fp64", 1e-8, 0), ("mixed", 1e-6, 1)):
        s = Solver(n, full.h, perm, cuts, tau=TAU, precision=prec)
        if prec == "fp64":
            assert s.N == 24
            So = ob.LocalProblem(rt0.Grid(n, full.h), perm, o.subs, i).schur()
            assert _relerr(s.schur(i), So) <= 1e-11
            rng = np.random.default_rng(4)
            xu = rng.standard_normal(o.subs.n_gamma)
            zu, _ = s.apply_precond(xu)
            assert _relerr(zu, o.precondition(xu)[0]) <= 1e-10
        u, p = s.solve(src, rtol=1e-8)
        st = s.stats()
        _say(f"uneven cutout {prec}: it {st['it']} (oracle {ref['it']}), flux {_relerr(u, ref['u']):.1e}, "
             f"pressure {_relerr(p, ref['p']):.1e}")
        assert abs(st["it"] - ref["it"]) <= dit
        assert _relerr(u, ref["u"]) <= tol and _relerr(p, ref["p"]) <= tol
        s.close()


@pytest.fixture(scope="module")
def full_batch():
    Solver = _gpu()
    full = _field()
    cuts = W.seeded_cuts(full.n, 4, 16, 0)
    srcs = np.stack([W.seeded_wells(full.n, np.random.default_rng(100 + k)) for k in range(32)])
    out = {"full": full, "cuts": cuts, "srcs": srcs}
    for prec in ("fp64", "mixed"):
        _say(f"uneven full size: {prec} setup")
        s = Solver(full.n, full.h, full.perm, cuts, tau=TAU, precision=prec, max_it=3000)
        flux, pres, its = s.solve_batch(srcs, rtol=1e-8)
        st = s.stats()
        _say(f"uneven full size: {prec}: N {st['n_sub']}, largest interface {s.max_gamma_local}, "
             f"iterations {its.min()}-{its.max()}, setup {st['t_setup_ms']:.0f} ms")
        out[prec] = (flux, pres, its, st)
        if prec == "fp64":
            out["solver"] = s
        else:
            s.close()
    yield out
    out["solver"].close()


def test_uneven_full_size_batch_properties(full_batch):
    full, srcs = full_batch["full"], full_batch["srcs"]
    g = rt0.Grid(full.n, full.h)
    A, B = rt0.global_matrices(g, full.perm)
    inner = ~g.boundary_faces()
    f64, mx = full_batch["fp64"], full_batch["mixed"]
    assert f64[3]["n_sub"] == 1260 and f64[3]["converged"] == 1
    assert (np.abs(f64[2] - mx[2]) <= 1).all()
    for k in (0, 13, 31):
        for name, (flux, pres, its, _) in (("fp64", f64), ("mixed", mx)):
            F = -srcs[k]
            div = np.linalg.norm(B @ flux[k] - F) / np.linalg.norm(F)
            Au = (A @ flux[k])[inner]
            fl = np.linalg.norm(Au + (B.T @ pres[k])[inner]) / np.linalg.norm(Au)
            _say(f"source {k} {name}: it {its[k]}, divergence rows {div:.1e}, flux rows {fl:.1e}")
            assert div <= 1e-9 and fl <= 1e-6
    for k in range(32):
        assert _relerr(mx[0][k], f64[0][k]) <= 1e-6
        assert _relerr(mx[1][k], f64[1][k]) <= 1e-6


def test_uneven_full_size_largest_box_schur(full_batch):
    full, cuts, s = full_batch["full"], full_batch["cuts"], full_batch["solver"]
    i, nsub = _largest_box(cuts)
    sub = (i % nsub[0], (i // nsub[0]) % nsub[1], i // (nsub[0] * nsub[1]))
    blo = [max(0, sub[d] - 1) for d in range(3)]
    bhi = [min(nsub[d], sub[d] + 2) for d in range(3)]
    c0 = [int(cuts[d][blo[d]]) for d in range(3)]
    ext = [int(cuts[d][bhi[d]]) - c0[d] for d in range(3)]
    perm = _sub_field(full, c0, ext)
    lcuts = [np.asarray(cuts[d][blo[d]:bhi[d] + 1]) - c0[d] for d in range(3)]
    g = rt0.Grid(tuple(ext), full.h)
    subs = ob.Substructuring(g, lcuts)
    loc = (sub[0] - blo[0]) + (bhi[0] - blo[0]) * ((sub[1] - blo[1]) + (bhi[1] - blo[1]) * (sub[2] - blo[2]))
    So = ob.LocalProblem(g, perm, subs, loc).schur()
    Sg = s.schur(i)
    _say(f"largest box {i}: n_gamma {Sg.shape[0]}, relerr {_relerr(Sg, So):.1e}")
    assert Sg.shape == So.shape and Sg.shape[0] > 500
    assert _relerr(Sg, So) <= 1e-11


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
@pytest.mark.parametrize("case", [
    ((48, 16, 16), 16, TAU),           # 4,096 cells: coefficients staged in LDS
    ((40, 20, 20), 20, float("inf")),  # 8,000 cells: read in place (faces of 400 dofs: no adaptive rows)
], ids=["16cube_staged", "20cube_in_place"])
def test_boxes_at_the_lds_limit(case, prec, tol):
    Solver = _gpu()
    n, b, tau = case
    full = _field()
    perm = _sub_field(full, (5, 100, 40), n)
    cuts = [np.arange(0, n[d] + 1, b) for d in range(3)]
    g = rt0.Grid(n, full.h)
    rng = np.random.default_rng(7)
    bnd = g.boundary_faces()
    bf = np.where(bnd, rng.standard_normal(g.nfaces), 0.0)
    dirs, coords = g.face_dir_coords()
    hi = coords[np.arange(g.nfaces), dirs] > 0
    outflow = np.sum(np.where(bnd & hi, bf, 0.0)) - np.sum(np.where(bnd & ~hi, bf, 0.0))
    src = W.seeded_wells(n, rng)
    src[0] += outflow
    ue, pe = rt0.direct_solve(g, perm, src, bflux=bf)
    pe = rt0.remove_mean(g, pe)
    s = Solver(n, full.h, perm, cuts, tau=tau, precision=prec, bflux=bf)
    try:
        u, p = s.solve(src, rtol=1e-11)
        st = s.stats()
    finally:
        s.close()
    _say(f"{b}^3 boxes {prec}: it {st['it']}, flux {_relerr(u, ue):.1e}, pressure {_relerr(p, pe):.1e}")
    assert st["converged"] == 1
    assert _relerr(u, ue) <= tol and _relerr(p, pe) <= tol
