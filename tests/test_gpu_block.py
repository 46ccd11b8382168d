"""Block CG (bddc_solve_block): several sources per CG iteration on the GPU.

Each source of a block keeps its own CG scalars and stopping test, so it must
give the result of its single solve (which the other GPU tests pin to the
oracle): FP64 within 1e-8 with equal iterations, mixed within 1e-6 and +-1
iteration.  Cases: the 16 x 16 square (partial block of 5), the 60 x 220
layer at tau = 10 (20 sources: a full block and a padded one), a ragged 3D
grid, and an uneven cutout of the reservoir field at tau = 5 with prescribed
boundary fluxes (18 sources).  Also: one block source against the oracle
directly, the captured-graph block iterations against eager launches (bit
for bit), device pointers against host buffers, and the argument checks.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bddc as ob
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


def _say(*a):
    print(*a, flush=True)


def _sources(n, k, seed, outflow=0.0):
    rng = np.random.default_rng(seed)
    srcs = np.stack([W.seeded_wells(n, rng) for _ in range(k)])
    srcs[:, 0] += outflow
    return srcs


def _ragged3d():
    rng = np.random.default_rng(3)
    n3 = (5, 4, 6)
    rng.normal(0, 2, (63, 2))
    k3 = np.exp(rng.normal(0, 1.5, (120, 3)))
    return n3, (1.0, 2.0, 0.5), k3, [np.array([0, 2, 5]), np.array([0, 3, 4]), np.array([0, 2, 4, 6])]


def _uneven():
    full = W.reservoir_3d(nz=85, seed=0, tau=5.0)
    n, lo = (30, 30, 16), (10, 90, 40)
    idx = np.arange(np.prod(full.n)).reshape(full.n, order="F")[
        lo[0]:lo[0] + n[0], lo[1]:lo[1] + n[1], lo[2]:lo[2] + n[2]].reshape(-1, order="F")
    return n, full.h, full.perm[idx], W.seeded_cuts(n, 4, 16, 2)


def _case(name):
    """(n, h, perm, cuts, tau, rtol, sources, bflux)"""
    if name == "square16":
        pr = W.unit_square_16(0)
        return pr.n, pr.h, pr.perm, pr.cuts, 3.0, 1e-10, _sources(pr.n, 5, 11), None
    if name == "layer":
        pr = W.layer_60x220(0, tau=10.0)
        return pr.n, pr.h, pr.perm, pr.cuts, 10.0, 1e-8, _sources(pr.n, 20, 12), None
    if name == "ragged3d":
        n, h, k, cuts = _ragged3d()
        return n, h, k, cuts, 3.0, 1e-10, _sources(n, 3, 13), None
    n, h, perm, cuts = _uneven()
    g = rt0.Grid(n, h)
    rng = np.random.default_rng(14)
    bnd = g.boundary_faces()
    bf = np.where(bnd, rng.standard_normal(g.nfaces), 0.0)
    dirs, coords = g.face_dir_coords()
    hi = coords[np.arange(g.nfaces), dirs] > 0
    outflow = np.sum(np.where(bnd & hi, bf, 0.0)) - np.sum(np.where(bnd & ~hi, bf, 0.0))
    return n, h, perm, cuts, 5.0, 1e-8, _sources(n, 18, 15, outflow), bf


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["square16", "layer", "ragged3d", "uneven_bflux"])
def test_block_equals_single_solves(name, prec):
    Solver = _gpu()
    n, h, perm, cuts, tau, rtol, srcs, bf = _case(name)
    s = Solver(n, h, perm, cuts, tau=tau, precision=prec, bflux=bf)
    try:
        fb, pb, itb = s.solve_block(srcs, rtol=rtol)
        stb = s.stats()
        worst = (0, 0.0, 0.0)
        for k in range(len(srcs)):
            u, p = s.solve(srcs[k], rtol=rtol)
            it = s.stats()["it"]
            eu, ep = _relerr(fb[k], u), _relerr(pb[k], p)
            worst = (max(worst[0], abs(int(itb[k]) - it)), max(worst[1], eu), max(worst[2], ep))
            if prec == "fp64":
                assert itb[k] == it, (k, itb[k], it)
                assert eu <= 1e-8 and ep <= 1e-8, (k, eu, ep)
            else:
                assert abs(int(itb[k]) - it) <= 1, (k, itb[k], it)
                assert eu <= 1e-6 and ep <= 1e-6, (k, eu, ep)
        _say(f"block {name} {prec}: {len(srcs)} sources, iterations {itb.min()}-{itb.max()}, "
             f"worst |d it| {worst[0]}, flux {worst[1]:.1e}, pressure {worst[2]:.1e}; last kappa {stb['kappa']:.3f}")
        assert stb["it"] == itb[-1]
    finally:
        s.close()


def test_block_source_matches_oracle():
    Solver = _gpu()
    pr = W.unit_square_16(0)
    srcs = _sources(pr.n, 3, 21)
    o = ob.BDDC(rt0.Grid(pr.n, pr.h), pr.perm, pr.cuts, tau=3.0)
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=3.0)
    try:
        fb, pb, itb = s.solve_block(srcs, rtol=1e-10)
    finally:
        s.close()
    for k in range(3):
        ref = o.solve(srcs[k], rtol=1e-10)
        assert itb[k] == ref["it"]
        assert _relerr(fb[k], ref["u"]) <= 1e-8 and _relerr(pb[k], ref["p"]) <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_graph_equals_eager_and_device_pointers(prec):
    import torch
    Solver = _gpu()
    pr = W.layer_60x220(0, tau=10.0)
    srcs = _sources(pr.n, 7, 31)
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0, precision=prec)
    try:
        f1, p1, i1 = s.solve_block(srcs, rtol=1e-8)
        f2, p2, i2 = s.solve_block(srcs, rtol=1e-8, eager=True)
        d_src = torch.tensor(srcs, dtype=torch.float64, device="cuda")
        d_f = torch.empty((7, s.n_faces_all), dtype=torch.float64, device="cuda")
        d_p = torch.empty((7, s.n_cells), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        i3 = s.solve_block_device(7, d_src.data_ptr(), 1e-8, d_f.data_ptr(), d_p.data_ptr())
        torch.cuda.synchronize()
        f3, p3 = d_f.cpu().numpy(), d_p.cpu().numpy()
    finally:
        s.close()
    assert np.array_equal(i1, i2) and np.array_equal(i1, i3)
    assert np.array_equal(f1, f2) and np.array_equal(p1, p2)
    assert np.array_equal(f1, f3) and np.array_equal(p1, p3)


def test_block_argument_checks():
    from paper_1901_02090_amd import BddcError
    Solver = _gpu()
    pr = W.unit_square_16(0)
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=3.0)
    try:
        f, p, its = s.solve_block(np.zeros((0, s.n_cells)))
        assert f.shape == (0, s.n_faces_all) and len(its) == 0
        bad = _sources(pr.n, 2, 1)
        bad[1, 0] += 1.0                      # does not sum to zero
        with pytest.raises(BddcError):
            s.solve_block(bad)
        # every source zero: each stops at once with zero flux
        f, p, its = s.solve_block(np.zeros((2, s.n_cells)))
        assert (its == 0).all() and not f.any()
    finally:
        s.close()
