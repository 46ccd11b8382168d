"""Bottom-subtree sweeps of the coarse solve (option coarse_subtree, GPU).

The levels 0 .. k-1 of the coarse tree are swept by one launch per direction,
one workgroup per subtree taking the subtree's levels in turn; the levels
above keep one launch per level.  Every sweep row and column is formed by the
same lane-group arithmetic as in the level launches, so the solves must give
the same bits as with one launch per level, for every k (k beyond the swept
levels takes them all; with a dense top block the subtrees stop below it).
The parity of the level launches with the oracle is covered by the other GPU
tests.  Rows and columns of at most sweep_single entries are taken by one
lane each (a row summed in another order than by a lane group): the same
solution to 1e-10 with the same iterations.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_02090_amd import Solver
    return Solver


def _uneven():
    full = W.reservoir_3d(nz=85, seed=0, tau=5.0)
    n, lo = (30, 30, 16), (10, 90, 40)
    idx = np.arange(np.prod(full.n)).reshape(full.n, order="F")[
        lo[0]:lo[0] + n[0], lo[1]:lo[1] + n[1], lo[2]:lo[2] + n[2]].reshape(-1, order="F")
    return n, full.h, full.perm[idx], W.seeded_cuts(n, 4, 16, 2), 5.0


def _case(name):
    """(n, h, perm, cuts, tau, coarse_top)"""
    if name == "layer_swept":
        pr = W.layer_60x220(0, tau=10.0)
        return pr.n, pr.h, pr.perm, pr.cuts, 10.0, -1
    if name == "layer_top300":
        pr = W.layer_60x220(0, tau=10.0)
        return pr.n, pr.h, pr.perm, pr.cuts, 10.0, 300
    n, h, perm, cuts, tau = _uneven()
    return n, h, perm, cuts, tau, 100   # a dense top block of at most 100 dofs, the levels below swept


@pytest.mark.parametrize("single", [0, 16], ids=["groups", "single16"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["layer_swept", "layer_top300", "uneven"])
def test_subtree_sweeps_give_the_level_launch_bits(name, prec, single):
    """single: rows and columns of up to 16 entries taken by one lane each."""
    Solver = _gpu()
    n, h, perm, cuts, tau, top = _case(name)
    rng = np.random.default_rng(7)
    src = W.seeded_wells(n, rng)
    s = Solver(n, h, perm, cuts, tau=tau, precision=prec, coarse_top=top, coarse_subtree=-1, sweep_single=single)
    try:
        u0, p0 = s.solve(src, rtol=1e-8)
        st0 = s.stats()
    finally:
        s.close()
    assert st0["sweep_subtree_levels"] == 0
    swept = st0["coarse_levels"] if top < 0 else None
    for k in (1, 2, 4, 99):
        s = Solver(n, h, perm, cuts, tau=tau, precision=prec, coarse_top=top, coarse_subtree=k,
                   sweep_single=single)
        try:
            u, p = s.solve(src, rtol=1e-8)
            st = s.stats()
        finally:
            s.close()
        lv = st["sweep_subtree_levels"]
        print(f"{name} {prec} single {single}: coarse_subtree {k} -> {lv} of {st['coarse_levels']} levels "
              f"(dense top {st['coarse_dense']} dofs), {st['it']} iterations", flush=True)
        assert 1 <= lv <= k
        if swept is not None:
            assert lv == min(k, swept)
        assert st["it"] == st0["it"]
        assert np.array_equal(u, u0) and np.array_equal(p, p0)


@pytest.mark.parametrize("single", [8, 32, 100000])
def test_single_lane_rows_solve_as_lane_groups(single):
    """Single-lane rows sum a row in another order than lane groups: the same
    iterations (FP64) and the same solution to 1e-10."""
    Solver = _gpu()
    n, h, perm, cuts, tau, top = _case("layer_swept")
    src = W.seeded_wells(n, np.random.default_rng(8))
    out = []
    for sg in (0, single):
        s = Solver(n, h, perm, cuts, tau=tau, coarse_top=top, sweep_single=sg)
        try:
            u, p = s.solve(src, rtol=1e-10)
            out.append((u, p, s.stats()["it"], s.stats()["sweep_wide1"]))
        finally:
            s.close()
    (u0, p0, it0, w0), (u1, p1, it1, w1) = out
    assert w0 == 0 and w1 == single
    assert it1 == it0
    assert np.linalg.norm(u1 - u0) <= 1e-10 * np.linalg.norm(u0)
    assert np.linalg.norm(p1 - p0) <= 1e-10 * np.linalg.norm(p0)
