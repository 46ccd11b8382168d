"""Oracle pins for stiffness scaling of the averaging operator E (Section 6).

The paper uses stiffness scaling (for RT0 the same as rho-scaling) when the
coefficient jumps follow the subdomain interfaces, and the multiplicity
weights 1/2 otherwise; the starting flux constraints need the weights to be
constant along each face.  Pinned by:
* weights: the two copies of every interface dof sum to 1, constant per face;
  a homogeneous field gives exactly 1/2 and the multiplicity results bit for bit;
* robustness: with permeability constant per subdomain (jumps of up to 1e4 on
  the interfaces) the stiffness-scaled preconditioned operator has a condition
  number below 3, the multiplicity-scaled one above 100 (the reason the paper
  switches scalings);
* solves reproduce the direct solution;
* adaptive rows with stiffness weights are refused (the pair eigenproblems
  assume 1/2).
"""

import numpy as np
import pytest

import workloads as W
from oracle import bddc as ob
from oracle import rt0

N2, H2 = (16, 16), (1 / 16, 1 / 16)


def _boxwise(kb):
    """Permeability constant on each 4 x 4 box of the 16 x 16 square."""
    k = np.array([kb[x // 4, y // 4] for y in range(16) for x in range(16)])
    return np.stack([k, k], 1)


def _fields():
    rng = np.random.default_rng(0)
    yield "lognormal", _boxwise(rng.lognormal(0, 3, (4, 4)))
    yield "checker", _boxwise(np.array([[1e4 if (bx + by) % 2 else 1.0 for by in range(4)] for bx in range(4)]))


def test_weights_partition_unity_and_homogeneous_limit():
    g = rt0.Grid(N2, H2)
    cuts = W.regular_cuts(N2, (4, 4))
    name, perm = next(_fields())
    o = ob.BDDC(g, perm, cuts, scaling="stiffness")
    tot = np.zeros(o.subs.n_gamma)
    for i, lp in enumerate(o.loc):
        tot[o.subs.gamma_pos[lp.G]] += o.weight[i]
    assert np.allclose(tot, 1.0, rtol=0, atol=1e-15)
    for k, (i, j) in enumerate(o.subs.face_pairs):
        pi, pj = o.face_pos[k]
        assert np.ptp(o.weight[i][pi]) == 0.0 and np.ptp(o.weight[j][pj]) == 0.0
    hom = W.homogeneous(N2, H2, cuts)
    a = ob.BDDC(g, hom.perm, cuts)
    b = ob.BDDC(g, hom.perm, cuts, scaling="stiffness")
    assert all(np.array_equal(w, np.full(len(w), 0.5)) for w in b.weight)
    ra, rb = a.solve(hom.source, rtol=1e-10), b.solve(hom.source, rtol=1e-10)
    assert ra["it"] == rb["it"] and np.array_equal(ra["u"], rb["u"])


@pytest.mark.parametrize("field", list(_fields()), ids=lambda f: f[0])
def test_stiffness_scaling_robust_for_aligned_jumps(field):
    _, perm = field
    g = rt0.Grid(N2, H2)
    cuts = W.regular_cuts(N2, (4, 4))
    src = W.corner_pair(N2)
    ue, _ = rt0.direct_solve(g, perm, src)
    kap = {}
    for sc in ("multiplicity", "stiffness"):
        out = ob.BDDC(g, perm, cuts, scaling=sc).solve(src, rtol=1e-10, maxit=400)
        kap[sc] = out["kappa"]
        if sc == "stiffness":
            assert out["converged"]
            assert np.linalg.norm(out["u"] - ue) <= 1e-8 * np.linalg.norm(ue)
    assert kap["stiffness"] < 3.0 < 100.0 < kap["multiplicity"]


def test_adaptive_rows_with_stiffness_weights_refused():
    g = rt0.Grid(N2, H2)
    name, perm = next(_fields())
    with pytest.raises(ValueError):
        ob.BDDC(g, perm, W.regular_cuts(N2, (4, 4)), tau=3.0, scaling="stiffness")
    ob.BDDC(g, perm, W.regular_cuts(N2, (4, 4)), multiscale=True, scaling="stiffness")   # allowed
