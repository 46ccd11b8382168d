"""Multiscale constraints (GPU): BDDC_MULTISCALE against the oracle's multiscale rows.

The face rows come from the Darcy problem on the two neighbours of each face
(Section 6), with the sources shaped by the wells of the solved source in the
subdomains that hold one (uniform elsewhere, and everywhere in the "uniform"
case); the oracle solves that problem literally, the GPU through the face's
reduced form (S^i_FF + S^j_FF)^{-1} (mu 1 - g), g the wells' face load.  On
the 16 x 16 square (two fields, and one with an extra interior well pair) and
a 20 x 20 x 10 cutout of the reservoir field (its injector column), both forms:
* the same number of rows per face;
* the preconditioner applied to a random interface vector (it depends on the
  span of the rows) within 1e-10 of the oracle's;
* solves: FP64 within 1e-8 with the oracle's iteration count, mixed within 1e-6
  and +-1 iteration.  On the cutout one row per face leaves the channels badly
  conditioned (about 700 iterations, where rounding moves the count by tens):
  there only the solutions are compared.
"""
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


def _case(name):
    if name == "square16_wells":
        pr = W.unit_square_16(2)
        src = pr.source.copy()
        src[5 + 16 * 6], src[6 + 16 * 6], src[0] = 0.7, -0.2, src[0] - 0.5
        return pr.n, pr.h, pr.perm, src, pr.cuts
    if name.startswith("square16"):
        pr = W.unit_square_16(int(name.split("_")[1]))
        return pr.n, pr.h, pr.perm, pr.source, pr.cuts
    full = W.reservoir_3d(nz=85, seed=0, tau=10.0)
    lo, ext = (20, 100, 30), (20, 20, 10)
    idx = np.arange(np.prod(full.n)).reshape(full.n, order="F")[
        lo[0]:lo[0] + ext[0], lo[1]:lo[1] + ext[1], lo[2]:lo[2] + ext[2]].reshape(-1, order="F")
    src = full.source[idx].copy()
    src -= src.mean()
    return ext, full.h, full.perm[idx], src, W.regular_cuts(ext, (10, 10, 5))


@pytest.mark.parametrize("name", ["square16_0", "square16_3", "square16_wells", "square16_0_uniform", "cutout"])
def test_multiscale_matches_oracle(name):
    Solver = _gpu()
    n, h, perm, src, cuts = _case(name)
    ms = None if name.endswith("uniform") else src
    o = ob.BDDC(rt0.Grid(n, h), perm, cuts, multiscale=True, ms_source=ms)
    ref = o.solve(src, rtol=1e-10)
    for prec, tol, dit in (("fp64", 1e-8, 0), ("mixed", 1e-6, 1)):
        s = Solver(n, h, perm, cuts, precision=prec, multiscale=True, ms_source=ms)
        try:
            st0 = s.stats()
            assert st0["n_adaptive"] == sum(o.face_k)
            assert np.array_equal(s.face_k(), np.array(o.face_k))
            if prec == "fp64":
                rng = np.random.default_rng(1)
                xu = rng.standard_normal(o.subs.n_gamma)
                zu, _ = s.apply_precond(xu)
                assert _relerr(zu, o.precondition(xu)[0]) <= 1e-10
            u, p = s.solve(src, rtol=1e-10)
            st = s.stats()
            print(f"{name} {prec}: rows {st0['n_adaptive']}, it {st['it']} (oracle {ref['it']}), "
                  f"flux {_relerr(u, ref['u']):.1e}", flush=True)
            # the cutout's channels leave the one-row-per-face space badly conditioned
            # (about 700 iterations, against 26 with the adaptive rows at tau = 10);
            # there rounding moves the count, which is compared only below 100
            if ref["it"] < 100:
                assert abs(st["it"] - ref["it"]) <= dit
            assert _relerr(u, ref["u"]) <= tol and _relerr(p, ref["p"]) <= tol
        finally:
            s.close()
