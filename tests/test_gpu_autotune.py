"""The autotuner of the per-iteration launch shapes (BDDC_AUTOTUNE, GPU).

It times four lane-group width policies of the coarse sweeps and four T^i
grids on the problem's own operators and keeps the fastest.  The tuned solver
must solve as the default one: the widths only change the order in which a
sweep row is summed, the grid only which workgroup takes which subdomain.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

WIDTHS = [(8, 32), (12, 48), (24, 96), (48, 192)]


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_02090_amd import Solver
    return Solver


def _relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("top", [0, -1], ids=["dense_top", "all_swept"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotuned_solver_solves_as_the_default(prec, top):
    """On the 60x220 layer the default dense top block takes the whole coarse
    problem (nothing to sweep, the sweep widths are not timed); with
    coarse_top = -1 every level is swept."""
    Solver = _gpu()
    pr = W.layer_60x220(0, tau=10.0)
    s0 = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0, precision=prec, coarse_top=top)
    u0, p0 = s0.solve(pr.source, rtol=1e-8)
    st0 = s0.stats()
    s0.close()
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0, precision=prec, autotune=True, coarse_top=top)
    st = s.stats()
    print(f"{prec}: tuned widths ({st['sweep_wide4']}, {st['sweep_wide16']}), T^i on {st['t_workgroups']} "
          f"workgroups, {st['t_tune_ms']:.1f} ms; coarse {np.round(st['tune_coarse_ms'], 4)} ms, "
          f"preconditioner {np.round(st['tune_precond_ms'], 4)} ms", flush=True)
    assert st["t_tune_ms"] > 0
    assert all(t > 0 for t in st["tune_precond_ms"])
    k = WIDTHS.index((st["sweep_wide4"], st["sweep_wide16"]))
    if top == 0:
        assert st["coarse_dense"] == st["n_coarse"] - 1 and not any(st["tune_coarse_ms"]) and k == 2
    else:
        assert st["coarse_dense"] == 0 and all(t > 0 for t in st["tune_coarse_ms"])
        assert st["tune_coarse_ms"][k] == min(st["tune_coarse_ms"])
        # bottom-subtree depths 0, 1, ... up to the swept levels, the fastest kept
        ts = st["tune_subtree_ms"]
        timed = [c for c in range(len(ts)) if ts[c] > 0]
        assert timed == list(range(len(timed))) and len(timed) >= 2
        assert ts[st["sweep_subtree_levels"]] == min(ts[c] for c in timed)
        print(f"  subtree levels {st['sweep_subtree_levels']}: coarse {np.round(ts, 4)} ms", flush=True)
        tw = st["tune_wide1_ms"]
        assert all(x > 0 for x in tw) and tw[[0, 8, 16, 32].index(st["sweep_wide1"])] == min(tw)
        print(f"  single-lane rows up to {st['sweep_wide1']}: coarse {np.round(tw, 4)} ms", flush=True)
    assert 1 <= st["t_workgroups"] <= st["n_sub"]
    u, p = s.solve(pr.source, rtol=1e-8)
    st1 = s.stats()
    s.close()
    assert abs(st1["it"] - st0["it"]) <= (0 if prec == "fp64" else 1)
    assert _relerr(u, u0) <= 1e-10 and _relerr(p, p0) <= 1e-10
