"""bddc_solve_noalloc: the solve that allocates no device memory (GPU).

Its CG scratch lives in the library's static device array; its result must be
that of bddc_solve on the same source.  Two calls in a row on two handles, the
second on a smaller problem, then the first again, each compared with the
existing entry point; neither call may reach the allocator.
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
    return torch, Solver


def _dev(torch, s, source):
    src = torch.tensor(source, dtype=torch.float64, device="cuda")
    flux = torch.empty(s.n_faces_all, dtype=torch.float64, device="cuda")
    pres = torch.empty(s.n_cells, dtype=torch.float64, device="cuda")
    return src, flux, pres


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_solve_matches_solve(prec):
    torch, Solver = _gpu()
    from paper_1901_02090_amd import set_allocator
    n_alloc, n_free = [0], [0]

    def alloc(n):
        n_alloc[0] += 1
        return torch.cuda.caching_allocator_alloc(n)

    def free(ptr):
        n_free[0] += 1
        torch.cuda.caching_allocator_delete(ptr)

    big = W.layer_60x220(0, tau=10.0)
    small = W.unit_square_16(0)
    set_allocator(alloc, free)
    try:
        sb = Solver(big.n, big.h, big.perm, big.cuts, tau=10.0, precision=prec)
        ss = Solver(small.n, small.h, small.perm, small.cuts, tau=3.0, precision=prec)
        cases = []
        for s, pr, rtol in ((sb, big, 1e-8), (ss, small, 1e-10)):
            src, flux, pres = _dev(torch, s, pr.source)
            s.solve_device(src.data_ptr(), rtol, flux.data_ptr(), pres.data_ptr())
            torch.cuda.synchronize()
            ref = (flux.cpu().numpy().copy(), pres.cpu().numpy().copy(), s.stats())
            cases.append((s, rtol, src, ref))
        torch.cuda.synchronize()
        before = (n_alloc[0], n_free[0])
        # big, then the smaller problem, then big again: every call against bddc_solve
        for s, rtol, src, (u_ref, p_ref, st_ref) in (cases[0], cases[1], cases[0]):
            flux = torch.full((s.n_faces_all,), np.nan, dtype=torch.float64, device="cuda")
            pres = torch.full((s.n_cells,), np.nan, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            mark = (n_alloc[0], n_free[0])
            s.solve_noalloc(src.data_ptr(), rtol, flux.data_ptr(), pres.data_ptr())
            torch.cuda.synchronize()
            assert (n_alloc[0], n_free[0]) == mark
            st = s.stats()
            print(f"noalloc N={st['n_sub']} it {st['it']} (solve {st_ref['it']}) kappa {st['kappa']:.4f}",
                  flush=True)
            assert st["it"] == st_ref["it"] and st["converged"] == 1
            assert st["kappa"] == pytest.approx(st_ref["kappa"], rel=1e-12)
            u, p = flux.cpu().numpy(), pres.cpu().numpy()
            assert np.array_equal(u, u_ref) and np.array_equal(p, p_ref)
        assert (n_alloc[0], n_free[0]) == before
        sb.close()
        ss.close()
        assert n_free[0] == n_alloc[0]
    finally:
        set_allocator()


def test_noalloc_refuses_a_history_beyond_the_scratch():
    torch, Solver = _gpu()
    from paper_1901_02090_amd.bddc import BddcError, BDDC_EINVAL
    pr = W.unit_square_16(0)
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, max_it=40000)
    src, flux, pres = _dev(torch, s, pr.source)
    with pytest.raises(BddcError) as e:
        s.solve_noalloc(src.data_ptr(), 1e-10, flux.data_ptr(), pres.data_ptr())
    assert e.value.code == BDDC_EINVAL and "max_it" in str(e.value)
    s.close()
