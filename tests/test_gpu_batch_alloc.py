"""Several sources on one resident problem, and a caller-supplied allocator (GPU)."""
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_of_sources_equals_single_solves(prec):
    """bddc_solve_batch gives, source by source, the bits of bddc_solve."""
    _, Solver = _gpu()
    pr = W.layer_60x220(0, tau=10.0)
    rng = np.random.default_rng(3)
    srcs = np.stack([pr.source] + [W.seeded_wells(pr.n, rng) for _ in range(2)])
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0, precision=prec)
    flux, pres, its = s.solve_batch(srcs, rtol=1e-8)
    for k in range(len(srcs)):
        u, p = s.solve(srcs[k], rtol=1e-8)
        assert its[k] == s.stats()["it"]
        assert np.array_equal(flux[k], u) and np.array_equal(pres[k], p)
    assert len(set(its.tolist())) >= 1 and (its > 0).all()
    s.close()


def test_caller_allocator_gives_the_same_solve():
    """Device memory from torch's caching allocator: same bits, every block handed back."""
    torch, Solver = _gpu()
    from paper_1901_02090_amd import set_allocator
    pr = W.layer_60x220(0, tau=10.0)
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0)
    u0, p0 = s.solve(pr.source, rtol=1e-8)
    s.close()
    live = {}

    def alloc(n):
        ptr = torch.cuda.caching_allocator_alloc(n)
        live[ptr] = n
        return ptr

    def free(ptr):
        live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, free)
    try:
        s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0)
        assert len(live) > 10
        held = sum(live.values())
        assert abs(held - s.stats()["device_bytes"]) <= 1e-6 * held
        u, p = s.solve(pr.source, rtol=1e-8)
        assert np.array_equal(u, u0) and np.array_equal(p, p0)
        s.close()
        assert not live
    finally:
        set_allocator()


def test_solves_after_setup_allocate_nothing():
    """Setup allocates every device buffer a solve uses: solves on device pointers (graph replay after the
    first one, and eager) call the allocator no more, free nothing, and match the host-buffer solve bit for bit."""
    torch, Solver = _gpu()
    from paper_1901_02090_amd import set_allocator
    pr = W.layer_60x220(0, tau=10.0)
    n_alloc, n_free = [0], [0]

    def alloc(n):
        n_alloc[0] += 1
        return torch.cuda.caching_allocator_alloc(n)

    def free(ptr):
        n_free[0] += 1
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, free)
    try:
        s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=10.0, precision="mixed")
        src = torch.tensor(pr.source, dtype=torch.float64, device="cuda")
        flux = torch.empty(s.n_faces_all, dtype=torch.float64, device="cuda")
        pres = torch.empty(s.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        after_setup = (n_alloc[0], n_free[0])
        assert after_setup[0] > 10
        outs = []
        for eager in (False, False, True):
            s.solve_device(src.data_ptr(), 1e-8, flux.data_ptr(), pres.data_ptr(), eager=eager)
            torch.cuda.synchronize()
            outs.append((flux.cpu().numpy().copy(), pres.cpu().numpy().copy()))
        assert (n_alloc[0], n_free[0]) == after_setup
        u, p = s.solve(pr.source, rtol=1e-8)
        for fu, fp in outs:
            assert np.array_equal(fu, u) and np.array_equal(fp, p)
        s.close()
        assert n_free[0] == n_alloc[0]
    finally:
        set_allocator()
