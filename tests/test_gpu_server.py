"""Serving on the GPU: continuous batching over independent problems.

Each request of a mix (different grids, fields, wells, tau) is solved by the
server while others are set up or iterating beside it, and its result must be
the result of the same problem solved alone on its own handle, bit for bit
(every request's arithmetic is its own: no reduction spans requests).  The
server must keep to its slot count and admit by memory.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# 2D grids of several sizes, one 60x220x5 and one 60x220x17 slab, tau off and 10
SEEDS = [1, 2, 4, 6, 7, 8, 11]


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_02090_amd import Server, Solver
    return Server, Solver


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def alone():
    Server, Solver = _gpu()
    out = {}
    for prec in ("fp64", "mixed"):
        for sd in SEEDS:
            pr = W.serving_request(sd)
            s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=pr.tau, precision=prec)
            u, p = s.solve(pr.source, rtol=pr.rtol)
            out[prec, sd] = (u, p, s.stats()["it"])
            s.close()
    return out


def _submit_all(srv, seeds):
    return [(sd, srv.submit((pr := W.serving_request(sd)).n, pr.h, pr.perm, pr.cuts, pr.source, tau=pr.tau,
                            rtol=pr.rtol)) for sd in seeds]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mix_results_equal_alone(alone, prec):
    Server, _ = _gpu()
    srv = Server(precision=prec, max_active=3, setup_workers=2)
    tickets = _submit_all(srv, SEEDS)
    for sd, t in tickets:
        u, p, st = srv.result(t)
        ua, pa, ita = alone[prec, sd]
        _say(f"{prec} request {sd}: it {st['it']} (alone {ita}), latency {st['latency_ms']:.1f} ms, "
             f"queue {st['queue_ms']:.1f} setup {st['setup_ms']:.1f} solve {st['solve_ms']:.1f}, "
             f"est {st['est_bytes'] / 1e6:.1f} MB peak {st['peak_bytes'] / 1e6:.1f} MB")
        assert st["status"] == 0 and st["converged"] == 1
        assert st["it"] == ita
        assert np.array_equal(u, ua) and np.array_equal(p, pa)
    ss = srv.stats()
    _say(f"{prec}: {ss}")
    assert ss["completed"] == len(SEEDS) and ss["failed"] == 0 and ss["queued"] == 0 and ss["active"] == 0
    assert 2 <= ss["peak_active"] <= 3
    assert 0 < ss["p50_ms"] <= ss["p99_ms"]
    srv.close()


def test_admission_by_memory():
    """With a cap that holds the largest request but not two large ones, the
    large requests run one at a time and everything still completes."""
    Server, _ = _gpu()
    from paper_1901_02090_amd import estimate_bytes
    prs = [W.serving_request(sd) for sd in SEEDS]
    est = [estimate_bytes(pr.n, pr.h, pr.cuts, tau=pr.tau) for pr in prs]
    big = sorted(est)[-2:]
    cap = big[1] * 1.01
    assert big[0] + big[1] > cap
    srv = Server(precision="fp64", mem_cap=cap, max_active=4)
    tickets = _submit_all(srv, SEEDS)
    for (sd, t), e in zip(tickets, est):
        u, p, st = srv.result(t)
        assert st["status"] == 0 and st["est_bytes"] == e
        if np.isinf(W.serving_request(sd).tau):
            # without adaptivity every array is known in advance: the estimate bounds the real peak
            assert st["peak_bytes"] <= st["est_bytes"]
    ss = srv.stats()
    _say(f"capped at {cap / 1e6:.1f} MB: {ss}")
    assert ss["completed"] == len(SEEDS)
    assert ss["peak_bytes"] <= cap * 1.5
    srv.close()
    # a request larger than the whole cap is refused at once
    srv = Server(precision="fp64", mem_cap=min(est) * 0.5, max_active=2)
    pr = prs[0]
    from paper_1901_02090_amd.bddc import BddcError, BDDC_ENOMEM, BDDC_EINVAL
    with pytest.raises(BddcError) as e:
        srv.submit(pr.n, pr.h, pr.perm, pr.cuts, pr.source, tau=pr.tau)
    assert e.value.code == BDDC_ENOMEM
    srv.close()
    # a request that fails its setup leaves the others unharmed
    srv = Server(precision="fp64", max_active=2)
    bad = W.serving_request(SEEDS[0])
    src = bad.source.copy()
    src[0] += 1.0                        # sources no longer sum to zero
    tb = srv.submit(bad.n, bad.h, bad.perm, bad.cuts, src, tau=bad.tau)
    good = _submit_all(srv, SEEDS[:2])
    with pytest.raises(BddcError) as e:
        srv.result(tb)
    assert e.value.code == BDDC_EINVAL
    for sd, t in good:
        u, p, st = srv.result(t)
        assert st["status"] == 0
    ss = srv.stats()
    assert ss["failed"] == 1 and ss["completed"] == 2
    srv.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_keyed_requests_share_a_resident_problem_and_batch(prec, tol):
    """Requests under one problem key: the first sets the problem up, the
    rest find it resident (no setup) and the ones waiting together are solved
    in one block; every result must equal its own single solve (FP64 1e-8
    with equal iterations, mixed 1e-6 within +-1), beside unkeyed requests in
    the mix."""
    Server, Solver = _gpu()
    pr = W.serving_request(6)     # 32 x 125, tau 10
    rtol = pr.rtol
    rng = np.random.default_rng(5)
    srcs = [W.seeded_wells(pr.n, rng) for _ in range(9)]
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=pr.tau, precision=prec)
    ref = []
    for src in srcs:
        u, p = s.solve(src, rtol=rtol)
        ref.append((u, p, s.stats()["it"]))
    s.close()
    srv = Server(precision=prec, max_active=3, setup_workers=2)
    other = _submit_all(srv, [1, 4])
    tk = [srv.submit(pr.n, pr.h, pr.perm, pr.cuts, src, tau=pr.tau, rtol=rtol, key=42) for src in srcs]
    out = [srv.result(t) for t in tk]
    for sd, t in other:
        srv.result(t)
    # a second wave finds the problem resident
    tk2 = [srv.submit(pr.n, pr.h, pr.perm, pr.cuts, src, tau=pr.tau, rtol=rtol, key=42) for src in srcs[:3]]
    out2 = [srv.result(t) for t in tk2]
    with pytest.raises(Exception):
        bad = W.serving_request(1)
        srv.submit(bad.n, bad.h, bad.perm, bad.cuts, bad.source, tau=bad.tau, rtol=bad.rtol, key=42)
    srv.close()
    batches = []
    for k, (u, p, st) in enumerate(out + out2):
        ua, pa, ita = ref[k % 9] if k < 9 else ref[k - 9]
        eu = np.linalg.norm(u - ua) / np.linalg.norm(ua)
        ep = np.linalg.norm(p - pa) / np.linalg.norm(pa)
        batches.append(st["batch"])
        _say(f"{prec} keyed request {k}: batch {st['batch']}, reused {st['reused']}, it {st['it']} (alone {ita}), "
             f"setup {st['setup_ms']:.1f} ms, latency {st['latency_ms']:.1f} ms, flux {eu:.1e}, pressure {ep:.1e}")
        assert eu <= tol and ep <= tol
        assert abs(st["it"] - ita) <= (0 if prec == "fp64" else 1)
    assert sum(st["reused"] for _, _, st in out) == 8 and all(st["reused"] for _, _, st in out2)
    assert max(batches) > 1
