"""Host side of serving: the admission estimate and the request generator (no GPU)."""
import math
import os

import numpy as np
import pytest

import workloads as W


def _lib():
    from paper_1901_02090_amd import bddc
    if not os.path.exists(bddc.LIB_PATH):
        pytest.skip("libbddc.so not built")
    return bddc


def test_estimate_is_host_only_and_grows_with_the_problem():
    b = _lib()
    sq = W.unit_square_16(0)
    small = b.estimate_bytes(sq.n, sq.h, sq.cuts)
    lay = W.layer_60x220(0)
    mid = b.estimate_bytes(lay.n, lay.h, lay.cuts)
    mid_ad = b.estimate_bytes(lay.n, lay.h, lay.cuts, tau=10.0)
    slab = W.serving_request(3)          # 60 x 220 x 34 slab
    big = b.estimate_bytes(slab.n, slab.h, slab.cuts)
    assert 0 < small < mid < mid_ad < big
    # the local dense workspaces alone are a lower bound: per subdomain
    # (2 n_c^2 + n_c (n_G + 1) + 3 n_G^2) doubles, with n_c cells
    nc = 10 * 10
    assert mid > 132 * 8 * 2 * nc * nc


def test_estimate_rejects_bad_partitions():
    b = _lib()
    lay = W.layer_60x220(0)
    bad = [np.array([0, 30, 30, 60]), lay.cuts[1]]
    with pytest.raises(b.BddcError) as e:
        b.estimate_bytes(lay.n, lay.h, bad)
    assert e.value.code == b.BDDC_EINVAL


def test_serving_requests_are_seeded_and_valid():
    for seed in range(24):
        pr = W.serving_request(seed)
        again = W.serving_request(seed)
        assert np.array_equal(pr.perm, again.perm) and np.array_equal(pr.source, again.source)
        assert abs(pr.source.sum()) <= 1e-12 and np.count_nonzero(pr.source) >= 2
        assert (pr.perm > 0).all() and np.isfinite(pr.perm).all()
        if pr.dim == 2:
            assert 32 <= pr.n[0] <= 60 and 32 <= pr.n[1] <= 220
        else:
            assert pr.n[:2] == (60, 220) and pr.n[2] in (5, 17, 34)
        for d in range(pr.dim):
            c = np.asarray(pr.cuts[d])
            assert c[0] == 0 and c[-1] == pr.n[d] and (np.diff(c) > 0).all() and np.diff(c).max() <= 32
        assert pr.tau == 10.0 or math.isinf(pr.tau)
    t = W.poisson_arrivals(50.0, 2000, 0)
    assert (np.diff(t) > 0).all() and abs(np.diff(t).mean() - 1 / 50.0) < 0.1 / 50.0
