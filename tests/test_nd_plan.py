"""Host logic of the coarse multifrontal solver: the nested-dissection plan.

The plan (csrc/nd.hpp) is compiled into a small host driver and checked here
without a GPU.  A random saddle point with the coarse problem's structure (one
dense SPD clique per subdomain on its face dofs, divergence rows -d_i * (+-1)
coupling each pressure to its face averages, last pressure pinned) is factored
and solved by a numpy transcription of the index arithmetic of the device
kernels (front assembly, extend-add, partial signed Cholesky, packed R storage,
push-form forward / backward sweeps).  The result must equal a dense solve, the
pivot signs must be +1 on face dofs and -1 on pressures, every packed entry and
every sweep row / column must be produced exactly once, and every B-vector
entry must be filled before it is read.  With a dense top block the levels
below it are swept, the top right-hand side is gathered through the plan's
map, and the top dofs are solved with the Schur complement of the coarse matrix
on them (formed here from the dense matrix, independently of the factor).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "nd_plan_dump.cpp")


@pytest.fixture(scope="module")
def dumper(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("nd") / "nd_plan_dump")
    subprocess.run([gxx, "-O1", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, SRC], check=True)
    return exe


SCALARS = ("N", "nF", "H", "nfr", "nk", "top", "nt", "sub_lv", "nsubt")


def load(exe, args, top=None, sub=None, w1=None):
    env = dict(os.environ)
    env.pop("ND_TOP", None)
    env.pop("ND_SUB", None)
    env.pop("ND_W1", None)
    if w1 is not None:
        env["ND_W1"] = str(w1)
    if top is not None:
        env["ND_TOP"] = str(top)
    if sub is not None:
        env["ND_SUB"] = str(sub)
    out = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, check=True,
                         env=env).stdout
    d = {}
    for line in out.splitlines():
        t = line.split()
        if t[0] in SCALARS:
            d[t[0]] = int(t[1])
        else:
            d[t[0]] = np.array([int(x) for x in t[2:]], dtype=np.int64)
            assert len(d[t[0]]) == int(t[1])
    return d


def coarse_matrix(P, rng):
    N, nk = P["N"], P["nk"]
    fk, sfo, sf, fm, cof, pidx = P["face_k"], P["sub_face_off"], P["sub_faces"], P["f_minus"], P["face_cofs"], P["pidx"]
    sub_coff, cmap = [0], []
    for i in range(N):
        for t in range(sfo[i], sfo[i + 1]):
            f = sf[t]
            cmap.extend(range(cof[f], cof[f] + fk[f] + 1))
        sub_coff.append(len(cmap))
    cmap = np.array(cmap, dtype=np.int64)
    K = np.zeros((nk, nk))
    Ac = []
    dsc = rng.uniform(0.5, 2.0, N)
    for i in range(N):
        nci = sub_coff[i + 1] - sub_coff[i]
        G = rng.standard_normal((nci, nci))
        A = G @ G.T / max(nci, 1) + np.eye(nci)
        Ac.append(A)
        idx = cmap[sub_coff[i]:sub_coff[i + 1]]
        K[np.ix_(idx, idx)] += A
        if pidx[i] >= 0:
            for t in range(sfo[i], sfo[i + 1]):
                f = sf[t]
                so = 1.0 if fm[f] == i else -1.0
                K[pidx[i], cof[f]] += -dsc[i] * so
                K[cof[f], pidx[i]] += -dsc[i] * so
    sg = np.ones(nk)
    sg[pidx[pidx >= 0]] = -1.0
    return K, Ac, cmap, np.array(sub_coff), dsc, sg


def factor(P, Ac, cmap, sub_coff, dsc, sg):
    """Front assembly and partial signed factorization as k_front_factor does it."""
    nfr = P["nfr"]
    first, n, m, ch, b_off, bidx, ext = P["first"], P["n"], P["m"], P["ch"], P["b_off"], P["bidx"], P["ext"]
    sfo, sf, fm, cof, pidx = P["sub_face_off"], P["sub_faces"], P["f_minus"], P["face_cofs"], P["pidx"]
    F = np.full(P["F_off"][nfr], np.nan)
    FR = np.full(P["r_off"][nfr], np.nan)
    BC = np.full(P["r_off"][nfr], np.nan)
    for lv in range(P["H"]):
        for p in range(P["lvl_off"][lv], P["lvl_off"][lv + 1]):
            fst, nn, mm = first[p], n[p], m[p]
            f = nn + mm
            Bp = bidx[b_off[p]:b_off[p] + mm]
            assert (np.diff(Bp) > 0).all() and (mm == 0 or Bp[0] >= fst + nn)
            fo = P["F_off"][p]
            assert P["F_off"][p + 1] - fo == f * f
            F[fo:fo + f * f] = 0.0

            def pos(u):
                if u < fst + nn:
                    return u - fst
                k = np.searchsorted(Bp, u)
                return nn + k if (k < mm and Bp[k] == u) else -1

            for t in range(P["touch_off"][p], P["touch_off"][p + 1]):
                i = P["touch"][t]
                idx = cmap[sub_coff[i]:sub_coff[i + 1]]
                for a, u in enumerate(idx):
                    for bb, v in enumerate(idx):
                        if u < v or v < fst or v >= fst + nn:
                            continue
                        pu = pos(u)
                        assert pu >= 0
                        F[fo + pu + (v - fst) * f] += Ac[i][a, bb]
                if pidx[i] >= 0:
                    for t2 in range(sfo[i], sfo[i + 1]):
                        fc = sf[t2]
                        jf = cof[fc]
                        if jf < fst or jf >= fst + nn:
                            continue
                        pp = pos(pidx[i])
                        assert pp >= 0 and pidx[i] > jf
                        F[fo + pp + (jf - fst) * f] += -dsc[i] * (1.0 if fm[fc] == i else -1.0)
            for k in range(2):
                c = ch[2 * p + k]
                if c < 0:
                    continue
                nc, mc = n[c], m[c]
                fc = nc + mc
                uo = P["F_off"][c] + nc + nc * fc
                ex = ext[b_off[c]:b_off[c] + mc]
                assert (ex >= 0).all() and (ex < f).all() and (np.diff(ex) > 0).all()
                for k2 in range(mc):
                    for k1 in range(k2, mc):
                        F[fo + ex[k1] + ex[k2] * f] += F[uo + k1 + k2 * fc]
            Fm = F[fo:fo + f * f].reshape(f, f, order="F")
            L = np.tril(Fm).copy()
            s = sg[fst:fst + nn]
            for j in range(nn):
                dj = s[j] * L[j, j]
                assert dj > 0, "pivot sign disagrees with s"
                L[j, j] = np.sqrt(dj)
                L[j + 1:, j] /= L[j, j] * s[j]
                L[j + 1:, j + 1:] -= s[j] * np.outer(L[j + 1:, j], L[j + 1:, j])
            Fm[np.tri(f, dtype=bool)] = L[np.tri(f, dtype=bool)]
            Wp = np.linalg.inv(Fm[:nn, :nn] * np.tri(nn))
            Qp = Fm[nn:, :nn] @ Wp
            ro = P["r_off"][p]
            tri = nn * (nn + 1) // 2
            assert P["r_off"][p + 1] - ro == tri + mm * nn
            for r in range(nn):
                for c in range(r + 1):
                    FR[ro + r * (r + 1) // 2 + c] = Wp[r, c]
                    BC[ro + c * f - c * (c - 1) // 2 + (r - c)] = Wp[r, c]
            for k in range(mm):
                for c in range(nn):
                    FR[ro + tri + k * nn + c] = Qp[k, c]
                    BC[ro + c * f - c * (c - 1) // 2 + (nn - c) + k] = Qp[k, c]
    assert not np.isnan(FR).any() and not np.isnan(BC).any()
    return FR, BC


def check_tasks(P):
    """Task list: level ranges partition it, dependencies point backwards with exact targets."""
    nfr, H = P["nfr"], P["H"]
    T = P["task"].reshape(-1, 16)
    nt = len(T)
    fo, blo, bhi = P["ftask_off"], P["btask_lo"], P["btask_hi"]
    assert fo[0] == 0 and fo[H] == blo[H - 1] and bhi[0] == nt
    for h in range(H - 1):
        assert bhi[h + 1] == blo[h]
    kind = T[:, 11]
    assert (kind[:fo[H]] == 0).all() and (kind[fo[H]:] == 1).all()
    # tasks per counter, and the last task index of each counter
    count = np.zeros(2 * nfr, int)
    last = np.full(2 * nfr, -1)
    for i, d in enumerate(T):
        c = d[0] + (nfr if d[11] else 0)
        count[c] += 1
        last[c] = i
    for i, d in enumerate(T):
        for dep, target in ((d[12], d[13]), (d[14], d[15])):
            if dep < 0:
                continue
            assert target == count[dep] and last[dep] < i, "dependency not strictly earlier"
        p = d[0]
        if d[11] == 0:
            kids = {c for c in P["ch"][2 * p:2 * p + 2] if c >= 0}
            assert {x for x in (d[12], d[14]) if x >= 0} == kids
        else:
            parent = [q for q in range(nfr) if p in P["ch"][2 * q:2 * q + 2]]
            want = nfr + parent[0] if parent else p
            assert d[12] == want and d[14] == -1


def launch_order(P, lvl):
    """(descriptor, subtree) in the order of the launches: with bottom
    subtrees (levels 0..sub_lv), each subtree's forward phases, then the
    forward levels above, the backward levels above, each subtree's backward
    phases; subtree -1 marks a level-launch task.  The subtree copies must be
    exactly the level tasks of levels <= sub_lv, phase k of a subtree holding
    level k forward and level sub_lv - k backward."""
    T = P["task"].reshape(-1, 16)
    sl = P["sub_lv"]
    if sl < 0:
        assert P["nsubt"] == 0 and len(P["stask"]) == 0
        return [(d, -1) for d in T]
    assert sl < P["top"]
    ns, npk = P["nsubt"], sl + 2
    ST, sph = P["stask"].reshape(-1, 16), P["sph"]
    assert len(sph) == 2 * ns * npk
    fwd, bwd = [], []
    for t in range(ns):
        for k in range(sl + 1):
            for i in range(sph[t * npk + k], sph[t * npk + k + 1]):
                assert ST[i][11] == 0 and lvl[ST[i][0]] == k
                fwd.append((ST[i], t))
            for i in range(sph[(ns + t) * npk + k], sph[(ns + t) * npk + k + 1]):
                assert ST[i][11] == 1 and lvl[ST[i][0]] == sl - k
                bwd.append((ST[i], t))
    low = [d for d in T if lvl[d[0]] <= sl]
    key = lambda d: tuple(int(v) for v in d[:12])
    assert sorted(map(key, low)) == sorted(map(key, [d for d, _ in fwd + bwd]))
    above_f = [(d, -1) for d in T if d[11] == 0 and lvl[d[0]] > sl]
    above_b = [(d, -1) for d in T if d[11] == 1 and lvl[d[0]] > sl]
    return fwd + above_f + above_b + bwd


def sweep(P, FR, BC, sg, b, K=None):
    """The sweep tasks serialised in launch order (what the level-by-level
    and subtree kernels compute).  With a dense top block (P["top"] < H)
    the tasks of the top levels are replaced by the gather of t_t and a dense
    solve with the Schur complement of K on the top dofs.  A subtree task may
    only push into (forward) or scatter into (backward) fronts of its own
    subtree, or, forward from the subtree's root, into a front above the
    subtree levels: subtrees of one launch never share data."""
    nfr, nk, H = P["nfr"], P["nk"], P["H"]
    top = P["top"]
    nv = P["v_off"][nfr]
    S = [np.zeros(nv), np.zeros(nv)]
    written = np.zeros((2, nv), bool)
    z = np.full(nk, np.nan)
    x = np.full(nk, np.nan)
    XB = np.full(max(1, P["b_off"][nfr]), np.nan)
    T = P["task"].reshape(-1, 16)
    lvl = np.empty(nfr, int)
    for h in range(H):
        lvl[P["lvl_off"][h]:P["lvl_off"][h + 1]] = h
    done_f, done_b = set(), set()
    topped = False

    def top_solve():
        d0 = P["lvl_dof"][top]
        nt = nk - d0
        assert P["nt"] == nt and len(P["tg_off"]) == nt + 1
        tg = P["tg"]
        v0 = P["v_off"][P["lvl_off"][top]]
        # every position of the top fronts' vectors feeds exactly one top dof
        assert np.array_equal(np.sort(tg), np.arange(v0, P["v_off"][nfr]))
        tt = np.array([b[d0 + j] + sum(S[0][q] + S[1][q] for q in tg[P["tg_off"][j]:P["tg_off"][j + 1]])
                       for j in range(nt)])
        bot = np.arange(d0)
        St = K[d0:, d0:] - K[d0:, :d0] @ np.linalg.solve(K[:d0, :d0], K[:d0, d0:]) if d0 else K.copy()
        xt = np.linalg.solve(St, tt)
        for jj in range(nt):
            dd = d0 + jj
            x[dd] = xt[jj]
            done_b.add(dd)
            for k in range(P["xsc_off"][dd], P["xsc_off"][dd + 1]):
                XB[P["xsc"][k]] = xt[jj]
        del bot

    sub_of = {}
    for d, t in launch_order(P, lvl):
        if t >= 0:
            sub_of.setdefault(int(d[0]), t)
            assert sub_of[int(d[0])] == t, "front in two subtrees"
    for d, tsub in launch_order(P, lvl):
        p, j, g, n, m, fst, vo, bo, rlo, rhi, slot, kind = (int(v) for v in d[:12])
        if tsub >= 0 and kind == 0:
            par = [q for q in range(nfr) if p in P["ch"][2 * q:2 * q + 2]]
            if par and lvl[par[0]] <= P["sub_lv"]:
                assert sub_of[par[0]] == tsub, "push into another subtree"
        if tsub >= 0 and kind == 1:
            for k in range(P["xsc_off"][fst + j], P["xsc_off"][min(fst + j + 256 // g, fst + n)]):
                owner = int(np.searchsorted(P["b_off"], P["xsc"][k], side="right")) - 1
                assert sub_of.get(owner) == tsub, "scatter into another subtree"
        if lvl[p] >= top:
            if kind == 1 and not topped:
                top_solve()
                topped = True
            continue
        if kind == 1 and not topped and top < H:
            top_solve()
            topped = True
        ro = (rhi & 0xffffffff) << 32 | (rlo & 0xffffffff)
        assert (n, m, fst, vo, bo, ro) == (P["n"][p], P["m"][p], P["first"][p], P["v_off"][p], P["b_off"][p],
                                           P["r_off"][p])
        assert g in (1, 4, 16, 64)
        if kind == 0:
            assert slot == P["cslot"][p]
            t = b[fst:fst + n] + S[0][vo:vo + n] + S[1][vo:vo + n]
            assert not np.isnan(t).any()
            for r in range(j, min(j + 256 // g, n + m)):
                assert (p, r) not in done_f
                done_f.add((p, r))
                if r < n:
                    o = ro + r * (r + 1) // 2
                    z[fst + r] = FR[o:o + r + 1] @ t[:r + 1]
                else:
                    o = ro + n * (n + 1) // 2 + (r - n) * n
                    dst = P["wdst"][bo + r - n]
                    assert not written[slot, dst]
                    written[slot, dst] = True
                    S[slot][dst] = S[0][vo + r] + S[1][vo + r] - FR[o:o + n] @ t
        else:
            f = n + m
            xb = XB[bo:bo + m].copy()
            assert not np.isnan(xb).any(), "B vector read before it was filled"
            for c in range(j, min(j + 256 // g, n)):
                dd = fst + c
                assert dd not in done_b
                done_b.add(dd)
                o = ro + c * f - c * (c - 1) // 2
                nl = n - c
                val = BC[o:o + nl] @ (sg[dd:dd + nl] * z[dd:dd + nl]) - BC[o + nl:o + nl + m] @ xb
                x[dd] = val
                for k in range(P["xsc_off"][dd], P["xsc_off"][dd + 1]):
                    q = P["xsc"][k]
                    assert P["bidx"][q] == dd
                    owner = int(np.searchsorted(P["b_off"], q, side="right")) - 1
                    assert lvl[owner] < lvl[p], "scatter into a front of the same or a higher level"
                    XB[q] = val
    if top < H and not topped:
        top_solve()
    swept = slice(0, P["lvl_off"][top])
    assert len(done_f) == int(sum(P["n"][swept]) + sum(P["m"][swept])) and len(done_b) == nk
    return x


CASES = [
    (3, 12, 16, 9, 3, 4, 3, 1, 0),     # 3D, single-subdomain leaves
    (3, 12, 16, 9, 3, 4, 3, 4, 1),     # leaf boxes of up to 4 subdomains
    (3, 12, 16, 9, 3, 4, 3, 100, 2),   # one dense front
    (2, 20, 30, 1, 4, 5, 1, 1, 3),     # 2D
    (2, 20, 30, 1, 4, 5, 1, 3, 4),
    (3, 20, 10, 5, 5, 2, 1, 2, 8),     # flat 3D grid
    (3, 6, 6, 6, 1, 1, 2, 1, 6),       # two subdomains
]


@pytest.mark.parametrize("top", [None, 40, 150, 100000], ids=["sweeps", "top40", "top150", "alldense"])
@pytest.mark.parametrize("args", CASES, ids=lambda a: "x".join(map(str, a[4:7])) + f"_leaf{a[7]}")
def test_plan_factor_and_sweeps_match_dense_solve(dumper, args, top):
    check_plan(dumper, args, top, None)


@pytest.mark.parametrize("sub", [0, 2, 99], ids=["sub1", "sub3", "suball"])
@pytest.mark.parametrize("top", [None, 150], ids=["sweeps", "top150"])
@pytest.mark.parametrize("args", CASES, ids=lambda a: "x".join(map(str, a[4:7])) + f"_leaf{a[7]}")
def test_subtree_sweeps_match_dense_solve(dumper, args, top, sub):
    """Bottom levels 0..sub swept by subtrees (one workgroup each), the rest by level launches."""
    P = check_plan(dumper, args, top, sub)
    want = min(sub, P["top"] - 1)
    assert P["sub_lv"] == (want if want >= 0 and P["nfr"] > 0 else -1)


@pytest.mark.parametrize("w1", [6, 1000], ids=["short1", "all1"])
@pytest.mark.parametrize("args", CASES, ids=lambda a: "x".join(map(str, a[4:7])) + f"_leaf{a[7]}")
def test_single_lane_rows_match_dense_solve(dumper, args, w1):
    """Rows / columns up to w1 entries as tasks of 256 single-lane rows, with bottom subtrees and a top block."""
    P = check_plan(dumper, args, 150, 2, w1)
    for g, ln in zip(P["gf"], P["n"]):
        assert (g == 1) == (ln <= w1)


def check_plan(dumper, args, top, sub, w1=None):
    P = load(dumper, args, top, sub, w1)
    if top is None:
        assert P["top"] == P["H"] and P["nt"] == 0
    else:
        # the top block: the lowest level whose dofs and all above fit the cap
        d0 = P["lvl_dof"][P["top"]]
        assert P["nk"] - d0 <= top
        assert P["top"] == 0 or P["nk"] - P["lvl_dof"][P["top"] - 1] > top
    rng = np.random.default_rng(args[-1])
    # numbering covers every coarse dof once, pinned pressure excluded
    fk, cof, pidx = P["face_k"], P["face_cofs"], P["pidx"]
    dofs = np.concatenate([np.arange(cof[f], cof[f] + fk[f] + 1) for f in range(P["nF"])] + [pidx[pidx >= 0]])
    assert np.array_equal(np.sort(dofs), np.arange(P["nk"]))
    assert pidx[-1] == -1 and (pidx[:-1] >= 0).all()
    # levels: children strictly below their parent
    lvl = np.empty(P["nfr"], int)
    for h in range(P["H"]):
        lvl[P["lvl_off"][h]:P["lvl_off"][h + 1]] = h
    for p in range(P["nfr"]):
        for c in P["ch"][2 * p:2 * p + 2]:
            if c >= 0:
                assert lvl[c] < lvl[p]
    check_tasks(P)
    K, Ac, cmap, sub_coff, dsc, sg = coarse_matrix(P, rng)
    FR, BC = factor(P, Ac, cmap, sub_coff, dsc, sg)
    b = rng.standard_normal(P["nk"])
    x = sweep(P, FR, BC, sg, b, K)
    ref = np.linalg.solve(K, b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10
    return P


def test_single_subdomain_has_no_coarse_dofs(dumper):
    P = load(dumper, (3, 6, 6, 6, 1, 1, 1, 1, 0))
    assert P["nk"] == 0 and P["nfr"] == 0 and P["H"] == 0


def test_weighted_cut_avoids_heavy_plane(dumper):
    """The root separator is a light plane, the heavy plane's faces go to small fronts.

    4 x 4 x 4 subdomains; the z-plane between subdomain layers 1 and 2 (the
    geometric middle) carries 20 adaptive rows per face, every other face none.
    """
    P = load(dumper, (3, 16, 16, 16, 4, 4, 4, 1, 0, 2, 1))
    fk, cof = P["face_k"], P["face_cofs"]
    root = P["nfr"] - 1
    assert P["lvl_off"][P["H"] - 1] == root
    own = set(range(P["first"][root], P["first"][root] + P["n"][root]))
    heavy = [f for f in range(P["nF"]) if fk[f] == 20]
    assert len(heavy) == 16
    assert not any(cof[f] in own for f in heavy)
    # root: a light 4 x 4 plane (16 face dofs) and the pressures placed on it
    assert P["n"][root] <= 16 + 32
    assert max(P["n"]) < 16 * 21
