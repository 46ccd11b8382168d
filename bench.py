#!/usr/bin/env python3
"""Benchmark of the BDDC-PCG solve on one MI355X.

A step is one complete ``bddc_solve`` (Algorithm "BDDC method": coarse step,
subdomain step, preconditioned CG on the interface correction to rtol 1e-8,
post-correction of interiors) of a resident problem whose source already sits
in device memory.  The setup (factorizations, face eigenproblems, coarse
problem) runs once before the timed region and is reported separately.

Prints one JSON line.  ``value`` is solves per second of the mixed form (FP32
local operators inside the FP64 CG); the FP64 form is reported beside it.
"""
import argparse
import faulthandler
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BDDC-PCG solve time & served solves/s (p50/p99), mixed vs FP64, rtol 1e-8"
HBM_PEAK_GBS = 8000.0


def make_workload(name):
    import workloads as W
    if name == "reservoir":
        pr = W.reservoir_3d(nz=85, seed=0, tau=10.0)
        desc = {"workload": "SPE10-shaped reservoir 60x220x85 (20x10x2 ft cells; smooth top 35 layers, channelised "
                            "bottom 50, kz=0.1kx), 10x10x5-cell boxes (N=2244), five-spot well columns, adaptive "
                            "tau=10, rtol 1e-8",
                "n": list(pr.n), "subdomains": 2244, "tau": 10.0, "rtol": 1e-8}
    elif name == "layer":
        pr = W.layer_60x220(0, tau=10.0)
        desc = {"workload": "SPE10-shaped channelised layer 60x220 (20x10 ft cells), 10x10-cell boxes (N=132), "
                            "five-spot wells, adaptive tau=10, rtol 1e-8",
                "n": list(pr.n), "subdomains": 132, "tau": 10.0, "rtol": 1e-8}
    elif name == "square":
        pr = W.unit_square_16(0)
        pr.rtol = 1e-10
        desc = {"workload": "unit square 16x16, GRF permeability, 4x4 boxes, no adaptivity, rtol 1e-10",
                "n": list(pr.n), "subdomains": 16, "tau": None, "rtol": 1e-10}
    else:
        raise SystemExit(f"unknown workload {name}")
    return pr, desc


def time_gpu(pr, precision, steps, warmup, kernel_reps=0):
    """Set up one solver, time `steps` solves of the resident problem, close it.

    One solver is alive at a time: each holds two streams (main and coarse
    side stream), and two of them plus torch's stream would exceed the four
    hardware queues a process gets, making streams share a queue.
    """
    import torch
    from paper_1901_02090_amd import Solver
    from paper_1901_02090_amd.bddc import K_SCHUR_APPLY, K_PRECOND_APPLY, K_PRECOND_FULL
    t0 = time.perf_counter()
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=pr.tau, precision=precision, max_it=5000, autotune=True)
    setup_s = time.perf_counter() - t0
    try:
        stream = torch.cuda.current_stream()
        s.set_stream(stream.cuda_stream)
        src = torch.tensor(pr.source, dtype=torch.float64, device="cuda")
        flux = torch.empty(s.n_faces_all, dtype=torch.float64, device="cuda")
        pres = torch.empty(s.n_cells, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for _ in range(warmup):
            s.solve_device(src.data_ptr(), pr.rtol, flux.data_ptr(), pres.data_ptr())
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            s.solve_device(src.data_ptr(), pr.rtol, flux.data_ptr(), pres.data_ptr())
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        st = s.stats()
        # host-buffer solves: source copied in, flux and pressure copied out over PCIe
        host_ms = None
        if kernel_reps > 0:
            s.solve(pr.source, rtol=pr.rtol)
            t_h = time.perf_counter()
            for _ in range(3):
                s.solve(pr.source, rtol=pr.rtol)
            host_ms = (time.perf_counter() - t_h) / 3 * 1e3
        # approximation quality of steps 1-2 (eq. epsilon): u_0 and u^* against the converged flux
        eps = None
        if kernel_reps > 0:
            fu = flux.cpu().numpy()
            ref = np.linalg.norm(fu)
            eps = {}
            for name, steps_flag in (("eps0", 1), ("eps_star", 12)):
                f2 = torch.empty_like(flux)
                p2 = torch.empty_like(pres)
                s.solve_device(src.data_ptr(), pr.rtol, f2.data_ptr(), p2.data_ptr(), steps=steps_flag)
                torch.cuda.synchronize()
                eps[name] = float(np.linalg.norm(f2.cpu().numpy() - fu) / ref)
        kern = {}
        if kernel_reps > 0:
            kern["schur"] = s.time_kernel(K_SCHUR_APPLY, kernel_reps)
            kern["precond"] = s.time_kernel(K_PRECOND_APPLY, kernel_reps)
            kern["precond_full"] = s.time_kernel(K_PRECOND_FULL, kernel_reps)
        return dict(setup_s=setup_s, total_s=total, lat=np.array(lat), stats=st, kernels=kern, host_ms=host_ms,
                    flux=flux.cpu().numpy(), pres=pres.cpu().numpy(), eps=eps)
    finally:
        s.close()


def multiscale_compare(pr, ref_flux):
    """Section 6's comparison: the multiscale rows (one per face) in place of the
    adaptive ones, mixed form, same source; one setup and one timed solve."""
    import torch
    from paper_1901_02090_amd import Solver
    t0 = time.perf_counter()
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, precision="mixed", max_it=5000, multiscale=True, ms_source=pr.source)
    setup_ms = (time.perf_counter() - t0) * 1e3
    try:
        stream = torch.cuda.current_stream()
        s.set_stream(stream.cuda_stream)
        src = torch.tensor(pr.source, dtype=torch.float64, device="cuda")
        flux = torch.empty(s.n_faces_all, dtype=torch.float64, device="cuda")
        pres = torch.empty(s.n_cells, dtype=torch.float64, device="cuda")
        out = {}
        for name, steps_flag in (("eps0", 1), ("eps_star", 12)):
            s.solve_device(src.data_ptr(), pr.rtol, flux.data_ptr(), pres.data_ptr(), steps=steps_flag)
            torch.cuda.synchronize()
            out[name] = float(np.linalg.norm(flux.cpu().numpy() - ref_flux) / np.linalg.norm(ref_flux))
        s.solve_device(src.data_ptr(), pr.rtol, flux.data_ptr(), pres.data_ptr())   # warm-up (graph capture)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.solve_device(src.data_ptr(), pr.rtol, flux.data_ptr(), pres.data_ptr())
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t1) * 1e3
        st = s.stats()
        out.update(iterations=st["it"], converged=bool(st["converged"]), n_rows=st["n_adaptive"],
                   n_coarse=st["n_coarse"], kappa=st["kappa"], setup_ms=setup_ms, ms_per_solve=solve_ms,
                   flux_relerr_vs_adaptive=float(np.linalg.norm(flux.cpu().numpy() - ref_flux) /
                                                 np.linalg.norm(ref_flux)))
        return out
    finally:
        s.close()


def _cutout(pr, lo, ext):
    """Sub-block of a 3D problem (same field), with the cut sources made compatible."""
    import workloads as W
    n = pr.n
    idx = np.arange(np.prod(n)).reshape(n, order="F")[lo[0]:lo[0] + ext[0], lo[1]:lo[1] + ext[1],
                                                       lo[2]:lo[2] + ext[2]].reshape(-1, order="F")
    src = pr.source[idx].copy()
    src -= src.mean()
    cuts = W.regular_cuts(tuple(ext), (10, 10, 5))
    return W.Problem("cutout", tuple(ext), pr.h, pr.perm[idx], src, cuts, tau=pr.tau, rtol=pr.rtol)


def host_info():
    """CPU model, logical CPUs this process may use, and RAM of the host."""
    model, ram = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 1024 ** 2, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "ram_gib": ram}


def _oracle_rate(sample, seconds, threads):
    """Complete oracle solves of `sample` (setup excluded) for about `seconds` with
    `threads` BLAS threads: (seconds per solve, solves, elapsed, last result)."""
    from threadpoolctl import threadpool_limits
    from oracle import bddc as ob, rt0
    with threadpool_limits(threads):
        g = rt0.Grid(sample.n, sample.h)
        o = ob.BDDC(g, sample.perm, sample.cuts, tau=sample.tau)
        n = 0
        t0 = time.perf_counter()
        while True:
            out = o.solve(sample.source, rtol=sample.rtol, maxit=5000)
            n += 1
            el = time.perf_counter() - t0
            if el >= seconds or n >= 1000:
                break
    return el / n, n, el, out, o


def cpu_baseline(pr, seconds, gpu_iters):
    """The oracle (plain CPU FP64 BDDC) timed on the host, setup excluded, with
    all the host's threads and with one.

    For the 2D layer the sample is the workload itself.  The reservoir's oracle
    setup (2,244 local saddle-point factorizations, 6,124 dense pair
    eigenproblems) does not fit a bench run, so the sample is a 20x20x10 cutout
    of the same field around the injector column (8 subdomains of the same
    10x10x5 shape), scaled by the subdomain count and the iteration ratio (the
    oracle's solve cost is linear in both).
    """
    host = host_info()
    # the threads this process may use (the machine's CPU share sets OMP_NUM_THREADS)
    nthr = int(os.environ.get("OMP_NUM_THREADS") or 0) or host["nproc"]
    sample = pr if len(pr.n) != 3 else _cutout(pr, (20, 100, 30), (20, 20, 10))
    runs = {}
    for thr in (nthr, 1):
        t_solve, n, el, out, o = _oracle_rate(sample, seconds / 2, thr)
        scale, what = 1.0, "the same workload"
        if sample is not pr:
            N_full = int(np.prod([len(c) - 1 for c in pr.cuts]))
            scale = (N_full / o.subs.N) * (gpu_iters / max(out["it"], 1))
            what = (f"a 20x20x10 cutout of the same field (x 20-40, y 100-120, z 30-40; {o.subs.N} subdomains, "
                    f"{out['it']} iterations), scaled x{scale:.1f} to {N_full} subdomains and {gpu_iters} iterations")
        runs[thr] = (1.0 / (t_solve * scale), n, el, what)
    v, n, el, what = runs[nthr]
    v1, n1, el1, _ = runs[1]
    return {"value": v, "unit": "solves/s", "cores": nthr, "kind": "oracle",
            "sample": f"{n} complete oracle solves (setup excluded, {el:.1f} s, {nthr} BLAS threads) of {what}",
            "one_thread": {"value": v1, "unit": "solves/s", "cores": 1,
                           "sample": f"{n1} solves in {el1:.1f} s with one BLAS thread"},
            "host": host}


COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "symv_reservoir_60x220x85_hbm_traffic.md")
KERNEL_SOURCES = ("paper_1901_02090_amd/csrc/solve.hip", "paper_1901_02090_amd/csrc/common.hpp")
PREC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "precond_apply_reservoir_60x220x85_hbm_traffic.md")
PREC_SOURCES = ("paper_1901_02090_amd/csrc/solve.hip", "paper_1901_02090_amd/csrc/coarse.hip",
                "paper_1901_02090_amd/csrc/common.hpp", "paper_1901_02090_amd/csrc/nd.hpp")


def measured_traffic(kernel, path=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch of `kernel` from a committed counter summary.

    Returns None when there is no entry or when the kernel sources changed
    since the counters were taken (their sha256 is stored beside the figure).
    """
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    for line in text.splitlines():
        t = line.split()
        if len(t) == 5 and t[0] == "traffic" and t[1] == kernel and t[3] == "sha256":
            return float(t[2]) if t[4] == h.hexdigest() else None
    return None


SERVE_DESC = ("Poisson stream (mean 50 requests/s, seeded) of independent solves: each request its own "
              "2D grid (32..60 x 32..220 cells) or 3D 60x220x{5,17,34} slab, own channelised field and seeded "
              "wells, tau off or 10, rtol 1e-8; setup and solve per request")


def serve_stream(precision, requests, arrivals, max_active=4, setup_workers=2, sources=None, keys=None):
    """Submit `requests` at their arrival times (s from start) and wait for all
    (sources / keys: per request, in place of the request's own source / 0)."""
    from paper_1901_02090_amd import Server
    srv = Server(precision=precision, max_active=max_active, setup_workers=setup_workers)
    try:
        tickets = []
        t0 = time.perf_counter()
        for k, (pr, ta) in enumerate(zip(requests, arrivals)):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            src = pr.source if sources is None else sources[k]
            key = 0 if keys is None else keys[k]
            tickets.append(srv.submit(pr.n, pr.h, pr.perm, pr.cuts, src, tau=pr.tau, rtol=pr.rtol, key=key))
        its, conv, batch, reused = [], 0, [], 0
        for t in tickets:
            _, _, st = srv.result(t)
            its.append(st["it"])
            conv += st["converged"]
            batch.append(st["batch"])
            reused += st["reused"]
        wall = time.perf_counter() - t0
        ss = srv.stats()
    finally:
        srv.close()
    return {"solves_per_s": ss["solves_per_s"], "p50_ms": ss["p50_ms"], "p99_ms": ss["p99_ms"],
            "completed": ss["completed"], "converged": conv, "wall_s": wall, "peak_active": ss["peak_active"],
            "peak_bytes": ss["peak_bytes"], "mean_iterations": float(np.mean(its)),
            "mean_batch": float(np.mean(batch)), "max_batch": int(max(batch)), "reused": int(reused)}


def serving(n_req, rate=50.0, seed=0):
    import workloads as W
    reqs = [W.serving_request(seed * 100000 + k) for k in range(n_req)]
    arr = W.poisson_arrivals(rate, n_req, seed)
    out = {"workload": SERVE_DESC, "requests": n_req, "arrival_rate_per_s": rate, "max_active": 4,
           "setup_workers": 2, "dims": {"2d": sum(r.dim == 2 for r in reqs), "3d": sum(r.dim == 3 for r in reqs)}}
    for prec in ("fp64", "mixed"):
        out[prec] = serve_stream(prec, reqs, arr)
    return out


SERVE_KEYED_DESC = ("Poisson stream (mean {rate:g} requests/s, seeded) over {np} resident problems (2D 32x125, 45x127, "
                    "55x80 and a 60x220x17 slab, channelised fields, tau 10, rtol 1e-8), each request its own seeded "
                    "wells, under problem keys: each problem is set up once and the waiting requests of a key are "
                    "solved together (bddc_solve_block)")


def serving_keyed(n_req, rate=200.0, seed=1):
    """The same problems requested again and again: keyed (resident, batched) against unkeyed."""
    import workloads as W
    base = [W.serving_request(sd) for sd in (6, 11, 12, 7)]
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(base), n_req)
    reqs = [base[p] for p in pick]
    srcs = [W.seeded_wells(base[p].n, rng) for p in pick]
    arr = W.poisson_arrivals(rate, n_req, seed)
    out = {"workload": SERVE_KEYED_DESC.format(rate=rate, np=len(base)), "requests": n_req,
           "arrival_rate_per_s": rate, "max_active": 4, "setup_workers": 2}
    for prec in ("fp64", "mixed"):
        out[prec] = serve_stream(prec, reqs, arr, sources=srcs, keys=[int(p) + 1 for p in pick])
    return out


def serving_child(n_req, timeout_s=600):
    """Both serving streams in a child process, started before this process
    touches the GPU (and done before it does), so that a failure there leaves
    the rest of the bench line intact; returns (serving, serving_resident) or
    error records."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serving-only", str(n_req)]
    try:
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired:
        err = {"error": f"serving child exceeded {timeout_s} s"}
        return err, err
    lines = [ln for ln in res.stdout.splitlines() if ln.startswith("{")]
    if res.returncode != 0 or not lines:
        err = {"error": f"serving child exited with status {res.returncode}", "stderr_tail": res.stderr[-600:]}
        return err, err
    d = json.loads(lines[-1])
    return d["serving"], d["serving_resident"]


def copy_rate(reps=20):
    """Device-to-device copy of COPY_BYTES, timed with events: GB/s moved (read + write)."""
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, c
    return 2.0 * COPY_BYTES / (ms * 1e-3) / 1e9


def kernels_only(pr, reps):
    """Launch the local apply kernels and a 1 GiB device-to-device copy alone.

    Under a hardware-counter profiler the copy gives the factor between the
    counters' byte figures and true bytes (it reads and writes exactly
    COPY_BYTES each).
    """
    import torch
    from paper_1901_02090_amd import Solver
    from paper_1901_02090_amd.bddc import K_SCHUR_APPLY, K_PRECOND_APPLY, K_PRECOND_FULL
    s = Solver(pr.n, pr.h, pr.perm, pr.cuts, tau=pr.tau, precision="mixed", max_it=5000)
    s.solve(pr.source, rtol=pr.rtol)
    ms_s, by_s = s.time_kernel(K_SCHUR_APPLY, reps)
    ms_t, by_t = s.time_kernel(K_PRECOND_APPLY, reps)
    ms_p, by_p = s.time_kernel(K_PRECOND_FULL, reps)
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        c.copy_(a)
    torch.cuda.synchronize()
    s.close()
    print(json.dumps({"schur_apply": {"avg_ms": ms_s, "bytes": by_s},
                      "precond_apply": {"avg_ms": ms_t, "bytes": by_t},
                      "precond_full": {"avg_ms": ms_p, "bytes": by_p},
                      "copy_bytes": COPY_BYTES, "reps": reps}), flush=True)


BLOCK_DESC = ("the same 60x220x85 field cut into uneven boxes (seeded cut planes, widths 4..16 cells; 1,260 "
              "subdomains, interfaces up to 1,224 dofs), tau=5, {k} seeded well placements solved together "
              "(bddc_solve_block: blocks of 16 sources per CG iteration), rtol 1e-8")
FP64_MFMA_PEAK_TFS = 78.6


def block_batch(nsrc):
    """Several sources on one resident problem: the block CG against one solve
    after the other (both device pointers), with the block kernels' rooflines."""
    import torch
    import workloads as W
    from paper_1901_02090_amd import Solver
    from paper_1901_02090_amd.bddc import K_BLOCK_SCHUR, K_BLOCK_PRECOND_FULL
    full = W.reservoir_3d(nz=85, seed=0, tau=5.0)
    cuts = W.seeded_cuts(full.n, 4, 16, 0)
    srcs = np.stack([W.seeded_wells(full.n, np.random.default_rng(100 + k)) for k in range(nsrc)])
    t0 = time.perf_counter()
    s = Solver(full.n, full.h, full.perm, cuts, tau=5.0, precision="mixed", max_it=3000)
    setup_s = time.perf_counter() - t0
    try:
        d_src = torch.tensor(srcs, dtype=torch.float64, device="cuda")
        d_f = torch.empty((nsrc, s.n_faces_all), dtype=torch.float64, device="cuda")
        d_p = torch.empty((nsrc, s.n_cells), dtype=torch.float64, device="cuda")
        s.solve_block_device(nsrc, d_src.data_ptr(), 1e-8, d_f.data_ptr(), d_p.data_ptr())   # first call allocates
        torch.cuda.synchronize()
        t = time.perf_counter()
        its_b = s.solve_block_device(nsrc, d_src.data_ptr(), 1e-8, d_f.data_ptr(), d_p.data_ptr())
        torch.cuda.synchronize()
        tb = time.perf_counter() - t
        st = s.stats()
        fb = d_f.cpu().numpy()
        t = time.perf_counter()
        its_1 = []
        for k in range(nsrc):
            s.solve_device(d_src[k].data_ptr(), 1e-8, d_f[k].data_ptr(), d_p[k].data_ptr())
            its_1.append(s.stats()["it"])
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t
        f1 = d_f.cpu().numpy()
        err = max(float(np.linalg.norm(fb[k] - f1[k]) / np.linalg.norm(f1[k])) for k in range(nsrc))
        ms_s, by_s = s.time_kernel(K_BLOCK_SCHUR, 20)
        ms_p, by_p = s.time_kernel(K_BLOCK_PRECOND_FULL, 16)
        fl = st["flops_block_local"]
    finally:
        s.close()
    ach = by_s / (ms_s * 1e-3) / 1e9
    tfs = fl / (ms_s * 1e-3) / 1e12
    return {"workload": BLOCK_DESC.format(k=nsrc), "n_sub": int(st["n_sub"]), "setup_ms": setup_s * 1e3,
            "solves_per_s": nsrc / tb, "ms": tb * 1e3,
            "one_by_one": {"solves_per_s": nsrc / t1, "ms": t1 * 1e3, "precision": "mixed"},
            "speedup": t1 / tb, "iterations": [int(its_b.min()), int(its_b.max())],
            "iterations_equal_one_by_one": bool((np.array(its_1) == its_b).all()),
            "max_flux_relerr_vs_one_by_one": err,
            "dtype": "f64",
            "roofline_block_schur": {
                "kernel": "k_blk_symv<double> (S^i against 16 columns, 64 x 16 tiles on v_mfma_f64_16x16x4f64)",
                "avg_launch_us": ms_s * 1e3, "bytes_per_launch": by_s, "flops_per_launch": fl,
                "hbm": {"achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS},
                "mfma": {"achieved": tfs, "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                         "frac": tfs / FP64_MFMA_PEAK_TFS},
                "note": "bytes count each packed entry once; the kernel reads the mirror half a second time"},
            "block_precond_apply": {"avg_us": ms_p * 1e3, "bytes": by_p,
                                    "achieved_gbs": by_p / (ms_p * 1e-3) / 1e9}}


def main():
    faulthandler.enable()
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="reservoir", choices=["reservoir", "layer", "square"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of a served Poisson stream (mean 50/s) through bddc_server_* in both forms "
                         "(0: not run)")
    ap.add_argument("--serving-only", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--block-sources", type=int, default=32,
                    help="sources of the block-solve workload (uneven boxes, tau 5), solved together and one by "
                         "one (0: not run)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set up the mixed form, solve once, launch the S^i and T^i apply kernels alone, the "
                         "whole preconditioner, and a plain device copy of known size (for scaling hardware "
                         "byte counters), then exit")
    ap.add_argument("--alloc", default="torch", choices=["torch", "hip"],
                    help="device memory of the solver handles: torch's caching allocator through "
                         "bddc_set_allocator (default), or the library's own hipMalloc / hipFree.  With hipFree "
                         "the tens of GB of setup workspace released at the end of a setup slow the solves of "
                         "the following half second or so by about 2%%")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on exactly one GPU: the solver is a single-GPU build "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    if args.serving_only > 0:
        # child of serving_child: the library's own hipMalloc, both streams
        print(json.dumps({"serving": dict(serving(args.serving_only), allocator="hipMalloc"),
                          "serving_resident": dict(serving_keyed(64), allocator="hipMalloc")}), flush=True)
        return
    srv_out = None
    if args.serve_requests > 0 and not args.kernels_only:
        # The serving streams run first, in a child process with the library's
        # own hipMalloc: two runs of independent-problem streams (one with
        # torch's allocator, one at 200 requests/s over repeated problems with
        # hipMalloc) ended in a host segmentation fault whose cause is not
        # known; a failure there must not take the rest of this line with it.
        srv_out = serving_child(args.serve_requests)
    if args.alloc == "torch":
        import torch
        from paper_1901_02090_amd import set_allocator
        set_allocator(torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete)
    pr, desc = make_workload(args.workload)
    desc = dict(desc, allocator="torch caching allocator" if args.alloc == "torch" else "hipMalloc")
    if args.kernels_only:
        kernels_only(pr, args.steps)
        return

    r64 = time_gpu(pr, "fp64", args.steps, args.warmup)
    rmx = time_gpu(pr, "mixed", args.steps, args.warmup, kernel_reps=200)
    msc = multiscale_compare(pr, rmx["flux"]) if args.workload == "reservoir" else None

    # dominant kernel of an iteration: the local S^i products (FP64 in both forms)
    ms_s, by_s = rmx["kernels"]["schur"]
    ms_t, by_t = rmx["kernels"]["precond"]
    kern = ("k_symv<double>", "local Schur products S^i of the CG operator", ms_s, by_s)
    if by_t / ms_t > by_s / ms_s and ms_t > ms_s:
        kern = ("k_symv<float>", "local substructure corrections T^i of the preconditioner", ms_t, by_t)
    achieved = kern[3] / (kern[2] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kern[0]),
            "kernel": f"{kern[0]} ({kern[1]})", "bytes_per_launch": kern[3], "avg_launch_us": kern[2] * 1e3}

    st = rmx["stats"]
    # the whole preconditioner of one CG iteration (Psi^T r, T^i beside the
    # coarse solve, Psi alpha, averaging), against the vendor HBM peak and the
    # copy rate measured here
    ms_p, by_p = rmx["kernels"]["precond_full"]
    cp = copy_rate()
    ach_p = by_p / (ms_p * 1e-3) / 1e9
    prec = {"avg_us": ms_p * 1e3, "bytes": by_p, "achieved_gbs": ach_p, "frac_of_peak": ach_p / HBM_PEAK_GBS,
            "copy_gbs": cp, "frac_of_copy": ach_p / cp,
            "traffic": measured_traffic("precond_full", PREC_TRAFFIC_FILE, PREC_SOURCES),
            "coarse_levels": st["coarse_levels"], "coarse_dense_dofs": st["coarse_dense"]}
    lat = rmx["lat"] * 1e3
    value = args.steps / rmx["total_s"]
    ref_u, ref_p = r64["flux"], r64["pres"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rmx["total_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": desc,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "iterations": st["it"],
        "kappa": st["kappa"],
        "n_coarse": st["n_coarse"],
        "omega_tilde": st["omega_tilde"],
        "setup_ms": rmx["setup_s"] * 1e3,
        "host_buffers_ms_per_step": rmx["host_ms"],
        "pcg_ms": st["t_pcg_ms"],
        "autotune": {"sweep_widths": [st["sweep_wide4"], st["sweep_wide16"]], "t_workgroups": st["t_workgroups"],
                     "tune_ms": st["t_tune_ms"], "coarse_ms_per_width": st["tune_coarse_ms"],
                     "precond_ms_per_t_grid": st["tune_precond_ms"],
                     "single_lane_rows_upto": st["sweep_wide1"],
                     "coarse_ms_per_single_lane_limit": st["tune_wide1_ms"],
                     "subtree_levels": st["sweep_subtree_levels"],
                     "coarse_ms_per_subtree_levels": st["tune_subtree_ms"],
                     "note": "coarse sweeps timed with lane-group widths (8,32) (12,48) (24,96) (48,192), then "
                             "with single-lane rows up to 0, 8, 16, 32 entries, then with the bottom 0..6 levels "
                             "swept by one launch per direction (a workgroup per subtree); preconditioner with T^i "
                             "on 3 n_cu/4, n_cu, 2 n_cu, N workgroups; all timed from graph replays"},
        "fp64": {"value": args.steps / r64["total_s"], "unit": "solves/s",
                 "ms_per_step": r64["total_s"] / args.steps * 1e3,
                 "latency_ms": {"p50": float(np.percentile(r64["lat"] * 1e3, 50)),
                                "p99": float(np.percentile(r64["lat"] * 1e3, 99))},
                 "iterations": r64["stats"]["it"], "setup_ms": r64["setup_s"] * 1e3},
        "mixed_vs_fp64": {"flux_relerr": float(np.linalg.norm(rmx["flux"] - ref_u) / np.linalg.norm(ref_u)),
                          "pressure_relerr": float(np.linalg.norm(rmx["pres"] - ref_p) / np.linalg.norm(ref_p))},
        "multiscale": dict(msc, note="one multiscale row per face (Section 6) in place of the adaptive rows, "
                                     "mixed form") if msc else None,
        "steps12": dict(rmx["eps"] or {}, note="relative flux errors of u_0 (step 1) and u^* (steps 1-2) "
                                              "against the converged solve, eq. epsilon"),
        "roofline": roof,
        "precond_apply": prec,
    }
    if args.block_sources > 0:
        out["batch"] = block_batch(args.block_sources)
    if srv_out is not None:
        out["serving"], out["serving_resident"] = srv_out
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds, st["it"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
