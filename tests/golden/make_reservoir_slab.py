"""Stored oracle solve of a 60x220x20 slab of the 60x220x85 reservoir workload.

Writes reservoir_slab_60x220x20_tau10.json next to this file, from the CPU
oracle only (``oracle/``; inputs from ``workloads/``): layers 30-49 of the
seeded SPE10-shaped reservoir field (the last five smooth layers and the first
fifteen channelised ones), the same 10x10x5-cell boxes (6 x 22 x 4 = 528
subdomains, interior ones with six faces), the same well columns, adaptive
tau = 10, conjugate gradients to rtol 1e-8.  The whole 60x220x85 problem does
not fit the oracle's sparse local factorizations in host memory (about 28 MB
per subdomain), so this slab stands in for it; the GPU test solves the same
slab and compares.

Stored: iterations, the condition estimate, omega-tilde, coarse-space sizes,
the norms of the flux and pressure, and their values at seeded sample
positions (flux at interior faces, pressure at cells).

usage: python tests/golden/make_reservoir_slab.py   (about 15 minutes, ~15 GB)
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import bddc as ob, rt0  # noqa: E402

OUT = os.path.join(HERE, "reservoir_slab_60x220x20_tau10.json")
Z0, NZ = 30, 20
N_FLUX_SAMPLES, N_PRES_SAMPLES = 6000, 3000


def slab_problem():
    """Layers Z0 .. Z0+NZ-1 of the reservoir workload, its boxes and wells."""
    full = W.reservoir_3d(nz=85, seed=0, tau=10.0)
    n = (full.n[0], full.n[1], NZ)
    idx = np.arange(np.prod(full.n)).reshape(full.n, order="F")[:, :, Z0:Z0 + NZ].reshape(-1, order="F")
    src = full.source[idx].copy()
    src -= src.mean()
    return W.Problem("reservoir_slab", n, full.h, full.perm[idx].copy(), src, W.regular_cuts(n, (10, 10, 5)),
                     tau=10.0, rtol=1e-8)


def sample_positions(n_faces, interior, n_cells):
    rng = np.random.default_rng(20260101)
    fpos = np.sort(rng.choice(interior, size=N_FLUX_SAMPLES, replace=False))
    cpos = np.sort(rng.choice(n_cells, size=N_PRES_SAMPLES, replace=False))
    return fpos, cpos


def main():
    pr = slab_problem()
    g = rt0.Grid(pr.n, pr.h)
    t0 = time.time()
    o = ob.BDDC(g, pr.perm, pr.cuts, tau=pr.tau)
    t1 = time.time()
    print(f"setup {t1 - t0:.0f} s: N {o.subs.N}, n_c {o.n_c}, omega {o.omega_tilde:.6f}", flush=True)
    out = o.solve(pr.source, rtol=pr.rtol, maxit=5000)
    t2 = time.time()
    lmin, lmax, kappa = ob.lanczos_kappa(out["alphas"], out["betas"])
    print(f"solve {t2 - t1:.0f} s: it {out['it']}, kappa {kappa:.6f}", flush=True)
    u, p = out["u"], out["p"]
    interior = np.flatnonzero(~g.boundary_faces())
    fpos, cpos = sample_positions(g.nfaces, interior, g.ncells)
    res = {
        "what": "oracle BDDC-PCG (FP64) on layers 30-49 of the 60x220x85 reservoir workload (seed 0), "
                "10x10x5-cell boxes, tau 10, rtol 1e-8",
        "script": "tests/golden/make_reservoir_slab.py",
        "n": list(pr.n), "z0": Z0, "N": int(o.subs.N), "n_gamma": int(o.subs.n_gamma),
        "n_faces": int(o.subs.n_faces), "n_adaptive": int(sum(o.face_k)), "n_coarse": int(o.n_c),
        "omega_tilde": float(o.omega_tilde), "it": int(out["it"]), "converged": bool(out["converged"]),
        "relres": float(out["relres"]), "kappa": float(kappa), "lambda_min": float(lmin),
        "lambda_max": float(lmax), "flux_norm": float(np.linalg.norm(u)), "pressure_norm": float(np.linalg.norm(p)),
        "flux_pos": fpos.tolist(), "flux": [float(v) for v in u[fpos]],
        "pressure_pos": cpos.tolist(), "pressure": [float(v) for v in p[cpos]],
        "oracle_seconds": {"setup": t1 - t0, "solve": t2 - t1},
    }
    with open(OUT, "w") as f:
        json.dump(res, f)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
