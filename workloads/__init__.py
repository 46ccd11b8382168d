"""Seeded synthetic inputs for the RT0/P0 Darcy problem and its box partitions.

This module only *generates* problem data (grids, permeability fields, well
sources, subdomain cut planes).  It holds none of the discretisation or solver
arithmetic, so both the CPU oracle and the GPU library can draw their inputs
from it without sharing any part of the method.

Conventions shared with every consumer:

* cells are numbered x-fastest: ``c = ix + nx*(iy + ny*iz)``;
* ``perm`` has shape ``[n_cells, dim]`` (diagonal tensor k_x, k_y[, k_z]), in mD;
* ``source`` has shape ``[n_cells]``: the cell-integrated volumetric source
  (injection > 0, production < 0) with zero sum, matching the compatibility
  condition of the no-flow problem (Section 2, eq. compatibility);
* ``cuts`` is a list with one increasing integer array per axis,
  ``cuts[d][0] == 0`` and ``cuts[d][-1] == n[d]``: box subdomains are the
  tensor product of the axis intervals (the regular and geometric partitions
  of Section 6, Table 1).

The SPE10 Model 2 data the paper uses is not available here; the fields below
reproduce its shape (layered smooth top, fluvial channelised bottom, six or
more decades of contrast, 20x10x2 ft cells, Section 6) from fixed seeds.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage


@dataclasses.dataclass
class Problem:
    """One synthetic workload: grid, field, sources and partition."""

    name: str
    n: tuple            # cells per axis
    h: tuple            # cell size per axis
    perm: np.ndarray    # [n_cells, dim] float64 > 0
    source: np.ndarray  # [n_cells] float64, sum 0
    cuts: list          # per-axis int arrays
    tau: float = math.inf
    rtol: float = 1e-8

    @property
    def dim(self):
        return len(self.n)

    @property
    def n_cells(self):
        return int(np.prod(self.n))


# ----------------------------------------------------------------------------
# partitions
# ----------------------------------------------------------------------------

def regular_cuts(n, sub):
    """Cut planes every ``sub[d]`` cells.

    A remainder shorter than half a block is merged into the last block, so
    220 cells at H/h = 30 give six 30-cell and one 40-cell interval (the 14
    subdomains of the 2D H/h = 30 partition in Table 1).
    """
    cuts = []
    for nd, sd in zip(n, sub):
        c = list(range(0, nd, sd)) + [nd]
        if len(c) > 2 and 2 * (c[-1] - c[-2]) < sd:
            c.pop(-2)
        cuts.append(np.asarray(c, dtype=np.int64))
    return cuts


def split_cuts(n, nsub):
    """``nsub[d]`` near-equal intervals per axis (larger intervals first)."""
    cuts = []
    for nd, k in zip(n, nsub):
        sizes = [nd // k + (1 if r < nd % k else 0) for r in range(k)]
        cuts.append(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64))
    return cuts


def seeded_cuts(n, lo, hi, seed):
    """Cut planes with interval widths drawn uniformly from [lo, hi]."""
    rng = np.random.default_rng(seed)
    cuts = []
    for nd in n:
        c = [0]
        while c[-1] < nd:
            w = int(rng.integers(lo, hi + 1))
            c.append(min(nd, c[-1] + w))
        if len(c) > 2 and c[-1] - c[-2] < lo:   # merge a short tail
            c.pop(-2)
        cuts.append(np.asarray(c, dtype=np.int64))
    return cuts


# ----------------------------------------------------------------------------
# permeability fields
# ----------------------------------------------------------------------------

def gaussian_field_exact(n, h, std, corr, seed):
    """Gaussian random field sampled exactly from its covariance.

    Squared-exponential covariance ``std^2 exp(-r^2 / (2 corr^2))`` between
    cell centres, plus a nugget of 1e-10 std^2 on the diagonal; the sample is
    ``L xi`` with L the Cholesky factor.  (The covariance is numerically rank
    deficient: an eigendecomposition would leave the basis of its near-null
    space, and so the sample, to the LAPACK build; the Cholesky factor of the
    regularised matrix is unique, so every machine draws the same field.)
    Only sensible for small grids (a few thousand cells).
    """
    axes = [(np.arange(nd) + 0.5) * hd for nd, hd in zip(n, h)]
    mesh = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([m.reshape(-1, order="F") for m in mesh], axis=1)
    d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    cov = std ** 2 * np.exp(-d2 / (2.0 * corr ** 2))
    cov[np.diag_indices_from(cov)] += 1e-10 * std ** 2
    chol = np.linalg.cholesky(cov)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(len(cov))
    return chol @ xi


def _smoothed_normal(shape, sigma, rng):
    """White noise smoothed by a Gaussian kernel and re-standardised."""
    g = rng.standard_normal(shape)
    g = ndimage.gaussian_filter(g, sigma=sigma, mode="reflect")
    g -= g.mean()
    s = g.std()
    return g / s if s > 0 else g


def channel_layer(nx, ny, rng, n_channels=6):
    """One fluvial layer (ln k, indexed [ix, iy]) in the spirit of SPE10's bottom.

    Background: ln k ~ N(ln 0.5, 1.5^2), correlation about 3 cells.
    Channels run along y with a sinuous centreline
    ``x(y) = x0 + A sin(2 pi y / lam + phi)``, A in [5, 15] cells,
    lam in [40, 120] cells, width 3..6 cells, ln k ~ N(7, 1) inside.
    """
    lnk = math.log(0.5) + 1.5 * _smoothed_normal((nx, ny), 3.0, rng)
    iy = np.arange(ny)
    ix = np.arange(nx)[:, None]
    for _ in range(n_channels):
        x0 = rng.uniform(0, nx)
        amp = rng.uniform(5, 15)
        lam = rng.uniform(40, 120)
        phi = rng.uniform(0, 2 * math.pi)
        width = rng.uniform(3, 6)
        centre = x0 + amp * np.sin(2 * math.pi * iy / lam + phi)
        inside = np.abs(ix - centre[None, :]) <= width / 2.0
        vals = rng.normal(7.0, 1.0, size=(nx, ny))
        lnk = np.where(inside, vals, lnk)
    return lnk


def clip_k(lnk):
    return np.clip(np.exp(lnk), 1e-3, 2e4)


# ----------------------------------------------------------------------------
# well sources
# ----------------------------------------------------------------------------

def _cell(n, idx):
    c = 0
    stride = 1
    for nd, i in zip(n, idx):
        c += int(i) * stride
        stride *= nd
    return c


def five_spot(n, centre, rate=1.0):
    """+rate at the centre cell (column in 3D), -rate/4 at the four corners."""
    ncell = int(np.prod(n))
    f = np.zeros(ncell)
    nz = n[2] if len(n) == 3 else 1
    corners = [(0, 0), (n[0] - 1, 0), (0, n[1] - 1), (n[0] - 1, n[1] - 1)]
    for iz in range(nz):
        tail = (iz,) if len(n) == 3 else ()
        f[_cell(n, tuple(centre) + tail)] += rate / nz
        for cx, cy in corners:
            f[_cell(n, (cx, cy) + tail)] -= rate / (4 * nz)
    return f


def corner_pair(n, rate=1.0):
    """Source in the first cell, sink in the last (opposite corner)."""
    f = np.zeros(int(np.prod(n)))
    f[0] += rate
    f[-1] -= rate
    return f


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def unit_square_16(seed=0):
    """16x16 unit square, k = exp(g) with g a GRF (std 2, corr 0.2), 4x4 boxes."""
    n, h = (16, 16), (1 / 16, 1 / 16)
    g = gaussian_field_exact(n, h, 2.0, 0.2, seed)
    k = np.exp(g)
    perm = np.stack([k, k], axis=1)
    return Problem(f"square16_s{seed}", n, h, perm, corner_pair(n), regular_cuts(n, (4, 4)),
                   tau=math.inf, rtol=1e-10)


def layer_60x220(seed=0, tau=10.0, sub=(10, 10)):
    """Single SPE10-shaped layer, 60x220 cells of 20x10 ft, channelised."""
    n, h = (60, 220), (20.0, 10.0)
    rng = np.random.default_rng(1000 + seed)
    lnk = channel_layer(60, 220, rng)
    k = clip_k(lnk).reshape(-1, order="F")
    perm = np.stack([k, k], axis=1)
    src = five_spot(n, (30, 110))
    return Problem(f"layer60x220_s{seed}", n, h, perm, src, regular_cuts(n, sub),
                   tau=tau, rtol=1e-8)


def reservoir_3d(nz=85, seed=0, tau=10.0, sub=(10, 10, 5), n_top=None):
    """60x220xnz field with 20x10x2 ft cells.

    The top ``n_top`` layers (35 of 85 by default, scaled with nz) are a smooth
    log-normal field with correlation (20, 20, 2) cells; the rest are fluvial
    channel layers whose channels persist across 2..4 layers.  k_z = 0.1 k_x.
    """
    nx, ny = 60, 220
    if n_top is None:
        n_top = int(round(35 * nz / 85))
    rng = np.random.default_rng(2000 + seed)
    lnk = np.empty((nx, ny, nz))
    if n_top > 0:
        top = math.log(0.5) + 1.5 * _smoothed_normal((nx, ny, n_top), (20.0, 20.0, 2.0), rng)
        lnk[:, :, :n_top] = top
    iz = n_top
    while iz < nz:
        span = int(rng.integers(2, 5))
        layer = channel_layer(nx, ny, rng)
        for j in range(iz, min(nz, iz + span)):
            jitter = 0.3 * rng.standard_normal((nx, ny))
            lnk[:, :, j] = layer + jitter
        iz += span
    k = clip_k(lnk).reshape(-1, order="F")
    perm = np.stack([k, k, 0.1 * k], axis=1)
    n = (nx, ny, nz)
    src = five_spot(n, (30, 110))
    return Problem(f"reservoir60x220x{nz}_s{seed}", n, (20.0, 10.0, 2.0), perm, src,
                   regular_cuts(n, sub), tau=tau, rtol=1e-8)


def homogeneous(n, h, cuts, source=None):
    """k = 1 everywhere (the homogeneous rows of Tables 2 and 5)."""
    ncell = int(np.prod(n))
    perm = np.ones((ncell, len(n)))
    src = corner_pair(n) if source is None else source
    return Problem("homogeneous", tuple(n), tuple(h), perm, src, cuts, tau=math.inf, rtol=1e-6)


# ----------------------------------------------------------------------------
# serving requests
# ----------------------------------------------------------------------------

def seeded_wells(n, rng, n_prod=None):
    """One injector and 1..4 producers at seeded cells (columns in 3D), zero total."""
    ncell = int(np.prod(n))
    f = np.zeros(ncell)
    nz = n[2] if len(n) == 3 else 1
    if n_prod is None:
        n_prod = int(rng.integers(1, 5))
    inj = (int(rng.integers(0, n[0])), int(rng.integers(0, n[1])))
    prods = []
    while len(prods) < n_prod:
        c = (int(rng.integers(0, n[0])), int(rng.integers(0, n[1])))
        if c != inj and c not in prods:
            prods.append(c)
    for iz in range(nz):
        tail = (iz,) if len(n) == 3 else ()
        f[_cell(n, inj + tail)] += 1.0 / nz
        for c in prods:
            f[_cell(n, c + tail)] -= 1.0 / (n_prod * nz)
    return f


def serving_request(seed):
    """One request of the serving stream: its own grid, field, wells and tau.

    2D: n_x in [32, 60], n_y in [32, 220] cells of 20 x 10 ft, one channelised
    layer, boxes of about 8 cells when the grid is 32 x 32 and about 10 cells
    otherwise.  3D (one request in four): a 60 x 220 x {5, 17, 34} slab of the
    layered channel field with 20 x 10 x 2 ft cells, 10 x 10 boxes in plane and
    about 5 layers per box.  tau is off or 10 with equal odds; rtol 1e-8.
    """
    rng = np.random.default_rng(5000 + seed)
    tau = math.inf if rng.random() < 0.5 else 10.0
    if rng.random() < 0.25:
        nz = int(rng.choice([5, 17, 34]))
        pr = reservoir_3d(nz=nz, seed=7000 + seed, tau=tau, sub=(10, 10, 5))
        nzs = max(1, round(nz / 5))
        cuts = split_cuts(pr.n, (6, 22, nzs))
        src = seeded_wells(pr.n, rng)
        return Problem(f"serve{seed}_3d{nz}", pr.n, pr.h, pr.perm, src, cuts, tau=tau, rtol=1e-8)
    nx = int(rng.integers(32, 61))
    ny = int(rng.integers(32, 221))
    n, h = (nx, ny), (20.0, 10.0)
    lnk = channel_layer(nx, ny, rng, n_channels=max(1, nx // 10))
    k = clip_k(lnk).reshape(-1, order="F")
    perm = np.stack([k, k], axis=1)
    box = 8 if (nx, ny) == (32, 32) else 10
    cuts = split_cuts(n, (max(1, round(nx / box)), max(1, round(ny / box))))
    src = seeded_wells(n, rng)
    return Problem(f"serve{seed}_2d{nx}x{ny}", n, h, perm, src, cuts, tau=tau, rtol=1e-8)


def poisson_arrivals(rate, count, seed):
    """Arrival times (s) of a Poisson stream with the given mean rate."""
    rng = np.random.default_rng(9000 + seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
