"""Pins of the oracle's RT0/P0 discretisation against closed forms and printed counts."""
import numpy as np
import pytest

from oracle import rt0


def _linear_case(n, h, k, a):
    g = rt0.Grid(n, h)
    dim = len(n)
    perm = np.tile(np.asarray(k, dtype=float), (g.ncells, 1))
    dirs, _ = g.face_dir_coords()
    area = np.array([np.prod([h[e] for e in range(dim) if e != d]) for d in range(dim)])
    # u = -k grad p with p = a . x, total flux through a face = u_d * area_d
    uex = -np.asarray(k)[dirs] * np.asarray(a)[dirs] * area[dirs]
    bnd = g.boundary_faces()
    u, p = rt0.direct_solve(g, perm, np.zeros(g.ncells), bflux=np.where(bnd, uex, 0.0))
    cc = g.cell_coords()
    pex = sum(a[d] * (cc[d] + 0.5) * h[d] for d in range(dim))
    return g, u, uex, rt0.remove_mean(g, p), rt0.remove_mean(g, pex)


@pytest.mark.parametrize("n,h,k,a", [
    ((5, 7), (0.3, 0.2), (2.0, 5.0), (0.7, -1.3)),
    ((6, 4), (20.0, 10.0), (1e-3, 1e-3), (2.0, 1.0)),
    ((3, 4, 5), (1.0, 2.0, 0.5), (1.5, 0.7, 3.0), (0.7, -1.3, 0.4)),
])
def test_linear_pressure_reproduced_exactly(n, h, k, a):
    """A linear pressure at constant k lies in RT0 x P0 (cell-centre values)."""
    _, u, uex, p, pex = _linear_case(n, h, k, a)
    assert np.abs(u - uex).max() <= 1e-12 * np.abs(uex).max()
    assert np.abs(p - pex).max() <= 1e-12 * np.abs(pex).max()


def test_dof_counts_printed_in_section6():
    # 60x220 layer: 39,880 dofs; 30^3 cutout: 110,700 dofs (faces + cells)
    g2 = rt0.Grid((60, 220), (20.0, 10.0))
    g3 = rt0.Grid((30, 30, 30), (20.0, 10.0, 2.0))
    assert g2.nfaces + g2.ncells == 39880
    assert g3.nfaces + g3.ncells == 110700


def test_mass_matrix_energy_closed_form():
    """u_x = x (linear in x) is exact in RT0; a(u,u) = int k^-1 x^2 dV."""
    n, h = (4, 3), (0.5, 2.0)
    g = rt0.Grid(n, h)
    kx = 3.0
    perm = np.tile([kx, 7.0], (g.ncells, 1))
    A, _ = rt0.global_matrices(g, perm)
    dirs, coords = g.face_dir_coords()
    x = coords[:, 0] * h[0]
    u = np.where(dirs == 0, x * h[1], 0.0)            # flux = u_x * face area
    Lx, Ly = n[0] * h[0], n[1] * h[1]
    exact = Ly * Lx ** 3 / 3.0 / kx
    assert abs(u @ (A @ u) - exact) <= 1e-12 * exact


def test_divergence_kernel_is_constants():
    g = rt0.Grid((5, 4, 3), (1.0, 1.0, 1.0))
    _, B = rt0.global_matrices(g, np.ones((g.ncells, 3)))
    inner = ~g.boundary_faces()
    r = B[:, inner].T @ np.ones(g.ncells)
    assert np.abs(r).max() == 0.0
    # and the divergence of a unit flux through one inner face is -1 / +1
    f = np.flatnonzero(inner)[0]
    col = B[:, f].toarray().ravel()
    assert sorted(col[col != 0]) == [-1.0, 1.0]
