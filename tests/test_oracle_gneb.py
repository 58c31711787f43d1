"""Pins of the oracle's GNEB (Sec. III.D; Appendices D and F).

Stoner-Wohlfarth: one spin with uniaxial anisotropy K along z in a field B
along z has its metastable minimum at -z, the saddle at cos(theta) = -h with
h = mu mu_B B / (2K), and the barrier K (1 - h)^2.  The converged chain's
highest image lies below the saddle by at most |E''| (dtheta/2)^2 / 2 for
image spacing dtheta, with E'' = -2K (1 - h^2) at the saddle.
"""

import math

import numpy as np
import pytest

import spin_inputs as si

MU_B = 9.2740100783e-24 / 1.602176634e-22


def _single_spin_system(ora, K=0.1, mu=2.0, B=1.0, n_cells=(1, 1, 1), J=()):
    geo = si.Geometry(((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 0, 0),), n_cells,
                      (1, 1, 0) if n_cells[0] > 1 else (0, 0, 0))
    ham = si.Hamiltonian(mu=(mu,), B=(0, 0, B), K=(K,), K_axis=((0, 0, 1),), J=J)
    return ora.System(geo, ham)


def _converge(g, max_iter=40000, tol=1e-9):
    for _ in range(max_iter // 500):
        g.iterate(500)
        if np.abs(g.F_prev).max() < tol:
            return True
    return False


def test_stoner_wohlfarth_values():
    K, mu, B = 0.1, 2.0, 1.0
    h = mu * MU_B * B / (2 * K)
    assert h == pytest.approx(0.578838, abs=1e-6)
    assert K * (1 - h) ** 2 == pytest.approx(0.0177377, abs=1e-7)


@pytest.mark.parametrize("M", [21, 41])
def test_gneb_single_spin_barrier(ora, M):
    K, mu, B = 0.1, 2.0, 1.0
    h = mu * MU_B * B / (2 * K)
    s = _single_spin_system(ora, K, mu, B)
    a = np.array([[0.0], [0.0], [-1.0]])
    b = np.array([[0.0], [0.0], [1.0]])
    chain = si.geodesic_chain(a, b, M, fallback_axis=(0, 1, 0))
    g = ora.Gneb(s, chain, k_spring=1.0, vp_dt=0.5, vp_mass=1.0)
    assert _converge(g)
    f = g.forces()
    E = f["E"]
    barrier = E.max() - E[0]
    exact = K * (1 - h) ** 2
    dtheta = math.pi / (M - 1)
    bound = 0.5 * 2 * K * (1 - h * h) * (dtheta / 2) ** 2
    assert barrier <= exact + 1e-12
    assert exact - barrier <= bound
    # images equidistant along the path (springs), path stays in the xz plane
    assert np.ptp(f["l"]) < 1e-6
    assert np.abs(g.chain[:, 1, :]).max() < 1e-10
    assert sum(f["l"]) == pytest.approx(math.pi, abs=1e-6)
    # forces on every spin are perpendicular to it and vanish at convergence
    assert np.abs(np.sum(f["F"] * g.chain, axis=1)).max() < 1e-12


def test_gneb_more_images_approach_the_saddle(ora):
    K, mu, B = 0.1, 2.0, 1.0
    h = mu * MU_B * B / (2 * K)
    exact = K * (1 - h) ** 2
    errs = []
    # image spacings 15 and 5 degrees: nearest images 120 and 125 degrees
    # from the saddle at arccos(-h) = 125.37 degrees
    for M in (13, 37):
        s = _single_spin_system(ora, K, mu, B)
        chain = si.geodesic_chain(np.array([[0.0], [0.0], [-1.0]]), np.array([[0.0], [0.0], [1.0]]), M)
        g = ora.Gneb(s, chain, vp_dt=0.5)
        assert _converge(g)
        E = g.forces()["E"]
        errs.append(exact - (E.max() - E[0]))
    assert 0 <= errs[1] < errs[0]


def test_gneb_coherent_rotation_of_a_ferromagnet(ora):
    """4x4 periodic ferromagnet, uniform initial path from -z to +z: by symmetry
    the path stays uniform and its barrier is N times the single-spin one."""
    K, mu, B = 0.1, 2.0, 1.0
    h = mu * MU_B * B / (2 * K)
    s = _single_spin_system(ora, K, mu, B, n_cells=(4, 4, 1), J=(1.0,))
    N = s.N
    a = np.tile([[0.0], [0.0], [-1.0]], (1, N))
    b = np.tile([[0.0], [0.0], [1.0]], (1, N))
    M = 21
    g = ora.Gneb(s, si.geodesic_chain(a, b, M, fallback_axis=(1, 0, 0)), vp_dt=0.5)
    assert _converge(g, tol=1e-8)
    E = g.forces()["E"]
    dtheta = math.pi / (M - 1)
    exact = N * K * (1 - h) ** 2
    assert E.max() - E[0] <= exact + 1e-10
    assert exact - (E.max() - E[0]) <= N * K * (1 - h * h) * (dtheta / 2) ** 2
    assert np.abs(g.chain - g.chain[:, :, :1]).max() < 1e-9
