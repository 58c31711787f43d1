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


# ------------------------------------------- climbing and falling images

GOLDEN = __import__("pathlib").Path(__file__).parent / "golden" / "gaussian_landscape_appendix_g.txt"


def gaussian_landscape():
    """The seven Gaussians of the single-spin landscape (Appendix G table)."""
    rows = [line.split() for line in GOLDEN.read_text().splitlines() if line.strip() and not line.startswith("#")]
    return tuple((float(r[0]), float(r[1]), (float(r[2]), float(r[3]), float(r[4]))) for r in rows)


def gaussian_system(ora):
    geo = si.Geometry(((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 0, 0),), (1, 1, 1), (0, 0, 0))
    ham = si.Hamiltonian(mu=(1.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), gauss=gaussian_landscape())
    return ora.System(geo, ham)


def _tangent_grad(s, n):
    g = s.gradient(n.reshape(3, 1))[:, 0]
    return g - g.dot(n) * n


def _descend(s, n, steps=40000, lr=0.002):
    """Projected gradient descent on the sphere (independent of GNEB)."""
    n = np.array(n, float) / np.linalg.norm(n)
    for _ in range(steps):
        n = n - lr * _tangent_grad(s, n)
        n /= np.linalg.norm(n)
    return n


def _tangent_hessian(s, n, h=1e-5):
    """2x2 Hessian of E on the sphere at n (central differences of the
    tangential gradient along an orthonormal tangent basis)."""
    a = np.cross(n, [1.0, 0, 0] if abs(n[0]) < 0.9 else [0, 1.0, 0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    H = np.zeros((2, 2))
    for j, t in enumerate((a, b)):
        gp = _tangent_grad(s, (n + h * t) / np.linalg.norm(n + h * t))
        gm = _tangent_grad(s, (n - h * t) / np.linalg.norm(n - h * t))
        d = (gp - gm) / (2 * h)
        H[0, j], H[1, j] = d.dot(a), d.dot(b)
    return 0.5 * (H + H.T)


def test_gaussian_landscape_gradient_matches_finite_differences(ora):
    s = gaussian_system(ora)
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        g = s.gradient(n.reshape(3, 1))[:, 0]
        h = 1e-6
        fd = np.array([(s.energy((n + h * e).reshape(3, 1)) - s.energy((n - h * e).reshape(3, 1))) / (2 * h)
                       for e in np.eye(3)])
        assert np.allclose(g, fd, atol=1e-7)
    # at a centre direction far from the others the energy is a_k plus tails
    c = np.array(gaussian_landscape()[0][2])
    c /= np.linalg.norm(c)
    assert s.energy(c.reshape(3, 1)) == pytest.approx(-1.1, abs=1e-3)


def geodesic(a, b, M):
    om = math.acos(float(np.clip(a.dot(b), -1, 1)))
    return np.array([(math.sin((1 - t) * om) * a + math.sin(t * om) * b) / math.sin(om)
                     for t in np.linspace(0, 1, M)])[:, :, None]


def test_climbing_and_falling_images_find_the_saddles_and_the_minimum(ora):
    """Chain between the minima near c6 and c7 of the Appendix G landscape:
    the relaxed path crosses two barriers with the deepest minimum (near c1)
    between them.  With two climbing images and one falling image the
    chain's critical points are exact: the falling image sits at the
    minimum found by plain descent from c1, and each climbing image has zero
    tangential gradient with one negative and one positive curvature."""
    s = gaussian_system(ora)
    gl = gaussian_landscape()
    m_start = _descend(s, np.array(gl[5][2]))
    m_end = _descend(s, np.array(gl[6][2]))
    m_deep = _descend(s, np.array(gl[0][2]))
    M = 40
    g = ora.Gneb(s, geodesic(m_start, m_end, M), k_spring=1.0, vp_dt=0.1)
    g.iterate(6000)
    E = g.forces()["E"]
    maxima = [k for k in range(1, M - 1) if E[k] > E[k - 1] and E[k] > E[k + 1]]
    minima = [k for k in range(1, M - 1) if E[k] < E[k - 1] and E[k] < E[k + 1]]
    assert len(maxima) == 2 and len(minima) == 1
    types = ["normal"] * M
    types[maxima[0]] = types[maxima[1]] = "climbing"
    types[minima[0]] = "falling"
    g.set_image_types(types)
    g.iterate(10000)
    f = g.forces()
    assert np.abs(f["F"]).max() < 1e-10
    fi = g.chain[minima[0]][:, 0]
    assert np.abs(fi - m_deep).max() < 1e-6
    assert f["E"][minima[0]] == pytest.approx(s.energy(m_deep.reshape(3, 1)), abs=1e-12)
    for k in maxima:
        n = g.chain[k][:, 0]
        assert np.linalg.norm(_tangent_grad(s, n)) < 1e-10
        ev = np.linalg.eigvalsh(_tangent_hessian(s, n))
        assert ev[0] < -1e-3 and ev[1] > 1e-3
        # climbing image above both neighbours; barrier heights from each side
        assert f["E"][k] > f["E"][k - 1] and f["E"][k] > f["E"][k + 1]
    # normal images keep the spring spacing between the special images
    assert np.all(f["l"] > 0)
