"""GPU GNEB chains (through the C ABI) against the FP64 oracle.

FP64 engine: iteration by iteration (the tangent rule and the velocity
projection take their discrete decisions from the same double-precision
values on both sides).  FP32 engine: the first iterations, and the converged
minimum-energy path; in between, FP32 and FP64 states can take different
tangent branches where neighbouring images have nearly equal energies, so
intermediate iterates are not comparable (the path the minimiser takes is
not unique, the converged path is)."""

import math

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, need_gpu

pytestmark = pytest.mark.gpu

MU_B = 9.2740100783e-24 / 1.602176634e-22
HAM0 = si.WORKLOADS["square32_fp64"].hamiltonian


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _single_spin(K=0.1, mu=2.0, B=1.0):
    geo = si.Geometry(((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 0, 0),), (1, 1, 1), (0, 0, 0))
    ham = si.Hamiltonian(mu=(mu,), B=(0, 0, B), K=(K,), K_axis=((0, 0, 1),))
    return geo, ham


def _bent_single_spin_chain(M):
    """-z to +z with unequal spacing and an out-of-plane bulge, so that both
    the energy force and the springs are non-zero."""
    v = np.arange(M) / (M - 1)
    theta = math.pi * (1.0 - v ** 1.3)
    phi = 0.5 * np.sin(math.pi * v)
    n = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], axis=1)
    n[0] = (0, 0, -1)
    n[-1] = (0, 0, 1)
    return n[:, :, None]


def _skyrmion_chain(geo, M, radius):
    a = si.skyrmion_ansatz(geo, radius=radius, width=1.5)
    b = si.ferromagnet(geo.n_sites, (0, 0, 1))
    return si.geodesic_chain(a, b, M, fallback_axis=(1, 0, 0))


def _pair(ora, geo, ham, precision, chain, **kw):
    import paper_1901_11350_amd as pk

    e = pk.Engine(0, precision)
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    g = pk.Gneb(e, chain, **kw)
    s = ora.System(geo, ham)
    o = ora.Gneb(s, chain, **kw)
    return e, g, o


def _case(name):
    if name == "single_spin":
        geo, ham = _single_spin()
        return geo, ham, _bent_single_spin_chain(21), dict(k_spring=1.0, vp_dt=0.5, vp_mass=1.0)
    if name == "square12x10":
        geo = si.square(12, 10)
        return geo, HAM0, _skyrmion_chain(geo, 8, 3.0), dict(k_spring=1.0, vp_dt=0.1, vp_mass=1.0)
    if name == "tri128x16_tiles":
        # sides divide into the 64 x 4 tiles of the stencil-path gradient:
        # three shells with interfacial DMI on the triangular stencil
        geo = si.triangular(128, 16)
        return (geo, si.WORKLOADS["triangular512_sllg"].hamiltonian, _skyrmion_chain(geo, 8, 3.0),
                dict(k_spring=1.0, vp_dt=0.1, vp_mass=1.0))
    geo = si.square(128, 128)
    return geo, HAM0, _skyrmion_chain(geo, 32, 5.0), dict(k_spring=1.0, vp_dt=0.1, vp_mass=1.0)


def chain_sensitivity(ora, geo, ham, chain, kw, iters, trials=3):
    """How far the oracle's own iteration map carries a rounding-size
    difference: chains whose interior images start 1e-15 apart (three random
    perturbations) are iterated beside the unperturbed one.  Returns the
    largest normwise chain difference (relative to the largest spin
    component) and force difference (relative to the initial force norm)
    over `iters` iterations.  The GPU sums in another order than the oracle,
    so its FP64 chain can part from the oracle's by as much as the map
    amplifies differences of that size."""
    s = ora.System(geo, ham)
    base = ora.Gneb(s, chain, **kw)
    F0 = np.linalg.norm(base.forces()["F"])
    rng = np.random.default_rng(12)
    others = []
    for _ in range(trials):
        c = np.array(chain, dtype=np.float64)
        c[1:-1] += 1e-15 * rng.standard_normal(c[1:-1].shape)
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        others.append(ora.Gneb(s, c, **kw))
    dc = dF = 0.0
    for _ in range(iters):
        base.iterate(1)
        fb = base.forces()["F"]
        for o in others:
            o.iterate(1)
            dc = max(dc, float(np.abs(o.chain - base.chain).max() / np.abs(base.chain).max()))
            dF = max(dF, float(np.linalg.norm(o.forces()["F"] - fb) / F0))
    return dc, dF


@pytest.mark.parametrize("case,iters", [("single_spin", 30), ("single_spin", 60), ("square12x10", 40),
                                        ("chain32x128x128", 20), ("tri128x16_tiles", 20)])
def test_gneb_fp64_iterations_match_oracle(ora, case, iters):
    """FP64 chain and forces after `iters` iterations within the 1e-12 bar,
    or within ten times what the oracle's own iteration map makes of 1e-15
    perturbations (measured here on the CPU), whichever is larger.  The
    velocity projection of the bent single-spin chain (vp_dt = 0.5) amplifies
    such differences about 1e5-fold between iterations 30 and 60, so only its
    60-iteration case needs the measured bound."""
    announce(f"gneb fp64 {case} {iters}")
    geo, ham, chain, kw = _case(case)
    e, g, o = _pair(ora, geo, ham, "f64", chain, **kw)
    f0, fo = g.forces(), o.forces()
    assert np.abs(fo["F"]).max() > 1e-3          # non-degenerate start
    assert_close(f0["F"], fo["F"], "f64", 1e-12, what="initial forces")
    assert np.allclose(f0["E"], fo["E"], rtol=1e-13, atol=1e-13 * np.abs(fo["E"]).max())
    assert np.allclose(f0["l"], fo["l"], rtol=1e-13)
    g.iterate(iters)
    o.iterate(iters)
    sens_c, sens_F = chain_sensitivity(ora, geo, ham, chain, kw, iters)
    tol_c = max(1e-12, 10 * sens_c)
    tol_F = max(1e-12, 10 * sens_F)
    print(f"[gneb] {case}: oracle divergence from 1e-15 over {iters} iterations: chain {sens_c:.2e}, "
          f"forces {sens_F:.2e}; bounds {tol_c:.1e} / {tol_F:.1e}", flush=True)
    assert_close(g.chain(), o.chain, "f64", tol_c, what=f"chain after {iters} iterations")
    fg, fo = g.forces(), o.forces()
    assert np.allclose(fg["E"], fo["E"], rtol=tol_c, atol=tol_c * np.abs(fo["E"]).max())
    # forces shrink as the chain converges: their difference is measured on
    # the scale of the initial forces, as the sensitivity is
    dF = np.linalg.norm(fg["F"] - fo["F"]) / np.linalg.norm(f0["F"])
    assert dF <= tol_F, f"forces: difference {dF:.3e} of the initial force norm > {tol_F:.1e}"


@pytest.mark.parametrize("case", ["single_spin", "square12x10", "chain32x128x128", "tri128x16_tiles"])
def test_gneb_fp32_first_iterations_match_oracle(ora, case):
    announce(f"gneb fp32 first iterations {case}")
    geo, ham, chain, kw = _case(case)
    e, g, o = _pair(ora, geo, ham, "f32", chain, **kw)
    assert_close(g.forces()["F"], o.forces()["F"], "f32", 1e-5, what="initial forces")
    g.iterate(3)
    o.iterate(3)
    assert_close(g.chain(), o.chain, "f32", 1e-5, what="chain after 3 iterations")


def test_gneb_fp32_converged_path_matches_oracle(ora):
    """Skyrmion-to-ferromagnet chain on a 12 x 10 lattice: after convergence
    the image energies and distances of the FP32 chain match the oracle's."""
    announce("gneb fp32 converged")
    geo, ham, chain, kw = _case("square12x10")
    e, g, o = _pair(ora, geo, ham, "f32", chain, **kw)
    g.iterate(1500)
    o.iterate(1500)
    fg, fo = g.forces(), o.forces()
    assert np.abs(fo["F"]).max() < 1e-9
    assert np.abs(fg["F"]).max() < 1e-3
    assert np.allclose(fg["E"], fo["E"], rtol=1e-5, atol=1e-5 * np.abs(fo["E"]).max())
    assert np.allclose(fg["l"], fo["l"], rtol=1e-4, atol=1e-4 * fo["l"].max())


def test_gneb_stoner_wohlfarth_barrier_fp32():
    import paper_1901_11350_amd as pk

    announce("gneb stoner-wohlfarth fp32")
    K, mu, B = 0.1, 2.0, 1.0
    h = mu * MU_B * B / (2 * K)
    geo, ham = _single_spin(K, mu, B)
    e = pk.Engine(0, "f32")
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    M = 37
    g = pk.Gneb(e, _bent_single_spin_chain(M), vp_dt=0.5)
    g.iterate(6000)
    f = g.forces()
    assert np.abs(f["F"]).max() < 1e-5
    barrier = f["E"].max() - f["E"][0]
    exact = K * (1 - h) ** 2
    bound = K * (1 - h * h) * (math.pi / (M - 1) / 2) ** 2
    assert -1e-6 <= exact - barrier <= bound + 1e-6


# ------------------------------------------- climbing and falling images

from test_oracle_gneb import _descend, gaussian_landscape, gaussian_system, geodesic  # noqa: E402


def _gauss_ham():
    return si.Hamiltonian(mu=(1.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), gauss=gaussian_landscape())


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gaussian_landscape_gradient_and_energy_match_oracle(ora, precision):
    """The on-site Gaussian potentials on a 9 x 7 lattice with exchange."""
    from gpu_util import make_pair

    announce(f"gaussian landscape field {precision}")
    geo = si.square(9, 7)
    ham = dataclasses_replace(_gauss_ham(), J=(0.3,))
    e, s = make_pair(ora, geo, ham, precision)
    n = si.uniform_sphere(geo.n_sites, 12)
    e.set_spins(n)
    assert_close(e.gradient(), s.gradient(n), precision, what="gradient with Gaussians")
    E, pt = e.energy(per_term=True)
    Eo, pto = s.energy(n, per_term=True)
    tol = 1e-12 if precision == "f64" else 1e-5
    assert abs(E - Eo) <= tol * np.abs(pto).sum()
    assert abs(pt[1] - pto[1]) <= tol * np.abs(pto).sum()


def _relaxed_gaussian_chain(ora):
    """Oracle chain between the minima of rows 6 and 7 of the Appendix G
    landscape, relaxed without special images, and the image types: the two
    interior energy maxima climb, the interior minimum falls.  The early
    iterations from a geodesic guess amplify rounding differences ~100x per
    ten iterations (tangent branches switch where neighbouring energies are
    nearly equal), so both engines start from this relaxed chain."""
    s = gaussian_system(ora)
    gl = gaussian_landscape()
    a, b = _descend(s, np.array(gl[5][2])), _descend(s, np.array(gl[6][2]))
    o = ora.Gneb(s, geodesic(a, b, 40), k_spring=1.0, vp_dt=0.1)
    o.iterate(3000)
    E = o.forces()["E"]
    M = len(E)
    maxima = [k for k in range(1, M - 1) if E[k] > E[k - 1] and E[k] > E[k + 1]]
    minima = [k for k in range(1, M - 1) if E[k] < E[k - 1] and E[k] < E[k + 1]]
    assert len(maxima) == 2 and len(minima) == 1
    types = ["normal"] * M
    types[maxima[0]] = types[maxima[1]] = "climbing"
    types[minima[0]] = "falling"
    return s, o.chain.copy(), types, maxima + minima


def _ci_pair(ora, precision, s, chain, types):
    import paper_1901_11350_amd as pk

    geo = si.Geometry(((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 0, 0),), (1, 1, 1), (0, 0, 0))
    e = pk.Engine(0, precision)
    e.set_geometry(geo)
    e.set_hamiltonian(_gauss_ham())
    g = pk.Gneb(e, chain, k_spring=1.0, vp_dt=0.1)
    o = ora.Gneb(s, chain, k_spring=1.0, vp_dt=0.1)
    g.set_image_types(types)
    o.set_image_types(types)
    return e, g, o


def test_climbing_falling_fp64_iterations_match_oracle(ora):
    announce("gneb climbing/falling fp64")
    s, chain, types, special = _relaxed_gaussian_chain(ora)
    e, g, o = _ci_pair(ora, "f64", s, chain, types)
    g.iterate(20)
    o.iterate(20)
    assert_close(g.chain(), o.chain, "f64", 1e-10, what="20 iterations with climbing and falling images")
    g.iterate(12000)
    o.iterate(12000)
    assert np.abs(o.forces()["F"]).max() < 1e-10
    assert_close(g.chain()[special], o.chain[special], "f64", 1e-9, what="converged critical points")


def test_climbing_falling_fp32_converge_to_the_oracle_critical_points(ora):
    """FP32 chain with two climbing and one falling image: the special images
    land on the oracle's converged saddles and minimum."""
    announce("gneb climbing/falling fp32")
    s, chain, types, special = _relaxed_gaussian_chain(ora)
    e, g, o = _ci_pair(ora, "f32", s, chain, types)
    g.iterate(12000)
    o.iterate(12000)
    fo = o.forces()
    assert np.abs(fo["F"]).max() < 1e-10
    cg, co = g.chain(), o.chain
    fg = g.forces()
    for k in special:
        assert np.abs(cg[k] - co[k]).max() < 2e-4, k
        assert fg["E"][k] == pytest.approx(fo["E"][k], abs=2e-6)


def dataclasses_replace(obj, **kw):
    import dataclasses

    return dataclasses.replace(obj, **kw)
