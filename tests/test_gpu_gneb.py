"""GPU GNEB chains (through the C ABI) against the FP64 oracle: iteration by
iteration in FP64 and FP32, the Stoner-Wohlfarth barrier, and the 32-image
128 x 128 chain of the batched workload."""

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


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["single_spin", "square12x10_skyrmion"])
def test_gneb_iterations_match_oracle(ora, case, precision):
    announce(f"gneb {case} {precision}")
    if case == "single_spin":
        geo, ham = _single_spin()
        chain = si.geodesic_chain(np.array([[0.0], [0.0], [-1.0]]), np.array([[0.0], [0.0], [1.0]]), 21)
        kw = dict(k_spring=1.0, vp_dt=0.5, vp_mass=1.0)
        iters = 60
    else:
        geo = si.square(12, 10)
        ham = HAM0
        chain = _skyrmion_chain(geo, 8, 3.0)
        kw = dict(k_spring=1.0, vp_dt=0.1, vp_mass=1.0)
        iters = 30
    e, g, o = _pair(ora, geo, ham, precision, chain, **kw)
    f0 = g.forces()
    fo = o.forces()
    tol = 1e-12 if precision == "f64" else 1e-5
    assert_close(f0["F"], fo["F"], precision, tol, what="initial forces")
    assert np.allclose(f0["E"], fo["E"], rtol=tol, atol=tol * np.abs(fo["E"]).max())
    g.iterate(iters)
    o.iterate(iters)
    tol = 1e-11 if precision == "f64" else 1e-5
    assert_close(g.chain(), o.chain, precision, tol, what=f"chain after {iters} iterations")
    fg, fo = g.forces(), o.forces()
    assert np.allclose(fg["l"], fo["l"], rtol=10 * tol)
    assert np.allclose(fg["E"], fo["E"], rtol=10 * tol, atol=10 * tol * np.abs(fo["E"]).max())


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
    chain = si.geodesic_chain(np.array([[0.0], [0.0], [-1.0]]), np.array([[0.0], [0.0], [1.0]]), M)
    g = pk.Gneb(e, chain, vp_dt=0.5)
    g.iterate(6000)
    f = g.forces()
    assert np.abs(f["F"]).max() < 1e-5
    barrier = f["E"].max() - f["E"][0]
    exact = K * (1 - h) ** 2
    bound = K * (1 - h * h) * (math.pi / (M - 1) / 2) ** 2
    assert -1e-6 <= exact - barrier <= bound + 1e-6


def test_gneb_full_chain_32x128x128(ora):
    """The 32-image chain of the batched workload (periodic 128 x 128 square
    lattice, square32 Hamiltonian, skyrmion to ferromagnet), FP32, 40 VP
    iterations against the oracle."""
    announce("gneb full chain 32 x 128^2")
    geo = si.square(128, 128)
    chain = _skyrmion_chain(geo, 32, 5.0)
    e, g, o = _pair(ora, geo, HAM0, "f32", chain, k_spring=1.0, vp_dt=0.1, vp_mass=1.0)
    g.iterate(40)
    o.iterate(40)
    assert_close(g.chain(), o.chain, "f32", what="chain after 40 iterations")
    fg, fo = g.forces(), o.forces()
    assert np.allclose(fg["E"], fo["E"], rtol=1e-5)
