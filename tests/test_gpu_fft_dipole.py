"""GPU tests of the FFT-convolution dipole field (SP_DDI_FFT) against the
FP64 oracle's direct pair sum: small lattices element by element (several
transform lengths, ragged sizes, a two-atom basis, a chain, a single site),
the 128 x 128 x 4 film on sampled sites, and Depondt trajectories."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, make_pair, need_gpu

pytestmark = pytest.mark.gpu

SP_DDI_FFT = 3
DIP = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), ddi=SP_DDI_FFT)


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _two_basis():
    geo = si.Geometry(((1, 0, 0), (0.5, 0.8660254037844386, 0), (0, 0, 1.3)),
                      ((0, 0, 0), (0.5, 0.2886751345948129, 0.4)), (9, 7, 2), (1, 0, 0))
    ham = si.Hamiltonian(mu=(2.0, 1.5), B=(0, 0, 0), K=(0.0, 0.0), K_axis=((0, 0, 1), (0, 0, 1)), ddi=SP_DDI_FFT)
    return geo, ham


CASES = {
    "single_site": (si.simple_cubic(1, 1, 1, periodic=(0, 0, 0)), DIP),
    "chain17": (si.simple_cubic(17, 1, 1, periodic=(1, 0, 0)), DIP),
    "square5x3x2": (si.simple_cubic(5, 3, 2, periodic=(0, 0, 0)), DIP),
    "triangular24x20": (si.triangular(24, 20), DIP),
    "film32x32x4": (si.simple_cubic(32, 32, 4, periodic=(0, 0, 0)), DIP),
    "film33x31x3": (si.simple_cubic(33, 31, 3, periodic=(0, 0, 0)), DIP),
    "two_basis9x7x2": _two_basis(),
}


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_fft_dipole_gradient_matches_direct_sum(ora, case, precision):
    announce(f"fft dipole {case} {precision}")
    geo, ham = CASES[case]
    e, s = make_pair(ora, geo, ham, precision)
    n = si.uniform_sphere(geo.n_sites, 17)
    e.set_spins(n)
    got = e.dipole_gradient()
    ref = s.gradient(n)           # the Hamiltonian has only the dipole term
    if geo.n_sites == 1:
        assert np.all(got == 0.0)
        return
    assert_close(got, ref, precision, what=f"FFT dipole {case}")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fft_dipole_full_film_sampled_sites(ora, precision):
    """128 x 128 x 4 film (the dipolar workload) with a skyrmion texture:
    the FFT field on 512 sampled sites against the oracle's pair sums there."""
    announce(f"fft dipole film128x4 {precision}")
    w = si.WORKLOADS["film128x4_dipolar"]
    ham = dataclasses.replace(w.hamiltonian, ddi=SP_DDI_FFT)
    import paper_1901_11350_amd as pk

    e = pk.Engine(0, precision)
    e.set_geometry(w.geometry)
    e.set_hamiltonian(dataclasses.replace(ham, B=(0, 0, 0), K=(0.0,), J=(), D=()))
    n = si.skyrmion_ansatz(w.geometry, radius=12.0, noise_rad=0.1, seed=4)
    e.set_spins(n)
    got = e.dipole_gradient()
    s = ora.System(w.geometry, dataclasses.replace(ham, ddi=True))
    sites = np.random.default_rng(7).choice(w.geometry.n_sites, 512, replace=False)
    sites = np.concatenate([sites, [0, w.geometry.n_sites - 1]])   # corners of the film
    ref = s.dipole_gradient_sites(n, sites)
    assert_close(got[:, sites], ref, precision, what="FFT dipole film sampled")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fft_dipole_llg_trajectory(ora, precision):
    """Depondt steps with exchange, anisotropy, Zeeman and the FFT dipole
    field on a 20 x 16 x 2 film, against the oracle's direct-sum trajectory."""
    announce(f"fft dipole llg {precision}")
    geo = si.simple_cubic(20, 16, 2, periodic=(0, 0, 0))
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0.2), K=(0.2,), K_axis=((0, 0, 1),), J=(1.0,), ddi=SP_DDI_FFT)
    e, s = make_pair(ora, geo, ham, precision)
    n0 = si.skyrmion_ansatz(geo, radius=5.0, noise_rad=0.2, seed=3)
    e.set_spins(n0)
    e.run(0.3, 0.001, 10)
    ref, _ = s.run(n0, 0.3, 0.001, 10)
    assert_close(e.get_spins(), ref, precision, what="FFT dipole trajectory")


def test_fft_mode_rejects_oversized_lattice_and_keeps_the_state():
    import paper_1901_11350_amd as pk
    from paper_1901_11350_amd.engine import SpError

    e = pk.Engine(0, "f32")
    e.set_geometry(si.simple_cubic(600, 2, 1, periodic=(0, 0, 0)))
    plain = dataclasses.replace(DIP, ddi=0, J=(1.0,))
    e.set_hamiltonian(plain)
    e.set_spins(si.uniform_sphere(e.N, 3))
    E0, path0, n0 = e.energy(), e.step_path, e.get_spins()
    with pytest.raises(SpError):
        e.set_hamiltonian(DIP)
    assert e.energy() == E0 and e.step_path == path0
    assert np.array_equal(e.get_spins(), n0)
