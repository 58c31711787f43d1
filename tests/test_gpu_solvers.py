"""GPU Heun and SIB integrators (Appendices B, C) against the FP64 oracle:
trajectories on every step path they run on (compile-time-stencil tiles and
the two-pass kernels), with and without the thermal field, generic lattices
with a two-atom basis and the dipole term, plus the single-spin precession
in closed form."""

import dataclasses
import math

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, make_pair, need_gpu

pytestmark = pytest.mark.gpu

W = si.WORKLOADS
HAM0 = W["square32_fp64"].hamiltonian
HAM1 = W["triangular512_sllg"].hamiltonian
HAM2 = W["cubic128_bulkdmi"].hamiltonian
HAM4 = W["film128x4_dipolar"].hamiltonian
GAMMA = 0.176085963023
BASIS2_GEO = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0.5, 0.5, 0.5)),
                         (10, 9, 7), (1, 1, 0))
BASIS2_HAM = si.Hamiltonian(mu=(2.0, 3.0), B=(0.2, 0.4, -0.3), K=(0.1, -0.2),
                            K_axis=((0, 0, 1), (0.6, 0.8, 0.0)), J=(1.0, 0.5), D=(0.1, 0.05),
                            dmi_kind=si.DMI_BULK)

SHAPE_CASES = {
    "sq20x12_small": (si.square(20, 12), HAM0),
    "tri40x24_ragged": (si.triangular(40, 24), HAM1),
    "tri37x29_open": (si.triangular(37, 29, periodic=(0, 1, 0)), HAM1),
    "sq45x33_2shell_nodmi": (si.square(45, 33), dataclasses.replace(HAM0, J=(1.0, 0.3), D=())),
}
GENERIC_CASES = {
    "cubic12x10x8": (si.simple_cubic(12, 10, 8), HAM2),
    "basis2": (BASIS2_GEO, BASIS2_HAM),
    "film12x10x2_dipole": (si.simple_cubic(12, 10, 2, periodic=(0, 0, 0)), HAM4),
    "film12x10x2_fft_dipole": (si.simple_cubic(12, 10, 2, periodic=(0, 0, 0)), dataclasses.replace(HAM4, ddi=3)),
}
SHAPE_TILE = {"f32": "64x16x1024", "f64": "32x16x256"}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("solver", ["heun", "sib"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(SHAPE_CASES))
def test_solver_paths_match_oracle_stencil_lattices(ora, case, precision, solver):
    geo, ham = SHAPE_CASES[case]
    announce(f"{solver} {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path.startswith("shape2d")
    n0 = si.uniform_sphere(s.N, 31)
    n_ora, _ = s.run(n0, 0.3, 0.001, 4, T=25.0, seed=77, step0=5, solver=solver)
    for path in ["twopass", "fused2d", "shape2d/" + SHAPE_TILE[precision]]:
        e.step_path = path
        e.set_spins(n0)
        e.step = 5
        e.run(0.3, 0.001, 4, T=25.0, seed=77, solver=solver)
        assert_close(e.get_spins(), n_ora, precision, what=f"{solver} {path} {case}")


@pytest.mark.parametrize("solver", ["heun", "sib"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("T", [0.0, 40.0])
@pytest.mark.parametrize("case", sorted(GENERIC_CASES))
def test_solver_generic_lattices_match_oracle(ora, case, precision, T, solver):
    geo, ham = GENERIC_CASES[case]
    announce(f"{solver} {case} {precision} T={T}")
    e, s = make_pair(ora, geo, ham, precision)
    n0 = si.uniform_sphere(s.N, 23)
    e.set_spins(n0)
    e.run(0.3, 0.001, 3, T=T, seed=5, solver=solver)
    n_ora, _ = s.run(n0, 0.3, 0.001, 3, T=T, seed=5, solver=solver)
    assert_close(e.get_spins(), n_ora, precision, what=f"{solver} {case} [{e.step_path}]")


@pytest.mark.parametrize("solver", ["heun", "sib"])
def test_solver_long_trajectory_fp64(ora, solver):
    """square 32x32 FP64 (the FP64 workload's Hamiltonian), 300 steps."""
    announce(f"{solver} square32 300 steps")
    w = W["square32_fp64"]
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f64")
    n0 = si.uniform_sphere(s.N, w.init_seed)
    e.set_spins(n0)
    e.run(0.3, 0.001, 300, solver=solver)
    n_ora, _ = s.run(n0, 0.3, 0.001, 300, solver=solver)
    assert_close(e.get_spins(), n_ora, "f64", what=f"{solver} 300 steps")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("solver", ["heun", "sib"])
def test_undamped_precession_closed_form_gpu(solver, precision):
    import paper_1901_11350_amd as pk

    announce(f"{solver} precession {precision}")
    geo = si.Geometry(((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 0, 0),), (1, 1, 1), (0, 0, 0))
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 1.0), K=(0.0,), K_axis=((0, 0, 1),))
    e = pk.Engine(0, precision)
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    e.set_spins(np.array([[1.0], [0.0], [0.0]]))
    K, dt = 300, 0.01
    e.run(0.0, dt, K, solver=solver)
    n = e.get_spins()[:, 0]
    b = GAMMA * dt
    if solver == "sib":
        step = 2 * math.atan(b / 2)
    else:
        c = 1 / math.sqrt(1 + b * b)
        step = math.atan2(0.5 * b * (1 + c), 1 - 0.5 * b * b * c)
    tol = 1e-12 if precision == "f64" else 2e-5
    assert abs(n[0] - math.cos(K * step)) < tol and abs(n[1] - math.sin(K * step)) < tol
    assert abs(n[2]) < tol


def test_batches_reject_other_solvers():
    import ctypes

    import paper_1901_11350_amd as pk
    from paper_1901_11350_amd.engine import SpError, lib, sp_llg_params

    e = pk.Engine(0, "f32")
    e.set_geometry(si.square(32, 32))
    e.set_hamiltonian(HAM0)
    e.set_spins(si.uniform_sphere(e.N, 1))
    b = pk.Batch(0)
    p = sp_llg_params(0.3, 0.001, 0.0, 1, 0, 1)   # solver = Heun
    with pytest.raises(SpError):
        b._check(lib().sp_batch_add(b._h, e._h, ctypes.byref(p)))
    assert b.add(e, 0.3, 0.001) == 0


TILE_CASES = {
    "honeycomb41x19_4shell": (si.honeycomb(41, 19),
                              si.Hamiltonian(mu=(2.0, 2.5), B=(0.1, -0.2, 0.5), K=(0.1, 0.05),
                                             K_axis=((0, 0, 1), (0.6, 0.0, 0.8)), J=(1.0, 0.2, -0.1, 0.05),
                                             D=(0.15,))),
    "kagome24x19_open": (si.kagome(24, 19, periodic=(1, 0, 0)),
                         si.Hamiltonian(mu=(2.0, 2.0, 3.0), B=(0.0, 0.0, 0.4), K=(0.1, 0.1, 0.2),
                                        K_axis=((0, 0, 1),) * 3, J=(1.0, -0.2, 0.1), D=(0.1,))),
    "basis2": (BASIS2_GEO, BASIS2_HAM),
}


@pytest.mark.parametrize("solver", ["heun", "sib"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(TILE_CASES))
def test_solver_fused_tile_matches_oracle(ora, case, precision, solver):
    """Heun and SIB on the fused tile path of lattices with a basis (and on
    the two-pass kernels) against the oracle's 4-step stochastic trajectory."""
    geo, ham = TILE_CASES[case]
    announce(f"{solver} fused tile {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path == "fusedtile"
    n0 = si.uniform_sphere(s.N, 31)
    n_ora, _ = s.run(n0, 0.3, 0.001, 4, T=25.0, seed=77, step0=5, solver=solver)
    for path in ["fusedtile", "twopass"]:
        e.step_path = path
        e.set_spins(n0)
        e.step = 5
        e.run(0.3, 0.001, 4, T=25.0, seed=77, solver=solver)
        assert_close(e.get_spins(), n_ora, precision, what=f"{solver} {path} {case}")
