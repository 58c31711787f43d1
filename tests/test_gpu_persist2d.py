"""GPU tests of the persistent 2D step path (persist2d): many Depondt steps
per launch, tiles synchronised through neighbour flags, against the FP64
oracle and against the one-launch-per-step kernel of the same tile.

Cases cover every compile-time stencil family, DMI on and off, open edges,
lattices of one tile row (a tile is its own neighbour), odd step counts
(the result ends in the other spin buffer), observation intervals that split
a run into several launches, the full 512 x 512 triangular workload, and
the time-out error path forced from the host (tiny spin limit)."""

import dataclasses
import os

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import TOL, announce, assert_close, make_pair, need_gpu, rel_err

pytestmark = pytest.mark.gpu

W = si.WORKLOADS
HAM0 = W["square32_fp64"].hamiltonian
HAM1 = W["triangular512_sllg"].hamiltonian

CASES = {
    "tri128x64": (si.triangular(128, 64), HAM1),
    "tri128x64_open_a": (si.triangular(128, 64, periodic=(0, 1, 0)), HAM1),
    "tri64x32_nodmi": (si.triangular(64, 32), dataclasses.replace(HAM1, D=())),
    "tri64x16_one_row": (si.triangular(64, 16), HAM1),
    "sq64x64": (si.square(64, 64), HAM0),
    "sq64x32_2shell_open": (si.square(64, 32, periodic=(0, 0, 0)), dataclasses.replace(HAM0, J=(1.0, 0.3), D=())),
    "sq32x32_3shell": (si.square(32, 32), dataclasses.replace(HAM0, J=(1.0, 0.3, -0.1))),
}
CFGS = {"f32": [(64, 16), (32, 32), (32, 16)], "f64": [(32, 16)]}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _cfgs(geo, precision):
    return [f"{tx}x{ty}" for tx, ty in CFGS[precision] if geo.n_cells[0] % tx == 0 and geo.n_cells[1] % ty == 0]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_persist_matches_oracle_and_one_step_kernel(ora, case, precision):
    geo, ham = CASES[case]
    cfgs = _cfgs(geo, precision)
    if not cfgs:
        pytest.skip("no persistent tile divides this lattice")
    announce(f"persist2d {case} {precision} {cfgs}")
    e, s = make_pair(ora, geo, ham, precision)
    n0 = si.uniform_sphere(s.N, 41)
    # 7 steps observed every 3: launches of 3, 3 and 1 steps
    n_ora, obs_o = s.run(n0, 0.3, 0.001, 7, T=25.0, seed=123, step0=9, observe_every=3)
    for cfg in cfgs:
        e.step_path = "persist2d/" + cfg
        assert e.step_path == "persist2d/" + cfg
        e.set_spins(n0)
        e.step = 9
        obs = e.run(0.3, 0.001, 7, T=25.0, seed=123, observe_every=3)
        assert e.step == 16
        got = e.get_spins()
        assert_close(got, n_ora, precision, what=f"persist2d/{cfg} {case}")
        assert [o["step"] for o in obs] == [o["step"] for o in obs_o]
        for a, b in zip(obs, obs_o):
            assert a["E"] == pytest.approx(b["E"], rel=10 * TOL[precision], abs=10 * TOL[precision] * s.N)
        # the one-step kernel of the same tile
        e.step_path = "shape2d/" + cfg + ("x256" if precision == "f64" else "x" + str(_threads(cfg)))
        e.set_spins(n0)
        e.step = 9
        e.run(0.3, 0.001, 7, T=25.0, seed=123)
        assert rel_err(got, e.get_spins()) <= 2 * TOL[precision]


def _threads(cfg):
    tx, ty = (int(v) for v in cfg.split("x"))
    return tx * ty


def test_persist_full_triangular512_two_thermal_steps(ora):
    """The 512 x 512 triangular workload on its benchmark configuration:
    every site of two stochastic steps against the oracle."""
    announce("persist2d triangular512 full")
    w = W["triangular512_sllg"]
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    e.step_path = "persist2d/64x16"
    n0 = si.uniform_sphere(s.N, w.init_seed)
    d = w.dynamics
    e.set_spins(n0)
    e.run(d.alpha, d.dt, 2, T=d.T, seed=d.seed)
    n_ora, _ = s.run(n0, d.alpha, d.dt, 2, T=d.T, seed=d.seed)
    assert_close(e.get_spins(), n_ora, "f32", what="persist2d triangular512")


def test_persist_long_trajectory_fp32(ora):
    """The triangular workload's dynamics (stochastic, T = 10 K) on a
    128 x 64 patch for 1000 steps in launches of 100, observations between:
    within 1e-5 of the oracle, as the one-step kernel is over this horizon."""
    announce("persist2d tri128x64 1000 steps")
    w = W["triangular512_sllg"]
    geo = w.geometry.with_cells((128, 64, 1))
    e, s = make_pair(ora, geo, w.hamiltonian, "f32")
    e.step_path = "persist2d/64x16"
    n0 = si.uniform_sphere(s.N, w.init_seed)
    d = w.dynamics
    e.set_spins(n0)
    obs = e.run(d.alpha, d.dt, 1000, T=d.T, seed=d.seed, observe_every=100)
    n_ora, obs_o = s.run(n0, d.alpha, d.dt, 1000, T=d.T, seed=d.seed, observe_every=100)
    assert_close(e.get_spins(), n_ora, "f32", what="persist2d 1000 steps")
    for a, b in zip(obs, obs_o):
        assert a["step"] == b["step"]
        assert a["E"] == pytest.approx(b["E"], rel=1e-5)


@pytest.mark.parametrize("solver", ["heun", "sib"])
def test_persist_path_other_solvers_step_one_launch_at_a_time(ora, solver):
    announce(f"persist2d path {solver}")
    geo, ham = CASES["tri64x32_nodmi"]
    e, s = make_pair(ora, geo, ham, "f32")
    e.step_path = "persist2d/32x16"
    n0 = si.uniform_sphere(s.N, 8)
    e.set_spins(n0)
    e.run(0.3, 0.001, 3, T=25.0, seed=4, solver=solver)
    n_ora, _ = s.run(n0, 0.3, 0.001, 3, T=25.0, seed=4, solver=solver)
    assert_close(e.get_spins(), n_ora, "f32", what=f"persist2d path {solver}")


def test_persist_rejects_unfit_lattices_and_tiles():
    import paper_1901_11350_amd as pk
    from paper_1901_11350_amd.engine import SpError

    announce("persist2d rejections")
    e = pk.Engine(0, "f32")
    e.set_geometry(si.triangular(40, 24))          # not a multiple of any tile
    e.set_hamiltonian(HAM1)
    keep = e.step_path
    with pytest.raises(SpError):
        e.step_path = "persist2d"
    assert e.step_path == keep
    e64 = pk.Engine(0, "f64")
    e64.set_geometry(si.square(64, 64))
    e64.set_hamiltonian(HAM0)
    with pytest.raises(SpError):
        e64.step_path = "persist2d/64x16"          # FP64 takes 32x16 only
    e64.step_path = "persist2d/32x16"
    with pytest.raises(SpError):
        e64.step_path = "persist2d/17x3"
    eb = pk.Engine(0, "f32")                        # generic lattice: no compile-time stencil
    eb.set_geometry(si.simple_cubic(64, 16, 2))
    eb.set_hamiltonian(W["cubic128_bulkdmi"].hamiltonian)
    with pytest.raises(SpError):
        eb.step_path = "persist2d"


def test_persist_timeout_path_reports_and_recovers(ora):
    """With a spin limit of zero a tile whose neighbours are not done at its
    first poll gives up: the run either completes or reports the time-out;
    the next run (normal limit) is again exact."""
    announce("persist2d forced time-out")
    geo, ham = CASES["tri128x64"]
    e, s = make_pair(ora, geo, ham, "f32")
    e.step_path = "persist2d/32x16"
    n0 = si.uniform_sphere(s.N, 77)
    os.environ["SP_PERSIST_SPIN_LIMIT"] = "0"
    try:
        e.set_spins(n0)
        _, rc = e.run(0.3, 0.001, 200, T=10.0, seed=3, check=False)
    finally:
        del os.environ["SP_PERSIST_SPIN_LIMIT"]
    if rc != 0:
        from paper_1901_11350_amd.engine import lib

        assert "timed out" in lib().sp_last_error(e._h).decode()
    announce(f"persist2d forced time-out rc={rc}")
    e.set_spins(n0)
    e.step = 0
    e.run(0.3, 0.001, 5, T=10.0, seed=3)
    n_ora, _ = s.run(n0, 0.3, 0.001, 5, T=10.0, seed=3)
    assert_close(e.get_spins(), n_ora, "f32", what="after a forced time-out")
