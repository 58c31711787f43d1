"""GPU tests of explicit pair interactions (sp_set_pairs) against the FP64
oracle with the same pair list: gradients, energies and stochastic Depondt
trajectories for long-range wrapping pairs, direction-dependent exchange,
arbitrary DMI vectors, a two-atom 3D basis and open edges; the shell table
written as pairs against the shell-built engine; rejected lists; and
sp_set_hamiltonian discarding the pairs."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import TOL, announce, assert_close, make_pair, need_gpu, rel_err

pytestmark = pytest.mark.gpu

HAM = si.Hamiltonian(mu=(2.0,), B=(0.1, -0.3, 0.8), K=(0.2,), K_axis=((0, 0, 1),))
LONG = [
    (0, 0, (1, 0, 0), 1.0, (0.1, -0.2, 0.3)),
    (0, 0, (0, 1, 0), 0.4, (0.0, 0.0, 0.0)),
    (0, 0, (2, -1, 0), -0.3, (0.05, 0.02, -0.1)),
    (0, 0, (27, 0, 0), 0.2, (0.0, 0.3, 0.0)),      # wraps past a 24-cell periodic axis
    (0, 0, (5, 9, 0), 0.15, (0.0, 0.0, 0.2)),
    (0, 0, (0, 20, 0), -0.1, (0.0, 0.0, 0.0)),     # onto the site itself on a 20-cell axis: dropped
]
SHORT = [
    (0, 0, (1, 0, 0), 1.0, (0.1, -0.2, 0.0)),
    (0, 0, (0, 1, 0), 0.6, (0.2, 0.1, 0.0)),
    (0, 0, (1, -1, 0), 0.8, (0.0, 0.0, 0.05)),
    (0, 0, (2, 0, 0), -0.2, (0.0, 0.0, 0.0)),
    (0, 0, (1, 1, 0), 0.1, (0.0, 0.1, 0.0)),
]
BASIS2_GEO = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0.3, 0.4, 0.5)),
                         (9, 7, 5), (1, 1, 0))
BASIS2_HAM = si.Hamiltonian(mu=(2.0, 1.5), B=(0.2, 0.1, 0.5), K=(0.1, 0.3), K_axis=((0, 0, 1), (1, 0, 0)))
BASIS2 = [(0, 1, (0, 0, 0), 0.8, (0.1, 0.0, -0.2)),
          (1, 0, (1, 0, 0), 0.3, (0.0, 0.2, 0.0)),
          (0, 0, (3, 1, 1), -0.2, (0.05, 0.05, 0.05)),
          (1, 1, (0, 2, -1), 0.5, (0.0, 0.0, 0.0)),
          (0, 1, (-5, 0, 1), 0.1, (0.2, -0.1, 0.0))]

CASES = {
    "long_range_tri24x20": (si.triangular(24, 20), HAM, LONG),
    "long_range_tri24x20_open_b": (si.triangular(24, 20, periodic=(1, 0, 0)), HAM, LONG),
    "short_range_tri40x24": (si.triangular(40, 24), HAM, SHORT),
    "basis2_9x7x5": (BASIS2_GEO, BASIS2_HAM, BASIS2),
}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _pair(ora, case, precision):
    geo, ham, pairs = CASES[case]
    e, s = make_pair(ora, geo, ham, precision)
    e.set_pairs(pairs)
    s.set_pairs(pairs)
    return e, s


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_pairs_gradient_and_energy_match_oracle(ora, case, precision):
    announce(f"pairs gradient {case} {precision}")
    e, s = _pair(ora, case, precision)
    n = si.uniform_sphere(s.N, 19)
    e.set_spins(n)
    assert_close(e.gradient(), s.gradient(n), precision, what=f"pairs gradient {case}")
    E = e.energy()
    assert E == pytest.approx(s.energy(n), rel=10 * TOL[precision], abs=10 * TOL[precision] * s.N)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_pairs_trajectory_matches_oracle_on_every_path(ora, case, precision):
    announce(f"pairs trajectory {case} {precision}")
    e, s = _pair(ora, case, precision)
    assert not e.step_path.startswith(("shape", "persist"))
    n0 = si.uniform_sphere(s.N, 7)
    ref, _ = s.run(n0, 0.3, 0.001, 4, T=20.0, seed=5, step0=3)
    paths = ["twopass"] + ([e.step_path] if e.step_path in ("fused2d", "fusedtile") else [])
    for path in paths:
        e.step_path = path
        e.set_spins(n0)
        e.step = 3
        e.run(0.3, 0.001, 4, T=20.0, seed=5)
        assert_close(e.get_spins(), ref, precision, what=f"pairs {path} {case}")


def test_short_pairs_take_the_runtime_stencil_path(ora):
    from paper_1901_11350_amd.engine import SpError

    e, _ = _pair(ora, "short_range_tri40x24", "f32")
    assert e.step_path == "fused2d"
    with pytest.raises(SpError):
        e.step_path = "shape2d"
    with pytest.raises(SpError):
        e.step_path = "persist2d"


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_shell_table_as_pairs_matches_shell_engine(ora, precision):
    """The 512^2 workload's Hamiltonian on a 64 x 48 patch: its shell bonds
    written as unique pairs give the shell engine's gradient and trajectory."""
    announce(f"pairs shell equivalence {precision}")
    w = si.WORKLOADS["triangular512_sllg"]
    geo = w.geometry.with_cells((64, 48, 1))
    a, s = make_pair(ora, geo, w.hamiltonian, precision)
    table = {(b[0], b[1], b[2], b[3], b[4]): b for b in s.bonds()}
    pairs = [(b[0], b[1], (b[2], b[3], b[4]), b[6], b[7]) for k, b in table.items()
             if k < (b[1], b[0], -b[2], -b[3], -b[4])]
    b_eng, _ = make_pair(ora, geo, dataclasses.replace(w.hamiltonian, J=(), D=()), precision)
    b_eng.set_pairs(pairs)
    n0 = si.uniform_sphere(s.N, 4)
    a.set_spins(n0)
    b_eng.set_spins(n0)
    assert rel_err(b_eng.gradient(), a.gradient()) <= 2 * TOL[precision]
    d = w.dynamics
    a.run(d.alpha, d.dt, 20, T=d.T, seed=d.seed)
    b_eng.run(d.alpha, d.dt, 20, T=d.T, seed=d.seed)
    assert a.step_path.startswith("shape2d") and b_eng.step_path == "fused2d"
    assert rel_err(b_eng.get_spins(), a.get_spins()) <= 4 * TOL[precision]


def test_rejected_pair_lists_leave_the_engine_unchanged(ora):
    from paper_1901_11350_amd.engine import SpError

    announce("pairs rejections")
    e, s = _pair(ora, "short_range_tri40x24", "f64")
    n = si.uniform_sphere(s.N, 2)
    e.set_spins(n)
    E0, path0 = e.energy(), e.step_path
    bad_lists = [
        [(0, 0, (0, 0, 0), 1.0, (0, 0, 0))],                                    # self pair
        [(0, 1, (1, 0, 0), 1.0, (0, 0, 0))],                                    # basis index
        [(0, 0, (1, 0, 0), 1.0, (0, 0, 0)), (0, 0, (1, 0, 0), 0.5, (0, 0, 0))],   # repeated
        [(0, 0, (1, 0, 0), 1.0, (0, 0, 0)), (0, 0, (-1, 0, 0), 0.5, (0, 0, 0))],  # reverse
        [(0, 0, (65, 0, 0), 1.0, (0, 0, 0))],                                   # offset beyond 64
        [(0, 0, (1, 0, 0), float("nan"), (0, 0, 0))],                           # non-finite
        [(0, 0, (k, 0, 0), 0.1, (0, 0, 0)) for k in range(1, 64)] +
        [(0, 0, (k, 1, 0), 0.1, (0, 0, 0)) for k in range(-64, 2)],             # > 256 bonds
    ]
    for bad in bad_lists:
        with pytest.raises(SpError):
            e.set_pairs(bad)
        assert e.energy() == E0 and e.step_path == path0
    e.set_pairs([])                       # no exchange / DMI left
    assert e.energy() == pytest.approx(ora.System(si.triangular(40, 24), HAM).energy(n), rel=1e-12)


def test_set_hamiltonian_discards_pairs(ora):
    announce("pairs discarded")
    w = si.WORKLOADS["triangular512_sllg"]
    geo = w.geometry.with_cells((64, 32, 1))
    e, s = make_pair(ora, geo, w.hamiltonian, "f64")
    n = si.uniform_sphere(s.N, 8)
    e.set_spins(n)
    e.set_pairs(SHORT)
    assert e.step_path == "fused2d"
    e.set_hamiltonian(w.hamiltonian)
    assert e.step_path.startswith("shape2d")
    assert_close(e.gradient(), s.gradient(n), "f64", what="after sp_set_hamiltonian")
