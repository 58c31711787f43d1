"""GPU parity: the HIP engine (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bar: max|engine - oracle| <= tol * max|oracle| with tol = 1e-12 for the
FP64 engine and 1e-5 for the FP32 engine (gradients, fields, spins);
Philox integers bit-exact.  Sizes span several tiles and ragged tails; the
full benchmark sizes are checked too.
"""

import dataclasses
import math

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import TOL, announce, assert_close, make_pair, need_gpu, rel_err

pytestmark = pytest.mark.gpu

W = si.WORKLOADS
HAM0 = W["square32_fp64"].hamiltonian
HAM1 = W["triangular512_sllg"].hamiltonian
HAM2 = W["cubic128_bulkdmi"].hamiltonian
HAM4 = W["film128x4_dipolar"].hamiltonian
BASIS2_GEO = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0.5, 0.5, 0.5)),
                         (10, 9, 7), (1, 1, 0))
BASIS2_HAM = si.Hamiltonian(mu=(2.0, 3.0), B=(0.2, 0.4, -0.3), K=(0.1, -0.2),
                            K_axis=((0, 0, 1), (0.6, 0.8, 0.0)), J=(1.0, 0.5), D=(0.1, 0.05),
                            dmi_kind=si.DMI_BULK)

HC_HAM = si.Hamiltonian(mu=(2.0, 2.5), B=(0.1, -0.2, 0.5), K=(0.1, 0.05),
                        K_axis=((0, 0, 1), (0.6, 0.0, 0.8)), J=(1.0, 0.2, -0.1), D=(0.15,))
KG_HAM = si.Hamiltonian(mu=(2.0, 2.0, 3.0), B=(0.0, 0.0, 0.4), K=(0.1, 0.1, 0.2),
                        K_axis=((0, 0, 1), (0, 0, 1), (0, 0, 1)), J=(1.0, -0.2, 0.1), D=(0.1,))
# the square lattice of spacing 1/2 written as a four-atom cell of spacing 1
SQ4_GEO = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)),
                      ((0, 0, 0), (0.5, 0, 0), (0, 0.5, 0), (0.5, 0.5, 0)), (16, 12, 1), (1, 1, 0))
SQ4_HAM = si.Hamiltonian(mu=(2.0,) * 4, B=(0.0, 0.0, 1.0), K=(0.1,) * 4, K_axis=((0, 0, 1),) * 4,
                         J=(1.0, 0.3), D=(0.3,))

CASES = {
    "square32": (W["square32_fp64"].geometry, HAM0),
    "honeycomb37x22": (si.honeycomb(37, 22), HC_HAM),
    "kagome24x19_open": (si.kagome(24, 19, periodic=(1, 0, 0)), KG_HAM),
    "square2x2": (si.square(2, 2), HAM0),
    "tri40x24_ragged": (si.triangular(40, 24), HAM1),
    "tri37x29_open": (si.triangular(37, 29, periodic=(0, 1, 0)), HAM1),
    "cubic12x10x8": (si.simple_cubic(12, 10, 8), HAM2),
    "basis2": (BASIS2_GEO, BASIS2_HAM),
    "film12x10x2_dipole": (si.simple_cubic(12, 10, 2, periodic=(0, 0, 0)), HAM4),
}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("case", sorted(CASES))
def test_bond_table_matches_oracle(ora, case):
    geo, ham = CASES[case]
    announce(f"bonds {case}")
    e, s = make_pair(ora, geo, ham, "f64")
    for beta in range(geo.n_basis):
        eb = {(int(r[0]), int(r[1]), int(r[2]), int(r[3]), int(r[4])): (r[5], tuple(r[6:9]))
              for r in e.bonds(beta)}
        ob = {(b[1], b[2], b[3], b[4], b[5]): (b[6], b[7]) for b in s.bonds()
              if b[0] == beta and (b[6] != 0.0 or any(b[7]))}
        assert set(eb) == set(ob)
        for k in eb:
            assert eb[k][0] == pytest.approx(ob[k][0], abs=1e-15)
            assert np.allclose(eb[k][1], ob[k][1], atol=1e-15)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_gradient_parity(ora, case, precision):
    geo, ham = CASES[case]
    announce(f"gradient {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    n = si.uniform_sphere(s.N, 17)
    e.set_spins(n)
    assert_close(e.gradient(), s.gradient(n), precision, what=f"gradient {case}")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_energy_parity(ora, case, precision):
    geo, ham = CASES[case]
    announce(f"energy {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    n = si.uniform_sphere(s.N, 19)
    e.set_spins(n)
    E, per = e.energy(per_term=True)
    Eo, per_o = s.energy(n, per_term=True)
    scale = np.abs(per_o).sum()
    tol = TOL[precision]
    assert abs(E - Eo) <= tol * scale
    assert np.abs(per - per_o).max() <= tol * scale
    obs = e.observe()
    oo = s.observe(n)
    assert obs["max_torque"] == pytest.approx(oo["max_torque"], rel=10 * tol)
    assert np.allclose(obs["M"], oo["M"], atol=10 * tol)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(200, 70), (2048, 1024)])
def test_observation_on_stencil_tiles_matches_oracle(ora, dims, precision):
    """Energy per term, largest torque, mean spin and norm deviation formed on
    the stencil path's tiles: 4 x 5 tiles with ragged edges, and 2,048 tiles
    (more than the partial rows, so each workgroup folds several tiles)
    against the oracle, and against the generic observation kernel of the
    same lattice with its bonds given as explicit pairs."""
    announce(f"observation on tiles {dims} {precision}")
    w = W["triangular512_sllg"]
    geo = w.geometry.with_cells((dims[0], dims[1], 1))
    e, s = make_pair(ora, geo, w.hamiltonian, precision)
    assert e.step_path.startswith("shape2d")
    n = si.uniform_sphere(s.N, 29)
    e.set_spins(n)
    obs = e.observe()
    oo = s.observe(n)
    tol = TOL[precision]
    scale = np.abs(oo["per_term"]).sum()
    assert np.abs(np.array(obs["per_term"]) - np.array(oo["per_term"])).max() <= tol * scale
    assert obs["E"] == pytest.approx(oo["E"], rel=tol, abs=tol * scale)
    assert obs["max_torque"] == pytest.approx(oo["max_torque"], rel=10 * tol)
    assert np.allclose(obs["M"], oo["M"], atol=10 * tol)
    if precision == "f64":
        assert obs["max_norm_dev"] == pytest.approx(oo["max_norm_dev"], abs=1e-14)
    else:
        assert obs["max_norm_dev"] < 1e-6
    table = {(b[0], b[1], b[2], b[3], b[4]): b for b in s.bonds()}
    pairs = [(b[0], b[1], (b[2], b[3], b[4]), b[6], b[7]) for k, b in table.items()
             if k < (b[1], b[0], -b[2], -b[3], -b[4])]
    g, _ = make_pair(ora, geo, dataclasses.replace(w.hamiltonian, J=(), D=()), precision)
    g.set_pairs(pairs)
    assert g.step_path == "fused2d"
    g.set_spins(n)
    og = g.observe()
    assert np.abs(np.array(obs["per_term"]) - np.array(og["per_term"])).max() <= 2 * tol * scale
    assert obs["max_torque"] == pytest.approx(og["max_torque"], rel=10 * tol)


def _step_case(ora, case, precision, T, steps, path=None, seed=99, alpha=0.3, dt=0.001):
    geo, ham = CASES[case]
    e, s = make_pair(ora, geo, ham, precision)
    if path:
        e.step_path = path
    n0 = si.uniform_sphere(s.N, 23)
    e.set_spins(n0)
    e.step = 5
    e.run(alpha, dt, steps, T=T, seed=seed)
    n_ora, _ = s.run(n0, alpha, dt, steps, T=T, seed=seed, step0=5)
    return e, s, e.get_spins(), n_ora


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("T", [0.0, 40.0])
@pytest.mark.parametrize("case", sorted(CASES))
def test_depondt_steps_parity(ora, case, precision, T):
    announce(f"depondt {case} {precision} T={T}")
    e, s, n_gpu, n_ora = _step_case(ora, case, precision, T, steps=3)
    assert_close(n_gpu, n_ora, precision, what=f"3 steps {case} [{e.step_path}]")
    assert e.step == 8


PATH_CASES = {
    "square32": (W["square32_fp64"].geometry, HAM0),
    "tri40x24_ragged": (si.triangular(40, 24), HAM1),
    "tri37x29_open": (si.triangular(37, 29, periodic=(0, 1, 0)), HAM1),
    "sq45x33_2shell_nodmi": (si.square(45, 33), dataclasses.replace(HAM0, J=(1.0, 0.3), D=())),
    "sq40x36_3shell_open": (si.square(40, 36, periodic=(1, 0, 0)), dataclasses.replace(HAM0, J=(1.0, 0.3, -0.1))),
    "tri50x20_1shell": (si.triangular(50, 20), dataclasses.replace(HAM1, J=(1.0,), D=(0.2,))),
    "tri66x34_2shell_bulk": (si.triangular(66, 34), dataclasses.replace(HAM1, J=(1.0, -0.3), D=(0.25,),
                                                                        dmi_kind=si.DMI_BULK)),
    # periodic lattices narrower than half a 64-wide tile plus halo: the
    # staged coordinates wrap more than once
    "sq20x12_small": (si.square(20, 12), HAM0),
    "tri24x20_small": (si.triangular(24, 20), HAM1),
}
SHAPE_CFGS = {"f32": ["32x16x256", "64x16x512", "32x16x512", "32x32x1024", "64x16x1024", "32x32x512",
                      "64x16x256"],
              "f64": ["32x16x256"]}


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(PATH_CASES))
def test_every_step_path_agrees_with_oracle(ora, case, precision):
    """Every step path and tile configuration the lattice allows gives the
    oracle's 4-step stochastic trajectory (ragged tiles, open edges)."""
    geo, ham = PATH_CASES[case]
    announce(f"paths {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path.startswith("shape2d"), e.step_path
    n0 = si.uniform_sphere(s.N, 23)
    n_ora, _ = s.run(n0, 0.3, 0.001, 4, T=25.0, seed=99, step0=5)
    res = {}
    for path in ["twopass", "fused2d"] + ["shape2d/" + c for c in SHAPE_CFGS[precision]]:
        e.step_path = path
        assert e.step_path == path
        e.set_spins(n0)
        e.step = 5
        e.run(0.3, 0.001, 4, T=25.0, seed=99)
        res[path] = e.get_spins()
        assert_close(res[path], n_ora, precision, what=f"{path} {case}")
    for path in res:
        assert rel_err(res[path], res["twopass"]) <= 2 * TOL[precision]


def test_autotune_restores_state_and_picks_a_path(ora):
    import paper_1901_11350_amd as pk

    announce("autotune")
    w = W["triangular512_sllg"]
    e = pk.engine_for(w)
    n0 = si.uniform_sphere(e.N, 1)
    e.set_spins(n0)
    e.step = 17
    before = e.get_spins()
    ms = e.autotune(w.dynamics.alpha, w.dynamics.dt, w.dynamics.T, w.dynamics.seed, n_steps=20)
    assert ms > 0
    assert e.step == 17
    assert np.array_equal(e.get_spins(), before)
    assert e.step_path in (["twopass", "fused2d"] + ["shape2d/" + c for c in SHAPE_CFGS["f32"]] +
                           ["persist2d/" + c for c in ("64x16", "32x32", "32x16")])
    announce(f"autotune picked {e.step_path} at {ms:.4f} ms/step")


def test_trajectory_square32_fp64_1000_steps(ora):
    """The FP64 workload: 1000 Depondt steps at T = 0 within 1e-12 of the oracle."""
    w = W["square32_fp64"]
    announce("trajectory square32 fp64 1000")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f64")
    n0 = si.uniform_sphere(s.N, w.init_seed)
    e.set_spins(n0)
    d = w.dynamics
    obs = e.run(d.alpha, d.dt, d.n_steps, T=d.T, seed=d.seed, observe_every=d.observe_every)
    n_ora, obs_o = s.run(n0, d.alpha, d.dt, d.n_steps, T=d.T, seed=d.seed,
                         observe_every=d.observe_every)
    assert_close(e.get_spins(), n_ora, "f64", what="1000 steps")
    for a, b in zip(obs, obs_o):
        assert a["step"] == b["step"]
        assert a["E"] == pytest.approx(b["E"], rel=1e-12)
    E = [o["E"] for o in obs]
    assert all(E[k + 1] <= E[k] for k in range(len(E) - 1))


@pytest.mark.parametrize("name,shape,steps", [
    ("triangular512_sllg", (64, 48, 1), 1000),
    ("square32_fp64", (32, 32, 1), 1000),
    ("cubic128_bulkdmi", (16, 12, 10), 300),
])
def test_trajectory_fp32_within_1e5(ora, name, shape, steps):
    """FP32 engine follows the FP64 oracle within 1e-5 over the measured
    horizon (perturbations of 1e-7 stay below 1e-5 for these step counts)."""
    w = W[name]
    announce(f"trajectory fp32 {name} {shape} {steps}")
    geo = w.geometry.with_cells(shape)
    e, s = make_pair(ora, geo, w.hamiltonian, "f32")
    n0 = si.uniform_sphere(s.N, w.init_seed)
    e.set_spins(n0)
    d = w.dynamics
    e.run(d.alpha, d.dt, steps, T=d.T, seed=d.seed)
    n_ora, _ = s.run(n0, d.alpha, d.dt, steps, T=d.T, seed=d.seed)
    assert_close(e.get_spins(), n_ora, "f32", what=f"{steps} steps")


def test_full_size_triangular512_steps(ora):
    """Benchmark workload at full size: 10 stochastic steps, every site."""
    w = W["triangular512_sllg"]
    announce("full triangular512 10 steps")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    assert e.step_path.startswith("shape2d")
    n0 = si.uniform_sphere(s.N, w.init_seed)
    e.set_spins(n0)
    d = w.dynamics
    assert_close(e.gradient(), s.gradient(n0), "f32", what="gradient")
    obs = e.run(d.alpha, d.dt, 10, T=d.T, seed=d.seed, observe_every=5)
    n_ora, obs_o = s.run(n0, d.alpha, d.dt, 10, T=d.T, seed=d.seed, observe_every=5)
    assert_close(e.get_spins(), n_ora, "f32", what="10 steps")
    for a, b in zip(obs, obs_o):
        assert a["E"] == pytest.approx(b["E"], rel=1e-5)


def test_full_size_cubic128_step(ora):
    w = W["cubic128_bulkdmi"]
    announce("full cubic128 1 step")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    n0 = si.conical_helix(w.geometry, seed=w.init_seed)
    e.set_spins(n0)
    d = w.dynamics
    assert_close(e.gradient(), s.gradient(n0), "f32", what="gradient")
    e.run(d.alpha, d.dt, 1)
    n_ora, _ = s.run(n0, d.alpha, d.dt, 1)
    assert_close(e.get_spins(), n_ora, "f32", what="1 step")


def test_full_size_dipole_film_sampled(ora):
    """128x128x4 dipolar film: the direct-sum dipole gradient at 192 sampled
    sites (every edge, corner and face class included) against the oracle's
    per-site direct sum; local terms at every site."""
    w = W["film128x4_dipolar"]
    announce("full film128x4 dipole sampled")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    n0 = si.skyrmion_ansatz(w.geometry, radius=12.0, noise_rad=0.3, seed=w.init_seed)
    e.set_spins(n0)
    gdd = e.dipole_gradient()
    rng = np.random.default_rng(5)
    N = s.N
    corners = [0, 127, 127 * 128, 128 * 128 - 1, N - 1, N - 128]
    sites = np.unique(np.concatenate([corners, rng.integers(0, N, 186)]))
    ref = s.dipole_gradient_sites(n0, sites)
    assert_close(gdd[:, sites], ref, "f32", what="dipole sampled")
    local = dataclasses.replace(w.hamiltonian, ddi=False)
    e2, s2 = make_pair(ora, w.geometry, local, "f32")
    e2.set_spins(n0)
    assert_close(e2.gradient(), s2.gradient(n0), "f32", what="local terms")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_philox_bits_and_normals(ora, precision):
    import paper_1901_11350_amd as pk

    announce(f"philox {precision}")
    e = pk.Engine(0, precision)
    for seed, step, replica, site0 in [(11351, 0, 0, 0), (2**40 + 7, 2**33 + 5, 3, 1000)]:
        eta, raw = e.thermal_normals(seed, step, site0, 4096, replica=replica)
        for i in range(0, 4096, 97):
            ctr = [site0 + i, step & 0xFFFFFFFF, step >> 32, replica]
            assert list(raw[i]) == ora.philox4x32_10(ctr, [seed & 0xFFFFFFFF, seed >> 32])
            ref = ora.thermal_normals(seed, step, site0 + i, replica)
            tol = 1e-13 if precision == "f64" else 2e-5 * max(1.0, np.abs(ref).max())
            assert np.abs(eta[:, i] - ref).max() <= tol


def test_invariants_norm_and_energy_fp32(ora):
    w = W["square32_fp64"]
    announce("invariants fp32")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    e.set_spins(si.uniform_sphere(s.N, 3))
    obs = e.run(0.3, 0.001, 2000, observe_every=100)
    assert max(o["max_norm_dev"] for o in obs) < 2e-6
    E = [o["E"] for o in obs]
    assert all(E[k + 1] <= E[k] + 1e-6 * abs(E[k]) for k in range(len(E) - 1))


def test_nonfinite_state_is_reported(ora):
    import torch
    import paper_1901_11350_amd as pk

    w = W["square32_fp64"]
    announce("nonfinite detection")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    bad = si.uniform_sphere(s.N, 3)
    bad[0, 5] = np.nan
    with pytest.raises(pk.SpError) as ei:
        e.set_spins(bad)
    assert ei.value.code == pk.SP_E_ARG
    t = torch.tensor(bad, dtype=torch.float32, device="cuda").contiguous()
    torch.cuda.synchronize()
    e.set_spins_dev(t)
    obs, rc = e.run(0.3, 0.001, 20, observe_every=5, check=False)
    assert rc == pk.SP_E_NONFINITE
    assert math.isnan(obs[0]["max_torque"])


def test_call_order_errors(ora):
    import paper_1901_11350_amd as pk

    announce("call order")
    e = pk.Engine(0, "f32")
    with pytest.raises(pk.SpError) as ei:
        e.llg_step(0.1, 0.001)
    assert ei.value.code == pk.SP_E_ORDER
    e.set_geometry(si.square(8, 8))
    with pytest.raises(pk.SpError) as ei:
        e.set_hamiltonian(dataclasses.replace(HAM0, J=(1.0,) * 9))
    assert ei.value.code == pk.SP_E_ARG
    e.set_hamiltonian(HAM0)
    with pytest.raises(pk.SpError) as ei:
        e.gradient()
    assert ei.value.code == pk.SP_E_ORDER
    with pytest.raises(pk.SpError):
        e.step_path = "nonsense"


@pytest.mark.parametrize("case", ["tri1540x1530", "tri1536x1472", "sq1600x1536_open_2shell"])
def test_stencil_gradient_large_tiles_match_oracle(ora, case):
    """Lattices large enough for the 64 x 64 tiles of the stand-alone stencil
    gradient (ragged tiles, open edges): every site against the oracle."""
    announce(f"stencil gradient large tiles {case}")
    if case == "tri1540x1530":
        geo, ham = si.triangular(1540, 1530), HAM1
    elif case == "tri1536x1472":   # whole 64 x 64 tiles: the 16-byte load and store kernel
        geo, ham = si.triangular(1536, 1472), HAM1
    else:
        geo, ham = si.square(1600, 1536, periodic=(0, 1, 0)), dataclasses.replace(HAM0, J=(1.0, 0.3))
    e, s = make_pair(ora, geo, ham, "f32")
    assert e.step_path.startswith("shape2d")
    n = si.uniform_sphere(s.N, 77)
    e.set_spins(n)
    assert_close(e.gradient(), s.gradient(n), "f32", what=f"stencil gradient {case}")


def test_stencil_gradient_to_unaligned_array_matches_aligned(ora):
    """A gradient written to a device array that is not 16-byte aligned takes
    the single-float kernel; on a lattice of whole 64 x 64 tiles it must equal,
    bit for bit, the 16-byte kernel's output to an aligned array."""
    import torch

    announce("stencil gradient unaligned output")
    geo, ham = si.square(1600, 1536, periodic=(0, 1, 0)), dataclasses.replace(HAM0, J=(1.0, 0.3))
    e, s = make_pair(ora, geo, ham, "f32")
    n = si.uniform_sphere(s.N, 78)
    e.set_spins(n)
    g_al = torch.zeros(3 * s.N, dtype=torch.float32, device="cuda")
    g_buf = torch.zeros(3 * s.N + 1, dtype=torch.float32, device="cuda")
    g_mis = g_buf[1:]
    assert g_mis.data_ptr() % 16 != 0
    e.gradient_dev(g_al)
    e.gradient_dev(g_mis)
    e.synchronize()
    assert torch.equal(g_al, g_mis)
    assert_close(g_al.double().cpu().numpy().reshape(3, -1), s.gradient(n), "f32", what="16-byte kernel")


@pytest.mark.parametrize("path", ["shape2d/64x16x1024", "persist2d/64x16", "twopass"])
def test_zero_work_calls_change_nothing(ora, path):
    """Empty runs: zero LLG steps, zero Monte Carlo sweeps, zero GNEB
    iterations and zero batch steps return OK and leave spins and step
    counters as they were; an observation interval longer than the run
    yields no observation; negative counts are rejected."""
    import paper_1901_11350_amd as pk

    announce(f"zero work {path}")
    e = pk.Engine(0, "f32")
    geo = si.triangular(128, 64)
    e.set_geometry(geo)
    e.set_hamiltonian(HAM1)
    e.step_path = path
    n0 = si.uniform_sphere(e.N, 3)
    e.set_spins(n0)
    e.step = 7
    before = e.get_spins()
    assert e.run(0.1, 0.001, 0, T=10.0, seed=1) == []
    assert e.run(0.1, 0.001, 0, T=10.0, seed=1, observe_every=5) == []
    assert e.step == 7 and np.array_equal(e.get_spins(), before)
    obs = e.run(0.1, 0.001, 3, T=10.0, seed=1, observe_every=5)   # interval longer than the run
    assert obs == [] and e.step == 10
    with pytest.raises(pk.SpError):
        e.run(0.1, 0.001, -1)
    m = pk.Engine(0, "f32")
    m.set_geometry(si.square(16, 16))
    m.set_hamiltonian(dataclasses.replace(HAM0, D=()))
    m.set_spins(si.uniform_sphere(m.N, 4))
    m0 = m.get_spins()
    obs, acc = m.mc_run(10.0, 30.0, 0, observe_every=1)
    assert obs == [] and acc == 0 and np.array_equal(m.get_spins(), m0)
    g_eng = pk.Engine(0, "f32")
    g_eng.set_geometry(si.square(16, 16))
    g_eng.set_hamiltonian(HAM0)
    chain = si.geodesic_chain(si.skyrmion_ansatz(si.square(16, 16), radius=3.0), si.ferromagnet(256, (0, 0, 1)), 5,
                              fallback_axis=(1, 0, 0))
    g = pk.Gneb(g_eng, chain)
    c0 = g.chain()
    g.iterate(0)
    assert np.array_equal(g.chain(), c0)
    with pytest.raises(pk.SpError):
        g.iterate(-1)
    b = pk.Batch(0)
    r = pk.Engine(0, "f32")
    r.set_geometry(si.square(32, 32))
    r.set_hamiltonian(HAM0)
    r.set_spins(si.uniform_sphere(r.N, 5))
    b.add(r, 0.3, 0.001)
    s0 = b.get_spins(0)
    b.run(0)
    assert b.step == 0 and np.array_equal(b.get_spins(0), s0)


TILE_CASES = {
    "honeycomb37x22": (si.honeycomb(37, 22), HC_HAM),
    "honeycomb41x19_4shell": (si.honeycomb(41, 19), dataclasses.replace(HC_HAM, J=(1.0, 0.2, -0.1, 0.05))),
    "honeycomb35x18_open": (si.honeycomb(35, 18, periodic=(0, 1, 0)), HC_HAM),
    "kagome24x19_open": (si.kagome(24, 19, periodic=(1, 0, 0)), KG_HAM),
    "square4atom16x12": (SQ4_GEO, SQ4_HAM),
    "basis2": (BASIS2_GEO, BASIS2_HAM),
    "bcc12x10x6": (BASIS2_GEO.with_cells((12, 10, 6), (1, 1, 1)), BASIS2_HAM),
    "fcc9x8x7": (si.fcc_primitive(9, 8, 7),
                 si.Hamiltonian(mu=(2.0,), B=(0.0, 0.0, 0.3), K=(0.05,), K_axis=((0, 0, 1),), J=(1.0, 0.1),
                                D=(0.1,), dmi_kind=si.DMI_BULK)),
}


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(TILE_CASES))
def test_fused_tile_path_matches_oracle(ora, case, precision):
    """Lattices with a basis (2D: two to four atoms, reach 1 and 2, ragged
    and open edges; 3D: two atoms, open and periodic c) and a 3D one-atom
    lattice without a compile-time stencil take the fused tile path by
    default; the field on its tiles and its 4-step stochastic trajectory
    match the oracle's, and the trajectory the two-pass path's."""
    geo, ham = TILE_CASES[case]
    announce(f"fused tile {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path == "fusedtile", e.step_path
    n0 = si.uniform_sphere(s.N, 31)
    e.set_spins(n0)
    assert_close(e.gradient(), s.gradient(n0), precision, what=f"gradient on tiles {case}")
    ref, _ = s.run(n0, 0.3, 0.001, 4, T=20.0, seed=13, step0=3)
    res = {}
    for path in ["fusedtile", "twopass"]:
        e.step_path = path
        e.set_spins(n0)
        e.step = 3
        e.run(0.3, 0.001, 4, T=20.0, seed=13)
        res[path] = e.get_spins()
        assert_close(res[path], ref, precision, what=f"4 steps {case} [{path}]")
    assert rel_err(res["fusedtile"], res["twopass"]) <= 2 * TOL[precision]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["honeycomb41x19_4shell", "kagome24x19_open", "bcc12x10x6"])
def test_fused_tile_trajectory_200_steps(ora, case, precision):
    """200 damped steps (T = 0) on the fused tile path against the oracle."""
    geo, ham = TILE_CASES[case]
    announce(f"fused tile 200 steps {case} {precision}")
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path == "fusedtile"
    n0 = si.uniform_sphere(s.N, 37)
    e.set_spins(n0)
    e.run(0.3, 0.001, 200)
    ref, _ = s.run(n0, 0.3, 0.001, 200)
    assert_close(e.get_spins(), ref, precision, what=f"200 steps {case}")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_four_atom_cell_equals_the_one_atom_lattice(ora, precision):
    """The square lattice of spacing 1/2 as a four-atom cell (fused tile path)
    and as a 32 x 24 one-atom lattice (compile-time stencil path): the same
    spins give the same trajectory, site by site."""
    announce(f"four-atom cell vs one-atom lattice {precision}")
    import paper_1901_11350_amd as pk

    a = pk.Engine(0, precision)
    a.set_geometry(SQ4_GEO)
    a.set_hamiltonian(SQ4_HAM)
    assert a.step_path == "fusedtile"
    one_geo = si.Geometry(((0.5, 0, 0), (0, 0.5, 0), (0, 0, 1.0)), ((0, 0, 0),), (32, 24, 1), (1, 1, 0))
    one_ham = si.Hamiltonian(mu=(2.0,), B=(0.0, 0.0, 1.0), K=(0.1,), K_axis=((0, 0, 1),), J=(1.0, 0.3), D=(0.3,))
    b = pk.Engine(0, precision)
    b.set_geometry(one_geo)
    b.set_hamiltonian(one_ham)
    # site (x, y) of the fine lattice is atom (x % 2) + 2 (y % 2) of cell (x // 2, y // 2)
    x, y = np.meshgrid(np.arange(32), np.arange(24))
    x, y = x.ravel(), y.ravel()
    four = (x // 2) + 16 * ((y // 2) + 12 * ((x % 2) + 2 * (y % 2)))
    one = x + 32 * y
    n_one = si.uniform_sphere(32 * 24, 41)
    n_four = np.zeros_like(n_one)
    n_four[:, four] = n_one[:, one]
    a.set_spins(n_four)
    b.set_spins(n_one)
    assert_close(a.gradient()[:, four], b.gradient()[:, one], precision, what="gradient")
    a.run(0.3, 0.001, 50, T=0.0)
    b.run(0.3, 0.001, 50, T=0.0)
    assert_close(a.get_spins()[:, four], b.get_spins()[:, one], precision, what="50 steps")
    a.close()
    b.close()


STACK3_GEO = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0, 0, 1 / 3), (0.5, 0.5, 2 / 3)),
                         (12, 10, 6), (1, 1, 1))
STACK3_HAM = si.Hamiltonian(mu=(2.0, 2.5, 3.0), B=(0.1, 0.0, 0.3), K=(0.1, 0.0, -0.1),
                            K_axis=((0, 0, 1), (1, 0, 0), (0, 0.6, 0.8)), J=(1.0, 0.4, 0.2), D=(0.1,),
                            dmi_kind=si.DMI_BULK)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_three_atom_cell_in_3d(ora, precision):
    """A 3D cell of three atoms (6, 6 and 22 bonds): the fused tile path in
    FP32 (8 x 8 x 4 tiles of the three atoms), the two-pass path in FP64
    (the tile would not fit in LDS); field and 4-step stochastic trajectory
    against the oracle."""
    announce(f"three-atom 3D cell {precision}")
    e, s = make_pair(ora, STACK3_GEO, STACK3_HAM, precision)
    assert e.step_path == ("fusedtile" if precision == "f32" else "twopass"), e.step_path
    n0 = si.uniform_sphere(s.N, 43)
    e.set_spins(n0)
    assert_close(e.gradient(), s.gradient(n0), precision, what="gradient three-atom 3D")
    e.step = 3
    e.run(0.3, 0.001, 4, T=20.0, seed=13)
    ref, _ = s.run(n0, 0.3, 0.001, 4, T=20.0, seed=13, step0=3)
    assert_close(e.get_spins(), ref, precision, what="4 steps three-atom 3D")
