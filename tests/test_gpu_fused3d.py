"""GPU parity of the streamed 3D fused step (compile-time simple-cubic
stencils, one to three shells, DMI on the first shell) against the FP64
oracle, for every tile configuration and integrator, ragged tiles, open and
periodic axes, thin lattices, the full 128^3 workload, and the largest
lattice the engine accepts (2^29 sites) on sampled sites."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import TOL, announce, assert_close, make_pair, need_gpu, rel_err

pytestmark = pytest.mark.gpu

HAM2 = si.WORKLOADS["cubic128_bulkdmi"].hamiltonian
CASES = {
    "sc2_bulk_12x10x8": (si.simple_cubic(12, 10, 8), HAM2),
    "sc2_bulk_ragged_37x21x11_openz": (si.simple_cubic(37, 21, 11, periodic=(1, 1, 0)), HAM2),
    "sc1_interfacial_20x18x6_open": (si.simple_cubic(20, 18, 6, periodic=(0, 0, 0)),
                                     dataclasses.replace(HAM2, J=(1.0,), D=(0.2,), dmi_kind=si.DMI_INTERFACIAL,
                                                         K=(0.1,), K_axis=((0.0, 0.6, 0.8),))),
    "sc3_nodmi_17x16x5": (si.simple_cubic(17, 16, 5), dataclasses.replace(HAM2, J=(1.0, 0.2, -0.05), D=())),
    "sc2_thin_9x9x2": (si.simple_cubic(9, 9, 2), HAM2),
    "sc1_40x4x3_periodic_small": (si.simple_cubic(40, 4, 3), dataclasses.replace(HAM2, J=(1.0,), D=(0.15,))),
}
CFGS = {"f32": ["32x16", "16x16", "32x8", "16x16z", "32x16b", "32x32"], "f64": ["16x16", "16x16z"]}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("solver", ["depondt", "heun", "sib"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_fused3d_matches_oracle(ora, case, precision, solver):
    geo, ham = CASES[case]
    announce(f"fused3d {case} {precision} {solver}")
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path.startswith("shape3d"), e.step_path
    n0 = si.uniform_sphere(s.N, 19)
    n_ora, _ = s.run(n0, 0.5, 0.001, 3, T=30.0, seed=4, step0=7, solver=solver)
    res = {}
    for path in ["twopass"] + ["shape3d/" + c for c in CFGS[precision]]:
        e.step_path = path
        assert e.step_path == path
        e.set_spins(n0)
        e.step = 7
        e.run(0.5, 0.001, 3, T=30.0, seed=4, solver=solver)
        res[path] = e.get_spins()
        assert_close(res[path], n_ora, precision, what=f"{path} {case} {solver}")
    for path in res:
        assert rel_err(res[path], res["twopass"]) <= 2 * TOL[precision]


def test_fused3d_full_cubic128_thermal(ora):
    """The 128^3 lattice (2,097,152 spins) on the streamed path: two steps with
    the thermal field on (T = 20 K, global site index as Philox counter)
    against the oracle over the whole lattice."""
    w = si.WORKLOADS["cubic128_bulkdmi"]
    announce("fused3d cubic128 full")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    assert e.step_path.startswith("shape3d")
    n0 = si.conical_helix(w.geometry, seed=w.init_seed)
    e.set_spins(n0)
    d = w.dynamics
    e.run(d.alpha, d.dt, 2, T=20.0, seed=d.seed)
    n_ora, _ = s.run(n0, d.alpha, d.dt, 2, T=20.0, seed=d.seed)
    assert_close(e.get_spins(), n_ora, "f32", what="cubic128 two thermal steps")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", ["sc2_bulk_ragged_37x21x11_openz", "sc1_interfacial_20x18x6_open",
                                  "sc3_nodmi_17x16x5", "sc2_thin_9x9x2", "sc1_40x4x3_periodic_small", "cubic128"])
def test_observation_on_3d_stencil_tiles_matches_oracle(ora, case, precision):
    """Energy per term, largest torque, mean spin and norm deviation formed on
    the 3D stencil tiles (32 x 8 tiles of one plane with its neighbours;
    ragged tiles, open axes, no DMI, and the 128^3 lattice, whose 8,192 work
    items exceed the partial rows) against the oracle, and for the ragged
    case against the generic kernel of the same bonds given as explicit
    pairs."""
    announce(f"3d observation {case} {precision}")
    if case == "cubic128":
        w = si.WORKLOADS["cubic128_bulkdmi"]
        geo, ham = w.geometry, w.hamiltonian
    else:
        geo, ham = CASES[case]
    e, s = make_pair(ora, geo, ham, precision)
    assert e.step_path.startswith("shape3d")
    n = si.uniform_sphere(s.N, 31)
    e.set_spins(n)
    obs, oo = e.observe(), s.observe(n)
    tol = TOL[precision]
    scale = np.abs(oo["per_term"]).sum()
    assert np.abs(np.array(obs["per_term"]) - np.array(oo["per_term"])).max() <= tol * scale
    assert obs["max_torque"] == pytest.approx(oo["max_torque"], rel=10 * tol)
    assert np.allclose(obs["M"], oo["M"], atol=10 * tol)
    if precision == "f64":
        assert obs["max_norm_dev"] == pytest.approx(oo["max_norm_dev"], abs=1e-14)
    else:
        assert obs["max_norm_dev"] < 1e-6
    if case == "sc2_bulk_ragged_37x21x11_openz":
        table = {(b[0], b[1], b[2], b[3], b[4]): b for b in s.bonds()}
        pairs = [(b[0], b[1], (b[2], b[3], b[4]), b[6], b[7]) for k, b in table.items()
                 if k < (b[1], b[0], -b[2], -b[3], -b[4])]
        g, _ = make_pair(ora, geo, dataclasses.replace(ham, J=(), D=()), precision)
        g.set_pairs(pairs)
        assert not g.step_path.startswith("shape3d")
        g.set_spins(n)
        og = g.observe()
        assert np.abs(np.array(obs["per_term"]) - np.array(og["per_term"])).max() <= 2 * tol * scale
        assert obs["max_torque"] == pytest.approx(og["max_torque"], rel=10 * tol)


def test_fused3d_max_size_lattice_follows_the_periodic_patch(ora):
    """A 1024 x 1024 x 512 periodic simple-cubic lattice (exactly 2^29 sites,
    the 128^3 workload's Hamiltonian, FP32) filled with a periodic tiling of a
    random 16^3 patch.  At T = 0 the dynamics commute with lattice
    translations, so after two steps on the streamed 3D path every sampled
    site (the eight corners included) must hold the oracle's trajectory of the
    16^3 periodic patch, and the energy per spin must be the patch's.  The
    spins are built and read on the device."""
    import torch

    import paper_1901_11350_amd as pk

    w = si.WORKLOADS["cubic128_bulkdmi"]
    d = w.dynamics
    P, BIG = 16, (1024, 1024, 512)
    announce(f"fused3d max size {BIG}")
    patch = si.uniform_sphere(P ** 3, 77)
    s = ora.System(w.geometry.with_cells((P, P, P)), w.hamiltonian)
    ref, _ = s.run(patch, d.alpha, d.dt, 2)            # T = 0
    e = pk.Engine(0, "f32")
    e.set_geometry(w.geometry.with_cells(BIG))
    e.set_hamiltonian(w.hamiltonian)
    assert e.N == 1 << 29
    assert e.step_path.startswith("shape3d"), e.step_path
    p = torch.tensor(patch.reshape(3, P, P, P), dtype=torch.float32, device="cuda")   # [3][c][b][a]
    n = p.repeat(1, BIG[2] // P, BIG[1] // P, BIG[0] // P).reshape(3, -1).contiguous()
    del p
    torch.cuda.synchronize()
    e.set_spins_dev(n)
    e.step = 0
    e.run(d.alpha, d.dt, 2)
    e.get_spins_dev(n)
    e.synchronize()
    rng = np.random.default_rng(8)
    xs = rng.integers(0, BIG[0], 8192)
    ys = rng.integers(0, BIG[1], 8192)
    zs = rng.integers(0, BIG[2], 8192)
    for k in range(8):                                  # the eight corners
        xs[k] = (BIG[0] - 1) * (k & 1)
        ys[k] = (BIG[1] - 1) * ((k >> 1) & 1)
        zs[k] = (BIG[2] - 1) * (k >> 2)
    idx = torch.tensor(xs + BIG[0] * (ys + BIG[1] * zs), device="cuda")
    got = n[:, idx].double().cpu().numpy()
    want = ref[:, (xs % P) + P * ((ys % P) + P * (zs % P))]
    assert_close(got, want, "f32", what="2^29-site 3D lattice")
    E_big = e.energy() / e.N
    E_patch = s.energy(ref) / P ** 3
    assert E_big == pytest.approx(E_patch, rel=1e-5)
    del n, e
    torch.cuda.empty_cache()
