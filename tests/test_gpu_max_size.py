"""The largest lattice the engine accepts (2^29 sites) and the limits around
it.

A 32768 x 16384 periodic triangular lattice (exactly 2^29 sites, the
512^2 workload's Hamiltonian, FP32) is filled with a periodic tiling of a
64 x 64 random patch.  At T = 0 the dynamics commute with lattice
translations, so every site of the big lattice must follow the oracle's
trajectory of the 64 x 64 periodic patch: checked on sampled sites after
Depondt steps on the default fused path and on the two-pass path, for the
energy per spin, and for the LDS-tiled stencil gradient.  The spins are built and read on the device (torch
tensors through the *_dev entry points), so no 2^29-site array crosses to
the host.  Also: 2^29 + 1 sites are rejected, the persistent path refuses a
lattice whose tiles cannot all be resident, and the Philox normals of the
last sites of the lattice are bit-exact."""

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, need_gpu

pytestmark = pytest.mark.gpu

W = si.WORKLOADS
P = 64                    # patch side
BIG = (32768, 16384)      # 2^29 sites


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def big_engine():
    import torch

    import paper_1901_11350_amd as pk

    need_gpu()
    w = W["triangular512_sllg"]
    e = pk.Engine(0, "f32")
    e.set_geometry(w.geometry.with_cells((BIG[0], BIG[1], 1)))
    e.set_hamiltonian(w.hamiltonian)
    assert e.N == 1 << 29
    yield e
    del e
    torch.cuda.empty_cache()


def _tiled(torch, patch):
    p = torch.tensor(patch.reshape(3, P, P), dtype=torch.float32, device="cuda")   # [3][y][x]
    return p.repeat(1, BIG[1] // P, BIG[0] // P).reshape(3, -1).contiguous()


@pytest.mark.parametrize("path,steps", [("shape2d/64x16x1024", 2), ("twopass", 1)])
def test_max_size_lattice_follows_the_periodic_patch(ora, big_engine, path, steps):
    import torch

    announce(f"max size {BIG} {path} {steps} steps")
    w = W["triangular512_sllg"]
    d = w.dynamics
    patch = si.uniform_sphere(P * P, 99)
    s = ora.System(w.geometry.with_cells((P, P, 1)), w.hamiltonian)
    ref, _ = s.run(patch, d.alpha, d.dt, steps)            # T = 0
    e = big_engine
    e.step_path = path
    n = _tiled(torch, patch)
    torch.cuda.synchronize()
    e.set_spins_dev(n)
    e.step = 0
    e.run(d.alpha, d.dt, steps)
    e.get_spins_dev(n)
    e.synchronize()
    rng = np.random.default_rng(5)
    xs = rng.integers(0, BIG[0], 8192)
    ys = rng.integers(0, BIG[1], 8192)
    xs[:4] = [0, BIG[0] - 1, 0, BIG[0] - 1]            # the four corners
    ys[:4] = [0, 0, BIG[1] - 1, BIG[1] - 1]
    idx = torch.tensor(xs + ys * BIG[0], device="cuda")
    got = n[:, idx].double().cpu().numpy()
    want = ref[:, (xs % P) + (ys % P) * P]
    assert_close(got, want, "f32", what=f"2^29 sites, {path}")
    # energy per spin of the big lattice = that of the patch
    E_big = e.energy() / e.N
    E_patch = s.energy(ref) / (P * P)
    assert E_big == pytest.approx(E_patch, rel=1e-5)
    del n
    torch.cuda.empty_cache()


def test_max_size_stencil_gradient_follows_the_periodic_patch(ora, big_engine):
    """The LDS-tiled stencil gradient of the 2^29-site lattice on sampled
    sites against the oracle's gradient of the 64 x 64 periodic patch."""
    import torch

    announce("max size stencil gradient")
    w = W["triangular512_sllg"]
    patch = si.uniform_sphere(P * P, 123)
    s = ora.System(w.geometry.with_cells((P, P, 1)), w.hamiltonian)
    ref = s.gradient(patch)
    e = big_engine
    n = _tiled(torch, patch)
    g = torch.empty_like(n)
    torch.cuda.synchronize()
    e.set_spins_dev(n)
    e.gradient_dev(g)
    e.synchronize()
    rng = np.random.default_rng(6)
    xs = rng.integers(0, BIG[0], 8192)
    ys = rng.integers(0, BIG[1], 8192)
    xs[:4] = [0, BIG[0] - 1, 0, BIG[0] - 1]
    ys[:4] = [0, 0, BIG[1] - 1, BIG[1] - 1]
    idx = torch.tensor(xs + ys * BIG[0], device="cuda")
    got = g[:, idx].double().cpu().numpy()
    assert_close(got, ref[:, (xs % P) + (ys % P) * P], "f32", what="2^29-site stencil gradient")
    del n, g
    torch.cuda.empty_cache()


def test_persistent_path_refuses_non_resident_tilings(big_engine):
    from paper_1901_11350_amd.engine import SpError

    announce("max size persist refused")
    keep = big_engine.step_path
    with pytest.raises(SpError):
        big_engine.step_path = "persist2d/64x16"        # 524,288 tiles
    assert big_engine.step_path == keep


def test_more_than_2_to_29_sites_rejected():
    import paper_1901_11350_amd as pk
    from paper_1901_11350_amd.engine import SpError

    e = pk.Engine(0, "f32")
    with pytest.raises(SpError):
        e.set_geometry(si.triangular(BIG[0] + 1, BIG[1]))
    e.set_geometry(si.triangular(BIG[0], BIG[1]))       # exactly 2^29: accepted


def test_philox_normals_of_the_last_sites_bit_exact(ora):
    import paper_1901_11350_amd as pk

    announce("philox last sites")
    e = pk.Engine(0, "f32")
    e.set_geometry(si.triangular(64, 64))
    e.set_hamiltonian(W["triangular512_sllg"].hamiltonian)
    site0 = (1 << 29) - 256
    eta, raw = e.thermal_normals(seed=0xDEADBEEF12345, step=(1 << 40) + 7, site0=site0, n_sites=256, replica=3)
    for k in range(0, 256, 17):
        want = ora.philox4x32_10((site0 + k, ((1 << 40) + 7) & 0xFFFFFFFF, ((1 << 40) + 7) >> 32, 3),
                                 (0xDEADBEEF12345 & 0xFFFFFFFF, 0xDEADBEEF12345 >> 32))
        assert tuple(int(v) for v in raw[k]) == tuple(want)
