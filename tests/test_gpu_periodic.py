"""The step instances for fully periodic lattices (FP32 Depondt: 64 x 16 x
1024 tiles in 2D, 32 x 32 columns in 3D) compile the boundary tests and the
zero fills of outside cells out and address the spins by 32-bit byte
offsets; their arithmetic is that of the general instances, term for term
and in the same order.  Only the rounding may differ: with a branch folded
away the compiler may fuse a product and the sum it feeds into one
multiply-add (one rounding instead of two) where the general instance keeps
them apart (measured: one FP32 unit in the last place on some components).
On periodic lattices -- tile-aligned and ragged, with and without
anisotropy, at T > 0 so the thermal field is drawn -- they must therefore
reproduce the general instances of other tile shapes to a few FP32
roundings (normwise 1e-6 after 10 steps, ten times below the parity bar),
and follow the FP64 oracle."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, make_pair, need_gpu, rel_err

pytestmark = pytest.mark.gpu

HAM3 = si.WORKLOADS["cubic128_bulkdmi"].hamiltonian
HAM3_K = dataclasses.replace(HAM3, K=(0.1,), K_axis=((0.0, 0.6, 0.8),))
HAM2 = si.WORKLOADS["triangular512_sllg"].hamiltonian

CASES = {
    # (geometry, Hamiltonian, periodic-instance path, general-instance path)
    "cubic64x64x16_bulk": (si.simple_cubic(64, 64, 16), HAM3, "shape3d/32x32", "shape3d/32x16b"),
    "cubic40x36x10_ragged_aniso": (si.simple_cubic(40, 36, 10), HAM3_K, "shape3d/32x32", "shape3d/32x16b"),
    "cubic12x10x8_small": (si.simple_cubic(12, 10, 8), HAM3, "shape3d/32x32", "shape3d/16x16"),
    "tri128x64": (si.triangular(128, 64), HAM2, "shape2d/64x16x1024", "shape2d/32x32x1024"),
    "tri100x37_ragged": (si.triangular(100, 37), HAM2, "shape2d/64x16x1024", "shape2d/32x16x512"),
}


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("case", sorted(CASES))
def test_periodic_instance_matches_the_general_one(ora, case):
    geo, ham, per_path, gen_path = CASES[case]
    announce(f"periodic instance {case}")
    e, s = make_pair(ora, geo, ham, "f32")
    n0 = si.uniform_sphere(s.N, 23)
    out = {}
    for path in (per_path, gen_path):
        e.step_path = path
        assert e.step_path == path
        e.set_spins(n0)
        e.step = 5
        e.run(0.3, 0.001, 10, T=25.0, seed=9)
        out[path] = e.get_spins()
    e.close()
    a, b = out[per_path], out[gen_path]
    assert rel_err(a, b) <= 1e-6, (rel_err(a, b), np.abs(a - b).max())
    n_ora, _ = s.run(n0, 0.3, 0.001, 10, T=25.0, seed=9, step0=5)
    assert_close(a, n_ora, "f32", what=f"periodic instance {case}")
