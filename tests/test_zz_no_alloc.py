"""The allocation-free dipole entry point (sp_dipole_gradient_dev_noalloc,
through the C ABI) against sp_dipole_gradient_dev on the same engine and
inputs: two calls in a row, the second on a smaller lattice (the static
scratch keeps the first call's partial sums), in both precisions; and the
size limit of the static scratch."""

import ctypes

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _film(na, nb, nc):
    geo = si.simple_cubic(na, nb, nc, periodic=(0, 0, 0))
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0.2), K=(0.2,), K_axis=((0, 0, 1),), J=(1.0,), ddi=1)
    return geo, ham


def _both(precision, geo, ham, seed):
    import torch

    import paper_1901_11350_amd as pk

    dt = torch.float64 if precision == "f64" else torch.float32
    e = pk.Engine(0, precision)
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    n = torch.tensor(si.uniform_sphere(e.N, seed), dtype=dt, device="cuda").contiguous()
    g_ref = torch.full((3, e.N), float("nan"), dtype=dt, device="cuda")
    g_new = torch.full((3, e.N), float("nan"), dtype=dt, device="cuda")
    e.dipole_gradient_dev(n, g_ref)
    rc = pk.lib().sp_dipole_gradient_dev_noalloc(e._h, ctypes.c_void_p(n.data_ptr()),
                                                 ctypes.c_void_p(g_new.data_ptr()), e.N)
    assert rc == 0, pk.lib().sp_last_error(e._h).decode()
    torch.cuda.synchronize()
    out = (n.double().cpu().numpy(), g_ref.double().cpu().numpy(), g_new.double().cpu().numpy())
    e.close()
    return out


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_noalloc_matches_the_allocating_entry_point(ora, precision):
    tol = 1e-12 if precision == "f64" else 1e-5
    for k, dims in enumerate([(24, 20, 4), (9, 7, 2)]):   # second call: smaller input
        announce(f"noalloc dipole {precision} {dims}")
        geo, ham = _film(*dims)
        n, g_ref, g_new = _both(precision, geo, ham, 40 + k)
        assert np.isfinite(g_new).all()
        assert_close(g_new, g_ref, precision, tol, what=f"noalloc vs sp_dipole_gradient_dev {dims}")
        # and the oracle's direct sum of the same spins
        s = ora.System(geo, ham)
        g_ora = s.dipole_gradient_sites(n, np.arange(s.N))
        assert_close(g_new, g_ora, precision, tol, what=f"noalloc vs oracle {dims}")


def test_noalloc_rejects_lattices_beyond_the_scratch():
    import torch

    import paper_1901_11350_amd as pk

    announce("noalloc size limit")
    geo, ham = _film(1200, 1200, 1)   # 1.44 M sites: 3 N x 8 B x 1 slice > 32 MiB in FP64
    e = pk.Engine(0, "f64")
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    n = torch.zeros((3, e.N), dtype=torch.float64, device="cuda")
    g = torch.zeros_like(n)
    rc = pk.lib().sp_dipole_gradient_dev_noalloc(e._h, ctypes.c_void_p(n.data_ptr()),
                                                 ctypes.c_void_p(g.data_ptr()), e.N)
    assert rc == pk.SP_E_ARG
    assert "static scratch" in pk.lib().sp_last_error(e._h).decode()
    e.close()
