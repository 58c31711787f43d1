"""Helpers shared by the GPU parity tests: build an engine and an oracle
system for the same workload, and the normwise tolerances.

Tolerances (relative to the largest component of the reference, i.e.
max|a - b| <= tol * max|b|): FP64 engine 1e-12, FP32 engine 1e-5.
"""

import numpy as np
import pytest

from conftest import gpu_available

TOL = {"f64": 1e-12, "f32": 1e-5}


def need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def make_pair(ora, geometry, hamiltonian, precision):
    import paper_1901_11350_amd as pk

    e = pk.Engine(0, precision)
    e.set_geometry(geometry)
    e.set_hamiltonian(hamiltonian)
    s = ora.System(geometry, hamiltonian)
    assert e.N == s.N
    return e, s


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def assert_close(a, b, precision, tol=None, what=""):
    t = TOL[precision] if tol is None else tol
    err = rel_err(a, b)
    assert err <= t, f"{what}: normwise relative error {err:.3e} > {t:.1e}"
    return err


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
