"""FP32 trajectory parity at full size, up to the measured horizon, and the
statistics beyond it.

The horizon H of a workload is the last step at which two FP64 oracle runs
whose initial states differ by about 1e-7 per component still agree within
1e-5 (tests/golden/make_fp32_horizon.py measures it on the CPU and stores
it with the two runs' observables every 100 steps).  Up to min(H, 1000)
steps the FP32 engine must follow the FP64 oracle within 1e-5 at every
site; beyond H trajectories may part, and the energy per spin and mean spin
of the engine's run must differ from the oracle's by no more than ten times
what the two oracle runs themselves differ by."""

import json
import os

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, make_pair, need_gpu

pytestmark = pytest.mark.gpu
W = si.WORKLOADS


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _horizon(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", "fp32_horizon.json")) as f:
        return json.load(f)[name]


def _initial(w):
    if w.init == "conical_helix":
        return si.conical_helix(w.geometry, seed=w.init_seed)
    return si.uniform_sphere(w.geometry.n_sites, w.init_seed)


@pytest.mark.parametrize("name", ["triangular512_sllg", "cubic128_bulkdmi"])
def test_full_size_fp32_follows_the_oracle_to_the_horizon(ora, name):
    h = _horizon(name)
    w = W[name]
    steps = min(h["horizon"], 1000)
    announce(f"full size fp32 {name} {steps} steps (horizon {h['horizon']})")
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f32")
    n0 = _initial(w)
    e.set_spins(n0)
    d = w.dynamics
    e.run(d.alpha, d.dt, steps, T=d.T, seed=d.seed)
    n_ora, _ = s.run(n0, d.alpha, d.dt, steps, T=d.T, seed=d.seed)
    assert_close(e.get_spins(), n_ora, "f32", 1e-5, what=f"{name} after {steps} steps")
    e.close()


def test_triangular512_statistics_beyond_the_horizon():
    """The stochastic 512^2 workload over its full 10,000 steps (H = the
    stored horizon): energy per spin and mean spin every 100 steps after H
    against the oracle's run."""
    name = "triangular512_sllg"
    h = _horizon(name)
    w = W[name]
    d = w.dynamics
    announce(f"statistics beyond the horizon {name} (H = {h['horizon']})")
    import paper_1901_11350_amd as pk

    e = pk.engine_for(w, 0, "f32")
    e.set_spins(_initial(w))
    obs = e.run(d.alpha, d.dt, d.n_steps, T=d.T, seed=d.seed, observe_every=100)
    e.close()
    ref = {o["step"]: o for o in h["observations_run"]}
    alt = {o["step"]: o for o in h["observations_perturbed"]}
    late = [o for o in obs if o["step"] > h["horizon"]]
    assert len(late) >= 50
    dE_pair = max(abs(ref[o["step"]]["E_per_spin"] - alt[o["step"]]["E_per_spin"]) for o in late)
    dM_pair = max(np.abs(np.subtract(ref[o["step"]]["M"], alt[o["step"]]["M"])).max() for o in late)
    dE = max(abs(o["E"] / e.N - ref[o["step"]]["E_per_spin"]) for o in late)
    dM = max(np.abs(np.subtract(o["M"], ref[o["step"]]["M"])).max() for o in late)
    print(f"[horizon] beyond H: |dE/N| {dE:.3e} (oracle pair {dE_pair:.3e}), |dM| {dM:.3e} "
          f"(oracle pair {dM_pair:.3e})", flush=True)
    assert dE <= 10 * dE_pair + 1e-9
    assert dM <= 10 * dM_pair + 1e-9
