"""Run control of the C ABI on the GPU: graph-replayed sp_run chunks against
direct launches, and the convergence tests of sp_run_tol (damped LLG as a
minimiser, Sec. III.C) and sp_gneb_iterate_tol (velocity projection of a
chain, Appendix D) against the FP64 oracle."""

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, make_pair, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _engine(geo, ham, precision, path=None):
    import paper_1901_11350_amd as pk

    e = pk.Engine(0, precision)
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    if path:
        e.step_path = path
    return e


CASES = {
    # 2D compile-time stencil, thermal field (the step comes from the device)
    "tri96x64_shape2d": (si.triangular(96, 64), si.WORKLOADS["triangular512_sllg"].hamiltonian, None),
    # generic two-pass kernels
    "tri40x24_twopass": (si.triangular(40, 24), si.WORKLOADS["triangular512_sllg"].hamiltonian, "twopass"),
    # 3D streamed stencil
    "cubic16_shape3d": (si.simple_cubic(16, 16, 16), si.WORKLOADS["cubic128_bulkdmi"].hamiltonian, None),
}


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("observe_every", [0, 5, 20])
def test_graph_replay_is_bit_identical_to_direct_launches(case, precision, observe_every):
    """Three consecutive sp_run calls (chunks replayed from the cache, the
    step advancing on the device, an odd chunk length swapping the buffers)
    give the same spins and observations, bit for bit, as direct launches."""
    geo, ham, path = CASES[case]
    announce(f"graph replay {case} {precision} observe_every={observe_every}")
    n0 = si.uniform_sphere(geo.n_sites, 3)
    out = []
    for graphs in (True, False):
        e = _engine(geo, ham, precision, path)
        e.set_graph_replay(graphs)
        e.set_spins(n0)
        obs = []
        for k, steps in enumerate((64, 40, 100)):
            obs += e.run(0.1, 0.0005, steps, T=10.0, seed=77, observe_every=observe_every)
        out.append((e.get_spins(), obs, e.step, e.step_path))
        e.close()
    (sa, oa, ka, pa), (sb, ob, kb, pb) = out
    assert pa == pb and ka == kb == 204
    assert np.array_equal(sa, sb)
    assert len(oa) == len(ob) == (sum(s // observe_every for s in (64, 40, 100)) if observe_every else 0)
    for a, b in zip(oa, ob):
        assert a == b


def test_graph_replay_follows_the_oracle_trajectory(ora):
    """A replayed stochastic run against the oracle's (FP64, 1e-12)."""
    announce("graph replay vs oracle")
    w = si.WORKLOADS["triangular512_sllg"]
    geo = si.triangular(64, 48)
    e, s = make_pair(ora, geo, w.hamiltonian, "f64")
    n0 = si.uniform_sphere(s.N, 5)
    e.set_spins(n0)
    obs = e.run(0.1, 0.0005, 96, T=10.0, seed=9, observe_every=32)
    n_ora, obs_ora = s.run(n0, 0.1, 0.0005, 96, T=10.0, seed=9, observe_every=32)
    assert_close(e.get_spins(), n_ora, "f64", 1e-12, what="spins after 96 replayed steps")
    for a, b in zip(obs, obs_ora):
        assert a["step"] == b["step"]
        assert abs(a["E"] - b["E"]) <= 1e-12 * abs(b["E"])
    e.close()


@pytest.mark.parametrize("precision,path", [("f64", None), ("f32", None), ("f64", "twopass"),
                                            ("f64", "persist2d/32x16")])
def test_run_tol_stops_at_the_first_converged_observation(ora, precision, path):
    """Damped relaxation of the 32 x 32 square workload: the run stops at the
    first observation whose maximum torque is below tol, with the state of
    that observation; the oracle's trajectory over the same number of steps
    gives the same state, and its torques decide the same stopping step."""
    announce(f"run_tol square32 {precision} {path}")
    w = si.WORKLOADS["square32_fp64"]
    e, s = make_pair(ora, w.geometry, w.hamiltonian, precision)
    if path:
        e.step_path = path
    # a ferromagnet with strong noise relaxes smoothly (no metastable walls)
    rng = np.random.default_rng(4)
    n0 = np.zeros((3, s.N))
    n0[2] = 1.0
    n0 += 0.4 * rng.standard_normal(n0.shape)
    n0 /= np.linalg.norm(n0, axis=0)
    e.set_spins(n0)
    tol, every, max_steps = 0.1, 50, 20000
    obs, done = e.run_tol(0.3, 0.001, max_steps, every, tol)
    assert 0 < done < max_steps and done % every == 0
    assert e.step == done
    assert len(obs) == done // every
    assert obs[-1]["max_torque"] < tol
    assert all(o["max_torque"] >= tol for o in obs[:-1])
    n_ora, obs_ora = s.run(n0, 0.3, 0.001, done, observe_every=every)
    t_ora = [o["max_torque"] for o in obs_ora]
    # the stopping decision: the oracle's torque crosses tol at the same observation
    margin = 1e-9 if precision == "f64" else 1e-4
    assert t_ora[-1] < tol * (1 + margin)
    assert all(t >= tol * (1 - margin) for t in t_ora[:-1])
    assert_close(e.get_spins(), n_ora, precision, 1e-12 if precision == "f64" else 1e-5,
                 what=f"state at the converged step {done}")
    # nothing moves after convergence within the call: the state is the observed one
    o_now = e.observe()
    assert abs(o_now["max_torque"] - obs[-1]["max_torque"]) <= 1e-12 * obs[-1]["max_torque"] + 1e-15
    # a converged state stops a new run at its first observation
    obs2, done2 = e.run_tol(0.3, 0.001, 1000, every, tol * 10)
    assert done2 == every and e.step == done + every
    e.close()


def test_run_tol_runs_to_the_limit_when_unconverged(ora):
    announce("run_tol unconverged")
    w = si.WORKLOADS["square32_fp64"]
    e, s = make_pair(ora, w.geometry, w.hamiltonian, "f64")
    n0 = si.uniform_sphere(s.N, 1)
    e.set_spins(n0)
    obs, done = e.run_tol(0.3, 0.001, 200, 50, 1e-9)
    assert done == 200 and len(obs) == 4 and e.step == 200
    n_ora, _ = s.run(n0, 0.3, 0.001, 200)
    assert_close(e.get_spins(), n_ora, "f64", 1e-12, what="200 unconverged steps")
    e.close()


def test_gneb_iterate_tol_stops_on_the_oracle_iteration(ora):
    """Skyrmion-collapse chain on a 12 x 10 lattice (FP64): iterations stop
    when the largest per-spin force falls below tol; the oracle's forces cross
    tol at the same iteration and its chain there matches, within the 1e-12
    bar or ten times the divergence the oracle's own iteration map gives two
    chains started 1e-15 apart, whichever is larger."""
    import paper_1901_11350_amd as pk

    from test_gpu_gneb import _case, chain_sensitivity

    announce("gneb iterate_tol square12x10")
    geo, ham, chain, kw = _case("square12x10")
    e = pk.Engine(0, "f64")
    e.set_geometry(geo)
    e.set_hamiltonian(ham)
    g = pk.Gneb(e, chain, **kw)
    tol = 1e-4
    assert g.iterate_tol(0, tol) == 0
    done = g.iterate_tol(2000, tol)
    assert 0 < done < 2000
    assert np.linalg.norm(g.forces()["F"], axis=1).max() < tol
    s = ora.System(geo, ham)
    o = ora.Gneb(s, chain, **kw)
    fmax = []
    for _ in range(done):
        o.iterate(1)
        fmax.append(np.linalg.norm(o.forces()["F"], axis=1).max())
    assert fmax[-1] < tol * (1 + 1e-9) and all(f >= tol * (1 - 1e-9) for f in fmax[:-1])
    bound = max(1e-12, 10 * chain_sensitivity(ora, geo, ham, chain, kw, done)[0])
    assert_close(g.chain(), o.chain, "f64", bound, what=f"chain after {done} iterations")
    g.close()
    e.close()
