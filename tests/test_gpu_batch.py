"""GPU tests of replica batches (LDS-resident small replicas, tiled large
replicas, HIP-graph chunks) against the FP64 oracle and against single-engine
runs of the same replica."""

import dataclasses

import numpy as np
import pytest

import spin_inputs as si
from gpu_util import announce, assert_close, need_gpu

pytestmark = pytest.mark.gpu

HAM0 = si.WORKLOADS["square32_fp64"].hamiltonian
HAM1 = si.WORKLOADS["triangular512_sllg"].hamiltonian


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _geo(lat, L):
    return si.square(L, L) if lat == "square" else si.triangular(L, L)


def _make(pk, lat, ham, specs, chunk=4):
    """specs: list of (side, T, alpha, dt, seed); replica index = position."""
    b = pk.Batch(0)
    b.set_chunk(chunk)
    inits = []
    for r, (L, T, alpha, dt, seed) in enumerate(specs):
        e = pk.Engine(0, "f32")
        e.set_geometry(_geo(lat, L))
        e.set_hamiltonian(ham)
        n0 = si.uniform_sphere(e.N, 1000 + r)
        e.set_spins(n0)
        assert b.add(e, alpha, dt, T=T, seed=seed, replica=r) == r
        inits.append(n0)
        e.close()
    return b, inits


SPECS = [(32, 0.0, 0.3, 0.001, 11353), (64, 40.0, 0.3, 0.001, 11353), (48, 100.0, 0.2, 0.0015, 7),
         (128, 10.0, 0.3, 0.001, 11353), (32, 75.0, 0.5, 0.001, 9), (80, 0.0, 0.3, 0.001, 11353)]


@pytest.mark.parametrize("lat,ham", [("square", HAM0), ("triangular", HAM1)])
def test_batch_replicas_match_oracle(ora, lat, ham):
    import paper_1901_11350_amd as pk

    announce(f"batch vs oracle {lat}")
    b, inits = _make(pk, lat, ham, SPECS, chunk=4)
    b.run(7)      # one graph replay + 3 direct steps (odd: buffers swap)
    b.run(6)      # graph re-captured for the new parity
    assert b.step == 13
    for r, (L, T, alpha, dt, seed) in enumerate(SPECS):
        n_sites, resident = b.info(r)
        assert resident == (L in (32, 64))
        s = ora.System(_geo(lat, L), ham)
        n_ora, _ = s.run(inits[r], alpha, dt, 13, T=T, seed=seed, replica=r)
        assert_close(b.get_spins(r), n_ora, "f32", what=f"replica {r} L={L} T={T}")


def test_batch_equals_single_engine_runs():
    """A tiled replica equals the single-engine run with the same tile
    configuration and Philox replica index bit for bit; resident replicas
    agree to FP32 rounding."""
    import paper_1901_11350_amd as pk

    announce("batch vs single engine")
    specs = [(32, 30.0, 0.3, 0.001, 5), (96, 30.0, 0.3, 0.001, 5), (64, 0.0, 0.3, 0.001, 5)]
    b, inits = _make(pk, "square", HAM0, specs, chunk=8)
    b.run(16)
    for r, (L, T, alpha, dt, seed) in enumerate(specs):
        e = pk.Engine(0, "f32")
        e.set_geometry(_geo("square", L))
        e.set_hamiltonian(HAM0)
        e.step_path = "shape2d/32x16x512"
        e.set_spins(inits[r])
        e.run(alpha, dt, 16, T=T, seed=seed, replica=r)
        single = e.get_spins()
        got = b.get_spins(r)
        if L in (32, 64):
            assert np.abs(got - single).max() <= 2e-6
        else:
            assert np.array_equal(got, single), np.abs(got - single).max()


def test_batch_autotune_restores_state(ora):
    import paper_1901_11350_amd as pk

    announce("batch autotune")
    specs = [(32, 10.0, 0.3, 0.001, 1), (128, 10.0, 0.3, 0.001, 1), (200, 0.0, 0.3, 0.001, 1)]
    b, inits = _make(pk, "square", HAM0, specs, chunk=2)
    b.run(2)
    before = [b.get_spins(r) for r in range(len(specs))]
    ms = b.autotune(8)
    assert ms > 0
    assert b.step == 2
    for r in range(len(specs)):
        assert np.array_equal(b.get_spins(r), before[r])
    b.run(4)
    for r, (L, T, alpha, dt, seed) in enumerate(specs):
        s = ora.System(_geo("square", L), HAM0)
        n_ora, _ = s.run(inits[r], alpha, dt, 6, T=T, seed=seed, replica=r)
        assert_close(b.get_spins(r), n_ora, "f32", what=f"replica {r}")


def test_batch_rejects_mixed_or_unsupported_replicas():
    import paper_1901_11350_amd as pk

    announce("batch errors")
    b = pk.Batch(0)
    e = pk.Engine(0, "f32")
    e.set_geometry(si.square(32, 32))
    e.set_hamiltonian(HAM0)
    e.set_spins(si.uniform_sphere(e.N, 1))
    b.add(e, 0.3, 0.001)
    e2 = pk.Engine(0, "f32")
    e2.set_geometry(si.square(32, 32))
    e2.set_hamiltonian(dataclasses.replace(HAM0, J=(1.5,)))
    e2.set_spins(si.uniform_sphere(e2.N, 1))
    with pytest.raises(pk.SpError) as ei:
        b.add(e2, 0.3, 0.001)
    assert ei.value.code == pk.SP_E_ARG
    e3 = pk.Engine(0, "f64")
    e3.set_geometry(si.square(32, 32))
    e3.set_hamiltonian(HAM0)
    e3.set_spins(si.uniform_sphere(e3.N, 1))
    with pytest.raises(pk.SpError) as ei:
        b.add(e3, 0.3, 0.001)
    assert ei.value.code == pk.SP_E_UNSUPPORTED
    b.run(2)
    with pytest.raises(pk.SpError) as ei:
        b.add(e, 0.3, 0.001)
    assert ei.value.code == pk.SP_E_ORDER
    with pytest.raises(pk.SpError):
        b.set_chunk(3)


def _chain(pk, L=48, M=10):
    e = pk.Engine(0, "f32")
    geo = si.square(L, L)
    e.set_geometry(geo)
    e.set_hamiltonian(HAM0)
    a = si.skyrmion_ansatz(geo, radius=4.0, width=1.5)
    c = si.geodesic_chain(a, si.ferromagnet(geo.n_sites, (0, 0, 1)), M, fallback_axis=(1, 0, 0))
    return e, c


def test_batch_advances_an_attached_gneb_chain():
    """A chain attached to a batch (its chunk of iterations a graph launched
    beside the replicas' chunk graph; a side branch of the direct chunks)
    ends bit-identical to the same chain iterated on its own, through graph
    replays, a re-capture and direct chunks; the replicas are the same as in
    a batch without the chain."""
    import paper_1901_11350_amd as pk
    from paper_1901_11350_amd.engine import SpError

    announce("batch + attached GNEB chain")
    e1, c = _chain(pk)
    g1 = pk.Gneb(e1, c, k_spring=1.0, vp_dt=0.1)
    e2, _ = _chain(pk)
    g2 = pk.Gneb(e2, c, k_spring=1.0, vp_dt=0.1)
    b, _ = _make(pk, "square", HAM0, SPECS, chunk=4)
    ref, _ = _make(pk, "square", HAM0, SPECS, chunk=4)
    g1.iterate(3)                       # the chain may have a history before it is attached
    g2.iterate(3)
    b.add_gneb(g1)
    with pytest.raises(SpError):
        g1.iterate(1)                   # the batch advances it now
    with pytest.raises(SpError):
        b.add_gneb(g2)                  # one chain per batch
    for n in (9, 6, 3):                 # replays + direct steps, a parity change, direct only
        b.run(n)
        ref.run(n)
        g2.iterate(n)
    assert np.array_equal(g1.chain(), g2.chain())
    f1, f2 = g1.forces(), g2.forces()
    assert np.array_equal(f1["E"], f2["E"]) and np.array_equal(f1["F"], f2["F"])
    for r in range(len(SPECS)):
        assert np.array_equal(b.get_spins(r), ref.get_spins(r))
    # destroying the chain detaches it; the batch keeps running
    g1.close()
    b.run(4)
    ref.run(4)
    assert np.array_equal(b.get_spins(0), ref.get_spins(0))


def test_attached_chain_survives_the_batch_and_fp64_is_refused():
    import paper_1901_11350_amd as pk
    from paper_1901_11350_amd.engine import SpError

    announce("batch + GNEB detach and refusals")
    e1, c = _chain(pk, L=32, M=6)
    g1 = pk.Gneb(e1, c)
    b, _ = _make(pk, "square", HAM0, SPECS[:2], chunk=2)
    b.add_gneb(g1)
    b.run(4)
    x = g1.chain()
    b.close()                           # detaches: the chain runs on its own again
    g1.iterate(2)
    assert not np.array_equal(g1.chain(), x)
    e64 = pk.Engine(0, "f64")
    e64.set_geometry(si.square(32, 32))
    e64.set_hamiltonian(HAM0)
    g64 = pk.Gneb(e64, c)
    b2, _ = _make(pk, "square", HAM0, SPECS[:1], chunk=2)
    with pytest.raises(SpError):
        b2.add_gneb(g64)
