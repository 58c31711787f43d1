"""Pins of the oracle's Metropolis Monte Carlo (Sec. III.B: every spin picked
once per sweep, sequentially in random order, cone trial steps, adaptive
cone): the local energy change against the full energy difference, the
visiting order as a uniformly random permutation, Boltzmann statistics of
non-interacting spins in a field (Langevin function) and with uniaxial
anisotropy (a one-dimensional integral), of an interacting pair (Langevin
function of the pair coupling), the cone trial distribution, the adaptive
cone's feedback and its fixed point, and order/disorder of the cubic
ferromagnet."""

import math

import numpy as np
import pytest
from scipy.integrate import quad

import spin_inputs as si

MU_B = 9.2740100783e-24 / 1.602176634e-22
K_B = 1.380649e-23 / 1.602176634e-22

GAUSS = ((-0.5, 0.2, (0.3, 0.1, 0.9)), (0.4, 0.3, (-1.0, 0.5, 0.0)))


@pytest.mark.parametrize("dmi", [si.DMI_BULK, si.DMI_INTERFACIAL])
def test_delta_energy_matches_energy_difference(ora, dmi):
    geo = si.simple_cubic(6, 4, 4, periodic=(1, 1, 0))
    ham = si.Hamiltonian(mu=(2.0,), B=(0.3, -0.2, 0.5), K=(0.2,), K_axis=((0.6, 0, 0.8),), J=(1.0,), D=(0.3,),
                         dmi_kind=dmi, gauss=GAUSS)
    s = ora.System(geo, ham)
    n = si.uniform_sphere(s.N, 3)
    rng = np.random.default_rng(0)
    E0 = s.energy(n)
    for i in rng.choice(s.N, 12, replace=False):
        nn = rng.standard_normal(3)
        nn /= np.linalg.norm(nn)
        m = n.copy()
        m[:, i] = nn
        assert s.mc_delta_energy(n, i, nn) == pytest.approx(s.energy(m) - E0, abs=1e-12 * abs(E0))


def _paramagnet(ora, ham, T, cone, sweeps=1500, burn=200, L=32):
    geo = si.simple_cubic(L, L, 2, periodic=(0, 0, 0))
    s = ora.System(geo, ham)
    n = si.uniform_sphere(s.N, 1)
    n, _, _ = s.mc_run(n, T, cone, burn, seed=3)
    n, obs, acc = s.mc_run(n, T, cone, sweeps, seed=3, sweep0=burn, observe_every=10)
    return s, n, obs, acc / (sweeps * s.N)


@pytest.mark.parametrize("B,T,expect", [(10.0, 10.0, 0.401776), (10.0, 100.0, 0.044727)])
def test_paramagnet_samples_the_langevin_function(ora, B, T, expect):
    mu = 2.0
    x = mu * MU_B * B / (K_B * T)
    assert 1 / math.tanh(x) - 1 / x == pytest.approx(expect, abs=2e-6)
    ham = si.Hamiltonian(mu=(mu,), B=(0, 0, B), K=(0.0,), K_axis=((0, 0, 1),))
    _, _, obs, rate = _paramagnet(ora, ham, T, 60.0)
    assert np.mean([o["M"][2] for o in obs]) == pytest.approx(expect, abs=0.006)
    assert 0.05 < rate < 1.0


def test_uniaxial_anisotropy_boltzmann_average(ora):
    """<(n.k)^2> of free spins with E = -K (n.k)^2 at temperature T equals
    int x^2 exp(b x^2) / int exp(b x^2) over x in [-1, 1], b = K / (k_B T)."""
    K, T = 0.5, 4.0
    b = K / (K_B * T)
    num = quad(lambda x: x * x * math.exp(b * x * x), -1, 1)[0]
    den = quad(lambda x: math.exp(b * x * x), -1, 1)[0]
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(K,), K_axis=((0, 0, 1),))
    s, n, obs, _ = _paramagnet(ora, ham, T, 90.0, sweeps=600, burn=100)
    assert np.mean(n[2] ** 2) == pytest.approx(num / den, abs=0.01)


def test_cone_trials_without_energy_are_always_accepted_and_uniform(ora):
    """With no Hamiltonian terms every trial is accepted; from n = z one sweep
    leaves cos(theta) = n_z uniform in [cos(cone), 1] and phi uniform."""
    geo = si.simple_cubic(64, 64, 2, periodic=(0, 0, 0))
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),))
    s = ora.System(geo, ham)
    n0 = si.ferromagnet(s.N, (0, 0, 1))
    cone = 40.0
    n, _, acc = s.mc_run(n0, 5.0, cone, 1, seed=9)
    assert acc == s.N
    c = math.cos(math.radians(cone))
    assert n[2].min() >= c - 1e-15 and n[2].max() <= 1.0
    assert np.mean(n[2]) == pytest.approx((1 + c) / 2, abs=3e-3 * (1 - c))
    assert np.var(n[2]) == pytest.approx((1 - c) ** 2 / 12, rel=0.03)
    assert abs(np.mean(n[0])) < 0.01 and abs(np.mean(n[1])) < 0.01
    assert np.allclose(np.linalg.norm(n, axis=0), 1.0, atol=1e-14)


def test_ferromagnet_orders_below_and_disorders_above_tc(ora):
    """Simple-cubic ferromagnet J = 1 meV (Tc = 1.44 J/k_B = 16.7 K): |M|
    stays near 1 far below Tc and falls to the 1/sqrt(N) level far above."""
    geo = si.simple_cubic(8, 8, 8)
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), J=(1.0,))
    s = ora.System(geo, ham)
    res = {}
    for T in (4.0, 40.0):
        n, _, _ = s.mc_run(si.ferromagnet(s.N, (0, 0, 1)), T, 60.0, 300, seed=5)
        n, obs, _ = s.mc_run(n, T, 60.0, 300, seed=5, sweep0=300, observe_every=5)
        res[T] = np.mean([np.linalg.norm(o["M"]) for o in obs])
    assert res[4.0] > 0.85
    assert res[40.0] < 0.12


def test_sweep_takes_any_lattice_but_not_the_dipole_term(ora):
    """The sequential sweep needs no colouring: odd rings, odd periodic
    lengths, bonds within a colour and a two-atom basis all sweep; the
    dipole term (not local) is rejected."""
    nn = si.Hamiltonian(mu=(2.0,), B=(0, 0, 1.0), K=(0.0,), K_axis=((0, 0, 1),), J=(1.0,))
    nnn = si.Hamiltonian(mu=(2.0,), B=(0, 0, 1.0), K=(0.0,), K_axis=((0, 0, 1),), J=(1.0, 0.5))
    two = si.Geometry(((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((0, 0, 0), (0.5, 0.5, 0)), (4, 4, 1), (1, 1, 0))
    ham2 = si.Hamiltonian(mu=(2.0, 1.0), B=(0, 0, 1.0), K=(0.0, 0.1), K_axis=((0, 0, 1), (0, 0, 1)), J=(1.0,))
    for geo, ham in [(si.triangular(8, 8), nn), (si.simple_cubic(5, 4, 4), nn), (si.square(8, 8), nnn),
                     (two, ham2)]:
        s = ora.System(geo, ham)
        n, _, acc = s.mc_run(si.uniform_sphere(s.N, 1), 5.0, 30.0, 2)
        assert 0 < acc <= 2 * s.N
        assert np.allclose(np.linalg.norm(n, axis=0), 1.0, atol=1e-14)
    film = ora.System(si.simple_cubic(4, 4, 1, periodic=(0, 0, 0)),
                      si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), ddi=1))
    with pytest.raises(ValueError):
        film.mc_run(si.uniform_sphere(film.N, 1), 5.0, 30.0, 1)


def test_visiting_order_is_a_uniform_random_permutation(ora):
    """Each sweep visits every site exactly once; over many sweeps every
    site is equally likely at every position (chi-square over the position
    of two sites), and the orders of different sweeps, seeds and replicas
    differ."""
    N, sweeps = 37, 20000
    pos = np.zeros((2, N))
    for t in range(sweeps):
        o = ora.mc_order(N, 11, t)
        assert np.array_equal(np.sort(o), np.arange(N))
        pos[0, np.flatnonzero(o == 0)[0]] += 1
        pos[1, np.flatnonzero(o == N - 1)[0]] += 1
    expect = sweeps / N
    for row in pos:
        chi2 = float(((row - expect) ** 2 / expect).sum())
        assert chi2 < 80.0      # 36 degrees of freedom: p ~ 5e-5
    assert not np.array_equal(ora.mc_order(N, 11, 0), ora.mc_order(N, 11, 1))
    assert not np.array_equal(ora.mc_order(N, 11, 0), ora.mc_order(N, 12, 0))
    assert not np.array_equal(ora.mc_order(N, 11, 0, 1), ora.mc_order(N, 11, 0, 0))


def test_interacting_pair_samples_the_langevin_function_of_its_coupling(ora):
    """Two sites on a periodic chain of length 2 are bonded twice (through
    +a and -a), so E = -2 J n1.n2 and <n1.n2> = L(2 J / k_B T) with
    L(x) = coth x - 1/x: an exact pin of the Boltzmann weight of an
    interacting system, the pair counting and the sequential updates."""
    J, T = 1.0, 20.0
    geo = si.simple_cubic(2, 1, 1, periodic=(1, 0, 0))
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), J=(J,))
    s = ora.System(geo, ham)
    x = 2 * J / (K_B * T)
    expect = 1 / math.tanh(x) - 1 / x
    n, _, _ = s.mc_run(si.uniform_sphere(2, 4), T, 90.0, 2000, seed=21)
    vals = []
    for k in range(40):
        n, obs, _ = s.mc_run(n, T, 90.0, 5000, seed=21, sweep0=2000 + 5000 * k, observe_every=1)
        # E = -2 J n1.n2 for this system
        vals.append(np.mean([-o["E"] / (2 * J) for o in obs]))
    mean, err = np.mean(vals), np.std(vals) / math.sqrt(len(vals))
    assert abs(mean - expect) < max(4 * err, 2e-3), (mean, err, expect)


def test_adaptive_cone_feedback(ora):
    """The cone grows while more than the target is accepted and shrinks
    while fewer are (multiplied by 1 + a - a*, capped at 180 degrees); a run
    with the feedback settles where the acceptance equals the target."""
    assert ora.mc_adapt_cone(30.0, 0.7, 0.5) == pytest.approx(36.0, rel=1e-15)
    assert ora.mc_adapt_cone(30.0, 0.2, 0.5) == pytest.approx(21.0, rel=1e-15)
    assert ora.mc_adapt_cone(170.0, 1.0, 0.5) == 180.0
    assert ora.mc_adapt_cone(30.0, 0.2, 0.0) == 30.0
    geo = si.simple_cubic(8, 8, 8)
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), J=(1.0,))
    s = ora.System(geo, ham)
    for start in (5.0, 150.0):
        n, _, _, cone = s.mc_run(si.ferromagnet(s.N, (0, 0, 1)), 10.0, start, 400, seed=2,
                                 target_acceptance=0.5, return_cone=True)
        n, _, acc = s.mc_run(n, 10.0, cone, 200, seed=2, sweep0=400)
        assert acc / (200 * s.N) == pytest.approx(0.5, abs=0.03), (start, cone)
