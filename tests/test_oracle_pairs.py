"""Pins of the oracle's explicit pair interactions (``ora_set_pairs``).

The Hamiltonian's exchange and DMI sums run over unique pairs <ij> of any
number, range and direction dependence (Sec. III.A).  The pins:
  * the shell-built bond table, written out as one entry per unique pair,
    reproduces the shell system's energy and gradient (the shell path is
    pinned by brute force elsewhere), so the expansion of a pair into two
    directed bonds (reverse bond with -D) is right;
  * long-range, direction-dependent pairs with arbitrary DMI vectors on tiny
    periodic and open lattices against a brute-force sum written directly
    from the pair form of the Hamiltonian (partner cell x + d wrapped on
    periodic axes, dropped on open ones, a pair onto its own site dropped),
    and the gradient against central differences of that sum;
  * rejected lists leave the system unchanged; an empty list removes the
    exchange and DMI terms."""

import dataclasses
import math

import numpy as np
import pytest

import spin_inputs as si

MU_B = 9.2740100783e-24 / 1.602176634e-22   # meV/T (CODATA 2018, SI values)
HAM = si.Hamiltonian(mu=(2.0,), B=(0.1, -0.3, 0.8), K=(0.2,), K_axis=((0, 0, 1),),
                     J=(1.0, -0.25, 0.1), D=(0.3,), dmi_kind=si.DMI_INTERFACIAL)


def _unique_pairs(bonds):
    """One entry per unique pair out of a directed bond table."""
    table = {(b[0], b[1], b[2], b[3], b[4]): b for b in bonds}
    out = []
    for key, b in table.items():
        rkey = (b[1], b[0], -b[2], -b[3], -b[4])
        assert rkey in table
        r = table[rkey]
        assert r[6] == b[6] and np.allclose(r[7], -np.asarray(b[7]), atol=0.0)
        if key < rkey:
            out.append((b[0], b[1], (b[2], b[3], b[4]), b[6], b[7]))
    return out


@pytest.mark.parametrize("case", ["tri6x5", "sq5x4_open", "basis2_3d"])
def test_shell_table_as_pairs_reproduces_shell_system(ora, case):
    if case == "tri6x5":
        geo, ham = si.triangular(6, 5), HAM
    elif case == "sq5x4_open":
        geo, ham = si.square(5, 4, periodic=(0, 1, 0)), dataclasses.replace(HAM, J=(1.0, 0.4), D=(0.2, 0.1))
    else:
        geo = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0.5, 0.5, 0.5)),
                          (4, 3, 3), (1, 1, 0))
        ham = si.Hamiltonian(mu=(2.0, 3.0), B=(0.2, 0.4, -0.3), K=(0.1, -0.2),
                             K_axis=((0, 0, 1), (0.6, 0.8, 0.0)), J=(1.0, 0.5), D=(0.1, 0.05),
                             dmi_kind=si.DMI_BULK)
    a = ora.System(geo, ham)
    pairs = _unique_pairs(a.bonds())
    assert 2 * len(pairs) == len(a.bonds())
    b = ora.System(geo, dataclasses.replace(ham, J=(), D=()))
    b.set_pairs(pairs)
    n = si.uniform_sphere(a.N, 3)
    assert b.energy(n) == pytest.approx(a.energy(n), rel=1e-13, abs=1e-12)
    np.testing.assert_allclose(b.gradient(n), a.gradient(n), rtol=0, atol=1e-12)


def _site(geo, a, b, c, beta):
    na, nb, nc = geo.n_cells
    return a + na * (b + nb * (c + nc * beta))


def brute_pair_energy(geo, ham, pairs, n):
    """Zeeman + anisotropy + the pair sums, straight from the definition:
    for every cell x and every listed pair, partner cell x + d (wrapped on
    periodic axes, absent past an open edge), a pair onto its own site
    skipped."""
    N = geo.n_sites
    cells = geo.n_cells[0] * geo.n_cells[1] * geo.n_cells[2]
    E = 0.0
    for i in range(N):
        beta = i // cells
        E -= ham.mu[beta] * MU_B * float(np.dot(ham.B, n[:, i]))
        E -= ham.K[beta] * float(np.dot(ham.K_axis[beta], n[:, i])) ** 2
    for a in range(geo.n_cells[0]):
        for b in range(geo.n_cells[1]):
            for c in range(geo.n_cells[2]):
                for bi, bj, d, J, D in pairs:
                    t = [a + d[0], b + d[1], c + d[2]]
                    ok = True
                    for k in range(3):
                        if not 0 <= t[k] < geo.n_cells[k]:
                            if geo.periodic[k]:
                                t[k] %= geo.n_cells[k]
                            else:
                                ok = False
                    if not ok:
                        continue
                    i = _site(geo, a, b, c, bi)
                    j = _site(geo, t[0], t[1], t[2], bj)
                    if i == j:
                        continue
                    E -= J * float(np.dot(n[:, i], n[:, j]))
                    E -= float(np.dot(D, np.cross(n[:, i], n[:, j])))
    return E


LONG_PAIRS = [
    (0, 0, (1, 0, 0), 1.0, (0.1, -0.2, 0.3)),     # anisotropic exchange: a1 and a2 differ
    (0, 0, (0, 1, 0), 0.4, (0.0, 0.0, 0.0)),
    (0, 0, (2, -1, 0), -0.3, (0.05, 0.02, -0.1)),
    (0, 0, (7, 0, 0), 0.2, (0.0, 0.3, 0.0)),      # beyond the shell search range, wraps past the lattice
    (0, 0, (5, 2, 0), 0.15, (0.0, 0.0, 0.2)),     # 5 cells along a1 of a 5-cell periodic axis
    (0, 0, (0, 6, 0), -0.1, (0.0, 0.0, 0.0)),     # wraps onto the site itself (3-cell periodic axis): dropped
]


@pytest.mark.parametrize("case", ["periodic", "open_a", "basis2"])
def test_long_range_pairs_against_brute_force(ora, case):
    if case == "basis2":
        geo = si.Geometry(((1.0, 0, 0), (0, 1.0, 0), (0, 0, 1.0)), ((0, 0, 0), (0.3, 0.4, 0.5)),
                          (4, 3, 2), (1, 1, 0))
        ham = si.Hamiltonian(mu=(2.0, 1.5), B=(0.2, 0.1, 0.5), K=(0.1, 0.3), K_axis=((0, 0, 1), (1, 0, 0)))
        pairs = [(0, 1, (0, 0, 0), 0.8, (0.1, 0.0, -0.2)),
                 (1, 0, (1, 0, 0), 0.3, (0.0, 0.2, 0.0)),
                 (0, 0, (3, 1, 1), -0.2, (0.05, 0.05, 0.05)),
                 (1, 1, (0, 2, -1), 0.5, (0.0, 0.0, 0.0)),
                 (0, 1, (-5, 0, 1), 0.1, (0.2, -0.1, 0.0))]
    else:
        geo = si.triangular(5, 3) if case == "periodic" else si.triangular(5, 3, periodic=(0, 1, 0))
        ham = dataclasses.replace(HAM, J=(), D=())
        pairs = LONG_PAIRS
    s = ora.System(geo, ham)
    s.set_pairs(pairs)
    n = si.uniform_sphere(s.N, 11)
    E_ref = brute_pair_energy(geo, ham, pairs, n)
    assert s.energy(n) == pytest.approx(E_ref, rel=1e-13, abs=1e-12)
    # gradient: central differences of the brute-force energy along each
    # embedding component (the energy is a polynomial of degree 2 in n)
    g = s.gradient(n)
    h = 1e-5
    for i in range(s.N):
        for k in range(3):
            npl, nmi = n.copy(), n.copy()
            npl[k, i] += h
            nmi[k, i] -= h
            fd = (brute_pair_energy(geo, ham, pairs, npl) - brute_pair_energy(geo, ham, pairs, nmi)) / (2 * h)
            assert g[k, i] == pytest.approx(fd, abs=1e-7)


def test_pair_lists_rejected_and_empty(ora):
    geo = si.triangular(6, 5)
    s = ora.System(geo, HAM)
    n = si.uniform_sphere(s.N, 2)
    E0 = s.energy(n)
    for bad in ([(0, 0, (0, 0, 0), 1.0, (0, 0, 0))],                                   # self pair
                [(0, 1, (1, 0, 0), 1.0, (0, 0, 0))],                                   # basis index
                [(0, 0, (1, 0, 0), 1.0, (0, 0, 0)), (0, 0, (1, 0, 0), 0.5, (0, 0, 0))],  # repeated
                [(0, 0, (1, 0, 0), 1.0, (0, 0, 0)), (0, 0, (-1, 0, 0), 0.5, (0, 0, 0))]):  # reverse
        with pytest.raises(ValueError):
            s.set_pairs(bad)
        assert s.energy(n) == E0
    s.set_pairs([])
    E, terms = s.energy(n, per_term=True)
    assert E == pytest.approx(brute_pair_energy(geo, HAM, [], n), rel=1e-13)
    assert terms[2] == 0.0 and terms[3] == 0.0


def test_pair_energy_closed_form_two_spin_chain(ora):
    """Two sites on an open chain, one pair: E = -J cos(theta) - D.(n1 x n2)
    for n1 = x, n2 = (cos t, sin t, 0), D = (0, 0, Dz): -J cos t - Dz sin t."""
    geo = si.simple_cubic(2, 1, 1, periodic=(0, 0, 0))
    ham = si.Hamiltonian(mu=(1.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),))
    s = ora.System(geo, ham)
    J, Dz = 0.7, 0.3
    s.set_pairs([(0, 0, (1, 0, 0), J, (0.0, 0.0, Dz))])
    for t in np.linspace(0.0, 2 * math.pi, 9):
        n = np.array([[1.0, math.cos(t)], [0.0, math.sin(t)], [0.0, 0.0]])
        assert s.energy(n) == pytest.approx(-J * math.cos(t) - Dz * math.sin(t), abs=1e-14)
