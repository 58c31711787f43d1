"""Workload descriptions: lattice geometry, Hamiltonian and dynamics parameters.

Units throughout: meV (energies, J, D, K), Tesla (B), Bohr magnetons (mu),
Angstrom (lattice constant), picoseconds (dt), Kelvin (T).

The named workloads are the five benchmark configurations of this project
plus a beyond-cache square-lattice probe; their parameters are listed in
the project's design notes together with the readings taken where the
source paper leaves a value open (dt, boundaries, damping of some configs).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

DMI_BULK = 1
DMI_INTERFACIAL = 2


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Bravais lattice with basis (rows of ``bravais`` are a1, a2, a3 in units
    of the lattice constant; ``basis`` holds cartesian basis positions in the
    same units)."""

    bravais: Tuple[Tuple[float, float, float], ...]
    basis: Tuple[Tuple[float, float, float], ...]
    n_cells: Tuple[int, int, int]
    periodic: Tuple[int, int, int]
    lattice_constant: float = 1.0

    @property
    def n_basis(self) -> int:
        return len(self.basis)

    @property
    def n_sites(self) -> int:
        na, nb, nc = self.n_cells
        return na * nb * nc * self.n_basis

    def with_cells(self, n_cells, periodic=None) -> "Geometry":
        return dataclasses.replace(
            self, n_cells=tuple(n_cells),
            periodic=tuple(periodic) if periodic is not None else self.periodic)


@dataclasses.dataclass(frozen=True)
class Hamiltonian:
    """Extended Heisenberg Hamiltonian parameters (per basis atom for mu, K
    and K_axis; per neighbour shell for J and D)."""

    mu: Tuple[float, ...]
    B: Tuple[float, float, float]
    K: Tuple[float, ...]
    K_axis: Tuple[Tuple[float, float, float], ...]
    J: Tuple[float, ...] = ()
    D: Tuple[float, ...] = ()
    dmi_kind: int = DMI_INTERFACIAL
    # dipole-dipole term: False/0 off; True/1 direct pair sum; the engine also
    # takes 2 (learned surrogate with residual check) and 3 (FFT convolution),
    # which define the same field
    ddi: int = False
    # on-site Gaussian potentials ((a, sigma, (cx, cy, cz)), ...) on every site
    gauss: Tuple[Tuple[float, float, Tuple[float, float, float]], ...] = ()


@dataclasses.dataclass(frozen=True)
class Dynamics:
    alpha: float
    dt: float           # ps
    T: float = 0.0      # K
    seed: int = 0
    n_steps: int = 1
    observe_every: int = 0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    geometry: Geometry
    hamiltonian: Hamiltonian
    dynamics: Dynamics
    precision: str          # "f32" or "f64"
    init: str               # name of the initial-state recipe
    init_seed: int
    description: str = ""


def square(n_a: int, n_b: int, periodic=(1, 1, 0)) -> Geometry:
    return Geometry(((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)),
                    ((0.0, 0.0, 0.0),), (n_a, n_b, 1), tuple(periodic))


def triangular(n_a: int, n_b: int, periodic=(1, 1, 0)) -> Geometry:
    return Geometry(((1.0, 0.0, 0.0), (0.5, math.sqrt(3.0) / 2.0, 0.0), (0.0, 0.0, 1.0)),
                    ((0.0, 0.0, 0.0),), (n_a, n_b, 1), tuple(periodic))


def honeycomb(n_a: int, n_b: int, periodic=(1, 1, 0)) -> Geometry:
    """Triangular Bravais lattice with a two-atom basis (nearest-neighbour
    distance 1/sqrt(3))."""
    return Geometry(((1.0, 0.0, 0.0), (0.5, math.sqrt(3.0) / 2.0, 0.0), (0.0, 0.0, 1.0)),
                    ((0.0, 0.0, 0.0), (0.5, math.sqrt(3.0) / 6.0, 0.0)), (n_a, n_b, 1), tuple(periodic))


def kagome(n_a: int, n_b: int, periodic=(1, 1, 0)) -> Geometry:
    """Triangular Bravais lattice with a three-atom basis (corner-sharing
    triangles, nearest-neighbour distance 1/2)."""
    return Geometry(((1.0, 0.0, 0.0), (0.5, math.sqrt(3.0) / 2.0, 0.0), (0.0, 0.0, 1.0)),
                    ((0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (0.25, math.sqrt(3.0) / 4.0, 0.0)), (n_a, n_b, 1),
                    tuple(periodic))


def fcc_primitive(n_a: int, n_b: int, n_c: int, periodic=(1, 1, 1)) -> Geometry:
    """Face-centred cubic lattice on its primitive (one-atom) cell."""
    return Geometry(((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)),
                    ((0.0, 0.0, 0.0),), (n_a, n_b, n_c), tuple(periodic))


def simple_cubic(n_a: int, n_b: int, n_c: int, periodic=(1, 1, 1)) -> Geometry:
    return Geometry(((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)),
                    ((0.0, 0.0, 0.0),), (n_a, n_b, n_c), tuple(periodic))


def _one_basis(mu: float, B: Sequence[float], K: float, J, D, dmi_kind, ddi=False) -> Hamiltonian:
    return Hamiltonian(mu=(mu,), B=tuple(B), K=(K,), K_axis=((0.0, 0.0, 1.0),),
                       J=tuple(J), D=tuple(D), dmi_kind=dmi_kind, ddi=ddi)


# Square 32x32 ferromagnet-with-DMI, FP64, 1000 damped steps at T=0.
CFG0_HAM = _one_basis(2.0, (0.0, 0.0, 1.0), 0.1, (1.0,), (0.3,), DMI_INTERFACIAL)

WORKLOADS = {
    "square32_fp64": Workload(
        "square32_fp64", square(32, 32), CFG0_HAM,
        Dynamics(alpha=0.3, dt=0.001, T=0.0, seed=11350, n_steps=1000, observe_every=100),
        "f64", "uniform_sphere", 11350,
        "2D square 32x32 periodic, J=1, interfacial D=0.3, K=0.1 z, B=1 T z, mu=2, T=0"),
    "triangular512_sllg": Workload(
        "triangular512_sllg", triangular(512, 512),
        _one_basis(2.0, (0.0, 0.0, 0.5), 0.05, (1.0, -0.2, -0.1), (0.2,), DMI_INTERFACIAL),
        Dynamics(alpha=0.1, dt=0.0005, T=10.0, seed=11351, n_steps=10000, observe_every=100),
        "f32", "uniform_sphere", 11351,
        "2D triangular 512x512 periodic, J1..J3 = 1,-0.2,-0.1, interfacial D=0.2, "
        "K=0.05, B=0.5 T, stochastic LLG T=10 K"),
    "cubic128_bulkdmi": Workload(
        "cubic128_bulkdmi", simple_cubic(128, 128, 128),
        _one_basis(2.0, (0.0, 0.0, 0.3), 0.0, (1.0, 0.1), (0.15,), DMI_BULK),
        Dynamics(alpha=0.5, dt=0.001, T=0.0, seed=11352, n_steps=1000, observe_every=100),
        "f32", "conical_helix", 11352,
        "3D simple cubic 128^3 periodic, J1=1, J2=0.1, bulk D=0.15, B=0.3 T"),
    "film128x4_dipolar": Workload(
        "film128x4_dipolar", simple_cubic(128, 128, 4, periodic=(0, 0, 0)),
        _one_basis(2.0, (0.0, 0.0, 0.2), 0.2, (1.0,), (), DMI_INTERFACIAL, ddi=True),
        Dynamics(alpha=0.3, dt=0.001, T=0.0, seed=11354, n_steps=5000, observe_every=100),
        "f32", "skyrmion_ansatz", 11354,
        "simple-cubic film 128x128x4, open boundaries, J=1, K=0.2, B=0.2 T, "
        "full dipole-dipole"),
    "square8192_probe": Workload(
        "square8192_probe", square(8192, 8192), CFG0_HAM,
        Dynamics(alpha=0.3, dt=0.001, T=0.0, seed=11355, n_steps=100, observe_every=0),
        "f32", "uniform_sphere", 11355,
        "square 8192x8192 periodic (beyond the last-level cache), square32 Hamiltonian"),
}


def batch_replica_table(n_replicas: int = 96, seed: int = 11353):
    """Replica table for the batched workload: side lengths drawn uniformly
    from {32, 64, 128, 256} and temperatures uniformly from [0, 100] K."""
    import numpy as np

    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.choice(np.array([32, 64, 128, 256]), size=n_replicas)
    temps = rng.uniform(0.0, 100.0, size=n_replicas)
    return [(int(s), float(t)) for s, t in zip(sides, temps)]


def describe(w: Workload) -> dict:
    return {"workload": w.name, "n_sites": w.geometry.n_sites, "precision": w.precision,
            "description": w.description}


def get(name: str) -> Workload:
    return WORKLOADS[name]


Optional  # re-export for type hints in callers
