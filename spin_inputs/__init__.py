"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This package holds no arithmetic of the spin method itself: it only
describes workloads (lattice, Hamiltonian parameters, dynamics parameters)
and draws seeded initial spin textures with NumPy's PCG64 generator.
Both the oracle and the HIP engine receive exactly these arrays.

Spin arrays are structure-of-arrays, shape (3, N), float64, with the site
index ``i = a + Na*(b + Nb*(c + Nc*beta))`` (cell a, b, c; basis atom beta).
"""

from .workloads import (  # noqa: F401
    Geometry,
    Hamiltonian,
    Dynamics,
    Workload,
    WORKLOADS,
    square,
    triangular,
    simple_cubic,
    honeycomb,
    kagome,
    fcc_primitive,
    DMI_BULK,
    DMI_INTERFACIAL,
)
from .generators import (  # noqa: F401
    uniform_sphere,
    conical_helix,
    skyrmion_ansatz,
    domain_walls,
    geodesic_chain,
    ferromagnet,
    spin_spiral,
    site_coords,
)
