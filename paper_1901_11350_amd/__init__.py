"""MI355X-native hot path of atomistic spin dynamics (arXiv:1901.11350).

``Engine`` wraps the C ABI of ``libsp_engine.so`` (hand-written HIP
kernels for gfx950): effective field of the extended Heisenberg
Hamiltonian, Depondt LLG steps with a Philox thermal field, dipole-dipole
direct sum, and double-precision observables.
"""

from .engine import (  # noqa: F401
    Batch,
    Engine,
    Gneb,
    close_all,
    SpError,
    engine_for,
    lib,
    EXPORTS,
    LIB_PATH,
    SP_OK,
    SP_E_ARG,
    SP_E_ORDER,
    SP_E_HIP,
    SP_E_NOMEM,
    SP_E_UNSUPPORTED,
    SP_E_NONFINITE,
)
