"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and
by the benchmark's CPU-baseline leg.  The HIP engine never imports it.

The wrapper marshals NumPy arrays; the arithmetic is in ``oracle.c``,
except the composition of the surrogate network in ``SurrogateNet`` (the
layer sequence, the relative squared-error loss and the chain rule between
layers), which is plain NumPy over the C layers.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_BASIS = 8
MAX_SHELLS = 8
MAX_GAUSS = 16
MAX_BONDS = MAX_BASIS * 256


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class Geometry(ctypes.Structure):
    _fields_ = [("bravais", ctypes.c_double * 9),
                ("n_basis", ctypes.c_int),
                ("basis", ctypes.c_double * (3 * MAX_BASIS)),
                ("n_cells", ctypes.c_int * 3),
                ("periodic", ctypes.c_int * 3),
                ("lattice_constant", ctypes.c_double)]


class Hamiltonian(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double * MAX_BASIS),
                ("B", ctypes.c_double * 3),
                ("K", ctypes.c_double * MAX_BASIS),
                ("K_axis", ctypes.c_double * (3 * MAX_BASIS)),
                ("n_exch", ctypes.c_int),
                ("J", ctypes.c_double * MAX_SHELLS),
                ("n_dmi", ctypes.c_int),
                ("D", ctypes.c_double * MAX_SHELLS),
                ("dmi_kind", ctypes.c_int),
                ("ddi", ctypes.c_int),
                ("n_gauss", ctypes.c_int),
                ("gauss_a", ctypes.c_double * MAX_GAUSS),
                ("gauss_sigma", ctypes.c_double * MAX_GAUSS),
                ("gauss_c", ctypes.c_double * (3 * MAX_GAUSS))]


class Bond(ctypes.Structure):
    _fields_ = [("bi", ctypes.c_int), ("bj", ctypes.c_int), ("da", ctypes.c_int),
                ("db", ctypes.c_int), ("dc", ctypes.c_int), ("shell", ctypes.c_int),
                ("J", ctypes.c_double), ("D", ctypes.c_double * 3)]


class LLGParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("dt", ctypes.c_double), ("T", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32), ("solver", ctypes.c_int32)]


SOLVERS = {"depondt": 0, "heun": 1, "sib": 2}


class McParams(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("cone_deg", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("target_acceptance", ctypes.c_double)]


class GnebParams(ctypes.Structure):
    _fields_ = [("k_spring", ctypes.c_double), ("vp_dt", ctypes.c_double),
                ("vp_mass", ctypes.c_double), ("image_type", ctypes.POINTER(ctypes.c_int))]


IMAGE_TYPES = {"normal": 0, "climbing": 1, "falling": 2}


class Observation(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("E", ctypes.c_double),
                ("per_term", ctypes.c_double * 5), ("max_torque", ctypes.c_double),
                ("M", ctypes.c_double * 3), ("max_norm_dev", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Hamiltonian)]
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_num_sites.restype = ctypes.c_int64
        L.ora_num_sites.argtypes = [ctypes.c_void_p]
        L.ora_bonds.restype = ctypes.c_int
        L.ora_bonds.argtypes = [ctypes.c_void_p, ctypes.POINTER(Bond), ctypes.c_int]
        ci_p = ctypes.POINTER(ctypes.c_int)
        L.ora_set_pairs.restype = ctypes.c_int
        L.ora_set_pairs.argtypes = [ctypes.c_void_p, ctypes.c_int, ci_p, ci_p, ci_p,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.ora_site_neighbours.restype = ctypes.c_int
        L.ora_site_neighbours.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.ora_shell_distances.restype = ctypes.c_int
        L.ora_shell_distances.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ctypes.c_int]
        L.ora_gradient.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.ora_dipole_gradient_sites.argtypes = [ctypes.c_void_p, dp,
                                                ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        L.ora_energy.restype = ctypes.c_double
        L.ora_energy.argtypes = [ctypes.c_void_p, dp, dp]
        L.ora_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint32)]
        L.ora_thermal_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint32, dp]
        L.ora_mc_delta_energy.restype = ctypes.c_double
        L.ora_mc_delta_energy.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64, dp]
        L.ora_mc_sweep.restype = ctypes.c_int64
        L.ora_mc_sweep.argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(McParams), ctypes.c_double, ctypes.c_uint64]
        L.ora_mc_order.restype = None
        L.ora_mc_order.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.POINTER(ctypes.c_int64)]
        L.ora_mc_adapt_cone.restype = ctypes.c_double
        L.ora_mc_adapt_cone.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.ora_mc_run.restype = ctypes.c_int64
        L.ora_mc_run.argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(McParams), ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_double)]
        for name in ("ora_depondt_step", "ora_heun_step", "ora_sib_step", "ora_llg_step"):
            getattr(L, name).argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(LLGParams), ctypes.c_uint64]
        L.ora_rotate.argtypes = [dp, dp, ctypes.c_double, dp]
        L.ora_observe.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64,
                                  ctypes.POINTER(Observation)]
        L.ora_run.restype = ctypes.c_int64
        L.ora_run.argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(LLGParams), ctypes.c_uint64,
                              ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(Observation)]
        for name in ("ora_const_mu_B", "ora_const_k_B", "ora_const_gamma", "ora_const_C_dd"):
            getattr(L, name).restype = ctypes.c_double
        L.ora_gneb_forces.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ctypes.POINTER(GnebParams),
                                      dp, dp, dp, dp]
        L.ora_gneb_vp.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp,
                                  ctypes.POINTER(GnebParams), ctypes.c_int]
        L.ora_bf16.restype = ctypes.c_double
        L.ora_bf16.argtypes = [ctypes.c_double]
        L.ora_conv_set_exact.argtypes = [ctypes.c_int]
        L.ora_ddr_check.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_ddr_moments.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.ora_ddr_backbone.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp]
        L.ora_ddr_project.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.ora_ddr_expand.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp]
        ci = ctypes.c_int
        L.ora_conv3x3_fwd.argtypes = [ci, ci, ci, ci, ci, dp, dp, dp, dp]
        L.ora_conv3x3_bwd.argtypes = [ci, ci, ci, ci, ci, dp, dp, dp, dp, dp, dp]
        L.ora_silu.argtypes = [ctypes.c_int64, dp, dp, dp]
        L.ora_adam.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ci]
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_num_threads.argtypes = []
        L.ora_set_num_threads.restype = None
        L.ora_set_num_threads.argtypes = [ci]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def constants() -> dict:
    L = lib()
    return {"mu_B": L.ora_const_mu_B(), "k_B": L.ora_const_k_B(),
            "gamma": L.ora_const_gamma(), "C_dd": L.ora_const_C_dd()}


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    lib().ora_set_num_threads(int(n))


def _geometry(geo) -> Geometry:
    g = Geometry()
    for r in range(3):
        for k in range(3):
            g.bravais[3 * r + k] = geo.bravais[r][k]
    g.n_basis = len(geo.basis)
    for b, p in enumerate(geo.basis):
        for k in range(3):
            g.basis[3 * b + k] = p[k]
    for k in range(3):
        g.n_cells[k] = geo.n_cells[k]
        g.periodic[k] = geo.periodic[k]
    g.lattice_constant = geo.lattice_constant
    return g


def _hamiltonian(ham) -> Hamiltonian:
    h = Hamiltonian()
    for b, m in enumerate(ham.mu):
        h.mu[b] = m
    for k in range(3):
        h.B[k] = ham.B[k]
    for b, kk in enumerate(ham.K):
        h.K[b] = kk
    for b, ax in enumerate(ham.K_axis):
        for k in range(3):
            h.K_axis[3 * b + k] = ax[k]
    h.n_exch = len(ham.J)
    for s, j in enumerate(ham.J):
        h.J[s] = j
    h.n_dmi = len(ham.D)
    for s, d in enumerate(ham.D):
        h.D[s] = d
    h.dmi_kind = ham.dmi_kind
    h.ddi = 1 if ham.ddi else 0
    gauss = getattr(ham, "gauss", ())
    h.n_gauss = len(gauss)
    for k, (a, sg, c) in enumerate(gauss):
        h.gauss_a[k] = a
        h.gauss_sigma[k] = sg
        for q in range(3):
            h.gauss_c[3 * k + q] = c[q]
    return h


class System:
    """One oracle system (geometry + Hamiltonian); see ``oracle.h``."""

    def __init__(self, geometry, hamiltonian):
        L = lib()
        self._g = _geometry(geometry)
        self._h = _hamiltonian(hamiltonian)
        self._p = L.ora_create(ctypes.byref(self._g), ctypes.byref(self._h))
        if not self._p:
            raise ValueError("oracle rejected the geometry/Hamiltonian")
        self.N = int(L.ora_num_sites(self._p))
        self.geometry = geometry
        self.hamiltonian = hamiltonian

    def __del__(self):
        p = getattr(self, "_p", None)
        if p and _lib is not None:
            _lib.ora_destroy(p)
            self._p = None

    def _spins(self, n) -> np.ndarray:
        n = np.ascontiguousarray(n, dtype=np.float64).reshape(3, self.N)
        return n

    def bonds(self):
        buf = (Bond * MAX_BONDS)()
        k = lib().ora_bonds(self._p, buf, MAX_BONDS)
        return [(b.bi, b.bj, b.da, b.db, b.dc, b.shell, b.J, tuple(b.D)) for b in buf[:k]]

    def set_pairs(self, pairs):
        """Explicit unique pairs (bi, bj, (da, db, dc), J, (Dx, Dy, Dz)) in place
        of the shell-built exchange and DMI bonds (``ora_set_pairs``)."""
        pairs = list(pairs)
        n = len(pairs)
        bi = np.ascontiguousarray([p[0] for p in pairs] or [0], dtype=np.int32)
        bj = np.ascontiguousarray([p[1] for p in pairs] or [0], dtype=np.int32)
        dc = np.ascontiguousarray([list(p[2]) for p in pairs] or [[0, 0, 0]], dtype=np.int32).reshape(-1)
        J = np.ascontiguousarray([p[3] for p in pairs] or [0.0], dtype=np.float64)
        D = np.ascontiguousarray([list(p[4]) for p in pairs] or [[0.0, 0.0, 0.0]], dtype=np.float64).reshape(-1)
        ip = ctypes.POINTER(ctypes.c_int)
        rc = lib().ora_set_pairs(self._p, n, bi.ctypes.data_as(ip), bj.ctypes.data_as(ip), dc.ctypes.data_as(ip),
                                 _dp(J), _dp(D))
        if rc != 0:
            raise ValueError(f"oracle rejected the pair list (code {rc})")

    def neighbours(self, i: int):
        js = (ctypes.c_int64 * 512)()
        bs = (ctypes.c_int * 512)()
        d = lib().ora_site_neighbours(self._p, i, js, bs, 512)
        return list(js[:d]), list(bs[:d])

    def shell_distances(self, beta: int = 0):
        out = np.zeros(MAX_SHELLS)
        k = lib().ora_shell_distances(self._p, beta, _dp(out), MAX_SHELLS)
        return out[:k]

    def gradient(self, n, terms: bool = False):
        n = self._spins(n)
        g = np.zeros((3, self.N))
        t = np.zeros((5, 3, self.N)) if terms else None
        lib().ora_gradient(self._p, _dp(n), _dp(g), _dp(t) if terms else None)
        return (g, t) if terms else g

    def dipole_gradient_sites(self, n, sites):
        n = self._spins(n)
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.zeros((len(sites), 3))
        lib().ora_dipole_gradient_sites(self._p, _dp(n),
                                        sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        len(sites), _dp(out))
        return out.T.copy()

    def energy(self, n, per_term: bool = False):
        n = self._spins(n)
        pt = np.zeros(5)
        E = lib().ora_energy(self._p, _dp(n), _dp(pt))
        return (E, pt) if per_term else E

    def depondt_step(self, n, alpha, dt, T=0.0, seed=0, step=0, replica=0) -> np.ndarray:
        return self.llg_step(n, alpha, dt, T, seed, step, replica, "depondt")

    def llg_step(self, n, alpha, dt, T=0.0, seed=0, step=0, replica=0, solver="depondt") -> np.ndarray:
        n = self._spins(n).copy()
        p = LLGParams(alpha, dt, T, seed, replica, SOLVERS[solver])
        lib().ora_llg_step(self._p, _dp(n), ctypes.byref(p), step)
        return n

    def mc_delta_energy(self, n, i, n_new) -> float:
        n = self._spins(n)
        return lib().ora_mc_delta_energy(self._p, _dp(n), int(i), _dp(np.ascontiguousarray(n_new, dtype=np.float64)))

    def mc_run(self, n, T, cone_deg, n_sweeps, seed=0, sweep0=0, replica=0, observe_every=0,
               target_acceptance=0.0, return_cone=False):
        """Metropolis sweeps in random order (Sec. III.B); returns (spins,
        observations, accepted trials[, final cone in degrees])."""
        n = self._spins(n).copy()
        p = McParams(T, cone_deg, seed, replica, target_acceptance)
        n_obs = n_sweeps // observe_every if observe_every > 0 else 0
        obs = (Observation * max(n_obs, 1))()
        acc = ctypes.c_int64()
        cone = ctypes.c_double()
        k = lib().ora_mc_run(self._p, _dp(n), ctypes.byref(p), sweep0, n_sweeps, observe_every,
                             ctypes.cast(obs, ctypes.c_void_p), ctypes.byref(acc), ctypes.byref(cone))
        if k < 0:
            raise ValueError("Monte Carlo sweeps do not support the dipole term")
        out = (n, [_obs_dict(o) for o in obs[:k]], acc.value)
        return out + (cone.value,) if return_cone else out

    # residual form of the learned dipole field (block images [qb][qa][12])
    def _ddr_dims(self, B):
        if lib().ora_ddr_check(self._p, B) != 0:
            raise ValueError("the residual form needs a one-atom film with sides divisible by the block")
        na, nb = self.geometry.n_cells[0], self.geometry.n_cells[1]
        return nb // B, na // B

    def ddr_moments(self, n, B) -> np.ndarray:
        h, w = self._ddr_dims(B)
        out = np.zeros((h, w, 12))
        lib().ora_ddr_moments(self._p, _dp(self._spins(n)), B, _dp(out))
        return out

    def ddr_backbone(self, n, B, reach, sites=None) -> np.ndarray:
        """Backbone field (units of C_dd mu^2), shape (3, len(sites))."""
        self._ddr_dims(B)
        sites = np.arange(self.N) if sites is None else np.asarray(sites)
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.zeros((len(sites), 3))
        lib().ora_ddr_backbone(self._p, _dp(self._spins(n)), B, reach,
                               sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sites), _dp(out))
        return out.T.copy()

    def ddr_project(self, r, B) -> np.ndarray:
        h, w = self._ddr_dims(B)
        out = np.zeros((h, w, 12))
        lib().ora_ddr_project(self._p, _dp(self._spins(r)), B, _dp(out))
        return out

    def ddr_expand(self, coef, B) -> np.ndarray:
        self._ddr_dims(B)
        out = np.zeros((3, self.N))
        lib().ora_ddr_expand(self._p, _dp(np.ascontiguousarray(coef, dtype=np.float64)), B, _dp(out))
        return out

    def observe(self, n, step=0) -> dict:
        n = self._spins(n)
        o = Observation()
        lib().ora_observe(self._p, _dp(n), step, ctypes.byref(o))
        return _obs_dict(o)

    def run(self, n, alpha, dt, n_steps, T=0.0, seed=0, step0=0, replica=0,
            observe_every=0, solver="depondt"):
        n = self._spins(n).copy()
        p = LLGParams(alpha, dt, T, seed, replica, SOLVERS[solver])
        n_obs = n_steps // observe_every if observe_every > 0 else 0
        obs = (Observation * max(n_obs, 1))()
        k = lib().ora_run(self._p, _dp(n), ctypes.byref(p), step0, n_steps, observe_every, obs)
        return n, [_obs_dict(o) for o in obs[:k]]


class Gneb:
    """GNEB chain on an oracle system: forces and velocity-projection
    iterations (state: chain, velocity, previous force)."""

    def __init__(self, system: "System", chain, k_spring=1.0, vp_dt=0.1, vp_mass=1.0):
        self.s = system
        self.chain = np.ascontiguousarray(chain, dtype=np.float64).reshape(-1, 3, system.N).copy()
        self.M = self.chain.shape[0]
        self.p = GnebParams(k_spring, vp_dt, vp_mass, None)
        self._types = None
        self.v = np.zeros_like(self.chain)
        f = self.forces()
        self.F_prev = f["F"].copy()

    def forces(self, chain=None) -> dict:
        c = self.chain if chain is None else np.ascontiguousarray(chain, dtype=np.float64)
        M, N = self.M, self.s.N
        E = np.zeros(M)
        tau = np.zeros((M, 3, N))
        l = np.zeros(max(M - 1, 1))
        F = np.zeros((M, 3, N))
        lib().ora_gneb_forces(self.s._p, M, _dp(c), ctypes.byref(self.p), _dp(E), _dp(tau),
                              _dp(l), _dp(F))
        return {"E": E, "tau": tau, "l": l[: M - 1], "F": F}

    def set_image_types(self, types):
        """types: M entries of "normal", "climbing", "falling" (endpoints ignored)."""
        arr = (ctypes.c_int * self.M)(*[IMAGE_TYPES[t] for t in types])
        self._types = arr
        self.p.image_type = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int))

    def iterate(self, n_iter: int):
        lib().ora_gneb_vp(self.s._p, self.M, _dp(self.chain), _dp(self.v), _dp(self.F_prev),
                          ctypes.byref(self.p), n_iter)


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even), as doubles."""
    a = np.asarray(x, dtype=np.float64)
    f = np.vectorize(lib().ora_bf16, otypes=[np.float64])
    return f(a) if a.size else a.copy()


class conv_exact:
    """Context manager: the conv layers skip their bfloat16 rounding."""

    def __enter__(self):
        lib().ora_conv_set_exact(1)

    def __exit__(self, *a):
        lib().ora_conv_set_exact(0)


def conv3x3_fwd(x, w, b) -> np.ndarray:
    """x (B,H,W,Cin), w (3,3,Cin,Cout), b (Cout,) -> pre-activation (B,H,W,Cout)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    B, H, W, Cin = x.shape
    Cout = w.shape[3]
    z = np.zeros((B, H, W, Cout))
    lib().ora_conv3x3_fwd(B, H, W, Cin, Cout, _dp(x), _dp(w), _dp(b), _dp(z))
    return z


def conv3x3_bwd(x, w, dz, need_dx=True):
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    dz = np.ascontiguousarray(dz, dtype=np.float64)
    B, H, W, Cin = x.shape
    Cout = w.shape[3]
    dx = np.zeros_like(x) if need_dx else None
    dw = np.zeros_like(w)
    db = np.zeros(Cout)
    lib().ora_conv3x3_bwd(B, H, W, Cin, Cout, _dp(x), _dp(w), _dp(dz), _dp(dx) if need_dx else None,
                          _dp(dw), _dp(db))
    return dx, dw, db


def silu(z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    y = np.zeros_like(z)
    d = np.zeros_like(z)
    lib().ora_silu(z.size, _dp(z), _dp(y), _dp(d))
    return y, d


def adam(p, m, v, g, lr, b1=0.9, b2=0.999, eps=1e-8, t=1):
    """In-place Adam step on float64 arrays p, m, v."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().ora_adam(p.size, _dp(p), _dp(m), _dp(v), _dp(g), lr, b1, b2, eps, t)


class SurrogateNet:
    """The surrogate network on the oracle: 3x3 convolutions with SiLU between
    them, forward with stored pre-activations, and the gradient of the
    per-sample relative squared error sum_b |y_b - t_b|^2 / |t_b|^2."""

    def __init__(self, weights, biases):
        self.w = [np.asarray(w, dtype=np.float64) for w in weights]
        self.b = [np.asarray(b, dtype=np.float64) for b in biases]

    def forward(self, x):
        acts, zs = [np.asarray(x, dtype=np.float64)], []
        for k, (w, b) in enumerate(zip(self.w, self.b)):
            z = conv3x3_fwd(acts[-1], w, b)
            zs.append(z)
            if k + 1 < len(self.w):
                acts.append(silu(z)[0])
        self.acts, self.zs = acts, zs
        return zs[-1]

    def loss_and_grads(self, x, target):
        y = self.forward(x)
        B = y.shape[0]
        nt = np.array([np.sum(target[b] ** 2) for b in range(B)])
        loss = sum(np.sum((y[b] - target[b]) ** 2) / nt[b] for b in range(B))
        dz = np.stack([2.0 * (y[b] - target[b]) / nt[b] for b in range(B)])
        gw, gb = [None] * len(self.w), [None] * len(self.w)
        for k in range(len(self.w) - 1, -1, -1):
            dx, gw[k], gb[k] = conv3x3_bwd(self.acts[k], self.w[k], dz, need_dx=k > 0)
            if k > 0:
                dz = dx * silu(self.zs[k - 1])[1]
        return loss, gw, gb


def _obs_dict(o: Observation) -> dict:
    return {"step": o.step, "E": o.E, "per_term": list(o.per_term),
            "max_torque": o.max_torque, "M": list(o.M), "max_norm_dev": o.max_norm_dev}


def mc_order(N, seed, sweep, replica=0) -> np.ndarray:
    """The random visiting order of one Metropolis sweep."""
    out = np.zeros(max(N, 1), dtype=np.int64)
    lib().ora_mc_order(N, seed, sweep, replica, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out[:N]


def mc_adapt_cone(cone_deg, acceptance, target) -> float:
    return lib().ora_mc_adapt_cone(cone_deg, acceptance, target)


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return list(o)


def thermal_normals(seed, step, site, replica=0) -> np.ndarray:
    out = np.zeros(3)
    lib().ora_thermal_normals(seed, step, site, replica, _dp(out))
    return out


def rotate(n, omega, dt) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64)
    w = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.zeros(3)
    lib().ora_rotate(_dp(n), _dp(w), dt, _dp(out))
    return out


Optional
