"""Thin ctypes binding of the C ABI in ``include/sp_engine.h``.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libsp_engine.so``.  PyTorch is used, where the caller wants it,
for device memory (``*_dev`` calls take CUDA/HIP tensors) and streams.
If the library is not built, importing works but creating an ``Engine``
raises ``RuntimeError`` -- there is no CPU fallback.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsp_engine.so")

SP_OK, SP_E_ARG, SP_E_ORDER, SP_E_HIP, SP_E_NOMEM, SP_E_UNSUPPORTED, SP_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
SP_F32, SP_F64 = 0, 1
SP_DMI_BULK, SP_DMI_INTERFACIAL = 1, 2
SP_DDI_OFF, SP_DDI_DIRECT = 0, 1

# every symbol the header declares
EXPORTS = [
    "sp_create", "sp_destroy", "sp_last_error", "sp_version", "sp_set_geometry",
    "sp_set_hamiltonian", "sp_set_pairs", "sp_num_sites", "sp_get_bonds", "sp_set_spins", "sp_get_spins",
    "sp_set_spins_dev", "sp_get_spins_dev", "sp_set_step", "sp_get_step", "sp_gradient",
    "sp_gradient_dev", "sp_energy", "sp_observe", "sp_llg_step", "sp_run", "sp_run_tol",
    "sp_set_graph_replay", "sp_synchronize",
    "sp_dipole_gradient", "sp_dipole_gradient_dev", "sp_dipole_gradient_dev_noalloc", "sp_thermal_normals", "sp_step_path",
    "sp_set_step_path", "sp_autotune", "sp_mc_run",
    "sp_batch_create", "sp_batch_destroy", "sp_batch_last_error", "sp_batch_add", "sp_batch_run",
    "sp_batch_get_spins", "sp_batch_replica_info", "sp_batch_set_chunk", "sp_batch_get_step",
    "sp_batch_autotune", "sp_batch_add_gneb",
    "sp_gneb_create", "sp_gneb_destroy", "sp_gneb_last_error", "sp_gneb_set_image_type", "sp_gneb_iterate",
    "sp_gneb_iterate_tol",
    "sp_gneb_get_chain", "sp_gneb_get_forces",
    "sp_ddi_init", "sp_ddi_init_residual", "sp_ddi_backbone_dev", "sp_ddi_num_params", "sp_ddi_set_params",
    "sp_ddi_get_params", "sp_ddi_label_dev",
    "sp_ddi_forward_dev", "sp_ddi_loss_grad_dev", "sp_ddi_train_dev", "sp_ddi_configure", "sp_ddi_stats",
]


class SpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sp_engine error {code}: {msg}")
        self.code = code


class sp_hamiltonian(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int),
                ("mu", ctypes.POINTER(ctypes.c_double)),
                ("B", ctypes.c_double * 3),
                ("K", ctypes.POINTER(ctypes.c_double)),
                ("K_axis", ctypes.POINTER(ctypes.c_double)),
                ("n_exch_shells", ctypes.c_int),
                ("J", ctypes.POINTER(ctypes.c_double)),
                ("n_dmi_shells", ctypes.c_int),
                ("D", ctypes.POINTER(ctypes.c_double)),
                ("dmi_kind", ctypes.c_int),
                ("ddi_mode", ctypes.c_int),
                ("n_gauss", ctypes.c_int),
                ("gauss_a", ctypes.POINTER(ctypes.c_double)),
                ("gauss_sigma", ctypes.POINTER(ctypes.c_double)),
                ("gauss_c", ctypes.POINTER(ctypes.c_double))]


class sp_llg_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("dt_ps", ctypes.c_double),
                ("T_K", ctypes.c_double), ("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32),
                ("solver", ctypes.c_int32)]


SOLVERS = {"depondt": 0, "heun": 1, "sib": 2}   # sp_solver


class sp_mc_params(ctypes.Structure):
    _fields_ = [("T_K", ctypes.c_double), ("cone_deg", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("target_acceptance", ctypes.c_double)]


class sp_observation(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("E", ctypes.c_double),
                ("per_term", ctypes.c_double * 5), ("max_torque", ctypes.c_double),
                ("M", ctypes.c_double * 3), ("max_norm_dev", ctypes.c_double)]


_lib = None

# Every live handle, closed at interpreter exit (batches, then chains, then
# engines) so that no HIP call is left to finalisers that run while the
# interpreter and the libraries it loaded are being torn down.
_live = weakref.WeakSet()


def close_all():
    """Close every Batch, Gneb and Engine still open (in that order)."""
    objs = list(_live)
    for kind in (Batch, Gneb, Engine):
        for o in objs:
            if isinstance(o, kind):
                o.close()


atexit.register(close_all)


def lib():
    """Load ``libsp_engine.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP engine library not built: {LIB_PATH} is missing "
                           "(run paper_1901_11350_amd/build.py or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i64, u64, ci = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    sig = {
        "sp_create": (ci, [ctypes.POINTER(vp), ci, ci, vp]),
        "sp_destroy": (None, [vp]),
        "sp_last_error": (ctypes.c_char_p, [vp]),
        "sp_version": (ctypes.c_char_p, []),
        "sp_set_geometry": (ci, [vp, dp, ci, dp, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.c_double]),
        "sp_set_hamiltonian": (ci, [vp, ctypes.POINTER(sp_hamiltonian)]),
        "sp_set_pairs": (ci, [vp, i64, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci), dp, dp]),
        "sp_num_sites": (i64, [vp]),
        "sp_get_bonds": (ci, [vp, ci, dp, ci]),
        "sp_set_spins": (ci, [vp, dp, i64]),
        "sp_get_spins": (ci, [vp, dp, i64]),
        "sp_set_spins_dev": (ci, [vp, vp, i64]),
        "sp_get_spins_dev": (ci, [vp, vp, i64]),
        "sp_set_step": (ci, [vp, u64]),
        "sp_get_step": (u64, [vp]),
        "sp_gradient": (ci, [vp, dp, i64]),
        "sp_gradient_dev": (ci, [vp, vp, i64]),
        "sp_energy": (ci, [vp, dp, dp]),
        "sp_observe": (ci, [vp, ctypes.POINTER(sp_observation)]),
        "sp_llg_step": (ci, [vp, ctypes.POINTER(sp_llg_params)]),
        "sp_run": (ci, [vp, ctypes.POINTER(sp_llg_params), i64, i64, ctypes.POINTER(sp_observation)]),
        "sp_run_tol": (ci, [vp, ctypes.POINTER(sp_llg_params), i64, i64, ctypes.c_double,
                            ctypes.POINTER(sp_observation), ctypes.POINTER(i64)]),
        "sp_set_graph_replay": (ci, [vp, ci]),
        "sp_synchronize": (ci, [vp]),
        "sp_dipole_gradient": (ci, [vp, dp, i64]),
        "sp_dipole_gradient_dev": (ci, [vp, vp, vp, i64]),
        "sp_dipole_gradient_dev_noalloc": (ci, [vp, vp, vp, i64]),
        "sp_thermal_normals": (ci, [vp, u64, u64, ctypes.c_uint32, ctypes.c_uint32, i64, dp,
                                    ctypes.POINTER(ctypes.c_uint32)]),
        "sp_step_path": (ctypes.c_char_p, [vp]),
        "sp_set_step_path": (ci, [vp, ctypes.c_char_p]),
        "sp_autotune": (ci, [vp, ctypes.POINTER(sp_llg_params), ci, dp]),
        "sp_mc_run": (ci, [vp, ctypes.POINTER(sp_mc_params), i64, i64, ctypes.POINTER(sp_observation),
                           ctypes.POINTER(i64), dp]),
        "sp_batch_create": (ci, [ctypes.POINTER(vp), ci, vp]),
        "sp_batch_destroy": (None, [vp]),
        "sp_batch_last_error": (ctypes.c_char_p, [vp]),
        "sp_batch_add": (ci, [vp, vp, ctypes.POINTER(sp_llg_params)]),
        "sp_batch_run": (ci, [vp, i64]),
        "sp_batch_get_spins": (ci, [vp, ci, dp, i64]),
        "sp_batch_replica_info": (ci, [vp, ci, ctypes.POINTER(i64), ctypes.POINTER(ci)]),
        "sp_batch_set_chunk": (ci, [vp, ci]),
        "sp_batch_get_step": (u64, [vp]),
        "sp_batch_autotune": (ci, [vp, ci, dp]),
        "sp_batch_add_gneb": (ci, [vp, vp]),
        "sp_gneb_create": (ci, [ctypes.POINTER(vp), vp, ci, dp, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double]),
        "sp_gneb_destroy": (None, [vp]),
        "sp_gneb_last_error": (ctypes.c_char_p, [vp]),
        "sp_gneb_set_image_type": (ci, [vp, ci, ci]),
        "sp_gneb_iterate": (ci, [vp, ci]),
        "sp_gneb_iterate_tol": (ci, [vp, ci, ctypes.c_double, ctypes.POINTER(ci)]),
        "sp_gneb_get_chain": (ci, [vp, dp]),
        "sp_gneb_get_forces": (ci, [vp, dp, dp, dp]),
        "sp_ddi_init": (ci, [vp, ci, ctypes.POINTER(ci), u64]),
        "sp_ddi_init_residual": (ci, [vp, ci, ctypes.POINTER(ci), u64, ci, ci]),
        "sp_ddi_backbone_dev": (ci, [vp, ci, vp, vp]),
        "sp_ddi_num_params": (i64, [vp]),
        "sp_ddi_set_params": (ci, [vp, dp, i64]),
        "sp_ddi_get_params": (ci, [vp, dp, i64]),
        "sp_ddi_label_dev": (ci, [vp, ci, vp, vp]),
        "sp_ddi_forward_dev": (ci, [vp, ci, vp, vp]),
        "sp_ddi_loss_grad_dev": (ci, [vp, ci, vp, vp, dp, dp]),
        "sp_ddi_train_dev": (ci, [vp, ci, vp, vp, ci, ci, ctypes.c_double, u64, dp]),
        "sp_ddi_configure": (ci, [vp, ctypes.c_double, ci]),
        "sp_ddi_stats": (ci, [vp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(values, n=None):
    a = np.ascontiguousarray(np.asarray(values, dtype=np.float64).ravel())
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def obs_dict(o: sp_observation) -> dict:
    return {"step": int(o.step), "E": o.E, "per_term": list(o.per_term),
            "max_torque": o.max_torque, "M": list(o.M), "max_norm_dev": o.max_norm_dev}


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _pair_arrays(pairs):
    pairs = list(pairs)
    bi = np.ascontiguousarray([p[0] for p in pairs], dtype=np.int32)
    bj = np.ascontiguousarray([p[1] for p in pairs], dtype=np.int32)
    dc = np.ascontiguousarray([list(p[2]) for p in pairs], dtype=np.int32).reshape(-1)
    J = np.ascontiguousarray([p[3] for p in pairs], dtype=np.float64)
    D = np.ascontiguousarray([list(p[4]) for p in pairs], dtype=np.float64).reshape(-1)
    if not pairs:   # valid pointers for an empty list
        bi, bj, dc = (np.zeros(3, np.int32) for _ in range(3))
        J, D = np.zeros(1), np.zeros(3)
    return len(pairs), bi, bj, dc, J, D


class Engine:
    """One engine instance (``sp_engine``) on one HIP device."""

    def __init__(self, device: int = 0, precision: str = "f32", stream=None):
        L = lib()
        self.precision = precision
        prec = {"f32": SP_F32, "f64": SP_F64}[precision]
        self._h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        rc = L.sp_create(ctypes.byref(self._h), device, prec, s)
        if rc != SP_OK:
            raise SpError(rc, "sp_create failed (no HIP device?)")
        _live.add(self)
        self.N = 0
        self._keep = []

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.sp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    def _check(self, rc: int):
        if rc != SP_OK:
            raise SpError(rc, lib().sp_last_error(self._h).decode())
        return rc

    # ------------------------------------------------------------- setup
    def set_geometry(self, geometry):
        br = _f64(geometry.bravais, 9)
        bs = _f64(geometry.basis, 3 * len(geometry.basis))
        nc = (ctypes.c_int * 3)(*geometry.n_cells)
        pe = (ctypes.c_int * 3)(*geometry.periodic)
        self._check(lib().sp_set_geometry(self._h, _dp(br), len(geometry.basis), _dp(bs), nc, pe,
                                          float(geometry.lattice_constant)))
        self.N = int(lib().sp_num_sites(self._h))

    def set_hamiltonian(self, ham):
        nb = len(ham.mu)
        arrs = {"mu": _f64(ham.mu, nb), "K": _f64(ham.K, nb), "Kax": _f64(ham.K_axis, 3 * nb),
                "J": _f64(ham.J if len(ham.J) else [0.0]), "D": _f64(ham.D if len(ham.D) else [0.0])}
        h = sp_hamiltonian()
        h.n_basis = nb
        h.mu = _dp(arrs["mu"])
        for k in range(3):
            h.B[k] = ham.B[k]
        h.K = _dp(arrs["K"])
        h.K_axis = _dp(arrs["Kax"])
        h.n_exch_shells = len(ham.J)
        h.J = _dp(arrs["J"])
        h.n_dmi_shells = len(ham.D)
        h.D = _dp(arrs["D"])
        h.dmi_kind = ham.dmi_kind
        # ddi: False/True (off / direct sum) or an sp_ddi_mode value
        h.ddi_mode = int(ham.ddi)
        gauss = getattr(ham, "gauss", ())
        h.n_gauss = len(gauss)
        if gauss:
            arrs["ga"] = _f64([a for a, _, _ in gauss])
            arrs["gs"] = _f64([sg for _, sg, _ in gauss])
            arrs["gc"] = _f64([x for _, _, c in gauss for x in c])
            h.gauss_a, h.gauss_sigma, h.gauss_c = _dp(arrs["ga"]), _dp(arrs["gs"]), _dp(arrs["gc"])
        self._check(lib().sp_set_hamiltonian(self._h, ctypes.byref(h)))

    def set_pairs(self, pairs):
        """Explicit pair interactions: a sequence of (bi, bj, (da, db, dc), J,
        (Dx, Dy, Dz)) replacing the shell-built exchange and DMI bonds."""
        n, bi, bj, dc, J, D = _pair_arrays(pairs)
        self._check(lib().sp_set_pairs(self._h, n, _ip(bi), _ip(bj), _ip(dc), _dp(J), _dp(D)))

    def bonds(self, beta: int = 0):
        k = lib().sp_get_bonds(self._h, beta, None, 0)
        if k < 0:
            self._check(k)
        out = np.zeros(10 * max(k, 1))
        lib().sp_get_bonds(self._h, beta, _dp(out), k)
        return out[: 10 * k].reshape(k, 10)

    # ------------------------------------------------------------- spins
    def set_spins(self, n):
        a = _f64(n, 3 * self.N)
        self._check(lib().sp_set_spins(self._h, _dp(a), self.N))

    def get_spins(self) -> np.ndarray:
        out = np.zeros(3 * self.N)
        self._check(lib().sp_get_spins(self._h, _dp(out), self.N))
        return out.reshape(3, self.N)

    def set_spins_dev(self, t):
        self._check(lib().sp_set_spins_dev(self._h, ctypes.c_void_p(t.data_ptr()), self.N))

    def get_spins_dev(self, t):
        self._check(lib().sp_get_spins_dev(self._h, ctypes.c_void_p(t.data_ptr()), self.N))

    @property
    def step(self) -> int:
        return int(lib().sp_get_step(self._h))

    @step.setter
    def step(self, v: int):
        self._check(lib().sp_set_step(self._h, int(v)))

    @property
    def step_path(self) -> str:
        return lib().sp_step_path(self._h).decode()

    @step_path.setter
    def step_path(self, name: str):
        self._check(lib().sp_set_step_path(self._h, name.encode()))

    # ----------------------------------------------------------- compute
    def gradient(self) -> np.ndarray:
        out = np.zeros(3 * self.N)
        self._check(lib().sp_gradient(self._h, _dp(out), self.N))
        return out.reshape(3, self.N)

    def gradient_dev(self, t):
        self._check(lib().sp_gradient_dev(self._h, ctypes.c_void_p(t.data_ptr()), self.N))

    def dipole_gradient(self) -> np.ndarray:
        out = np.zeros(3 * self.N)
        self._check(lib().sp_dipole_gradient(self._h, _dp(out), self.N))
        return out.reshape(3, self.N)

    def dipole_gradient_dev(self, n_t, g_t):
        self._check(lib().sp_dipole_gradient_dev(self._h, ctypes.c_void_p(n_t.data_ptr()),
                                                 ctypes.c_void_p(g_t.data_ptr()), self.N))

    def energy(self, per_term: bool = False):
        E = ctypes.c_double()
        pt = np.zeros(5)
        self._check(lib().sp_energy(self._h, ctypes.byref(E), _dp(pt)))
        return (E.value, pt) if per_term else E.value

    def observe(self) -> dict:
        o = sp_observation()
        self._check(lib().sp_observe(self._h, ctypes.byref(o)))
        return obs_dict(o)

    def llg_step(self, alpha: float, dt: float, T: float = 0.0, seed: int = 0, replica: int = 0,
                 solver: str = "depondt"):
        p = sp_llg_params(alpha, dt, T, seed, replica, SOLVERS[solver])
        self._check(lib().sp_llg_step(self._h, ctypes.byref(p)))

    def run(self, alpha: float, dt: float, n_steps: int, T: float = 0.0, seed: int = 0,
            observe_every: int = 0, check: bool = True, replica: int = 0, solver: str = "depondt"):
        p = sp_llg_params(alpha, dt, T, seed, replica, SOLVERS[solver])
        n_obs = n_steps // observe_every if observe_every > 0 else 0
        obs = (sp_observation * max(n_obs, 1))()
        rc = lib().sp_run(self._h, ctypes.byref(p), n_steps, observe_every, obs if n_obs else None)
        if check:
            self._check(rc)
        res = [obs_dict(o) for o in obs[:n_obs]]
        return (res, rc) if not check else res

    def run_tol(self, alpha: float, dt: float, max_steps: int, observe_every: int, tol: float, T: float = 0.0,
                seed: int = 0, replica: int = 0, solver: str = "depondt"):
        """Run until an observation's maximum torque is below tol (or
        max_steps); returns (observations, steps taken)."""
        p = sp_llg_params(alpha, dt, T, seed, replica, SOLVERS[solver])
        n_obs = max_steps // observe_every if observe_every > 0 else 0
        obs = (sp_observation * max(n_obs, 1))()
        done = ctypes.c_int64()
        self._check(lib().sp_run_tol(self._h, ctypes.byref(p), max_steps, observe_every, tol,
                                     obs if n_obs else None, ctypes.byref(done)))
        n_kept = done.value // observe_every if observe_every > 0 else 0
        return [obs_dict(o) for o in obs[:min(n_obs, n_kept)]], done.value

    def set_graph_replay(self, enable: bool):
        self._check(lib().sp_set_graph_replay(self._h, 1 if enable else 0))

    def mc_run(self, T: float, cone_deg: float, n_sweeps: int, seed: int = 0, replica: int = 0,
               observe_every: int = 0, target_acceptance: float = 0.0, return_cone: bool = False):
        """Metropolis sweeps; returns (observations, accepted trials[, final cone])."""
        p = sp_mc_params(T, cone_deg, seed, replica, target_acceptance)
        n_obs = n_sweeps // observe_every if observe_every > 0 else 0
        obs = (sp_observation * max(n_obs, 1))()
        acc = ctypes.c_int64()
        cone = ctypes.c_double()
        self._check(lib().sp_mc_run(self._h, ctypes.byref(p), n_sweeps, observe_every, obs if n_obs else None,
                                    ctypes.byref(acc), ctypes.byref(cone)))
        out = ([obs_dict(o) for o in obs[:n_obs]], acc.value)
        return out + (cone.value,) if return_cone else out

    def autotune(self, alpha: float, dt: float, T: float = 0.0, seed: int = 0, n_steps: int = 50,
                 solver: str = "depondt") -> float:
        """Time every allowed step path / tile configuration, keep the fastest;
        returns its milliseconds per step."""
        p = sp_llg_params(alpha, dt, T, seed, 0, SOLVERS[solver])
        ms = ctypes.c_double()
        self._check(lib().sp_autotune(self._h, ctypes.byref(p), n_steps, ctypes.byref(ms)))
        return ms.value

    def synchronize(self):
        self._check(lib().sp_synchronize(self._h))

    # ------------------------------------------- learned dipole surrogate
    def ddi_init(self, channels, seed: int = 0):
        ch = (ctypes.c_int * len(channels))(*channels)
        self._check(lib().sp_ddi_init(self._h, len(channels) - 1, ch, seed))

    def ddi_init_residual(self, channels, seed: int = 0, block: int = 4, reach: int = 2):
        ch = (ctypes.c_int * len(channels))(*channels)
        self._check(lib().sp_ddi_init_residual(self._h, len(channels) - 1, ch, seed, block, reach))

    def ddi_backbone_dev(self, batch: int, spins_t, field_t):
        self._check(lib().sp_ddi_backbone_dev(self._h, batch, ctypes.c_void_p(spins_t.data_ptr()),
                                              ctypes.c_void_p(field_t.data_ptr())))

    def ddi_num_params(self) -> int:
        return int(lib().sp_ddi_num_params(self._h))

    def ddi_set_params(self, params):
        p = _f64(params, self.ddi_num_params())
        self._check(lib().sp_ddi_set_params(self._h, _dp(p), p.size))

    def ddi_get_params(self) -> np.ndarray:
        p = np.zeros(self.ddi_num_params())
        self._check(lib().sp_ddi_get_params(self._h, _dp(p), p.size))
        return p

    def ddi_label_dev(self, batch: int, spins_t, labels_t):
        self._check(lib().sp_ddi_label_dev(self._h, batch, ctypes.c_void_p(spins_t.data_ptr()),
                                           ctypes.c_void_p(labels_t.data_ptr())))

    def ddi_forward_dev(self, batch: int, spins_t, field_t):
        self._check(lib().sp_ddi_forward_dev(self._h, batch, ctypes.c_void_p(spins_t.data_ptr()),
                                             ctypes.c_void_p(field_t.data_ptr())))

    def ddi_loss_grad_dev(self, batch: int, spins_t, labels_t):
        loss = ctypes.c_double()
        g = np.zeros(self.ddi_num_params())
        self._check(lib().sp_ddi_loss_grad_dev(self._h, batch, ctypes.c_void_p(spins_t.data_ptr()),
                                               ctypes.c_void_p(labels_t.data_ptr()), ctypes.byref(loss),
                                               _dp(g)))
        return loss.value, g

    def ddi_train_dev(self, n: int, spins_t, labels_t, epochs: int, batch: int, lr: float,
                      seed: int = 0) -> np.ndarray:
        out = np.zeros(max(epochs, 1))
        self._check(lib().sp_ddi_train_dev(self._h, n, ctypes.c_void_p(spins_t.data_ptr()),
                                           ctypes.c_void_p(labels_t.data_ptr()), epochs, batch, lr, seed,
                                           _dp(out)))
        return out[:epochs]

    def ddi_configure(self, tol: float, n_check: int):
        self._check(lib().sp_ddi_configure(self._h, tol, n_check))

    def ddi_stats(self) -> dict:
        s = np.zeros(4)
        self._check(lib().sp_ddi_stats(self._h, _dp(s)))
        return {"evaluations": int(s[0]), "fallbacks": int(s[1]), "last_error": s[2], "max_error": s[3]}

    def thermal_normals(self, seed: int, step: int, site0: int, n_sites: int, replica: int = 0):
        eta = np.zeros(3 * n_sites)
        raw = (ctypes.c_uint32 * (4 * n_sites))()
        self._check(lib().sp_thermal_normals(self._h, seed, step, replica, site0, n_sites, _dp(eta), raw))
        return eta.reshape(3, n_sites), np.frombuffer(raw, dtype=np.uint32).reshape(n_sites, 4).copy()


class Batch:
    """A replica batch (``sp_batch``): replicas sharing one Hamiltonian advance
    together (LDS-resident small replicas, tiled large ones, HIP-graph chunks)."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        self._h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        rc = L.sp_batch_create(ctypes.byref(self._h), device, s)
        if rc != SP_OK:
            raise SpError(rc, "sp_batch_create failed (no HIP device?)")
        _live.add(self)
        self.sizes = []

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.sp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    def _check(self, rc: int):
        if rc < 0:
            raise SpError(rc, lib().sp_batch_last_error(self._h).decode())
        return rc

    def add(self, engine: "Engine", alpha: float, dt: float, T: float = 0.0, seed: int = 0,
            replica: int = 0) -> int:
        p = sp_llg_params(alpha, dt, T, seed, replica)
        slot = self._check(lib().sp_batch_add(self._h, engine._h, ctypes.byref(p)))
        self.sizes.append(engine.N)
        return slot

    def run(self, n_steps: int):
        self._check(lib().sp_batch_run(self._h, n_steps))

    def get_spins(self, slot: int) -> np.ndarray:
        n = self.sizes[slot]
        out = np.zeros(3 * n)
        self._check(lib().sp_batch_get_spins(self._h, slot, _dp(out), n))
        return out.reshape(3, n)

    def info(self, slot: int):
        n = ctypes.c_int64()
        r = ctypes.c_int()
        self._check(lib().sp_batch_replica_info(self._h, slot, ctypes.byref(n), ctypes.byref(r)))
        return int(n.value), bool(r.value)

    def set_chunk(self, steps: int):
        self._check(lib().sp_batch_set_chunk(self._h, steps))

    @property
    def step(self) -> int:
        return int(lib().sp_batch_get_step(self._h))

    def autotune(self, n_steps: int = 20) -> float:
        ms = ctypes.c_double()
        self._check(lib().sp_batch_autotune(self._h, n_steps, ctypes.byref(ms)))
        return ms.value

    def add_gneb(self, chain: "Gneb"):
        """Advance a GNEB chain (FP32) with every run, in the same chunk graph."""
        self._check(lib().sp_batch_add_gneb(self._h, chain._h))
        self._gneb = chain   # keep it alive while attached


class Gneb:
    """GNEB chain (``sp_gneb``) on an engine's lattice and Hamiltonian; the
    engine must stay alive while the chain is used."""

    def __init__(self, engine: "Engine", chain, k_spring: float = 1.0, vp_dt: float = 0.1,
                 vp_mass: float = 1.0):
        c = np.ascontiguousarray(np.asarray(chain, dtype=np.float64))
        self.M = c.shape[0]
        self.N = engine.N
        assert c.size == self.M * 3 * self.N
        self.engine = engine
        self._h = ctypes.c_void_p()
        rc = lib().sp_gneb_create(ctypes.byref(self._h), engine._h, self.M, _dp(c), k_spring, vp_dt,
                                  vp_mass)
        engine._check(rc)
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.sp_gneb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        self.close()

    def _check(self, rc: int):
        if rc != SP_OK:
            raise SpError(rc, lib().sp_gneb_last_error(self._h).decode())

    def set_image_types(self, types):
        """types: one of "normal", "climbing", "falling" per image (endpoints ignored)."""
        codes = {"normal": 0, "climbing": 1, "falling": 2}
        for v, t in enumerate(types):
            if 0 < v < len(types) - 1:
                self._check(lib().sp_gneb_set_image_type(self._h, v, codes[t]))

    def iterate(self, n_iter: int):
        self._check(lib().sp_gneb_iterate(self._h, n_iter))

    def iterate_tol(self, max_iter: int, tol: float) -> int:
        """Iterate until the largest per-spin force is below tol; returns the
        iterations taken."""
        done = ctypes.c_int()
        self._check(lib().sp_gneb_iterate_tol(self._h, max_iter, tol, ctypes.byref(done)))
        return done.value

    def chain(self) -> np.ndarray:
        out = np.zeros(self.M * 3 * self.N)
        self._check(lib().sp_gneb_get_chain(self._h, _dp(out)))
        return out.reshape(self.M, 3, self.N)

    def forces(self) -> dict:
        E = np.zeros(self.M)
        l = np.zeros(self.M - 1)
        F = np.zeros(self.M * 3 * self.N)
        self._check(lib().sp_gneb_get_forces(self._h, _dp(E), _dp(l), _dp(F)))
        return {"E": E, "l": l, "F": F.reshape(self.M, 3, self.N)}


def engine_for(workload, device: int = 0, precision: Optional[str] = None, stream=None) -> Engine:
    """Engine with the workload's geometry and Hamiltonian set (spins not set)."""
    e = Engine(device, precision or workload.precision, stream)
    e.set_geometry(workload.geometry)
    e.set_hamiltonian(workload.hamiltonian)
    return e


Sequence
