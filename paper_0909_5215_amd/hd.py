"""ctypes binding of libhd.so (include/hd.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The library is loaded from this package directory; if it is
missing, or no gfx950 device is present, the calls fail loudly (there is no
CPU fallback).  PyTorch, when used, only supplies a HIP stream and device
buffers for the *_device copies.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhd.so")

HD_OK, HD_E_ARG, HD_E_OOM, HD_E_HIP, HD_E_STATE, HD_E_UNSTABLE, HD_E_NOGPU = 0, -1, -2, -3, -4, -5, -6
HD_FP64, HD_FP32C = 0, 1
HD_EXEC_BATCHED, HD_EXEC_GRID, HD_EXEC_SEQUENTIAL = 0, 1, 2
HD_FORCE_TOTAL, HD_FORCE_LJ, HD_FORCE_BIAS, HD_HU, HD_TUU = 0, 1, 2, 3, 4
HD_BIAS_SLOPE, HD_BIAS_CURVATURE, HD_BIAS_DISTANCE, HD_BIAS_EIGENVALUE = 0, 1, 2, 3
HD_FLAG_UNSTABLE, HD_FLAG_NBR_OVERFLOW = 1, 2
HD_LAUNCH_LDS, HD_LAUNCH_PERSISTENT_LARGE = 1, 2
HD_QUENCH_CHECK, HD_QUENCH_SET_REFERENCE = 0, 1
HD_ALL_SYSTEMS = -1
HD_FIELD_POSITIONS, HD_FIELD_VELOCITIES, HD_FIELD_FORCES, HD_FIELD_FORCES_LJ, HD_FIELD_FORCES_BIAS, HD_FIELD_HU = \
    0, 1, 2, 3, 4, 5

_c = ctypes
_dp = _c.POINTER(_c.c_double)


class hd_system_desc(_c.Structure):
    _fields_ = [("dim", _c.c_int32), ("n_atoms", _c.c_int32), ("box", _c.c_double * 3),
                ("periodic", _c.c_int32 * 3), ("pos", _dp), ("type", _c.POINTER(_c.c_uint8)),
                ("role", _c.POINTER(_c.c_uint8)), ("mass", _c.c_double)]


class hd_lj_params(_c.Structure):
    _fields_ = [("eps", (_c.c_double * 2) * 2), ("sig", (_c.c_double * 2) * 2),
                ("rc", _c.c_double), ("skin", _c.c_double)]


class hd_thermo_params(_c.Structure):
    _fields_ = [("dt", _c.c_double), ("gamma", _c.c_double), ("kT", _c.c_double), ("seed", _c.c_uint64)]


class hd_drive_params(_c.Structure):
    _fields_ = [("k_spring", _c.c_double), ("f_normal", _c.c_double),
                ("x_slider", _c.c_double), ("v_slider", _c.c_double)]


class hd_bias_params(_c.Structure):
    _fields_ = [("enabled", _c.c_int32), ("m_b", _c.c_int32), ("dv_max", _c.c_double),
                ("g_lo", _c.c_double), ("g_hi", _c.c_double)]


class hd_scalars(_c.Structure):
    _fields_ = [("e_pot", _c.c_double), ("e_kin", _c.c_double), ("dv", _c.c_double),
                ("dvp", _c.c_double), ("g", _c.c_double), ("d", _c.c_double),
                ("t_md", _c.c_double), ("t_hyper", _c.c_double), ("x_slider", _c.c_double),
                ("x_tip", _c.c_double), ("f_lat", _c.c_double), ("step", _c.c_int64),
                ("flags", _c.c_int32), ("n_rebuilds", _c.c_int32),
                ("kappa", _c.c_double), ("dv1", _c.c_double), ("dv2", _c.c_double),
                ("e_nhc", _c.c_double), ("lambda_", _c.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


class hd_schedule(_c.Structure):
    _fields_ = [("lds_resident", _c.c_int32), ("small_block", _c.c_int32),
                ("persistent_large", _c.c_int32), ("large_block", _c.c_int32),
                ("small_half_lists", _c.c_int32), ("ms_per_step", _c.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes)
_P = _c.c_void_p
_SIGS = {
    "hd_create": (_c.c_int, [_c.c_int, _c.c_int, _c.c_void_p, _c.POINTER(_c.c_void_p)]),
    "hd_set_exec": (_c.c_int, [_P, _c.c_int]),
    "hd_set_launch": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_int32]),
    "hd_add_system": (_c.c_int, [_P, _c.POINTER(hd_system_desc), _c.POINTER(hd_lj_params),
                                 _c.POINTER(hd_thermo_params), _c.POINTER(hd_drive_params),
                                 _c.POINTER(_c.c_int32)]),
    "hd_set_reference": (_c.c_int, [_P, _c.c_int32, _dp]),
    "hd_set_bias": (_c.c_int, [_P, _c.c_int32, _c.POINTER(hd_bias_params)]),
    "hd_set_slider": (_c.c_int, [_P, _c.c_int32, _c.c_double]),
    "hd_set_thermo": (_c.c_int, [_P, _c.c_int32, _c.POINTER(hd_thermo_params)]),
    "hd_init_velocities": (_c.c_int, [_P, _c.c_int32]),
    "hd_set_positions": (_c.c_int, [_P, _c.c_int32, _dp]),
    "hd_set_velocities": (_c.c_int, [_P, _c.c_int32, _dp]),
    "hd_finalize": (_c.c_int, [_P]),
    "hd_step": (_c.c_int, [_P, _c.c_int64]),
    "hd_compute": (_c.c_int, [_P]),
    "hd_sync": (_c.c_int, [_P]),
    "hd_read_forces": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _dp]),
    "hd_read_positions": (_c.c_int, [_P, _c.c_int32, _dp]),
    "hd_read_velocities": (_c.c_int, [_P, _c.c_int32, _dp]),
    "hd_read_scalars": (_c.c_int, [_P, _c.c_int32, _c.POINTER(hd_scalars)]),
    "hd_read_scalars_batch": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.POINTER(hd_scalars)]),
    "hd_copy_positions_device": (_c.c_int, [_P, _c.c_int32, _c.c_void_p]),
    "hd_copy_forces_device": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_void_p]),
    "hd_get_state": (_c.c_int, [_P, _c.c_int32, _c.c_void_p, _c.POINTER(_c.c_size_t)]),
    "hd_set_state": (_c.c_int, [_P, _c.c_int32, _c.c_void_p, _c.c_size_t]),
    "hd_debug_pairs": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int32), _c.c_int64,
                                  _c.POINTER(_c.c_int64)]),
    "hd_system_info": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    "hd_num_systems": (_c.c_int32, [_P]),
    "hd_last_step_timing": (_c.c_int, [_P, _dp, _c.POINTER(_c.c_int64)]),
    "hd_get_schedule": (_c.c_int, [_P, _c.POINTER(hd_schedule)]),
    "hd_set_schedule": (_c.c_int, [_P, _c.POINTER(hd_schedule)]),
    "hd_autotune": (_c.c_int, [_P, _c.c_double, _c.c_int64, _c.POINTER(hd_schedule), _c.c_int32,
                               _c.POINTER(_c.c_int32)]),
    "hd_quench": (_c.c_int, [_P, _c.POINTER(_c.c_int32), _c.c_int32, _c.c_double, _c.c_int64, _c.c_int32,
                             _c.POINTER(_c.c_int64), _dp, _dp]),
    "hd_quench_noalloc": (_c.c_int, [_P, _c.POINTER(_c.c_int32), _c.c_int32, _c.c_double, _c.c_int64, _c.c_int32,
                                     _c.POINTER(_c.c_int64), _dp, _dp]),
    "hd_min_mode": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_double, _c.c_uint64, _dp,
                               _c.POINTER(_c.c_int32), _dp]),
    "hd_min_mode_gradient": (_c.c_int, [_P, _c.c_int32, _dp, _dp]),
    "hd_set_tip_bonds": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_double, _c.c_double, _c.c_double]),
    "hd_set_bias_variables": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_double, _c.c_double]),
    "hd_set_nose_hoover": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_double]),
    "hd_set_min_mode": (_c.c_int, [_P, _c.c_int32, _dp, _c.c_double]),
    "hd_read_min_mode": (_c.c_int, [_P, _c.c_int32, _dp]),
    "hd_bind_device": (_c.c_int, [_P, _c.c_int32, _c.c_int32, _c.c_void_p]),
    "hd_batch_layout": (_c.c_int, [_P, _c.c_int32, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64)]),
    "hd_last_error": (_c.c_char_p, [_P]),
    "hd_destroy": (None, [_P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libhd.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        # one HIP runtime per process: PyTorch ships its own, and when it is
        # installed it is loaded first so that libhd.so binds to the same one
        # (device pointers and streams are then shared; two runtimes in one
        # process cannot both open the device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> List[str]:
    return list(_SIGS)


class HDError(RuntimeError):
    pass


def _check(ctx, status: int, what: str):
    if status != HD_OK:
        msg = load().hd_last_error(ctx).decode() if ctx else ""
        raise HDError(f"{what} failed with status {status}: {msg}")


def _darr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class Context:
    """One hd_ctx: a batch of AFM model instances on one GPU."""

    def __init__(self, precision: int = HD_FP32C, device: int = 0, stream=None,
                 exec_mode: int = HD_EXEC_BATCHED, block_threads: int = 0, max_neighbors: int = 0,
                 lds_resident: bool = True, persistent_large: bool = False):
        L = load()
        h = ctypes.c_void_p()
        st = L.hd_create(int(precision), int(device), stream, ctypes.byref(h))
        if st != HD_OK:
            raise HDError(f"hd_create failed with status {st} (gfx950 device required)")
        self._h = h
        self.precision = precision
        self.dims: List[int] = []
        self.sizes: List[int] = []
        _check(h, L.hd_set_exec(h, int(exec_mode)), "hd_set_exec")
        flags = (HD_LAUNCH_LDS if lds_resident else 0) | (HD_LAUNCH_PERSISTENT_LARGE if persistent_large else 0)
        _check(h, L.hd_set_launch(h, int(block_threads), int(max_neighbors), flags), "hd_set_launch")

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().hd_destroy(self._h)
            self._h = None
        self._bound = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- construction -----------------------------------------------------
    def add_system(self, spec) -> int:
        """Add one hd_inputs.SystemSpec (geometry + run parameters)."""
        L = load()
        pos = np.ascontiguousarray(spec.pos, dtype=np.float64)
        typ = np.ascontiguousarray(spec.type, dtype=np.uint8)
        rol = np.ascontiguousarray(spec.role, dtype=np.uint8)
        d = hd_system_desc()
        d.dim, d.n_atoms = spec.dim, spec.n
        for k in range(3):
            d.box[k] = float(spec.box[k])
            d.periodic[k] = int(spec.periodic[k])
        d.pos = _darr(pos)
        d.type = typ.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        d.role = rol.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        d.mass = spec.mass
        lj = hd_lj_params()
        for a in range(2):
            for b in range(2):
                lj.eps[a][b] = float(spec.eps[a, b])
                lj.sig[a][b] = float(spec.sig[a, b])
        lj.rc, lj.skin = spec.rc, spec.skin
        th = hd_thermo_params(spec.dt, spec.gamma, spec.kT, int(spec.seed))
        dr = hd_drive_params(spec.k_spring, spec.f_normal, spec.x_slider, spec.v_slider)
        sid = ctypes.c_int32()
        _check(self._h, L.hd_add_system(self._h, ctypes.byref(d), ctypes.byref(lj), ctypes.byref(th),
                                        ctypes.byref(dr), ctypes.byref(sid)), "hd_add_system")
        s = sid.value
        self.dims.append(spec.dim)
        self.sizes.append(spec.n)
        if spec.rO is not None:
            self.set_reference(s, spec.rO)
        v1, v2 = int(getattr(spec, "bias_var1", 0)), int(getattr(spec, "bias_var2", -1))
        if v1 != HD_BIAS_SLOPE or v2 >= 0:
            self.set_bias_variables(s, v1, v2, getattr(spec, "b2_lo", 0.0), getattr(spec, "b2_hi", 1.0))
        if spec.bias_on:
            self.set_bias(s, True, spec.m_b, spec.dv_max, spec.g_lo, spec.g_hi)
        if HD_BIAS_EIGENVALUE in (v1, v2) and getattr(spec, "mode", None) is not None:
            self.set_min_mode(s, spec.mode, float(getattr(spec, "mode_alpha", 0.0)))
        if int(getattr(spec, "thermostat", 0)) == 1:
            self.set_nose_hoover(s, int(getattr(spec, "nhc_len", 3)), float(getattr(spec, "nhc_tau", 0.5)))
        if getattr(spec, "tip_bonds", 0):
            self.set_tip_bonds(s, True, spec.k_bond, spec.r_bond, spec.r_bond_cut)
        return s

    def set_tip_bonds(self, s: int, enabled: bool, k_bond: float, r_bond: float, r_cut: float):
        _check(self._h, load().hd_set_tip_bonds(self._h, s, int(bool(enabled)), float(k_bond), float(r_bond),
                                                float(r_cut)), "hd_set_tip_bonds")

    def set_min_mode(self, s: int, mode: np.ndarray, alpha: float):
        """Mode estimate of the eigenvalue variable ([dim][n], hd_min_mode's
        layout) and the step of its per-step rotation (hd_set_min_mode)."""
        a = np.ascontiguousarray(mode, dtype=np.float64)
        _check(self._h, load().hd_set_min_mode(self._h, int(s), _darr(a), float(alpha)), "hd_set_min_mode")

    def min_mode_estimate(self, s: int) -> np.ndarray:
        """The current mode estimate, unit over the degrees of freedom
        (hd_read_min_mode)."""
        o = self._out(s)
        _check(self._h, load().hd_read_min_mode(self._h, int(s), _darr(o)), "hd_read_min_mode")
        return o

    def set_nose_hoover(self, s: int, chain_len: int, tau: float = 0.5):
        _check(self._h, load().hd_set_nose_hoover(self._h, s, int(chain_len), float(tau)), "hd_set_nose_hoover")

    def set_bias_variables(self, s: int, var1: int, var2: int = -1, lo2: float = 0.0, hi2: float = 1.0):
        _check(self._h, load().hd_set_bias_variables(self._h, s, int(var1), int(var2), float(lo2), float(hi2)),
               "hd_set_bias_variables")

    def set_reference(self, s: int, rO: np.ndarray):
        a = np.ascontiguousarray(rO, dtype=np.float64)
        _check(self._h, load().hd_set_reference(self._h, s, _darr(a)), "hd_set_reference")

    def set_bias(self, s: int, enabled: bool, m_b: int, dv_max: float, g_lo: float, g_hi: float):
        b = hd_bias_params(int(enabled), int(m_b), float(dv_max), float(g_lo), float(g_hi))
        _check(self._h, load().hd_set_bias(self._h, s, ctypes.byref(b)), "hd_set_bias")

    def set_slider(self, s: int, x: float):
        _check(self._h, load().hd_set_slider(self._h, s, float(x)), "hd_set_slider")

    def set_thermo(self, s: int, dt: float, gamma: float, kT: float, seed: int):
        t = hd_thermo_params(dt, gamma, kT, int(seed))
        _check(self._h, load().hd_set_thermo(self._h, s, ctypes.byref(t)), "hd_set_thermo")

    def init_velocities(self, s: int):
        _check(self._h, load().hd_init_velocities(self._h, s), "hd_init_velocities")

    def set_positions(self, s: int, x: np.ndarray):
        a = np.ascontiguousarray(x, dtype=np.float64)
        _check(self._h, load().hd_set_positions(self._h, s, _darr(a)), "hd_set_positions")

    def set_velocities(self, s: int, v: np.ndarray):
        a = np.ascontiguousarray(v, dtype=np.float64)
        _check(self._h, load().hd_set_velocities(self._h, s, _darr(a)), "hd_set_velocities")

    def finalize(self):
        _check(self._h, load().hd_finalize(self._h), "hd_finalize")

    # -- running ----------------------------------------------------------
    def step(self, n: int):
        _check(self._h, load().hd_step(self._h, int(n)), "hd_step")

    def compute(self):
        _check(self._h, load().hd_compute(self._h), "hd_compute")

    def sync(self):
        _check(self._h, load().hd_sync(self._h), "hd_sync")

    def last_step_timing(self):
        ms = ctypes.c_double()
        nl = ctypes.c_int64()
        _check(self._h, load().hd_last_step_timing(self._h, ctypes.byref(ms), ctypes.byref(nl)),
               "hd_last_step_timing")
        return ms.value, nl.value

    def schedule(self) -> dict:
        out = hd_schedule()
        _check(self._h, load().hd_get_schedule(self._h, ctypes.byref(out)), "hd_get_schedule")
        return out.as_dict()

    def set_schedule(self, shape: dict):
        sh = hd_schedule(**{k: shape[k] for k, _ in hd_schedule._fields_ if k in shape})
        _check(self._h, load().hd_set_schedule(self._h, ctypes.byref(sh)), "hd_set_schedule")

    def autotune(self, min_ms: float = 20.0, max_steps: int = 8192):
        """Time every launch shape on this batch, keep the fastest (the
        trajectory is left where it was).  Returns (chosen, trials)."""
        cap = 128   # more than the candidate shapes of any batch
        buf = (hd_schedule * cap)()
        n = ctypes.c_int32()
        _check(self._h, load().hd_autotune(self._h, float(min_ms), int(max_steps), buf, cap, ctypes.byref(n)),
               "hd_autotune")
        return self.schedule(), [buf[k].as_dict() for k in range(min(n.value, cap))]

    def num_systems(self) -> int:
        return int(load().hd_num_systems(self._h))

    def quench(self, systems, ftol: float = 1e-10, max_iters: int = 100000, set_reference: bool = False,
               no_alloc: bool = False):
        """FIRE minimisation of the listed systems from their current
        positions (hd_quench); the run state is left as it was.  Returns
        (iters, max_disp, minima): per system the iterations used (negative:
        not converged), the largest displacement from r_O (or, with
        set_reference, from the start; the minimum then becomes r_O), and the
        minimum positions [dim][n].  no_alloc: hd_quench_noalloc (no device
        allocation; scratch in the library's static device array)."""
        systems = [int(k) for k in systems]
        n = len(systems)
        ids = (ctypes.c_int32 * n)(*systems)
        iters = (ctypes.c_int64 * n)()
        disp = np.zeros(n, dtype=np.float64)
        valid = [k for k in systems if 0 <= k < len(self.dims)]   # the library rejects the rest
        tot = sum(self.dims[k] * self.sizes[k] for k in valid)
        xm = np.zeros(tot, dtype=np.float64)
        mode = HD_QUENCH_SET_REFERENCE if set_reference else HD_QUENCH_CHECK
        fn = load().hd_quench_noalloc if no_alloc else load().hd_quench
        _check(self._h, fn(self._h, ids, n, float(ftol), int(max_iters), mode, iters, _darr(disp), _darr(xm)),
               "hd_quench_noalloc" if no_alloc else "hd_quench")
        minima, o = [], 0
        for k in systems:
            m = self.dims[k] * self.sizes[k]
            minima.append(xm[o:o + m].reshape(self.dims[k], self.sizes[k]).copy())
            o += m
        return [int(v) for v in iters], disp, minima

    def min_mode(self, s: int, max_iter: int = 300, tol: float = 1e-10, seed: int = 1):
        """Lowest Hessian eigenvalue over system s's degrees of freedom and its
        mode (hd_min_mode).  Returns (eps, iters, mode [dim][n])."""
        eps = ctypes.c_double()
        it = ctypes.c_int32()
        m = self._out(s) if 0 <= s < len(self.dims) else np.zeros(1)
        _check(self._h, load().hd_min_mode(self._h, int(s), int(max_iter), float(tol), int(seed), ctypes.byref(eps),
                                           ctypes.byref(it), _darr(m)), "hd_min_mode")
        return eps.value, it.value, m

    def min_mode_gradient(self, s: int, mode: np.ndarray) -> np.ndarray:
        """Gradient of the lowest eigenvalue over system s's degrees of
        freedom (hd_min_mode_gradient), [dim][n]: mobile atoms' rows, the
        rigid body's on each rigid atom."""
        g = self._out(s) if 0 <= s < len(self.dims) else np.zeros(1)
        q = np.ascontiguousarray(mode, dtype=np.float64)
        _check(self._h, load().hd_min_mode_gradient(self._h, int(s), _darr(q), _darr(g)), "hd_min_mode_gradient")
        return g

    # -- read-outs --------------------------------------------------------
    def _out(self, s):
        return np.zeros((self.dims[s], self.sizes[s]), dtype=np.float64)

    def forces(self, s: int, which: int = HD_FORCE_TOTAL) -> np.ndarray:
        o = self._out(s)
        _check(self._h, load().hd_read_forces(self._h, s, int(which), _darr(o)), "hd_read_forces")
        return o

    def positions(self, s: int) -> np.ndarray:
        o = self._out(s)
        _check(self._h, load().hd_read_positions(self._h, s, _darr(o)), "hd_read_positions")
        return o

    def velocities(self, s: int) -> np.ndarray:
        o = self._out(s)
        _check(self._h, load().hd_read_velocities(self._h, s, _darr(o)), "hd_read_velocities")
        return o

    def scalars(self, s: int) -> dict:
        sc = hd_scalars()
        _check(self._h, load().hd_read_scalars(self._h, s, ctypes.byref(sc)), "hd_read_scalars")
        return sc.as_dict()

    def scalars_batch(self, first: int = 0, count: Optional[int] = None) -> List[dict]:
        """Scalars of systems first .. first + count - 1 (default: all from
        first) in one device-to-host copy."""
        if count is None:
            count = self.num_systems() - first
        arr = (hd_scalars * max(count, 1))()
        _check(self._h, load().hd_read_scalars_batch(self._h, first, count, arr), "hd_read_scalars_batch")
        return [arr[k].as_dict() for k in range(count)]

    def copy_positions_device(self, s: int, dev_ptr: int):
        _check(self._h, load().hd_copy_positions_device(self._h, s, ctypes.c_void_p(dev_ptr)),
               "hd_copy_positions_device")

    def copy_forces_device(self, s: int, which: int, dev_ptr: int):
        _check(self._h, load().hd_copy_forces_device(self._h, s, int(which), ctypes.c_void_p(dev_ptr)),
               "hd_copy_forces_device")

    def batch_layout(self, s: int):
        """(offset, ntot): system s occupies atoms offset .. offset + n - 1 of
        the batch arrays, which hold ntot atoms."""
        off, nt = ctypes.c_int64(), ctypes.c_int64()
        _check(self._h, load().hd_batch_layout(self._h, int(s), ctypes.byref(off), ctypes.byref(nt)),
               "hd_batch_layout")
        return off.value, nt.value

    def bind_device(self, field: int, tensor=None):
        """Bind a batch field (HD_FIELD_*) to a caller-owned device tensor of
        shape (3, ntot), float64, contiguous, on the context's device
        (hd_bind_device); None unbinds.  The tensor is kept referenced here
        while bound."""
        if not hasattr(self, "_bound"):
            self._bound = {}
        ptr = None
        if tensor is not None:
            _, nt = self.batch_layout(0)
            shape = tuple(tensor.shape)
            if shape != (3, nt) or str(tensor.dtype) != "torch.float64" or not tensor.is_contiguous():
                raise ValueError(f"bind_device needs a contiguous float64 tensor of shape (3, {nt}), got "
                                 f"{shape} {tensor.dtype}")
            ptr = ctypes.c_void_p(tensor.data_ptr())
        _check(self._h, load().hd_bind_device(self._h, HD_ALL_SYSTEMS, int(field), ptr), "hd_bind_device")
        if tensor is None:
            self._bound.pop(int(field), None)
        else:
            self._bound[int(field)] = tensor

    def get_state(self, s: int) -> bytes:
        n = ctypes.c_size_t()
        L = load()
        _check(self._h, L.hd_get_state(self._h, s, None, ctypes.byref(n)), "hd_get_state")
        buf = ctypes.create_string_buffer(n.value)
        _check(self._h, L.hd_get_state(self._h, s, buf, ctypes.byref(n)), "hd_get_state")
        return buf.raw

    def set_state(self, s: int, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._h, load().hd_set_state(self._h, s, buf, len(blob)), "hd_set_state")

    def debug_pairs(self, s: int) -> np.ndarray:
        L = load()
        n = ctypes.c_int64()
        _check(self._h, L.hd_debug_pairs(self._h, s, None, 0, ctypes.byref(n)), "hd_debug_pairs")
        out = np.zeros((max(n.value, 1), 2), dtype=np.int32)
        _check(self._h, L.hd_debug_pairs(self._h, s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         n.value, ctypes.byref(n)), "hd_debug_pairs")
        return out[: n.value]


def make_context(specs: Sequence, precision: int = HD_FP32C, exec_mode: int = HD_EXEC_BATCHED,
                 init_velocities: bool = True, block_threads: int = 0, stream=None,
                 max_neighbors: int = 0, lds_resident: bool = True,
                 persistent_large: bool = False) -> Context:
    """Context holding every spec, finalized, with Maxwell-Boltzmann velocities."""
    ctx = Context(precision, 0, stream, exec_mode, block_threads, max_neighbors, lds_resident,
                  persistent_large)
    for sp in specs:
        s = ctx.add_system(sp)
        if init_velocities:
            ctx.init_velocities(s)
    ctx.finalize()
    return ctx
