"""ctypes wrapper for the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark.  The GPU product path never imports
this module, and this module never imports the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "hd_oracle.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with plain gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB_PATH, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32),
        ("box", ctypes.c_double * 3), ("periodic", ctypes.c_int32 * 3),
        ("mass", ctypes.c_double),
        ("eps", (ctypes.c_double * 2) * 2), ("sig", (ctypes.c_double * 2) * 2),
        ("rc", ctypes.c_double), ("skin", ctypes.c_double),
        ("dt", ctypes.c_double), ("gamma", ctypes.c_double), ("kT", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("k_spring", ctypes.c_double), ("f_normal", ctypes.c_double),
        ("x_slider", ctypes.c_double), ("v_slider", ctypes.c_double),
        ("bias_on", ctypes.c_int32), ("m_b", ctypes.c_int32),
        ("dv_max", ctypes.c_double), ("g_lo", ctypes.c_double), ("g_hi", ctypes.c_double),
        ("tip_bonds", ctypes.c_int32), ("pad_tb", ctypes.c_int32),
        ("k_bond", ctypes.c_double), ("r_bond", ctypes.c_double), ("r_bond_cut", ctypes.c_double),
        ("bias_var1", ctypes.c_int32), ("bias_var2", ctypes.c_int32),
        ("b2_lo", ctypes.c_double), ("b2_hi", ctypes.c_double),
        ("thermostat", ctypes.c_int32), ("nhc_len", ctypes.c_int32), ("nhc_tau", ctypes.c_double),
        ("mode_alpha", ctypes.c_double),
    ]


class OrcScalars(ctypes.Structure):
    _fields_ = [
        ("e_lj", ctypes.c_double), ("v_drive", ctypes.c_double),
        ("e_pot", ctypes.c_double), ("e_kin", ctypes.c_double),
        ("d", ctypes.c_double), ("g", ctypes.c_double),
        ("dv", ctypes.c_double), ("dvp", ctypes.c_double),
        ("x_slider", ctypes.c_double), ("x_tip", ctypes.c_double), ("f_lat", ctypes.c_double),
        ("t_md", ctypes.c_double), ("t_hyper", ctypes.c_double),
        ("step", ctypes.c_int64), ("flags", ctypes.c_int32), ("pad_f", ctypes.c_int32),
        ("kappa", ctypes.c_double), ("dv1", ctypes.c_double), ("dv2", ctypes.c_double),
        ("e_nhc", ctypes.c_double), ("lambda_", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        u8 = P(ctypes.c_uint8)
        vp = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.orc_normals.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, dp]
        for fn in (L.orc_pairs_brute, L.orc_pairs_cells):
            fn.argtypes = [P(OrcParams), dp, u8, ctypes.c_double, ctypes.c_int,
                           P(ctypes.c_int32), ctypes.c_int64]
            fn.restype = ctypes.c_int64
        L.orc_create.argtypes = [P(OrcParams), dp, u8, u8, dp]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_set_params.argtypes = [vp, P(OrcParams)]
        L.orc_set_positions.argtypes = [vp, dp]
        L.orc_set_velocities.argtypes = [vp, dp]
        L.orc_set_reference.argtypes = [vp, dp]
        L.orc_init_velocities.argtypes = [vp]
        L.orc_set_pair_method.argtypes = [vp, ctypes.c_int]
        L.orc_compute.argtypes = [vp, dp, dp, dp, dp, dp, P(OrcScalars)]
        L.orc_step.argtypes = [vp, ctypes.c_int64]
        L.orc_get_positions.argtypes = [vp, dp]
        L.orc_get_velocities.argtypes = [vp, dp]
        L.orc_get_scalars.argtypes = [vp, P(OrcScalars)]
        L.orc_get_rigid.argtypes = [vp, dp, dp, dp]
        L.orc_get_tuu.argtypes = [vp, dp]
        L.orc_get_nhc.argtypes = [vp, dp, dp]
        L.orc_set_nhc.argtypes = [vp, dp, dp]
        L.orc_set_mode.argtypes = [vp, dp]
        L.orc_get_mode.argtypes = [vp, dp]
        L.orc_rotate_mode.argtypes = [vp]
        L.orc_fire.argtypes = [vp, ctypes.c_double, ctypes.c_int64]
        L.orc_fire.restype = ctypes.c_int64
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def params_from_spec(spec, **over) -> OrcParams:
    p = OrcParams()
    p.dim, p.n = spec.dim, spec.n
    for k in range(3):
        p.box[k] = float(spec.box[k])
        p.periodic[k] = int(spec.periodic[k])
    p.mass = spec.mass
    for a in range(2):
        for b in range(2):
            p.eps[a][b] = float(spec.eps[a, b])
            p.sig[a][b] = float(spec.sig[a, b])
    p.rc, p.skin = spec.rc, spec.skin
    p.dt, p.gamma, p.kT = spec.dt, spec.gamma, spec.kT
    p.seed = int(spec.seed)
    p.k_spring, p.f_normal = spec.k_spring, spec.f_normal
    p.x_slider, p.v_slider = spec.x_slider, spec.v_slider
    p.bias_on, p.m_b = int(spec.bias_on), int(spec.m_b)
    p.dv_max, p.g_lo, p.g_hi = spec.dv_max, spec.g_lo, spec.g_hi
    p.tip_bonds = int(getattr(spec, "tip_bonds", 0))
    p.k_bond = float(getattr(spec, "k_bond", 0.0))
    p.r_bond = float(getattr(spec, "r_bond", 0.0))
    p.r_bond_cut = float(getattr(spec, "r_bond_cut", 0.0))
    p.bias_var1 = int(getattr(spec, "bias_var1", 0))
    p.bias_var2 = int(getattr(spec, "bias_var2", -1))
    p.b2_lo = float(getattr(spec, "b2_lo", 0.0))
    p.b2_hi = float(getattr(spec, "b2_hi", 1.0))
    p.thermostat = int(getattr(spec, "thermostat", 0))
    p.nhc_len = int(getattr(spec, "nhc_len", 3))
    p.nhc_tau = float(getattr(spec, "nhc_tau", 0.5))
    p.mode_alpha = float(getattr(spec, "mode_alpha", 0.0))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def normals(seed: int, step: int, particle: int, tag: int) -> np.ndarray:
    z = np.zeros(4)
    lib().orc_normals(int(seed), int(step), int(particle), int(tag), _dp(z))
    return z


def _pairs(fn, spec, x, rl, exclude):
    p = params_from_spec(spec)
    x = np.ascontiguousarray(x, dtype=np.float64)
    role = np.ascontiguousarray(spec.role, dtype=np.uint8)
    cap = 64
    while True:
        out = np.zeros((cap, 2), dtype=np.int32)
        cnt = fn(ctypes.byref(p), _dp(x), _u8(role), float(rl), int(exclude),
                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
        if cnt <= cap:
            return out[:cnt]
        cap = int(cnt)


def pairs_brute(spec, x, rl, exclude=True) -> np.ndarray:
    """(i, j), i < j, with r^2 < rl^2 by brute force."""
    return _pairs(lib().orc_pairs_brute, spec, x, rl, exclude)


def pairs_cells(spec, x, rl, exclude=True) -> np.ndarray:
    """Same set through the oracle's own cell list."""
    return _pairs(lib().orc_pairs_cells, spec, x, rl, exclude)


class OracleSystem:
    """One AFM model instance advanced by the FP64 oracle."""

    def __init__(self, spec, x=None, rO=None, brute=False, **param_over):
        self.spec = spec
        self.dim, self.n = spec.dim, spec.n
        self._p = params_from_spec(spec, **param_over)
        x = np.ascontiguousarray(spec.pos if x is None else x, dtype=np.float64)
        rO = np.ascontiguousarray(spec.reference() if rO is None else rO, dtype=np.float64)
        self._type = np.ascontiguousarray(spec.type, dtype=np.uint8)
        self._role = np.ascontiguousarray(spec.role, dtype=np.uint8)
        self._h = lib().orc_create(ctypes.byref(self._p), _dp(x), _u8(self._type),
                                   _u8(self._role), _dp(rO))
        lib().orc_set_pair_method(self._h, 1 if brute else 0)
        if getattr(spec, "mode", None) is not None:
            self.set_mode(spec.mode)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_params(self, **over):
        for k, v in over.items():
            setattr(self._p, k, v)
        lib().orc_set_params(self._h, ctypes.byref(self._p))

    def set_positions(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        lib().orc_set_positions(self._h, _dp(x))

    def set_velocities(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        lib().orc_set_velocities(self._h, _dp(v))

    def set_reference(self, rO):
        rO = np.ascontiguousarray(rO, dtype=np.float64)
        lib().orc_set_reference(self._h, _dp(rO))

    def init_velocities(self):
        lib().orc_init_velocities(self._h)

    def compute(self) -> dict:
        nd = (self.dim, self.n)
        f, hu, fb, ft = (np.zeros(nd) for _ in range(4))
        e = np.zeros(self.n)
        sc = OrcScalars()
        lib().orc_compute(self._h, _dp(f), _dp(hu), _dp(fb), _dp(ft), _dp(e), ctypes.byref(sc))
        t = np.zeros(nd)
        lib().orc_get_tuu(self._h, _dp(t))
        return {"f_lj": f, "hu": hu, "f_b": fb, "f_tot": ft, "e_atom": e, "tuu": t, **sc.as_dict()}

    def step(self, nsteps: int):
        lib().orc_step(self._h, int(nsteps))

    def positions(self) -> np.ndarray:
        x = np.zeros((self.dim, self.n))
        lib().orc_get_positions(self._h, _dp(x))
        return x

    def velocities(self) -> np.ndarray:
        v = np.zeros((self.dim, self.n))
        lib().orc_get_velocities(self._h, _dp(v))
        return v

    def scalars(self) -> dict:
        sc = OrcScalars()
        lib().orc_get_scalars(self._h, ctypes.byref(sc))
        return sc.as_dict()

    def rigid(self):
        a, b, c = np.zeros(3), np.zeros(3), np.zeros(3)
        lib().orc_get_rigid(self._h, _dp(a), _dp(b), _dp(c))
        return a, b, c

    def nhc(self):
        xi, eta = np.zeros(4), np.zeros(4)
        lib().orc_get_nhc(self._h, _dp(xi), _dp(eta))
        return xi, eta

    def set_nhc(self, xi, eta):
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        lib().orc_set_nhc(self._h, _dp(xi), _dp(eta))

    def set_mode(self, q):
        """Mode estimate of the eigenvalue variable, atom layout [dim][n]
        (rigid body read from its first atom)."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        lib().orc_set_mode(self._h, _dp(q))

    def mode(self) -> np.ndarray:
        """The mode estimate normalised over the degrees of freedom."""
        q = np.zeros((self.dim, self.n))
        lib().orc_get_mode(self._h, _dp(q))
        return q

    def rotate_mode(self):
        """Evaluate at the current positions and rotate the mode once."""
        lib().orc_rotate_mode(self._h)

    def fire(self, ftol=1e-10, maxit=200000) -> int:
        return int(lib().orc_fire(self._h, float(ftol), int(maxit)))


# --------------------------------------------------------------------------
# The eigenvalue bias variable (§2.2; eq. 15 uses it): the lowest eigenvalue
# of the Hessian of the unbiased potential over the degrees of freedom.
# --------------------------------------------------------------------------
ROLE_MOBILE_, ROLE_RIGID_ = 0, 2


def dof_layout(spec):
    """Degrees of freedom of a model: each mobile atom's coordinates (atom by
    atom, dim each), then the rigid body's (dim), when it has rigid atoms."""
    mob = np.flatnonzero(spec.role == ROLE_MOBILE_)
    rig = np.flatnonzero(spec.role == ROLE_RIGID_)
    return mob, rig, spec.dim * len(mob) + (spec.dim if len(rig) else 0)


def dof_to_atoms(spec, q):
    """Atom displacements [dim][n] of a degree-of-freedom vector: fixed atoms
    stay, every rigid atom moves with the rigid body."""
    mob, rig, m = dof_layout(spec)
    w = np.zeros((spec.dim, spec.n))
    w[:, mob] = np.asarray(q[:spec.dim * len(mob)]).reshape(len(mob), spec.dim).T
    if len(rig):
        w[:, rig] = np.asarray(q[spec.dim * len(mob):]).reshape(spec.dim, 1)
    return w


def reduced_hessian(spec, x=None) -> np.ndarray:
    """Hessian of the unbiased potential (pairs and drive) over the degrees of
    freedom at positions x, assembled column by column from the oracle's
    Hessian-vector product: column q is H applied to the unit displacement of
    degree of freedom q (u = x - r_O with r_O moved by it), the rigid body's
    row collecting its atoms' rows.  Slow (one evaluation per degree of
    freedom): small models only."""
    x = np.asarray(spec.pos if x is None else x, dtype=np.float64)
    mob, rig, m = dof_layout(spec)
    o = OracleSystem(spec, x=x)
    o.set_params(bias_on=0)
    H = np.zeros((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        o.set_reference(x - dof_to_atoms(spec, e))
        hu = o.compute()["hu"]
        col = list(hu[:, mob].T.reshape(-1))
        if len(rig):
            col += list(hu[:, rig].sum(axis=1))
        H[:, c] = col
    return H


def lowest_hessian_eigenvalue(spec, x=None):
    """The eigenvalue bias variable: the smallest eigenvalue of
    reduced_hessian (library symmetric eigensolver) and its unit eigenvector
    over the degrees of freedom."""
    H = reduced_hessian(spec, x)
    vals, vecs = np.linalg.eigh(0.5 * (H + H.T))
    return float(vals[0]), vecs[:, 0]


def dof_project(spec, a):
    """An atom vector [dim][n] projected onto the degrees of freedom (the
    transpose of dof_to_atoms): mobile atoms' entries, then the sum over the
    rigid atoms."""
    mob, rig, m = dof_layout(spec)
    out = list(np.asarray(a)[:, mob].T.reshape(-1))
    if len(rig):
        out += list(np.asarray(a)[:, rig].sum(axis=1))
    return np.array(out)


def eigenvalue_gradient(spec, x=None):
    """Gradient of the lowest eigenvalue eps over the degrees of freedom
    (its derivative for the eigenvalue bias of eq. 13 and eq. 15): for a
    simple eigenvalue with unit eigenvector q, d eps = q^T dH q, i.e. the
    third derivatives of V contracted twice with the atom displacement
    w = P q -- the oracle's T[u,u] at u = w -- projected back by P^T.
    Returns (eps, q, gradient)."""
    x = np.asarray(spec.pos if x is None else x, dtype=np.float64)
    eps, q = lowest_hessian_eigenvalue(spec, x)
    o = OracleSystem(spec, x=x, rO=x - dof_to_atoms(spec, q))
    o.set_params(bias_on=0)
    return eps, q, dof_project(spec, o.compute()["tuu"])
