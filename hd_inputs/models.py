"""Seeded synthetic inputs for the AFM tip/substrate models.

This module only lays atoms on lattices and draws seeded workload parameters.
It holds none of the method's arithmetic (no potential, no force, no
integrator) so that the CPU oracle and the GPU path can both consume it
without sharing any computation.

Geometry follows the paper's model descriptions: a 2D close-packed
("FCC in 2D") substrate with a tip in registry (Sec. 3.1.1) and a 3D fcc
substrate joined to an fcc tip along [001] (Sec. 3.2.1).  Sizes are those
of the benchmark workloads (40x10 + 10x8 in 2D; 20x20x6 cells + a
hemispherical tip in 3D; 1M-atom slab; uneven batches).

Conventions
-----------
* reduced LJ units (eps = sigma = m = 1);
* nearest-neighbour distance 2**(1/6) (the LJ minimum, which is also the
  bond length the paper quotes for its harmonic tip bonds, eq. 12);
* roles: 0 mobile, 1 fixed (bottom substrate layer), 2 rigid (top tip layer);
* types: 0 substrate, 1 tip;
* positions are SoA float64 arrays of shape (dim, n);
* periodic along x (2D) or x, y (3D); open along the normal axis.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ROLE_MOBILE, ROLE_FIXED, ROLE_RIGID = 0, 1, 2
TYPE_SUB, TYPE_TIP = 0, 1

A2D = 2.0 ** (1.0 / 6.0)          # 2D triangular nearest-neighbour distance
PITCH2D = A2D * math.sqrt(3.0) / 2.0
AFCC = 2.0 ** (2.0 / 3.0)         # fcc cube edge with NN distance 2**(1/6)
_TOL = 1e-9


@dataclasses.dataclass
class SystemSpec:
    """One AFM model instance: geometry plus all run parameters."""
    dim: int
    pos: np.ndarray                  # (dim, n) float64
    type: np.ndarray                 # (n,) uint8
    role: np.ndarray                 # (n,) uint8
    box: np.ndarray                  # (3,) float64; 0 on open axes
    periodic: np.ndarray             # (3,) int32
    mass: float = 1.0
    # Lennard-Jones table (energy-shifted at rc)
    eps: np.ndarray = dataclasses.field(default_factory=lambda: np.ones((2, 2)))
    sig: np.ndarray = dataclasses.field(default_factory=lambda: np.ones((2, 2)))
    rc: float = 2.5
    skin: float = 0.3
    # thermostat: 0 Langevin (gamma), 1 Nose-Hoover chain of nhc_len
    # thermostats with relaxation time nhc_tau
    dt: float = 0.005
    gamma: float = 1.0
    kT: float = 0.1
    seed: int = 1
    thermostat: int = 0
    nhc_len: int = 3
    nhc_tau: float = 0.5
    # slider drive on the rigid layer
    k_spring: float = 1.0
    f_normal: float = 5.0
    x_slider: float = 0.0
    v_slider: float = 0.0
    # slope bias (eq. 14); disabled by default
    bias_on: int = 0
    m_b: int = 2
    dv_max: float = 0.5
    g_lo: float = 0.0
    g_hi: float = 1.0
    # bias variables: bias_var1 enters the switch above, bias_var2 (-1: none)
    # a second switch with b2_lo, b2_hi, combined by eq. 13; 0 slope (eq. 5),
    # 1 curvature (eq. 6), 2 distance (eq. 7)
    bias_var1: int = 0
    bias_var2: int = -1
    b2_lo: float = 0.0
    b2_hi: float = 1.0
    # harmonic tip bonds (eq. 12): tip-tip pairs closer than r_bond_cut are
    # springs of stiffness k_bond and rest length r_bond, farther tip-tip
    # pairs do not interact; off by default (tip-tip pairs are then LJ)
    tip_bonds: int = 0
    k_bond: float = 72.0 * 2.0 ** (-1.0 / 3.0)
    r_bond: float = 2.0 ** (1.0 / 6.0)
    r_bond_cut: float = 1.36
    # eigenvalue bias variable (bias_var 3): the mode estimate, atom layout
    # (dim, n) (rigid atoms the rigid body's component, fixed atoms 0), and
    # the step of its per-step rotation towards the lowest mode
    mode: Optional[np.ndarray] = None
    mode_alpha: float = 0.0
    # basin reference r_O (defaults to the lattice positions)
    rO: Optional[np.ndarray] = None
    label: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    def reference(self) -> np.ndarray:
        return self.pos.copy() if self.rO is None else self.rO

    def copy(self) -> "SystemSpec":
        c = dataclasses.replace(self)
        for f in ("pos", "type", "role", "box", "periodic", "eps", "sig"):
            setattr(c, f, getattr(self, f).copy())
        if self.rO is not None:
            c.rO = self.rO.copy()
        if self.mode is not None:
            c.mode = self.mode.copy()
        return c


# ----------------------------------------------------------------------------
# 2D: triangular lattice
# ----------------------------------------------------------------------------
def _tri_site(i: int, row: int) -> tuple:
    return ((i + 0.5 * (row & 1)) * A2D, row * PITCH2D)


def build_2d(nx: int = 40, ny: int = 10, tip: str = "block", tip_w: int = 10,
             tip_h: int = 8, R: float = 8.0, n_fixed_rows: int = 2,
             eps_ts: float = 0.5) -> SystemSpec:
    """2D close-packed substrate of nx x ny atoms (periodic in x, bottom
    n_fixed_rows rows fixed) with a tip in registry above it.

    tip='block': tip_w x tip_h block continuing the lattice, centred; its top
    row is rigid.  tip='halfdisk': lattice sites inside a half disk of radius
    R whose flat top row is rigid and whose lowest row sits one lattice row
    above the substrate.  tip='trapezoid': tip_h rows continuing the lattice,
    tip_w atoms in the lowest row and one more in each row above, all rows
    centred on one vertical line (the 2D counterpart of a cone with flat
    ends); its top row is rigid.
    """
    xs, ys, types, roles = [], [], [], []
    for row in range(ny):
        for i in range(nx):
            x, y = _tri_site(i, row)
            xs.append(x); ys.append(y)
            types.append(TYPE_SUB)
            roles.append(ROLE_FIXED if row < n_fixed_rows else ROLE_MOBILE)
    L = nx * A2D
    if tip == "block":
        i0 = (nx - tip_w) // 2
        for r in range(tip_h):
            row = ny + r
            for i in range(tip_w):
                x, y = _tri_site(i0 + i, row)
                xs.append(x); ys.append(y)
                types.append(TYPE_TIP)
                roles.append(ROLE_RIGID if r == tip_h - 1 else ROLE_MOBILE)
    elif tip == "trapezoid":
        # rows of width w = tip_w + r share the centre c (in units of A2D):
        # c = i0 + (w - 1)/2 + (row & 1)/2 for the first site i0 of each row,
        # an integer for every row since w and the row parity change together
        row0 = ny
        c2 = 2 * (nx // 2 - tip_w // 2) + (tip_w - 1) + (row0 & 1)    # 2c
        for r in range(tip_h):
            row, w = ny + r, tip_w + r
            twice_i0 = c2 - (w - 1) - (row & 1)
            assert twice_i0 % 2 == 0
            for j in range(w):
                x, y = _tri_site(twice_i0 // 2 + j, row)
                xs.append(x); ys.append(y)
                types.append(TYPE_TIP)
                roles.append(ROLE_RIGID if r == tip_h - 1 else ROLE_MOBILE)
    elif tip == "halfdisk":
        # find how many rows below the centre row the half disk reaches
        sites = []
        m = int(math.floor(R / PITCH2D)) + 1
        for drow in range(-m, 1):
            for di in range(-int(R / A2D) - 3, int(R / A2D) + 4):
                # centre on an even row: relative x uses the parity of drow
                dx = (di + 0.5 * (drow & 1)) * A2D
                dy = drow * PITCH2D
                if dx * dx + dy * dy <= R * R + _TOL:
                    sites.append((di, drow))
        apex = -min(d for _, d in sites)
        crow = ny + apex                      # absolute row of the centre
        ci = int(round((L / 2) / A2D))        # centre column
        if 2 * R + 2 * 2.8 > L:
            raise ValueError("half-disk tip wider than the periodic box")
        for di, drow in sites:
            row = crow + drow
            # keep registry: column index chosen so that x matches the
            # relative offset computed for an even centre row
            rel = (di + 0.5 * (drow & 1)) * A2D
            xc = (ci + 0.5 * (crow & 1)) * A2D
            x = xc + rel
            y = row * PITCH2D
            xs.append(x % L); ys.append(y)
            types.append(TYPE_TIP)
            roles.append(ROLE_RIGID if drow == 0 else ROLE_MOBILE)
    else:
        raise ValueError(tip)
    pos = np.array([xs, ys], dtype=np.float64)
    pos[0] = np.mod(pos[0], L)
    eps = np.array([[1.0, eps_ts], [eps_ts, 1.0]])
    return SystemSpec(dim=2, pos=pos, type=np.array(types, np.uint8),
                      role=np.array(roles, np.uint8),
                      box=np.array([L, 0.0, 0.0]), periodic=np.array([1, 0, 0], np.int32),
                      eps=eps, label=f"2d_{nx}x{ny}_{tip}")


def build_2d_paper() -> SystemSpec:
    """The paper's 2D model (§3.1.1): 80 substrate atoms (20 x 4 rows, bottom
    row fixed, periodic in x) and a 33-atom tip in registry (rows of 3, 4,
    ..., 8 atoms from the contact row up, top row rigid), spring k = 5,
    normal load F_N = 5, eps_ts = 0.5."""
    s = build_2d(nx=20, ny=4, tip="trapezoid", tip_w=3, tip_h=6, n_fixed_rows=1)
    s.k_spring, s.f_normal = 5.0, 5.0
    s.label = "2d_paper_80+33"
    return s


# ----------------------------------------------------------------------------
# 3D: fcc lattice, (001) layers stacked along z with spacing AFCC/2
# ----------------------------------------------------------------------------
def _fcc_halfsites(R: float):
    """Integer half-lattice coordinates (px, py, pz) (units of AFCC/2) of fcc
    sites with px+py+pz even, pz <= 0 and |p|*AFCC/2 <= R."""
    h = AFCC / 2.0
    m = int(math.floor(R / h)) + 1
    out = []
    for pz in range(-m, 1):
        for py in range(-m, m + 1):
            for px in range(-m, m + 1):
                if (px + py + pz) & 1:
                    continue
                r2 = (px * px + py * py + pz * pz) * h * h
                if r2 <= R * R + _TOL:
                    out.append((px, py, pz))
    return out


def build_3d(nx: int = 20, ny: int = 20, nz: int = 6, R: float = 8.0,
             eps_st: float = 0.2) -> SystemSpec:
    """fcc slab of nx x ny x nz cubic cells (periodic in x, y; bottom (001)
    layer fixed) with a hemispherical fcc tip of radius R in registry: the
    tip holds the lattice sites within R of a centre site and not above it;
    its flat top layer is rigid and its apex layer sits one layer spacing
    above the substrate's top layer."""
    h = AFCC / 2.0
    basis = ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1))   # in units of h
    px, py, pz = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for b in basis:
                    px.append(2 * i + b[0]); py.append(2 * j + b[1]); pz.append(2 * k + b[2])
    px = np.array(px); py = np.array(py); pz = np.array(pz)
    n_sub = px.size
    roles = np.where(pz == 0, ROLE_FIXED, ROLE_MOBILE).astype(np.uint8)
    types = np.zeros(n_sub, np.uint8)
    Lx, Ly = nx * AFCC, ny * AFCC
    if 2 * R + 2 * 2.8 > min(Lx, Ly):
        raise ValueError("tip wider than the periodic box")
    rel = _fcc_halfsites(R)
    apex = -min(p[2] for p in rel)
    cz = 2 * nz + apex                      # top substrate layer is 2nz-1
    cx, cy = nx, ny                         # box centre in units of h
    if (cx + cy + cz) & 1:
        cx += 1
    tpx = np.array([cx + p[0] for p in rel])
    tpy = np.array([cy + p[1] for p in rel])
    tpz = np.array([cz + p[2] for p in rel])
    troles = np.where(tpz == cz, ROLE_RIGID, ROLE_MOBILE).astype(np.uint8)
    px = np.concatenate([px, tpx]); py = np.concatenate([py, tpy]); pz = np.concatenate([pz, tpz])
    pos = np.stack([px * h, py * h, pz * h]).astype(np.float64)
    pos[0] = np.mod(pos[0], Lx)
    pos[1] = np.mod(pos[1], Ly)
    eps = np.array([[1.0, eps_st], [eps_st, 1.0]])
    return SystemSpec(dim=3, pos=pos,
                      type=np.concatenate([types, np.ones(len(rel), np.uint8)]),
                      role=np.concatenate([roles, troles]),
                      box=np.array([Lx, Ly, 0.0]), periodic=np.array([1, 1, 0], np.int32),
                      eps=eps, label=f"3d_{nx}x{ny}x{nz}_R{R:g}")


def _cone_sites(layers: int, r_apex: float, tan_half: float):
    """Half-lattice coordinates of an fcc cone along [001] with flat ends:
    layer t (t = 0 at the apex) holds the in-layer sites within
    r_apex + t h tan_half of the axis, which passes through a site."""
    h = AFCC / 2.0
    out = []
    for t in range(layers):
        r = r_apex + t * h * tan_half
        m = int(r / h) + 2
        for py in range(-m, m + 1):
            for px in range(-m, m + 1):
                if (px + py + t) & 1:
                    continue
                if (px * px + py * py) * h * h <= r * r + _TOL:
                    out.append((px, py, t))
    return out


def build_3d_cone(nx: int = 15, ny: int = 15, nz: int = 2, layers: int = 6, r_apex: float = 1.9,
                  tan_half: float = 0.78, eps_st: float = 0.2) -> SystemSpec:
    """The paper's 3D model (§3.2.1): an fcc substrate of nx x ny x nz cubic
    cells (1800 atoms by default; periodic in x, y, bottom layer fixed) and a
    conical fcc tip with flat ends in registry above it, its apex layer of 9
    atoms one layer spacing above the substrate, 183 atoms in 6 layers by
    default, top layer rigid; tip-tip interactions are the harmonic bonds of
    eq. 12, the slider spring k = 10."""
    h = AFCC / 2.0
    basis = ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1))
    px, py, pz = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for b in basis:
                    px.append(2 * i + b[0]); py.append(2 * j + b[1]); pz.append(2 * k + b[2])
    px = np.array(px); py = np.array(py); pz = np.array(pz)
    n_sub = px.size
    roles = np.where(pz == 0, ROLE_FIXED, ROLE_MOBILE).astype(np.uint8)
    Lx, Ly = nx * AFCC, ny * AFCC
    rel = _cone_sites(layers, r_apex, tan_half)
    top_r = r_apex + (layers - 1) * h * tan_half
    if 2 * top_r + 2 * 2.8 > min(Lx, Ly):
        raise ValueError("tip wider than the periodic box")
    cz = 2 * nz                              # apex layer: one spacing above the top layer 2nz-1
    cx, cy = nx, ny
    if (cx + cy + cz) & 1:
        cx += 1
    tpx = np.array([cx + p[0] for p in rel])
    tpy = np.array([cy + p[1] for p in rel])
    tpz = np.array([cz + p[2] for p in rel])
    troles = np.where(tpz == cz + layers - 1, ROLE_RIGID, ROLE_MOBILE).astype(np.uint8)
    px = np.concatenate([px, tpx]); py = np.concatenate([py, tpy]); pz = np.concatenate([pz, tpz])
    pos = np.stack([px * h, py * h, pz * h]).astype(np.float64)
    pos[0] = np.mod(pos[0], Lx)
    pos[1] = np.mod(pos[1], Ly)
    eps = np.array([[1.0, eps_st], [eps_st, 1.0]])
    return SystemSpec(dim=3, pos=pos,
                      type=np.concatenate([np.zeros(n_sub, np.uint8), np.ones(len(rel), np.uint8)]),
                      role=np.concatenate([roles, troles]),
                      box=np.array([Lx, Ly, 0.0]), periodic=np.array([1, 1, 0], np.int32),
                      eps=eps, k_spring=10.0, tip_bonds=1,
                      label=f"3d_cone_{nx}x{ny}x{nz}_{len(rel)}")


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
def seed_for(base: int, k: int) -> int:
    """Per-system seed of system k of a batch drawn from a base seed."""
    return (int(base) << 20) + int(k)


def config_c1() -> List[SystemSpec]:
    """2D plain MD, one slider position, continuous sliding at v = 0.01."""
    s = build_2d()
    s.k_spring, s.v_slider, s.kT, s.gamma, s.dt = 1.0, 0.01, 0.1, 1.0, 0.005
    s.seed = seed_for(1001, 0)
    s.label = "C1"
    return [s]


def config_c2(n_sys: int = 32) -> List[SystemSpec]:
    """2D model at n_sys stepped slider positions spread over one lattice
    period; slope bias on (its thresholds are set by the harness)."""
    out = []
    for k in range(n_sys):
        s = build_2d()
        s.k_spring, s.kT, s.gamma, s.dt = 1.0, 0.1, 1.0, 0.005
        s.x_slider = k * A2D / n_sys
        s.seed = seed_for(1002, k)
        s.bias_on = 1
        s.label = f"C2[{k}]"
        out.append(s)
    return out


def config_c3(n_sys: int = 64, nx: int = 20, nz: int = 6, R: float = 8.0) -> List[SystemSpec]:
    """3D fcc 20x20x6 slab + R=8 hemispherical tip at n_sys slider positions."""
    base = build_3d(nx, nx, nz, R)
    out = []
    for k in range(n_sys):
        s = base.copy()
        s.k_spring, s.f_normal, s.kT, s.gamma, s.dt = 1.0, 5.0, 0.1, 1.0, 0.005
        s.x_slider = k * AFCC / n_sys
        s.seed = seed_for(1003, k)
        s.bias_on = 1
        s.label = f"C3[{k}]"
        out.append(s)
    return out


def config_c4(n_sys: int = 128, seed: int = 1004, n_min: int = 500,
              n_max: int = 50000) -> List[SystemSpec]:
    """Uneven batch: seeded mix of 2D and 3D instances, log-uniform sizes,
    tip radii U[4, 12], temperatures U[0.05, 0.2]."""
    rng = np.random.default_rng(seed)
    out = []
    k = 0
    while len(out) < n_sys:
        dim = 2 if rng.random() < 0.5 else 3
        n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        R = rng.uniform(4.0, 12.0)
        kT = rng.uniform(0.05, 0.2)
        try:
            if dim == 2:
                ny = max(10, int(round(math.sqrt(n_target / 4.0))))
                nx = max(8, int(round(n_target / ny)))
                s = build_2d(nx, ny, tip="halfdisk", R=R)
            else:
                nxy = max(4, int(round(math.sqrt(n_target / 24.0))))
                s = build_3d(nxy, nxy, 6, R)
        except ValueError:
            continue                      # box narrower than the tip: redraw
        s.kT = kT
        s.k_spring, s.f_normal, s.gamma, s.dt = 1.0, 5.0, 1.0, 0.005
        a = A2D if dim == 2 else AFCC
        s.x_slider = (k % 16) * a / 16
        s.seed = seed_for(seed, k)
        s.bias_on = 1
        s.label = f"C4[{k}]"
        out.append(s)
        k += 1
    return out


def config_c5a() -> List[SystemSpec]:
    """One 1.0M-atom fcc slab (100x100x25 cells) with an R=20 tip."""
    s = build_3d(100, 100, 25, 20.0)
    s.k_spring, s.f_normal, s.kT, s.gamma, s.dt = 1.0, 5.0, 0.1, 1.0, 0.005
    s.seed = seed_for(1005, 0)
    s.bias_on = 1
    s.label = "C5a"
    return [s]


def config_c5b(n_sys: int = 256) -> List[SystemSpec]:
    """256 slider positions of an 8,072-atom 3D model (18x18x6 + R=5)."""
    base = build_3d(18, 18, 6, 5.0)
    out = []
    for k in range(n_sys):
        s = base.copy()
        s.k_spring, s.f_normal, s.kT, s.gamma, s.dt = 1.0, 5.0, 0.1, 1.0, 0.005
        s.x_slider = k * AFCC / n_sys
        s.seed = seed_for(1005, 1000 + k)
        s.bias_on = 1
        s.label = f"C5b[{k}]"
        out.append(s)
    return out


DX_SLIDER = 0.01   # the paper's slider step (§3.1.1)


def config_p2(n_sys: int = 256) -> List[SystemSpec]:
    """The paper's 2D model (113 atoms, spring k = 5) at n_sys consecutive
    slider positions k dx_S, dx_S = 0.01, T = 0.01, slope bias on."""
    base = build_2d_paper()
    out = []
    for k in range(n_sys):
        s = base.copy()
        s.kT, s.gamma, s.dt = 0.01, 1.0, 0.005
        s.x_slider = k * DX_SLIDER
        s.seed = seed_for(1007, k)
        s.bias_on = 1
        s.label = f"P2[{k}]"
        out.append(s)
    return out


def config_p3(n_sys: int = 256) -> List[SystemSpec]:
    """The paper's 3D model (1800-atom substrate, 183-atom conical tip with
    harmonic tip bonds, spring k = 10) at n_sys consecutive slider positions
    k dx_S, dx_S = 0.01, T = 0.1, slope bias on."""
    base = build_3d_cone()
    out = []
    for k in range(n_sys):
        s = base.copy()
        s.f_normal, s.kT, s.gamma, s.dt = 5.0, 0.1, 1.0, 0.005
        s.x_slider = k * DX_SLIDER
        s.seed = seed_for(1006, k)
        s.bias_on = 1
        s.label = f"P3[{k}]"
        out.append(s)
    return out


CONFIGS = {"C1": config_c1, "C2": config_c2, "C3": config_c3, "C4": config_c4,
           "C5a": config_c5a, "C5b": config_c5b, "P2": config_p2, "P3": config_p3}


def perturbed(spec: SystemSpec, amp: float, seed: int) -> np.ndarray:
    """Positions with seeded uniform jitter of amplitude amp on non-fixed atoms
    (rigid atoms move together), wrapped into the periodic box.  Used to make
    off-lattice snapshots for parity cases."""
    rng = np.random.default_rng(seed)
    x = spec.pos.copy()
    mob = spec.role == ROLE_MOBILE
    x[:, mob] += rng.uniform(-amp, amp, size=(spec.dim, int(mob.sum())))
    rig = spec.role == ROLE_RIGID
    if rig.any():
        x[:, rig] += rng.uniform(-amp, amp, size=(spec.dim, 1))
    for k in range(spec.dim):
        if spec.periodic[k]:
            x[k] = np.mod(x[k], spec.box[k])
    return x
