"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test below checks the oracle against something other than itself:
closed forms of eq. 9, the tip-bond constants printed with eq. 12, finite
differences of the energy (forces, Hu, slope g of eq. 5, bias force), the
boundary values of eq. 14, limits of eq. 3, Newton's third law, known-answer
vectors of Philox4x32-10, the exact stationary statistics of BAOAB on a
harmonic oscillator, time reversibility of velocity Verlet, and brute-force
neighbour sets.
"""
import math

import numpy as np
import pytest

from hd_inputs import (AFCC, A2D, ROLE_FIXED, ROLE_MOBILE, ROLE_RIGID, SystemSpec, build_3d_cone,
                       build_2d, build_3d, config_c5a, perturbed)
from tests.conftest import golden


def small2d(**kw):
    s = build_2d(nx=12, ny=4, tip_w=4, tip_h=3, n_fixed_rows=1)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def small3d(**kw):
    s = build_3d(7, 7, 2, R=2.0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def small_cone(**kw):
    """A small conical tip with harmonic tip bonds (eq. 12) on a thin slab."""
    s = build_3d_cone(nx=9, ny=9, nz=1, layers=4)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def pair_system(r, types=(0, 0), eps_ts=0.5):
    """Two mobile atoms on the x axis of a wide open 2D box."""
    pos = np.array([[10.0, 10.0 + r], [0.0, 0.0]])
    return SystemSpec(dim=2, pos=pos, type=np.array(types, np.uint8),
                      role=np.array([ROLE_MOBILE, ROLE_MOBILE], np.uint8),
                      box=np.array([40.0, 0.0, 0.0]), periodic=np.array([1, 0, 0], np.int32),
                      eps=np.array([[1.0, eps_ts], [eps_ts, 1.0]]))


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def test_philox_known_answers(oracle_mod):
    with open("tests/golden/philox4x32_10_kat.txt") as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(v, 16) for v in r]
        out = oracle_mod.philox4x32_10(vals[0:4], vals[4:6])
        assert list(out) == vals[6:10]


def test_normals_moments(oracle_mod):
    z = np.array([oracle_mod.normals(12345, s, p, 0) for s in range(50) for p in range(100)]).ravel()
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / z.size)
    # fourth moment of a standard normal is 3
    assert abs((z ** 4).mean() - 3.0) < 0.25
    # different tags and steps give different streams
    assert not np.array_equal(oracle_mod.normals(1, 0, 0, 0), oracle_mod.normals(1, 0, 0, 1))
    assert not np.array_equal(oracle_mod.normals(1, 0, 0, 0), oracle_mod.normals(1, 1, 0, 0))


# --------------------------------------------------------------------------
# Lennard-Jones closed forms (eq. 9) and the tip-bond constants (eq. 12)
# --------------------------------------------------------------------------
def test_lj_closed_forms(oracle_mod):
    g = golden("lj_closed_forms.txt")
    rmin = 2.0 ** (1.0 / 6.0)
    assert rmin == pytest.approx(float(g["r_min"]), rel=1e-15)
    o = oracle_mod.OracleSystem(pair_system(rmin))
    r = o.compute()
    assert np.abs(r["f_lj"]).max() < 1e-13
    assert r["e_lj"] == pytest.approx(float(g["well_depth_shifted"]), abs=1e-12)
    # force magnitude at r = sigma is 24 eps/sigma, repulsive
    o = oracle_mod.OracleSystem(pair_system(1.0))
    r = o.compute()
    assert r["f_lj"][0, 0] == pytest.approx(-float(g["force_at_sigma"]), rel=1e-14)
    assert r["f_lj"][0, 1] == pytest.approx(float(g["force_at_sigma"]), rel=1e-14)
    assert r["e_lj"] == pytest.approx(0.0 - float(g["phi_rc"]), abs=1e-14)
    # mixed pair scales with eps_ab
    o = oracle_mod.OracleSystem(pair_system(1.0, types=(0, 1), eps_ts=0.5))
    assert o.compute()["f_lj"][0, 1] == pytest.approx(12.0, rel=1e-14)
    # beyond the cutoff nothing interacts
    o = oracle_mod.OracleSystem(pair_system(2.5000001))
    r = o.compute()
    assert r["e_lj"] == 0.0 and np.all(r["f_lj"] == 0.0)


def test_hessian_at_minimum_matches_eq12(oracle_mod):
    """H u with u along the bond gives phi''(r_min) = 72 * 2^(-1/3), which the
    paper rounds to the harmonic stiffness k = 57.2 at r_O = 1.12 (eq. 12)."""
    g = golden("eq12_tip_bond.txt")
    c = golden("lj_closed_forms.txt")
    rmin = 2.0 ** (1.0 / 6.0)
    spec = pair_system(rmin)
    # reference r_O displaced so that u = (+1, 0) on atom 0 and 0 on atom 1
    rO = spec.pos.copy()
    rO[0, 0] -= 1.0
    o = oracle_mod.OracleSystem(spec, rO=rO)
    hu = o.compute()["hu"]
    # (Hu)_0 = H_pair (u_0 - u_1); along the bond that is phi''
    assert hu[0, 0] == pytest.approx(float(c["curvature_min"]), rel=1e-12)
    assert hu[0, 0] == pytest.approx(72.0 * 2.0 ** (-1.0 / 3.0), rel=1e-13)
    assert hu[0, 0] == pytest.approx(float(g["k"]), rel=float(g["rtol"]))
    assert rmin == pytest.approx(float(g["r_O"]), rel=float(g["rtol"]))
    # transverse direction: phi'(r_min)/r_min = 0
    rO = spec.pos.copy(); rO[1, 0] -= 1.0
    o = oracle_mod.OracleSystem(spec, rO=rO)
    assert abs(o.compute()["hu"][1, 0]) < 1e-12


# --------------------------------------------------------------------------
# Forces, Hu, slope and bias force against finite differences
# --------------------------------------------------------------------------
_SYSCACHE = {}


def _energy(oracle_mod, spec, x, rO, key="e_pot"):
    """Energy at positions x on a system created once per (spec, rO), so the
    drive's reference position X_R(0) stays that of the unperturbed model."""
    ck = (id(spec), None if rO is None else rO.tobytes())
    if ck not in _SYSCACHE:
        _SYSCACHE.clear()
        _SYSCACHE[ck] = (spec, oracle_mod.OracleSystem(spec, rO=rO))
    o = _SYSCACHE[ck][1]
    o.set_positions(x)
    r = o.compute()
    if key == "all":
        return r
    return r[key] if key != "bias" else r["dv"]


def _at(oracle_mod, spec, x, rO=None):
    """Full evaluation at x on the cached system (same X_R(0) as _energy)."""
    return _energy(oracle_mod, spec, x, rO, "all")


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone])
def test_forces_match_energy_gradient(oracle_mod, maker):
    spec = maker()
    x = perturbed(spec, 0.06, 7)
    r = _at(oracle_mod, spec, x)
    h = 1e-6
    mob = np.where(spec.role == ROLE_MOBILE)[0]
    for i in mob[:: max(1, len(mob) // 12)]:
        for k in range(spec.dim):
            xp = x.copy(); xp[k, i] += h
            xm = x.copy(); xm[k, i] -= h
            fd = -(_energy(oracle_mod, spec, xp, None) - _energy(oracle_mod, spec, xm, None)) / (2 * h)
            assert r["f_lj"][k, i] == pytest.approx(fd, rel=2e-6, abs=2e-6)


def test_rigid_body_force_matches_energy_gradient(oracle_mod):
    spec = small2d(x_slider=0.3)
    x = perturbed(spec, 0.05, 3)
    r = _at(oracle_mod, spec, x, spec.pos)
    rig = spec.role == ROLE_RIGID
    FR = r["f_lj"][:, rig].sum(axis=1)
    h = 1e-6
    for k in range(spec.dim):
        xp = x.copy(); xp[k, rig] += h
        xm = x.copy(); xm[k, rig] -= h
        fd = -(_energy(oracle_mod, spec, xp, spec.pos) - _energy(oracle_mod, spec, xm, spec.pos)) / (2 * h)
        assert FR[k] == pytest.approx(fd, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone])
def test_newton_third_law(oracle_mod, maker):
    """Internal LJ forces sum to zero; what remains is the drive on the rigid
    layer (spring along x, anchor along y in 3D, -F_N along the normal)."""
    spec = maker(x_slider=0.2)
    x = perturbed(spec, 0.05, 11)
    o = oracle_mod.OracleSystem(spec, x=x)
    r = o.compute()
    XR, _, XR0 = o.rigid()
    drive = np.zeros(spec.dim)
    drive[0] = spec.k_spring * (spec.x_slider - (XR[0] - XR0[0]))
    if spec.dim == 3:
        drive[1] = -spec.k_spring * (XR[1] - XR0[1])
    drive[-1] += -spec.f_normal
    total = r["f_lj"].sum(axis=1)
    scale = np.abs(r["f_lj"]).sum()
    assert np.all(np.abs(total - drive) <= 1e-12 * scale)
    assert r["f_lat"] == pytest.approx(drive[0], abs=1e-14)


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone])
def test_hu_matches_force_difference(oracle_mod, maker):
    """H u = -(F(r + h u) - F(r - h u)) / 2h (Hessian-vector product)."""
    spec = maker(x_slider=0.1)
    x = perturbed(spec, 0.05, 5)
    rO = spec.pos.copy()
    r = _at(oracle_mod, spec, x, rO)
    u = x - rO
    for k in range(spec.dim):
        if spec.periodic[k]:
            L = spec.box[k]
            u[k] = u[k] - L * np.round(u[k] / L)
    u[:, spec.role == ROLE_FIXED] = 0.0
    h = 1e-5
    fp = _at(oracle_mod, spec, x + h * u, rO)["f_lj"]
    fm = _at(oracle_mod, spec, x - h * u, rO)["f_lj"]
    fd = -(fp - fm) / (2 * h)
    nf = spec.role != ROLE_FIXED
    err = np.abs(fd[:, nf] - r["hu"][:, nf]).max() / np.abs(r["hu"][:, nf]).max()
    assert err < 1e-7


@pytest.mark.parametrize("maker", [small2d, small3d])
def test_slope_is_directional_derivative(oracle_mod, maker):
    """g = grad V . s with s = u/d (eq. 5, eq. 7)."""
    spec = maker(x_slider=0.1)
    x = perturbed(spec, 0.05, 9)
    rO = spec.pos.copy()
    r = _at(oracle_mod, spec, x, rO)
    u = x - rO
    for k in range(spec.dim):
        if spec.periodic[k]:
            u[k] -= spec.box[k] * np.round(u[k] / spec.box[k])
    u[:, spec.role == ROLE_FIXED] = 0.0
    d = math.sqrt((u * u).sum())
    assert r["d"] == pytest.approx(d, rel=1e-13)
    s = u / d
    h = 1e-6
    ep = _energy(oracle_mod, spec, x + h * s, rO)
    em = _energy(oracle_mod, spec, x - h * s, rO)
    assert r["g"] == pytest.approx((ep - em) / (2 * h), rel=1e-6)


def _bias_spec(oracle_mod, maker, x, rO, frac=0.4, m_b=2):
    """Thresholds placed so that the current g sits inside (g_L, g_U)."""
    spec = maker(x_slider=0.1)
    o = oracle_mod.OracleSystem(spec, rO=rO)
    o.set_positions(x)
    g0 = o.compute()["g"]
    span = 2.0 * abs(g0) + 1.0
    spec.bias_on, spec.m_b, spec.dv_max = 1, m_b, 0.7
    spec.g_lo = g0 - frac * span
    spec.g_hi = g0 + (1.0 - frac) * span
    return spec


def test_bias_switch_boundaries_and_derivative(oracle_mod):
    spec = small2d()
    x = perturbed(spec, 0.05, 2)
    rO = spec.pos.copy()
    base = _bias_spec(oracle_mod, small2d, x, rO)
    g0 = oracle_mod.OracleSystem(base, x=x, rO=rO).compute()["g"]

    def dv_at(shift, m_b=2):
        # dV(g0 + shift) == dV evaluated with both thresholds moved by -shift
        s = base.copy(); s.m_b = m_b
        s.g_lo, s.g_hi = base.g_lo - shift, base.g_hi - shift
        r = oracle_mod.OracleSystem(s, x=x, rO=rO).compute()
        return r["dv"], r["dvp"]

    # plateau values of eq. 14
    assert dv_at(base.g_hi - g0)[0] == base.dv_max      # g = g_U
    assert dv_at(base.g_hi - g0 + 1.0)[0] == base.dv_max
    assert dv_at(base.g_lo - g0)[0] == 0.0              # g = g_L
    assert dv_at(base.g_lo - g0 - 1.0)[0] == 0.0
    # range [0, dV_max] (stated under eq. 15)
    for t in np.linspace(-1.2, 1.2, 25):
        v, _ = dv_at(t * (base.g_hi - base.g_lo))
        assert 0.0 <= v <= base.dv_max
    # derivative: analytic vs central difference; C1 at both ends for m >= 2
    for m_b in (1, 2, 3):
        for t in (0.1, 0.5, 0.9):
            sh = base.g_lo + t * (base.g_hi - base.g_lo) - g0
            h = 1e-6 * (base.g_hi - base.g_lo)
            _, dvp = dv_at(sh, m_b)
            fd = (dv_at(sh + h, m_b)[0] - dv_at(sh - h, m_b)[0]) / (2 * h)
            assert dvp == pytest.approx(fd, rel=1e-6)
    eps = 1e-7 * (base.g_hi - base.g_lo)
    assert dv_at(base.g_hi - g0 - eps)[1] < 1e-5
    assert dv_at(base.g_lo - g0 + eps)[1] < 1e-5
    # closed form in the middle for m = 2: xi = 1/2 -> dV = dVmax (1 - 1/4)^2
    mid = 0.5 * (base.g_lo + base.g_hi) - g0
    assert dv_at(mid)[0] == pytest.approx(base.dv_max * 0.75 ** 2, rel=1e-12)


@pytest.mark.parametrize("maker", [small2d, small3d])
def test_bias_force_matches_bias_gradient(oracle_mod, maker):
    spec0 = maker()
    x = perturbed(spec0, 0.05, 4)
    rO = spec0.pos.copy()
    spec = _bias_spec(oracle_mod, maker, x, rO)
    r = _at(oracle_mod, spec, x, rO)
    assert 0.0 < r["dv"] < spec.dv_max
    h = 1e-6
    mob = np.where(spec.role == ROLE_MOBILE)[0]
    worst = 0.0
    scale = np.abs(r["f_b"]).max()
    for i in mob[:: max(1, len(mob) // 10)]:
        for k in range(spec.dim):
            xp = x.copy(); xp[k, i] += h
            xm = x.copy(); xm[k, i] -= h
            fd = -(_energy(oracle_mod, spec, xp, rO, "bias") - _energy(oracle_mod, spec, xm, rO, "bias")) / (2 * h)
            worst = max(worst, abs(fd - r["f_b"][k, i]) / scale)
    assert worst < 1e-6
    # the rigid body as a whole
    rig = spec.role == ROLE_RIGID
    FbR = r["f_b"][:, rig].sum(axis=1)
    for k in range(spec.dim):
        xp = x.copy(); xp[k, rig] += h
        xm = x.copy(); xm[k, rig] -= h
        fd = -(_energy(oracle_mod, spec, xp, rO, "bias") - _energy(oracle_mod, spec, xm, rO, "bias")) / (2 * h)
        assert abs(fd - FbR[k]) / scale < 1e-6
    np.testing.assert_array_equal(r["f_tot"], r["f_lj"] + r["f_b"])


# --------------------------------------------------------------------------
# Boosted clock (eq. 3) limits
# --------------------------------------------------------------------------
def test_clock_limits(oracle_mod):
    spec = small2d(kT=0.1)
    spec.bias_on, spec.dv_max = 1, 0.3
    # dV == dVmax everywhere: bias force vanishes, trajectory equals the
    # unbiased one bit for bit, t_hyper = t_MD exp(dVmax/kT)
    full = spec.copy(); full.g_lo, full.g_hi = -2e30, -1e30
    off = spec.copy(); off.bias_on = 0
    a = oracle_mod.OracleSystem(full); a.init_velocities(); a.step(60)
    b = oracle_mod.OracleSystem(off); b.init_velocities(); b.step(60)
    np.testing.assert_array_equal(a.positions(), b.positions())
    np.testing.assert_array_equal(a.velocities(), b.velocities())
    sa = a.scalars()
    assert sa["dv"] == spec.dv_max
    assert sa["t_hyper"] == pytest.approx(sa["t_md"] * math.exp(spec.dv_max / spec.kT), rel=1e-13)
    assert sa["t_md"] == pytest.approx(60 * spec.dt, rel=1e-13)
    # dV == 0 everywhere: t_hyper == t_MD
    zero = spec.copy(); zero.g_lo, zero.g_hi = 1e30, 2e30
    c = oracle_mod.OracleSystem(zero); c.init_velocities(); c.step(30)
    sc = c.scalars()
    assert sc["t_hyper"] == sc["t_md"]


# --------------------------------------------------------------------------
# Integrator
# --------------------------------------------------------------------------
def test_velocity_verlet_time_reversible(oracle_mod):
    """gamma = 0, kT = 0: BAOAB is velocity Verlet, exactly time reversible."""
    spec = small2d(gamma=0.0, kT=0.0, x_slider=0.2)
    x = perturbed(spec, 0.05, 21)
    o = oracle_mod.OracleSystem(spec, x=x)
    v0 = np.zeros((2, spec.n))
    rng = np.random.default_rng(0)
    v0[:, spec.role == ROLE_MOBILE] = rng.normal(0, 0.3, size=(2, int((spec.role == ROLE_MOBILE).sum())))
    v0[:, spec.role == ROLE_RIGID] = 0.05
    o.set_velocities(v0)
    x0 = o.positions()
    o.step(200)
    o.set_velocities(-o.velocities())
    o.step(200)
    d = o.positions() - x0
    d[0] -= spec.box[0] * np.round(d[0] / spec.box[0])
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-o.velocities(), v0, atol=1e-9)


@pytest.mark.parametrize("bias", [0, 1])
def test_nve_energy_error_is_second_order(oracle_mod, bias):
    """Energy fluctuation of velocity Verlet scales as dt^2; with the bias on
    the conserved quantity is K + V + dV."""
    spec = small2d(gamma=0.0, kT=0.0, x_slider=0.15)
    x = perturbed(spec, 0.04, 8)
    if bias:
        spec = _bias_spec(oracle_mod, small2d, x, spec.pos.copy(), frac=0.3)
        spec.gamma, spec.kT = 0.0, 1.0   # kT only scales the clock here

    def spread(dt, nsteps):
        s = spec.copy(); s.dt = dt
        o = oracle_mod.OracleSystem(s, x=x)
        rng = np.random.default_rng(1)
        v = np.zeros((2, s.n))
        v[:, s.role == ROLE_MOBILE] = rng.normal(0, 0.2, size=(2, int((s.role == ROLE_MOBILE).sum())))
        o.set_velocities(v)
        tot = []
        for _ in range(nsteps):
            o.step(1)
            sc = o.scalars()
            tot.append(sc["e_pot"] + sc["e_kin"] + sc["dv"])
        tot = np.array(tot)
        return tot.max() - tot.min()

    e1 = spread(0.004, 250)
    e2 = spread(0.002, 500)
    assert e1 < 5e-3 * spec.n
    assert 3.0 < e1 / e2 < 5.0


def _harmonic_rigid_system(k, nR, kT, gamma, dt):
    """nR rigid atoms only: the drive spring makes X_R,x a harmonic oscillator
    of stiffness k and mass nR; no LJ (rigid-rigid pairs are excluded)."""
    pos = np.array([[1.0 + 1.2 * i for i in range(nR)], [5.0] * nR])
    return SystemSpec(dim=2, pos=pos, type=np.ones(nR, np.uint8),
                      role=np.full(nR, ROLE_RIGID, np.uint8),
                      box=np.array([50.0, 0, 0]), periodic=np.array([1, 0, 0], np.int32),
                      k_spring=k, f_normal=0.0, kT=kT, gamma=gamma, dt=dt, seed=99)


@pytest.mark.slow
def test_baoab_harmonic_stationary_statistics(oracle_mod):
    """BAOAB samples a harmonic oscillator's positions exactly for any stable
    dt: <x^2> = kT/k, while <v^2> = (kT/M)(1 - w^2 dt^2/4)."""
    k, nR, kT, gamma, dt = 4.0, 10, 1.0, 1.0, 1.0
    spec = _harmonic_rigid_system(k, nR, kT, gamma, dt)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(200)
    xs, vs = [], []
    for _ in range(60000):
        o.step(1)
        XR, VR, XR0 = o.rigid()
        xs.append(XR[0] - XR0[0]); vs.append(VR[0])
    xs, vs = np.array(xs), np.array(vs)
    M = float(nR)
    w2 = k / M
    assert (xs ** 2).mean() == pytest.approx(kT / k, rel=0.03)
    assert (vs ** 2).mean() == pytest.approx(kT / M * (1 - w2 * dt * dt / 4), rel=0.03)
    # and clearly not the continuous-time value kT/M
    assert abs((vs ** 2).mean() - kT / M) > 0.05 * kT / M


@pytest.mark.slow
def test_equipartition(oracle_mod):
    spec = small2d(kT=0.1, gamma=1.0)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(500)
    ndof = 2 * int((spec.role == ROLE_MOBILE).sum()) + 2
    ks = []
    for _ in range(200):
        o.step(10)
        ks.append(o.scalars()["e_kin"])
    assert np.mean(ks) / (0.5 * ndof) == pytest.approx(spec.kT, rel=0.04)


def test_maxwell_boltzmann_init(oracle_mod):
    spec = build_2d()
    spec.kT = 0.25
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    v = o.velocities()[:, spec.role == ROLE_MOBILE]
    assert v.var() == pytest.approx(spec.kT, rel=0.08)
    assert np.all(o.velocities()[:, spec.role == ROLE_FIXED] == 0.0)
    # draws follow the counter definition: atom i, tag 1, step 0
    i = int(np.where(spec.role == ROLE_MOBILE)[0][3])
    z = oracle_mod.normals(spec.seed, 0, i, 1)
    np.testing.assert_array_equal(o.velocities()[:, i], math.sqrt(spec.kT) * z[:2])


def _rigid_cluster(n_rigid, n_mobile=1, **kw):
    """A 2D model of n_rigid rigid atoms in a row (one body of mass
    n_rigid m) plus n_mobile mobile atoms far above it, out of reach."""
    n = n_rigid + n_mobile
    pos = np.zeros((2, n))
    pos[0, :n_rigid] = 1.0 + 1.2 * np.arange(n_rigid)
    pos[0, n_rigid:] = 1.0 + 1.2 * np.arange(n_mobile)
    pos[1, n_rigid:] = 10.0
    role = np.array([ROLE_RIGID] * n_rigid + [ROLE_MOBILE] * n_mobile, np.uint8)
    typ = np.ones(n, np.uint8)
    L = max(8.0, 1.2 * max(n_rigid, n_mobile) + 6.0)
    spec = SystemSpec(dim=2, pos=pos, type=typ, role=role, box=np.array([L, 0.0, 0.0]),
                      periodic=np.array([1, 0, 0], np.int32))
    for k, v in kw.items():
        setattr(spec, k, v)
    return spec


def test_rigid_body_maxwell_boltzmann_draw(oracle_mod):
    """The rigid top layer is one body of mass n_R m (Sec. 3.1.1): its
    Maxwell-Boltzmann velocity has variance kT/(n_R m) per axis, each of its
    atoms moves with it, and the draw is the counter-based one of particle
    index n (tag 1, step 0)."""
    n_rigid, kT = 10, 0.25
    vr = []
    for seed in range(1, 1501):
        spec = _rigid_cluster(n_rigid, kT=kT, seed=seed)
        o = oracle_mod.OracleSystem(spec)
        o.init_velocities()
        _, VR, _ = o.rigid()
        v = o.velocities()
        np.testing.assert_array_equal(v[:, :n_rigid], np.repeat(VR[:2, None], n_rigid, axis=1))
        vr.append(VR[:2])
        if seed == 1:
            z = oracle_mod.normals(seed, 0, spec.n, 1)
            np.testing.assert_allclose(VR[:2], math.sqrt(kT / n_rigid) * z[:2], rtol=1e-15)
    vr = np.array(vr)
    # 3000 samples: the variance is known to about 2.6 % (one sigma)
    assert vr.var() == pytest.approx(kT / n_rigid, rel=0.1)
    assert abs(vr.mean()) < 4.0 * math.sqrt(kT / n_rigid / vr.size)


@pytest.mark.parametrize("n_rigid", [1, 4])
def test_continuous_sliding_drives_the_exact_oscillator(oracle_mod, n_rigid):
    """Continuous sliding (Sec. 2.3, Fig. 1): the slider moves at constant
    velocity, x_S(t) = x_S(0) + v_S t, and pulls the rigid layer (mass
    M = n_R m) through the spring k.  Alone, started at rest at x_S(0) = 0,
    the layer obeys M Y'' = k (v_S t - Y), whose solution is
    Y(t) = v_S t - (v_S / w) sin(w t), w = sqrt(k/M).  Without friction the
    step is velocity Verlet, second order: after 2000 steps the layer is
    within 1e-6 of the solution (the error is ~1e-7); evaluating the slider
    one step late or early shifts it by ~5e-5."""
    v_s, dt, k, N = 0.01, 0.005, 1.0, 2000
    spec = _rigid_cluster(n_rigid, gamma=0.0, kT=0.1, dt=dt, k_spring=k, f_normal=0.0,
                          x_slider=0.0, v_slider=v_s)
    o = oracle_mod.OracleSystem(spec)
    o.step(N)
    XR, VR, XR0 = o.rigid()
    w = math.sqrt(k / n_rigid)
    t = N * dt
    sc = o.scalars()
    assert sc["t_md"] == pytest.approx(t, rel=1e-12)
    assert XR[0] - XR0[0] == pytest.approx(v_s * t - v_s / w * math.sin(w * t), abs=1e-6)
    assert VR[0] == pytest.approx(v_s * (1.0 - math.cos(w * t)), abs=1e-6)
    assert XR[1] == XR0[1] and VR[1] == 0.0
    # read-outs: the slider at the last evaluation and the lateral force
    # k (x_S - x_T) of eq. 10
    assert sc["x_slider"] == pytest.approx(v_s * sc["t_md"], rel=1e-12)
    assert sc["f_lat"] == pytest.approx(k * (sc["x_slider"] - sc["x_tip"]), rel=1e-12)
    assert sc["x_tip"] == pytest.approx(XR[0] - XR0[0], rel=1e-12)


def test_fixed_atoms_never_move_and_rigid_layer_stays_rigid(oracle_mod):
    spec = small3d(kT=0.2)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(40)
    x = o.positions()
    fx = spec.role == ROLE_FIXED
    np.testing.assert_array_equal(x[:, fx], spec.pos[:, fx])
    rig = np.where(spec.role == ROLE_RIGID)[0]
    d0 = spec.pos[:, rig] - spec.pos[:, rig[:1]]
    d1 = x[:, rig] - x[:, rig[:1]]
    for k in range(2):
        d1[k] -= spec.box[k] * np.round((d1[k] - d0[k]) / spec.box[k])
    np.testing.assert_allclose(d1, d0, atol=1e-12)


def test_fire_relaxes_to_a_minimum(oracle_mod):
    spec = small2d(x_slider=0.0)
    o = oracle_mod.OracleSystem(spec, x=perturbed(spec, 0.05, 1))
    e0 = o.compute()["e_pot"]
    it = o.fire(ftol=1e-8, maxit=100000)
    assert it >= 0
    r = o.compute()
    assert r["e_pot"] < e0
    mob = spec.role == ROLE_MOBILE
    assert np.sqrt((r["f_lj"][:, mob] ** 2).sum(0)).max() < 1e-8
    # at the minimum with r_O there, d = 0 and the guard sets g = 0
    o2 = oracle_mod.OracleSystem(spec, x=o.positions(), rO=o.positions())
    r2 = o2.compute()
    assert r2["d"] == 0.0 and r2["g"] == 0.0


# --------------------------------------------------------------------------
# Neighbour sets
# --------------------------------------------------------------------------
@pytest.mark.parametrize("maker", [small2d, small3d, lambda: build_2d(), lambda: build_3d(9, 9, 3, 3.0)])
def test_cell_pairs_equal_brute_force(oracle_mod, maker):
    spec = maker()
    x = perturbed(spec, 0.1, 13)
    for rl in (2.5, 2.8):
        for excl in (True, False):
            a = oracle_mod.pairs_brute(spec, x, rl, excl)
            b = oracle_mod.pairs_cells(spec, x, rl, excl)
            sa = set(map(tuple, a)); sb = set(map(tuple, b))
            assert len(sa) == len(a) and sa == sb


def test_pair_edge_cases(oracle_mod):
    # exactly r = rl (2.75 is exact in binary) is excluded; strict <
    spec = pair_system(2.75)
    assert len(oracle_mod.pairs_brute(spec, spec.pos, 2.75)) == 0
    assert len(oracle_mod.pairs_brute(spec, spec.pos, 2.7500000001)) == 1
    # pairs straddling the periodic wrap are found by both methods
    pos = np.array([[0.3, 39.5], [1.0, 1.0]])
    s2 = SystemSpec(dim=2, pos=pos, type=np.zeros(2, np.uint8), role=np.zeros(2, np.uint8),
                    box=np.array([40.0, 0, 0]), periodic=np.array([1, 0, 0], np.int32))
    assert len(oracle_mod.pairs_brute(s2, pos, 2.8)) == 1
    assert len(oracle_mod.pairs_cells(s2, pos, 2.8)) == 1
    # fixed-fixed and rigid-rigid pairs are excluded from the interaction set
    spec = build_2d()
    pairs = oracle_mod.pairs_brute(spec, spec.pos, 2.8, True)
    ro = spec.role
    assert not np.any((ro[pairs[:, 0]] == ROLE_FIXED) & (ro[pairs[:, 1]] == ROLE_FIXED))
    assert not np.any((ro[pairs[:, 0]] == ROLE_RIGID) & (ro[pairs[:, 1]] == ROLE_RIGID))


def test_model_sizes():
    g = golden("model_sizes.txt")
    s = build_2d()
    assert s.n == int(g["2d_total"])
    assert int((s.role == ROLE_FIXED).sum()) == int(g["2d_fixed"])
    assert int((s.role == ROLE_RIGID).sum()) == int(g["2d_rigid"])
    assert int((s.type == 1).sum()) == int(g["2d_tip"])
    t = build_3d()
    assert int((t.type == 0).sum()) == int(g["3d_substrate"])
    assert int((t.role == ROLE_FIXED).sum()) == int(g["3d_fixed"])
    # the 1M-atom slab of the large single-instance workload, as built
    (c5a,) = config_c5a()
    assert int((c5a.type == 0).sum()) == int(g["3d_large_substrate"])
    assert int((c5a.type == 1).sum()) == int(g["3d_large_tip"])
    assert c5a.n == int(g["3d_large_total"])
    assert int((c5a.role == ROLE_FIXED).sum()) == int(g["3d_large_fixed"])


@pytest.mark.parametrize("maker", [lambda: build_2d(), lambda: build_3d()])
def test_lattice_in_registry(oracle_mod, maker):
    """Nearest-neighbour distance everywhere (tip included) is 2^(1/6)."""
    spec = maker()
    pairs = oracle_mod.pairs_brute(spec, spec.pos, 1.2, False)
    d = spec.pos[:, pairs[:, 0]] - spec.pos[:, pairs[:, 1]]
    for k in range(spec.dim):
        if spec.periodic[k]:
            d[k] -= spec.box[k] * np.round(d[k] / spec.box[k])
    r = np.sqrt((d * d).sum(0))
    np.testing.assert_allclose(r, 2 ** (1 / 6), rtol=1e-12)
    # every atom has at least one nearest neighbour
    assert len(np.unique(pairs)) == spec.n


# --------------------------------------------------------------------------
# The eigenvalue bias variable: reduced Hessian and its lowest eigenvalue
# --------------------------------------------------------------------------
@pytest.mark.parametrize("maker", [small2d, small3d], ids=["2d", "3d"])
def test_reduced_hessian_is_the_energy_curvature(oracle_mod, maker):
    """q^T H q equals the second difference of the energy along the
    degree-of-freedom displacement q (mobile atoms and the rigid body), and
    H is symmetric: a wrong rigid-body row, a missing drive term or a sign
    slip fails this."""
    spec = maker(x_slider=0.3)
    x = perturbed(spec, 0.04, 3)
    H = oracle_mod.reduced_hessian(spec, x)
    assert np.abs(H - H.T).max() <= 1e-9 * np.abs(H).max()
    rng = np.random.default_rng(5)
    o = oracle_mod.OracleSystem(spec, x=x)
    o.set_params(bias_on=0)
    e0 = o.compute()["e_pot"]
    h = 1e-4
    for _ in range(3):
        q = rng.normal(size=H.shape[0])
        q /= np.linalg.norm(q)
        w = oracle_mod.dof_to_atoms(spec, q)
        ep = []
        for sgn in (1.0, -1.0):
            o2 = oracle_mod.OracleSystem(spec, x=x)
            o2.set_params(bias_on=0)
            o2.set_positions(x + sgn * h * w)
            ep.append(o2.compute()["e_pot"])
        fd = (ep[0] - 2.0 * e0 + ep[1]) / h ** 2
        assert fd == pytest.approx(q @ H @ q, rel=2e-4, abs=1e-4)


def test_lowest_eigenvalue_positive_at_a_minimum(oracle_mod):
    """At a FIRE minimum every curvature is positive, and the lowest
    eigenvalue bounds every Rayleigh quotient from below."""
    spec = small2d()
    o = oracle_mod.OracleSystem(spec, x=perturbed(spec, 0.05, 7))
    assert o.fire(ftol=1e-9, maxit=200000) >= 0
    x = o.positions()
    eps, v = oracle_mod.lowest_hessian_eigenvalue(spec, x)
    assert eps > 0.0
    H = oracle_mod.reduced_hessian(spec, x)
    assert v @ H @ v == pytest.approx(eps, rel=1e-10)
    rng = np.random.default_rng(9)
    for _ in range(5):
        q = rng.normal(size=H.shape[0])
        assert q @ H @ q / (q @ q) >= eps - 1e-12


# --------------------------------------------------------------------------
# Harmonic tip bonds (eq. 12)
# --------------------------------------------------------------------------
def test_harmonic_tip_bond_closed_forms(oracle_mod):
    """Two tip atoms with bonds on: energy k (r - r0)^2 / 2, force -k (r - r0)
    along the bond (zero at r0), H u = k u along the bond at r0 and
    (k (r - r0)/r) u across it; beyond the bond cut no interaction at all
    (not LJ, although within rc); substrate pairs stay LJ."""
    k, r0 = 72.0 * 2.0 ** (-1.0 / 3.0), 2.0 ** (1.0 / 6.0)
    for r in (r0, 1.05, 1.3, 1.5):
        spec = pair_system(r, types=(1, 1))
        spec.tip_bonds, spec.k_bond, spec.r_bond, spec.r_bond_cut = 1, k, r0, 1.36
        res = oracle_mod.OracleSystem(spec).compute()
        if r < 1.36:
            assert res["e_pot"] == pytest.approx(0.5 * k * (r - r0) ** 2, rel=1e-13, abs=1e-15)
            # Delta = x_0 - x_1 points along -x: F_0 = -k (r - r0)/r Delta
            assert res["f_lj"][0, 0] == pytest.approx(k * (r - r0), rel=1e-12, abs=1e-14)
            assert res["f_lj"][0, 1] == pytest.approx(-k * (r - r0), rel=1e-12, abs=1e-14)
        else:
            assert res["e_pot"] == 0.0 and np.all(res["f_lj"] == 0.0)
    # H u at r0: along the bond k u, across it 0
    spec = pair_system(r0, types=(1, 1))
    spec.tip_bonds, spec.k_bond, spec.r_bond, spec.r_bond_cut = 1, k, r0, 1.36
    for u_dir, want in (((1.0, 0.0), k), ((0.0, 1.0), 0.0)):
        rO = spec.pos.copy()
        rO[:, 0] -= 1e-3 * np.array(u_dir)          # u_0 = x - r_O = 1e-3 u_dir
        res = oracle_mod.OracleSystem(spec, rO=rO).compute()
        hu = res["hu"][:, 0]
        assert hu[0 if u_dir[0] else 1] == pytest.approx(want * 1e-3, rel=1e-9, abs=1e-15)
    # without bonds the same pair is LJ
    spec = pair_system(1.5, types=(1, 1))
    assert oracle_mod.OracleSystem(spec).compute()["e_pot"] != 0.0


def test_cone_model_is_the_papers():
    """§3.2.1: 1800 substrate atoms, 183 tip atoms with 9 at the apex in
    registry with the substrate, spring k = 10, tip bonds on."""
    s = build_3d_cone()
    tip = s.type == 1
    assert (~tip).sum() == 1800 and tip.sum() == 183
    z = np.round(s.pos[2, tip], 6)
    assert np.sum(z == z.min()) == 9
    assert s.k_spring == 10.0 and s.tip_bonds == 1


# --------------------------------------------------------------------------
# Curvature (eq. 6) and distance (eq. 7) as bias variables; eq. 13
# --------------------------------------------------------------------------
def _lj_derivs(r):
    """phi', phi'', phi''' of 4 (r^-12 - r^-6) (eq. 9, eps = sigma = 1)."""
    return (4.0 * (-12.0 * r ** -13 + 6.0 * r ** -7),
            4.0 * (156.0 * r ** -14 - 42.0 * r ** -8),
            4.0 * (-2184.0 * r ** -15 + 336.0 * r ** -9))


@pytest.mark.parametrize("bond", [False, True])
def test_curvature_and_third_derivative_closed_forms(oracle_mod, bond):
    """One pair, u = a e on atom 0 only (d = a): along the bond
    kappa = phi''(r) and T[u,u]_0 = a^2 phi'''(r) Delta/r; across it
    kappa = phi'(r)/r and T[u,u]_0 = a^2 (phi'' - phi'/r) Delta / r^2.
    For a harmonic tip bond (eq. 12) phi'' = k and phi''' = 0."""
    a = 1e-3
    k, r0 = 72.0 * 2.0 ** (-1.0 / 3.0), 2.0 ** (1.0 / 6.0)
    for r in (1.05, 1.12, 1.3):
        spec = pair_system(r, types=(1, 1) if bond else (0, 0))
        if bond:
            spec.tip_bonds, spec.k_bond, spec.r_bond, spec.r_bond_cut = 1, k, r0, 1.36
            d1, d2, d3 = k * (r - r0), k, 0.0
        else:
            d1, d2, d3 = _lj_derivs(r)
        Dx = -r                                  # Delta = x_0 - x_1 along x
        for along in (True, False):
            rO = spec.pos.copy()
            rO[0 if along else 1, 0] -= a
            res = oracle_mod.OracleSystem(spec, rO=rO).compute()
            assert res["d"] == pytest.approx(a, rel=1e-12)
            if along:
                assert res["kappa"] == pytest.approx(d2, rel=1e-9)
                assert res["tuu"][0, 0] == pytest.approx(a * a * d3 * Dx / r, rel=1e-9, abs=1e-15)
            else:
                assert res["kappa"] == pytest.approx(d1 / r, rel=1e-9, abs=1e-12)
                assert res["tuu"][0, 0] == pytest.approx(a * a * (d2 - d1 / r) * Dx / r ** 2, rel=1e-9)
            np.testing.assert_allclose(res["tuu"][:, 1], -res["tuu"][:, 0], rtol=1e-14)


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone])
def test_curvature_is_the_second_directional_derivative(oracle_mod, maker):
    """kappa = d2V/ds2 (eq. 6): along the ray r + h s the direction s stays
    u/d, so kappa is the derivative of the slope g (eq. 5) there, and the
    second difference of V."""
    spec = maker(x_slider=0.1)
    x = perturbed(spec, 0.05, 21)
    rO = spec.pos.copy()
    r = _at(oracle_mod, spec, x, rO)
    u = x - rO
    for k in range(spec.dim):
        if spec.periodic[k]:
            u[k] -= spec.box[k] * np.round(u[k] / spec.box[k])
    u[:, spec.role == ROLE_FIXED] = 0.0
    s = u / math.sqrt((u * u).sum())
    h = 1e-6
    gp = _at(oracle_mod, spec, x + h * s, rO)["g"]
    gm = _at(oracle_mod, spec, x - h * s, rO)["g"]
    assert r["kappa"] == pytest.approx((gp - gm) / (2 * h), rel=1e-6)
    # a step small enough that no pair crosses a cutoff inside it (the force
    # jumps there; in the cone model a pair crosses one within 1e-4)
    h = 2e-5
    e0 = _energy(oracle_mod, spec, x, rO)
    ep = _energy(oracle_mod, spec, x + h * s, rO)
    em = _energy(oracle_mod, spec, x - h * s, rO)
    # (a loose check: the rounding of E, ~1e-11 over a few thousand pair
    # terms, is divided by h^2)
    assert r["kappa"] == pytest.approx((ep - 2 * e0 + em) / h ** 2, rel=1e-3)


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone])
def test_third_derivative_matches_hessian_difference(oracle_mod, maker):
    """T[u,u] = grad of u.H(r) u at fixed u: moving one atom and its r_O
    together keeps u and changes only H."""
    spec = maker(x_slider=0.1)
    x = perturbed(spec, 0.05, 23)
    rO = spec.pos.copy()
    ref = oracle_mod.OracleSystem(spec, x=x, rO=rO).compute()
    nf = spec.role != ROLE_FIXED

    def uhu(xx, rr):
        o = oracle_mod.OracleSystem(spec, x=xx, rO=rr)
        res = o.compute()
        return res["kappa"] * res["d"] ** 2

    h = 1e-5
    mob = np.where(spec.role == ROLE_MOBILE)[0]
    scale = np.abs(ref["tuu"][:, nf]).max()
    for i in mob[:: max(1, len(mob) // 8)]:
        for k in range(spec.dim):
            e = np.zeros_like(x); e[k, i] = h
            fd = (uhu(x + e, rO + e) - uhu(x - e, rO - e)) / (2 * h)
            assert abs(fd - ref["tuu"][k, i]) <= 1e-6 * scale


def _var_spec(oracle_mod, maker, x, rO, v1, v2, frac1=0.4, frac2=0.6):
    """Bias on variables v1 (and v2), thresholds placed so that each variable
    sits inside its switch; the distance switch runs the other way (lo > hi)."""
    spec = maker(x_slider=0.1)
    if 3 in (v1, v2):
        # the eigenvalue variable along a seeded mode estimate
        spec.mode = np.random.default_rng(7).standard_normal((spec.dim, spec.n))
        spec.bias_var1 = 3
    res = oracle_mod.OracleSystem(spec, x=x, rO=rO).compute()
    val = {0: res["g"], 1: res["kappa"], 2: res["d"], 3: res["lambda"]}

    def thresholds(v, frac):
        span = 2.0 * abs(val[v]) + 1.0
        lo, hi = val[v] - frac * span, val[v] + (1.0 - frac) * span
        return (hi, lo) if v == 2 else (lo, hi)

    spec.bias_on, spec.m_b, spec.dv_max = 1, 2, 0.7
    spec.bias_var1, spec.bias_var2 = v1, v2
    spec.g_lo, spec.g_hi = thresholds(v1, frac1)
    if v2 >= 0:
        spec.b2_lo, spec.b2_hi = thresholds(v2, frac2)
    return spec


VAR_PAIRS = [(1, -1), (2, -1), (0, 1), (0, 2), (1, 2), (2, 0), (3, -1), (0, 3)]


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone], ids=["2d", "3d", "cone"])
@pytest.mark.parametrize("v1,v2", VAR_PAIRS)
def test_bias_force_matches_gradient_for_every_variable(oracle_mod, maker, v1, v2):
    spec0 = maker()
    x = perturbed(spec0, 0.05, 4)
    rO = spec0.pos.copy()
    spec = _var_spec(oracle_mod, maker, x, rO, v1, v2)
    r = _at(oracle_mod, spec, x, rO)
    assert 0.0 < r["dv"] < spec.dv_max
    h = 1e-6
    scale = np.abs(r["f_b"]).max()
    assert scale > 0.0
    mob = np.where(spec.role == ROLE_MOBILE)[0]
    for i in mob[:: max(1, len(mob) // 8)]:
        for k in range(spec.dim):
            xp = x.copy(); xp[k, i] += h
            xm = x.copy(); xm[k, i] -= h
            fd = -(_energy(oracle_mod, spec, xp, rO, "bias") - _energy(oracle_mod, spec, xm, rO, "bias")) / (2 * h)
            assert abs(fd - r["f_b"][k, i]) / scale < 1e-6
    rig = spec.role == ROLE_RIGID
    FbR = r["f_b"][:, rig].sum(axis=1)
    for k in range(spec.dim):
        xp = x.copy(); xp[k, rig] += h
        xm = x.copy(); xm[k, rig] -= h
        fd = -(_energy(oracle_mod, spec, xp, rO, "bias") - _energy(oracle_mod, spec, xm, rO, "bias")) / (2 * h)
        assert abs(fd - FbR[k]) / scale < 1e-6


def test_eq13_plateaus_and_symmetry(oracle_mod):
    """Eq. 13: dV2 = dV_max gives dV = dV_max with no force whatever dV1 is;
    dV2 = 0 gives exactly the one-variable bias; the two variables may be
    swapped; dV stays in [0, dV_max]."""
    spec0 = small3d()
    x = perturbed(spec0, 0.05, 8)
    rO = spec0.pos.copy()
    one = _var_spec(oracle_mod, small3d, x, rO, 0, -1)
    r1 = oracle_mod.OracleSystem(one, x=x, rO=rO).compute()
    assert 0.0 < r1["dv"] < one.dv_max
    d = r1["d"]
    for full in (True, False):
        s = one.copy()
        s.bias_var2 = 2
        # distance switch: full for d <= b2_hi, zero for d >= b2_lo
        s.b2_hi, s.b2_lo = (2 * d + 1, 3 * d + 2) if full else (0.1 * d, 0.5 * d)
        r = oracle_mod.OracleSystem(s, x=x, rO=rO).compute()
        if full:
            assert r["dv2"] == s.dv_max and r["dv"] == s.dv_max
            assert np.all(r["f_b"] == 0.0)
        else:
            assert r["dv2"] == 0.0 and r["dv"] == r1["dv"]
            np.testing.assert_array_equal(r["f_b"], r1["f_b"])
    a = _var_spec(oracle_mod, small3d, x, rO, 0, 1)
    b = a.copy()
    b.bias_var1, b.bias_var2 = 1, 0
    b.g_lo, b.g_hi, b.b2_lo, b.b2_hi = a.b2_lo, a.b2_hi, a.g_lo, a.g_hi
    ra = oracle_mod.OracleSystem(a, x=x, rO=rO).compute()
    rb = oracle_mod.OracleSystem(b, x=x, rO=rO).compute()
    assert ra["dv"] == rb["dv"] and 0.0 < ra["dv"] < a.dv_max
    np.testing.assert_array_equal(ra["f_b"], rb["f_b"])
    assert ra["dv"] == pytest.approx(ra["dv1"] + ra["dv2"] - ra["dv1"] * ra["dv2"] / a.dv_max, rel=1e-15)


def test_2d_paper_model():
    """§3.1.1: 80 substrate atoms with the bottom layer fixed, 33 tip atoms in
    registry (every tip site is a site of the substrate's lattice continued
    upwards), top tip row rigid, spring k = 5, F_N = 5, eps_ts = 0.5."""
    from hd_inputs import build_2d_paper
    s = build_2d_paper()
    tip = s.type == 1
    assert (~tip).sum() == 80 and tip.sum() == 33
    assert (s.role == ROLE_FIXED).sum() == 20 and np.all(s.type[s.role == ROLE_FIXED] == 0)
    a = 2.0 ** (1.0 / 6.0)
    pitch = a * math.sqrt(3.0) / 2.0
    rows = np.round(s.pos[1] / pitch).astype(int)
    np.testing.assert_allclose(s.pos[1], rows * pitch, atol=1e-12)
    # lattice sites: x = (i + (row mod 2)/2) a
    frac = s.pos[0] / a - 0.5 * (rows & 1)
    np.testing.assert_allclose(frac, np.round(frac), atol=1e-9)
    trow = rows[tip]
    widths = [int((trow == r).sum()) for r in range(trow.min(), trow.max() + 1)]
    assert widths == [3, 4, 5, 6, 7, 8]
    assert trow.min() == rows[~tip].max() + 1                # the contact row sits on the substrate
    assert np.all(s.role[tip & (rows == trow.max())] == ROLE_RIGID)
    assert s.k_spring == 5.0 and s.f_normal == 5.0 and s.eps[0, 1] == 0.5


# --------------------------------------------------------------------------
# Nose-Hoover chain thermostat (Sec. 3.1.1; Martyna, Klein, Tuckerman 1992)
# --------------------------------------------------------------------------
def _nhc(spec, tau=0.5, M=3):
    spec.thermostat, spec.nhc_len, spec.nhc_tau = 1, M, tau
    return spec


@pytest.mark.parametrize("M", [1, 3])
def test_nhc_time_reversible(oracle_mod, M):
    """The chain integrator is a symmetric splitting: reversing the particle
    and thermostat velocities retraces the trajectory."""
    spec = _nhc(small2d(kT=0.1, x_slider=0.2), M=M)
    x = perturbed(spec, 0.05, 21)
    o = oracle_mod.OracleSystem(spec, x=x)
    o.init_velocities()
    o.step(20)                               # the thermostats pick up speed
    x0, v0 = o.positions(), o.velocities()
    xi0, eta0 = o.nhc()
    assert np.abs(xi0[:M]).min() > 0.0
    o.step(150)
    o.set_velocities(-o.velocities())
    xi, eta = o.nhc()
    o.set_nhc(-xi, eta)
    o.step(150)
    d = o.positions() - x0
    d[0] -= spec.box[0] * np.round(d[0] / spec.box[0])
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-o.velocities(), v0, atol=1e-9)
    xi1, eta1 = o.nhc()
    np.testing.assert_allclose(-xi1, xi0, atol=1e-9)
    np.testing.assert_allclose(eta1, eta0, atol=1e-9)


@pytest.mark.parametrize("bias", [0, 1])
def test_nhc_extended_energy_error_is_second_order(oracle_mod, bias):
    """K + V (+ dV) + the chain's energy is the conserved quantity of the
    Nose-Hoover chain; velocity Verlet keeps it to O(dt^2)."""
    base = small2d(kT=0.1, x_slider=0.15)
    x = perturbed(base, 0.04, 8)
    spec = _bias_spec(oracle_mod, small2d, x, base.pos.copy(), frac=0.3) if bias else base
    spec.kT = 0.1
    _nhc(spec)

    def spread(dt, nsteps):
        s = spec.copy(); s.dt = dt
        o = oracle_mod.OracleSystem(s, x=x)
        o.init_velocities()
        tot = []
        for _ in range(nsteps):
            o.step(1)
            sc = o.scalars()
            tot.append(sc["e_pot"] + sc["e_kin"] + sc["dv"] + sc["e_nhc"])
        tot = np.array(tot)
        return tot.max() - tot.min(), o.nhc()[0]

    e1, xi = spread(0.004, 250)
    e2, _ = spread(0.002, 500)
    assert np.abs(xi).max() > 1e-3            # the chain did work
    assert 3.0 < e1 / e2 < 5.0


@pytest.mark.slow
def test_nhc_equipartition(oracle_mod):
    """The chain holds the kinetic temperature at kT: <K> = N_f kT / 2 with
    N_f the integrated degrees of freedom (mobile atoms and the rigid body)."""
    spec = _nhc(small2d(kT=0.1))
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(1000)
    ndof = 2 * int((spec.role == ROLE_MOBILE).sum()) + 2
    ks = []
    for _ in range(400):
        o.step(10)
        ks.append(o.scalars()["e_kin"])
    assert np.mean(ks) / (0.5 * ndof) == pytest.approx(spec.kT, rel=0.04)


def test_nhc_single_thermostat_fixes_the_mean_kinetic_energy(oracle_mod):
    """With one thermostat, Q dxi/dt = 2K - N_f kT: over a long bounded run
    its time average vanishes, so <2K> = N_f kT whatever the dynamics.  The
    rigid body alone (a harmonic oscillator along x, free along y) has
    N_f = 2."""
    spec = _nhc(_harmonic_rigid_system(4.0, 10, 1.0, 0.0, 0.05), tau=0.5, M=1)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    k2 = []
    for _ in range(40000):
        o.step(1)
        k2.append(2.0 * o.scalars()["e_kin"])
    assert np.mean(k2[5000:]) == pytest.approx(2 * spec.kT, rel=0.05)


@pytest.mark.parametrize("maker", [small2d, small_cone], ids=["2d", "cone"])
def test_eigenvalue_gradient_matches_eigenvalue_differences(oracle_mod, maker):
    """d eps / d y for a degree of freedom y against central differences of
    the library eigenvalue of the reduced Hessian (mobile atoms and the
    rigid body)."""
    spec = maker(x_slider=0.1)
    spec.pos = perturbed(spec, 0.04, 31)
    eps, q, grad = oracle_mod.eigenvalue_gradient(spec)
    mob, rig, m = oracle_mod.dof_layout(spec)
    h = 1e-5
    scale = np.abs(grad).max()
    picks = list(range(0, spec.dim * len(mob), max(1, spec.dim * len(mob) // 6))) + [m - 2, m - 1]
    for c in picks:
        e = np.zeros(m)
        e[c] = h
        dx = oracle_mod.dof_to_atoms(spec, e)
        ep = oracle_mod.lowest_hessian_eigenvalue(spec, spec.pos + dx)[0]
        em = oracle_mod.lowest_hessian_eigenvalue(spec, spec.pos - dx)[0]
        assert abs((ep - em) / (2 * h) - grad[c]) <= 1e-5 * scale, c


# --------------------------------------------------------------------------
# The eigenvalue variable along the trajectory (eq. 13, eq. 15)
# --------------------------------------------------------------------------
def _dof_vector(oracle_mod, spec, q_atoms):
    """Atom-layout mode -> vector over the degrees of freedom (mobile atoms,
    then the rigid body's component read from one rigid atom)."""
    mob, rig, m = oracle_mod.dof_layout(spec)
    out = list(np.asarray(q_atoms)[:, mob].T.reshape(-1))
    if len(rig):
        out += list(np.asarray(q_atoms)[:, rig[0]])
    return np.array(out)


def test_mode_rotation_converges_to_the_lowest_eigenvalue(oracle_mod):
    """One rotation step per time step, q <- q - alpha (H q - lambda q), is a
    gradient step on the Rayleigh quotient: at a fixed configuration the
    steps reach the library eigensolver's lowest eigenvalue of the reduced
    Hessian and its eigenvector (a model with a rigid layer, whose body's
    row and drive term take part)."""
    spec = small2d()
    o = oracle_mod.OracleSystem(spec)
    assert o.fire(1e-8) >= 0
    x = o.positions()
    H = oracle_mod.reduced_hessian(spec, x)
    w, V = np.linalg.eigh(0.5 * (H + H.T))
    assert w[1] - w[0] > 1.0            # a simple lowest eigenvalue
    s = spec.copy()
    s.pos, s.bias_var1, s.bias_on = x, 3, 0
    s.mode_alpha = 0.9 / w[-1]
    s.mode = np.random.default_rng(1).standard_normal((s.dim, s.n))
    r = oracle_mod.OracleSystem(s)
    lam = []
    for it in range(3000):
        r.rotate_mode()
        lam.append(r.scalars()["lambda"])
    assert lam[-1] == pytest.approx(w[0], rel=1e-10)
    assert lam[10] > lam[100] > lam[1000] > w[0] - 1e-9     # from above
    q = _dof_vector(oracle_mod, spec, r.mode())
    assert abs(np.linalg.norm(q) - 1.0) < 1e-12
    assert abs(float(q @ V[:, 0])) > 1.0 - 1e-9


@pytest.mark.parametrize("maker", [small2d, small_cone], ids=["2d", "cone"])
def test_eigen_variable_is_the_rayleigh_quotient(oracle_mod, maker):
    """Along the library eigenvector the variable is the lowest eigenvalue,
    and its gradient at fixed mode is the eigenvalue's gradient (pinned
    against differences of the library eigenvalue above); a scaled mode
    gives the same values (normalisation over the degrees of freedom)."""
    spec = maker()
    x = perturbed(spec, 0.03, 5)
    eps, q, grad = oracle_mod.eigenvalue_gradient(spec, x)
    s = spec.copy()
    s.pos, s.bias_var1, s.bias_on = x, 3, 0
    s.mode = 3.7 * oracle_mod.dof_to_atoms(spec, q)
    r = oracle_mod.OracleSystem(s).compute()
    assert r["lambda"] == pytest.approx(eps, rel=1e-10)
    g = oracle_mod.dof_project(spec, r["tuu"])
    np.testing.assert_allclose(g, grad, rtol=0, atol=1e-10 * np.abs(grad).max())
