"""The eigenvalue bias variable of eq. 15 in the dynamics, on the GPU,
against the oracle (through the C ABI).

The variable is the Rayleigh quotient along each system's mode estimate, its
gradient T[w,w] comes from the same pair pass, and every step rotates the
mode once towards the lowest Hessian mode (the oracle's scheme, pinned there
against the library eigensolver).

Tolerances as in test_gpu_parity: float64 evaluations 1e-11 relative (1e-10
for T[w,w], which sums larger cancelling terms), 20-step float64
trajectories 1e-10; float32 forces 1e-5 relative L2 and
|dV - dV_ref| <= 1e-6 dV_max.
"""
import numpy as np
import pytest

from hd_inputs import build_2d, build_3d, build_3d_cone, perturbed

pytestmark = pytest.mark.gpu

ALPHA = 2e-4   # below 2 / (largest - smallest eigenvalue) of these models: a stable rotation


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def model_3d():
    return build_3d(10, 10, 4, 4.0)


MAKERS = {"2d": build_2d, "3d": model_3d, "cone": build_3d_cone}


def eig_spec(oracle_mod, name, seed, v1=3, v2=-1, kT=0.1):
    """Jittered model (r_O = lattice) biased on the eigenvalue (v1 = 3) or
    on the slope and the eigenvalue (v1 = 0, v2 = 3), thresholds bracketing
    the snapshot's values, a seeded mode estimate."""
    s = MAKERS[name]()
    s.x_slider, s.kT = 0.2, kT
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.mode = np.random.default_rng(seed).standard_normal((s.dim, s.n))
    s.mode_alpha = ALPHA
    s.bias_var1, s.bias_var2 = 3, -1
    r = oracle_mod.OracleSystem(s).compute()
    val = {0: r["g"], 3: r["lambda"]}

    def thresholds(v, frac):
        span = 2.0 * abs(val[v]) + 1.0
        return val[v] - frac * span, val[v] + (1.0 - frac) * span

    s.bias_on, s.m_b, s.dv_max = 1, 2, 5.0 * kT
    s.bias_var1, s.bias_var2 = v1, v2
    s.g_lo, s.g_hi = thresholds(v1, 0.4)
    if v2 >= 0:
        s.b2_lo, s.b2_hi = thresholds(v2, 0.6)
    return s


def min_image(spec, dx):
    dx = dx.copy()
    for k in range(spec.dim):
        if spec.periodic[k]:
            dx[k] -= spec.box[k] * np.round(dx[k] / spec.box[k])
    return dx


@pytest.mark.parametrize("name", ["2d", "3d", "cone"])
@pytest.mark.parametrize("v1,v2", [(3, -1), (0, 3)])
def test_evaluation_matches_oracle(hd, oracle_mod, name, v1, v2):
    spec = eig_spec(oracle_mod, name, 21, v1, v2)
    ref = oracle_mod.OracleSystem(spec).compute()
    assert 0.0 < ref["dv"] < spec.dv_max
    ctx = hd.make_context([spec], precision=hd.HD_FP64, init_velocities=False)
    sc = ctx.scalars(0)
    assert sc["lambda"] == pytest.approx(ref["lambda"], rel=1e-11)
    assert abs(sc["dv"] - ref["dv"]) <= 1e-11 * spec.dv_max
    assert sc["dv1"] == pytest.approx(ref["dv1"], rel=1e-10, abs=1e-12)
    assert sc["dv2"] == pytest.approx(ref["dv2"], rel=1e-10, abs=1e-12)
    assert rel(ctx.forces(0, hd.HD_TUU), ref["tuu"]) < 1e-10
    assert rel(ctx.forces(0, hd.HD_FORCE_BIAS), ref["f_b"]) < 1e-10
    assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) < 1e-11
    ctx.close()
    # float32 pair arithmetic: the stated tolerances
    ctx = hd.make_context([spec], precision=hd.HD_FP32C, init_velocities=False)
    sc = ctx.scalars(0)
    assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) <= 1e-5
    assert abs(sc["dv"] - ref["dv"]) <= 1e-6 * spec.dv_max
    ctx.close()


@pytest.mark.parametrize("name", ["2d", "3d", "cone"])
def test_trajectory_with_rotating_mode_matches_oracle(hd, oracle_mod, name):
    """20 biased steps (slope and eigenvalue, eq. 13): positions, the
    variable, dV and the rotated mode against the oracle's run from the same
    state and Philox stream."""
    spec = eig_spec(oracle_mod, name, 22, 0, 3)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(20)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, init_velocities=True)
    ctx.step(20)
    assert np.abs(min_image(spec, ctx.positions(0) - o.positions())).max() < 1e-10
    sc, so = ctx.scalars(0), o.scalars()
    assert sc["lambda"] == pytest.approx(so["lambda"], rel=1e-9)
    assert abs(sc["dv"] - so["dv"]) <= 1e-10 * spec.dv_max
    assert sc["t_hyper"] == pytest.approx(so["t_hyper"], rel=1e-10)
    q_gpu, q_ref = ctx.min_mode_estimate(0), o.mode()
    assert np.abs(q_gpu - q_ref).max() < 1e-9
    ctx.close()
    # float32: the same run within reach of the force tolerance (a force
    # error of 1e-5 |F_ref| held over n steps moves an atom by at most
    # (n dt)^2/2 times it; a factor 4 for its growth, as for the C3 batch)
    f_ref = oracle_mod.OracleSystem(spec).compute()["f_tot"]
    bound = 4.0 * 0.5 * (20 * spec.dt) ** 2 * 1e-5 * np.linalg.norm(f_ref)
    ctx = hd.make_context([spec], precision=hd.HD_FP32C, init_velocities=True)
    ctx.step(20)
    sc = ctx.scalars(0)
    assert np.abs(min_image(spec, ctx.positions(0) - o.positions())).max() < bound
    assert abs(sc["dv"] - so["dv"]) <= 1e-6 * spec.dv_max
    assert np.abs(ctx.min_mode_estimate(0) - q_ref).max() < 1e-4
    ctx.close()


def test_mode_converges_to_the_lowest_eigenvalue_on_the_gpu(hd, oracle_mod):
    """At rest at a minimum (no noise, no friction, bias off) the positions
    stay and the per-step rotation turns the mode to the reduced Hessian's
    lowest eigenvector: lambda reaches the library eigensolver's value."""
    spec = build_2d(nx=12, ny=4, tip_w=4, tip_h=3, n_fixed_rows=1)
    o = oracle_mod.OracleSystem(spec)
    assert o.fire(1e-10) >= 0
    x = o.positions()
    XR, _, XR0 = o.rigid()
    H = oracle_mod.reduced_hessian(spec, x)
    w = np.linalg.eigvalsh(0.5 * (H + H.T))
    s = spec.copy()
    s.pos = x
    s.rO = x.copy()
    s.gamma, s.kT = 0.0, 0.1
    # the drive measures the tip from its starting position: keep the
    # spring's stretch of the minimum
    s.x_slider = spec.x_slider - (XR[0] - XR0[0])
    s.bias_var1, s.bias_on = 3, 0
    s.mode = np.random.default_rng(3).standard_normal((s.dim, s.n))
    s.mode_alpha = 0.9 / w[-1]
    ctx = hd.make_context([s], precision=hd.HD_FP64, exec_mode=hd.HD_EXEC_GRID, init_velocities=False)
    ctx.step(3000)
    assert np.abs(min_image(s, ctx.positions(0) - x)).max() < 1e-9
    assert ctx.scalars(0)["lambda"] == pytest.approx(w[0], rel=1e-9)
    ctx.close()


def test_batch_with_lds_resident_slope_systems_and_checkpoint(hd, oracle_mod):
    """Eigenvalue-biased systems run on the grid kernels beside LDS-resident
    slope-biased ones; a checkpoint carries the mode, so a restored run
    continues bit for bit."""
    a = eig_spec(oracle_mod, "3d", 23, 0, 3)
    b = build_2d()
    b.rO = b.pos.copy()
    b.pos = perturbed(b, 0.05, 24)
    ctx = hd.make_context([b, a], precision=hd.HD_FP64, init_velocities=True)
    ctx.step(10)
    o = oracle_mod.OracleSystem(a)
    o.init_velocities()
    o.step(10)
    assert np.abs(min_image(a, ctx.positions(1) - o.positions())).max() < 1e-10
    st = ctx.get_state(1)
    ctx.step(10)
    x20, q20 = ctx.positions(1), ctx.min_mode_estimate(1)
    ctx.set_state(1, st)
    ctx.step(10)
    np.testing.assert_array_equal(ctx.positions(1), x20)
    np.testing.assert_array_equal(ctx.min_mode_estimate(1), q20)
    ctx.close()


def test_eigen_bias_argument_errors(hd, oracle_mod):
    spec = build_2d()
    ctx = hd.Context(hd.HD_FP64)
    s = ctx.add_system(spec)
    with pytest.raises(hd.HDError):
        ctx.set_min_mode(s, np.ones((2, spec.n)), 1e-3)      # not biased on the eigenvalue
    with pytest.raises(hd.HDError):
        ctx.set_bias_variables(s, hd.HD_BIAS_CURVATURE, hd.HD_BIAS_EIGENVALUE, 0.0, 1.0)
    ctx.set_bias_variables(s, hd.HD_BIAS_EIGENVALUE)
    with pytest.raises(hd.HDError):
        ctx.set_min_mode(s, np.ones((2, spec.n)), -1.0)
    ctx.set_min_mode(s, np.ones((2, spec.n)), 1e-3)
    ctx.finalize()
    q = ctx.min_mode_estimate(s)
    assert np.isfinite(q).all()
    ctx.close()
