"""Curvature (eq. 6) and distance (eq. 7) as bias variables and eq. 13 with
two variables, on the GPU against the oracle: bias force, total force,
T[u,u], the switches and the curvature, in both precisions and both
schedulers; a short biased trajectory; a batch mixing them with slope-only
systems; argument errors."""
import numpy as np
import pytest

from hd_inputs import build_2d, build_3d, build_3d_cone, perturbed

pytestmark = pytest.mark.gpu

VAR_PAIRS = [(1, -1), (2, -1), (0, 1), (0, 2), (1, 2), (2, 0)]


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


MAKERS = {
    "2d": lambda: build_2d(),
    "3d": lambda: build_3d(7, 7, 3, 2.0),
    "cone": lambda: build_3d_cone(nx=9, ny=9, nz=1, layers=4),
}


def biased(oracle_mod, model, v1, v2, seed, frac1=0.4, frac2=0.6):
    """A jittered snapshot biased on (v1, v2), each variable inside its
    switch (the distance switch the other way round)."""
    s = MAKERS[model]()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.x_slider = 0.1
    res = oracle_mod.OracleSystem(s).compute()
    val = {0: res["g"], 1: res["kappa"], 2: res["d"]}

    def th(v, frac):
        span = 2.0 * abs(val[v]) + 1.0
        lo, hi = val[v] - frac * span, val[v] + (1.0 - frac) * span
        return (hi, lo) if v == 2 else (lo, hi)

    s.bias_on, s.m_b, s.dv_max = 1, 2, 0.5
    s.bias_var1, s.bias_var2 = v1, v2
    s.g_lo, s.g_hi = th(v1, frac1)
    if v2 >= 0:
        s.b2_lo, s.b2_hi = th(v2, frac2)
    return s


@pytest.mark.parametrize("exec_mode", [0, 1])
@pytest.mark.parametrize("model", ["2d", "3d", "cone"])
@pytest.mark.parametrize("v1,v2", VAR_PAIRS)
def test_bias_variables_fp64(hd, oracle_mod, v1, v2, model, exec_mode):
    spec = biased(oracle_mod, model, v1, v2, 50 + v1 + 3 * v2)
    ref = oracle_mod.OracleSystem(spec).compute()
    assert 0.0 < ref["dv"] < spec.dv_max
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    sc = ctx.scalars(0)
    assert sc["dv"] == pytest.approx(ref["dv"], rel=1e-10)
    assert sc["dv1"] == pytest.approx(ref["dv1"], rel=1e-10, abs=1e-14)
    assert sc["dv2"] == pytest.approx(ref["dv2"], rel=1e-10, abs=1e-14)
    assert sc["dvp"] == pytest.approx(ref["dvp"], rel=1e-9)
    assert sc["g"] == pytest.approx(ref["g"], rel=1e-10)
    if 1 in (v1, v2):
        assert sc["kappa"] == pytest.approx(ref["kappa"], rel=1e-10)
        assert rel(ctx.forces(0, hd.HD_TUU), ref["tuu"]) < 1e-10
    assert rel(ctx.forces(0, hd.HD_FORCE_BIAS), ref["f_b"]) < 1e-9
    assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) < 1e-11


@pytest.mark.parametrize("model", ["2d", "3d", "cone"])
@pytest.mark.parametrize("v1,v2", [(1, -1), (0, 1), (0, 2), (1, 2)])
def test_bias_variables_fp32c(hd, oracle_mod, v1, v2, model):
    spec = biased(oracle_mod, model, v1, v2, 70 + v1 + 3 * v2)
    ref = oracle_mod.OracleSystem(spec).compute()
    ctx = hd.make_context([spec], precision=hd.HD_FP32C, init_velocities=False)
    sc = ctx.scalars(0)
    assert abs(sc["dv"] - ref["dv"]) <= 1e-6 * spec.dv_max
    assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) <= 1e-5
    assert rel(ctx.forces(0, hd.HD_FORCE_BIAS), ref["f_b"]) <= 1e-4
    if 1 in (v1, v2):
        assert sc["kappa"] == pytest.approx(ref["kappa"], rel=1e-5)


@pytest.mark.parametrize("v1,v2", [(0, 1), (2, -1)])
def test_biased_trajectory_fp64(hd, oracle_mod, v1, v2):
    spec = biased(oracle_mod, "3d", v1, v2, 90)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, init_velocities=True)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    ctx.step(20)
    o.step(20)
    d = ctx.positions(0) - o.positions()
    for k in range(2):
        d[k] -= spec.box[k] * np.round(d[k] / spec.box[k])
    assert float(np.abs(d).max()) < 1e-9
    a, b = ctx.scalars(0), o.scalars()
    assert a["t_hyper"] == pytest.approx(b["t_hyper"], rel=1e-11)
    assert a["dv"] == pytest.approx(b["dv"], rel=1e-8, abs=1e-12)


def test_mixed_batch(hd, oracle_mod):
    """Slope-only systems stay on the LDS-resident kernel, the others take
    the grid; every one matches the oracle."""
    specs = [biased(oracle_mod, "2d", 0, -1, 100), biased(oracle_mod, "2d", 1, 2, 101),
             biased(oracle_mod, "3d", 0, -1, 102), biased(oracle_mod, "cone", 2, 0, 103)]
    ctx = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=False)
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        assert rel(ctx.forces(k, hd.HD_FORCE_BIAS), ref["f_b"]) < 1e-9, k
        assert ctx.scalars(k)["dv"] == pytest.approx(ref["dv"], rel=1e-10), k


def test_at_the_reference(hd, oracle_mod):
    """x = r_O: d = 0, no bias force, curvature reported as 0."""
    s = build_3d(7, 7, 3, 2.0)
    s.bias_on, s.dv_max, s.bias_var1, s.bias_var2 = 1, 0.5, 1, 2
    s.g_lo, s.g_hi, s.b2_lo, s.b2_hi = -1.0, 1.0, 2.0, 1.0
    ctx = hd.make_context([s], precision=hd.HD_FP64, init_velocities=False)
    sc = ctx.scalars(0)
    assert sc["d"] == 0.0 and sc["kappa"] == 0.0
    assert np.all(ctx.forces(0, hd.HD_FORCE_BIAS) == 0.0)
    ref = oracle_mod.OracleSystem(s).compute()
    assert sc["dv"] == ref["dv"]


def test_bias_variable_arguments(hd):
    ctx = hd.Context(hd.HD_FP64)
    k = ctx.add_system(build_2d())
    # 4 is no variable; the curvature and the eigenvalue (3) are not combined
    for bad in ((4, -1), (-1, -1), (0, 0), (1, 3), (3, 1), (0, 4)):
        with pytest.raises(hd.HDError):
            ctx.set_bias_variables(k, *bad)
    ctx.set_bias_variables(k, 0, 2, 1.0, 2.0)            # bias off: not checked ...
    with pytest.raises(hd.HDError):
        ctx.set_bias(k, True, 2, 0.5, 0.0, 1.0)          # ... until it is enabled
    ctx.set_bias_variables(k, 0, 2, 2.0, 1.0)
    ctx.set_bias(k, True, 2, 0.5, 0.0, 1.0)
    with pytest.raises(hd.HDError):
        ctx.set_bias_variables(k, 0, 2, 1.0, 2.0)        # distance needs lo2 > hi2
    ctx.set_bias(k, False, 2, 0.5, 0.0, 1.0)
    ctx.set_bias_variables(k, 2)
    with pytest.raises(hd.HDError):
        ctx.set_bias(k, True, 2, 0.5, 0.0, 1.0)          # distance needs g_lo > g_hi
    ctx.set_bias(k, True, 2, 0.5, 1.0, 0.0)
    with pytest.raises(hd.HDError):
        ctx.set_bias_variables(k, 0)                     # those thresholds do not suit the slope
    ctx.set_bias(k, True, 2, 0.0, 1.0, 0.0)
    with pytest.raises(hd.HDError):
        ctx.set_bias_variables(k, 2, 0, 0.0, 1.0)        # two variables with dv_max = 0
    ctx.finalize()
    with pytest.raises(hd.HDError):
        ctx.set_bias_variables(k, 1)                     # after finalize


def test_bias_off_with_two_variables(hd, oracle_mod):
    """Bias disabled, two variables chosen, dv_max left at 0: no bias, the
    boosted clock equals the MD clock, the run follows the oracle's."""
    s = build_3d(7, 7, 3, 2.0)
    s.pos = perturbed(s, 0.05, 120)
    s.rO = build_3d(7, 7, 3, 2.0).pos
    s.bias_on, s.dv_max, s.bias_var1, s.bias_var2 = 0, 0.0, 1, 2
    s.b2_lo, s.b2_hi = 2.0, 1.0
    ctx = hd.make_context([s], precision=hd.HD_FP64, init_velocities=True)
    o = oracle_mod.OracleSystem(s)
    o.init_velocities()
    ctx.step(10)
    o.step(10)
    sc = ctx.scalars(0)
    assert sc["dv"] == 0.0 and sc["t_hyper"] == sc["t_md"]
    assert np.all(ctx.forces(0, hd.HD_FORCE_BIAS) == 0.0)
    d = ctx.positions(0) - o.positions()
    for k in range(2):
        d[k] -= s.box[k] * np.round(d[k] / s.box[k])
    assert float(np.abs(d).max()) < 1e-10
