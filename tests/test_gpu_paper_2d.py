"""The paper's 2D model (§3.1.1: 80 + 33 atoms, k = 5) on the GPU against the
oracle: forces, H u, energy and the slope bias at a jittered snapshot, and a
short biased trajectory, through the LDS-resident kernel and the grid
kernels in both precisions; the P2 batch of stepped slider positions."""
import numpy as np
import pytest

from hd_inputs import CONFIGS, build_2d_paper, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def snapshot(oracle_mod, seed, x_slider=0.3, narrow=True):
    """Jittered snapshot (u = the jitter) with slope thresholds around its g
    (about 60 here): a window 3 wide (narrow), or one of width 2|g| + 1 with
    g at 40 % of it, as in the other parity tests."""
    s = build_2d_paper()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.x_slider, s.kT = x_slider, 0.01
    g = oracle_mod.OracleSystem(s).compute()["g"]
    s.bias_on, s.m_b, s.dv_max = 1, 2, 0.05
    if narrow:
        s.g_lo, s.g_hi = g - 1.0, g + 2.0
    else:
        span = 2.0 * abs(g) + 1.0
        s.g_lo, s.g_hi = g - 0.4 * span, g + 0.6 * span
    return s


# In the narrow window dDV/dg is 2.5 % of DV_max per unit of g, so the stated
# 1e-6 DV_max asks for g to 3e-8 relative: within reach of float64 only.
# Float32 pair forces give g to about 1e-7 relative (checked directly), and
# meet the DV tolerance in the window that scales with g.
@pytest.mark.parametrize("seed", [7, 8, 9, 10, 11])
@pytest.mark.parametrize("exec_mode", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_paper_2d_evaluation(hd, oracle_mod, precision, exec_mode, seed):
    spec = snapshot(oracle_mod, seed, narrow=(precision == 0))
    ref = oracle_mod.OracleSystem(spec).compute()
    ctx = hd.make_context([spec], precision=precision, exec_mode=exec_mode, init_velocities=False)
    tol = 1e-11 if precision == 0 else 1e-5
    assert rel(ctx.forces(0, hd.HD_FORCE_LJ), ref["f_lj"]) <= tol
    assert rel(ctx.forces(0, hd.HD_HU), ref["hu"]) <= tol
    assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) <= tol
    sc = ctx.scalars(0)
    assert 0.0 < ref["dv"] < spec.dv_max
    assert abs(sc["dv"] - ref["dv"]) <= (1e-11 if precision == 0 else 1e-6) * spec.dv_max
    assert abs(sc["g"] - ref["g"]) <= (1e-12 if precision == 0 else 2e-7) * abs(ref["g"])
    assert sc["f_lat"] == pytest.approx(ref["f_lat"], rel=1e-12)


@pytest.mark.parametrize("exec_mode", [0, 1])
def test_paper_2d_trajectory_fp64(hd, oracle_mod, exec_mode):
    spec = snapshot(oracle_mod, 8)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=True)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    ctx.step(40)
    o.step(40)
    d = ctx.positions(0) - o.positions()
    d[0] -= spec.box[0] * np.round(d[0] / spec.box[0])
    assert float(np.abs(d).max()) < 1e-10
    assert ctx.scalars(0)["t_hyper"] == pytest.approx(o.scalars()["t_hyper"], rel=1e-12)


def test_p2_batch_sampled(hd, oracle_mod):
    """The P2 workload (256 positions, dx_S = 0.01) in one float32 batch:
    sampled systems against the oracle at a jittered snapshot."""
    specs = CONFIGS["P2"]()
    for k, s in enumerate(specs):
        s.rO = s.pos.copy()
        s.pos = perturbed(s, 0.05, 500 + k)
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=False)
    assert ctx.schedule()["lds_resident"] == 1
    for k in (0, 77, 255):
        ref = oracle_mod.OracleSystem(specs[k]).compute()
        assert rel(ctx.forces(k, hd.HD_FORCE_LJ), ref["f_lj"]) <= 1e-5, k
        assert ctx.scalars(k)["x_slider"] == pytest.approx(0.01 * k, abs=1e-15)
