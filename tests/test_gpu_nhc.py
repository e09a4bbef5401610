"""The Nose-Hoover chain thermostat (§3.1.1) on the GPU against the oracle:
trajectories, the chain's energy and the boosted clock in both precisions;
the extended energy's O(dt^2) error; a batch mixing it with Langevin
systems; checkpoint and restore; argument errors."""
import numpy as np
import pytest

from hd_inputs import build_2d, build_3d, build_3d_cone, build_2d_paper, perturbed

pytestmark = pytest.mark.gpu

MAKERS = {
    "2d": lambda: build_2d(),
    "3d": lambda: build_3d(7, 7, 3, 2.0),
    "cone": lambda: build_3d_cone(nx=9, ny=9, nz=1, layers=4),
    "paper2d": build_2d_paper,
}


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def nhc_spec(oracle_mod, model, seed, M=3, bias=True):
    s = MAKERS[model]()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.x_slider, s.kT = 0.1, 0.1
    s.thermostat, s.nhc_len, s.nhc_tau = 1, M, 0.5
    if bias:
        g = oracle_mod.OracleSystem(s).compute()["g"]
        s.bias_on, s.m_b, s.dv_max = 1, 2, 0.5
        s.g_lo, s.g_hi = g - 2.0, g + 3.0
    return s


def min_image_diff(spec, a, b):
    d = a - b
    for k in range(spec.dim):
        if spec.periodic[k]:
            d[k] -= spec.box[k] * np.round(d[k] / spec.box[k])
    return d


@pytest.mark.parametrize("exec_mode", [0, 1], ids=["lds", "grid"])
@pytest.mark.parametrize("M", [1, 3])
@pytest.mark.parametrize("model", ["2d", "3d", "cone", "paper2d"])
def test_nhc_trajectory_fp64(hd, oracle_mod, model, M, exec_mode):
    """Batched: the 2D and 3D models run LDS-resident (the cone model, with
    tip bonds, on the grid); grid: every model on the grid kernels."""
    spec = nhc_spec(oracle_mod, model, 11, M)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=True)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    ctx.step(40)
    o.step(40)
    assert float(np.abs(min_image_diff(spec, ctx.positions(0), o.positions())).max()) < 1e-10
    assert float(np.abs(ctx.velocities(0) - o.velocities()).max()) < 1e-9
    a, b = ctx.scalars(0), o.scalars()
    assert b["e_nhc"] != 0.0
    assert a["e_nhc"] == pytest.approx(b["e_nhc"], rel=1e-9, abs=1e-12)
    assert a["e_kin"] == pytest.approx(b["e_kin"], rel=1e-11)
    assert a["t_hyper"] == pytest.approx(b["t_hyper"], rel=1e-12)


@pytest.mark.parametrize("exec_mode", [0, 1], ids=["lds", "grid"])
@pytest.mark.parametrize("model", ["2d", "3d"])
def test_nhc_trajectory_fp32c(hd, oracle_mod, model, exec_mode):
    spec = nhc_spec(oracle_mod, model, 12)
    ctx = hd.make_context([spec], precision=hd.HD_FP32C, exec_mode=exec_mode, init_velocities=True)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    ctx.step(20)
    o.step(20)
    assert float(np.abs(min_image_diff(spec, ctx.positions(0), o.positions())).max()) < 1e-6
    assert ctx.scalars(0)["e_nhc"] == pytest.approx(o.scalars()["e_nhc"], rel=1e-4, abs=1e-8)


def test_nhc_extended_energy_second_order(hd, oracle_mod):
    """On the GPU alone: K + V + dV + the chain's energy drifts as dt^2."""
    def spread(dt, nsteps):
        s = nhc_spec(oracle_mod, "2d", 13)
        s.dt = dt
        ctx = hd.make_context([s], precision=hd.HD_FP64, init_velocities=True)
        tot = []
        for _ in range(nsteps // 10):
            ctx.step(10)
            sc = ctx.scalars(0)
            tot.append(sc["e_pot"] + sc["e_kin"] + sc["dv"] + sc["e_nhc"])
        return max(tot) - min(tot)

    e1, e2 = spread(0.004, 400), spread(0.002, 800)
    assert 3.0 < e1 / e2 < 5.0


def test_nhc_and_langevin_in_one_batch(hd, oracle_mod):
    specs = [nhc_spec(oracle_mod, "2d", 20), MAKERS["2d"](), nhc_spec(oracle_mod, "cone", 21), MAKERS["3d"]()]
    for k in (1, 3):
        specs[k].pos = perturbed(specs[k], 0.05, 30 + k)
    ctx = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=True)
    oracles = [oracle_mod.OracleSystem(s) for s in specs]
    for o in oracles:
        o.init_velocities()
        o.step(20)
    ctx.step(20)
    for k, (s, o) in enumerate(zip(specs, oracles)):
        assert float(np.abs(min_image_diff(s, ctx.positions(k), o.positions())).max()) < 1e-9, k


def test_nhc_checkpoint_restore(hd, oracle_mod):
    spec = nhc_spec(oracle_mod, "3d", 40)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, init_velocities=True)
    ctx.step(15)
    blob = ctx.get_state(0)
    ctx.step(25)
    ref_x, ref_s = ctx.positions(0), ctx.scalars(0)
    other = hd.make_context([spec], precision=hd.HD_FP64, init_velocities=False)
    other.set_state(0, blob)
    other.step(25)
    np.testing.assert_array_equal(other.positions(0), ref_x)
    assert other.scalars(0)["e_nhc"] == ref_s["e_nhc"]


def test_nhc_arguments(hd):
    ctx = hd.Context(hd.HD_FP64)
    k = ctx.add_system(build_2d())
    for bad in ((5, 0.5), (-1, 0.5), (3, 0.0)):
        with pytest.raises(hd.HDError):
            ctx.set_nose_hoover(k, *bad)
    s0 = build_2d()
    s0.kT = 0.0
    other = hd.Context(hd.HD_FP64)
    k0 = other.add_system(s0)
    with pytest.raises(hd.HDError):
        other.set_nose_hoover(k0, 3, 0.5)                # kT = 0
    ctx.set_nose_hoover(k, 3, 0.5)
    ctx.finalize()
    with pytest.raises(hd.HDError):
        ctx.set_nose_hoover(k, 0, 0.5)                   # after finalize


@pytest.mark.parametrize("exec_mode", [0, 1], ids=["lds", "grid"])
def test_nhc_across_launches(hd, oracle_mod, exec_mode):
    """A run split into several launches (each opening the chain itself)
    follows the oracle's uninterrupted run."""
    spec = nhc_spec(oracle_mod, "paper2d", 14)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=True)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    for n in (7, 13, 1, 19):
        ctx.step(n)
    o.step(40)
    assert float(np.abs(min_image_diff(spec, ctx.positions(0), o.positions())).max()) < 1e-10
    assert ctx.scalars(0)["e_nhc"] == pytest.approx(o.scalars()["e_nhc"], rel=1e-9)


def test_nhc_lds_batch_p2(hd, oracle_mod):
    """The P2 workload under the chain: 256 positions LDS-resident, sampled
    systems against the oracle after 30 steps."""
    from hd_inputs import CONFIGS
    specs = CONFIGS["P2"]()
    for k, s in enumerate(specs):
        s.rO = s.pos.copy()
        s.pos = perturbed(s, 0.05, 700 + k)
        s.thermostat, s.nhc_len, s.nhc_tau = 1, 3, 0.5
        s.bias_on = 0
    ctx = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=True)
    assert ctx.schedule()["lds_resident"] == 1
    ctx.step(30)
    for k in (0, 131, 255):
        o = oracle_mod.OracleSystem(specs[k])
        o.init_velocities()
        o.step(30)
        assert float(np.abs(min_image_diff(specs[k], ctx.positions(k), o.positions())).max()) < 1e-10, k
