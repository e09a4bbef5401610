"""Harmonic tip bonds (eq. 12) on the GPU: the paper's conical-tip 3D model
against the oracle -- forces, H u, energy and a short trajectory -- through
both schedulers and in both precisions.  Models with tip bonds run on the
grid kernels (never LDS-resident)."""
import numpy as np
import pytest

from hd_inputs import build_3d, build_3d_cone, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def snapshot(maker, seed):
    s = maker()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.x_slider = 0.3
    return s


def jittered_plain(seed):
    s = build_3d(7, 7, 3, 2.0)
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    return s


MAKERS = {"paper": build_3d_cone, "small": lambda: build_3d_cone(nx=9, ny=9, nz=1, layers=4)}


@pytest.mark.parametrize("exec_mode", [0, 1])
@pytest.mark.parametrize("model", ["paper", "small"])
def test_tip_bonds_evaluation_fp64(hd, oracle_mod, exec_mode, model):
    spec = snapshot(MAKERS[model], 31)
    ref = oracle_mod.OracleSystem(spec).compute()
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    assert rel(ctx.forces(0, hd.HD_FORCE_LJ), ref["f_lj"]) < 1e-11
    assert rel(ctx.forces(0, hd.HD_HU), ref["hu"]) < 1e-11
    assert ctx.scalars(0)["e_pot"] == pytest.approx(ref["e_pot"], rel=1e-11)


def test_bonded_and_plain_systems_in_one_batch(hd, oracle_mod):
    """A batch mixing bonded cone models with plain LJ systems small enough
    for the LDS-resident kernel: the bonded ones go to the grid kernels, the
    others stay where they were, and every system matches the oracle."""
    specs = [snapshot(MAKERS["small"], 40), jittered_plain(41), snapshot(MAKERS["paper"], 42), jittered_plain(43)]
    ctx = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=False)
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        assert rel(ctx.forces(k, hd.HD_FORCE_LJ), ref["f_lj"]) < 1e-11, k
        assert rel(ctx.forces(k, hd.HD_HU), ref["hu"]) < 1e-11, k


@pytest.mark.parametrize("exec_mode", [0, 1])
def test_tip_bonds_evaluation_fp32c(hd, oracle_mod, exec_mode):
    spec = snapshot(build_3d_cone, 32)
    ref = oracle_mod.OracleSystem(spec).compute()
    ctx = hd.make_context([spec], precision=hd.HD_FP32C, exec_mode=exec_mode, init_velocities=False)
    assert rel(ctx.forces(0, hd.HD_FORCE_LJ), ref["f_lj"]) <= 1e-5
    assert rel(ctx.forces(0, hd.HD_HU), ref["hu"]) <= 1e-5


@pytest.mark.parametrize("large_block", [64, 320, 1024])
@pytest.mark.parametrize("precision", [0, 1])
def test_tip_bonds_every_lane_count(hd, oracle_mod, precision, large_block):
    """The bonded pair loop gathers list entries and records four at a time,
    so every lane's list ends in a ragged block: four, two and one lanes per
    atom (64-, 320- and 1024-atom tiles, the 320-atom ones ragged against the
    system) against the oracle."""
    specs = [snapshot(MAKERS["paper"], 34), snapshot(MAKERS["small"], 35)]
    ctx = hd.make_context(specs, precision=precision, init_velocities=False)
    ctx.set_schedule({"lds_resident": 0, "small_block": 0, "persistent_large": 0,
                      "large_block": large_block, "ms_per_step": 0.0})
    ctx.compute()
    assert ctx.schedule()["large_block"] == large_block
    tol = 1e-11 if precision == hd.HD_FP64 else 1e-5
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        assert rel(ctx.forces(k, hd.HD_FORCE_LJ), ref["f_lj"]) <= tol, k
        assert rel(ctx.forces(k, hd.HD_HU), ref["hu"]) <= tol, k
        assert ctx.scalars(k)["e_pot"] == pytest.approx(ref["e_pot"], rel=1e-11 if precision == hd.HD_FP64 else 1e-6)


def test_tip_bonds_trajectory_fp64(hd, oracle_mod):
    spec = snapshot(build_3d_cone, 33)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, init_velocities=True)
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    ctx.step(20)
    o.step(20)
    d = ctx.positions(0) - o.positions()
    for k in range(2):
        d[k] -= spec.box[k] * np.round(d[k] / spec.box[k])
    assert float(np.abs(d).max()) < 1e-9
    # a bonded tip keeps its bonds: every tip nearest-neighbour distance
    # stays near the rest length
    tip = np.flatnonzero(spec.type == 1)
    x = ctx.positions(0)[:, tip]
    dd = x[:, :, None] - x[:, None, :]
    for k in range(2):
        dd[k] -= spec.box[k] * np.round(dd[k] / spec.box[k])
    r = np.sqrt((dd ** 2).sum(0))
    near = r[(r > 0) & (r < 1.36)]
    assert near.size > 0 and np.abs(near - spec.r_bond).max() < 0.2


def test_tip_bonds_arguments(hd):
    s = build_3d_cone(nx=9, ny=9, nz=1, layers=4)
    ctx = hd.Context(hd.HD_FP64)
    k = ctx.add_system(s)
    with pytest.raises(hd.HDError):
        ctx.set_tip_bonds(k, True, 57.0, 1.12, 3.0)     # cut beyond rc
    ctx.finalize()
    with pytest.raises(hd.HDError):
        ctx.set_tip_bonds(k, False, 0.0, 1.0, 1.0)      # after finalize
