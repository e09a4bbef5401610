"""The autotuner and launch-shape switching (hd_autotune, hd_set_schedule).

* hd_autotune times every candidate shape, keeps the fastest, and leaves
  every system's state (positions, velocities, step, clocks) bit for bit
  where it was;
* a run tuned at step k continues bit for bit like a run that switched to the
  same shape at step k with hd_set_schedule (a shape switch rebuilds lists
  from the recorded build positions, as a checkpoint restore does);
* every shape follows the oracle on an evaluation.
"""
import numpy as np
import pytest

from tests.test_gpu_parity import biased, rel, snapshot_2d, snapshot_3d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def mixed_specs(oracle_mod):
    small = [biased(oracle_mod, snapshot_2d(seed=80 + k, x_slider=0.3 * k)) for k in range(2)]
    large = [biased(oracle_mod, snapshot_3d(seed=82, nx=10, nz=4, R=4.0))]
    return small + large


def state(ctx, k):
    sc = ctx.scalars(k)
    return ctx.positions(k), ctx.velocities(k), sc["step"], sc["t_md"], sc["t_hyper"]


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_keeps_state_and_picks_fastest(hd, oracle_mod, precision):
    specs = mixed_specs(oracle_mod)
    ctx = hd.make_context(specs, precision=precision)
    ctx.step(30)
    before = [state(ctx, k) for k in range(len(specs))]
    chosen, trials = ctx.autotune(min_ms=2.0, max_steps=256)
    # LDS on (block 512 or 1024; float32 also with or without half lists)
    # x 7 shapes for the large system (grid tiles of 64 to 512 atoms, the
    # one-workgroup kernel at 256 to 1024 threads), then LDS off x 7
    assert len(trials) == (21 if precision == 0 else 35)
    assert all(t["ms_per_step"] > 0 for t in trials)
    best = min(trials, key=lambda t: t["ms_per_step"])
    assert chosen["ms_per_step"] == best["ms_per_step"]
    for key in ("lds_resident", "persistent_large", "large_block", "small_half_lists"):
        assert chosen[key] == best[key]
    for k in range(len(specs)):
        after = state(ctx, k)
        np.testing.assert_array_equal(after[0], before[k][0])
        np.testing.assert_array_equal(after[1], before[k][1])
        assert after[2:] == before[k][2:]


def test_tuned_run_equals_switched_run(hd, oracle_mod):
    specs = mixed_specs(oracle_mod)
    a = hd.make_context(specs, precision=hd.HD_FP64)
    a.step(30)
    chosen, _ = a.autotune(min_ms=2.0, max_steps=256)
    a.step(40)
    b = hd.make_context(specs, precision=hd.HD_FP64)
    b.step(30)
    b.set_schedule(chosen)
    assert b.schedule()["lds_resident"] == chosen["lds_resident"]
    b.step(40)
    for k in range(len(specs)):
        np.testing.assert_array_equal(a.positions(k), b.positions(k))
        np.testing.assert_array_equal(a.velocities(k), b.velocities(k))
        assert a.scalars(k)["t_hyper"] == b.scalars(k)["t_hyper"]


@pytest.mark.parametrize("shape", [
    {"lds_resident": 1, "small_block": 1024, "persistent_large": 0, "large_block": 128, "small_half_lists": 1},
    {"lds_resident": 1, "small_block": 512, "persistent_large": 1, "large_block": 1024, "small_half_lists": 0},
    {"lds_resident": 1, "small_block": 512, "persistent_large": 0, "large_block": 256, "small_half_lists": 1},
    {"lds_resident": 0, "small_block": 0, "persistent_large": 0, "large_block": 512},
    {"lds_resident": 0, "small_block": 0, "persistent_large": 1, "large_block": 256},
])
def test_every_shape_follows_the_oracle(hd, oracle_mod, shape):
    specs = mixed_specs(oracle_mod)
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=False)
    ctx.set_schedule(dict(shape, ms_per_step=0.0))
    ctx.compute()
    got = ctx.schedule()
    assert got["lds_resident"] == shape["lds_resident"] and got["large_block"] == shape["large_block"]
    assert got["small_half_lists"] == shape.get("small_half_lists", 0)
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        assert rel(ctx.forces(k), ref["f_tot"]) <= 1e-5, k
        assert abs(ctx.scalars(k)["dv"] - ref["dv"]) <= 1e-6 * s.dv_max, k
    ctx.step(20)
    assert all(ctx.scalars(k)["flags"] == 0 for k in range(len(specs)))


def test_schedule_argument_errors(hd, oracle_mod):
    specs = mixed_specs(oracle_mod)[:1]
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=False)
    with pytest.raises(hd.HDError):
        ctx.set_schedule({"lds_resident": 1, "small_block": 384, "persistent_large": 0, "large_block": 256})
    with pytest.raises(hd.HDError):
        ctx.set_schedule({"lds_resident": 1, "small_block": 512, "persistent_large": 0, "large_block": 100})
    with pytest.raises(hd.HDError):
        ctx.autotune(min_ms=0.0)
    seq = hd.make_context(specs, precision=hd.HD_FP64, exec_mode=hd.HD_EXEC_SEQUENTIAL, init_velocities=False)
    with pytest.raises(hd.HDError):
        seq.autotune()


SHAPES = {
    "lds+grid": {"lds_resident": 1, "small_block": 512, "persistent_large": 0, "large_block": 256,
                 "small_half_lists": 1},
    "lds-full": {"lds_resident": 1, "small_block": 512, "persistent_large": 0, "large_block": 256,
                 "small_half_lists": 0},
    "grid": {"lds_resident": 0, "small_block": 0, "persistent_large": 0, "large_block": 128},
    "persistent": {"lds_resident": 0, "small_block": 0, "persistent_large": 1, "large_block": 512},
}


@pytest.mark.parametrize("first,second,precision", [
    ("persistent", "grid", 0),       # one-workgroup rebuild, then the grid's counting sort
    ("lds+grid", "persistent", 1),   # half lists in LDS, then full lists in global memory
    ("grid", "lds+grid", 1),
    ("lds+grid", "lds-full", 1),     # half lists, then full lists, both in LDS
])
def test_switch_equals_restore_into_fresh_context(hd, oracle_mod, first, second, precision):
    """Switching shape mid-run gives the same trajectory as checkpointing and
    restoring into a fresh context that uses the second shape."""
    specs = mixed_specs(oracle_mod)
    a = hd.make_context(specs, precision=precision)
    a.set_schedule(SHAPES[first])
    a.step(25)
    blobs = [a.get_state(k) for k in range(len(specs))]
    a.set_schedule(SHAPES[second])
    a.step(25)
    b = hd.make_context(specs, precision=precision, init_velocities=False)
    b.set_schedule(SHAPES[second])
    for k, blob in enumerate(blobs):
        b.set_state(k, blob)
    b.step(25)
    for k in range(len(specs)):
        np.testing.assert_array_equal(a.positions(k), b.positions(k))
        np.testing.assert_array_equal(a.velocities(k), b.velocities(k))
        assert a.scalars(k)["t_hyper"] == b.scalars(k)["t_hyper"]
