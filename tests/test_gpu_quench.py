"""FIRE quench on the GPU (hd_quench): basin minima r_O and the quench-and-
compare transition check of the parallel slider-position algorithm (§2.3).

* the GPU minimum is a minimum by the oracle's own forces (every degree of
  freedom below the tolerance, up to the float64 summation order), and it is
  the oracle FIRE's minimum from the same start;
* the run state is untouched: a run quenched at step k continues bit for bit
  like one that was not;
* a configuration in r_O's basin reports a small displacement, one whose r_O
  is a lattice spacing away reports the spacing (a transition);
* with set_reference the minimum becomes r_O.
"""
import numpy as np
import pytest

from hd_inputs import ROLE_MOBILE, ROLE_RIGID, build_2d, build_3d, perturbed

pytestmark = pytest.mark.gpu

FTOL = 1e-9


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def jittered(spec, seed):
    s = spec.copy()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    return s


def small_3d():
    return build_3d(7, 7, 3, 2.0)     # 614 atoms


def dof_fmax(spec, res):
    """Largest force on a degree of freedom: mobile atoms, the rigid body."""
    f = res["f_lj"]
    mob = spec.role == ROLE_MOBILE
    fm = float(np.sqrt((f[:, mob] ** 2).sum(0)).max()) if mob.any() else 0.0
    rig = spec.role == ROLE_RIGID
    if rig.any():
        fm = max(fm, float(np.linalg.norm(res["f_tot"][:, rig].sum(1))))
    return fm


def min_image(spec, d):
    d = d.copy()
    for k in range(spec.dim):
        if spec.periodic[k]:
            d[k] -= spec.box[k] * np.round(d[k] / spec.box[k])
    return d


@pytest.mark.parametrize("path", ["lds", "grid"])
@pytest.mark.parametrize("maker", [lambda: build_2d(), small_3d], ids=["2d", "3d"])
def test_quench_reaches_the_oracle_minimum(hd, oracle_mod, path, maker):
    spec = jittered(maker(), 11)
    spec.x_slider = 0.2
    exec_mode = hd.HD_EXEC_BATCHED if path == "lds" else hd.HD_EXEC_GRID
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    iters, disp, (xm,) = ctx.quench([0], ftol=FTOL, max_iters=200000)
    assert iters[0] > 0
    # a minimum by the oracle's forces (the rigid body moved from its
    # starting position, which fixes the drive's zero)
    o = oracle_mod.OracleSystem(spec)
    o.set_positions(xm)
    res = o.compute()
    assert dof_fmax(spec, res) < 10 * FTOL
    # the oracle's FIRE from the same start lands on the same minimum
    ref = oracle_mod.OracleSystem(spec)
    assert ref.fire(ftol=FTOL, maxit=200000) >= 0
    d = min_image(spec, xm - ref.positions())
    assert float(np.abs(d).max()) < 1e-6
    assert res["e_pot"] == pytest.approx(ref.compute()["e_pot"], rel=1e-12, abs=1e-12)
    # the displacement reported is the minimum's distance from r_O
    want = float(np.sqrt((min_image(spec, xm - spec.rO) ** 2).sum(0)).max())
    assert disp[0] == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("precision,exec_mode", [(0, 0), (1, 0), (1, 1)])
def test_quench_leaves_the_run_untouched(hd, oracle_mod, precision, exec_mode):
    specs = [jittered(build_2d(), 20 + k) for k in range(2)] + [jittered(small_3d(), 22)]
    for s in specs:
        s.bias_on, s.m_b, s.dv_max = 1, 2, 0.5
        g = oracle_mod.OracleSystem(s).compute()["g"]
        s.g_lo, s.g_hi = g - 2.0, g + 3.0
    runs = []
    for quench in (False, True):
        ctx = hd.make_context(specs, precision=precision, exec_mode=exec_mode)
        ctx.step(40)
        if quench:
            # float32 pair forces carry rounding of ~1e-6 of their terms: a
            # coarser tolerance there
            it, _, _ = ctx.quench([2, 0], ftol=1e-6 if precision == 0 else 1e-3, max_iters=50000)
            assert all(v > 0 for v in it)
        ctx.step(40)
        runs.append([(ctx.positions(k), ctx.velocities(k), ctx.scalars(k)) for k in range(len(specs))])
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        for key in ("step", "t_md", "t_hyper", "dv", "e_pot", "n_rebuilds"):
            assert a[2][key] == b[2][key], key


def test_transition_check_and_new_reference(hd, oracle_mod):
    base = build_2d()
    same = jittered(base, 31)
    # a reference one lattice spacing away along the sliding direction: the
    # tip atoms' basin as if the tip had slipped by one spacing
    moved = jittered(base, 32)
    a = float(2.0 ** (1.0 / 6.0))
    tip = moved.type == 1
    moved.rO = moved.rO.copy()
    moved.rO[0, tip] = (moved.rO[0, tip] + a) % moved.box[0]
    ctx = hd.make_context([same, moved], precision=hd.HD_FP64, init_velocities=False)
    iters, disp, _ = ctx.quench([0, 1], ftol=1e-8)
    assert min(iters) > 0
    assert disp[0] < 0.35         # same basin (relaxation under the normal load only)
    assert disp[1] > 0.8 * a      # a transition of one spacing
    # the minimum becomes r_O: checked again, it is at distance ~0
    it2, d2, (xm,) = ctx.quench([1], ftol=1e-8, set_reference=True)
    assert it2[0] > 0 and d2[0] > 0.0
    it3, d3, _ = ctx.quench([1], ftol=1e-8)
    assert d3[0] < 1e-6
    # and with r_O at a minimum and x there, d = 0: no bias force
    assert np.isfinite(ctx.scalars(1)["e_pot"])


def test_quench_argument_errors(hd):
    ctx = hd.make_context([build_2d()], precision=hd.HD_FP64, init_velocities=False)
    for bad in ([1], [0, 0], [-1]):
        with pytest.raises(hd.HDError):
            ctx.quench(bad)
    with pytest.raises(hd.HDError):
        ctx.quench([0], ftol=0.0)
    with pytest.raises(hd.HDError):
        ctx.quench([0], max_iters=0)


def test_lds_and_grid_fire_reach_the_same_minima_in_one_call(hd, oracle_mod):
    """LDS-resident systems take the whole quench in one launch of the LDS
    kernel's FIRE mode, grid systems iterate FIRE kernels and evaluations:
    in one call over a mixed batch (listed out of order) every system's
    results sit at its own listed index, and every minimum is the oracle
    FIRE's.  Quenched again from its minimum, a system converges at once."""
    big = jittered(build_3d(10, 10, 4, 4.0), 41)     # 1743 atoms: grid kernels
    small = jittered(build_2d(), 42)                 # 480 atoms: LDS-resident
    small3 = jittered(small_3d(), 43)                # 614 atoms: LDS-resident
    specs = [small, big, small3]
    for s in specs:
        s.x_slider = 0.2
    ctx = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=False)
    order = [2, 1, 0]
    iters, disp, xms = ctx.quench(order, ftol=1e-8, max_iters=200000)
    for k, sidx in enumerate(order):
        spec = specs[sidx]
        assert iters[k] > 0
        ref = oracle_mod.OracleSystem(spec)
        assert ref.fire(ftol=1e-8, maxit=200000) >= 0
        assert float(np.abs(min_image(spec, xms[k] - ref.positions())).max()) < 1e-5
        want = float(np.sqrt((min_image(spec, xms[k] - spec.rO) ** 2).sum(0)).max())
        assert disp[k] == pytest.approx(want, rel=1e-12)
    # from the minimum: converged at the first test, on both paths
    for sidx in (0, 1):
        ctx.set_positions(sidx, xms[order.index(sidx)])
    it2, _, _ = ctx.quench([1, 0], ftol=1e-8, max_iters=1000)
    assert list(it2) == [0, 0]
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_lds_fire_matches_the_grid_fire(hd, precision):
    """The same systems quenched on the LDS kernel and on the grid kernels
    land on the same minimum: float64 to 1e-8 within 1e-6; float32 pair
    forces converge only to a coarser tolerance (1e-3), which leaves soft
    modes undetermined to about ftol / (their curvature): the same basin,
    within a tenth of a lattice spacing."""
    specs = [jittered(build_2d(), 50), jittered(small_3d(), 51)]
    ftol = 1e-8 if precision == 0 else 1e-3
    out = []
    for mode in (hd.HD_EXEC_BATCHED, hd.HD_EXEC_GRID):
        ctx = hd.make_context(specs, precision=precision, exec_mode=mode, init_velocities=False)
        iters, disp, xms = ctx.quench([0, 1], ftol=ftol, max_iters=200000)
        assert all(v > 0 for v in iters)
        out.append(xms)
        ctx.close()
    tol = 1e-6 if precision == 0 else 0.1
    for s, a, b in zip(specs, *out):
        assert float(np.abs(min_image(s, a - b)).max()) < tol


def test_scalars_batch_matches_single_reads(hd):
    specs = [jittered(build_2d(), 60 + k) for k in range(3)]
    ctx = hd.make_context(specs, precision=hd.HD_FP32C)
    ctx.step(25)
    got = ctx.scalars_batch()
    assert got == [ctx.scalars(k) for k in range(3)]
    assert ctx.scalars_batch(1, 2) == got[1:]
    assert ctx.scalars_batch(3, 0) == []
    for first, count in ((-1, 1), (2, 2), (0, 4)):
        with pytest.raises(hd.HDError):
            ctx.scalars_batch(first, count)
    ctx.close()
