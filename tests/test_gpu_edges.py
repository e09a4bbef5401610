"""Edge cases of the GPU path: tiny and degenerate systems, the size limit of
the LDS-resident kernel, neighbour-capacity overflow, d = 0, argument errors
and the per-system instability flag (a system whose energy becomes
non-finite is frozen while the others continue)."""
import numpy as np
import pytest

from hd_inputs import (ROLE_FIXED, ROLE_MOBILE, ROLE_RIGID, SystemSpec, build_2d, perturbed)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def custom(pos, role, typ=None, L=30.0):
    pos = np.array(pos, dtype=np.float64)
    n = pos.shape[1]
    return SystemSpec(dim=2, pos=np.array(pos, dtype=np.float64), role=np.array(role, np.uint8),
                      type=np.zeros(n, np.uint8) if typ is None else np.array(typ, np.uint8),
                      box=np.array([L, 0.0, 0.0]), periodic=np.array([1, 0, 0], np.int32))


@pytest.mark.parametrize("lds", [True, False])
def test_single_atom_and_tiny_systems(hd, oracle_mod, lds):
    one = custom([[1.0], [2.0]], [ROLE_MOBILE])
    two = custom([[1.0, 2.2], [2.0, 2.1]], [ROLE_MOBILE, ROLE_MOBILE])
    nodrive = custom([[1.0, 2.2, 3.3], [2.0, 2.1, 2.0]], [ROLE_MOBILE, ROLE_FIXED, ROLE_MOBILE])
    specs = [one, two, nodrive]
    ctx = hd.make_context(specs, precision=hd.HD_FP64, lds_resident=lds)
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        np.testing.assert_allclose(ctx.forces(k), ref["f_tot"], rtol=1e-12, atol=1e-12)
        assert ctx.scalars(k)["e_pot"] == pytest.approx(ref["e_pot"], abs=1e-12)
    ctx.step(30)
    for k in range(3):
        assert ctx.scalars(k)["step"] == 30
        assert np.all(np.isfinite(ctx.positions(k)))
    assert ctx.scalars(0)["e_pot"] == 0.0


def test_all_fixed_system_never_moves(hd):
    s = build_2d(nx=12, ny=4, tip_w=4, tip_h=3)
    s.role[:] = ROLE_FIXED
    ctx = hd.make_context([s], precision=hd.HD_FP32C)
    x0 = ctx.positions(0)
    ctx.step(25)
    np.testing.assert_array_equal(ctx.positions(0), x0)


def _exactly(nsub_x, nsub_y, tip_w, tip_h, extra=0):
    s = build_2d(nx=nsub_x, ny=nsub_y, tip_w=tip_w, tip_h=tip_h)
    if extra:
        xs = np.concatenate([s.pos, np.array([[s.box[0] / 3], [s.pos[1].max() + 6.0]])], axis=1)
        s = SystemSpec(dim=2, pos=xs, type=np.append(s.type, 0).astype(np.uint8),
                       role=np.append(s.role, ROLE_MOBILE).astype(np.uint8), box=s.box, periodic=s.periodic,
                       eps=s.eps)
    return s


@pytest.mark.parametrize("extra", [0, 1])
def test_lds_kernel_size_limit(hd, oracle_mod, extra):
    """1024 atoms is the largest LDS-resident system; 1025 goes to the global
    kernel.  Both agree with the oracle."""
    s = _exactly(64, 14, 16, 8, extra)
    assert s.n == 1024 + extra
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, 9)
    ref = oracle_mod.OracleSystem(s).compute()
    ctx = hd.make_context([s], precision=hd.HD_FP32C, init_velocities=False)
    assert rel(ctx.forces(0), ref["f_tot"]) <= 1e-5
    ctx.step(10)
    assert ctx.scalars(0)["flags"] == 0


@pytest.mark.parametrize("lds", [True, False])
def test_neighbour_overflow_is_flagged(hd, lds):
    s = build_2d()
    ctx = hd.make_context([s], precision=hd.HD_FP32C, max_neighbors=8, lds_resident=lds)
    assert ctx.scalars(0)["flags"] & hd.HD_FLAG_NBR_OVERFLOW
    ctx.step(5)
    assert ctx.scalars(0)["step"] == 5


def test_zero_distance_guard(hd, oracle_mod):
    """At x = r_O the distance d is 0: g is set to 0 and there is no bias force."""
    s = build_2d()
    s.bias_on, s.g_lo, s.g_hi, s.dv_max = 1, -1.0, 1.0, 0.3
    ctx = hd.make_context([s], precision=hd.HD_FP64, init_velocities=False)
    sc = ctx.scalars(0)
    ref = oracle_mod.OracleSystem(s).compute()
    assert sc["d"] == 0.0 and sc["g"] == 0.0
    assert sc["dv"] == pytest.approx(ref["dv"], abs=1e-15)
    assert np.all(ctx.forces(0, hd.HD_FORCE_BIAS) == 0.0)


def test_argument_errors(hd):
    s = build_2d()
    ctx = hd.Context(hd.HD_FP32C)
    with pytest.raises(hd.HDError):
        ctx.step(1)                                  # before finalize
    k = ctx.add_system(s)
    with pytest.raises(hd.HDError):
        ctx.set_bias(k, True, 2, 0.5, 1.0, 0.0)      # g_lo >= g_hi
    with pytest.raises(hd.HDError):
        ctx.set_bias(k, True, 0, 0.5, 0.0, 1.0)      # m_b < 1
    ctx.finalize()
    with pytest.raises(hd.HDError):
        ctx.scalars(5)                               # bad system index
    with pytest.raises(hd.HDError):
        ctx.add_system(s)                            # after finalize
    bad = build_2d(nx=4, ny=4, tip_w=2, tip_h=2)     # box shorter than 2 (rc + skin)
    c2 = hd.Context(hd.HD_FP32C)
    with pytest.raises(hd.HDError):
        c2.add_system(bad)


def test_unstable_system_is_frozen_others_continue(hd, oracle_mod):
    """Two atoms 0.05 apart are frozen by the set-up evaluation; two atoms
    0.6 apart blow up within the first launch (the oracle's force passes
    1e6 at its third step).  The healthy system runs on."""
    good = build_2d()
    early, late = build_2d(), build_2d()
    i, j = 150, 151                                  # two mobile substrate atoms
    for s, gap in ((early, 0.05), (late, 0.6)):
        s.pos[0, j] = s.pos[0, i] + gap
        s.pos[1, j] = s.pos[1, i]
    ctx = hd.make_context([good, early, late], precision=hd.HD_FP64)
    e0 = ctx.scalars(1)["e_pot"]
    assert e0 == pytest.approx(oracle_mod.OracleSystem(early).compute()["e_pot"], rel=1e-12)
    ctx.step(50)
    assert ctx.scalars(0)["flags"] == 0
    assert ctx.scalars(0)["step"] == 50
    for k in (1, 2):
        assert ctx.scalars(k)["flags"] & hd.HD_FLAG_UNSTABLE
    # frozen before its first step: the readout keeps the evaluation's
    # (finite, huge) energy
    assert ctx.scalars(1)["step"] == 0
    assert ctx.scalars(1)["e_pot"] == e0
    # frozen within a launch of the LDS-resident kernel, which evaluates the
    # pair energy on a launch's last step only: the frozen system reports a
    # pair energy of zero, so e_pot is the (finite, small) drive energy alone
    # rather than the blown-up pair energy
    sc = ctx.scalars(2)
    assert 0 < sc["step"] < 50
    assert np.isfinite(sc["e_pot"]) and abs(sc["e_pot"]) < 10.0


def test_crowded_stencil_rows_fall_back_to_one_lane_build(hd, oracle_mod):
    """A slab compressed twofold along z puts more neighbours in one stencil
    row than the row-parallel build holds; those atoms take the one-lane
    build, and the lists still equal the brute-force set."""
    from hd_inputs import build_3d
    s = build_3d(10, 10, 4, 4.0)
    z0 = s.pos[2].min()
    s.pos[2] = z0 + 0.5 * (s.pos[2] - z0)
    ctx = hd.make_context([s], precision=hd.HD_FP64, init_velocities=False, max_neighbors=512)
    got = set(map(tuple, ctx.debug_pairs(0).tolist()))
    ref = set(map(tuple, oracle_mod.pairs_brute(s, s.pos, s.rc + s.skin, exclude=True).tolist()))
    assert max(np.bincount(np.array(sorted(ref)).ravel())) > 48
    assert got == ref


@pytest.mark.parametrize("path", ["lds", "grid"])
@pytest.mark.parametrize("dim", [2, 3])
def test_narrow_periodic_box_takes_general_minimum_image(hd, oracle_mod, path, dim):
    """A periodic box narrower than three list radii has one cell on that
    axis: every pair shares it, with either image, and the list build takes
    the general minimum image there.  Forces and, after rebuilds, the lists
    match the oracle."""
    from hd_inputs import build_3d
    from tests.test_gpu_parity import _build_positions
    s = build_2d(nx=6, ny=6, tip_w=3, tip_h=3) if dim == 2 else build_3d(5, 5, 3, 1.0)
    assert s.box[0] < 3 * (s.rc + s.skin)
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, 70 + dim)
    exec_mode = hd.HD_EXEC_BATCHED if path == "lds" else hd.HD_EXEC_GRID
    ctx = hd.make_context([s], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    ref = oracle_mod.OracleSystem(s).compute()
    assert rel(ctx.forces(0), ref["f_tot"]) < 1e-11
    ctx.init_velocities(0)
    ctx.step(300)
    assert ctx.scalars(0)["flags"] == 0 and ctx.scalars(0)["n_rebuilds"] >= 1
    xb = _build_positions(ctx.get_state(0), s.dim, s.n)
    got = set(map(tuple, ctx.debug_pairs(0).tolist()))
    want = set(map(tuple, oracle_mod.pairs_brute(s, xb, s.rc + s.skin, exclude=True).tolist()))
    assert got == want
