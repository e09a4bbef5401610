"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances
* neighbour lists: bit-exact set equality with the oracle's brute force;
* float64 path: relative L2 error of forces / H u per system <= 1e-11 and
  scalars to 1e-11 (summation order differs: full lists on the GPU, half
  pairs in the oracle);
* float32 path: relative L2 force error <= 1e-5 and |dV - dV_ref| <= 1e-6 dV_max
  (the stated tolerances of the hot path);
* short trajectories (identical Philox streams): float64 positions within
  1e-10, float32 within a bound that follows from the force tolerance.
"""
import numpy as np
import pytest

from hd_inputs import (AFCC, A2D, ROLE_FIXED, ROLE_MOBILE, ROLE_RIGID, build_2d, build_3d,
                       config_c4, perturbed)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def biased(oracle_mod, spec, frac=0.4, dv_max=0.5):
    """Copy of spec whose slope thresholds bracket the snapshot's g."""
    g = oracle_mod.OracleSystem(spec).compute()["g"]
    s = spec.copy()
    span = 2.0 * abs(g) + 1.0
    s.bias_on, s.m_b, s.dv_max = 1, 2, dv_max
    s.g_lo, s.g_hi = g - frac * span, g + (1.0 - frac) * span
    return s


def snapshot_2d(seed=3, x_slider=0.25):
    """Perturbed 2D model; r_O is the lattice, so u = x - r_O is the jitter."""
    s = build_2d()
    s.x_slider = x_slider
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    return s


def snapshot_3d(seed=5, nx=20, nz=6, R=8.0, x_slider=0.4):
    s = build_3d(nx, nx, nz, R)
    s.x_slider = x_slider
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    return s


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("maker", [snapshot_2d, lambda: snapshot_3d(nx=10, nz=4, R=4.0)])
@pytest.mark.parametrize("exec_mode", [0, 2])
def test_neighbour_pairs_bit_exact(hd, oracle_mod, maker, exec_mode):
    spec = maker()
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    got = ctx.debug_pairs(0)
    ref = oracle_mod.pairs_brute(spec, spec.pos, spec.rc + spec.skin, exclude=True)
    sg = set(map(tuple, got.tolist()))
    sr = set(map(tuple, ref.tolist()))
    assert len(sg) == len(got)
    assert sg == sr


def _build_positions(blob, dim, n):
    """Recorded build positions from a checkpoint: header, then x, v, r_O,
    x_build, F and the eigenvalue variable's mode (each dim x n float64)."""
    nd = dim * n
    body = np.frombuffer(blob[len(blob) - 6 * nd * 8:], dtype=np.float64)
    return body[3 * nd:4 * nd].reshape(dim, n).copy()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("path", ["lds", "grid", "grid3d", "grid3d-wide"])
def test_lists_after_rebuilds_bit_exact(hd, oracle_mod, path, precision):
    """After many steps (several list rebuilds, the grid's in cell-sorted
    order), the current lists are exactly the oracle's pair set at the
    recorded build positions.  grid3d-wide is a wider slab (4400 cells,
    26063 atoms)."""
    if path == "grid3d":
        spec = snapshot_3d(seed=91, nx=10, nz=4, R=4.0)
    elif path == "grid3d-wide":
        spec = snapshot_3d(seed=92, nx=36, nz=5, R=4.0)
    else:
        spec = snapshot_2d(seed=90)
    exec_mode = hd.HD_EXEC_BATCHED if path == "lds" else hd.HD_EXEC_GRID
    ctx = hd.make_context([spec], precision=precision, exec_mode=exec_mode)
    ctx.step(300)
    assert ctx.scalars(0)["n_rebuilds"] >= 3
    xb = _build_positions(ctx.get_state(0), spec.dim, spec.n)
    got = set(map(tuple, ctx.debug_pairs(0).tolist()))
    # the oracle's cell-list pair set (pinned to brute force on the CPU)
    pairs = oracle_mod.pairs_cells if spec.n > 5000 else oracle_mod.pairs_brute
    ref = set(map(tuple, pairs(spec, xb, spec.rc + spec.skin, exclude=True).tolist()))
    assert got == ref


def _compare_eval(hd, oracle_mod, spec, precision, exec_mode=0, ftol=None):
    ref = oracle_mod.OracleSystem(spec).compute()
    ctx = hd.make_context([spec], precision=precision, exec_mode=exec_mode, init_velocities=False)
    sc = ctx.scalars(0)
    out = {w: ctx.forces(0, w) for w in (hd.HD_FORCE_TOTAL, hd.HD_FORCE_LJ, hd.HD_FORCE_BIAS, hd.HD_HU)}
    return ref, sc, out


@pytest.mark.parametrize("exec_mode", [0, 1, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_evaluation_fp64(hd, oracle_mod, exec_mode, dim):
    spec = snapshot_2d() if dim == 2 else snapshot_3d(nx=12, nz=4, R=5.0)
    spec = biased(oracle_mod, spec)
    ref, sc, out = _compare_eval(hd, oracle_mod, spec, hd.HD_FP64, exec_mode)
    assert 0.0 < ref["dv"] < spec.dv_max
    assert rel(out[hd.HD_FORCE_LJ], ref["f_lj"]) < 1e-11
    assert rel(out[hd.HD_HU], ref["hu"]) < 1e-11
    assert rel(out[hd.HD_FORCE_BIAS], ref["f_b"]) < 1e-10
    assert rel(out[hd.HD_FORCE_TOTAL], ref["f_tot"]) < 1e-11
    for k in ("e_pot", "g", "d"):
        assert sc[k] == pytest.approx(ref[k], rel=1e-11), k
    assert abs(sc["dv"] - ref["dv"]) <= 1e-11 * spec.dv_max
    assert sc["f_lat"] == pytest.approx(ref["f_lat"], rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("exec_mode", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_evaluation_fp32c(hd, oracle_mod, exec_mode, dim):
    spec = snapshot_2d(seed=7) if dim == 2 else snapshot_3d(seed=9)
    spec = biased(oracle_mod, spec)
    ref, sc, out = _compare_eval(hd, oracle_mod, spec, hd.HD_FP32C, exec_mode)
    assert rel(out[hd.HD_FORCE_TOTAL], ref["f_tot"]) <= 1e-5
    assert rel(out[hd.HD_FORCE_LJ], ref["f_lj"]) <= 1e-5
    assert abs(sc["dv"] - ref["dv"]) <= 1e-6 * spec.dv_max
    assert sc["e_pot"] == pytest.approx(ref["e_pot"], rel=1e-6)
    assert sc["g"] == pytest.approx(ref["g"], rel=1e-5)


def _trajectory(hd, oracle_mod, spec, precision, nsteps, exec_mode=0):
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(nsteps)
    ctx = hd.make_context([spec], precision=precision, exec_mode=exec_mode, init_velocities=True)
    ctx.step(nsteps)
    return o, ctx


@pytest.mark.parametrize("exec_mode", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_short_trajectory_fp64(hd, oracle_mod, exec_mode, dim):
    spec = snapshot_2d(seed=11) if dim == 2 else snapshot_3d(seed=12, nx=10, nz=4, R=4.0)
    spec.kT, spec.gamma = 0.1, 1.0
    spec = biased(oracle_mod, spec)
    o, ctx = _trajectory(hd, oracle_mod, spec, hd.HD_FP64, 10, exec_mode)
    dx = ctx.positions(0) - o.positions()
    for k in range(spec.dim):
        if spec.periodic[k]:
            dx[k] -= spec.box[k] * np.round(dx[k] / spec.box[k])
    assert np.abs(dx).max() < 1e-10
    assert np.abs(ctx.velocities(0) - o.velocities()).max() < 1e-9
    sc, so = ctx.scalars(0), o.scalars()
    assert sc["step"] == so["step"] == 10
    assert sc["t_hyper"] == pytest.approx(so["t_hyper"], rel=1e-10)
    assert sc["t_md"] == pytest.approx(so["t_md"], rel=1e-14)
    assert sc["e_kin"] == pytest.approx(so["e_kin"], rel=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_short_trajectory_fp32c(hd, oracle_mod, dim):
    """Force errors of ~1e-6 relative move positions by ~dt^2 |dF| per step."""
    spec = snapshot_2d(seed=13) if dim == 2 else snapshot_3d(seed=14, nx=10, nz=4, R=4.0)
    spec = biased(oracle_mod, spec)
    o, ctx = _trajectory(hd, oracle_mod, spec, hd.HD_FP32C, 10)
    dx = ctx.positions(0) - o.positions()
    for k in range(spec.dim):
        if spec.periodic[k]:
            dx[k] -= spec.box[k] * np.round(dx[k] / spec.box[k])
    assert np.abs(dx).max() < 1e-8
    sc, so = ctx.scalars(0), o.scalars()
    assert sc["t_hyper"] == pytest.approx(so["t_hyper"], rel=1e-6)


def test_clock_limits_on_gpu(hd, oracle_mod):
    spec = snapshot_2d(seed=4)
    spec.bias_on, spec.dv_max, spec.kT = 1, 0.3, 0.1
    spec.g_lo, spec.g_hi = -2e30, -1e30
    ctx = hd.make_context([spec], precision=hd.HD_FP64)
    ctx.step(40)
    sc = ctx.scalars(0)
    assert sc["dv"] == spec.dv_max
    assert sc["t_hyper"] == pytest.approx(sc["t_md"] * np.exp(spec.dv_max / spec.kT), rel=1e-13)
    assert np.all(ctx.forces(0, hd.HD_FORCE_BIAS) == 0.0)


def test_batch_matches_single_and_order(hd, oracle_mod):
    """Each system of a batch gives the same bits as when run alone, in any order."""
    specs = []
    for k in range(4):
        s = snapshot_2d(seed=20 + k, x_slider=k * A2D / 4)
        specs.append(biased(oracle_mod, s))
    big = hd.make_context(specs, precision=hd.HD_FP64, block_threads=512)
    big.step(25)
    rev = hd.make_context(specs[::-1], precision=hd.HD_FP64, block_threads=512)
    rev.step(25)
    for k in (0, 3):
        one = hd.make_context([specs[k]], precision=hd.HD_FP64, block_threads=512)
        one.step(25)
        np.testing.assert_array_equal(big.positions(k), one.positions(0))
        np.testing.assert_array_equal(rev.positions(3 - k), one.positions(0))
        assert big.scalars(k)["t_hyper"] == one.scalars(0)["t_hyper"]


def test_mixed_uneven_batch(hd, oracle_mod):
    """2D and 3D instances of different sizes in one launch, each checked
    against the oracle (float32 tolerances)."""
    specs = [s for s in config_c4(12, seed=77, n_max=6000)]
    specs = [biased(oracle_mod, s) for s in specs[:6]]
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=False)
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        assert rel(ctx.forces(k), ref["f_tot"]) <= 1e-5, k
        assert abs(ctx.scalars(k)["dv"] - ref["dv"]) <= 1e-6 * s.dv_max


@pytest.mark.parametrize("precision,half", [(0, 0), (1, 0), (1, 1)])
def test_lds_energy_after_a_multistep_launch(hd, oracle_mod, precision, half):
    """The LDS-resident kernel evaluates the pair energy on a launch's last
    step only: after a 30-step launch the energy, dV and slope match the
    oracle's same trajectory (float64 1e-10; float32 1e-6 relative, full and
    half lists)."""
    spec = biased(oracle_mod, snapshot_2d(seed=61))
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(30)
    ctx = hd.make_context([spec], precision=precision)
    shape = ctx.schedule()
    assert shape["lds_resident"] == 1
    if precision == 1:
        shape["small_half_lists"] = half
        ctx.set_schedule(shape)
    ctx.step(30)
    sc, so = ctx.scalars(0), o.scalars()
    tol = 1e-10 if precision == 0 else 1e-6
    assert sc["step"] == 30
    assert sc["e_pot"] == pytest.approx(so["e_pot"], rel=tol)
    assert abs(sc["dv"] - so["dv"]) <= tol * spec.dv_max
    assert sc["g"] == pytest.approx(so["g"], rel=10 * tol, abs=tol)
    ctx.close()


@pytest.mark.parametrize("lds", [True, False])
def test_fp64_determinism_and_checkpoint(hd, oracle_mod, lds):
    """Chunked runs equal one long run bit for bit, and a checkpoint restored
    into a fresh context continues bit-identically."""
    spec = biased(oracle_mod, snapshot_2d(seed=31))
    a = hd.make_context([spec], precision=hd.HD_FP64, lds_resident=lds)
    a.step(30)
    blob = a.get_state(0)
    a.step(40)
    b = hd.make_context([spec], precision=hd.HD_FP64, lds_resident=lds)
    b.step(70)
    np.testing.assert_array_equal(a.positions(0), b.positions(0))
    np.testing.assert_array_equal(a.velocities(0), b.velocities(0))
    c = hd.make_context([spec], precision=hd.HD_FP64, lds_resident=lds)
    c.set_state(0, blob)
    c.step(40)
    np.testing.assert_array_equal(c.positions(0), a.positions(0))
    np.testing.assert_array_equal(c.velocities(0), a.velocities(0))
    assert c.scalars(0)["t_hyper"] == a.scalars(0)["t_hyper"]
    assert c.scalars(0)["step"] == 70


@pytest.mark.parametrize("precision", [0, 1])
def test_lds_resident_matches_global_kernel(hd, oracle_mod, precision):
    """The LDS-resident kernel and the global-memory kernel follow the same
    trajectory (same arithmetic, different memory); both match the oracle."""
    specs = [biased(oracle_mod, snapshot_2d(seed=40 + k, x_slider=k * A2D / 3)) for k in range(3)]
    a = hd.make_context(specs, precision=precision, lds_resident=True)
    b = hd.make_context(specs, precision=precision, lds_resident=False)
    for ctx in (a, b):
        ctx.step(60)
    for k in range(3):
        dx = a.positions(k) - b.positions(k)
        dx[0] -= specs[k].box[0] * np.round(dx[0] / specs[k].box[0])
        assert np.abs(dx).max() < (1e-11 if precision == 0 else 1e-7)
        sa, sb = a.scalars(k), b.scalars(k)
        assert sa["step"] == sb["step"] == 60
        assert sa["t_hyper"] == pytest.approx(sb["t_hyper"], rel=1e-9 if precision == 0 else 1e-5)
    # an evaluation through the LDS-resident kernel against the oracle
    ref = oracle_mod.OracleSystem(specs[1]).compute()
    c = hd.make_context([specs[1]], precision=precision, lds_resident=True, init_velocities=False)
    tol = 1e-11 if precision == 0 else 1e-5
    assert rel(c.forces(0), ref["f_tot"]) <= tol
    assert rel(c.forces(0, hd.HD_HU), ref["hu"]) <= tol
    assert abs(c.scalars(0)["dv"] - ref["dv"]) <= (1e-11 if precision == 0 else 1e-6) * specs[1].dv_max
    pairs = set(map(tuple, c.debug_pairs(0).tolist()))
    refp = set(map(tuple, oracle_mod.pairs_brute(specs[1], specs[1].pos, 2.8).tolist()))
    assert pairs == refp


@pytest.mark.parametrize("precision", [0, 1])
def test_large_systems_on_both_schedulers(hd, oracle_mod, precision):
    """Systems above the LDS limit run on the grid kernels by default, or on
    the persistent one-workgroup kernel on request; both follow the oracle."""
    specs = [biased(oracle_mod, snapshot_3d(seed=70 + k, nx=10, nz=4, R=4.0, x_slider=0.1 * k)) for k in range(2)]
    specs.append(biased(oracle_mod, snapshot_2d(seed=72)))       # a small one alongside
    a = hd.make_context(specs, precision=precision)
    b = hd.make_context(specs, precision=precision, persistent_large=True)
    tol = 1e-11 if precision == 0 else 1e-5
    for k, s in enumerate(specs):
        ref = oracle_mod.OracleSystem(s).compute()
        for ctx in (a, b):
            assert rel(ctx.forces(k), ref["f_tot"]) <= tol, k
    for ctx in (a, b):
        ctx.step(60)
    for k, s in enumerate(specs):
        dx = a.positions(k) - b.positions(k)
        for d in range(s.dim):
            if s.periodic[d]:
                dx[d] -= s.box[d] * np.round(dx[d] / s.box[d])
        assert np.abs(dx).max() < (1e-10 if precision == 0 else 1e-6), k
        assert a.scalars(k)["step"] == b.scalars(k)["step"] == 60


@pytest.mark.parametrize("exec_mode", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_continuous_sliding_trajectory(hd, oracle_mod, exec_mode, precision):
    """The plain-MD workload (one position, slider moving at v = 0.01, bias
    off) over 200 steps: the drive's slider position and lateral force follow
    the oracle (reading: x_S(step) = x_S + v_S step dt)."""
    from hd_inputs import config_c1
    spec = config_c1()[0]
    o = oracle_mod.OracleSystem(spec)
    o.init_velocities()
    o.step(200)
    ctx = hd.make_context([spec], precision=precision, exec_mode=exec_mode, init_velocities=True)
    ctx.step(200)
    sc, so = ctx.scalars(0), o.scalars()
    assert sc["x_slider"] == pytest.approx(so["x_slider"], rel=1e-14, abs=1e-14)
    assert sc["x_slider"] == pytest.approx(spec.x_slider + 200 * spec.dt * spec.v_slider, rel=1e-12)
    tol = 1e-9 if precision == 0 else 1e-4
    assert sc["f_lat"] == pytest.approx(so["f_lat"], rel=tol, abs=tol)
    assert sc["x_tip"] == pytest.approx(so["x_tip"], rel=tol, abs=tol)
    assert sc["t_hyper"] == sc["t_md"]       # no bias: the clocks agree


@pytest.mark.parametrize("exec_mode", [0, 1])
def test_parameter_changes_after_finalize(hd, oracle_mod, exec_mode):
    """Slider position, bias and thermostat changed after hd_finalize take
    effect at the next evaluation, as in an oracle built with the new values."""
    spec = biased(oracle_mod, snapshot_2d(seed=13))
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    new = spec.copy()
    new.x_slider = spec.x_slider + 0.37
    new.dv_max, new.m_b = 0.8, 3
    new = biased(oracle_mod, new, frac=0.3, dv_max=0.8)
    new.m_b = 3
    new.kT, new.gamma = 0.15, 2.0
    ctx.set_slider(0, new.x_slider)
    ctx.set_bias(0, True, new.m_b, new.dv_max, new.g_lo, new.g_hi)
    ctx.set_thermo(0, new.dt, new.gamma, new.kT, new.seed)
    ctx.compute()
    ref = oracle_mod.OracleSystem(new).compute()
    sc = ctx.scalars(0)
    assert sc["x_slider"] == pytest.approx(new.x_slider, rel=1e-15)
    assert sc["f_lat"] == pytest.approx(ref["f_lat"], rel=1e-11, abs=1e-12)
    assert abs(sc["dv"] - ref["dv"]) <= 1e-11 * new.dv_max
    assert rel(ctx.forces(0), ref["f_tot"]) <= 1e-11
    # the thermostat change shows in a short trajectory from the same state
    # (velocities zero on both sides)
    o = oracle_mod.OracleSystem(new)
    o.step(10)
    ctx.step(10)
    dx = ctx.positions(0) - o.positions()
    dx[0] -= new.box[0] * np.round(dx[0] / new.box[0])
    assert np.abs(dx).max() < 1e-10
    assert np.abs(ctx.velocities(0) - o.velocities()).max() < 1e-9
