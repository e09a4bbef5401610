"""Lowest Hessian eigenvalue on the GPU (hd_min_mode): Lanczos over the
degrees of freedom with the pair pass's H u as the product, against the
oracle's dense reduced Hessian (§2.2, the eigenvalue bias variable)."""
import numpy as np
import pytest

from hd_inputs import build_2d, build_3d, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def small2d():
    return build_2d(nx=12, ny=4, tip_w=4, tip_h=3, n_fixed_rows=1)


def small3d():
    return build_3d(7, 7, 2, R=2.0)


@pytest.mark.parametrize("path", ["lds", "grid"])
@pytest.mark.parametrize("maker", [small2d, small3d], ids=["2d", "3d"])
def test_min_mode_matches_the_dense_eigenvalue(hd, oracle_mod, path, maker):
    spec = maker()
    spec.x_slider = 0.3
    spec.pos = perturbed(spec, 0.05, 21)
    exec_mode = hd.HD_EXEC_BATCHED if path == "lds" else hd.HD_EXEC_GRID
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=False)
    eps, it, mode = ctx.min_mode(0, max_iter=2000, tol=1e-13)
    assert it > 0
    ref, _ = oracle_mod.lowest_hessian_eigenvalue(spec, spec.pos)
    assert eps == pytest.approx(ref, rel=1e-8, abs=1e-9)
    # the Ritz vector is the eigenvector: its Rayleigh quotient on the
    # oracle's Hessian is the eigenvalue
    H = oracle_mod.reduced_hessian(spec, spec.pos)
    mob, rig, m = oracle_mod.dof_layout(spec)
    v = list(mode[:, mob].T.reshape(-1)) + (list(mode[:, rig[0]]) if len(rig) else [])
    v = np.array(v)
    assert np.linalg.norm(v) == pytest.approx(1.0, rel=1e-10)
    assert v @ H @ v == pytest.approx(ref, rel=1e-6, abs=1e-7)


def test_min_mode_leaves_the_run_untouched(hd):
    specs = [small2d(), small3d()]
    for s in specs:
        s.pos = perturbed(s, 0.05, 23)
    runs = []
    for probe in (False, True):
        ctx = hd.make_context(specs, precision=hd.HD_FP64)
        ctx.step(30)
        if probe:
            ctx.min_mode(1, max_iter=50, tol=1e-8)
        ctx.step(30)
        runs.append([(ctx.positions(k), ctx.velocities(k), ctx.scalars(k)["t_hyper"]) for k in range(2)])
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        assert a[2] == b[2]


def test_min_mode_argument_errors(hd):
    ctx = hd.make_context([small2d()], precision=hd.HD_FP64, init_velocities=False)
    with pytest.raises(hd.HDError):
        ctx.min_mode(1)
    with pytest.raises(hd.HDError):
        ctx.min_mode(0, max_iter=0)
    with pytest.raises(hd.HDError):
        ctx.min_mode(0, tol=0.0)


def small_cone():
    from hd_inputs import build_3d_cone
    return build_3d_cone(nx=9, ny=9, nz=1, layers=4)


@pytest.mark.parametrize("maker", [small2d, small3d, small_cone], ids=["2d", "3d", "cone"])
def test_eigenvalue_gradient(hd, oracle_mod, maker):
    """d eps/dy on the GPU (one pair pass with u = P q accumulating T[u,u])
    against the oracle's: with the oracle's eigenvector as the mode the two
    are the same contraction; with the GPU's own Lanczos mode the gradient
    agrees to the mode's accuracy."""
    spec = maker()
    spec.x_slider = 0.3
    spec.pos = perturbed(spec, 0.05, 25)
    ctx = hd.make_context([spec], precision=hd.HD_FP64, exec_mode=hd.HD_EXEC_GRID, init_velocities=False)
    eps_ref, q_ref, g_ref = oracle_mod.eigenvalue_gradient(spec)
    mob, rig, m = oracle_mod.dof_layout(spec)

    def dof(g):
        return np.array(list(g[:, mob].T.reshape(-1)) + (list(g[:, rig[0]]) if len(rig) else []))

    g = dof(ctx.min_mode_gradient(0, oracle_mod.dof_to_atoms(spec, q_ref)))
    assert np.linalg.norm(g - g_ref) <= 1e-10 * np.linalg.norm(g_ref)
    eps, it, mode = ctx.min_mode(0, max_iter=2000, tol=1e-13)
    assert it > 0 and eps == pytest.approx(eps_ref, rel=1e-8, abs=1e-9)
    g2 = dof(ctx.min_mode_gradient(0, mode))
    assert np.linalg.norm(g2 - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert np.all(ctx.min_mode_gradient(0, mode)[:, spec.role == 1] == 0.0)   # fixed atoms


def test_eigenvalue_gradient_leaves_the_run_untouched(hd, oracle_mod):
    specs = [small2d(), small3d()]
    for s in specs:
        s.pos = perturbed(s, 0.05, 27)
    runs = []
    for probe in (False, True):
        ctx = hd.make_context(specs, precision=hd.HD_FP64, exec_mode=hd.HD_EXEC_GRID)
        ctx.step(30)
        if probe:
            _, _, mode = ctx.min_mode(1, max_iter=40, tol=1e-8)
            ctx.min_mode_gradient(1, mode)
            # the gradient's evaluation rebuilds the lists at the current
            # positions (32-bit entries, on the curvature kernels): read
            # back before the next step, they hold the brute-force pair set
            got = set(map(tuple, ctx.debug_pairs(1).tolist()))
            s1 = specs[1]
            want = oracle_mod.pairs_brute(s1, ctx.positions(1), s1.rc + s1.skin, exclude=True)
            assert got == set(map(tuple, want.tolist()))
        ctx.step(30)
        runs.append([(ctx.positions(k), ctx.velocities(k), ctx.scalars(k)["t_hyper"]) for k in range(2)])
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        assert a[2] == b[2]


def test_eigenvalue_gradient_errors(hd):
    s = small2d()
    lds = hd.make_context([s], precision=hd.HD_FP64, init_velocities=False)
    if lds.schedule()["lds_resident"]:
        with pytest.raises(hd.HDError):
            lds.min_mode_gradient(0, np.ones((2, s.n)))     # LDS-resident: not on the grid kernels
    grid = hd.make_context([s], precision=hd.HD_FP64, exec_mode=hd.HD_EXEC_GRID, init_velocities=False)
    with pytest.raises(hd.HDError):
        grid.min_mode_gradient(0, np.zeros((2, s.n)))
