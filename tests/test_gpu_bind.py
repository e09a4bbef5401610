"""Caller-owned device storage (hd_bind_device) and what a checkpoint carries.

Bound fields: the kernels step the batch inside torch tensors' storage, and
the trajectories still match the oracle's (float64: 1e-10, as in
test_gpu_parity).  Checkpoints: the run state moves, the seed and the slider
stay with the system it is restored into.
"""
import ctypes

import numpy as np
import pytest

from hd_inputs import build_2d, build_3d, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def _spec2d(seed, x_slider=0.25):
    s = build_2d()
    s.x_slider = x_slider
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.seed = 7000 + seed
    return s


def _spec3d(seed, x_slider=0.4):
    s = build_3d(10, 10, 4, 4.0)
    s.x_slider = x_slider
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.seed = 7100 + seed
    return s


def _min_image(spec, dx):
    dx = dx.copy()
    for k in range(spec.dim):
        if spec.periodic[k]:
            dx[k] -= spec.box[k] * np.round(dx[k] / spec.box[k])
    return dx


def _oracle_run(oracle_mod, spec, nsteps, v0=None):
    o = oracle_mod.OracleSystem(spec)
    if v0 is None:
        o.init_velocities()
    else:
        o.set_velocities(v0)
    o.step(nsteps)
    return o


@pytest.mark.parametrize("exec_mode", [0, 1])
def test_bound_fields_step_in_caller_storage(hd, oracle_mod, exec_mode):
    import torch
    specs = [_spec2d(1), _spec3d(2)]
    ctx = hd.make_context(specs, precision=hd.HD_FP64, exec_mode=exec_mode, init_velocities=True)
    off = [ctx.batch_layout(k)[0] for k in range(2)]
    nt = ctx.batch_layout(0)[1]
    assert nt == sum(s.n for s in specs) and off == [0, specs[0].n]
    x0 = [ctx.positions(k) for k in range(2)]
    X = torch.full((3, nt), float("nan"), dtype=torch.float64, device="cuda")
    V = torch.zeros((3, nt), dtype=torch.float64, device="cuda")
    F = torch.zeros((3, nt), dtype=torch.float64, device="cuda")
    ctx.bind_device(hd.HD_FIELD_POSITIONS, X)
    ctx.bind_device(hd.HD_FIELD_VELOCITIES, V)
    ctx.bind_device(hd.HD_FIELD_FORCES, F)
    ctx.sync()
    torch.cuda.synchronize()
    # binding moves the current contents into the caller's storage
    for k, s in enumerate(specs):
        np.testing.assert_array_equal(X[:s.dim, off[k]:off[k] + s.n].cpu().numpy(), x0[k])
    ctx.step(10)
    ctx.sync()
    torch.cuda.synchronize()
    for k, s in enumerate(specs):
        sl = slice(off[k], off[k] + s.n)
        np.testing.assert_array_equal(X[:s.dim, sl].cpu().numpy(), ctx.positions(k))
        np.testing.assert_array_equal(V[:s.dim, sl].cpu().numpy(), ctx.velocities(k))
        np.testing.assert_array_equal(F[:s.dim, sl].cpu().numpy(), ctx.forces(k, hd.HD_FORCE_TOTAL))
        o = _oracle_run(oracle_mod, s, 10)
        assert np.abs(_min_image(s, ctx.positions(k) - o.positions())).max() < 1e-10
        assert np.abs(ctx.velocities(k) - o.velocities()).max() < 1e-9
    # unbinding copies the field back; the caller's tensor is then left alone
    ctx.bind_device(hd.HD_FIELD_POSITIONS, None)
    kept = X.clone()
    ctx.step(5)
    ctx.sync()
    torch.cuda.synchronize()
    assert torch.equal(X, kept)
    for k, s in enumerate(specs):
        o = _oracle_run(oracle_mod, s, 15)
        assert np.abs(_min_image(s, ctx.positions(k) - o.positions())).max() < 1e-10
        sl = slice(off[k], off[k] + s.n)
        np.testing.assert_array_equal(V[:s.dim, sl].cpu().numpy(), ctx.velocities(k))
    # positions written through the library land in the bound storage
    ctx.bind_device(hd.HD_FIELD_POSITIONS, X)
    ctx.set_positions(0, specs[0].pos)
    ctx.sync()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(X[:2, off[0]:off[0] + specs[0].n].cpu().numpy(), ctx.positions(0))
    ctx.close()


def test_bind_device_argument_errors(hd):
    import torch
    L = hd.load()
    spec = _spec2d(3)
    ctx = hd.Context(hd.HD_FP64)
    ctx.add_system(spec)
    X = torch.zeros((3, spec.n), dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(X.data_ptr())
    assert L.hd_bind_device(ctx.handle, hd.HD_ALL_SYSTEMS, hd.HD_FIELD_POSITIONS, p) == hd.HD_E_STATE
    ctx.finalize()
    assert L.hd_bind_device(ctx.handle, 0, hd.HD_FIELD_POSITIONS, p) == hd.HD_E_ARG
    assert L.hd_bind_device(ctx.handle, hd.HD_ALL_SYSTEMS, 6, p) == hd.HD_E_ARG
    assert L.hd_bind_device(ctx.handle, hd.HD_ALL_SYSTEMS, -1, p) == hd.HD_E_ARG
    host = np.zeros(3 * spec.n)
    assert L.hd_bind_device(ctx.handle, hd.HD_ALL_SYSTEMS, hd.HD_FIELD_POSITIONS,
                            ctypes.c_void_p(host.ctypes.data)) == hd.HD_E_ARG
    assert L.hd_bind_device(ctx.handle, hd.HD_ALL_SYSTEMS, hd.HD_FIELD_POSITIONS,
                            ctypes.c_void_p(X.data_ptr() + 4)) == hd.HD_E_ARG
    with pytest.raises(ValueError):
        ctx.bind_device(hd.HD_FIELD_POSITIONS, torch.zeros((3, spec.n + 1), dtype=torch.float64, device="cuda"))
    # the context still works after the refusals
    ctx.step(3)
    assert ctx.scalars(0)["step"] == 3
    ctx.close()


def test_checkpoint_keeps_the_targets_seed_and_slider(hd, oracle_mod):
    """A state restored into another system continues with that system's
    own Philox stream and slider position (the redistribution of Sec. 2.3
    seeds several positions from one state)."""
    a, b = _spec2d(4, x_slider=0.1), _spec2d(4, x_slider=0.6)
    b.seed = a.seed + 1
    ctx = hd.make_context([a, b], precision=hd.HD_FP64, init_velocities=True)
    v0 = ctx.velocities(0)
    ctx.set_state(1, ctx.get_state(0))
    sc = ctx.scalars(1)
    assert sc["step"] == 0
    ctx.step(10)
    # the target's seed: the oracle from the same state with b's seed and slider
    o = _oracle_run(oracle_mod, b, 10, v0=v0)
    assert np.abs(_min_image(b, ctx.positions(1) - o.positions())).max() < 1e-10
    assert ctx.scalars(1)["x_slider"] == pytest.approx(b.x_slider, abs=1e-15)
    # ... and so a different trajectory from the source's
    assert np.abs(_min_image(a, ctx.positions(1) - ctx.positions(0))).max() > 1e-6
    # restored into its own system (same seed), the run continues bit for bit
    st = ctx.get_state(0)
    ctx.step(7)
    x7 = ctx.positions(0)
    ctx.set_state(0, st)
    ctx.step(7)
    np.testing.assert_array_equal(ctx.positions(0), x7)
    ctx.close()
