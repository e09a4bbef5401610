"""hd_quench_noalloc (no device allocation, scratch in the library's static
device array) against hd_quench, called through the C ABI.

Both run the same FIRE kernels on the same inputs, so iterations, the
displacements and the minima agree bit for bit; two calls in a row, the
second on a smaller input, check that the shared scratch carries nothing
from one call to the next.  The run state is untouched afterwards: stepping
continues bit for bit like a run that was never quenched.
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


def _jittered(spec, seed):
    s = spec.copy()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    s.x_slider = 0.15
    return s


def _specs(oracle_mod):
    specs = [_jittered(build_2d(), 40), _jittered(build_3d(7, 7, 3, 2.0), 41), _jittered(build_2d(), 42)]
    for s in specs:
        s.bias_on, s.m_b, s.dv_max = 1, 2, 0.5
        g = oracle_mod.OracleSystem(s).compute()["g"]
        s.g_lo, s.g_hi = g - 2.0, g + 3.0
    return specs


def _call(hd, ctx, fn, systems, ftol, max_iters, mode):
    n = len(systems)
    ids = (ctypes.c_int32 * n)(*systems)
    iters = (ctypes.c_int64 * n)()
    disp = np.zeros(n)
    tot = sum(ctx.dims[k] * ctx.sizes[k] for k in systems)
    xm = np.zeros(tot)
    st = fn(ctx.handle, ids, n, float(ftol), int(max_iters), int(mode), iters,
            disp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            xm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert st == hd.HD_OK, load_error(hd, ctx)
    return list(iters), disp, xm


def load_error(hd, ctx):
    return hd.load().hd_last_error(ctx.handle).decode()


@pytest.mark.parametrize("precision,exec_mode", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_noalloc_quench_matches_hd_quench(hd, oracle_mod, precision, exec_mode):
    L = hd.load()
    specs = _specs(oracle_mod)
    ftol = 1e-6 if precision == 0 else 1e-3
    calls = [([1, 0, 2], hd.HD_QUENCH_CHECK), ([2], hd.HD_QUENCH_CHECK)]
    ref = hd.make_context(specs, precision=precision, exec_mode=exec_mode)
    new = hd.make_context(specs, precision=precision, exec_mode=exec_mode)
    plain = hd.make_context(specs, precision=precision, exec_mode=exec_mode)
    for c in (ref, new, plain):
        c.step(30)
    for systems, mode in calls:
        a = _call(hd, ref, L.hd_quench, systems, ftol, 50000, mode)
        b = _call(hd, new, L.hd_quench_noalloc, systems, ftol, 50000, mode)
        assert all(v > 0 for v in a[0])
        assert a[0] == b[0]
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_array_equal(a[2], b[2])
    # the run continues as if never quenched
    for c in (ref, new, plain):
        c.step(30)
    for k in range(len(specs)):
        np.testing.assert_array_equal(new.positions(k), plain.positions(k))
        np.testing.assert_array_equal(new.velocities(k), plain.velocities(k))
        np.testing.assert_array_equal(new.forces(k, hd.HD_FORCE_TOTAL), plain.forces(k, hd.HD_FORCE_TOTAL))
        sa, sb = new.scalars(k), plain.scalars(k)
        for key in ("step", "t_md", "t_hyper", "dv", "e_pot", "n_rebuilds"):
            assert sa[key] == sb[key], key
    for c in (ref, new, plain):
        c.close()


def test_noalloc_set_reference(hd, oracle_mod):
    """With set_reference the minimum becomes r_O, as with hd_quench."""
    L = hd.load()
    specs = _specs(oracle_mod)[:1]
    ref = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=False)
    new = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=False)
    a = _call(hd, ref, L.hd_quench, [0], 1e-8, 50000, hd.HD_QUENCH_SET_REFERENCE)
    b = _call(hd, new, L.hd_quench_noalloc, [0], 1e-8, 50000, hd.HD_QUENCH_SET_REFERENCE)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[2], b[2])
    _, d, _ = _call(hd, new, L.hd_quench_noalloc, [0], 1e-8, 50000, hd.HD_QUENCH_CHECK)
    assert d[0] < 1e-6
    ref.close()
    new.close()
