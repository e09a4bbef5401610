"""Run-to-run bit identity of the float32 half-list pass of the LDS-resident
kernel: the partner's share of each pair lands through LDS atomics in an
order that varies between runs, and is summed in fixed point so that the
total does not depend on it.  Two contexts stepping the same batch agree bit
for bit, as do a run and its checkpointed continuation."""
import numpy as np
import pytest

from hd_inputs import config_c2, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def _batch():
    specs = []
    for k, s in enumerate(config_c2(8)):
        s = s.copy()
        s.rO = s.pos.copy()
        s.pos = perturbed(s, 0.05, 500 + k)
        s.bias_on, s.m_b, s.dv_max, s.g_lo, s.g_hi = 1, 2, 0.5, -3.0, 3.0
        specs.append(s)
    return specs


def _half_list_ctx(hd, specs):
    ctx = hd.make_context(specs, precision=hd.HD_FP32C)
    shape = ctx.schedule()
    assert shape["lds_resident"] == 1
    shape["small_half_lists"] = 1
    ctx.set_schedule(shape)
    assert ctx.schedule()["small_half_lists"] == 1
    return ctx


def test_half_lists_repeat_bit_for_bit(hd):
    specs = _batch()
    runs = []
    for _ in range(2):
        ctx = _half_list_ctx(hd, specs)
        ctx.step(600)
        runs.append([(ctx.positions(k), ctx.velocities(k), ctx.forces(k, hd.HD_FORCE_TOTAL), ctx.scalars(k))
                     for k in range(len(specs))])
        ctx.close()
    for a, b in zip(*runs):
        for q in range(3):
            np.testing.assert_array_equal(a[q], b[q])
        for key in ("e_pot", "dv", "g", "t_hyper", "n_rebuilds"):
            assert a[3][key] == b[3][key], key
