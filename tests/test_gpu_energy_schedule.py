"""The grid kernels evaluate the pair energy only on the last step of each
replayed sequence of steps (the steps before it run the pair pass without the
energy terms): after any call of hd_step the reported energy is that of the
final positions, the same as a fresh evaluation there."""
import numpy as np
import pytest

from hd_inputs import build_2d, build_3d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


# calls of one sequence (50), a full sequence and a remainder (60), and calls
# that start and end inside sequences
@pytest.mark.parametrize("calls", [(50,), (60,), (7, 50, 3)])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("lds", [False, True])
def test_energy_after_step_calls(hd, calls, precision, lds):
    specs = [build_3d(7, 7, 3, 2.0), build_2d()]
    prec = hd.HD_FP64 if precision == "fp64" else hd.HD_FP32C
    ctx = hd.make_context(specs, precision=prec, lds_resident=lds)
    for n in calls:
        ctx.step(n)
        got = [ctx.scalars(s) for s in range(len(specs))]
        ctx.compute()
        ref = [ctx.scalars(s) for s in range(len(specs))]
        for s, (g, r) in enumerate(zip(got, ref)):
            assert g["flags"] == 0, (s, g["flags"])
            assert np.isfinite(g["e_pot"]) and g["e_pot"] != 0.0, (s, g["e_pot"])
            # the same pair terms at the same positions: only their order of
            # summation may differ
            assert abs(g["e_pot"] - r["e_pot"]) <= 1e-9 * abs(r["e_pot"]), (s, n, g["e_pot"], r["e_pot"])
            assert g["step"] == r["step"]
