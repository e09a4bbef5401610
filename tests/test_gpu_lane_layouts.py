"""The grid pair kernels at one, two and four lanes per atom (tiles of 1024,
512 and 128 atoms): the four-lane kernels gather the neighbour records per
quad through LDS, the others per lane.  Each pair-term variant -- LJ only,
the curvature terms, the eigenvalue terms, tip bonds -- against the oracle
in float64 (10^-10) and float32 (the stated tolerances)."""
import numpy as np
import pytest

from test_gpu_bias_vars import biased
from test_gpu_eigen_bias import eig_spec

pytestmark = pytest.mark.gpu

BLOCKS = [128, 512, 1024]


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check(hd, oracle_mod, spec, block, curv=False, eig=False):
    ref = oracle_mod.OracleSystem(spec).compute()
    assert 0.0 < ref["dv"] < spec.dv_max
    for prec in (hd.HD_FP64, hd.HD_FP32C):
        ctx = hd.make_context([spec], precision=prec, exec_mode=hd.HD_EXEC_GRID, block_threads=block,
                              init_velocities=False)
        sc = ctx.scalars(0)
        if prec == hd.HD_FP64:
            assert rel(ctx.forces(0, hd.HD_FORCE_LJ), ref["f_lj"]) < 1e-11
            assert rel(ctx.forces(0, hd.HD_HU), ref["hu"]) < 1e-11
            assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) < 1e-10
            assert abs(sc["dv"] - ref["dv"]) <= 1e-10 * spec.dv_max
            if curv or eig:
                assert rel(ctx.forces(0, hd.HD_TUU), ref["tuu"]) < 1e-10
            if eig:
                assert sc["lambda"] == pytest.approx(ref["lambda"], rel=1e-10)
        else:
            assert rel(ctx.forces(0, hd.HD_FORCE_TOTAL), ref["f_tot"]) <= 1e-5
            assert abs(sc["dv"] - ref["dv"]) <= 1e-6 * spec.dv_max
        ctx.close()


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("model", ["3d", "cone"])
def test_slope_and_curvature(hd, oracle_mod, model, block):
    check(hd, oracle_mod, biased(oracle_mod, model, 0, 1, 91), block, curv=True)


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("model", ["3d", "cone"])
def test_slope_and_eigenvalue(hd, oracle_mod, model, block):
    check(hd, oracle_mod, eig_spec(oracle_mod, model, 92, 0, 3), block, eig=True)


@pytest.mark.parametrize("block", BLOCKS)
def test_slope_only(hd, oracle_mod, block):
    check(hd, oracle_mod, biased(oracle_mod, "3d", 0, -1, 93), block)
