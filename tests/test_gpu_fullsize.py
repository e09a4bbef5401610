"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (batched scheduler, float32 pair arithmetic with float64
per-atom sums).  The oracle evaluates sampled systems of each batch in full; every
system's scalars must be finite.

Tolerances as in test_gpu_parity: relative L2 force error <= 1e-5 per system,
|dV - dV_ref| <= 1e-6 dV_max.
"""
import numpy as np
import pytest

from hd_inputs import config_c2, config_c3, config_c4, config_c5a, config_c5b, perturbed

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-5     # relative L2 force error of the float32 path, per system
DV_TOL = 1e-6        # |dV - dV_ref| / dV_max


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def snapshot(oracle_mod, spec, seed, need_bias=True):
    """Jittered lattice snapshot with r_O = lattice and thresholds that
    bracket the snapshot's slope."""
    s = spec.copy()
    s.rO = s.pos.copy()
    s.pos = perturbed(s, 0.05, seed)
    if need_bias:
        g = oracle_mod.OracleSystem(s).compute()["g"]
        span = 2.0 * abs(g) + 1.0
        s.bias_on, s.m_b, s.dv_max = 1, 2, 5.0 * s.kT
        s.g_lo, s.g_hi = g - 0.4 * span, g + 0.6 * span
    return s


def check_batch(hd, oracle_mod, specs, sample, block=0):
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=False, block_threads=block)
    for k in range(len(specs)):
        sc = ctx.scalars(k)
        assert np.isfinite(sc["e_pot"]) and sc["flags"] == 0, k
    for k in sample:
        ref = oracle_mod.OracleSystem(specs[k]).compute()
        assert rel(ctx.forces(k), ref["f_tot"]) <= FORCE_TOL, k
        sc = ctx.scalars(k)
        assert abs(sc["dv"] - ref["dv"]) <= DV_TOL * specs[k].dv_max, k
        assert sc["e_pot"] == pytest.approx(ref["e_pot"], rel=1e-6), k
    return ctx


def test_c2_full_batch(hd, oracle_mod):
    specs = [snapshot(oracle_mod, s, 100 + k) for k, s in enumerate(config_c2())]
    check_batch(hd, oracle_mod, specs, range(len(specs)))


# the grid tile sizes the autotuner picks for the 3D batches (64 or 128
# atoms), and the default
@pytest.mark.parametrize("block", [64, 128, 256])
def test_c3_sampled(hd, oracle_mod, block):
    base = config_c3()
    sample = [0, 21, 42, 63]
    specs = [snapshot(oracle_mod, s, 200 + k, need_bias=(k in sample)) for k, s in enumerate(base)]
    check_batch(hd, oracle_mod, specs, sample, block)


@pytest.mark.parametrize("block", [64, 128, 256])
def test_c5b_sampled(hd, oracle_mod, block):
    base = config_c5b()
    sample = [0, 101, 255]
    specs = [snapshot(oracle_mod, s, 300 + k, need_bias=(k in sample)) for k, s in enumerate(base)]
    check_batch(hd, oracle_mod, specs, sample, block)


def test_c4_sampled(hd, oracle_mod):
    base = config_c4()
    sizes = np.array([s.n for s in base])
    sample = sorted({int(sizes.argmin()), int(sizes.argmax()), 7, 77})
    specs = [snapshot(oracle_mod, s, 400 + k, need_bias=(k in sample)) for k, s in enumerate(base)]
    check_batch(hd, oracle_mod, specs, sample)


@pytest.mark.slow
def test_c5a_one_million_atoms(hd, oracle_mod):
    spec = snapshot(oracle_mod, config_c5a()[0], 500)
    check_batch(hd, oracle_mod, [spec], [0])


def test_c3_short_trajectory_sampled(hd, oracle_mod):
    """20 steps of the full C3 batch; two sampled systems against the oracle's
    trajectories from the same state and Philox stream."""
    base = config_c3()
    sample = [5, 50]
    specs = [snapshot(oracle_mod, s, 600 + k, need_bias=(k in sample)) for k, s in enumerate(base)]
    nsteps = 20
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=True)
    f0 = {k: ctx.forces(k) for k in sample}
    ctx.step(nsteps)
    for k in sample:
        o = oracle_mod.OracleSystem(specs[k])
        f_ref = o.compute()["f_tot"]
        # the stated float32 tolerance first: relative L2 force error <= 1e-5
        rel = np.linalg.norm(f0[k] - f_ref) / np.linalg.norm(f_ref)
        assert rel <= FORCE_TOL, (k, rel)
        # a force error within that tolerance is at most FORCE_TOL |F_ref|_2
        # on any one atom; held over n steps it moves an atom by at most
        # (n dt)^2 / 2 times that (unit mass), and the dynamics can amplify a
        # displacement error over t = n dt by at most about
        # (cosh(w t) - 1) / ((w t)^2 / 2) ~ 1.4 for the stiffest mode of the
        # fcc lattice (w ~ 20 / tau at t = 0.1 tau): a factor 4 covers it
        bound = 4.0 * 0.5 * (nsteps * specs[k].dt) ** 2 * FORCE_TOL * np.linalg.norm(f_ref)
        o.init_velocities()
        o.step(nsteps)
        dx = ctx.positions(k) - o.positions()
        for d in range(3):
            if specs[k].periodic[d]:
                dx[d] -= specs[k].box[d] * np.round(dx[d] / specs[k].box[d])
        err = float(np.abs(dx).max())
        assert err < bound, (k, err, bound)
        assert ctx.scalars(k)["t_hyper"] == pytest.approx(o.scalars()["t_hyper"], rel=1e-6)
