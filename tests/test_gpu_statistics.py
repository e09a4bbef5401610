"""Long-run statistics on the GPU: trajectories of a chaotic system agree
with the oracle's only for a short horizon, so longer runs are compared by
what they sample -- equipartition under both thermostats, and the boosted
clock's mean boost <exp(dV/kT)> (eq. 3) against the oracle's own run."""
import numpy as np
import pytest

from hd_inputs import ROLE_MOBILE, build_2d, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def ndof(spec):
    return spec.dim * (int((spec.role == ROLE_MOBILE).sum()) + 1)


@pytest.mark.parametrize("thermostat", ["langevin", "nhc"])
def test_equipartition(hd, thermostat):
    """<K> = N_f kT / 2 over a long run (mobile atoms and the rigid body)."""
    specs = []
    for k in range(8):
        s = build_2d()
        s.kT, s.seed, s.x_slider = 0.1, 300 + k, 0.05 * k
        if thermostat == "nhc":
            s.thermostat, s.nhc_len, s.nhc_tau = 1, 3, 0.5
        specs.append(s)
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=True)
    ctx.step(4000)
    ek = []
    for _ in range(100):
        ctx.step(100)
        ek.append([ctx.scalars(k)["e_kin"] for k in range(len(specs))])
    mean = np.mean(ek) / (0.5 * ndof(specs[0]))
    assert mean == pytest.approx(0.1, rel=0.03)


def test_mean_boost_matches_the_oracle(hd, oracle_mod):
    """A biased run on the GPU (float32 pairs) and the oracle's (float64)
    from the same state decorrelate, but sample the same boost: the ratio
    t_hyper / t_MD of the two agrees within the statistical spread of
    independent runs."""
    base = build_2d()
    base.kT, base.x_slider = 0.1, 0.2
    base.rO = base.pos.copy()
    g = oracle_mod.OracleSystem(base).compute()["g"]
    runs_gpu, runs_orc = [], []
    for k in range(4):
        s = base.copy()
        s.seed = 900 + k
        s.pos = perturbed(s, 0.02, 40 + k)
        s.bias_on, s.m_b, s.dv_max = 1, 2, 0.5
        s.g_lo, s.g_hi = g - 4.0, g + 4.0
        ctx = hd.make_context([s], precision=hd.HD_FP32C, init_velocities=True)
        ctx.step(3000)
        sc = ctx.scalars(0)
        runs_gpu.append(sc["t_hyper"] / sc["t_md"])
        o = oracle_mod.OracleSystem(s)
        o.init_velocities()
        o.step(3000)
        so = o.scalars()
        runs_orc.append(so["t_hyper"] / so["t_md"])
    a, b = np.array(runs_gpu), np.array(runs_orc)
    assert np.all(a > 1.0) and np.all(b > 1.0)
    spread = max(a.std(), b.std(), 1e-3 * a.mean())
    assert abs(a.mean() - b.mean()) <= 4.0 * spread
