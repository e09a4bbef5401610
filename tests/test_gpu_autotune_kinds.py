"""Launch shapes and the autotuner over a batch holding every kind of
system: a Nose-Hoover-chain model (LDS-resident when the shape allows), a
curvature-and-distance-biased model and a conical tip with tip bonds (grid
kernels always), and plain slope-biased models.  Every shape follows the
oracle; tuning leaves the run state as it was."""
import numpy as np
import pytest

from hd_inputs import build_2d, build_3d, build_3d_cone, perturbed

pytestmark = pytest.mark.gpu

SHAPES = [
    {"lds_resident": 1, "small_block": 1024, "persistent_large": 0, "large_block": 128, "small_half_lists": 0},
    {"lds_resident": 1, "small_block": 512, "persistent_large": 1, "large_block": 1024, "small_half_lists": 0},
    {"lds_resident": 0, "small_block": 0, "persistent_large": 0, "large_block": 512},
    {"lds_resident": 0, "small_block": 0, "persistent_large": 0, "large_block": 64},
    {"lds_resident": 0, "small_block": 0, "persistent_large": 1, "large_block": 256},
]


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def kinds(oracle_mod):
    out = []
    for maker, seed in ((lambda: build_2d(), 1), (lambda: build_2d(), 2), (lambda: build_3d(7, 7, 3, 2.0), 3),
                        (lambda: build_3d_cone(nx=9, ny=9, nz=1, layers=4), 4)):
        s = maker()
        s.rO = s.pos.copy()
        s.pos = perturbed(s, 0.04, 60 + seed)
        s.seed, s.x_slider = 500 + seed, 0.1 * seed
        g = oracle_mod.OracleSystem(s).compute()
        s.bias_on, s.m_b, s.dv_max = 1, 2, 0.5
        s.g_lo, s.g_hi = g["g"] - 3.0, g["g"] + 3.0
        out.append(s)
    out[0].thermostat, out[0].nhc_len, out[0].nhc_tau = 1, 3, 0.5
    k = oracle_mod.OracleSystem(out[1]).compute()
    out[1].bias_var1, out[1].bias_var2 = 1, 2
    out[1].g_lo, out[1].g_hi = k["kappa"] - 50.0, k["kappa"] + 50.0
    out[1].b2_lo, out[1].b2_hi = k["d"] + 1.0, k["d"] - 0.1
    return out


def min_image(spec, d):
    for k in range(spec.dim):
        if spec.periodic[k]:
            d[k] -= spec.box[k] * np.round(d[k] / spec.box[k])
    return d


@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_every_shape_follows_the_oracle(hd, oracle_mod, shape):
    specs = kinds(oracle_mod)
    ctx = hd.make_context(specs, precision=hd.HD_FP64, init_velocities=True)
    ctx.set_schedule(dict(SHAPES[shape], ms_per_step=0.0))
    ctx.step(20)
    for k, s in enumerate(specs):
        o = oracle_mod.OracleSystem(s)
        o.init_velocities()
        o.step(20)
        d = min_image(s, ctx.positions(k) - o.positions())
        assert float(np.abs(d).max()) < 1e-10, k
        assert ctx.scalars(k)["t_hyper"] == pytest.approx(o.scalars()["t_hyper"], rel=1e-12), k


def test_autotune_keeps_state(hd, oracle_mod):
    specs = kinds(oracle_mod)
    ctx = hd.make_context(specs, precision=hd.HD_FP32C, init_velocities=True)
    ctx.step(20)
    before = [(ctx.positions(k), ctx.velocities(k), ctx.scalars(k)["t_hyper"], ctx.scalars(k)["e_nhc"])
              for k in range(len(specs))]
    chosen, trials = ctx.autotune(min_ms=2.0, max_steps=256)
    assert len(trials) > 0 and chosen["ms_per_step"] > 0
    for k in range(len(specs)):
        np.testing.assert_array_equal(ctx.positions(k), before[k][0])
        np.testing.assert_array_equal(ctx.velocities(k), before[k][1])
        assert ctx.scalars(k)["t_hyper"] == before[k][2]
        assert ctx.scalars(k)["e_nhc"] == before[k][3]
    ctx.step(20)
    assert all(ctx.scalars(k)["flags"] == 0 for k in range(len(specs)))
