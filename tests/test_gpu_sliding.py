"""The parallel slider-position algorithm (paper_0909_5215_amd.sliding) over
the GPU path: cycles of S positions, the transition check, and the
redistribution that seeds the next cycle from the latest transitioning
position (or from the last position when none had a transition)."""
import numpy as np
import pytest

from hd_inputs import build_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_0909_5215_amd import hd as _hd
    _hd.load()
    return _hd


def batch(S, seed0=500):
    specs = []
    for k in range(S):
        s = build_2d()
        s.seed = seed0 + k            # independent noise for each copy
        s.bias_on, s.m_b, s.dv_max, s.g_lo, s.g_hi = 1, 2, 0.5, -1.0, 1.0
        specs.append(s)
    return specs


def test_cycle_without_transition_advances_by_S(hd):
    from paper_0909_5215_amd.sliding import ParallelSliding
    S = 3
    ctx = hd.make_context(batch(S), precision=hd.HD_FP64)
    ps = ParallelSliding(ctx, x0=0.0, dx=0.01, dtau=1.0, threshold=0.5, chunk=50, check_every=4)
    ps.start(0)
    for j in range(S):
        assert ctx.scalars(j)["x_slider"] == pytest.approx(0.01 * j)
    r = ps.run_cycle()
    assert r.k_star == -1 and not any(r.transitions)
    assert r.next_base == S
    assert all(h >= 1.0 for h in r.hyper_time) and all(st > 0 for st in r.steps)
    seed_x = None
    ps.advance(r)
    for j in range(S):
        x = ctx.positions(j)
        if seed_x is None:
            seed_x = x
        np.testing.assert_array_equal(x, seed_x)      # every system holds the last position's state
        assert ctx.scalars(j)["x_slider"] == pytest.approx(0.01 * (S + j))


def test_latest_transition_seeds_the_next_cycle(hd):
    from paper_0909_5215_amd.sliding import ParallelSliding
    S = 4
    ctx = hd.make_context(batch(S, 600), precision=hd.HD_FP64)
    ps = ParallelSliding(ctx, x0=0.0, dx=0.01, dtau=50.0, threshold=0.5, chunk=50, check_every=2)
    ps.start(0)
    # positions 1 and 2 see their basin move by a lattice spacing (as after a
    # slip of the tip): both read as transitions, the latest (2) seeds
    a = float(2.0 ** (1.0 / 6.0))
    tip = build_2d().type == 1
    for j in (1, 2):
        spec = build_2d()
        rO = ctx.positions(j).copy()
        rO[0, tip] = (rO[0, tip] + a) % spec.box[0]
        ctx.set_reference(j, rO)
    r = ps.run_cycle()
    assert r.transitions[1] and r.transitions[2]
    assert not r.transitions[0] and not r.transitions[3]
    assert r.k_star == 2 and r.next_base == 2
    ps.advance(r)
    x2 = ctx.positions(0)
    for j in range(S):
        np.testing.assert_array_equal(ctx.positions(j), x2)
        assert ctx.scalars(j)["x_slider"] == pytest.approx(0.01 * (2 + j))
    # the new cycle's references are the minima at the new slider positions:
    # no transition reads from them
    _, d, _ = ctx.quench(range(S), ftol=1e-6)
    assert float(np.max(d)) < 1e-4



def test_cycle_detects_a_spontaneous_slip(hd):
    """No reference is moved: the spring pulls the tip, and at the two
    strongest slider positions (lateral force near 10 eps/sigma) the tip
    slips by a lattice spacing during plain MD at kT = 0.1 (at x_S = 10
    no slip comes within the cycle).  The check quench reads the slip as a
    transition (a displacement of one spacing, two if it slipped twice
    between checks), and the latest slipping position seeds the next
    cycle."""
    from paper_0909_5215_amd.sliding import ParallelSliding
    S = 4
    specs = []
    for k in range(S):
        s = build_2d()
        s.seed = 700 + k
        specs.append(s)
    ctx = hd.make_context(specs, precision=hd.HD_FP64)
    dt = specs[0].dt
    ps = ParallelSliding(ctx, x0=10.0, dx=0.5, dtau=8000 * dt, threshold=0.5, chunk=500, check_every=2)
    ps.start(0)
    r = ps.run_cycle()
    a = float(2.0 ** (1.0 / 6.0))
    assert not r.transitions[0]
    assert r.transitions[2] or r.transitions[3]
    assert r.k_star >= 2 and r.next_base == r.k_star
    for j in range(S):
        if r.transitions[j]:
            assert 0.8 * a < r.max_disp[j] < 2.5 * a
            assert r.steps[j] < 8000
    ps.advance(r)
    for j in range(S):
        assert ctx.scalars(j)["x_slider"] == pytest.approx(10.0 + 0.5 * (r.k_star + j))


def test_argument_errors(hd):
    from paper_0909_5215_amd.sliding import ParallelSliding
    ctx = hd.make_context(batch(2), precision=hd.HD_FP64)
    with pytest.raises(ValueError):
        ParallelSliding(ctx, 0.0, 0.01, dtau=0.0)
