"""Bookkeeping of the parallel slider-position algorithm on the CPU, against
a scripted stand-in for the GPU context: which positions finish when, the
latest transitioning position k*, the next cycle's base and its seed state."""
import pytest

from paper_0909_5215_amd.sliding import ParallelSliding


class FakeContext:
    """S systems whose boosted clocks advance at given rates per step and
    whose quench displacement jumps above 1 at a given step (a transition)."""

    def __init__(self, rates, jump_at):
        self.S = len(rates)
        self.rates, self.jump_at = rates, jump_at
        self.step_n = [0] * self.S
        self.th = [0.0] * self.S
        self.slider = [0.0] * self.S
        self.states = [f"s{j}" for j in range(self.S)]
        self.quenched = []

    def num_systems(self):
        return self.S

    def set_state(self, j, blob):
        self.states[j] = blob

    def get_state(self, j):
        return f"{self.states[j]}@{self.step_n[j]}"

    def set_slider(self, j, x):
        self.slider[j] = x

    def step(self, n):
        for j in range(self.S):
            self.step_n[j] += n
            self.th[j] += n * self.rates[j]

    def scalars(self, j):
        return {"t_hyper": self.th[j], "step": self.step_n[j], "f_lat": 0.1 * j, "x_slider": self.slider[j]}

    def scalars_batch(self, first=0, count=None):
        count = self.S - first if count is None else count
        return [self.scalars(j) for j in range(first, first + count)]

    def quench(self, systems, ftol=1e-6, max_iters=1000, set_reference=False):
        systems = list(systems)
        self.quenched.append((systems, set_reference))
        d = [2.0 if self.jump_at[j] is not None and self.step_n[j] >= self.jump_at[j] else 0.01 for j in systems]
        return [1] * len(systems), d, [None] * len(systems)


def run(rates, jump_at, **kw):
    ctx = FakeContext(rates, jump_at)
    ps = ParallelSliding(ctx, x0=1.0, dx=0.5, dtau=10.0, chunk=10, check_every=3, **kw)
    ps.start(4)
    return ctx, ps, ps.run_cycle()


def test_positions_finish_at_their_own_boosted_interval():
    ctx, ps, r = run([1.0, 0.5, 0.25], [None, None, None])
    assert r.transitions == [False, False, False] and r.k_star == -1
    assert r.steps == [10, 20, 40] and r.hyper_time == [10.0, 10.0, 10.0]
    assert r.next_base == 4 + 3
    assert ps.seed_state == "s2@40"                  # the last position seeds
    assert ctx.slider == [1.0 + 0.5 * 4, 1.0 + 0.5 * 5, 1.0 + 0.5 * 6]
    ps.advance(r)
    assert ctx.states == ["s2@40"] * 3
    assert ctx.slider == [1.0 + 0.5 * 7, 1.0 + 0.5 * 8, 1.0 + 0.5 * 9]
    assert ctx.quenched[-1] == ([0, 1, 2], True)     # new references


def test_latest_transition_is_k_star():
    # position 0 jumps early, position 2 later, position 3 never; position 1
    # reaches its interval first
    ctx, ps, r = run([0.01, 1.0, 0.01, 0.01], [20, None, 50, None])
    assert r.transitions == [True, False, True, False]
    assert r.k_star == 2 and r.next_base == 4 + 2
    assert ps.seed_state == "s2@60"                  # found at the check after step 50
    assert r.steps[0] == 30 and r.steps[1] == 10


def test_runs_end_at_the_chunk_cap():
    ctx, ps, r = run([0.0, 0.0], [None, None], max_chunks=5)
    assert r.transitions == [False, False] and r.steps == [50, 50]
    assert r.next_base == 4 + 2


def test_arguments():
    with pytest.raises(ValueError):
        ParallelSliding(FakeContext([1.0], [None]), 0.0, 0.1, dtau=-1.0)
