"""The parallel slider-position algorithm of §2.3 (stepped sliding with S
slider positions simulated at once), driven from the host over the C ABI.

A cycle simulates S consecutive slider positions x0 + (base + j) dx,
j = 0 .. S-1, one system each, all started from the same configuration (the
frontier).  Each system is first relaxed to its basin minimum at its own
slider position (GPU FIRE), which becomes its r_O -- the reference the bias
of eq. 7 and eq. 13-14 measures from -- and then runs biased MD until its
boosted clock has advanced by dtau (the shortened interval of eq. 8), checked
at chunk boundaries.  At every check, and when a system reaches dtau, its
minimum is compared with r_O: a largest atom displacement above `threshold`
is a transition, which ends that position's run.

When the cycle ends, the latest position k* that saw a transition seeds the
next cycle: its state after the transition is copied into every system and
the positions become base + k*, ..., base + k* + S - 1; results of the
positions after k* are discarded.  Without a transition the last position
seeds base + S, ...  (the dice argument of §2.3: transitions at different
fixed slider positions are independent, so they may be tried at once).

Every system needs its own thermostat seed, so that the copies of a seed
state follow independent noise.
"""
import time
from dataclasses import dataclass
from typing import List, Optional


@dataclass
class Cycle:
    base: int                 # slider index of position 0
    transitions: List[bool]   # per position: a transition before its interval ended
    steps: List[int]          # MD steps each position ran until it finished
    hyper_time: List[float]   # boosted time each position accumulated
    f_lat: List[float]        # lateral force on the tip when it finished
    max_disp: List[float]     # largest displacement from r_O at the last check
    k_star: int               # latest transitioning position, or -1
    next_base: int            # slider index of the next cycle's position 0


class ParallelSliding:
    """Cycles of the parallel slider-position algorithm over the systems of a
    finalized context (system j = position j of a cycle)."""

    def __init__(self, ctx, x0: float, dx: float, dtau: float, threshold: float = 0.5,
                 ftol: float = 1e-6, max_quench: int = 20000, chunk: int = 100, check_every: int = 10,
                 max_chunks: int = 10000, check_ftol: float = 1e-4):
        """ftol: force tolerance of the quench that sets r_O; check_ftol: of
        the transition checks, which only compare a minimum's displacement
        with `threshold` (a residual force f moves a minimum by about f/k, k
        the stiffest curvature, ~57 here: far below any threshold)."""
        if not (dtau > 0 and threshold > 0 and chunk > 0 and check_every > 0 and max_chunks > 0
                and ftol > 0 and check_ftol > 0):
            raise ValueError("dtau, threshold, tolerances, chunk, check_every and max_chunks must be positive")
        self.ctx = ctx
        self.S = ctx.num_systems()
        self.x0, self.dx, self.dtau = float(x0), float(dx), float(dtau)
        self.threshold, self.ftol, self.max_quench = float(threshold), float(ftol), int(max_quench)
        self.check_ftol = float(check_ftol)
        self.quench_seconds = 0.0      # wall time spent in transition checks
        self.chunk, self.check_every, self.max_chunks = int(chunk), int(check_every), int(max_chunks)
        self.base = 0
        self.seed_state: Optional[bytes] = None
        self._t0 = [0.0] * self.S
        self._step0 = [0] * self.S

    def slider(self, index: int) -> float:
        return self.x0 + index * self.dx

    def start(self, base: int, seed_state: Optional[bytes] = None):
        """Place a cycle: copy seed_state (if given) into every system, move
        system j's slider to position base + j, relax each system to its basin
        minimum there and make it r_O."""
        ctx = self.ctx
        for j in range(self.S):
            if seed_state is not None:
                ctx.set_state(j, seed_state)
            ctx.set_slider(j, self.slider(base + j))
        ctx.quench(range(self.S), ftol=self.ftol, max_iters=self.max_quench, set_reference=True)
        self.base = base
        sc = ctx.scalars_batch(0, self.S)
        self._t0 = [s["t_hyper"] for s in sc]
        self._step0 = [s["step"] for s in sc]

    def run_cycle(self) -> Cycle:
        """Biased MD of every position until each has a transition or has
        advanced its boosted clock by dtau."""
        ctx, S = self.ctx, self.S
        done = [False] * S
        trans = [False] * S
        steps, hyper, flat, disp = [0] * S, [0.0] * S, [0.0] * S, [0.0] * S
        states: List[Optional[bytes]] = [None] * S
        for c in range(self.max_chunks):
            ctx.step(self.chunk)
            sc = ctx.scalars_batch(0, S)
            reached = [not done[j] and sc[j]["t_hyper"] - self._t0[j] >= self.dtau for j in range(S)]
            last = c == self.max_chunks - 1
            if not ((c + 1) % self.check_every == 0 or any(reached) or last):
                continue
            live = [j for j in range(S) if not done[j]]
            t0 = time.perf_counter()
            _, d, _ = ctx.quench(live, ftol=self.check_ftol, max_iters=self.max_quench)
            self.quench_seconds += time.perf_counter() - t0
            for j, dj in zip(live, d):
                disp[j] = float(dj)
                if dj > self.threshold or reached[j] or last:
                    done[j] = True
                    trans[j] = bool(dj > self.threshold)
                    states[j] = ctx.get_state(j)
                    steps[j] = sc[j]["step"] - self._step0[j]
                    hyper[j] = sc[j]["t_hyper"] - self._t0[j]
                    flat[j] = sc[j]["f_lat"]
            if all(done):
                break
        k_star = max((j for j in range(S) if trans[j]), default=-1)
        seed = k_star if k_star >= 0 else S - 1
        self.seed_state = states[seed]
        next_base = self.base + (k_star if k_star >= 0 else S)
        return Cycle(self.base, trans, steps, hyper, flat, disp, k_star, next_base)

    def advance(self, r: Cycle):
        """Start the cycle that r's outcome seeds."""
        self.start(r.next_base, self.seed_state)
