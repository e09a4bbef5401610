"""Seeded synthetic model inputs shared by the oracle tests, the GPU tests and
the benchmark.  Pure lattice geometry and parameter draws: no physics."""
from .models import *  # noqa: F401,F403
