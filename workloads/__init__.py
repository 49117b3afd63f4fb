"""Seeded synthetic inputs for the two-electron Hall-HOM propagator.

This package only builds *inputs*: grid/box/time-step settings, the external
potential table V(x, y), the two single-particle edge packets psi_a, psi_b and
the top/bottom region weight table.  It holds none of the propagation
arithmetic; both the FP64 oracle and the HIP library consume what it returns.
"""
from .presets import Workload, preset, PRESETS, mid_sweep  # noqa: F401
