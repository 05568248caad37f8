"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only builds input fields (phase maps, material fields, load
schedules, random fields).  It contains none of the method's arithmetic, so
that the CPU oracle and the HIP path stay independent of each other.
"""
from .microstructure import *  # noqa: F401,F403
from .workloads import *  # noqa: F401,F403
