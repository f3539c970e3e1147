"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package only draws numbers and lays out region boxes.  It holds none of
the multigrid arithmetic: no operators, transfers, smoothers or solvers.
"""
from .workloads import *  # noqa: F401,F403
