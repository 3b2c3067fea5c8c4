"""Seeded synthetic inputs (wavenumber fields, sources, random vectors).

This package holds no arithmetic of the solver itself: it only draws the inputs
that both the CPU oracle and the GPU library are run on.
"""
from .workloads import *  # noqa: F401,F403
