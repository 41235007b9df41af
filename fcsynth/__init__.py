"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds none of the fast-convolution method's arithmetic: no
transforms of the FC chain, no block schedules, no CP rule. Callers pass the
per-symbol low-rate CP lengths in. It only draws random QAM grids, builds
standard CP-OFDM waveforms from them, adds noise, and describes the
benchmark workloads as plain parameter lists.
"""
from .signals import qam, qam_grid, cp_ofdm, cp_ofdm_highrate, awgn  # noqa: F401
from . import workloads  # noqa: F401
