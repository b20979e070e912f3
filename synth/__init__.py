"""Seeded synthetic inputs shared by the oracle, the GPU library tests and the bench.

This package only draws data (SSP spectra, filters, line tables, dust tables,
parameter batches, request streams).  It contains none of the forward model's
arithmetic: weights, contraction, attenuation, redshifting, projection and the
likelihood live separately in the oracle and in the HIP library.
"""
from .workloads import *  # noqa: F401,F403
