"""Seeded synthetic shot gathers shared by the tests, the benchmark and smoke().

This package holds no arithmetic of the EMD method: it only builds signed
seismograms (Pcal, Pobs) and their grid spacings.  Both the HIP path and the CPU
oracle consume what it produces; neither is imported here.
"""
from .gathers import (  # noqa: F401
    Gather,
    ricker,
    hyperbolic_gather,
    config1_pairs,
    config2_gather,
    config3_batch,
    config4_batch,
    config5_batch,
    random_small_pair,
    blob_pair,
    pack_batch,
)
