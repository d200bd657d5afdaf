"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package only *generates inputs*: sparse-matrix structure (CSR column
indices), row splits, dense vectors and the synthetic exchange lists of the
batched workload.  It contains none of the method's arithmetic (no halo
discovery, no send-list transpose, no dedup, no pack/unpack, no sums).
"""
from .gen import *  # noqa: F401,F403
