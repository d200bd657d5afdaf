import functools
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: large CPU-side workload (tens of seconds)")


@functools.lru_cache(maxsize=None)
def cached_grid2d():
    from workloads import grid2d_5pt, equal_row_starts
    rp, cols = grid2d_5pt(512, 512)
    return equal_row_starts(512 * 512, 16), rp, cols


@functools.lru_cache(maxsize=None)
def cached_grid3d():
    from workloads import grid3d_27pt, equal_row_starts
    rp, cols = grid3d_27pt(128, 16)
    return equal_row_starts(128 ** 3, 512), rp, cols


@functools.lru_cache(maxsize=None)
def cached_random_rows():
    from workloads import random_rows, equal_row_starts
    rp, cols = random_rows(1 << 22, 32, 4096, 2309)
    return equal_row_starts(1 << 22, 4096), rp, cols
