"""Pins of the seeded input generators (CPU): the SplitMix64 stream against
the published generator's first outputs, the native (C/OpenMP) fills
against the pure-numpy definitions, and the sizes of the batched workload's
256 plans."""
import os

import numpy as np
import pytest

import workloads as W
from workloads import gen as G

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_splitmix64_seed0():
    vals = []
    for line in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            vals.append(int(line, 16))
    return np.array(vals, np.uint64)


def pm1_numpy(seed, start, count):
    z = G.splitmix64_numpy(seed, start, count)
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def test_splitmix64_matches_published_outputs():
    want = golden_splitmix64_seed0()
    assert want.size == 3
    assert np.array_equal(G.splitmix64_numpy(0, 0, 3), want)
    assert np.array_equal(W.splitmix64(0, 0, 3), want)
    # output i of a stream started at i0 is output i0 + i of the stream
    assert np.array_equal(G.splitmix64_numpy(0, 1, 2), want[1:])


def test_native_fill_is_built():
    G.build_native()
    assert W.native_available()


@pytest.mark.parametrize("seed,start,count", [(0, 0, 1000), (2309, 123_456_789, 5000), (7337, 0, 300_001),
                                              (2 ** 64 - 1, 2 ** 40, 777)])
def test_native_streams_equal_numpy(seed, start, count):
    assert W.native_available()
    assert np.array_equal(W.splitmix64(seed, start, count), G.splitmix64_numpy(seed, start, count))
    ref = pm1_numpy(seed, start, count)
    got = W.uniform_pm1(seed, count, start)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    assert got.min() >= -1.0 and got.max() < 1.0
    # FP32 values: the FP64 values rounded to nearest even
    got32 = W.uniform_pm1_f32(seed, count, start)
    assert np.array_equal(got32.view(np.uint32), ref.astype(np.float32).view(np.uint32))


def test_random_rows_native_equals_numpy_small():
    assert W.native_available()
    rp, cols = W.random_rows(1 << 14, 32, 16, 2309)
    assert np.array_equal(rp, np.arange((1 << 14) + 1, dtype=np.int64) * 32)
    assert np.array_equal(cols, G.random_rows_numpy_cols(1 << 14, 32, 16, 2309))


def test_random_rows_full_size_slices():
    """Slices of the 2^22 x 32 matrix (4096 ranks, seed 2309) against the
    definition, computed from the stream directly."""
    assert W.native_available()
    nrows, k, R, seed = 1 << 22, 32, 4096, 2309
    blk = nrows // R
    _, cols = W.random_rows(nrows, k, R, seed)
    assert cols.size == nrows * k
    for e0 in (0, 31 * 1_000_003, nrows * k - 4096, 1511 * blk * k):
        z = G.splitmix64_numpy(seed, e0, 4096)
        e = np.arange(e0, e0 + 4096, dtype=np.int64)
        glob = (z >> np.uint64(40)) < np.uint64(5033164)
        want = np.where(glob, (z & np.uint64(nrows - 1)).astype(np.int64),
                        (e // k // blk) * blk + (z & np.uint64(blk - 1)).astype(np.int64))
        assert np.array_equal(cols[e0:e0 + 4096], want), e0
    # about 30 % of the entries are global: threshold floor(0.3 * 2^24)
    assert G.GLOBAL_THRESHOLD_24 == 5033164 == int(0.3 * 2 ** 24)
    frac = np.mean((cols[: 1 << 20] // blk) != (np.arange(1 << 20) // k // blk))
    assert 0.29 < frac < 0.31


def test_batched_plan_sizes_pins():
    h, k = W.batched_plan_sizes()
    assert h.size == k.size == 256
    assert int(h.sum()) == 34_696_856
    assert int(h.min()) == 1048 and int(h.max()) == 970_052
    assert int(k.min()) == 1 and int(k.max()) == 3929
    assert int(np.median(k)) == 55
    assert np.all(k <= h)
