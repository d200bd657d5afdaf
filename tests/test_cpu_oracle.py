"""Pins of the multithreaded C oracle loops (oracle/cpu_move.c, the all-cores
CPU baseline): brute force on tiny inputs written as plain Python loops,
index-encoded values, signed zeros, order-sensitive sums and equality with
the numpy oracle on random plans."""
import numpy as np
import pytest

from oracle import cpu as OC
from oracle import move as OM
from oracle import plan as OP


@pytest.fixture(scope="module", autouse=True)
def built():
    OC.build_cpu()
    OC.load()


def test_gather_encodes_every_index():
    rng = np.random.default_rng(1)
    x = np.arange(50 * 3, dtype=np.float64).reshape(50, 3)   # row i holds 3i, 3i+1, 3i+2
    idx = rng.integers(0, 50, 777).astype(np.int32)
    got = OC.gather(x, idx)
    for k in range(idx.size):
        assert list(got[k]) == [3 * idx[k], 3 * idx[k] + 1, 3 * idx[k] + 2]
    # identity copy, FP32 rows of one value
    y = np.arange(1000, dtype=np.float32).reshape(1000, 1)
    assert np.array_equal(OC.gather(y, None), y)
    # empty list
    assert OC.gather(x, np.zeros(0, np.int32)).shape == (0, 3)


def _brute_sum(g, ptr, perm):
    out = np.zeros((len(ptr) - 1,) + g.shape[1:], g.dtype)
    for i in range(len(ptr) - 1):
        for c in range(g.shape[1]):
            acc = None
            for e in range(ptr[i], ptr[i + 1]):
                v = g[perm[e], c]
                acc = v if acc is None else g.dtype.type(acc + v)
            out[i, c] = g.dtype.type(0) if acc is None else acc
    return out


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_transpose_sum_brute_force(dt):
    rng = np.random.default_rng(2)
    idx = rng.integers(0, 40, 300).astype(np.int32)
    ptr, perm = OP.transpose_csr(idx, 45)           # rows 40..44 are empty
    g = rng.standard_normal((300, 4)).astype(dt)
    want = _brute_sum(g, ptr, perm)
    got = OC.transpose_sum(g, ptr, perm)
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))
    assert np.array_equal(got.view(np.uint8), OM.pack_transpose(g, ptr, perm).view(np.uint8))


def test_transpose_sum_order_and_zeros():
    # (1e16 + 1) - 1e16 = 0 in order, but (1e16 - 1e16) + 1 = 1 with the last two swapped
    g = np.array([[1e16], [1.0], [-1e16], [-0.0], [-0.0], [0.0], [-0.0], [-0.0]])
    ptr = np.array([0, 3, 4, 6, 8, 8], np.int32)
    perm = np.arange(8, dtype=np.int32)
    got = OC.transpose_sum(g, ptr, perm)[:, 0]
    assert got[0] == 0.0
    assert got[1] == 0.0 and np.signbit(got[1])          # a lone -0.0 survives
    assert got[2] == 0.0 and not np.signbit(got[2])      # -0.0 + 0.0 = +0.0
    assert got[3] == 0.0 and np.signbit(got[3])          # -0.0 + -0.0 = -0.0
    assert got[4] == 0.0 and not np.signbit(got[4])      # empty row: +0.0
    perm_rev = np.array([0, 2, 1, 3, 4, 5, 6, 7], np.int32)
    assert OC.transpose_sum(g, ptr, perm_rev)[0, 0] == 1.0


def test_transpose_sum_integer_closed_form():
    # every slot carries its row's id: the sum is count(i) * i exactly
    rng = np.random.default_rng(3)
    n = 2000
    idx = rng.integers(0, n, 20_000).astype(np.int32)
    ptr, perm = OP.transpose_csr(idx, n)
    g = idx.astype(np.float64).reshape(-1, 1)
    got = OC.transpose_sum(g, ptr, perm)[:, 0]
    assert np.array_equal(got, np.bincount(idx, minlength=n) * np.arange(n, dtype=np.float64))
