"""Seeded input generators (matrix structure, row splits, vectors, synthetic lists).

Every random number comes from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): output ``i`` (0-based)
of the stream seeded with ``s`` is ``mix(s + (i + 1) * GAMMA)`` with the
published golden-gamma constant and the variant-13 mixer (shifts 30/27/31).

Workloads (sizes as used by the benchmark and the parity tests):

* ``grid2d_5pt``     2D 5-point Laplacian structure, natural ordering
                     ``i = y * nx + x`` (x fastest).
* ``grid3d_27pt``    3D 27-point stencil on a cube split into equal cubic
                     blocks; rows are numbered block by block so that each
                     rank owns a contiguous row range.
* ``random_rows``    random sparse rows: each entry independently "global"
                     with probability ~0.3 (uniform over all columns), else
                     uniform inside the row's own rank block.
* ``batched_plans``  independent synthetic exchange lists with log-uniform
                     halo sizes and neighbor counts (the batched workload).

Nothing here computes a halo, a send list, a dedup set or moves any vector
data: those belong to the method and are implemented separately by the oracle
and by the HIP library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "GAMMA", "splitmix64", "uniform53", "uniform_pm1", "uniform_pm1_f32",
    "equal_row_starts", "grid2d_5pt", "grid3d_27pt", "random_rows",
    "random_small_csr", "batched_plan_sizes", "batched_plan",
    "GLOBAL_THRESHOLD_24", "native_available", "build_native",
]

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 20

# An entry of the random-rows workload is "global" iff (z >> 40) < floor(0.3 * 2^24).
GLOBAL_THRESHOLD_24 = 5033164


_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsm64.so")
_native = None


def build_native() -> str:
    """Compile the multithreaded SplitMix64 fill (sm64.c) next to this file."""
    import subprocess
    src = os.path.join(_HERE, "sm64.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


def _load_native():
    global _native
    if _native is None:
        if os.path.exists(_SO) and not os.environ.get("HX_GEN_NUMPY"):
            lib = ctypes.CDLL(_SO)
            for name, ptr in (("sm64_fill_u64", ctypes.c_uint64), ("sm64_fill_pm1_f64", ctypes.c_double),
                              ("sm64_fill_pm1_f32", ctypes.c_float)):
                fn = getattr(lib, name)
                fn.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ptr)]
                fn.restype = None
            lib.gen_random_rows_cols.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                                 ctypes.c_int64, ctypes.c_uint64,
                                                 ctypes.POINTER(ctypes.c_int32)]
            lib.gen_random_rows_cols.restype = None
            _native = lib
        else:
            _native = False
    return _native or None


def native_available() -> bool:
    return _load_native() is not None


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream for ``seed`` (uint64)."""
    lib = _load_native()
    if lib is not None:
        out = np.empty(int(count), np.uint64)
        lib.sm64_fill_u64(int(seed) & 0xFFFFFFFFFFFFFFFF, int(start), int(count),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        return out
    return splitmix64_numpy(seed, start, count)


def splitmix64_numpy(seed: int, start: int, count: int) -> np.ndarray:
    """Pure-numpy SplitMix64 (the definition; the native fill must match it)."""
    count = int(count)
    out = np.empty(count, np.uint64)
    tmp = np.empty(min(count, _CHUNK), np.uint64)
    s = np.uint64(int(seed) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for lo in range(0, count, _CHUNK):
            hi = min(count, lo + _CHUNK)
            z = out[lo:hi]
            t = tmp[: hi - lo]
            z[:] = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            z *= GAMMA
            z += s
            np.right_shift(z, np.uint64(30), out=t); z ^= t; z *= _MIX1
            np.right_shift(z, np.uint64(27), out=t); z ^= t; z *= _MIX2
            np.right_shift(z, np.uint64(31), out=t); z ^= t
    return out


def uniform53(seed: int, start: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) with 53 random bits: ``(z >> 11) * 2^-53``."""
    z = splitmix64(seed, start, count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, count: int, start: int = 0) -> np.ndarray:
    """FP64 values in [-1, 1): ``(z >> 11) * 2^-52 - 1`` (exact in FP64)."""
    lib = _load_native()
    if lib is not None:
        out = np.empty(int(count), np.float64)
        lib.sm64_fill_pm1_f64(int(seed) & 0xFFFFFFFFFFFFFFFF, int(start), int(count),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out
    out = np.empty(int(count), np.float64)
    for lo in range(0, int(count), _CHUNK * 8):
        hi = min(int(count), lo + _CHUNK * 8)
        z = splitmix64(seed, start + lo, hi - lo)
        out[lo:hi] = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
    return out


def uniform_pm1_f32(seed: int, count: int, start: int = 0) -> np.ndarray:
    """FP32 values: the FP64 values above rounded to nearest-even."""
    lib = _load_native()
    if lib is not None:
        out = np.empty(int(count), np.float32)
        lib.sm64_fill_pm1_f32(int(seed) & 0xFFFFFFFFFFFFFFFF, int(start), int(count),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        return out
    out = np.empty(int(count), np.float32)
    for lo in range(0, int(count), _CHUNK * 8):
        hi = min(int(count), lo + _CHUNK * 8)
        out[lo:hi] = uniform_pm1(seed, hi - lo, start + lo).astype(np.float32)
    return out


def equal_row_starts(n: int, nranks: int) -> np.ndarray:
    """Contiguous equal row blocks (n must be divisible by nranks)."""
    if n % nranks:
        raise ValueError("n must be divisible by nranks")
    return (np.arange(nranks + 1, dtype=np.int64) * (n // nranks))


def _csr_from_candidates(cand: np.ndarray, valid: np.ndarray):
    counts = valid.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(cand.shape[0] + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols = cand[valid].astype(np.int32)
    return row_ptr, cols


def grid2d_5pt(nx: int = 512, ny: int = 512):
    """CSR structure (row_ptr int64, cols int32) of the 5-point stencil, x fastest."""
    n = nx * ny
    i = np.arange(n, dtype=np.int64)
    x = i % nx
    y = i // nx
    cand = np.stack([i - nx, i - 1, i, i + 1, i + nx], axis=1)
    valid = np.stack([y > 0, x > 0, np.ones(n, bool), x < nx - 1, y < ny - 1], axis=1)
    return _csr_from_candidates(cand, valid)


def grid3d_27pt(g: int = 128, b: int = 16):
    """CSR structure of the 27-point stencil on a g^3 grid cut into (g/b)^3 blocks.

    Block (bx, by, bz) is rank ``bx + nb*by + nb^2*bz`` (nb = g/b); the point with
    in-block offsets (lx, ly, lz) is row ``rank*b^3 + lx + b*(ly + b*lz)``.
    Columns of a row are listed in (dz, dy, dx) lexicographic offset order.
    The row id is separable, ``FX[X] + FY[Y] + FZ[Z]``, which the code uses.
    """
    nb = g // b
    b3 = b * b * b
    n = g * g * g
    ax = np.arange(g, dtype=np.int64)
    FX = (ax // b) * b3 + (ax % b)
    FY = (ax // b) * nb * b3 + (ax % b) * b
    FZ = (ax // b) * nb * nb * b3 + (ax % b) * b * b
    bad = -(1 << 29)

    def padded(F):
        return np.concatenate([[bad], F, [bad]]).astype(np.int32)

    FXp, FYp, FZp = padded(FX), padded(FY), padded(FZ)
    rows = np.arange(n, dtype=np.int64)
    p = rows // b3
    l = rows % b3
    X = ((p % nb) * b + (l % b)).astype(np.int32) + 1
    Y = (((p // nb) % nb) * b + ((l // b) % b)).astype(np.int32) + 1
    Z = ((p // (nb * nb)) * b + (l // (b * b))).astype(np.int32) + 1
    del p, l, rows
    cand = np.empty((27, n), np.int32)
    t = 0
    for dz in (-1, 0, 1):
        cz = FZp[Z + dz]
        for dy in (-1, 0, 1):
            cyz = FYp[Y + dy] + cz
            for dx in (-1, 0, 1):
                np.add(FXp[X + dx], cyz, out=cand[t])
                t += 1
    cand = np.ascontiguousarray(cand.T)
    valid = cand >= 0
    counts = valid.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols = cand.ravel()[valid.ravel()]
    return row_ptr, cols


def random_rows(nrows: int = 1 << 22, nnz_per_row: int = 32, nranks: int = 4096,
                seed: int = 2309):
    """Random rows: entry e = row*k + j draws z = SM64(seed, e).

    The entry is global iff ``(z >> 40) < GLOBAL_THRESHOLD_24``; its column is
    then ``z & (nrows - 1)`` (nrows a power of two), otherwise
    ``blk * floor(row / blk) + (z & (blk - 1))`` with ``blk = nrows / nranks``
    (a power of two).  Columns are kept in draw order; duplicates are allowed.
    """
    blk = nrows // nranks
    assert nrows & (nrows - 1) == 0 and blk & (blk - 1) == 0
    nnz = nrows * nnz_per_row
    cols = np.empty(nnz, np.int32)
    row_ptr = np.arange(nrows + 1, dtype=np.int64) * nnz_per_row
    lib = _load_native()
    if lib is not None:
        lib.gen_random_rows_cols(int(seed), nrows, nnz_per_row, blk, GLOBAL_THRESHOLD_24,
                                 cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        return row_ptr, cols
    return row_ptr, random_rows_numpy_cols(nrows, nnz_per_row, nranks, seed)


def random_rows_numpy_cols(nrows: int, nnz_per_row: int, nranks: int, seed: int) -> np.ndarray:
    """Pure-numpy columns of ``random_rows`` (the definition the native fill must match)."""
    blk = nrows // nranks
    nnz = nrows * nnz_per_row
    cols = np.empty(nnz, np.int32)
    step = _CHUNK * 8
    for lo in range(0, nnz, step):
        hi = min(nnz, lo + step)
        z = splitmix64(seed, lo, hi - lo)
        e = np.arange(lo, hi, dtype=np.int64)
        row = e // nnz_per_row
        glob = (z >> np.uint64(40)) < np.uint64(GLOBAL_THRESHOLD_24)
        gcol = (z & np.uint64(nrows - 1)).astype(np.int64)
        lcol = (row // blk) * blk + (z & np.uint64(blk - 1)).astype(np.int64)
        cols[lo:hi] = np.where(glob, gcol, lcol)
    return cols


def random_small_csr(n: int, nranks: int, max_nnz_row: int, p_far: float, seed: int,
                     uneven: bool = False):
    """Tiny random CSR for brute-force tests.

    Row split: equal blocks, or (``uneven``) random cut points that may leave
    ranks empty.  Each row draws ``1 + (z % max_nnz_row)`` entries; an entry is
    "far" (uniform over all columns) with probability ``p_far``, else within
    +-3 of the row (clipped).  Returns (row_starts, row_ptr, cols).
    """
    ctr = 0

    def draw(cnt):
        nonlocal ctr
        z = splitmix64(seed, ctr, cnt)
        ctr += cnt
        return z

    if uneven:
        cuts = np.sort((draw(nranks - 1) % np.uint64(n + 1)).astype(np.int64))
        row_starts = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    else:
        base = n // nranks
        extra = n % nranks
        sizes = np.array([base + (1 if r < extra else 0) for r in range(nranks)], np.int64)
        row_starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    lens = 1 + (draw(n) % np.uint64(max_nnz_row)).astype(np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    nnz = int(row_ptr[-1])
    row = np.repeat(np.arange(n, dtype=np.int64), lens)
    u = (draw(nnz) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    far = u < p_far
    zc = draw(nnz)
    far_col = (zc % np.uint64(n)).astype(np.int64)
    near_col = np.clip(row + (zc % np.uint64(7)).astype(np.int64) - 3, 0, n - 1)
    cols = np.where(far, far_col, near_col).astype(np.int32)
    return row_starts, row_ptr, cols


# ---------------------------------------------------------------------------
# Batched workload: independent synthetic exchange lists.
# ---------------------------------------------------------------------------

def batched_plan_sizes(nplans: int = 256, seed: int = 3, nranks: int = 4096):
    """Halo size h_b and neighbor count k_b of each plan.

    u, v are 53-bit uniforms SM64(seed, 2b), SM64(seed, 2b+1);
    ``h = floor(10^(3 + 3u))`` (log-uniform in [1e3, 1e6)),
    ``k = min(h, max(1, floor(nranks^v)))`` (log-uniform in [1, nranks)).
    """
    z = splitmix64(seed, 0, 2 * nplans)
    uv = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    u = uv[0::2]
    v = uv[1::2]
    h = np.floor(10.0 ** (3.0 + 3.0 * u)).astype(np.int64)
    k = np.minimum(h, np.maximum(1, np.floor(float(nranks) ** v).astype(np.int64)))
    return h, k


def _distinct_sorted_per_group(sizes: np.ndarray, universe: int, seed: int) -> list:
    """For group i draw ``sizes[i]`` distinct integers uniform in [0, universe), sorted.

    Sparse groups (4*size <= universe) use rejection in draw order; dense groups
    take the first ``size`` entries of a random permutation (argsort of SM64 keys).
    """
    k = len(sizes)
    result = [None] * k
    dense = sizes * 4 > universe
    ctr = 0
    # dense groups
    for i in np.nonzero(dense)[0]:
        keys = splitmix64(seed + 0x100000 + int(i), 0, universe)
        perm = np.argsort(keys, kind="stable")
        result[i] = np.sort(perm[: sizes[i]]).astype(np.int64)
    # sparse groups, vectorised rejection
    idx = np.nonzero(~dense)[0]
    if idx.size:
        sz = sizes[idx].astype(np.int64)
        acc_grp = np.empty(0, np.int64)
        acc_val = np.empty(0, np.int64)
        have = np.zeros(idx.size, np.int64)
        while True:
            need = sz - have
            if not need.any():
                break
            draw = np.where(need > 0, need + need // 2 + 4, 0)
            total = int(draw.sum())
            z = splitmix64(seed, ctr, total)
            ctr += total
            vals = ((z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * universe).astype(np.int64)
            grp = np.repeat(np.arange(idx.size, dtype=np.int64), draw)
            key_new = grp * universe + vals
            key_old = acc_grp * universe + acc_val
            keep = ~np.isin(key_new, key_old)
            key_new = key_new[keep]
            grp = grp[keep]
            vals = vals[keep]
            _, first = np.unique(key_new, return_index=True)
            first = np.sort(first)
            key_new, grp, vals = key_new[first], grp[first], vals[first]
            # rank of each new value within its group, in draw order
            order = np.argsort(grp, kind="stable")
            g_sorted = grp[order]
            starts = np.searchsorted(g_sorted, g_sorted, side="left")
            rank = np.empty_like(order)
            rank[order] = np.arange(order.size) - starts
            take = rank < need[grp]
            acc_grp = np.concatenate([acc_grp, grp[take]])
            acc_val = np.concatenate([acc_val, vals[take]])
            have = np.bincount(acc_grp, minlength=idx.size).astype(np.int64)
        order = np.lexsort((acc_val, acc_grp))
        acc_grp, acc_val = acc_grp[order], acc_val[order]
        bounds = np.searchsorted(acc_grp, np.arange(idx.size + 1))
        for j, i in enumerate(idx):
            result[i] = acc_val[bounds[j]:bounds[j + 1]]
    return result


def batched_plan(b: int, h: int, k: int, nranks: int = 4096):
    """Exchange lists of batched plan ``b`` (its own rank is 0 of ``nranks``).

    * neighbors: the first k of a random permutation of ranks 1..nranks-1, ascending;
    * per-neighbor sizes: 1 + a multinomial split of the remaining h - k entries;
    * send lists mirror the recv sizes: for each neighbor, ``size`` distinct local
      rows uniform in [0, h), ascending (so n_local = h and E = H = h).

    Returns dict(procs, counts, displs, send_idx).  The neighbor's data that
    would arrive (the recv buffer) is an input filled separately.
    """
    keys = splitmix64(10_000 + b, 0, nranks - 1)
    nbrs = np.sort(1 + np.argsort(keys, kind="stable")[:k]).astype(np.int32)
    extra = h - k
    u = uniform53(20_000 + b, 0, extra)
    sizes = 1 + np.bincount(np.minimum((u * k).astype(np.int64), k - 1), minlength=k)
    sizes = sizes.astype(np.int64)
    rows = _distinct_sorted_per_group(sizes, h, 30_000 + b * 0x1000)
    send_idx = np.concatenate(rows).astype(np.int32) if k else np.empty(0, np.int32)
    displs = np.zeros(k, np.int64)
    if k:
        displs[1:] = np.cumsum(sizes)[:-1]
    return dict(procs=nbrs, counts=sizes.astype(np.int32), displs=displs.astype(np.int32),
                send_idx=send_idx)
