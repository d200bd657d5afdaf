"""ctypes loader of the multithreaded C data-movement loops (``cpu_move.c``),
the all-cores CPU baseline.

TEST INFRASTRUCTURE (see the package docstring).  ``build_cpu()`` compiles
the library with gcc and OpenMP; the loaders below raise if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_move.c")
LIB = os.path.join(HERE, "libcpu_move.so")

_lib = None


def build_cpu() -> str:
    """Compiles cpu_move.c (IEEE arithmetic: no fast-math, no contraction)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-o", tmp, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise ImportError(f"{LIB} is missing: run oracle.cpu.build_cpu()")
    lib = C.CDLL(LIB)
    vp, i64 = C.c_void_p, C.c_int64
    lib.oc_threads.restype = C.c_int
    lib.oc_threads.argtypes = []
    lib.oc_gather.restype = None
    lib.oc_gather.argtypes = [vp, vp, i64, i64, vp]
    for name in ("oc_transpose_sum_f64", "oc_transpose_sum_f32"):
        f = getattr(lib, name)
        f.restype = None
        f.argtypes = [vp, vp, vp, i64, i64, vp]
    _lib = lib
    return lib


def threads() -> int:
    """Threads the OpenMP loops use (OMP_NUM_THREADS, else the host's cores)."""
    return int(load().oc_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def gather(src: np.ndarray, idx, out: np.ndarray | None = None) -> np.ndarray:
    """out[k] = src[idx[k]] (idx None: the identity copy of len(out) rows)."""
    src = np.ascontiguousarray(src)
    if idx is not None:
        idx = np.ascontiguousarray(np.asarray(idx, np.int32))
        n = idx.size
    else:
        n = src.shape[0] if out is None else out.shape[0]
    if out is None:
        out = np.empty((n,) + src.shape[1:], src.dtype)
    rb = src.dtype.itemsize * int(np.prod(src.shape[1:], dtype=np.int64))
    load().oc_gather(_ptr(src), _ptr(idx), n, rb, _ptr(out))
    return out


def transpose_sum(g: np.ndarray, ptr, perm, out: np.ndarray | None = None) -> np.ndarray:
    """gx[i] = sum of g[perm[e]] over e in [ptr[i], ptr[i+1]), in order."""
    g = np.ascontiguousarray(g)
    ptr = np.ascontiguousarray(np.asarray(ptr, np.int32))
    perm = np.ascontiguousarray(np.asarray(perm, np.int32))
    n = ptr.size - 1
    ncols = int(np.prod(g.shape[1:], dtype=np.int64))
    if out is None:
        out = np.empty((n,) + g.shape[1:], g.dtype)
    fn = {np.dtype(np.float64): load().oc_transpose_sum_f64, np.dtype(np.float32): load().oc_transpose_sum_f32}
    fn[g.dtype](_ptr(g), _ptr(ptr), _ptr(perm), n, ncols, _ptr(out))
    return out
