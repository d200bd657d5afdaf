"""Helpers shared by the GPU parity tests (marshalling only)."""
import sys

import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import plan as OP


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def variant_id(v: str) -> int:
    return {"plain": P.HX_PLAIN, "locality": P.HX_LOCALITY_2STEP, "locality3": P.HX_LOCALITY_3STEP}[v]


def gpu_plan(rs, rp, cols, ppn, variant, node_map="block"):
    return P.hx_plan_from_csr(len(rs) - 1, rs, ppn, variant_id(variant), dev(np.asarray(rp, np.int64)),
                              dev(np.asarray(cols, np.int32)), node_map=node_map)


def plan_rank(plan, r) -> dict:
    return {f: P.hx_plan_field(plan, r, f) for f in P.FIELDS}


def assert_plan_equal(got: dict, want: dict, ctx=""):
    for k in OP.PLAN_KEYS:
        g = np.asarray(got[k], np.int64)
        w = np.asarray(want[k], np.int64)
        if g.shape != w.shape or not np.array_equal(g, w):
            raise AssertionError(f"{ctx} field {k}: got {g[:12]} ({g.size}) want {w[:12]} ({w.size})")


def bits_equal(a, b) -> bool:
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.shape == b.shape and a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))
