"""The C-ABI library loads and exports every entry point of include/hx.h;
host-side argument validation works without a GPU (no compute calls)."""
import os
import re

import numpy as np
import pytest

import paper_2309_07337_amd as P
from paper_2309_07337_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "hx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hx_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTED) == names


def test_version_and_error_strings():
    assert "gfx950" in P.hx_version()
    assert P.hx_error_string(0) == "success"
    assert P.hx_error_string(P.HX_ERR_STATE) == "invalid request state"
    assert P.hx_error_string(12345) == "unknown error"


def test_topology_validation():
    with pytest.raises(P.HXError) as e:
        P.hx_topo_create(0, 4, [1], [2], reorder=1)
    assert e.value.code == P.HX_ERR_UNSUPPORTED
    for bad in ([0], [4], [-1], [1, 1]):
        with pytest.raises(P.HXError) as e:
            P.hx_topo_create(0, 4, bad, [2])
        assert e.value.code == P.HX_ERR_RANGE
    with pytest.raises(P.HXError) as e:
        P.hx_topo_create(5, 4, [1], [2])
    assert e.value.code == P.HX_ERR_ARG
    t = P.hx_topo_create(0, 4, [1, 3], [2], recv_weights=[1, 1], send_weights=[7])
    t.free()
    t.free()


class FakeTensor:
    """Shape/dtype/pointer stand-in: validation fails before any device call."""

    def __init__(self, rows, ncols=1):
        import torch
        self.shape = (rows, ncols)
        self.dtype = torch.float64

    def dim(self):
        return 2

    def data_ptr(self):
        return 4096


@pytest.mark.parametrize("kind", ["displs", "range", "negative"])
def test_init_validation_on_host(kind):
    topo = P.hx_topo_create(1, 4, [0, 2], [0, 2])
    x, halo = FakeTensor(10), FakeTensor(5)
    sc, sd, idx = [2, 3], [0, 2], [0, 1, 2, 3, 4]
    rc, rd = [2, 3], [0, 2]
    if kind == "displs":
        sd = [0, 3]
        code = P.HX_ERR_ARG
    elif kind == "range":
        idx = [0, 1, 2, 3, 10]
        code = P.HX_ERR_RANGE
    else:
        rc = [-1, 6]
        code = P.HX_ERR_ARG
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_alltoallv_init(x, sc, sd, idx, halo, rc, rd, topo)
    assert e.value.code == code


def test_plan_validation_on_host():
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(2, [0, 3, 2], 1, P.HX_PLAIN, [0, 0, 0], None, stream=0)
    assert e.value.code == P.HX_ERR_ARG
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(P.HX_PLAN_MAX_RANKS + 1, np.arange(P.HX_PLAN_MAX_RANKS + 2), 1, P.HX_PLAIN,
                             np.zeros(P.HX_PLAN_MAX_RANKS + 2), None, stream=0)
    assert e.value.code == P.HX_ERR_UNSUPPORTED
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(2, [0, 2, 4], 0, P.HX_LOCALITY_2STEP, [0, 0, 0], None, stream=0)
    assert e.value.code == P.HX_ERR_ARG
    # node map: unknown value, and the 3-step variant (contiguous node rows) under a cyclic map
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(2, [0, 2, 4], 1, P.HX_LOCALITY_2STEP, [0, 0, 0], None, stream=0, node_map=7)
    assert e.value.code == P.HX_ERR_ARG
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(2, [0, 2, 4], 1, P.HX_LOCALITY_3STEP, [0, 0, 0], None, stream=0,
                             node_map="cyclic")
    assert e.value.code == P.HX_ERR_UNSUPPORTED
    lib = P.load()
    rs = np.array([0, 2, 4], np.int64)
    out = __import__("ctypes").c_void_p()
    assert lib.hx_plan_from_halos(2, rs.ctypes.data_as(P._lib.I64P), None, rs.ctypes.data_as(P._lib.I64P), None,
                                  None, __import__("ctypes").byref(out)) == P.HX_ERR_ARG   # null info


def test_product_path_has_no_cpu_fallback(monkeypatch, tmp_path):
    """With the library missing, loading fails loudly instead of falling back."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L.load()


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs one GPU's share: --gpus 2 exits with a JSON error line
    (before touching any GPU)."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_allocator_failure_is_nomem_without_a_gpu():
    """The first allocation of an init call fails in the installed allocator:
    HX_ERR_NOMEM, and nothing is handed to the free callback."""
    import ctypes as C
    from paper_2309_07337_amd import _lib as L
    lib = P.load()
    calls, frees = [], []
    try:
        P.hx_set_allocator(lambda n, s, c: calls.append(n), lambda p, c: frees.append(p))
        topo = P.hx_topo_create(0, 2, [1], [1])
        sc = np.array([2], np.int32)
        si = np.array([0, 3], np.int32)
        out = C.c_void_p()
        rc = lib.hx_neighbor_alltoallv_init(0x1000, 4, sc.ctypes.data_as(L.I32P), None, si.ctypes.data_as(L.I32P),
                                            0x2000, sc.ctypes.data_as(L.I32P), None, P.HX_F64, 1, topo.ptr,
                                            C.byref(out))
        assert rc == P.HX_ERR_NOMEM and not out.value
        assert len(calls) == 1 and not frees
        # exactly one of the two callbacks: an argument error
        assert lib.hx_set_allocator(L._TORCH_ALLOC, L.FREE_FN(0), None) == P.HX_ERR_ARG
    finally:
        L.use_torch_allocator()


def test_collective_locality_init_checks_on_host():
    """The per-rank locality-aware init: a joined request is pending (every
    call on it refuses), a rank cannot join twice, and a completing call
    whose ranks' lists do not match fails before any device work, leaving
    the set over.  A 3-step rank packs from its node's rows (block placement
    only), so its vector has the node's row count."""
    with pytest.raises(P.HXError) as e:
        P.hx_comm_create(2, [0, 3, 6], 1, P.HX_LOCALITY_3STEP, node_map="cyclic", stream=0)
    assert e.value.code == P.HX_ERR_UNSUPPORTED
    comm3 = P.hx_comm_create(2, [0, 3, 6], 2, P.HX_LOCALITY_3STEP, stream=0)
    t0 = P.hx_topo_create(0, 2, [1], [1])
    with pytest.raises(P.HXError) as e:       # its own 3 rows, not the node's 6
        P.hx_neighbor_locality_alltoallv_init(FakeTensor(3), [1], None, [1], FakeTensor(2), [2], None, [3, 4],
                                              t0, comm3)
    assert e.value.code == P.HX_ERR_ARG
    r3 = P.hx_neighbor_locality_alltoallv_init(FakeTensor(6), [1], None, [1], FakeTensor(2), [2], None, [3, 4],
                                               t0, comm3)
    with pytest.raises(P.HXError) as e:
        P.hx_start(r3, stream=0)
    assert e.value.code == P.HX_ERR_STATE
    r3.free()
    comm3.free()
    with pytest.raises(P.HXError) as e:
        P.hx_comm_create(2, [0, 3, 6], 1, P.HX_LOCALITY_2STEP, node_map=5, stream=0)
    assert e.value.code == P.HX_ERR_ARG
    comm = P.hx_comm_create(2, [0, 3, 6], 1, P.HX_LOCALITY_2STEP, stream=0)
    t0 = P.hx_topo_create(0, 2, [1], [1])
    t1 = P.hx_topo_create(1, 2, [0], [0])
    x, h = FakeTensor(3), FakeTensor(2)
    r0 = P.hx_neighbor_locality_alltoallv_init(x, [1], None, [1], h, [2], None, [3, 4], t0, comm)
    with pytest.raises(P.HXError) as e:
        P.hx_start(r0, stream=0)
    assert e.value.code == P.HX_ERR_STATE
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_locality_alltoallv_init(x, [1], None, [1], h, [2], None, [3, 4], t0, comm)
    assert e.value.code == P.HX_ERR_STATE
    # rank 1 sends [3, 4] (as rank 0 expects) but expects [0] where rank 0 sends [1]
    x1, h1 = FakeTensor(3), FakeTensor(1)
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_locality_alltoallv_init(x1, [2], None, [3, 4], h1, [1], None, [0], t1, comm)
    assert e.value.code == P.HX_ERR_ARG
    with pytest.raises(P.HXError) as e:
        P.hx_start(r0, stream=0)
    assert e.value.code == P.HX_ERR_STATE
    # an index the source does not own, and a wrong row count
    comm2 = P.hx_comm_create(2, [0, 3, 6], 1, P.HX_PLAIN, stream=0)
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_locality_alltoallv_init(x, [1], None, [1], h, [2], None, [2, 4], t0, comm2)
    assert e.value.code == P.HX_ERR_RANGE
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_locality_alltoallv_init(FakeTensor(4), [1], None, [1], h, [2], None, [3, 4], t0, comm2)
    assert e.value.code == P.HX_ERR_ARG
    r0.free()
    comm.free()
    comm2.free()
