"""ctypes binding of ``libhx.so`` (include/hx.h): same entry-point names,
argument marshalling only.  Every step of the exchange runs in the library's
HIP kernels; PyTorch only supplies device memory and the current stream.

The binding fails loudly when the library is missing: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhx.so")

HX_SUCCESS = 0
HX_ERR_ARG, HX_ERR_RANGE, HX_ERR_STATE, HX_ERR_NOMEM, HX_ERR_UNSUPPORTED, HX_ERR_HIP = -1, -2, -3, -4, -5, -6
HX_F32, HX_F64 = 0, 1
HX_PLAIN, HX_LOCALITY_2STEP, HX_LOCALITY_3STEP = 0, 1, 2
HX_NODES_BLOCK, HX_NODES_CYCLIC = 0, 1
NODE_MAPS = {"block": HX_NODES_BLOCK, "cyclic": HX_NODES_CYCLIC}
HX_ARENA_SEND, HX_ARENA_RECV, HX_ARENA_GRAD_SEND = 0, 1, 4
HX_WORLD_SIM_TRANSFER, HX_WORLD_STAGED_BACKWARD = 1, 2
HX_REPLAY_GRAPH, HX_REPLAY_DIRECT = 0, 1
HX_PLAN_MAX_RANKS = 16384
HX_NOALLOC_SCRATCH_BYTES = 1 << 20
PHASES = ("pack", "redist", "unpack", "backward")

FIELDS = ("halo", "s1_procs", "s1_counts", "s1_displs", "s1_idx",
          "r1_procs", "r1_counts", "r1_displs",
          "s2_procs", "s2_counts", "s2_displs", "s2_src",
          "r2_procs", "r2_counts", "r2_displs",
          "unpack_src", "bt_ptr", "bt_perm")
FIELD_ID = {k: i for i, k in enumerate(FIELDS)}

EXPORTED = (
    "hx_error_string", "hx_last_hip_error", "hx_last_error_message", "hx_version", "hx_set_allocator",
    "hx_topo_create", "hx_topo_free", "hx_neighbor_alltoallv_init",
    "hx_comm_create", "hx_comm_free", "hx_neighbor_locality_alltoallv_init",
    "hx_plan_from_csr", "hx_plan_from_halos", "hx_plan_free", "hx_plan_field_size",
    "hx_plan_field_copy", "hx_plan_field_all", "hx_plan_describe", "hx_req_from_plan", "hx_start", "hx_wait", "hx_req_arena",
    "hx_req_bind_grad", "hx_req_enable_ready", "hx_backward", "hx_backward_noalloc", "hx_req_free", "hx_batch_init", "hx_batch_from_plan",
    "hx_batch_start", "hx_batch_wait", "hx_batch_start_plain", "hx_batch_wait_plain",
    "hx_batch_bind_grad", "hx_batch_backward", "hx_batch_backward_plain", "hx_batch_tune",
    "hx_batch_launch_phase", "hx_batch_get_sched", "hx_batch_set_sched", "hx_batch_set_replay", "hx_batch_get_replay",
    "hx_batch_arena", "hx_batch_arena_offset", "hx_batch_bytes", "hx_batch_free",
)


class HXError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hx error {code}: {msg}")
        self.code = code


class hx_sched(C.Structure):
    _fields_ = [("tile_rows", C.c_int), ("block_threads", C.c_int), ("blocks_per_cu", C.c_int),
                ("nontemporal", C.c_int), ("per_neighbor", C.c_int), ("unroll", C.c_int),
                ("push_pack", C.c_int), ("lds_window", C.c_int), ("pair_rows", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class hx_info(C.Structure):
    _fields_ = [("variant", C.c_int), ("ppn", C.c_int), ("node_map", C.c_int)]


_lib = None
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
VP = C.c_void_p
PP = C.POINTER(C.c_void_p)
I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)


def load() -> C.CDLL:
    """Loads libhx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2309_07337_amd.build)")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "hx_error_string": (C.c_char_p, [C.c_int]),
        "hx_last_hip_error": (C.c_int, []),
        "hx_last_error_message": (C.c_char_p, []),
        "hx_version": (C.c_char_p, []),
        "hx_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, VP]),
        "hx_topo_create": (C.c_int, [C.c_int, C.c_int, C.c_int, I32P, I32P, C.c_int, I32P, I32P, C.c_int, PP]),
        "hx_topo_free": (C.c_int, [PP]),
        "hx_neighbor_alltoallv_init": (C.c_int, [VP, C.c_int64, I32P, I32P, I32P, VP, I32P, I32P, C.c_int,
                                                 C.c_int, VP, PP]),
        "hx_comm_create": (C.c_int, [C.c_int, I64P, C.POINTER(hx_info), VP, PP]),
        "hx_comm_free": (C.c_int, [PP]),
        "hx_neighbor_locality_alltoallv_init": (C.c_int, [VP, C.c_int64, I32P, I32P, I64P, VP, I32P, I32P, I64P,
                                                          C.c_int, C.c_int, VP, VP, PP]),
        "hx_plan_from_csr": (C.c_int, [C.c_int, I64P, C.POINTER(hx_info), VP, VP, VP, PP]),
        "hx_plan_from_halos": (C.c_int, [C.c_int, I64P, C.POINTER(hx_info), I64P, VP, VP, PP]),
        "hx_plan_free": (C.c_int, [PP]),
        "hx_plan_field_size": (C.c_int, [VP, C.c_int, C.c_int, I64P]),
        "hx_plan_field_copy": (C.c_int, [VP, C.c_int, C.c_int, I32P]),
        "hx_plan_field_all": (C.c_int, [VP, C.c_int, I64P, I32P]),
        "hx_plan_describe": (C.c_int, [VP, C.POINTER(C.c_int), I64P, C.POINTER(hx_info), I64P]),
        "hx_req_from_plan": (C.c_int, [VP, C.c_int, VP, VP, C.c_int, C.c_int, PP]),
        "hx_start": (C.c_int, [VP, VP]),
        "hx_wait": (C.c_int, [VP, VP]),
        "hx_req_arena": (C.c_int, [VP, C.c_int, PP, I64P]),
        "hx_req_bind_grad": (C.c_int, [VP, VP, VP]),
        "hx_backward": (C.c_int, [VP, VP]),
        "hx_backward_noalloc": (C.c_int, [VP, VP, VP, VP]),
        "hx_req_free": (C.c_int, [PP]),
        "hx_batch_init": (C.c_int, [PP, C.c_int, C.POINTER(hx_sched), PP]),
        "hx_batch_from_plan": (C.c_int, [VP, VP, VP, C.c_int, C.c_int, C.c_int, C.POINTER(hx_sched), PP]),
        "hx_batch_start": (C.c_int, [VP, VP]),
        "hx_batch_wait": (C.c_int, [VP, VP]),
        "hx_batch_start_plain": (C.c_int, [VP, VP]),
        "hx_batch_wait_plain": (C.c_int, [VP, VP]),
        "hx_batch_bind_grad": (C.c_int, [VP, VP, VP]),
        "hx_batch_backward": (C.c_int, [VP, VP]),
        "hx_batch_backward_plain": (C.c_int, [VP, VP]),
        "hx_batch_tune": (C.c_int, [VP, VP]),
        "hx_req_enable_ready": (C.c_int, [VP, PP]),
        "hx_batch_launch_phase": (C.c_int, [VP, C.c_int, VP]),
        "hx_batch_get_sched": (C.c_int, [VP, C.c_int, C.POINTER(hx_sched)]),
        "hx_batch_set_sched": (C.c_int, [VP, C.c_int, C.POINTER(hx_sched)]),
        "hx_batch_set_replay": (C.c_int, [VP, C.c_int]),
        "hx_batch_get_replay": (C.c_int, [VP, C.POINTER(C.c_int)]),
        "hx_batch_arena": (C.c_int, [VP, C.c_int, PP, I64P]),
        "hx_batch_arena_offset": (C.c_int, [VP, C.c_int, C.c_int, I64P]),
        "hx_batch_bytes": (C.c_int, [VP, C.c_int, I64P]),
        "hx_batch_free": (C.c_int, [PP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    use_torch_allocator()
    return lib


# ---------------------------------------------------------------------------
# Device memory: the library allocates through torch's caching allocator, so
# torch sees (torch.cuda.memory_allocated) and reuses the arenas and plan
# arrays.  The callbacks run at init / free time only, never in Start / Wait.
# ---------------------------------------------------------------------------
_shutting_down = False


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        s = int(stream) if stream else torch.cuda.current_stream().cuda_stream
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), s)
    except Exception:      # out of memory (or no device): the library reports HX_ERR_NOMEM
        return None


def _torch_free(ptr, ctx):
    if _shutting_down or not ptr:
        return             # the interpreter is exiting: the process releases the memory
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


_TORCH_ALLOC = ALLOC_FN(_torch_alloc)
_TORCH_FREE = FREE_FN(_torch_free)
_allocator_keep = []        # callbacks installed by hx_set_allocator stay alive here


def _at_exit():
    global _shutting_down
    _shutting_down = True


import atexit  # noqa: E402
atexit.register(_at_exit)


def hx_set_allocator(alloc_fn=None, free_fn=None, ctx=None) -> None:
    """Installs device allocation callbacks (ctypes ALLOC_FN / FREE_FN
    objects, or plain Python callables wrapped here); None, None restores
    hipMalloc / hipFree.  Allocations made afterwards go through them."""
    if alloc_fn is not None and not isinstance(alloc_fn, ALLOC_FN):
        alloc_fn = ALLOC_FN(alloc_fn)
    if free_fn is not None and not isinstance(free_fn, FREE_FN):
        free_fn = FREE_FN(free_fn)
    _check(load().hx_set_allocator(alloc_fn if alloc_fn is not None else ALLOC_FN(0),
                                   free_fn if free_fn is not None else FREE_FN(0), ctx))
    _allocator_keep.extend([f for f in (alloc_fn, free_fn) if f is not None])


def use_torch_allocator() -> None:
    """Routes the library's device allocations through torch's caching allocator."""
    _check(_lib.hx_set_allocator(_TORCH_ALLOC, _TORCH_FREE, None))


def _check(rc: int) -> None:
    if rc != HX_SUCCESS:
        msg = load().hx_last_error_message().decode(errors="replace")
        raise HXError(rc, msg)


def _i32(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _p32(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(I32P)


def _p64(a: np.ndarray):
    return a.ctypes.data_as(I64P)


def _dptr(t) -> Optional[int]:
    """Device address of a tensor (None for None)."""
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream=None) -> Optional[int]:
    if stream is not None:
        return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _dtype_of(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return HX_F64
    if t.dtype == torch.float32:
        return HX_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ncols(t) -> int:
    return 1 if t.dim() == 1 else int(np.prod(t.shape[1:]))


class _Handle:
    _free_name = ""

    def __init__(self, ptr: C.c_void_p, keep=()):
        self.ptr = ptr
        self._keep = list(keep)

    @property
    def value(self):
        return self.ptr

    def free(self):
        if self.ptr is not None and self.ptr.value:
            rc = getattr(load(), self._free_name)(C.byref(self.ptr))
            if rc != HX_SUCCESS:   # e.g. a request still active or held by a batch: kept
                _check(rc)
        self.ptr = None
        self._keep = []

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Topo(_Handle):
    _free_name = "hx_topo_free"


class Plan(_Handle):
    _free_name = "hx_plan_free"


class Req(_Handle):
    _free_name = "hx_req_free"


class Batch(_Handle):
    _free_name = "hx_batch_free"


class Comm(_Handle):
    _free_name = "hx_comm_free"


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def hx_version() -> str:
    return load().hx_version().decode()


def hx_error_string(code: int) -> str:
    return load().hx_error_string(code).decode()


def hx_topo_create(rank: int, nranks: int, recv_procs: Sequence[int], send_procs: Sequence[int],
                   recv_weights=None, send_weights=None, reorder: int = 0) -> Topo:
    rp, sp = _i32(recv_procs), _i32(send_procs)
    rw, sw = _i32(recv_weights), _i32(send_weights)
    out = C.c_void_p()
    _check(load().hx_topo_create(rank, nranks, len(rp), _p32(rp), _p32(rw), len(sp), _p32(sp), _p32(sw),
                                 reorder, C.byref(out)))
    return Topo(out)


def hx_neighbor_alltoallv_init(x_local, sendcounts, sdispls, send_idx, halo, recvcounts, rdispls,
                               topo: Topo) -> Req:
    sc, sd, si = _i32(sendcounts), _i32(sdispls), _i32(send_idx)
    rc, rd = _i32(recvcounts), _i32(rdispls)
    out = C.c_void_p()
    n_local = int(x_local.shape[0])
    _check(load().hx_neighbor_alltoallv_init(_dptr(x_local), n_local, _p32(sc), _p32(sd), _p32(si),
                                             _dptr(halo), _p32(rc), _p32(rd), _dtype_of(x_local),
                                             _ncols(x_local), topo.ptr, C.byref(out)))
    return Req(out, keep=(x_local, halo, topo))


def _info(ppn: int, variant: int, node_map) -> hx_info:
    nm = NODE_MAPS[node_map] if isinstance(node_map, str) else int(node_map)
    return hx_info(int(variant), int(ppn), nm)


def hx_comm_create(nranks: int, row_starts, ppn: int, variant: int, node_map="block", stream=None) -> Comm:
    """A simulated communicator for the collective per-rank locality-aware init."""
    rs = _i64(row_starts)
    info = _info(ppn, variant, node_map)
    out = C.c_void_p()
    _check(load().hx_comm_create(nranks, _p64(rs), C.byref(info), _stream(stream), C.byref(out)))
    return Comm(out)


def hx_neighbor_locality_alltoallv_init(x_local, sendcounts, sdispls, global_sindices, halo, recvcounts, rdispls,
                                        global_rindices, topo: Topo, comm: Comm) -> Req:
    """One rank joins the collective init (pending until every rank has joined)."""
    sc, sd, rc, rd = _i32(sendcounts), _i32(sdispls), _i32(recvcounts), _i32(rdispls)
    gs, gr = _i64(global_sindices), _i64(global_rindices)
    out = C.c_void_p()
    _check(load().hx_neighbor_locality_alltoallv_init(
        _dptr(x_local), int(x_local.shape[0]), _p32(sc), _p32(sd), _p64(gs), _dptr(halo), _p32(rc), _p32(rd),
        _p64(gr), _dtype_of(x_local), _ncols(x_local), topo.ptr, comm.ptr, C.byref(out)))
    return Req(out, keep=(x_local, halo, topo, comm))


def hx_plan_from_csr(nranks: int, row_starts, ppn: int, variant: int, row_ptr, cols, stream=None,
                     node_map="block") -> Plan:
    """node_map: "block" / "cyclic" (or HX_NODES_*); with ppn and variant it
    fills the hx_info argument."""
    rs = _i64(row_starts)
    info = _info(ppn, variant, node_map)
    out = C.c_void_p()
    _check(load().hx_plan_from_csr(nranks, _p64(rs), C.byref(info), _dptr(row_ptr), _dptr(cols),
                                   _stream(stream), C.byref(out)))
    return Plan(out)


def hx_plan_from_halos(nranks: int, row_starts, ppn: int, variant: int, halo_ptr, halo_cols,
                       stream=None, node_map="block") -> Plan:
    rs, hp = _i64(row_starts), _i64(halo_ptr)
    info = _info(ppn, variant, node_map)
    out = C.c_void_p()
    _check(load().hx_plan_from_halos(nranks, _p64(rs), C.byref(info), _p64(hp), _dptr(halo_cols),
                                     _stream(stream), C.byref(out)))
    return Plan(out)


def hx_plan_field(plan: Plan, rank: int, field: str) -> np.ndarray:
    """hx_plan_field_size + hx_plan_field_copy: one per-rank plan array on the host."""
    fid = FIELD_ID[field]
    n = C.c_int64()
    _check(load().hx_plan_field_size(plan.ptr, rank, fid, C.byref(n)))
    out = np.empty(n.value, np.int32)
    _check(load().hx_plan_field_copy(plan.ptr, rank, fid, _p32(out)))
    return out


def hx_plan_field_all(plan: Plan, field: str):
    """(offsets [nranks+1], concatenation of every rank's array) of one field."""
    fid = FIELD_ID[field]
    R = hx_plan_describe(plan)["nranks"]
    off = np.empty(R + 1, np.int64)
    _check(load().hx_plan_field_all(plan.ptr, fid, _p64(off), None))
    out = np.empty(int(off[-1]), np.int32)
    _check(load().hx_plan_field_all(plan.ptr, fid, None, _p32(out)))
    return off, out


def hx_plan_describe(plan: Plan) -> dict:
    """nranks, n, variant, ppn, node_map ("block" / "cyclic") and row_starts of a plan."""
    R, n, info = C.c_int(), C.c_int64(), hx_info()
    _check(load().hx_plan_describe(plan.ptr, C.byref(R), C.byref(n), C.byref(info), None))
    rs = np.empty(R.value + 1, np.int64)
    _check(load().hx_plan_describe(plan.ptr, None, None, None, _p64(rs)))
    nm = {v: k for k, v in NODE_MAPS.items()}[info.node_map]
    return dict(nranks=R.value, n=n.value, variant=info.variant, ppn=info.ppn, node_map=nm, row_starts=rs)


def hx_req_from_plan(plan: Plan, rank: int, x_local, halo) -> Req:
    out = C.c_void_p()
    _check(load().hx_req_from_plan(plan.ptr, rank, _dptr(x_local), _dptr(halo), _dtype_of(x_local),
                                   _ncols(x_local), C.byref(out)))
    return Req(out, keep=(plan, x_local, halo))


def hx_start(req: Req, stream=None) -> None:
    _check(load().hx_start(req.ptr, _stream(stream)))


def hx_wait(req: Req, stream=None) -> None:
    _check(load().hx_wait(req.ptr, _stream(stream)))


def hx_req_arena(req: Req, which: int):
    p, rows = C.c_void_p(), C.c_int64()
    _check(load().hx_req_arena(req.ptr, which, C.byref(p), C.byref(rows)))
    return (p.value or 0), rows.value


def hx_req_bind_grad(req: Req, g_send, g_x) -> None:
    _check(load().hx_req_bind_grad(req.ptr, _dptr(g_send), _dptr(g_x)))
    req._keep += [g_send, g_x]


def hx_req_enable_ready(req: Req) -> int:
    """Per-message completion counters of the pack (device address of
    len(send list) uint64 counters owned by the request)."""
    p = C.c_void_p()
    _check(load().hx_req_enable_ready(req.ptr, C.byref(p)))
    return p.value or 0


def hx_backward(req: Req, stream=None) -> None:
    _check(load().hx_backward(req.ptr, _stream(stream)))


def hx_backward_noalloc(req: Req, g_send, g_x, stream=None) -> None:
    """The request's backward into g_x from g_send, allocating nothing (the
    launch table goes to the library's fixed per-device area)."""
    _check(load().hx_backward_noalloc(req.ptr, _dptr(g_send), _dptr(g_x), _stream(stream)))


def _sched_ptr(sched):
    if sched is None:
        return None
    s = hx_sched(**{k: int(sched.get(k, 0)) for k, _ in hx_sched._fields_}) if isinstance(sched, dict) else sched
    return C.pointer(s)


def hx_batch_init(reqs: Sequence[Req], sched=None) -> Batch:
    arr = (C.c_void_p * len(reqs))(*[r.ptr.value for r in reqs])
    out = C.c_void_p()
    _check(load().hx_batch_init(arr, len(reqs), _sched_ptr(sched), C.byref(out)))
    return Batch(out, keep=list(reqs))


def hx_batch_from_plan(plan: Plan, x_global, halo_all, flags: int = 0, sched=None) -> Batch:
    out = C.c_void_p()
    _check(load().hx_batch_from_plan(plan.ptr, _dptr(x_global), _dptr(halo_all), _dtype_of(x_global),
                                     _ncols(x_global), flags, _sched_ptr(sched), C.byref(out)))
    return Batch(out, keep=(plan, x_global, halo_all))


def hx_batch_start(b: Batch, stream=None) -> None:
    _check(load().hx_batch_start(b.ptr, _stream(stream)))


def hx_batch_wait(b: Batch, stream=None) -> None:
    _check(load().hx_batch_wait(b.ptr, _stream(stream)))


def hx_batch_start_plain(b: Batch, stream=None) -> None:
    _check(load().hx_batch_start_plain(b.ptr, _stream(stream)))


def hx_batch_wait_plain(b: Batch, stream=None) -> None:
    _check(load().hx_batch_wait_plain(b.ptr, _stream(stream)))


def hx_batch_bind_grad(b: Batch, g_in, g_out) -> None:
    _check(load().hx_batch_bind_grad(b.ptr, _dptr(g_in), _dptr(g_out)))
    b._keep += [g_in, g_out]


def hx_batch_backward(b: Batch, stream=None) -> None:
    _check(load().hx_batch_backward(b.ptr, _stream(stream)))


def hx_batch_backward_plain(b: Batch, stream=None) -> None:
    _check(load().hx_batch_backward_plain(b.ptr, _stream(stream)))


def hx_batch_launch_phase(b: Batch, phase: int, stream=None) -> None:
    _check(load().hx_batch_launch_phase(b.ptr, phase, _stream(stream)))


def hx_batch_tune(b: Batch, stream=None) -> None:
    _check(load().hx_batch_tune(b.ptr, _stream(stream)))


def hx_batch_get_sched(b: Batch, phase: int) -> dict:
    s = hx_sched()
    _check(load().hx_batch_get_sched(b.ptr, phase, C.byref(s)))
    return s.as_dict()


def hx_batch_set_sched(b: Batch, phase: int, sched) -> None:
    """Applies a schedule (dict of hx_sched fields, or hx_sched) to one phase."""
    _check(load().hx_batch_set_sched(b.ptr, phase, _sched_ptr(sched)))


def hx_batch_set_replay(b: Batch, mode: int) -> None:
    _check(load().hx_batch_set_replay(b.ptr, mode))


def hx_batch_get_replay(b: Batch) -> int:
    m = C.c_int()
    _check(load().hx_batch_get_replay(b.ptr, C.byref(m)))
    return m.value


def hx_batch_arena(b: Batch, which: int):
    p, rows = C.c_void_p(), C.c_int64()
    _check(load().hx_batch_arena(b.ptr, which, C.byref(p), C.byref(rows)))
    return (p.value or 0), rows.value


def hx_batch_arena_offset(b: Batch, which: int, rank: int) -> int:
    v = C.c_int64()
    _check(load().hx_batch_arena_offset(b.ptr, which, rank, C.byref(v)))
    return v.value


def hx_batch_bytes(b: Batch, phase: int) -> int:
    v = C.c_int64()
    _check(load().hx_batch_bytes(b.ptr, phase, C.byref(v)))
    return v.value


class _ArrayInterface:
    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def device_view(ptr: int, rows: int, ncols: int, dtype):
    """Zero-copy torch view of library-owned device memory (an arena).

    The view must not outlive the handle that owns the memory.
    """
    import torch
    if rows == 0 or not ptr:
        return torch.empty((rows, ncols), dtype=dtype, device="cuda")
    typestr = {torch.float64: "<f8", torch.float32: "<f4", torch.int32: "<i4", torch.int64: "<i8"}[dtype]
    return torch.as_tensor(_ArrayInterface(ptr, (rows, ncols), typestr), device="cuda")


def req_arena_view(req: Req, which: int, ncols: int, dtype):
    p, rows = hx_req_arena(req, which)
    return device_view(p, rows, ncols, dtype)


def batch_arena_view(b: Batch, which: int, ncols: int, dtype):
    p, rows = hx_batch_arena(b, which)
    return device_view(p, rows, ncols, dtype)
