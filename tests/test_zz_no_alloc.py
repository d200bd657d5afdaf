"""The backward entry point that allocates nothing (hx_backward_noalloc),
called through the C ABI: bit-equal to the request's bound backward
(hx_req_bind_grad + hx_backward) and to the oracle's transpose sum, on calls
in a row of shrinking size, without a single device allocation, replayed
from a captured graph, and rejecting sizes beyond its fixed area."""
import gc

import numpy as np
import pytest

import paper_2309_07337_amd as P
from paper_2309_07337_amd import _lib as L
from oracle import move as OM
from oracle import plan as OP
from tests.gpu_util import bits_equal, dev, host, need_gpu, say
from workloads import batched_plan, batched_plan_sizes, uniform_pm1, uniform_pm1_f32

pytestmark = pytest.mark.gpu


def _request(b, cap, ncols, f32, torch):
    h_all, k_all = batched_plan_sizes()
    h = int(min(h_all[b], cap))
    lists = batched_plan(b, h, int(min(k_all[b], h)))
    dt = torch.float32 if f32 else torch.float64
    x = torch.zeros(h, ncols, dtype=dt, device="cuda")
    halo = torch.zeros(h, ncols, dtype=dt, device="cuda")
    topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
    req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                       lists["counts"], lists["displs"], topo)
    E = int(np.sum(lists["counts"]))
    gen = uniform_pm1_f32 if f32 else uniform_pm1
    g = gen(500 + b, E * ncols).reshape(E, ncols)
    # a lone -0.0 must survive (first term first)
    g[0, 0] = -0.0
    return req, lists, h, g, dt


class _NoAlloc:
    """Allocator that records and refuses every request."""

    def __init__(self):
        self.calls = 0
        self.alloc = L.ALLOC_FN(self._alloc)
        self.free = L.FREE_FN(self._free)

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        return None

    def _free(self, ptr, ctx):
        self.calls += 1


def _bound_backward(req, g_dev, h, ncols, dt, torch):
    gx = torch.full((h, ncols), float("nan"), dtype=dt, device="cuda")
    P.hx_req_bind_grad(req, g_dev, gx)
    P.hx_backward(req)
    return host(gx)


@pytest.mark.parametrize("shape", [(16, False), (1, True), (3, False)], ids=["f64x16", "f32x1", "f64x3"])
def test_noalloc_backward_equals_bound_backward(shape):
    need_gpu()
    import torch
    ncols, f32 = shape
    # two calls in a row, the second on a smaller request
    # (FP32 x 1: the second request's send slots fit the sum's LDS term window)
    cases = [(7, 400_000), (0, 6_000)] if ncols > 1 else [(5, 400_000), (8, 12_000)]
    prepared = []
    for b, cap in cases:
        req, lists, h, g, dt = _request(b, cap, ncols, f32, torch)
        g_dev = dev(g)
        want = _bound_backward(req, g_dev, h, ncols, dt, torch)
        ptr, perm = OP.transpose_csr(lists["send_idx"], h)
        assert bits_equal(want, OM.pack_transpose(g, ptr, perm))
        prepared.append((req, g_dev, h, dt, want))
    outs = [torch.full((h, ncols), float("nan"), dtype=dt, device="cuda") for _, _, h, dt, _ in prepared]
    gc.collect()  # nothing of earlier tests is freed inside the measured window
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    refuse = _NoAlloc()
    try:
        P.hx_set_allocator(refuse.alloc, refuse.free)
        for (req, g_dev, h, dt, want), gx in zip(prepared, outs):
            say("noalloc backward: rows", h, "ncols", ncols, "f32" if f32 else "f64")
            P.hx_backward_noalloc(req, g_dev, gx)
        torch.cuda.synchronize()
    finally:
        L.use_torch_allocator()
    assert refuse.calls == 0
    assert torch.cuda.memory_allocated() == before
    for (req, g_dev, h, dt, want), gx in zip(prepared, outs):
        assert bits_equal(host(gx), want)
    # the bound gradients are untouched: the bound backward still writes its own buffer
    req, g_dev, h, dt, want = prepared[0]
    assert bits_equal(_bound_backward(req, g_dev, h, ncols, dt, torch), want)


def test_noalloc_backward_replays_from_a_graph():
    need_gpu()
    import torch
    req, lists, h, g, dt = _request(7, 50_000, 16, False, torch)
    small, lists_s, h_s, g_s, _ = _request(1, 3_000, 16, False, torch)
    g_dev, gs_dev = dev(g), dev(g_s)
    want = _bound_backward(req, g_dev, h, 16, dt, torch)
    want_s = _bound_backward(small, gs_dev, h_s, 16, dt, torch)
    gx = torch.zeros(h, 16, dtype=dt, device="cuda")
    gx_s = torch.zeros(h_s, 16, dtype=dt, device="cuda")
    P.hx_backward_noalloc(req, g_dev, gx)  # first call on the device, outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            P.hx_backward_noalloc(req, g_dev, gx, stream=s)
            P.hx_backward_noalloc(small, gs_dev, gx_s, stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        gx.fill_(float("nan"))
        gx_s.fill_(float("nan"))
        # eager use of the same area between replays
        other = torch.full_like(gx_s, float("nan"))
        P.hx_backward_noalloc(small, gs_dev, other)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert bits_equal(host(gx), want), rep
        assert bits_equal(host(gx_s), want_s), rep
        assert bits_equal(host(other), want_s), rep


def test_noalloc_backward_limits_and_errors():
    need_gpu()
    import torch
    req, lists, h, g, dt = _request(2, 5_000, 2, False, torch)
    gx = torch.zeros(h, 2, dtype=dt, device="cuda")
    with pytest.raises(P.HXError) as e:
        P.hx_backward_noalloc(req, None, gx)
    assert e.value.code == P.HX_ERR_ARG
    with pytest.raises(P.HXError) as e:
        P.hx_backward_noalloc(req, dev(g), None)
    assert e.value.code == P.HX_ERR_ARG
    # one tile (512 rows of 4 bytes) more than the area holds: refused, nothing launched
    max_tiles = (P.HX_NOALLOC_SCRATCH_BYTES - 512) // 8
    n = (max_tiles + 1) * 512
    x = torch.zeros(n, 1, dtype=torch.float32, device="cuda")
    topo = P.hx_topo_create(0, 2, [], [])
    big = P.hx_neighbor_alltoallv_init(x, [], None, [], torch.zeros(0, 1, dtype=torch.float32, device="cuda"),
                                       [], None, topo)
    with pytest.raises(P.HXError) as e:
        P.hx_backward_noalloc(big, None, x)
    assert e.value.code == P.HX_ERR_UNSUPPORTED
    # at the limit it runs: every row of a request without sends gets +0.0
    n_ok = max_tiles * 512
    x_ok = x[:n_ok]
    ok = P.hx_neighbor_alltoallv_init(x_ok, [], None, [], torch.zeros(0, 1, dtype=torch.float32, device="cuda"),
                                      [], None, topo)
    x_ok.fill_(-1.0)
    P.hx_backward_noalloc(ok, None, x_ok)
    got = host(x_ok)
    assert not np.signbit(got).any() and not got.any()
    big.free()
    ok.free()
    del e
    gc.collect()
