"""Device memory through the installed allocator (torch's caching allocator
by default), allocation failures injected through the allocator callback,
gradient rebinding of batch members, and the autograd Function's output
buffers."""
import ctypes as C
import gc

import numpy as np
import pytest

import paper_2309_07337_amd as P
from paper_2309_07337_amd import _lib as L
from oracle import move as OM
from oracle import plan as OP
from tests.gpu_util import bits_equal, dev, gpu_plan, host, need_gpu, say
from workloads import batched_plan, batched_plan_sizes, random_small_csr, uniform_pm1, uniform_pm1_f32

pytestmark = pytest.mark.gpu


def _plan_lists(b, cap):
    h, k = batched_plan_sizes()
    hb = int(min(h[b], cap))
    return hb, batched_plan(b, hb, int(min(k[b], hb)))


def _init(lists, h, ncols, torch):
    x = dev(uniform_pm1(11, h * ncols).reshape(h, ncols))
    halo = torch.zeros(h, ncols, dtype=torch.float64, device="cuda")
    topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
    req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                       lists["counts"], lists["displs"], topo)
    return req, x, halo


def test_torch_allocator_accounts_for_arenas():
    need_gpu()
    import torch
    h, lists = _plan_lists(3, 200_000)
    ncols = 16
    x = dev(uniform_pm1(11, h * ncols).reshape(h, ncols))
    halo = torch.zeros(h, ncols, dtype=torch.float64, device="cuda")
    topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
    gc.collect()  # handles of earlier tests still held by reference cycles free their memory now
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                       lists["counts"], lists["displs"], topo)
    torch.cuda.synchronize()
    E = int(np.sum(lists["counts"]))
    arenas = 2 * E * ncols * 8                      # send + receive arenas
    grown = torch.cuda.memory_allocated() - before
    say("allocated through torch:", grown, "arenas:", arenas)
    assert grown >= arenas
    P.hx_start(req)
    P.hx_wait(req)
    assert bits_equal(host(P.req_arena_view(req, P.HX_ARENA_SEND, ncols, torch.float64)),
                      OM.pack(host(x), lists["send_idx"]))
    req.free()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


class _Counting:
    """Allocator over torch's that fails after `ok` successful allocations
    and tracks the blocks it handed out."""

    def __init__(self, ok):
        import torch
        self.torch = torch
        self.ok = ok
        self.live = {}
        self.calls = 0
        self.alloc = L.ALLOC_FN(self._alloc)
        self.free = L.FREE_FN(self._free)

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.calls > self.ok:
            return None
        p = self.torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream) if stream else 0)
        self.live[p] = nbytes
        return p

    def _free(self, ptr, ctx):
        self.live.pop(int(ptr))
        self.torch.cuda.caching_allocator_delete(int(ptr))


def test_nomem_injected_through_the_allocator_leaks_nothing():
    need_gpu()
    import torch
    h, lists = _plan_lists(5, 20_000)
    rs, rp, cols = random_small_csr(96, 8, 6, 0.5, 2309, False)
    rp_d, cols_d = dev(np.asarray(rp, np.int64)), dev(np.asarray(cols, np.int32))
    try:
        # count the allocations of each call when nothing fails
        probe = _Counting(10 ** 9)
        P.hx_set_allocator(probe.alloc, probe.free)
        req, x, halo = _init(lists, h, 2, torch)
        n_req = probe.calls
        plan = P.hx_plan_from_csr(len(rs) - 1, rs, 3, P.HX_LOCALITY_2STEP, rp_d, cols_d)
        n_plan = probe.calls - n_req
        req.free()
        plan.free()
        assert not probe.live
        say("allocations: request", n_req, "plan", n_plan)
        assert n_req >= 3 and n_plan >= 10
        # fail at every allocation in turn
        for fail_at in range(n_req):
            a = _Counting(fail_at)
            P.hx_set_allocator(a.alloc, a.free)
            with pytest.raises(P.HXError) as e:
                _init(lists, h, 2, torch)
            assert e.value.code == P.HX_ERR_NOMEM, fail_at
            assert not a.live, (fail_at, a.live)
        for fail_at in range(0, n_plan, max(1, n_plan // 12)):
            a = _Counting(fail_at)
            P.hx_set_allocator(a.alloc, a.free)
            with pytest.raises(P.HXError) as e:
                P.hx_plan_from_csr(len(rs) - 1, rs, 3, P.HX_LOCALITY_2STEP, rp_d, cols_d)
            assert e.value.code == P.HX_ERR_NOMEM, fail_at
            assert not a.live, (fail_at, a.live)
    finally:
        L.use_torch_allocator()
    # the library works normally afterwards
    req, x, halo = _init(lists, h, 2, torch)
    P.hx_start(req)
    P.hx_wait(req)
    assert bits_equal(host(P.req_arena_view(req, P.HX_ARENA_SEND, 2, torch.float64)),
                      OM.pack(host(x), lists["send_idx"]))


def test_hipmalloc_restored():
    need_gpu()
    import torch
    h, lists = _plan_lists(2, 5_000)
    try:
        P.hx_set_allocator(None, None)
        x = dev(uniform_pm1(11, h * 3).reshape(h, 3))
        halo = torch.zeros(h, 3, dtype=torch.float64, device="cuda")
        topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
        gc.collect()
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                           lists["counts"], lists["displs"], topo)
        # the arenas and lists came from hipMalloc, not from torch
        assert torch.cuda.memory_allocated() == before
        P.hx_start(req)
        P.hx_wait(req)
        assert bits_equal(host(P.req_arena_view(req, P.HX_ARENA_SEND, 3, torch.float64)),
                          OM.pack(host(x), lists["send_idx"]))
        req.free()
    finally:
        L.use_torch_allocator()


def test_member_gradients_rebound_to_new_buffers():
    need_gpu()
    import torch
    members = []
    for b in (0, 1, 4):
        h, lists = _plan_lists(b, 8_000)
        req, x, halo = _init(lists, h, 4, torch)
        members.append((req, x, lists, h))
    for req, x, lists, h in members:
        P.hx_req_bind_grad(req, dev(uniform_pm1(1, h * 4).reshape(h, 4)), torch.zeros_like(x))
    batch = P.hx_batch_init([m[0] for m in members])
    P.hx_batch_backward(batch)
    for rnd in range(2):
        # rebind every member to fresh buffers of the same size
        fresh = []
        for i, (req, x, lists, h) in enumerate(members):
            g = dev(uniform_pm1(100 * rnd + i, h * 4).reshape(h, 4))
            gx = torch.full_like(x, float("nan"))
            P.hx_req_bind_grad(req, g, gx)
            fresh.append((g, gx))
        if rnd == 0:
            P.hx_batch_backward(batch)
        else:
            P.hx_batch_backward_plain(batch)
        for (req, x, lists, h), (g, gx) in zip(members, fresh):
            ptr, perm = OP.transpose_csr(lists["send_idx"], h)
            assert bits_equal(host(gx), OM.pack_transpose(host(g), ptr, perm)), rnd


def test_halo_gather_outputs_do_not_alias():
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange, halo_gather
    n, R, ppn, C = 96, 8, 3, 3
    rs, rp, cols = random_small_csr(n, R, 6, 0.5, 2309, False)
    halos = OP.all_halos(rp, cols, rs)
    plan = gpu_plan(rs, rp, cols, ppn, "locality")
    H = sum(h.size for h in halos)
    hcat = np.concatenate(halos)
    ex = HaloExchange(plan, n, H, C, dtype=torch.float32)
    xa = uniform_pm1_f32(1, n * C).reshape(n, C)
    xb = uniform_pm1_f32(2, n * C).reshape(n, C)
    ya = halo_gather(dev(xa), ex)
    yb = halo_gather(dev(xb), ex)
    assert bits_equal(host(ya), xa[hcat]) and bits_equal(host(yb), xb[hcat])
    # aliased output: a later forward invalidates its backward
    x = ex.x
    x.copy_(dev(xa))
    xr = x.detach().requires_grad_(True)
    y = halo_gather(xr, ex, copy_out=False)
    assert y.data_ptr() == ex.halo.data_ptr()
    halo_gather(dev(xb), ex, copy_out=False)
    with pytest.raises(RuntimeError, match="overwritten"):
        y.backward(torch.ones_like(y))
    # the zero-copy path: input in ex.x, gradient in ex.g_halo
    xr = ex.x.detach().requires_grad_(True)
    y = halo_gather(xr, ex, copy_out=False)
    g = uniform_pm1_f32(3, H * C).reshape(H, C)
    ex.g_halo.copy_(dev(g))
    y.backward(ex.g_halo)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    ref = OM.exchange_adjoint_reference(halos, gy, n)
    assert bits_equal(host(xr.grad), ref)
