"""Persistent requests initialised from explicit lists (the paper's init call):
pack / unpack / backward vs the oracle, bit for bit, plus the request state
machine and edge cases."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.gpu_util import bits_equal, dev, host, need_gpu, say
from workloads import batched_plan, batched_plan_sizes, uniform_pm1

pytestmark = pytest.mark.gpu


def make_req(lists, n_local, ncols, dtype, seed):
    import torch
    x = dev(uniform_pm1(seed, n_local * ncols).reshape(n_local, ncols)).to(dtype)
    H = int(np.sum(lists["counts"]))
    halo = torch.full((H, ncols), float("nan"), dtype=dtype, device="cuda")
    topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
    req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                       lists["counts"], lists["displs"], topo)
    return req, x, halo


def small_plans(cap=6000):
    h, k = batched_plan_sizes()
    out = []
    for b in (0, 1, 2, 5, 11, 40):
        hb = int(min(h[b], cap))
        kb = int(min(k[b], hb))
        out.append((b, hb, batched_plan(b, hb, kb)))
    return out


@pytest.mark.parametrize("dtype_name,ncols", [("f64", 1), ("f32", 1), ("f64", 16), ("f32", 64),
                                               ("f64", 3), ("f32", 5), ("f32", 2), ("f64", 64)])
def test_list_request_pack_unpack_backward(dtype_name, ncols):
    need_gpu()
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    for b, h, lists in small_plans():
        say("req", dtype_name, ncols, "plan", b, h)
        req, x, halo = make_req(lists, h, ncols, dtype, 500 + b)
        # simulated peers: the receive arena holds what the neighbors sent
        recv = dev(uniform_pm1(900 + b, h * ncols).reshape(h, ncols)).to(dtype)
        P.req_arena_view(req, P.HX_ARENA_RECV, ncols, dtype).copy_(recv)
        P.hx_start(req)
        P.hx_wait(req)
        send = P.req_arena_view(req, P.HX_ARENA_SEND, ncols, dtype)
        assert bits_equal(host(send), OM.pack(host(x), lists["send_idx"]))
        assert bits_equal(host(halo), host(recv))
        # backward of the pack
        g_send = dev(uniform_pm1(1300 + b, h * ncols).reshape(h, ncols)).to(dtype)
        g_x = torch.full_like(x, float("nan"))
        P.hx_req_bind_grad(req, g_send, g_x)
        P.hx_backward(req)
        ptr, perm = OP.transpose_csr(lists["send_idx"], h)
        assert bits_equal(host(g_x), OM.pack_transpose(host(g_send), ptr, perm))
        req.free()


def test_state_machine_and_repeat():
    need_gpu()
    import torch
    b, h, lists = small_plans()[1]
    req, x, halo = make_req(lists, h, 4, torch.float32, 3)
    P.hx_wait(req)                         # inactive: no-op
    P.hx_start(req)
    with pytest.raises(P.HXError) as e:
        P.hx_start(req)
    assert e.value.code == P.HX_ERR_STATE
    P.hx_wait(req)
    for it in range(3):                    # persistent: re-start with new values
        x.copy_(dev(uniform_pm1(40 + it, h * 4).reshape(h, 4)).float())
        P.hx_start(req)
        P.hx_wait(req)
        send = P.req_arena_view(req, P.HX_ARENA_SEND, 4, torch.float32)
        assert bits_equal(host(send), OM.pack(host(x), lists["send_idx"]))


def test_edge_cases():
    need_gpu()
    import torch
    # no neighbors at all
    topo = P.hx_topo_create(0, 2, [], [])
    x = torch.zeros(7, 2, dtype=torch.float64, device="cuda")
    req = P.hx_neighbor_alltoallv_init(x, [], [], [], None, [], [], topo)
    P.hx_start(req)
    P.hx_wait(req)
    g_x = torch.full_like(x, 5.0)
    P.hx_req_bind_grad(req, None, g_x)
    P.hx_backward(req)
    assert np.all(host(g_x) == 0.0) and not np.any(np.signbit(host(g_x)))
    # zero-count neighbors, one row, a single value sent many times
    topo = P.hx_topo_create(1, 5, [0, 2, 3, 4], [0, 2, 3, 4])
    x = dev(np.array([[-0.0], [2.5]], np.float32))
    counts, displs = [0, 3, 0, 1], [0, 0, 3, 3]
    idx = [1, 0, 1, 0]
    halo = torch.zeros(4, 1, dtype=torch.float32, device="cuda")
    req = P.hx_neighbor_alltoallv_init(x, counts, displs, idx, halo, counts, displs, topo)
    P.req_arena_view(req, P.HX_ARENA_RECV, 1, torch.float32).copy_(dev(np.arange(4, dtype=np.float32)[:, None]))
    P.hx_start(req)
    P.hx_wait(req)
    assert host(P.req_arena_view(req, P.HX_ARENA_SEND, 1, torch.float32))[:, 0].tolist() == [2.5, -0.0, 2.5, -0.0]
    assert host(halo)[:, 0].tolist() == [0, 1, 2, 3]
    g_send = dev(np.array([[1.0], [-0.0], [2.0], [-0.0]], np.float32))
    g_x = torch.full_like(x, 9.0)
    P.hx_req_bind_grad(req, g_send, g_x)
    P.hx_backward(req)
    gx = host(g_x)[:, 0]
    assert gx[1] == 3.0 and gx[0] == 0.0 and np.signbit(gx[0])   # -0 + -0 = -0


def test_misaligned_and_bad_arguments():
    need_gpu()
    import torch
    topo = P.hx_topo_create(0, 2, [1], [1])
    x = torch.zeros(8, 1, dtype=torch.float64, device="cuda")
    halo = torch.zeros(2, 1, dtype=torch.float64, device="cuda")
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_alltoallv_init(x, [2], [0], [0, 8], halo, [2], [0], topo)
    assert e.value.code == P.HX_ERR_RANGE
    with pytest.raises(P.HXError) as e:
        P.hx_neighbor_alltoallv_init(x, [2], [1], [0, 1], halo, [2], [0], topo)
    assert e.value.code == P.HX_ERR_ARG


def counters_view(ptr, n):
    import torch
    return P.device_view(ptr, n, 1, torch.int64)   # uint64 counters, small values


@pytest.mark.parametrize("ncols", [16, 1])
def test_partition_ready_counters(ncols):
    """Per-message completion counters: after the k-th pack each counter
    equals k times its message size; the packed data stay exact; batches with
    such members pack in the pull form and the tuner's trials do not count."""
    need_gpu()
    import torch
    (b0, h0, l0), (b1, h1, l1), (b2, h2, l2) = small_plans()[2:5]
    say("ready counters", ncols)
    reqs = []
    for b, h, lists in ((b0, h0, l0), (b1, h1, l1), (b2, h2, l2)):
        req, x, halo = make_req(lists, h, ncols, torch.float64, 900 + b)
        reqs.append((req, x, halo, lists))
    ptrs = [P.hx_req_enable_ready(r[0]) for r in reqs[:2]]     # the third member keeps no counters
    assert ptrs[0] == P.hx_req_enable_ready(reqs[0][0])      # enabling twice keeps the counters
    counts = [np.asarray(r[3]["counts"], np.int64) for r in reqs[:2]]
    # single request, three Start/Wait rounds
    req, x, halo, lists = reqs[0]
    for k in (1, 2, 3):
        P.hx_start(req)
        P.hx_wait(req)
        torch.cuda.synchronize()
        assert np.array_equal(host(counters_view(ptrs[0], counts[0].size))[:, 0], k * counts[0])
    send = host(P.req_arena_view(req, P.HX_ARENA_SEND, ncols, torch.float64))
    assert bits_equal(send, OM.pack(host(x), lists["send_idx"]))
    # batch of the three members: default schedule, then tuned
    bt = P.hx_batch_init([r[0] for r in reqs])
    assert P.hx_batch_get_sched(bt, 0)["push_pack"] == 2
    P.hx_batch_start(bt)
    P.hx_batch_wait(bt)
    P.hx_batch_tune(bt)
    P.hx_batch_start(bt)
    P.hx_batch_wait(bt)
    torch.cuda.synchronize()
    assert np.array_equal(host(counters_view(ptrs[0], counts[0].size))[:, 0], 5 * counts[0])
    assert np.array_equal(host(counters_view(ptrs[1], counts[1].size))[:, 0], 2 * counts[1])
    for req, x, halo, lists in reqs:
        send = host(P.req_arena_view(req, P.HX_ARENA_SEND, ncols, torch.float64))
        assert bits_equal(send, OM.pack(host(x), lists["send_idx"]))
    bt.free()


@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_request_steps_replayed_from_a_captured_graph(variant):
    """Start, Wait and the backward of one rank's request (built from a GPU
    plan, 2 FP64 columns) recorded in a CUDA graph after one eager step, then
    replayed four times with new vector, receive-arena and gradient values
    written eagerly between the replays (and unrelated eager work): every
    replay's send arena, halo and gradient equal the oracle's for that
    replay's inputs."""
    need_gpu()
    import torch
    from tests.gpu_util import gpu_plan
    from tests.test_oracle_brute import CASES
    from workloads import random_small_csr
    n, R, mx, pf, seed, uneven, ppn = CASES[4]
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    plans = [D.plan(q, variant) for q in range(R)]
    r = max(range(R), key=lambda q: halos[q].size)
    C = 2
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    nl = int(rs[r + 1] - rs[r])
    x_local = torch.zeros(nl, C, dtype=torch.float64, device="cuda")
    halo = torch.full((halos[r].size, C), float("nan"), dtype=torch.float64, device="cuda")
    req = P.hx_req_from_plan(plan, r, x_local, halo)
    recv = P.req_arena_view(req, P.HX_ARENA_RECV, C, torch.float64)
    send = P.req_arena_view(req, P.HX_ARENA_SEND, C, torch.float64)
    E1 = int(plans[r]["s1_idx"].size)
    g_send = torch.zeros(E1, C, dtype=torch.float64, device="cuda")
    g_x = torch.full_like(x_local, float("nan"))
    P.hx_req_bind_grad(req, g_send, g_x)

    def step():
        P.hx_start(req)
        P.hx_wait(req)
        P.hx_backward(req)

    step()                      # eager: builds the launch tables
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    other = torch.zeros(1 << 20, device="cuda")
    for it in range(4):
        xh = uniform_pm1(4000 + it, int(rs[-1]) * C).reshape(-1, C)
        out = OM.forward_all(plans, xh, rs)
        gh = uniform_pm1(5000 + it, E1 * C).reshape(E1, C)
        x_local.copy_(dev(xh[rs[r]:rs[r + 1]]))
        recv.copy_(dev(out["arena"][r]))
        g_send.copy_(dev(gh))
        halo.fill_(float("nan"))
        g_x.fill_(float("nan"))
        other.add_(1.0)          # unrelated eager work between replays
        torch.cuda.synchronize()
        say("captured request step, replay", variant, it)
        graph.replay()
        torch.cuda.synchronize()
        assert bits_equal(host(send), np.concatenate([out["send1"][r], out["send2"][r]])), it
        assert bits_equal(host(halo), out["halo"][r]), it
        want = OM.pack_transpose(gh, plans[r]["bt_ptr"], plans[r]["bt_perm"])
        assert bits_equal(host(g_x), want), it
    del graph
    req.free()


def test_free_refused_while_active_or_batched():
    """A request cannot be freed between Start and Wait, nor while a batch
    holds it as a member; both are HX_ERR_STATE and leave it intact."""
    need_gpu()
    import torch
    b, h, lists = small_plans()[0]
    req, x, halo = make_req(lists, h, 2, torch.float64, 7)
    P.hx_start(req)
    with pytest.raises(P.HXError) as e:
        req.free()
    assert e.value.code == P.HX_ERR_STATE and req.ptr is not None
    P.hx_wait(req)
    batch = P.hx_batch_init([req, req])
    with pytest.raises(P.HXError) as e:
        req.free()
    assert e.value.code == P.HX_ERR_STATE and req.ptr is not None
    P.hx_batch_start(batch)     # the member is intact
    P.hx_batch_wait(batch)
    batch.free()
    req.free()
    assert req.ptr is None
