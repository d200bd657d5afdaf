"""Batched persistent launches (hipGraph) vs the plain one-launch-per-plan
form vs the oracle, bit for bit, under several schedules and the tuner."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.gpu_util import bits_equal, dev, host, need_gpu, say
from workloads import batched_plan, batched_plan_sizes, uniform_pm1

pytestmark = pytest.mark.gpu


def build_members(nplans, cap, ncols, dtype):
    import torch
    h, k = batched_plan_sizes()
    mem = []
    for b in range(nplans):
        hb = int(min(h[b], cap))
        kb = int(min(k[b], hb))
        lists = batched_plan(b, hb, kb)
        x = dev(uniform_pm1(100 + b, hb * ncols).reshape(hb, ncols)).to(dtype)
        halo = torch.full((hb, ncols), float("nan"), dtype=dtype, device="cuda")
        topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
        req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                           lists["counts"], lists["displs"], topo)
        recv = dev(uniform_pm1(200 + b, hb * ncols).reshape(hb, ncols)).to(dtype)
        P.req_arena_view(req, P.HX_ARENA_RECV, ncols, dtype).copy_(recv)
        g_send = dev(uniform_pm1(300 + b, hb * ncols).reshape(hb, ncols)).to(dtype)
        g_x = torch.full_like(x, float("nan"))
        P.hx_req_bind_grad(req, g_send, g_x)
        mem.append(dict(lists=lists, x=x, halo=halo, req=req, recv=recv, g_send=g_send, g_x=g_x, h=hb))
    return mem


def check_members(mem, ncols, dtype):
    for m in mem:
        send = host(P.req_arena_view(m["req"], P.HX_ARENA_SEND, ncols, dtype))
        assert bits_equal(send, OM.pack(host(m["x"]), m["lists"]["send_idx"]))
        assert bits_equal(host(m["halo"]), host(m["recv"]))
        ptr, perm = OP.transpose_csr(m["lists"]["send_idx"], m["h"])
        assert bits_equal(host(m["g_x"]), OM.pack_transpose(host(m["g_send"]), ptr, perm))


def reset(mem):
    for m in mem:
        m["halo"].fill_(float("nan"))
        m["g_x"].fill_(float("nan"))
        P.req_arena_view(m["req"], P.HX_ARENA_SEND, m["x"].shape[1], m["x"].dtype).fill_(float("nan"))


SCHEDS = [None,
          dict(tile_rows=64, block_threads=256, blocks_per_cu=1, unroll=1, push_pack=1),
          dict(tile_rows=1000, block_threads=512, blocks_per_cu=3, nontemporal=1, unroll=4, push_pack=2),
          dict(tile_rows=4096, block_threads=256, blocks_per_cu=8, per_neighbor=1, push_pack=2),
          dict(tile_rows=17, block_threads=512, blocks_per_cu=2, nontemporal=1, per_neighbor=1, unroll=4,
               push_pack=1),
          dict(tile_rows=333, block_threads=256, blocks_per_cu=4, nontemporal=1, unroll=4, push_pack=1),
          dict(tile_rows=2048, block_threads=256, blocks_per_cu=2, unroll=2, push_pack=1),
          dict(tile_rows=50, block_threads=512, blocks_per_cu=2, unroll=2, push_pack=2, lds_window=1),
          dict(tile_rows=3000, unroll=4, push_pack=2, lds_window=1, per_neighbor=1),
          dict(tile_rows=256, push_pack=2, lds_window=2),
          # 1024 lanes: segmented sums only (gathers run 512, term windows off)
          dict(tile_rows=512, block_threads=1024, blocks_per_cu=8, unroll=4, nontemporal=1),
          dict(tile_rows=100, block_threads=1024, blocks_per_cu=2, unroll=2, lds_window=1, per_neighbor=1),
          # one workgroup per tile (one-shot grid), small segmented-sum term buffers
          dict(tile_rows=24, blocks_per_cu=1 << 20, block_threads=1024, unroll=2),
          dict(tile_rows=300, blocks_per_cu=1 << 20, push_pack=1, unroll=4, nontemporal=1, lds_window=2),
          dict(tile_rows=7, blocks_per_cu=1 << 20, lds_window=1, per_neighbor=1),
          # 8-byte rows two per lane (even tiles; odd job ends are half pairs)
          dict(tile_rows=64, blocks_per_cu=1 << 20, pair_rows=1, unroll=4),
          dict(tile_rows=1000, pair_rows=1, unroll=2, nontemporal=1, per_neighbor=1, push_pack=2),
          dict(tile_rows=33, pair_rows=1, unroll=1),
          # 1024-lane gathers (the push pack runs 512), with windows and pairs
          dict(tile_rows=4096, block_threads=1024, blocks_per_cu=2, lds_window=1, push_pack=2, unroll=2),
          dict(tile_rows=128, block_threads=1024, blocks_per_cu=1 << 20, pair_rows=1, push_pack=1)]


@pytest.mark.parametrize("dtype_name,ncols", [("f64", 16), ("f32", 1), ("f64", 1), ("f32", 64)])
def test_batch_graph_equals_plain_equals_oracle(dtype_name, ncols):
    need_gpu()
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    say("batch", dtype_name, ncols)
    mem = build_members(24, 20000, ncols, dtype)
    reqs = [m["req"] for m in mem]
    for sched in SCHEDS:
        say("  sched", sched)
        b = P.hx_batch_init(reqs, sched=sched)
        reset(mem)
        P.hx_batch_start(b)
        P.hx_batch_wait(b)
        P.hx_batch_backward(b)
        check_members(mem, ncols, dtype)
        for rep in range(2):      # graph replays with eager work in between
            reset(mem)
            torch.cuda.synchronize()
            P.hx_batch_start(b)
            P.hx_batch_wait(b)
            P.hx_batch_backward(b)
            check_members(mem, ncols, dtype)
        reset(mem)
        P.hx_batch_start_plain(b)
        P.hx_batch_wait_plain(b)
        P.hx_batch_backward_plain(b)
        check_members(mem, ncols, dtype)
        b.free()


@pytest.mark.parametrize("dtype_name,ncols", [("f64", 16), ("f64", 1)])
def test_direct_replay_equals_graph_and_oracle(dtype_name, ncols):
    """Start / wait / backward launched directly from the prepared tables give
    the graph replay's results bit for bit, also after a re-prepare (bind)."""
    need_gpu()
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    say("direct replay", dtype_name, ncols)
    mem = build_members(12, 20000, ncols, dtype)
    b = P.hx_batch_init([m["req"] for m in mem])
    assert P.hx_batch_get_replay(b) == P.HX_REPLAY_GRAPH
    P.hx_batch_set_replay(b, P.HX_REPLAY_DIRECT)
    assert P.hx_batch_get_replay(b) == P.HX_REPLAY_DIRECT
    for rep in range(3):
        reset(mem)
        torch.cuda.synchronize()
        P.hx_batch_start(b)
        P.hx_batch_wait(b)
        P.hx_batch_backward(b)
        check_members(mem, ncols, dtype)
    P.hx_batch_set_replay(b, P.HX_REPLAY_GRAPH)
    reset(mem)
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    P.hx_batch_backward(b)
    check_members(mem, ncols, dtype)
    with pytest.raises(P.HXError) as e:
        P.hx_batch_set_replay(b, 2)
    assert e.value.code == P.HX_ERR_ARG
    b.free()


def test_tuner_keeps_results_and_caches(tmp_path, monkeypatch):
    need_gpu()
    import torch
    monkeypatch.setenv("HX_TUNE_CACHE", str(tmp_path / "tune.txt"))
    mem = build_members(16, 30000, 16, torch.float64)
    b = P.hx_batch_init([m["req"] for m in mem])
    P.hx_batch_tune(b)
    scheds = [P.hx_batch_get_sched(b, ph) for ph in range(4)]
    reset(mem)
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    P.hx_batch_backward(b)
    check_members(mem, 16, torch.float64)
    text = (tmp_path / "tune.txt").read_text()
    assert "gfx950" in text and len(text.splitlines()) >= 3
    # a new batch of the same shape picks the cached schedules up
    b2 = P.hx_batch_init([m["req"] for m in mem])
    assert [P.hx_batch_get_sched(b2, ph) for ph in range(4)] == scheds
    assert all(P.hx_batch_bytes(b, ph) > 0 for ph in (0, 2, 3))
    # the tuner also chose a replay; results hold in it
    assert P.hx_batch_get_replay(b) in (P.HX_REPLAY_GRAPH, P.HX_REPLAY_DIRECT)
    reset(mem)
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    P.hx_batch_backward(b)
    check_members(mem, 16, torch.float64)


def test_tuning_cache_keeps_the_staged_backward_apart(tmp_path, monkeypatch):
    """A locality world's staged backward (forwarder sums, then owner sums)
    runs other kernels than its closed-form backward: each is tuned and
    cached under a key of its own, and a new world of either kind picks up
    its own schedule."""
    need_gpu()
    import torch
    from tests.conftest import cached_grid2d
    from tests.gpu_util import gpu_plan
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HX_TUNE_CACHE", str(cache))
    rs, rp, cols = cached_grid2d()
    plan = gpu_plan(rs, rp, cols, 4, "locality")
    n = int(rs[-1])
    H = sum(int(P.hx_plan_field(plan, r, "halo").size) for r in range(len(rs) - 1))
    keep, tuned = [], {}
    for staged in (True, False):
        x = torch.zeros(n, 1, dtype=torch.float64, device="cuda")
        halo = torch.zeros(H, 1, dtype=torch.float64, device="cuda")
        g_halo, g_x = torch.ones_like(halo), torch.zeros_like(x)
        b = P.hx_batch_from_plan(plan, x, halo, flags=P.HX_WORLD_STAGED_BACKWARD if staged else 0)
        P.hx_batch_bind_grad(b, g_halo, g_x)
        P.hx_batch_tune(b)
        tuned[staged] = P.hx_batch_get_sched(b, 3)
        keep += [b, x, halo, g_halo, g_x]
    keys = [ln.split()[0] for ln in cache.read_text().splitlines() if "|p3|" in ln.split()[0]]
    assert any(k.endswith("|staged") for k in keys) and any(not k.endswith("|staged") for k in keys), keys
    for staged in (True, False):
        x = torch.zeros(n, 1, dtype=torch.float64, device="cuda")
        halo = torch.zeros(H, 1, dtype=torch.float64, device="cuda")
        b = P.hx_batch_from_plan(plan, x, halo, flags=P.HX_WORLD_STAGED_BACKWARD if staged else 0)
        P.hx_batch_bind_grad(b, torch.ones_like(halo), torch.zeros_like(x))
        assert P.hx_batch_get_sched(b, 3) == tuned[staged], staged
        b.free()


def test_batch_state_machine():
    need_gpu()
    import torch
    mem = build_members(3, 2000, 2, torch.float32)
    b = P.hx_batch_init([m["req"] for m in mem])
    P.hx_batch_wait(b)
    P.hx_batch_start(b)
    with pytest.raises(P.HXError) as e:
        P.hx_batch_start(b)
    assert e.value.code == P.HX_ERR_STATE
    P.hx_batch_wait(b)
    x64 = torch.zeros(4, 2, dtype=torch.float64, device="cuda")
    topo = P.hx_topo_create(0, 2, [1], [1])
    other = P.hx_neighbor_alltoallv_init(x64, [1], [0], [0], torch.zeros(1, 2, dtype=torch.float64, device="cuda"),
                                         [1], [0], topo)
    with pytest.raises(P.HXError) as e:
        P.hx_batch_init([mem[0]["req"], other])
    assert e.value.code == P.HX_ERR_ARG


@pytest.mark.parametrize("sched", [dict(tile_rows=16, push_pack=1), dict(tile_rows=64, push_pack=1, unroll=2),
                                   dict(tile_rows=4096, push_pack=1), dict(tile_rows=64, push_pack=2),
                                   dict(tile_rows=16, blocks_per_cu=1 << 20, block_threads=1024)])
def test_high_fan_out(sched):
    """Every source row goes to 100 neighbors: push tiles whose entries do not
    fit the staging buffer (64 rows x 100 slots) take the row-parallel form,
    smaller tiles the entry-parallel one; the backward sums 100 terms per row
    (more than a 16-row tile's 4 KiB term buffer holds: such a row is summed
    straight from global memory)."""
    need_gpu()
    import torch
    n, k, C = 90, 100, 16
    say("high fan-out", sched)
    x = dev(uniform_pm1(77, n * C).reshape(n, C))
    idx = np.tile(np.arange(n, dtype=np.int32), k)
    counts = np.full(k, n, np.int32)
    displs = (np.arange(k) * n).astype(np.int32)
    halo = torch.full((k, C), float("nan"), dtype=torch.float64, device="cuda")
    procs = list(range(1, k + 1))
    topo = P.hx_topo_create(0, k + 1, procs, procs)
    req = P.hx_neighbor_alltoallv_init(x, counts, displs, idx, halo, np.ones(k, np.int32),
                                       np.arange(k, dtype=np.int32), topo)
    g_send = dev(uniform_pm1(78, n * k * C).reshape(n * k, C))
    g_x = torch.full_like(x, float("nan"))
    P.hx_req_bind_grad(req, g_send, g_x)
    b = P.hx_batch_init([req], sched=sched)
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    P.hx_batch_backward(b)
    send = host(P.req_arena_view(req, P.HX_ARENA_SEND, C, torch.float64))
    assert bits_equal(send, OM.pack(host(x), idx))
    ptr, perm = OP.transpose_csr(idx, n)
    assert bits_equal(host(g_x), OM.pack_transpose(host(g_send), ptr, perm))
    b.free()


def test_batched256_full_size_all_plans(tmp_path, monkeypatch):
    """The benchmark workload at full size (256 plans, 34.7 M halo rows, 16
    FP64 columns) under the default and the tuned schedules: every plan's
    send arena, halo and backward equal the oracle (the pinned OpenMP loops
    of oracle/cpu_move.c, for speed at this size)."""
    need_gpu()
    import torch
    from oracle import cpu as OC
    OC.build_cpu()
    monkeypatch.setenv("HX_TUNE_CACHE", str(tmp_path / "tune.txt"))
    say("batched256 full size: building 256 plans")
    mem = build_members(256, 10 ** 7, 16, torch.float64)
    hs = np.array([m["h"] for m in mem])
    assert hs.sum() == 34_696_856
    b = P.hx_batch_init([m["req"] for m in mem])
    for tuned in (False, True):
        if tuned:
            P.hx_batch_tune(b)
        say("  tuned" if tuned else "  default", [P.hx_batch_get_sched(b, ph) for ph in (0, 2, 3)])
        reset(mem)
        P.hx_batch_start(b)
        P.hx_batch_wait(b)
        P.hx_batch_backward(b)
        torch.cuda.synchronize()
        for i, m in enumerate(mem):
            idx = m["lists"]["send_idx"]
            send = host(P.req_arena_view(m["req"], P.HX_ARENA_SEND, 16, torch.float64))
            assert bits_equal(send, OC.gather(host(m["x"]), idx)), i
            assert bits_equal(host(m["halo"]), host(m["recv"])), i
            ptr, perm = OP.transpose_csr(idx, m["h"])
            assert bits_equal(host(m["g_x"]), OC.transpose_sum(host(m["g_send"]), ptr, perm)), i
    b.free()
