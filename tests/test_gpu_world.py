"""Whole-decomposition exchange on one GPU (every rank's Start/Wait with the
simulated transfer) vs the oracle; per-rank requests built from a GPU plan."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.conftest import cached_grid2d, cached_grid3d, cached_random_rows
from tests.gpu_util import bits_equal, dev, gpu_plan, host, need_gpu, say
from tests.test_oracle_brute import CASES
from workloads import random_small_csr, uniform_pm1

pytestmark = pytest.mark.gpu


def run_world(plan, x, H, plain_launch=False, sched=None):
    """plain_launch: False = graph replay, True = one launch per rank,
    "direct" = the batched tables launched directly (no graph)."""
    import torch
    halo = torch.full((H, x.shape[1]), float("nan"), dtype=x.dtype, device="cuda")
    b = P.hx_batch_from_plan(plan, x, halo, flags=P.HX_WORLD_SIM_TRANSFER, sched=sched)
    if plain_launch == "direct":
        P.hx_batch_set_replay(b, P.HX_REPLAY_DIRECT)
        P.hx_batch_start(b)
        P.hx_batch_wait(b)
    elif plain_launch:
        P.hx_batch_start_plain(b)
        P.hx_batch_wait_plain(b)
    else:
        P.hx_batch_start(b)
        P.hx_batch_wait(b)
    return b, halo


def check_world_against_oracle(rs, rp, cols, ppn, variant, ncols, dtype_name, seed=11, full_stages=True,
                               node_map="block", n_variants=None):
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn, node_map)
    R = len(rs) - 1
    n = int(rs[-1])
    xh = uniform_pm1(seed, n * ncols).reshape(n, ncols)
    if dtype_name == "f32":
        xh = xh.astype(np.float32)
    x = dev(xh)
    plan = gpu_plan(rs, rp, cols, ppn, variant, node_map)
    H = sum(h.size for h in halos)
    variants = [(False, None), (True, None), (False, dict(push_pack=1, unroll=4, tile_rows=77)),
                (False, dict(push_pack=2, unroll=2, nontemporal=1)),
                (False, dict(push_pack=2, lds_window=1, tile_rows=64, unroll=2)),
                (True, dict(push_pack=2, lds_window=1, unroll=1)),
                (False, dict(push_pack=2, lds_window=2, tile_rows=5000)),
                (False, dict(push_pack=2, lds_window=2, pair_rows=1, tile_rows=50, unroll=4)),
                (True, dict(push_pack=2, lds_window=2, pair_rows=1, blocks_per_cu=1 << 20)),
                ("direct", None), ("direct", dict(push_pack=1, tile_rows=40, blocks_per_cu=1 << 20)),
                (False, dict(push_pack=2, lds_window=1, block_threads=1024, blocks_per_cu=2, tile_rows=300)),
                (False, dict(push_pack=1, pair_rows=1, block_threads=1024, blocks_per_cu=1 << 20)),
                # short rows in 16-byte groups per lane with LDS windows
                (False, dict(push_pack=2, lds_window=1, pair_rows=1, tile_rows=50, unroll=8)),
                (True, dict(push_pack=2, lds_window=1, pair_rows=1, block_threads=1024, blocks_per_cu=2,
                            tile_rows=333, unroll=2)),
                ("direct", dict(push_pack=2, lds_window=1, pair_rows=1, blocks_per_cu=1 << 20, tile_rows=4096,
                                unroll=4, nontemporal=1)),
                (False, dict(push_pack=2, lds_window=1, pair_rows=1, block_threads=256, blocks_per_cu=1,
                             tile_rows=7, unroll=1))]
    variants = variants[:n_variants]
    ref = np.concatenate([xh[h] for h in halos]) if H else np.zeros((0, ncols), xh.dtype)
    out = OM.forward_all([D.plan(r, variant) for r in range(R)], xh, rs) if full_stages else None
    for plain_launch, sched in variants:
        b, halo = run_world(plan, x, H, plain_launch, sched)
        got = host(halo)
        assert bits_equal(got, ref)
        if full_stages:
            send = host(P.batch_arena_view(b, P.HX_ARENA_SEND, ncols, dtype))
            recv = host(P.batch_arena_view(b, P.HX_ARENA_RECV, ncols, dtype))
            for r in range(R):
                s1 = P.hx_batch_arena_offset(b, P.HX_ARENA_SEND, r)
                s2 = P.hx_batch_arena_offset(b, P.HX_ARENA_SEND | 2, r)
                r1 = P.hx_batch_arena_offset(b, P.HX_ARENA_RECV, r)
                r2 = P.hx_batch_arena_offset(b, P.HX_ARENA_RECV | 2, r)
                e1, e2 = out["send1"][r].shape[0], out["send2"][r].shape[0]
                q1, q2 = out["recv1"][r].shape[0], out["recv2"][r].shape[0]
                assert bits_equal(send[s1:s1 + e1], out["send1"][r]), r
                assert bits_equal(send[s2:s2 + e2], out["send2"][r]), r
                assert bits_equal(recv[r1:r1 + q1], out["recv1"][r]), r
                assert bits_equal(recv[r2:r2 + q2], out["recv2"][r]), r
        b.free()


@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
@pytest.mark.parametrize("case", CASES)
def test_world_tiny(case, variant):
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = case
    say("world tiny", case, variant)
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    for ncols, dt in ((1, "f64"), (1, "f32"), (3, "f32"), (16, "f64")):
        check_world_against_oracle(rs, rp, cols, ppn, variant, ncols, dt)


@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_world_grid2d(variant):
    need_gpu()
    say("world grid2d", variant)
    rs, rp, cols = cached_grid2d()
    check_world_against_oracle(rs, rp, cols, 4, variant, 1, "f64")


@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
def test_world_grid3d(variant):
    need_gpu()
    say("world grid3d", variant)
    rs, rp, cols = cached_grid3d()
    check_world_against_oracle(rs, rp, cols, 64, variant, 1, "f64")
    check_world_against_oracle(rs, rp, cols, 64, variant, 8, "f32", full_stages=False)


@pytest.mark.parametrize("dtype_name,variant", [("f64", "locality"), ("f32", "locality"),
                                                ("f64", "locality3")])
def test_world_random_rows_full_size(dtype_name, variant):
    """4096 ranks, locality-aware (2-step, 3-step): every halo equals the
    direct gather x[N_r]."""
    need_gpu()
    import torch
    say("world random_rows", dtype_name, variant)
    rs, rp, cols = cached_random_rows()
    halos = OP.all_halos(rp, cols, rs)
    n = int(rs[-1])
    xh = uniform_pm1(7337, n).reshape(n, 1)
    if dtype_name == "f32":
        xh = xh.astype(np.float32)
    plan = gpu_plan(rs, rp, cols, 128, variant)
    H = sum(h.size for h in halos)
    want = xh[np.concatenate(halos)]
    # default schedule; short rows in 16-byte groups per lane with LDS windows
    # (one-shot and persistent grids) and without
    for sched in (None, dict(pair_rows=1, lds_window=1, unroll=8, tile_rows=16384, block_threads=1024,
                             blocks_per_cu=1 << 20, push_pack=2),
                  dict(pair_rows=1, lds_window=1, unroll=2, tile_rows=3000, block_threads=512, blocks_per_cu=2,
                       push_pack=2),
                  dict(pair_rows=1, lds_window=2, unroll=4, tile_rows=2048, push_pack=2, nontemporal=1)):
        say("  schedule", sched)
        b, halo = run_world(plan, dev(xh), H, sched=sched)
        assert bits_equal(host(halo), want)
        b.free()
    b, halo = run_world(plan, dev(xh), H)
    if variant == "locality3":   # one stage-1 message per node pair that needs one
        inter = 0
        for r in range(4096):
            procs = P.hx_plan_field(plan, r, "s1_procs")
            inter += int(np.sum(procs // 128 != r // 128))
        assert inter == 32 * 31
        # rank 5 aggregates node 0's data for node 5: its own request packs
        # from the node's rows (node-shared memory)
        nb = int(rs[128])
        s1 = P.hx_plan_field(plan, 5, "s1_idx")
        assert s1.size > 0 and int(s1.max()) >= int(rs[6])   # reads node-mates' rows
        req = P.hx_req_from_plan(plan, 5, dev(xh[:nb]), torch.empty(halos[5].size, 1, device="cuda", dtype=halo.dtype))
        P.hx_start(req)
        P.hx_wait(req)
        send = host(P.req_arena_view(req, P.HX_ARENA_SEND, 1, halo.dtype))
        assert bits_equal(send[:s1.size], xh[:nb][s1])
        req.free()


@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_rank_requests_from_plan(variant):
    """One rank's request (its arrays alone): the receive arena is filled with
    what its peers send (oracle transfer), Wait produces the oracle's
    redistribution buffer and halo."""
    need_gpu()
    import torch
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 64)
    plans = [D.plan(r, variant) for r in range(512)]
    n = int(rs[-1])
    C = 4
    xh = uniform_pm1(21, n * C).reshape(n, C)
    out = OM.forward_all(plans, xh, rs)
    plan = gpu_plan(rs, rp, cols, 64, variant)
    for r in (0, 219, 300, 511):
        say("rank request", variant, r)
        x_local = dev(xh[rs[r]:rs[r + 1]])
        halo = torch.full((halos[r].size, C), float("nan"), dtype=torch.float64, device="cuda")
        req = P.hx_req_from_plan(plan, r, x_local, halo)
        P.req_arena_view(req, P.HX_ARENA_RECV, C, torch.float64).copy_(dev(out["arena"][r]))
        P.hx_start(req)
        P.hx_wait(req)
        send = host(P.req_arena_view(req, P.HX_ARENA_SEND, C, torch.float64))
        assert bits_equal(send, np.concatenate([out["send1"][r], out["send2"][r]]))
        assert bits_equal(host(halo), out["halo"][r])
        req.free()


def _node_rows(rs, ppn, r):
    nd = r // ppn
    return int(rs[nd * ppn]), int(rs[min(len(rs) - 1, (nd + 1) * ppn)])


def _check_3step_requests(rs, rp, cols, ppn, ranks, C, seed):
    import torch
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    R = len(rs) - 1
    plans = [D.plan(r, "locality3") for r in range(R)]
    n = int(rs[-1])
    xh = uniform_pm1(seed, n * C).reshape(n, C)
    out = OM.forward_all(plans, xh, rs)
    plan = gpu_plan(rs, rp, cols, ppn, "locality3")
    for r in ranks:
        say("3-step rank request", R, ppn, r)
        a, b = _node_rows(rs, ppn, r)
        x_node = dev(xh[a:b])
        halo = torch.full((halos[r].size, C), float("nan"), dtype=torch.float64, device="cuda")
        req = P.hx_req_from_plan(plan, r, x_node, halo)
        P.req_arena_view(req, P.HX_ARENA_RECV, C, torch.float64).copy_(dev(out["arena"][r]))
        P.hx_start(req)
        P.hx_wait(req)
        send = host(P.req_arena_view(req, P.HX_ARENA_SEND, C, torch.float64))
        assert bits_equal(send, np.concatenate([out["send1"][r], out["send2"][r]])), r
        assert bits_equal(host(halo), out["halo"][r]), r
        # the backward of its own pack, over the node's rows
        E1 = int(plans[r]["s1_idx"].size)
        gh = uniform_pm1(seed + 1000 + r, E1 * C).reshape(E1, C)
        g_x = torch.full((b - a, C), float("nan"), dtype=torch.float64, device="cuda")
        P.hx_req_bind_grad(req, dev(gh), g_x)
        P.hx_backward(req)
        assert bits_equal(host(g_x), OM.pack_transpose(gh, plans[r]["bt_ptr"], plans[r]["bt_perm"])), r
        req.free()


def test_rank_requests_from_3step_plan():
    """One rank's request of a 3-step plan reads the rows of its whole node
    (node-shared memory: an aggregator packs its node-mates' rows): with the
    receive arena filled by the oracle's transfer, Start/Wait give the
    oracle's send arena and halo, and the backward of its pack (over the
    node's rows) the oracle's transpose sum; on the 27-point grid (64 ranks
    per node) an aggregator (5), a receiver (64) and ranks that are
    neither."""
    need_gpu()
    rs, rp, cols = cached_grid3d()
    _check_3step_requests(rs, rp, cols, 64, (0, 5, 64, 219, 300, 511), 3, 23)


@pytest.mark.parametrize("case", CASES)
def test_rank_requests_from_3step_plan_tiny(case):
    """The same on the tiny decompositions (uneven rows, partial last nodes,
    ranks that own nothing), every rank."""
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    _check_3step_requests(rs, rp, cols, ppn, range(R), 2, seed + 5)


@pytest.mark.parametrize("case", [CASES[2], CASES[3], CASES[4]])
def test_3step_requests_in_a_member_batch(case):
    """Every rank's 3-step request (each reading its node's rows, with ranks
    of one node sharing one copy of them) in one member batch: the batched
    pack, redistribution and unpack (receive arenas filled by the oracle's
    transfer) and the batched backward of every request's pack equal the
    oracle bit for bit."""
    need_gpu()
    import torch
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    plans = [D.plan(r, "locality3") for r in range(R)]
    C = 2
    xh = uniform_pm1(seed + 3, int(rs[-1]) * C).reshape(-1, C)
    out = OM.forward_all(plans, xh, rs)
    plan = gpu_plan(rs, rp, cols, ppn, "locality3")
    nodes = {}
    reqs, halos_d, gs, gxs = [], [], [], []
    for r in range(R):
        a, b = _node_rows(rs, ppn, r)
        if r // ppn not in nodes:
            nodes[r // ppn] = dev(xh[a:b])
        halo = torch.full((halos[r].size, C), float("nan"), dtype=torch.float64, device="cuda")
        req = P.hx_req_from_plan(plan, r, nodes[r // ppn], halo)
        E1 = int(plans[r]["s1_idx"].size)
        g = dev(uniform_pm1(seed + 500 + r, E1 * C).reshape(E1, C))
        g_x = torch.full((b - a, C), float("nan"), dtype=torch.float64, device="cuda")
        P.hx_req_bind_grad(req, g, g_x)
        reqs.append(req); halos_d.append(halo); gs.append(g); gxs.append(g_x)
    bt = P.hx_batch_init(reqs)
    for r in range(R):
        P.req_arena_view(reqs[r], P.HX_ARENA_RECV, C, torch.float64).copy_(dev(out["arena"][r]))
    say("3-step member batch", case)
    P.hx_batch_start(bt)
    P.hx_batch_wait(bt)
    P.hx_batch_backward(bt)
    for r in range(R):
        send = host(P.req_arena_view(reqs[r], P.HX_ARENA_SEND, C, torch.float64))
        assert bits_equal(send, np.concatenate([out["send1"][r], out["send2"][r]])), r
        assert bits_equal(host(halos_d[r]), out["halo"][r]), r
        want = OM.pack_transpose(host(gs[r]), plans[r]["bt_ptr"], plans[r]["bt_perm"])
        assert bits_equal(host(gxs[r]), want), r
    bt.free()
    for q in reqs:
        q.free()


@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_launch_phase_matches_graphs(variant):
    """Each phase's kernel launched alone rewrites exactly what the graphs wrote."""
    need_gpu()
    import torch
    n, R, mx, pf, seed, uneven, ppn = case = CASES[4]
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    say("launch_phase", variant, case)
    halos = OP.all_halos(rp, cols, rs)
    H = sum(h.size for h in halos)
    C = 3
    x = dev(uniform_pm1(seed, n * C).reshape(n, C))
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    b, halo = run_world(plan, x, H)
    g_halo = dev(uniform_pm1(seed + 1, H * C).reshape(H, C))
    g_x = torch.full_like(x, float("nan"))
    P.hx_batch_bind_grad(b, g_halo, g_x)
    P.hx_batch_backward(b)
    send_v = P.batch_arena_view(b, P.HX_ARENA_SEND, C, torch.float64)
    ref_send, ref_halo, ref_gx = host(send_v).copy(), host(halo).copy(), host(g_x).copy()
    send_v.fill_(float("nan"))
    halo.fill_(float("nan"))
    g_x.fill_(float("nan"))
    for ph in range(4):
        P.hx_batch_launch_phase(b, ph)
    torch.cuda.synchronize()
    assert bits_equal(host(send_v), ref_send)
    assert bits_equal(host(halo), ref_halo)
    assert bits_equal(host(g_x), ref_gx)
    P.hx_batch_start(b)
    with pytest.raises(P.HXError):
        P.hx_batch_launch_phase(b, 0)
    P.hx_batch_wait(b)
    b.free()


def test_set_sched_applies_and_rejects():
    """hx_batch_set_sched: a phase's schedule is applied (and read back), the
    results stay bit-exact, and an invalid schedule leaves the previous one."""
    need_gpu()
    import torch
    n, R, mx, pf, seed, uneven, ppn = CASES[4]
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    H = sum(h.size for h in halos)
    xh = uniform_pm1(seed, n).reshape(n, 1)
    plan = gpu_plan(rs, rp, cols, ppn, "locality")
    b, halo = run_world(plan, dev(xh), H)
    want = xh[np.concatenate(halos)]
    s1 = dict(tile_rows=24, block_threads=256, blocks_per_cu=3, unroll=2, pair_rows=1, lds_window=1)
    for ph in (0, 1, 2):
        P.hx_batch_set_sched(b, ph, s1)
        got = P.hx_batch_get_sched(b, ph)
        assert (got["tile_rows"], got["block_threads"], got["blocks_per_cu"], got["unroll"], got["pair_rows"],
                got["lds_window"]) == (24, 256, 3, 2, 1, 1)
    halo.fill_(float("nan"))
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    assert bits_equal(host(halo), want)
    with pytest.raises(P.HXError) as e:
        P.hx_batch_set_sched(b, 1, dict(block_threads=300))
    assert e.value.code == P.HX_ERR_ARG
    assert P.hx_batch_get_sched(b, 1)["block_threads"] == 256
    halo.fill_(float("nan"))
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    assert bits_equal(host(halo), want)
    P.hx_batch_start(b)
    with pytest.raises(P.HXError) as e:
        P.hx_batch_set_sched(b, 0, s1)
    assert e.value.code == P.HX_ERR_STATE
    P.hx_batch_wait(b)
    b.free()
