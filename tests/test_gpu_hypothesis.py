"""Property-based GPU parity: hypothesis draws small decompositions (rows,
ranks, entries per row, share of far entries, uneven splits, ranks per node,
placement, plan variant, columns and dtype); for each, the GPU plan, every
stage buffer of the world exchange and the staged backward equal the
oracle's, bit for bit.  Derandomized, so every run takes the same
examples."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.gpu_util import assert_plan_equal, bits_equal, dev, gpu_plan, host, need_gpu, plan_rank, say
from tests.test_gpu_grad import staged_exchange
from workloads import random_small_csr, uniform_pm1

pytestmark = pytest.mark.gpu


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(n=st.integers(1, 300), R=st.integers(1, 24), mx=st.integers(1, 8), pf=st.floats(0.0, 1.0),
       seed=st.integers(0, 10_000), uneven=st.booleans(), ppn=st.integers(1, 7),
       placement=st.sampled_from(["block", "cyclic"]), variant=st.sampled_from(["plain", "locality", "locality3"]),
       ncols=st.sampled_from([1, 2, 3, 16]), f32=st.booleans())
def test_random_decompositions_on_the_gpu(n, R, mx, pf, seed, uneven, ppn, placement, variant, ncols, f32):
    need_gpu()
    import torch
    if variant == "locality3" and placement == "cyclic":
        placement = "block"   # the 3-step variant needs contiguous node rows
    R = min(R, n)
    say("hypothesis", n, R, mx, round(pf, 3), seed, uneven, ppn, placement, variant, ncols, f32)
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn, placement)
    plans = [D.plan(r, variant) for r in range(R)]
    plan = gpu_plan(rs, rp, cols, ppn, variant, placement)
    for r in range(R):
        assert_plan_equal(plan_rank(plan, r), plans[r], f"rank {r}")
    dt = torch.float32 if f32 else torch.float64
    xh = uniform_pm1(seed + 3, n * ncols).reshape(n, ncols)
    if f32:
        xh = xh.astype(np.float32)
    out = OM.forward_all(plans, xh, rs)
    H = sum(h.size for h in halos)
    x = dev(xh)
    halo = torch.full((H, ncols), float("nan"), dtype=dt, device="cuda")
    b = P.hx_batch_from_plan(plan, x, halo, flags=P.HX_WORLD_SIM_TRANSFER)
    P.hx_batch_start(b)
    P.hx_batch_wait(b)
    send = host(P.batch_arena_view(b, P.HX_ARENA_SEND, ncols, dt))
    recv = host(P.batch_arena_view(b, P.HX_ARENA_RECV, ncols, dt))
    for r in range(R):
        s1 = P.hx_batch_arena_offset(b, P.HX_ARENA_SEND, r)
        s2 = P.hx_batch_arena_offset(b, P.HX_ARENA_SEND | 2, r)
        r1 = P.hx_batch_arena_offset(b, P.HX_ARENA_RECV, r)
        r2 = P.hx_batch_arena_offset(b, P.HX_ARENA_RECV | 2, r)
        assert bits_equal(send[s1:s1 + out["send1"][r].shape[0]], out["send1"][r]), r
        assert bits_equal(send[s2:s2 + out["send2"][r].shape[0]], out["send2"][r]), r
        assert bits_equal(recv[r1:r1 + out["recv1"][r].shape[0]], out["recv1"][r]), r
        assert bits_equal(recv[r2:r2 + out["recv2"][r].shape[0]], out["recv2"][r]), r
    want_halo = np.concatenate(out["halo"]) if H else np.zeros((0, ncols), xh.dtype)
    assert bits_equal(host(halo), want_halo)
    b.free()
    # staged backward (the closed form for the plain plan)
    ex, _ = staged_exchange(rs, rp, cols, ppn, variant, ncols, dt, node_map=placement)
    g = uniform_pm1(seed + 5, H * ncols).reshape(H, ncols)
    if f32:
        g = g.astype(np.float32)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want = OM.staged_adjoint_reference(plans, gy, rs)["g_x"]
    ex.g_halo.copy_(dev(g))
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)


@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_world_without_halo_binds_empty_gradients(variant):
    """One rank (no halo entries): its empty halo-gradient buffer may be a
    null pointer; the backward writes +0.0 to every row."""
    need_gpu()
    import torch
    rs, rp, cols = random_small_csr(10, 1, 3, 0.5, 4, False)
    ex, _ = staged_exchange(rs, rp, cols, 2, variant, 2, torch.float64)
    assert ex.halo.shape[0] == 0
    ex.g_x.fill_(float("nan"))
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    got = host(ex.g_x)
    assert np.all(got == 0) and not np.signbit(got).any()


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(members=st.lists(st.tuples(st.integers(0, 10_000), st.integers(1, 3000), st.integers(1, 200)),
                        min_size=1, max_size=6),
       ncols=st.sampled_from([1, 2, 3, 4, 16, 64]), f32=st.booleans(),
       tile=st.sampled_from([0, 1, 7, 64, 300, 4096]), bt=st.sampled_from([0, 256, 512, 1024]),
       bpc=st.sampled_from([0, 1, 2, 8, 1 << 20]), unroll=st.sampled_from([0, 1, 2, 4, 8]),
       nt=st.sampled_from([0, 1, 2]), push=st.sampled_from([0, 1, 2]), win=st.sampled_from([0, 1, 2]),
       pair=st.sampled_from([0, 1, 2]), per_nbr=st.booleans())
def test_member_batches_under_random_schedules(members, ncols, f32, tile, bt, bpc, unroll, nt, push, win, pair,
                                                per_nbr):
    """Batches of requests built from random exchange lists, under a random
    launch schedule: every member's send arena (pack), halo (unpack of its
    receive arena) and backward equal the oracle's."""
    need_gpu()
    import torch
    from workloads import batched_plan
    sched = dict(tile_rows=tile, block_threads=bt, blocks_per_cu=bpc, unroll=unroll, nontemporal=int(nt),
                 push_pack=push, lds_window=win, pair_rows=pair, per_neighbor=int(per_nbr))
    if push == 1 and bt == 1024:
        sched["block_threads"] = 512   # the push pack runs at most 512 lanes
    say("hypothesis batch", members, ncols, f32, sched)
    dt = torch.float32 if f32 else torch.float64
    reqs, keep, want = [], [], []
    for i, (b, h, k) in enumerate(members):
        lists = batched_plan(b, h, min(k, h))
        xh = uniform_pm1(b + 7, h * ncols).reshape(h, ncols)
        rh = uniform_pm1(b + 8, h * ncols).reshape(h, ncols)
        gh = uniform_pm1(b + 9, h * ncols).reshape(h, ncols)
        if f32:
            xh, rh, gh = xh.astype(np.float32), rh.astype(np.float32), gh.astype(np.float32)
        x, halo = dev(xh), torch.full((h, ncols), float("nan"), dtype=dt, device="cuda")
        topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
        req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                           lists["counts"], lists["displs"], topo)
        P.req_arena_view(req, P.HX_ARENA_RECV, ncols, dt).copy_(dev(rh))
        g, gx = dev(gh), torch.full_like(x, float("nan"))
        P.hx_req_bind_grad(req, g, gx)
        ptr, perm = OP.transpose_csr(lists["send_idx"], h)
        reqs.append(req)
        keep.append((x, halo, g, gx, topo))
        want.append((OM.pack(xh, lists["send_idx"]), rh, OM.pack_transpose(gh, ptr, perm)))
    batch = P.hx_batch_init(reqs, sched=sched)
    P.hx_batch_start(batch)
    P.hx_batch_wait(batch)
    P.hx_batch_backward(batch)
    torch.cuda.synchronize()
    for req, (x, halo, g, gx, topo), (w_send, w_halo, w_gx) in zip(reqs, keep, want):
        assert bits_equal(host(P.req_arena_view(req, P.HX_ARENA_SEND, ncols, dt)), w_send)
        assert bits_equal(host(halo), w_halo)
        assert bits_equal(host(gx), w_gx)
    batch.free()
    for req in reqs:
        req.free()


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(n=st.integers(2, 400), R=st.integers(2, 20), mx=st.integers(1, 8), pf=st.floats(0.0, 1.0),
       seed=st.integers(0, 10_000), ppn=st.integers(1, 6), variant=st.sampled_from(["plain", "locality", "locality3"]),
       ncols=st.sampled_from([1, 2, 5]), f32=st.booleans(),
       tile=st.sampled_from([0, 3, 64, 1000]), bt=st.sampled_from([0, 256, 1024]),
       bpc=st.sampled_from([0, 2, 1 << 20]), unroll=st.sampled_from([0, 1, 4]), nt=st.sampled_from([0, 1, 2]),
       win=st.sampled_from([0, 1, 2]), pair=st.sampled_from([0, 1, 2]), direct=st.booleans())
def test_worlds_under_random_schedules(n, R, mx, pf, seed, ppn, variant, ncols, f32, tile, bt, bpc, unroll, nt, win,
                                       pair, direct):
    """A world's exchange and staged backward under a random schedule for all
    four phases, replayed from graphs or launched directly: halos equal the
    direct gather, gradients the oracle's staged adjoint."""
    need_gpu()
    import torch
    R = min(R, n)
    sched = dict(tile_rows=tile, block_threads=bt, blocks_per_cu=bpc, unroll=unroll, nontemporal=int(nt),
                 lds_window=win, pair_rows=pair, push_pack=2)
    say("hypothesis world", n, R, mx, round(pf, 3), seed, ppn, variant, ncols, f32, sched, direct)
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, False)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    plans = [D.plan(r, variant) for r in range(R)]
    dt = torch.float32 if f32 else torch.float64
    ex, _ = staged_exchange(rs, rp, cols, ppn, variant, ncols, dt)
    for ph in range(4):
        P.hx_batch_set_sched(ex.batch, ph, sched)
    P.hx_batch_set_replay(ex.batch, P.HX_REPLAY_DIRECT if direct else P.HX_REPLAY_GRAPH)
    H = ex.halo.shape[0]
    xh = uniform_pm1(seed + 11, n * ncols).reshape(n, ncols)
    g = uniform_pm1(seed + 12, H * ncols).reshape(H, ncols)
    if f32:
        xh, g = xh.astype(np.float32), g.astype(np.float32)
    ex.x.copy_(dev(xh))
    ex.halo.fill_(float("nan"))
    ex.forward()
    torch.cuda.synchronize()
    want_halo = xh[np.concatenate(halos)] if H else np.zeros((0, ncols), xh.dtype)
    assert bits_equal(host(ex.halo), want_halo)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want = OM.staged_adjoint_reference(plans, gy, rs)["g_x"]
    ex.g_halo.copy_(dev(g))
    ex.g_x.fill_(float("nan"))
    ex.backward()
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)


@settings(max_examples=25, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(n=st.integers(2, 300), R=st.integers(1, 16), mx=st.integers(1, 6), pf=st.floats(0.0, 1.0),
       seed=st.integers(0, 10_000), uneven=st.booleans(), ppn=st.integers(1, 5),
       node_map=st.sampled_from(["block", "cyclic"]), variant=st.sampled_from(["plain", "locality", "locality3"]),
       shuffle=st.booleans())
def test_collective_init_random_decompositions(n, R, mx, pf, seed, uneven, ppn, node_map, variant, shuffle):
    """The per-rank locality-aware init on random decompositions, ranks
    joining in a random order with (optionally) shuffled receive orders
    (3-step ranks join with their node's rows)."""
    need_gpu()
    from tests.test_gpu_comm import run_collective
    R = min(R, n)
    if variant == "locality3":
        node_map = "block"   # the 3-step variant needs contiguous node rows
    say("hypothesis collective init", n, R, mx, round(pf, 3), seed, uneven, ppn, node_map, variant, shuffle)
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    run_collective(rs, halos, ppn, variant, node_map, 2, seed + 13, shuffle)


@settings(max_examples=30, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
@given(n=st.integers(1, 500), R=st.integers(1, 20), density=st.floats(0.0, 1.0), seed=st.integers(0, 10_000),
       uneven=st.booleans(), ppn=st.integers(1, 6), node_map=st.sampled_from(["block", "cyclic"]),
       variant=st.sampled_from(["plain", "locality", "locality3"]))
def test_plans_from_arbitrary_halos(n, R, density, seed, uneven, ppn, node_map, variant):
    """Plans built from halos drawn directly (each rank needs a random subset
    of the columns it does not own, from none to all), not from a matrix:
    every field of every rank equals the oracle's."""
    need_gpu()
    from workloads import splitmix64
    if variant == "locality3":
        node_map = "block"
    R = min(R, n)
    if uneven and R > 1:
        cuts = np.sort((splitmix64(seed, 0, R - 1) % np.uint64(n + 1)).astype(np.int64))
        rs = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    else:
        rs = (np.arange(R + 1, dtype=np.int64) * n) // R
    z = splitmix64(seed + 1, 0, R * n)
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    halos = []
    for r in range(R):
        row = u[r * n:(r + 1) * n] < density
        row[rs[r]:rs[r + 1]] = False
        halos.append(np.nonzero(row)[0].astype(np.int64))
    say("hypothesis halos", n, R, round(density, 3), seed, uneven, ppn, node_map, variant)
    D = OP.Decomposition(halos, rs, ppn, node_map)
    hp = np.concatenate([[0], np.cumsum([h.size for h in halos])]).astype(np.int64)
    flat = np.concatenate(halos).astype(np.int32) if hp[-1] else np.zeros(0, np.int32)
    vid = {"plain": P.HX_PLAIN, "locality": P.HX_LOCALITY_2STEP, "locality3": P.HX_LOCALITY_3STEP}[variant]
    plan = P.hx_plan_from_halos(R, rs, ppn, vid, hp, dev(flat) if flat.size else None, node_map=node_map)
    for r in range(R):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"rank {r}")
