"""Cyclic (round-robin) rank-to-node placement on the GPU: plans, the whole-
decomposition exchange, per-rank requests and the staged backward against
the oracle under the same placement, bit for bit (integer lists exact,
values bit-exact).  Under this placement the 5-point grid's neighbors of a
rank sit on other nodes, so every message crosses a node and partners
forward to their node-mates."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.conftest import cached_grid2d, cached_grid3d, cached_random_rows
from tests.gpu_util import assert_plan_equal, bits_equal, dev, gpu_plan, host, need_gpu, plan_rank, say
from tests.test_gpu_grad import staged_exchange
from tests.test_gpu_world import check_world_against_oracle, run_world
from tests.test_oracle_brute import CASES
from workloads import random_small_csr, uniform_pm1, uniform_pm1_f32

pytestmark = pytest.mark.gpu

CYC = "cyclic"


def _staged_backward_check(rs, rp, cols, ppn, ncols, seed):
    import torch
    halos = OP.all_halos(rp, cols, rs)
    R = len(rs) - 1
    D = OP.Decomposition(halos, rs, ppn, CYC)
    ex, _ = staged_exchange(rs, rp, cols, ppn, "locality", ncols, torch.float32, node_map=CYC)
    H = ex.halo.shape[0]
    g = uniform_pm1_f32(seed, H * ncols).reshape(H, ncols)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want = OM.staged_adjoint_reference([D.plan(r, "locality") for r in range(R)], gy, rs)["g_x"]
    ex.g_halo.copy_(dev(g))
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)
    ex.g_x.fill_(float("nan"))
    P.hx_batch_backward_plain(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)


@pytest.mark.parametrize("case", CASES)
def test_tiny_plans_world_and_backward(case):
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn, CYC)
    for variant in ("plain", "locality"):
        say("cyclic tiny", case, variant)
        plan = gpu_plan(rs, rp, cols, ppn, variant, CYC)
        for r in range(R):
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"{variant} rank {r}")
    for ncols, dt in ((1, "f64"), (1, "f32"), (3, "f32")):
        check_world_against_oracle(rs, rp, cols, ppn, "locality", ncols, dt, node_map=CYC, n_variants=6)
    _staged_backward_check(rs, rp, cols, ppn, 3, seed + 5)


@pytest.mark.parametrize("seed", range(6))
def test_random_shapes(seed):
    need_gpu()
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(50, 3000))
    R = int(rng.integers(2, 40))
    ppn = int(rng.integers(1, 9))
    say("cyclic random plan", seed, n, R, ppn)
    rs, rp, cols = random_small_csr(n, R, int(rng.integers(1, 12)), float(rng.random()), 300 + seed,
                                    bool(seed % 2))
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn, CYC)
    plan = gpu_plan(rs, rp, cols, ppn, "locality", CYC)
    for r in range(R):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, "locality"), f"rank {r}")


@pytest.mark.parametrize("ppn", [3, 4])
def test_grid2d(ppn):
    """5-point 512 x 512 grid in 16 strips: rank 5's neighbors 4 and 6 sit on
    other nodes, and the exchange forwards entries on every node."""
    need_gpu()
    rs, rp, cols = cached_grid2d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn, CYC)
    say("cyclic grid2d plan", ppn)
    plan = gpu_plan(rs, rp, cols, ppn, "locality", CYC)
    for r in range(16):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, "locality"), f"rank {r}")
    s1 = P.hx_plan_field(plan, 5, "s1_procs")
    assert s1.size and all(D.node(int(q)) != D.node(5) for q in s1)
    assert sum(int(P.hx_plan_field(plan, r, "s2_counts").sum()) for r in range(16)) > 0
    say("cyclic grid2d world", ppn)
    check_world_against_oracle(rs, rp, cols, ppn, "locality", 1, "f64", node_map=CYC, n_variants=6)
    say("cyclic grid2d staged backward", ppn)
    _staged_backward_check(rs, rp, cols, ppn, 2, 40 + ppn)


def test_grid3d():
    """27-point 128^3, 512 ranks on 8 nodes of 64: plans of every rank, the
    exchange with every stage buffer, per-rank requests and the staged
    backward."""
    need_gpu()
    import torch
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 64, CYC)
    plans = [D.plan(r, "locality") for r in range(512)]
    say("cyclic grid3d plan")
    plan = gpu_plan(rs, rp, cols, 64, "locality", CYC)
    for r in range(512):
        assert_plan_equal(plan_rank(plan, r), plans[r], f"rank {r}")
    say("cyclic grid3d world")
    check_world_against_oracle(rs, rp, cols, 64, "locality", 1, "f64", node_map=CYC, n_variants=4)
    say("cyclic grid3d rank requests")
    n, C = int(rs[-1]), 2
    xh = uniform_pm1(23, n * C).reshape(n, C)
    out = OM.forward_all(plans, xh, rs)
    for r in (0, 5, 300, 511):
        x_local = dev(xh[rs[r]:rs[r + 1]])
        halo = torch.full((halos[r].size, C), float("nan"), dtype=torch.float64, device="cuda")
        req = P.hx_req_from_plan(plan, r, x_local, halo)
        P.req_arena_view(req, P.HX_ARENA_RECV, C, torch.float64).copy_(dev(out["arena"][r]))
        P.hx_start(req)
        P.hx_wait(req)
        send = host(P.req_arena_view(req, P.HX_ARENA_SEND, C, torch.float64))
        assert bits_equal(send, np.concatenate([out["send1"][r], out["send2"][r]])), r
        assert bits_equal(host(halo), out["halo"][r]), r
        req.free()
    say("cyclic grid3d staged backward")
    _staged_backward_check(rs, rp, cols, 64, 4, 77)


def test_random_rows_full_size():
    """2^22 rows in 4096 ranks, 32 nodes of 128 ranks dealt round robin:
    sampled ranks' plans against the oracle, and every halo of the exchange
    equal to the direct gather."""
    need_gpu()
    rs, rp, cols = cached_random_rows()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 128, CYC)
    say("cyclic random_rows plan")
    plan = gpu_plan(rs, rp, cols, 128, "locality", CYC)
    for r in (0, 31, 1511, 4095):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, "locality"), f"rank {r}")
    n = int(rs[-1])
    xh = uniform_pm1(2309, n).reshape(n, 1)
    H = sum(h.size for h in halos)
    say("cyclic random_rows world")
    b, halo = run_world(plan, dev(xh), H)
    assert bits_equal(host(halo), xh[np.concatenate(halos)])
    b.free()
