"""Segmented sums of rows of one value, one row per lane (schedules with
pair_rows = 1): the owner sums and the staged backward's forwarder sums, bit
for bit against the oracle, with and without LDS term windows, in FP32 and
FP64, on tiny decompositions, the 27-point one and member batches."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.conftest import cached_grid3d
from tests.gpu_util import bits_equal, dev, gpu_plan, host, need_gpu, say
from tests.test_oracle_brute import CASES
from workloads import batched_plan, batched_plan_sizes, random_small_csr, uniform_pm1, uniform_pm1_f32

pytestmark = pytest.mark.gpu

SCHEDS = [dict(pair_rows=1, lds_window=1, tile_rows=16384, block_threads=512, blocks_per_cu=1 << 20, unroll=4),
          dict(pair_rows=1, lds_window=2, tile_rows=64, block_threads=256, blocks_per_cu=1 << 20, unroll=2),
          dict(pair_rows=1, lds_window=1, tile_rows=7, block_threads=256, blocks_per_cu=2, unroll=1),
          dict(pair_rows=1, lds_window=1, tile_rows=300, block_threads=1024, blocks_per_cu=3, unroll=2,
               nontemporal=1)]


def _grads(seed, H, f32):
    g = (uniform_pm1_f32 if f32 else uniform_pm1)(seed, H).reshape(H, 1)
    if H:
        g[0, 0] = -0.0          # a lone -0.0 must survive where it is a row's only term
    return g


@pytest.mark.parametrize("f32", [True, False], ids=["f32", "f64"])
@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
@pytest.mark.parametrize("case", CASES)
def test_staged_and_adjoint_backward_one_value_rows(case, variant, f32):
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    H = sum(h.size for h in halos)
    g = _grads(seed + 41, H, f32)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want_staged = OM.staged_adjoint_reference([D.plan(r, variant) for r in range(R)], gy, rs)["g_x"]
    want_adj = OM.exchange_adjoint_reference(halos, gy, n)
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    dt = torch.float32 if f32 else torch.float64
    for sched in SCHEDS:
        say("one-value segsum", case, variant, "f32" if f32 else "f64", sched)
        for staged, want in ((True, want_staged), (False, want_adj)):
            ex = HaloExchange(plan, n, H, 1, dtype=dt, staged_backward=staged, sched=sched)
            assert P.hx_batch_get_sched(ex.batch, 3)["pair_rows"] == 1
            ex.g_halo.copy_(dev(g))
            ex.g_x.fill_(float("nan"))
            P.hx_batch_backward(ex.batch)
            torch.cuda.synchronize()
            assert bits_equal(host(ex.g_x), want), (staged, sched)
            ex.g_x.fill_(float("nan"))
            P.hx_batch_backward_plain(ex.batch)
            torch.cuda.synchronize()
            assert bits_equal(host(ex.g_x), want), (staged, sched)


def test_staged_backward_grid3d_one_value_rows():
    """27-point 128^3, 512 ranks, locality plan, one FP64 value per row."""
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 64)
    R, n = len(rs) - 1, int(rs[-1])
    H = sum(h.size for h in halos)
    g = _grads(6, H, False)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want = OM.staged_adjoint_reference([D.plan(r, "locality") for r in range(R)], gy, rs)["g_x"]
    plan = gpu_plan(rs, rp, cols, 64, "locality")
    for sched in SCHEDS[:2]:
        say("one-value segsum grid3d", sched)
        ex = HaloExchange(plan, n, H, 1, dtype=torch.float64, staged_backward=True, sched=sched)
        ex.g_halo.copy_(dev(g))
        P.hx_batch_backward(ex.batch)
        torch.cuda.synchronize()
        assert bits_equal(host(ex.g_x), want)


@pytest.mark.parametrize("f32", [True, False], ids=["f32", "f64"])
def test_member_batch_backward_one_value_rows(f32):
    """Requests of the batched workload (high fan-out rows), one value per row."""
    need_gpu()
    import torch
    dt = torch.float32 if f32 else torch.float64
    h_all, k_all = batched_plan_sizes()
    members = []
    for b in (0, 3, 5, 9):
        h = int(min(h_all[b], 60_000))
        lists = batched_plan(b, h, int(min(k_all[b], h)))
        x = torch.zeros(h, 1, dtype=dt, device="cuda")
        halo = torch.zeros(h, 1, dtype=dt, device="cuda")
        topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
        req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                           lists["counts"], lists["displs"], topo)
        E = int(np.sum(lists["counts"]))
        g = _grads(700 + b, E, f32)
        gx = torch.full_like(x, float("nan"))
        P.hx_req_bind_grad(req, dev(g), gx)
        ptr, perm = OP.transpose_csr(lists["send_idx"], h)
        members.append((req, gx, OM.pack_transpose(g, ptr, perm)))
    for sched in SCHEDS:
        say("member one-value segsum", sched)
        batch = P.hx_batch_init([m[0] for m in members], sched=sched)
        for _, gx, _ in members:
            gx.fill_(float("nan"))
        P.hx_batch_backward(batch)
        torch.cuda.synchronize()
        for _, gx, want in members:
            assert bits_equal(host(gx), want)
        batch.free()
