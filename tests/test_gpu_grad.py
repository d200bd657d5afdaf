"""Backward of the exchange: the library's fixed-order transpose sum vs the
oracle (bit-exact) and vs central finite differences; the autograd Function."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.conftest import cached_grid3d, cached_random_rows
from tests.gpu_util import bits_equal, dev, gpu_plan, host, need_gpu, say
from tests.test_oracle_brute import CASES
from workloads import random_small_csr, uniform_pm1, uniform_pm1_f32

pytestmark = pytest.mark.gpu


def exchange_for(rs, rp, cols, ppn, variant, ncols):
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    H = sum(int(P.hx_plan_field(plan, r, "halo").size) for r in range(len(rs) - 1))
    return HaloExchange(plan, int(rs[-1]), H, ncols, dtype=torch.float32), plan


@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
@pytest.mark.parametrize("case", CASES[:6])
def test_backward_tiny_bit_exact(case, variant):
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import halo_gather
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    ex, _ = exchange_for(rs, rp, cols, ppn, variant, 3)
    x = dev(uniform_pm1_f32(seed, n * 3).reshape(n, 3)).requires_grad_(True)
    y = halo_gather(x, ex)
    H = y.shape[0]
    assert bits_equal(host(y), host(x)[np.concatenate(halos)] if H else np.zeros((0, 3), np.float32))
    g = uniform_pm1_f32(seed + 9, H * 3).reshape(H, 3)
    y.backward(dev(g))
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    assert bits_equal(host(x.grad), OM.exchange_adjoint_reference(halos, gy, n))


def test_backward_grid3d_64_columns():
    """The 27-point decomposition with 64 FP32 features per row."""
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import halo_gather
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    n = int(rs[-1])
    C = 64
    say("grad grid3d")
    ex, _ = exchange_for(rs, rp, cols, 64, "plain", C)
    x = dev(uniform_pm1_f32(1, n * C).reshape(n, C)).requires_grad_(True)
    y = halo_gather(x, ex)
    H = y.shape[0]
    g = uniform_pm1_f32(2, H * C).reshape(H, C)
    y.backward(dev(g))
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    assert bits_equal(host(x.grad), OM.exchange_adjoint_reference(halos, gy, n))


def test_backward_random_rows_every_row():
    """Full size (4096 ranks, 64 FP32 columns, the differentiation workload):
    every row of the backward, in 16-column chunks, against the closed-form
    adjoint in ascending rank order (the pinned OpenMP loops of
    oracle/cpu_move.c over the adjoint CSR), and every halo row of the
    forward against the direct gather."""
    need_gpu()
    import torch
    from oracle import cpu as OC
    OC.build_cpu()
    rs, rp, cols = cached_random_rows()
    halos = OP.all_halos(rp, cols, rs)
    n = int(rs[-1])
    C = 64
    say("grad random_rows, every row")
    ex, _ = exchange_for(rs, rp, cols, 128, "plain", C)
    H = ex.halo.shape[0]
    ex.x.copy_(dev(uniform_pm1_f32(5, n * C).reshape(n, C)))
    y = ex.forward()
    g = torch.empty_like(ex.g_halo)
    step = 1 << 22
    for lo in range(0, H, step):
        hi = min(H, lo + step)
        g[lo:hi] = dev(uniform_pm1_f32(6, (hi - lo) * C, start=lo * C).reshape(hi - lo, C))
    ex.g_halo.copy_(g)
    gx = ex.backward()
    torch.cuda.synchronize()
    allcols = np.concatenate(halos)
    # adjoint CSR: column -> halo entries holding it, ascending (= ascending rank)
    perm = np.argsort(allcols, kind="stable").astype(np.int32)
    ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(allcols, minlength=n), out=ptr[1:])
    ptr = ptr.astype(np.int32)
    for c0 in range(0, C, 16):
        vals = np.ascontiguousarray(host(g[:, c0:c0 + 16]))
        want = OC.transpose_sum(vals, ptr, perm)
        assert bits_equal(np.ascontiguousarray(host(gx[:, c0:c0 + 16])), want), c0
        del vals, want
    xs = host(ex.x)
    for lo in range(0, H, step):
        hi = min(H, lo + step)
        assert bits_equal(host(y[lo:hi]), xs[allcols[lo:hi]]), lo


def test_finite_differences():
    """Central differences of L = sum(w * Y) (float64 on the device) at
    h = 1e-3 in FP32, divided by the realised step, against the backward for
    inputs drawn from every fan-out class: |g_fd - g| <= 1e-6 * max(1, |g|)."""
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import halo_gather
    rs, rp, cols = cached_grid3d()
    n = int(rs[-1])
    C = 2
    ex, plan = exchange_for(rs, rp, cols, 64, "plain", C)
    x0 = dev(uniform_pm1_f32(3, n * C).reshape(n, C))
    H = ex.halo.shape[0]
    w = dev(uniform_pm1_f32(4, H * C).reshape(H, C)).double()
    x = x0.clone().requires_grad_(True)
    y = halo_gather(x, ex)
    (y.double() * w).sum().backward()
    grad = host(x.grad)
    halos = [P.hx_plan_field(plan, r, "halo") for r in range(512)]
    counts = np.bincount(np.concatenate(halos), minlength=n)
    rng = np.random.default_rng(1)
    picks = []
    for f in np.unique(counts):
        rows = np.nonzero(counts == f)[0]
        picks += [(int(r), int(rng.integers(C))) for r in rng.choice(rows, size=min(4, rows.size), replace=False)]
    h = np.float32(1e-3)
    for (r, c) in picks:
        v = float(x0[r, c])
        vp, vm = np.float32(v) + h, np.float32(v) - h
        losses = []
        for val in (vp, vm):
            xp = x0.clone()
            xp[r, c] = float(val)
            ex.x.copy_(xp)
            losses.append(float((ex.forward().double() * w).sum()))
        fd = (losses[0] - losses[1]) / (float(vp) - float(vm))
        g = float(grad[r, c])
        assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (r, c, counts[r], fd, g)


def test_finite_differences_random_rows_64_columns():
    """The differentiation workload at full size: random-matrix plan (4096
    ranks), 64 FP32 features.  Central differences of L = sum(w * Y) at
    h = 1e-3, for inputs drawn from every fan-out class, evaluated as the
    float64 sum of w * (Y(x + h) - Y(x - h)) over the halo entries that
    changed (every other entry of that difference is exactly zero, so no
    rounding of the 2.6 G-term loss enters), divided by the realised step,
    against the backward with w as the halo gradient:
    |g_fd - g| <= 1e-6 * max(1, |g|)."""
    need_gpu()
    import torch
    rs, rp, cols = cached_random_rows()
    halos = OP.all_halos(rp, cols, rs)
    n = int(rs[-1])
    C = 64
    say("finite differences random_rows, 64 columns")
    ex, _ = exchange_for(rs, rp, cols, 128, "plain", C)
    H = ex.halo.shape[0]
    x0 = dev(uniform_pm1_f32(9, n * C).reshape(n, C))
    step = 1 << 22
    for lo in range(0, H, step):
        hi = min(H, lo + step)
        ex.g_halo[lo:hi] = dev(uniform_pm1_f32(10, (hi - lo) * C, start=lo * C).reshape(hi - lo, C))
    ex.x.copy_(x0)
    ex.forward()
    gx = ex.backward()
    torch.cuda.synchronize()
    counts = np.bincount(np.concatenate(halos), minlength=n)
    rng = np.random.default_rng(2)
    picks = []
    for f in np.unique(counts):
        rows = np.nonzero(counts == f)[0]
        picks += [(int(r), int(rng.integers(C))) for r in rng.choice(rows, size=min(2, rows.size), replace=False)]
    h = np.float32(1e-3)
    for (r, c) in picks[:48]:
        v = float(x0[r, c])
        vp, vm = np.float32(v) + h, np.float32(v) - h
        ex.x[r, c] = float(vp)
        yp = ex.forward()[:, c].clone()
        ex.x[r, c] = float(vm)
        ym = ex.forward()[:, c]
        ch = (yp != ym).nonzero().flatten()
        assert ch.numel() == counts[r], (r, c)   # every halo entry that reads row r, and no other
        fd = float((ex.g_halo[ch, c].double() * (yp[ch].double() - ym[ch].double())).sum()) / (float(vp) - float(vm))
        ex.x[r, c] = v
        g = float(gx[r, c])
        assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (r, c, counts[r], fd, g)


@pytest.mark.parametrize("sim", [True, False])
@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_world_backward_plain_launch_equals_graph(variant, sim):
    """The one-launch-per-rank form of the world backward gives the same bits
    as the captured graph, and both equal the oracle's adjoint.  Without the
    simulated transport, a plain world's gradient send slots are filled by the
    caller (here: copied from a simulated-transport world of the same plan)."""
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange
    n, R, mx, pf, seed, uneven, ppn = case = CASES[3]
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    H = sum(h.size for h in halos)
    C = 5
    say(f"world backward plain vs graph {variant} sim={sim} case={case}")
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    g = dev(uniform_pm1_f32(seed + 17, H * C).reshape(H, C))
    ref = HaloExchange(plan, n, H, C, dtype=torch.float32, sim_transfer=True)
    ref.g_halo.copy_(g)
    ref.backward()
    ex = ref if sim else HaloExchange(plan, n, H, C, dtype=torch.float32, sim_transfer=False)
    if not sim:
        ex.g_halo.copy_(g)
        if variant == "plain":
            P.batch_arena_view(ex.batch, P.HX_ARENA_GRAD_SEND, C, torch.float32).copy_(
                P.batch_arena_view(ref.batch, P.HX_ARENA_GRAD_SEND, C, torch.float32))
        else:
            with pytest.raises(P.HXError):
                P.hx_batch_arena(ex.batch, P.HX_ARENA_GRAD_SEND)
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    g_graph = host(ex.g_x).copy()
    ex.g_x.fill_(float("nan"))
    P.hx_batch_backward_plain(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), g_graph)
    gy = np.split(host(g), np.cumsum([h.size for h in halos])[:-1])
    assert bits_equal(g_graph, OM.exchange_adjoint_reference(halos, gy, n))


def staged_exchange(rs, rp, cols, ppn, variant, ncols, dtype, sim=True, node_map="block"):
    from paper_2309_07337_amd.autograd import HaloExchange
    plan = gpu_plan(rs, rp, cols, ppn, variant, node_map)
    H = sum(int(P.hx_plan_field(plan, r, "halo").size) for r in range(len(rs) - 1))
    return HaloExchange(plan, int(rs[-1]), H, ncols, dtype=dtype, sim_transfer=sim, staged_backward=True), plan


@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
@pytest.mark.parametrize("case", CASES)
def test_staged_backward_tiny_bit_exact(case, variant):
    """Backward through the plan's stages == the oracle's staged adjoint, bit
    for bit, in the graph, in the one-launch-per-rank form and launched
    directly from the batched tables."""
    need_gpu()
    import torch
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    say("staged backward", variant, case)
    ex, _ = staged_exchange(rs, rp, cols, ppn, variant, 3, torch.float32)
    H = ex.halo.shape[0]
    g = uniform_pm1_f32(seed + 31, H * 3).reshape(H, 3)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want = OM.staged_adjoint_reference([D.plan(r, variant) for r in range(R)], gy, rs)["g_x"]
    ex.g_halo.copy_(dev(g))
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)
    ex.g_x.fill_(float("nan"))
    P.hx_batch_backward_plain(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)
    ex.g_x.fill_(float("nan"))
    P.hx_batch_set_replay(ex.batch, P.HX_REPLAY_DIRECT)   # same tables, no graph
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)
    P.hx_batch_set_replay(ex.batch, P.HX_REPLAY_GRAPH)
    if variant == "plain":   # the closed form, whichever flag
        assert bits_equal(want, OM.exchange_adjoint_reference(halos, gy, n))


def test_staged_backward_grid3d_full():
    """27-point 128^3, 512 ranks, locality plan, 4 FP32 columns: bit-exact
    against the oracle's staged adjoint at full size."""
    need_gpu()
    import torch
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 64)
    say("staged backward grid3d")
    ex, _ = staged_exchange(rs, rp, cols, 64, "locality", 4, torch.float32)
    H = ex.halo.shape[0]
    g = uniform_pm1_f32(5, H * 4).reshape(H, 4)
    gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
    want = OM.staged_adjoint_reference([D.plan(r, "locality") for r in range(len(rs) - 1)], gy, rs)["g_x"]
    ex.g_halo.copy_(dev(g))
    P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    assert bits_equal(host(ex.g_x), want)


def test_staged_backward_random_rows_exact_values():
    """2^22 x 32, 4096 ranks, locality plan, 1 FP64 column: with small-integer
    gradients every grouping is exact, so the staged backward must equal the
    closed-form one (the library's own, checked bit-exact elsewhere) and the
    oracle's closed form on sampled rows."""
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange
    rs, rp, cols = cached_random_rows()
    say("staged backward random_rows")
    plan = gpu_plan(rs, rp, cols, 128, "locality")
    R, n = len(rs) - 1, int(rs[-1])
    H = sum(int(P.hx_plan_field(plan, r, "halo").size) for r in range(R))
    staged = HaloExchange(plan, n, H, 1, dtype=torch.float64, staged_backward=True)
    flat = HaloExchange(plan, n, H, 1, dtype=torch.float64)
    g = ((torch.arange(H, dtype=torch.int64, device="cuda") * 7919) % 17 - 8).to(torch.float64).view(H, 1)
    for ex in (staged, flat):
        ex.g_halo.copy_(g)
        P.hx_batch_backward(ex.batch)
    torch.cuda.synchronize()
    assert torch.equal(staged.g_x, flat.g_x)
    halos = [P.hx_plan_field(plan, r, "halo").astype(np.int64) for r in range(R)]
    allh = np.concatenate(halos)
    gh = host(g)[:, 0]
    rng = np.random.default_rng(3)
    rows = rng.choice(n, 2000, replace=False)
    got = host(staged.g_x)[:, 0]
    order = np.argsort(allh, kind="stable")
    sh = allh[order]
    for c in rows:
        lo, hi = np.searchsorted(sh, c), np.searchsorted(sh, c, side="right")
        assert got[c] == float(np.sum(gh[order[lo:hi]]))


@pytest.mark.parametrize("variant", ["locality", "locality3"])
def test_staged_backward_random_rows_fp32_by_definition(variant):
    """2^22 x 32, 4096 ranks, 2-step or 3-step locality plan, one FP32 value
    per row: the staged backward at full size (with the simulated reverse
    transfers), every owned row of a dozen ranks recomputed from the stages'
    definition (reading R15) by walking the plan's lists: each stage-1 send
    slot that packs the row (3-step: the slots of every rank of its node, in
    ascending rank, then slot), ascending, contributes its receiver's stage-1
    receive-slot sum, which is the receiver's own halo term (if its halo
    reads the slot) followed by the gradients of the redistribution entries
    forwarding that slot, in ascending entry, each being the gradient of the
    halo entry its destination unpacks it into; all additions sequential in
    FP32."""
    need_gpu()
    import torch
    from paper_2309_07337_amd.autograd import HaloExchange
    rs, rp, cols = cached_random_rows()
    say("staged backward random_rows by definition", variant)
    ppn = 128
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    R, n = len(rs) - 1, int(rs[-1])
    hsz = np.array([P.hx_plan_field(plan, r, "halo").size for r in range(R)], np.int64)
    hoff = np.concatenate([[0], np.cumsum(hsz)])
    H = int(hoff[-1])
    ex = HaloExchange(plan, n, H, 1, dtype=torch.float32, staged_backward=True)
    gh = uniform_pm1_f32(9, H)
    ex.g_halo.copy_(dev(gh.reshape(H, 1)))
    P.hx_batch_backward(ex.batch)
    got = host(ex.g_x)[:, 0]
    cache = {}

    def F(r, name):
        key = (r, name)
        if key not in cache:
            cache[key] = P.hx_plan_field(plan, r, name).astype(np.int64)
        return cache[key]

    def inv_unpack(t):
        key = (t, "inv")
        if key not in cache:
            us = F(t, "unpack_src")
            nslots = int(F(t, "r1_counts").sum() + F(t, "r2_counts").sum())
            inv = np.full(nslots, -1, np.int64)
            inv[us] = np.arange(us.size)
            cache[key] = inv
        return cache[key]

    def forwards(t, q):
        """Redistribution entries of t that forward its stage-1 slot q, ascending."""
        key = (t, "fwd")
        if key not in cache:
            s2src = F(t, "s2_src")
            o = np.argsort(s2src, kind="stable")
            cache[key] = (o, s2src[o])
        o, srt = cache[key]
        return o[np.searchsorted(srt, q):np.searchsorted(srt, q, side="right")]

    def seq_sum(vals):
        acc = np.float32(vals[0])
        for v in vals[1:]:
            acc = np.float32(acc + np.float32(v))
        return acc

    def recv1_slot_sum(t, q):
        terms = []
        own = inv_unpack(t)[q]
        if own >= 0:
            terms.append(gh[hoff[t] + own])
        s2d, s2p = F(t, "s2_displs"), F(t, "s2_procs")
        for e in forwards(t, q):
            m2 = int(np.searchsorted(s2d, e, side="right") - 1)
            d = int(s2p[m2])
            pos = int(np.nonzero(F(d, "r2_procs") == t)[0][0])
            slot = int(F(d, "r1_counts").sum()) + int(F(d, "r2_displs")[pos]) + int(e - s2d[m2])
            j = inv_unpack(d)[slot]
            assert j >= 0
            terms.append(gh[hoff[d] + j])
        assert terms, (t, q)
        return seq_sum(terms)

    def packers(r):
        """(rank, global row of each of its send slots) of the ranks whose packs read r's rows."""
        if variant == "locality":
            return [(r, int(rs[r]) + F(r, "s1_idx"))]
        nd = r // ppn
        base = int(rs[nd * ppn])
        return [(q, base + F(q, "s1_idx")) for q in range(nd * ppn, min(R, (nd + 1) * ppn))]

    checked = 0
    for r in (0, 1, 1511, 2048, 2300, 4095, 777, 3001, 127, 128, 3968, 1023):
        # every send slot packing one of r's rows, in ascending (rank, slot)
        q_all, k_all, row_all = [], [], []
        for q, rows in packers(r):
            sel = np.nonzero((rows >= rs[r]) & (rows < rs[r + 1]))[0]
            q_all.append(np.full(sel.size, q)); k_all.append(sel); row_all.append(rows[sel])
        q_all, k_all, row_all = np.concatenate(q_all), np.concatenate(k_all), np.concatenate(row_all)
        order = np.argsort(row_all, kind="stable")
        bounds = np.searchsorted(row_all[order], np.arange(int(rs[r]), int(rs[r + 1]) + 1))
        for lc in range(int(rs[r + 1] - rs[r])):
            sl = order[bounds[lc]:bounds[lc + 1]]          # ascending (rank, slot)
            if sl.size == 0:
                want = np.float32(0.0)
            else:
                parts = []
                for i in sl:
                    q, k = int(q_all[i]), int(k_all[i])
                    s1d, s1p = F(q, "s1_displs"), F(q, "s1_procs")
                    m = int(np.searchsorted(s1d, k, side="right") - 1)
                    t = int(s1p[m])
                    pos = int(np.nonzero(F(t, "r1_procs") == q)[0][0])
                    parts.append(recv1_slot_sum(t, int(F(t, "r1_displs")[pos]) + int(k - s1d[m])))
                want = seq_sum(parts)
            c = int(rs[r]) + lc
            assert got[c].view(np.uint32) == np.float32(want).view(np.uint32), (variant, r, lc, sl.size)
            checked += 1
    say("  rows checked:", checked)
