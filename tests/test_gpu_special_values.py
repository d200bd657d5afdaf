"""IEEE special values through every path.

The forward moves (pack, redistribution, unpack, in every kernel form) are
copies, so any 32- or 64-bit pattern -- NaN payloads, infinities,
subnormals, signed zeros -- must arrive bit for bit.  The fixed-order sums of
the backward must keep subnormals (no flush to zero) and equal the oracle bit
for bit; where a sum is NaN only the NaN-ness is compared (IEEE 754 does not
fix which payload a NaN result carries)."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.gpu_util import dev, gpu_plan, host, need_gpu, say
from tests.test_gpu_grad import staged_exchange
from tests.test_oracle_brute import CASES
from workloads import random_small_csr, splitmix64

pytestmark = pytest.mark.gpu

SCHEDS = [None,
          dict(pair_rows=1, lds_window=1, tile_rows=64, unroll=2, push_pack=2),
          dict(pair_rows=2, lds_window=1, tile_rows=100, unroll=1, push_pack=2),
          dict(push_pack=1, tile_rows=33, unroll=4),
          dict(pair_rows=1, lds_window=2, blocks_per_cu=2, tile_rows=4096, unroll=4, push_pack=2, nontemporal=1)]


def random_bits(seed, shape, f32):
    """Arbitrary bit patterns viewed as floats (NaNs with payloads included)."""
    z = splitmix64(seed, 0, int(np.prod(shape)))
    if f32:
        return (z & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).reshape(shape)
    return z.view(np.float64).reshape(shape)


PALETTE64 = np.array([5e-324, 2.2250738585072e-308, -1e-310, 3e-320, 0.0, -0.0, np.inf, -np.inf, np.nan, 1.0, -1.5,
                      1e308, -1e308, 0.25], np.float64)
PALETTE32 = np.array([1e-45, 1.1754942e-38, -1e-40, 3e-42, 0.0, -0.0, np.inf, -np.inf, np.nan, 1.0, -1.5, 3e38,
                      -3e38, 0.25], np.float32)


def special_terms(seed, shape, f32, weights=None):
    """Gradients drawn from a palette of subnormals, signed zeros, infinities,
    NaN, large values (sums that overflow) and ordinary values."""
    pal = PALETTE32 if f32 else PALETTE64
    z = splitmix64(seed, 0, int(np.prod(shape)))
    if weights is None:   # mostly subnormals and zeros, so many sums stay finite
        k = (z % np.uint64(4 * pal.size)).astype(np.int64)
        k = np.where(k < pal.size, k, k % 6)
    else:
        k = (z % np.uint64(pal.size)).astype(np.int64)
    return pal[k].reshape(shape)


def same_bits_or_both_nan(got, want):
    got, want = np.ascontiguousarray(got), np.ascontiguousarray(want)
    if got.shape != want.shape or got.dtype != want.dtype:
        return False
    gn, wn = np.isnan(got), np.isnan(want)
    if not np.array_equal(gn, wn):
        return False
    u = np.uint32 if got.dtype == np.float32 else np.uint64
    return np.array_equal(got.view(u)[~gn], want.view(u)[~wn])


@pytest.mark.parametrize("f32,ncols", [(False, 1), (True, 1), (False, 3), (True, 16)], ids=["f64x1", "f32x1", "f64x3",
                                                                                          "f32x16"])
@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
def test_forward_moves_any_bit_pattern(variant, f32, ncols):
    need_gpu()
    import torch
    for case in (CASES[2], CASES[4]):
        n, R, mx, pf, seed, uneven, ppn = case
        rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
        halos = OP.all_halos(rp, cols, rs)
        H = sum(h.size for h in halos)
        plan = gpu_plan(rs, rp, cols, ppn, variant)
        xh = random_bits(seed + 1000 * ncols, (n, ncols), f32)
        x = dev(xh)
        want = xh[np.concatenate(halos)] if H else np.zeros((0, ncols), xh.dtype)
        for sched in SCHEDS:
            say("special forward", variant, case, f32, ncols, sched)
            halo = torch.zeros(H, ncols, dtype=torch.float32 if f32 else torch.float64, device="cuda")
            b = P.hx_batch_from_plan(plan, x, halo, flags=P.HX_WORLD_SIM_TRANSFER, sched=sched)
            P.hx_batch_start(b)
            P.hx_batch_wait(b)
            got = host(halo)
            u = np.uint32 if f32 else np.uint64
            assert np.array_equal(got.view(u), want.view(u)), sched
            b.free()


@pytest.mark.parametrize("f32,ncols", [(False, 1), (True, 1), (False, 3), (True, 5)], ids=["f64x1", "f32x1", "f64x3",
                                                                                         "f32x5"])
@pytest.mark.parametrize("variant", ["plain", "locality"])
def test_backward_sums_keep_subnormals_and_special_values(variant, f32, ncols):
    """Staged backward of a world (forwarder and owner sums) and the
    closed-form backward, against the oracle, with gradients drawn from
    subnormals, signed zeros, infinities, NaN and overflowing values."""
    need_gpu()
    import torch
    dt = torch.float32 if f32 else torch.float64
    for case in (CASES[2], CASES[4]):
        n, R, mx, pf, seed, uneven, ppn = case
        rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
        halos = OP.all_halos(rp, cols, rs)
        D = OP.Decomposition(halos, rs, ppn)
        for weights in (None, "uniform"):
            say("special backward", variant, case, f32, ncols, weights)
            ex, _ = staged_exchange(rs, rp, cols, ppn, variant, ncols, dt)
            H = ex.halo.shape[0]
            g = special_terms(seed + 77, (H, ncols), f32, weights)
            gy = np.split(g, np.cumsum([h.size for h in halos])[:-1])
            with np.errstate(all="ignore"):
                want = OM.staged_adjoint_reference([D.plan(r, variant) for r in range(R)], gy, rs)["g_x"]
                want_cf = OM.exchange_adjoint_reference(halos, gy, n)
            ex.g_halo.copy_(dev(g))
            P.hx_batch_backward(ex.batch)
            torch.cuda.synchronize()
            got = host(ex.g_x)
            assert same_bits_or_both_nan(got, want)
            if weights is None:   # mostly subnormal terms: their sums must not flush to zero
                tiny = np.finfo(got.dtype).tiny
                sub = (np.abs(want) > 0) & (np.abs(want) < tiny)
                assert sub.any() and np.array_equal(got[sub].view(np.uint32 if f32 else np.uint64),
                                                    want[sub].view(np.uint32 if f32 else np.uint64))
            if variant == "plain":
                assert same_bits_or_both_nan(got, want_cf)


@pytest.mark.parametrize("f32,ncols", [(False, 1), (True, 1), (False, 16), (True, 64)], ids=["f64x1", "f32x1",
                                                                                           "f64x16", "f32x64"])
def test_request_backward_special_values(f32, ncols):
    """One request's backward of its pack (chunked, windowed and one-value
    segmented sums) with special-value gradients, and its pack of arbitrary
    bit patterns (pull and push forms)."""
    need_gpu()
    import torch
    from workloads import batched_plan, batched_plan_sizes
    dt = torch.float32 if f32 else torch.float64
    h_all, k_all = batched_plan_sizes()
    for b in (0, 3):
        h = int(min(h_all[b], 5000))
        lists = batched_plan(b, h, int(min(k_all[b], h)))
        E = int(np.sum(lists["counts"]))
        xh = random_bits(50 + b, (h, ncols), f32)
        x = dev(xh)
        halo = torch.zeros(E, ncols, dtype=dt, device="cuda")
        topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
        req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                           lists["counts"], lists["displs"], topo)
        g = special_terms(60 + b, (E, ncols), f32)
        gx = torch.zeros_like(x)
        P.hx_req_bind_grad(req, dev(g), gx)
        ptr, perm = OP.transpose_csr(lists["send_idx"], h)
        with np.errstate(all="ignore"):
            want = OM.pack_transpose(g, ptr, perm)
        for sched in SCHEDS:
            say("special request", b, f32, ncols, sched)
            batch = P.hx_batch_init([req], sched=sched)
            P.hx_batch_start(batch)
            P.hx_batch_wait(batch)
            u = np.uint32 if f32 else np.uint64
            send = host(P.req_arena_view(req, P.HX_ARENA_SEND, ncols, dt))
            assert np.array_equal(send.view(u), xh[lists["send_idx"]].view(u)), sched
            gx.fill_(float("nan"))
            P.hx_batch_backward(batch)
            torch.cuda.synchronize()
            assert same_bits_or_both_nan(host(gx), want), sched
            batch.free()
        req.free()
