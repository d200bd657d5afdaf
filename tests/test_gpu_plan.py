"""GPU plan kernels vs the oracle, element for element (integer arrays: bit-exact).

Covers halo discovery, owner segmentation (receive lists), the send-list
transpose, the 2-step and 3-step locality lists (node dedup, stage-1
aggregated messages, redistribution lists, unpack map) and the transpose of
the pack map.
"""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import plan as OP
from tests.conftest import cached_grid2d, cached_grid3d, cached_random_rows
from tests.gpu_util import assert_plan_equal, dev, gpu_plan, host, need_gpu, plan_rank, say, variant_id
from tests.test_oracle_brute import CASES
from workloads import random_small_csr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", ["plain", "locality", "locality3"])
@pytest.mark.parametrize("case", CASES)
def test_tiny_decompositions(case, variant):
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = case
    say("plan tiny", case, variant)
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    plan = gpu_plan(rs, rp, cols, ppn, variant)
    for r in range(R):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"rank {r}")


@pytest.mark.parametrize("variant,node_map", [("locality", "block"), ("locality", "cyclic"), ("locality3", "block")])
def test_more_ranks_per_node_than_ranks(variant, node_map):
    """ppn above the rank count (up to INT32_MAX) is one node of every rank:
    the plan equals the oracle's for ppn = R, and records R."""
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = CASES[5]
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    D = OP.Decomposition(OP.all_halos(rp, cols, rs), rs, R, node_map)
    for big in (R + 1, 1000, 2 ** 31 - 1):
        say("plan ppn", variant, node_map, big)
        plan = gpu_plan(rs, rp, cols, big, variant, node_map)
        assert P.hx_plan_describe(plan)["ppn"] == R
        for r in range(R):
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"ppn {big}, rank {r}")


@pytest.mark.parametrize("seed", range(6))
def test_more_random_shapes(seed):
    need_gpu()
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50, 3000))
    R = int(rng.integers(2, 40))
    ppn = int(rng.integers(1, 9))
    say("plan random", seed, n, R, ppn)
    rs, rp, cols = random_small_csr(n, R, int(rng.integers(1, 12)), float(rng.random()), 100 + seed,
                                    bool(seed % 2))
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    for variant in ("plain", "locality", "locality3"):
        plan = gpu_plan(rs, rp, cols, ppn, variant)
        for r in range(R):
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"{variant} rank {r}")


def test_grid2d_all_ranks():
    need_gpu()
    rs, rp, cols = cached_grid2d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 4)
    for variant in ("plain", "locality", "locality3"):
        say("plan grid2d", variant)
        plan = gpu_plan(rs, rp, cols, 4, variant)
        for r in range(16):
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"{variant} rank {r}")


def test_grid3d_all_ranks():
    need_gpu()
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 64)
    for variant in ("plain", "locality", "locality3"):
        say("plan grid3d", variant)
        plan = gpu_plan(rs, rp, cols, 64, variant)
        for r in range(512):
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"{variant} rank {r}")


def test_random_rows_sampled_ranks():
    """Full-size random workload: the ranks the oracle can afford, incl. the
    one with the most neighbors, the first, the last and a few others."""
    need_gpu()
    rs, rp, cols = cached_random_rows()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 128)
    sample = [0, 1, 31, 127, 128, 1511, 2048, 3001, 4095]
    for variant in ("plain", "locality", "locality3"):
        say("plan random_rows", variant)
        plan = gpu_plan(rs, rp, cols, 128, variant)
        for r in sample:
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"{variant} rank {r}")
        # every rank's halo, and the totals
        allh = np.concatenate([P.hx_plan_field(plan, r, "halo") for r in range(4096)])
        assert np.array_equal(allh, np.concatenate(halos))


def test_from_halos_matches_from_csr_and_validates():
    need_gpu()
    rs, rp, cols = random_small_csr(300, 12, 6, 0.5, 77, False)
    for variant in ("plain", "locality", "locality3"):
        a = gpu_plan(rs, rp, cols, 3, variant)
        hs = [P.hx_plan_field(a, r, "halo") for r in range(12)]
        hp = np.concatenate([[0], np.cumsum([h.size for h in hs])])
        b = P.hx_plan_from_halos(12, rs, 3, variant_id(variant), hp,
                                 dev(np.concatenate(hs).astype(np.int32)))
        for r in range(12):
            assert_plan_equal(plan_rank(b, r), plan_rank(a, r), f"rank {r}")
    hs = [P.hx_plan_field(a, r, "halo") for r in range(12)]
    hp = np.concatenate([[0], np.cumsum([h.size for h in hs])])
    flat = np.concatenate(hs).astype(np.int32)
    j = int(np.argmax(np.diff(hp) > 2))
    bad = flat.copy()
    bad[hp[j]], bad[hp[j] + 1] = bad[hp[j] + 1], bad[hp[j]]      # not increasing
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(12, rs, 3, 0, hp, dev(bad))
    assert e.value.code == P.HX_ERR_RANGE
    bad = flat.copy()
    bad[hp[j]] = rs[j]                                          # owned by its own rank
    with pytest.raises(P.HXError) as e:
        P.hx_plan_from_halos(12, rs, 3, 0, hp, dev(np.sort(bad)))
    assert e.value.code == P.HX_ERR_RANGE
    bad = cols.copy()
    bad[5] = 300                                                # column out of range
    with pytest.raises(P.HXError) as e:
        gpu_plan(rs, rp, bad, 3, "plain")
    assert e.value.code == P.HX_ERR_RANGE


def test_degenerate_decompositions():
    need_gpu()
    # one rank: no halo at all; empty ranks; a rank with no rows
    for (n, R, uneven) in [(40, 1, False), (20, 6, True), (5, 5, False)]:
        rs, rp, cols = random_small_csr(n, R, 4, 0.7, 9, uneven)
        halos = OP.all_halos(rp, cols, rs)
        for ppn in (1, 2, R):
            D = OP.Decomposition(halos, rs, ppn)
            for variant in ("plain", "locality"):
                plan = gpu_plan(rs, rp, cols, ppn, variant)
                for r in range(R):
                    assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"n{n} R{R} ppn{ppn} r{r}")


@pytest.fixture
def bitmap_budget(monkeypatch):
    """Sets the halo-discovery bitmap budget (bytes) for the calls of a test."""
    def set_budget(nbytes):
        monkeypatch.setenv("HX_PLAN_BITMAP_BYTES", str(int(nbytes)))
    return set_budget


@pytest.mark.parametrize("case", CASES)
def test_halo_discovery_one_rank_at_a_time(case, bitmap_budget):
    """A bitmap budget below two ranks' bitmaps: every rank's halo is
    discovered alone, and the plans still equal the oracle's."""
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, ppn)
    bitmap_budget(1)
    for variant in ("plain", "locality"):
        say("plan one rank per bitmap group", case, variant)
        plan = gpu_plan(rs, rp, cols, ppn, variant)
        for r in range(R):
            assert_plan_equal(plan_rank(plan, r), D.plan(r, variant), f"{variant} rank {r}")


def test_halo_discovery_in_groups_random_rows(bitmap_budget):
    """The 2^22-row matrix (2 GiB of bitmaps for 4096 ranks) discovered 128
    ranks at a time (64 MiB): every halo equals the oracle's, sampled ranks'
    full plans too."""
    need_gpu()
    rs, rp, cols = cached_random_rows()
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 128)
    bitmap_budget(64 << 20)
    say("plan random_rows in bitmap groups")
    plan = gpu_plan(rs, rp, cols, 128, "locality")
    for r in range(4096):
        assert np.array_equal(P.hx_plan_field(plan, r, "halo"), halos[r]), r
    for r in (0, 127, 128, 1511, 4095):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, "locality"), f"rank {r}")


@pytest.mark.parametrize("variant,node_map", [("plain", "block"), ("locality", "cyclic"), ("locality3", "block")])
def test_plan_save_and_restore(tmp_path, variant, node_map):
    """A saved plan (27-point grid, 512 ranks) is rebuilt from its halos with
    every field equal, and its description round-trips; a tampered file is
    refused."""
    need_gpu()
    from paper_2309_07337_amd.planio import load_plan, save_plan
    rs, rp, cols = cached_grid3d()
    plan = gpu_plan(rs, rp, cols, 64, variant, node_map)
    d = P.hx_plan_describe(plan)
    assert d["nranks"] == 512 and d["n"] == 128 ** 3 and d["ppn"] == 64 and d["node_map"] == node_map
    assert d["variant"] == variant_id(variant) and np.array_equal(d["row_starts"], rs)
    off, h = P.hx_plan_field_all(plan, "halo")
    assert np.array_equal(h[off[219]:off[220]], P.hx_plan_field(plan, 219, "halo"))
    path = tmp_path / "plan.npz"
    say("plan save/restore", variant, node_map)
    save_plan(plan, path)
    back = load_plan(path)
    for r in (0, 219, 511):
        assert_plan_equal(plan_rank(back, r), plan_rank(plan, r), f"rank {r}")
    z = dict(np.load(path))
    z["unpack_src"] = z["unpack_src"].copy()
    z["unpack_src"][0] ^= 1
    np.savez(tmp_path / "bad.npz", **z)
    with pytest.raises(ValueError):
        load_plan(tmp_path / "bad.npz")


def test_plan_and_exchange_at_the_rank_cap():
    """HX_PLAN_MAX_RANKS ranks (16384) of a 2^21-row random matrix (128 rows
    per rank, 8 entries per row, 64 ranks per node): halo discovery in four
    1 GiB bitmap groups, sampled ranks' full locality plans against the
    oracle, every halo, and the exchange of all ranks equal to the direct
    gather."""
    need_gpu()
    import torch
    from tests.test_gpu_world import run_world
    from workloads import equal_row_starts, random_rows, uniform_pm1
    R = P.HX_PLAN_MAX_RANKS
    n = 1 << 21
    rp, cols = random_rows(n, 8, R, 77)
    rs = equal_row_starts(n, R)
    halos = OP.all_halos(rp, cols, rs)
    D = OP.Decomposition(halos, rs, 64)
    say("plan at the rank cap")
    plan = gpu_plan(rs, rp, cols, 64, "locality")
    off, h = P.hx_plan_field_all(plan, "halo")
    assert np.array_equal(np.diff(off), [x.size for x in halos])
    assert np.array_equal(h, np.concatenate(halos))
    for r in (0, 63, 64, 8191, R - 1):
        assert_plan_equal(plan_rank(plan, r), D.plan(r, "locality"), f"rank {r}")
    say("exchange at the rank cap")
    xh = uniform_pm1(78, n).reshape(n, 1)
    b, halo = run_world(plan, dev(xh), int(off[-1]))
    assert np.array_equal(host(halo), xh[h])
    b.free()
    del plan
    torch.cuda.empty_cache()
