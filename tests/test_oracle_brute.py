"""Pins of the oracle by brute force on tiny decompositions (no GPU).

Each check is written independently of the oracle's code path: Python sets
and explicit loops for the halo and the node dedup, the direct global gather
x[N_r] for the exchange result, explicit per-row loops for the fixed-order
backward.  A dropped term, a wrong index or a transposed operand in the
oracle fails at least one of them.
"""
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import move as M
from oracle import plan as P
from workloads import random_small_csr, uniform_pm1

CASES = [
    # (n, R, max_nnz_row, p_far, seed, uneven, ppn)
    (40, 4, 4, 0.3, 1, False, 2),
    (64, 8, 5, 0.5, 2, False, 4),
    (64, 8, 5, 0.5, 2, False, 3),      # partial last node
    (97, 7, 6, 0.4, 3, True, 2),       # uneven split, empty ranks possible
    (128, 16, 3, 0.9, 4, False, 4),
    (200, 10, 8, 0.2, 5, True, 3),
    (256, 16, 6, 0.6, 6, False, 16),   # one node
    (256, 16, 6, 0.6, 6, False, 1),    # one rank per node
    (33, 5, 7, 1.0, 7, False, 2),
    (10, 10, 3, 0.5, 8, False, 3),     # one row per rank
]


def brute_halo(row_starts, row_ptr, cols, r):
    lo, hi = int(row_starts[r]), int(row_starts[r + 1])
    s = set()
    for i in range(lo, hi):
        for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            c = int(cols[e])
            if not (lo <= c < hi):
                s.add(c)
    return sorted(s)


def build(case, placement="block"):
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = P.all_halos(rp, cols, rs)
    return rs, rp, cols, halos, P.Decomposition(halos, rs, ppn, placement)


def placement_fns(R, ppn, placement):
    """Node of a rank, the ranks of a node (ascending) and a rank's partner
    on a node, written out independently of the oracle (reading R2)."""
    NN = (R + ppn - 1) // ppn
    if placement == "block":
        node = lambda p: p // ppn
        lrank = lambda p: p % ppn
    else:
        node = lambda p: p % NN
        lrank = lambda p: p // NN
    members = lambda m: [s for s in range(R) if node(s) == m]

    def partner(q, m):
        mem = members(m)
        want = lrank(q) % len(mem)
        return [s for s in mem if lrank(s) == want][0]
    return node, members, partner, NN


PLACEMENTS = ["block", "cyclic"]


@pytest.mark.parametrize("case", CASES)
def test_halo_matches_brute_force(case):
    rs, rp, cols, halos, _ = build(case)
    for r in range(len(rs) - 1):
        assert list(halos[r]) == brute_halo(rs, rp, cols, r)


@pytest.mark.parametrize("placement", PLACEMENTS)
@pytest.mark.parametrize("variant", ["plain", "locality"])
@pytest.mark.parametrize("case", CASES)
def test_exchange_equals_direct_global_gather(case, variant, placement):
    rs, rp, cols, halos, D = build(case, placement)
    R = len(rs) - 1
    n = int(rs[-1])
    plans = [D.plan(r, variant) for r in range(R)]
    for C in (1, 3):
        x = uniform_pm1(99, n * C).reshape(n, C)
        out = M.forward_all(plans, x, rs)
        for r in range(R):
            ref = x[np.asarray(brute_halo(rs, rp, cols, r), np.int64)]
            assert np.array_equal(out["halo"][r], ref)


@pytest.mark.parametrize("case", CASES)
def test_plain_symmetry_and_conservation(case):
    rs, rp, cols, halos, D = build(case)
    R = len(rs) - 1
    plans = [D.plain_plan(r) for r in range(R)]
    tot_e = sum(p["s1_idx"].size for p in plans)
    tot_h = sum(h.size for h in halos)
    assert tot_e == tot_h
    for q in range(R):
        p = plans[q]
        for s, c, d in zip(p["s1_procs"], p["s1_counts"], p["s1_displs"]):
            sent = set((p["s1_idx"][d:d + c] + rs[q]).tolist())
            need = {x for x in brute_halo(rs, rp, cols, s) if rs[q] <= x < rs[q + 1]}
            assert sent == need and c == len(need)
            # the receiver lists q with the same count
            pr = plans[s]
            k = list(pr["r1_procs"]).index(q)
            assert pr["r1_counts"][k] == c
        assert q not in list(p["s1_procs"]) and q not in list(p["r1_procs"])
        assert list(p["s1_procs"]) == sorted(set(p["s1_procs"].tolist()))
        assert np.all(p["s1_counts"] > 0) and np.all(p["r1_counts"] > 0)


@pytest.mark.parametrize("placement", PLACEMENTS)
@pytest.mark.parametrize("case", CASES)
def test_locality_dedup_and_routing(case, placement):
    """A value crosses from rank q to node m at most once, all of node m's needs
    from q cross, inter-node traffic only goes to partners, forwarding stays
    on-node, and every halo entry is delivered exactly once."""
    rs, rp, cols, halos, D = build(case, placement)
    R = len(rs) - 1
    node, members, partner, NN = placement_fns(R, D.ppn, placement)
    plans = [D.locality_plan(r) for r in range(R)]
    need = [set(brute_halo(rs, rp, cols, r)) for r in range(R)]
    for q in range(R):
        p = plans[q]
        inter = {}
        for t, c, d in zip(p["s1_procs"], p["s1_counts"], p["s1_displs"]):
            vals = (p["s1_idx"][d:d + c] + rs[q]).tolist()
            assert len(vals) == len(set(vals))
            if node(t) != node(q):
                assert node(t) not in inter          # one message per remote node
                assert t == partner(q, node(t))      # to the partner on that node
                inter[node(t)] = set(vals)
            else:
                assert set(vals) == {x for x in need[t] if rs[q] <= x < rs[q + 1]}
        for m in range(NN):
            if m == node(q):
                continue
            want = set()
            for s in members(m):
                want |= {x for x in need[s] if rs[q] <= x < rs[q + 1]}
            assert inter.get(m, set()) == want
        for t in p["s2_procs"]:
            assert node(t) == node(q) and t != q
    # exactly-once delivery, using x[i] = i so every arena slot names its column
    n = int(rs[-1])
    x = np.arange(n, dtype=np.float64).reshape(n, 1)
    out = M.forward_all(plans, x, rs)
    for r in range(R):
        p = plans[r]
        R1 = out["recv1"][r].shape[0]
        src = p["unpack_src"].astype(np.int64)
        assert src.size == len(set(src.tolist()))           # no slot read twice
        assert np.all(src[src >= R1] < R1 + out["recv2"][r].shape[0])
        # every stage-2 slot is used by the unpack exactly once
        assert sorted(src[src >= R1].tolist()) == list(range(R1, R1 + out["recv2"][r].shape[0]))
        assert out["arena"][r][src, 0].tolist() == sorted(need[r])
        direct = sum(c for t, c in zip(p["r1_procs"], p["r1_counts"]) if node(t) == node(r))
        self_ = int(np.sum((src < R1))) - direct
        assert direct + self_ + out["recv2"][r].shape[0] == halos[r].size


@pytest.mark.parametrize("placement", PLACEMENTS)
@pytest.mark.parametrize("case", [c for c in CASES])
def test_locality_special_cases(case, placement):
    """ppn == 1 (every neighbor remote, nothing to merge) and one node (no
    inter-node traffic) both reduce the 2-step plan to the plain plan."""
    n, R, mx, pf, seed, uneven, _ = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = P.all_halos(rp, cols, rs)
    for ppn in (1, R, R + 3):
        D = P.Decomposition(halos, rs, ppn, placement)
        for r in range(R):
            a, b = D.plain_plan(r), D.locality_plan(r)
            for k in P.PLAN_KEYS:
                assert np.array_equal(a[k], b[k]), (ppn, r, k)


def test_transpose_csr_brute_force():
    rng_idx = [np.array([3, 1, 3, 0, 3, 1], np.int32), np.zeros(0, np.int32),
               np.array([5, 5, 5, 5], np.int32)]
    for idx in rng_idx:
        n_local = 7
        ptr, perm = P.transpose_csr(idx, n_local)
        for i in range(n_local):
            assert perm[ptr[i]:ptr[i + 1]].tolist() == [k for k in range(idx.size) if idx[k] == i]


def loop_sum(vals, groups):
    out = []
    for g in groups:
        if not g:
            out.append(np.zeros(vals.shape[1:], vals.dtype))
            continue
        acc = vals[g[0]].copy()
        for k in g[1:]:
            acc = (acc + vals[k]).astype(vals.dtype)
        out.append(acc)
    return np.stack(out)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fixed_order_sum_matches_loop(dtype):
    idx = np.array([2, 0, 2, 2, 5, 0, 2, 1], np.int32)
    vals = uniform_pm1(5, idx.size * 3).reshape(-1, 3).astype(dtype) * dtype(1e3)
    ptr, perm = P.transpose_csr(idx, 6)
    got = M.pack_transpose(vals, ptr, perm)
    want = loop_sum(vals, [[k for k in range(idx.size) if idx[k] == i] for i in range(6)])
    assert got.dtype == dtype and np.array_equal(got.view(np.uint8), want.view(np.uint8))


def test_fixed_order_sum_order_and_signed_zero():
    # ascending order matters: (1e8 + 1) - 1e8 = 0 in FP32, any other order differs
    vals = np.array([[1e8], [1.0], [-1e8], [-0.0], [-0.0]], np.float32)
    ptr = np.array([0, 3, 4, 5, 5], np.int64)
    perm = np.array([0, 1, 2, 3, 4], np.int64)
    out = M.segmented_sum_fixed_order(vals, ptr, perm)
    assert out[0, 0] == 0.0
    alt = (vals[0] + vals[2]) + vals[1]
    assert alt[0] == 1.0                       # a different order gives another value
    assert np.signbit(out[1, 0]) and out[1, 0] == 0.0    # lone -0.0 survives
    assert np.signbit(out[2, 0])
    assert not np.signbit(out[3, 0]) and out[3, 0] == 0.0  # empty row -> +0.0


@pytest.mark.parametrize("case", CASES[:6])
def test_backward_is_adjoint_of_forward(case):
    """<G x, y> == <x, G^T y> exactly (small integers, FP64), where G is the
    whole exchange x -> halos and G^T is computed two ways: the closed form
    and the per-rank pack transpose after transferring halo gradients back."""
    rs, rp, cols, halos, D = build(case)
    R = len(rs) - 1
    n = int(rs[-1])
    C = 2
    x = (np.arange(n * C) % 7 - 3).astype(np.float64).reshape(n, C)
    plans = [D.plain_plan(r) for r in range(R)]
    out = M.forward_all(plans, x, rs)
    gy = [((np.arange(h.size * C) * 5 + r) % 11 - 5).astype(np.float64).reshape(h.size, C)
          for r, h in enumerate(halos)]
    lhs = sum(float(np.sum(a * b)) for a, b in zip(out["halo"], gy))
    gx = M.exchange_adjoint_reference(halos, gy, n)
    assert lhs == float(np.sum(x * gx))
    # per-rank route: halo gradient -> reverse transfer -> pack transpose
    g_send = M.transfer(gy, [(p["r1_procs"], p["r1_counts"], p["r1_displs"]) for p in plans],
                        [(p["s1_procs"], p["s1_counts"], p["s1_displs"]) for p in plans])
    gx2 = np.concatenate([M.pack_transpose(g_send[q], plans[q]["bt_ptr"], plans[q]["bt_perm"])
                          for q in range(R)])
    assert np.array_equal(gx, gx2)


@settings(max_examples=25, deadline=None)
@given(n=st.integers(1, 120), R=st.integers(1, 12), mx=st.integers(1, 6),
       pf=st.floats(0.0, 1.0), seed=st.integers(0, 10_000), uneven=st.booleans(),
       ppn=st.integers(1, 6), placement=st.sampled_from(PLACEMENTS))
def test_random_decompositions(n, R, mx, pf, seed, uneven, ppn, placement):
    R = min(R, n)
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = P.all_halos(rp, cols, rs)
    D = P.Decomposition(halos, rs, ppn, placement)
    x = uniform_pm1(seed + 1, n).reshape(n, 1)
    for variant in ("plain", "locality"):
        plans = [D.plan(r, variant) for r in range(R)]
        out = M.forward_all(plans, x, rs)
        for r in range(R):
            assert np.array_equal(out["halo"][r], x[np.asarray(brute_halo(rs, rp, cols, r), np.int64)])


class Sym:
    """A symbolic gradient: addition builds the expression it stands for, so
    the order and grouping of every sum the oracle performs can be read back."""

    def __init__(self, s):
        self.s = s

    def __add__(self, o):
        return Sym(f"({self.s}+{o.s})")

    def __eq__(self, o):
        return isinstance(o, Sym) and self.s == o.s

    def __repr__(self):
        return self.s


def _fold(terms):
    acc = terms[0]
    for t in terms[1:]:
        acc = acc + t
    return acc


def brute_staged_expression(halos, row_starts, ppn, placement="block"):
    """Expected expression of every row's gradient under reading R15, built
    from the definitions alone: the owner p sends row c once to each on-node
    rank that needs it and once per remote node m that needs it, to the
    partner m*ppn + (lrank(p) mod cnt(m)); the partner sums its own need
    first, then its node's other needers in ascending rank; the owner adds
    its send slots in ascending destination rank."""
    R = len(row_starts) - 1
    node, _, partner, _ = placement_fns(R, ppn, placement)
    needers = {}
    for s, h in enumerate(halos):
        for c in np.asarray(h).tolist():
            needers.setdefault(c, []).append(s)
    out = {}
    for c, ss in needers.items():
        p = int(np.searchsorted(row_starts, c, side="right") - 1)
        node_p = node(p)
        slots = {}
        for s in ss:
            m = node(s)
            if m == node_p:
                slots[s] = [s]
            else:
                t = partner(p, m)
                slots.setdefault(t, [])
                slots[t].append(s)
        terms = []
        for dest in sorted(slots):
            grp = sorted(slots[dest])
            grp = ([dest] if dest in grp else []) + [s for s in grp if s != dest]
            terms.append(_fold([Sym(f"g{s}_{c}") for s in grp]))
        out[c] = _fold(terms)
    return out


@pytest.mark.parametrize("placement", PLACEMENTS)
@pytest.mark.parametrize("variant", ["plain", "locality"])
@pytest.mark.parametrize("case", CASES)
def test_staged_adjoint_order_brute_force(case, variant, placement):
    """Every row's gradient is the sum the reading prescribes, term for term
    and in that grouping (symbolic values), for both plans."""
    rs, rp, cols, halos, D = build(case, placement)
    n, R = int(rs[-1]), len(rs) - 1
    ppn = case[-1] if variant == "locality" else 1   # the plain plan = one rank per node
    plans = [D.plan(r, variant) for r in range(R)]
    gy = [np.array([Sym(f"g{r}_{c}") for c in np.asarray(h).tolist()], dtype=object) for r, h in enumerate(halos)]
    got = M.staged_adjoint_reference(plans, gy, rs)["g_x"]
    want = brute_staged_expression(halos, rs, ppn, placement)
    for c in range(n):
        if c in want:
            assert got[c] == want[c], (c, got[c], want[c])
        else:
            assert not isinstance(got[c], Sym) and got[c] == 0


@pytest.mark.parametrize("case", CASES)
def test_staged_adjoint_plain_is_closed_form(case):
    """Plain plan: the staged backward is the closed-form adjoint, bit for bit
    (random FP32 gradients, so the summation order is visible)."""
    rs, rp, cols, halos, D = build(case)
    n, R = int(rs[-1]), len(rs) - 1
    plans = [D.plan(r, "plain") for r in range(R)]
    gy = [uniform_pm1(50 + r, h.size * 3).astype(np.float32).reshape(h.size, 3) for r, h in enumerate(halos)]
    got = M.staged_adjoint_reference(plans, gy, rs)["g_x"]
    assert np.array_equal(got.view(np.uint32), M.exchange_adjoint_reference(halos, gy, n).view(np.uint32))


@pytest.mark.parametrize("case", CASES)
def test_staged_adjoint_locality_exact_values(case):
    """Locality plan: with small-integer gradients (exact in FP64 whatever the
    order) the staged backward equals the closed-form adjoint, and it is the
    adjoint of the forward: <G x, y> == <x, G^T y>."""
    rs, rp, cols, halos, D = build(case)
    n, R = int(rs[-1]), len(rs) - 1
    plans = [D.plan(r, "locality") for r in range(R)]
    gy = [((np.arange(h.size * 2) * 7 + 3 * r) % 13 - 6).astype(np.float64).reshape(h.size, 2)
          for r, h in enumerate(halos)]
    got = M.staged_adjoint_reference(plans, gy, rs)["g_x"]
    assert np.array_equal(got, M.exchange_adjoint_reference(halos, gy, n))
    x = (np.arange(n * 2) % 9 - 4).astype(np.float64).reshape(n, 2)
    fw = M.forward_all(plans, x, rs)["halo"]
    assert sum(float(np.sum(a * b)) for a, b in zip(fw, gy)) == float(np.sum(x * got))


# --- the 3-step variant (reading R16) ----------------------------------------
def _node_of(row_starts, c, ppn):
    return int(np.searchsorted(row_starts, c, side="right") - 1) // ppn


@pytest.mark.parametrize("case", CASES)
def test_locality3_exchange_and_node_pairs(case):
    """3-step plan: the exchange equals the direct gather x[N_r]; exactly one
    inter-node message per node pair that needs one, from the pair's
    aggregator to its receiver, carrying the node's distinct columns the
    other node needs (Python sets, written from the definitions)."""
    rs, rp, cols, halos, D = build(case)
    n, R, ppn = int(rs[-1]), len(rs) - 1, case[-1]
    NN = (R + ppn - 1) // ppn
    cnt = [min(ppn, R - m * ppn) for m in range(NN)]
    plans = [D.plan(r, "locality3") for r in range(R)]
    x = (np.arange(n * 2) + 1).astype(np.float64).reshape(n, 2)
    out = M.forward_all(plans, x, rs)
    for r in range(R):
        assert np.array_equal(out["halo"][r], x[halos[r]])
    need = {}   # (source node, destination node) -> set of columns
    for s in range(R):
        for c in np.asarray(halos[s]).tolist():
            a, b = _node_of(rs, c, ppn), s // ppn
            if a != b:
                need.setdefault((a, b), set()).add(c)
    seen = {}
    for r in range(R):
        p = plans[r]
        base = p["pack_base"]
        for q, cnt_, d in zip(p["s1_procs"], p["s1_counts"], p["s1_displs"]):
            if int(q) // ppn == r // ppn:
                continue
            key = (r // ppn, int(q) // ppn)
            assert key not in seen, "two messages for one node pair"
            seen[key] = (r, int(q), set((base + p["s1_idx"][int(d):int(d) + int(cnt_)]).tolist()))
    assert set(seen) == set(need)
    for (a, b), (snd, rcv, colset) in seen.items():
        assert snd == a * ppn + b % cnt[a] and rcv == b * ppn + a % cnt[b]
        assert colset == need[(a, b)]


@pytest.mark.parametrize("case", CASES)
def test_locality3_special_cases(case):
    """One rank per node: the 3-step plan is the plain plan (each node pair is
    a rank pair).  One node: no inter-node traffic, so it is the 2-step plan
    (same messages, pack indices from the node's first row)."""
    rs, rp, cols, halos, _ = build(case)
    R = len(rs) - 1
    D1 = P.Decomposition(halos, rs, 1)
    for r in range(R):
        a, b = D1.plan(r, "locality3"), D1.plan(r, "plain")
        for k in ("s1_procs", "s1_counts", "r1_procs", "r1_counts", "s2_counts", "r2_counts"):
            assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a["s1_idx"].astype(np.int64) + a["pack_base"] - rs[r], b["s1_idx"])
        assert np.array_equal(a["unpack_src"], b["unpack_src"])
    DA = P.Decomposition(halos, rs, R)
    for r in range(R):
        a, b = DA.plan(r, "locality3"), DA.plan(r, "locality")
        for k in ("s1_procs", "s1_counts", "r1_procs", "r1_counts", "s2_counts", "r2_counts", "unpack_src"):
            assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a["s1_idx"].astype(np.int64) + a["pack_base"], b["s1_idx"] + rs[r])


def brute_staged_expression3(halos, row_starts, ppn):
    """Expected gradient expression of every row under R15 on the 3-step plan
    (R16): the slots of row c are the owner's direct on-node slots and one
    node-pair slot per remote node needing c, held by that pair's
    aggregator; the receiver sums its own need first, then its node's other
    needers ascending; slots add in ascending (sender rank, destination)."""
    R = len(row_starts) - 1
    NN = (R + ppn - 1) // ppn
    cnt = [min(ppn, R - m * ppn) for m in range(NN)]
    needers = {}
    for s, h in enumerate(halos):
        for c in np.asarray(h).tolist():
            needers.setdefault(c, []).append(s)
    out = {}
    for c, ss in needers.items():
        p = int(np.searchsorted(row_starts, c, side="right") - 1)
        n = p // ppn
        slots = {}   # (sender, destination) -> needers served
        for s in ss:
            m = s // ppn
            if m == n:
                slots[(p, s)] = [s]
            else:
                a, b = n * ppn + m % cnt[n], m * ppn + n % cnt[m]
                slots.setdefault((a, b), []).append(s)
        terms = []
        for key in sorted(slots):
            grp = sorted(slots[key])
            dest = key[1]
            grp = ([dest] if dest in grp else []) + [s for s in grp if s != dest]
            terms.append(_fold([Sym(f"g{s}_{c}") for s in grp]))
        out[c] = _fold(terms)
    return out


@pytest.mark.parametrize("case", CASES)
def test_locality3_staged_adjoint(case):
    """Staged backward on the 3-step plan: the order the reading prescribes
    (symbolic brute force), and the closed form in exact arithmetic."""
    rs, rp, cols, halos, D = build(case)
    n, R, ppn = int(rs[-1]), len(rs) - 1, case[-1]
    plans = [D.plan(r, "locality3") for r in range(R)]
    gy = [np.array([Sym(f"g{r}_{c}") for c in np.asarray(h).tolist()], dtype=object) for r, h in enumerate(halos)]
    got = M.staged_adjoint_reference(plans, gy, rs)["g_x"]
    want = brute_staged_expression3(halos, rs, ppn)
    for c in range(n):
        if c in want:
            assert got[c] == want[c], (c, got[c], want[c])
        else:
            assert not isinstance(got[c], Sym) and got[c] == 0
    gi = [((np.arange(h.size) * 5 + r) % 9 - 4).astype(np.float64) for r, h in enumerate(halos)]
    assert np.array_equal(M.staged_adjoint_reference(plans, gi, rs)["g_x"], M.exchange_adjoint_reference(halos, gi, n))
