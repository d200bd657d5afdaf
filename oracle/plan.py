"""Exchange plans of a persistent neighborhood all-to-all-v, built step by step.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU baseline may use this module.

Source passages (MPI Advance, Bienz, Schafer, Skjellum, 2023):

* Sec. 2.2, first paragraph: a neighborhood collective exchanges data between
  each process and a subset of the others; the persistent form pays every
  setup cost once, at initialisation, and that is what lets the library apply
  locality-aware aggregation underneath the standard call.
* Listings 3 and 4: the neighbor topology is given as ``n_recvs, recv_procs,
  n_sends, send_procs``; the exchange as ``sendcounts, sdispls`` /
  ``recvcounts, rdispls`` (all-to-all-v layout); the persistent request is
  created once and then driven by Start / Wait.
* Sec. 2.2, last paragraph: the locality-aware extension is given unique
  (global) indices of every value sent and received and uses them so that a
  value crosses between a pair of nodes only once.

Readings of what the paper leaves open:

* R1  contiguous ownership: rank p owns rows/columns [row_starts[p], row_starts[p+1]).
* R2  placement of R ranks on NN = ceil(R / ppn) nodes, block (the default):
      node(p) = p // ppn, lrank(p) = p % ppn, the last node may hold fewer
      ranks, cnt(m) = min(ppn, R - m*ppn); or cyclic (round robin):
      node(p) = p mod NN, lrank(p) = p // NN, cnt(m) = (R - 1 - m) // NN + 1.
      The rank of node m with local rank l is m*ppn + l (block) or l*NN + m
      (cyclic); a node's ranks are listed in ascending rank order.
* R3  orders: neighbor lists ascending by rank; entries of one message
      ascending by global index; displacements are exclusive prefix sums;
      empty messages are omitted; a rank never messages itself.  The halo is
      ordered by ascending global column, which equals the plain receive order.
* R4  locality-aware variant = "2-step": rank q sends the deduplicated union
      D(q -> m) of what node m needs from it to its partner
      partner(q, m) = the rank of node m with local rank lrank(q) mod cnt(m)
      (block: m*ppn + (lrank(q) mod cnt(m))) on each remote node m; on-node
      neighbors are served directly, as in the plain variant; the partner then
      forwards to every other rank of its node the entries of that rank's halo
      it received (redistribution), ordered by destination, then source rank,
      then position.
"""
from __future__ import annotations

import numpy as np

I32 = np.int32


def owner(cols, row_starts) -> np.ndarray:
    """Owning rank of each global column under contiguous ownership (reading R1)."""
    return np.searchsorted(np.asarray(row_starts, np.int64), np.asarray(cols, np.int64),
                           side="right") - 1


def halo(row_ptr, cols, row_starts, r: int) -> np.ndarray:
    """Halo discovery for rank r: sorted distinct columns of r's rows owned elsewhere.

    Sec. 2.2: the values a rank receives in the exchange are exactly the
    off-process entries its rows reference; each is received once.
    """
    lo, hi = int(row_starts[r]), int(row_starts[r + 1])
    c = np.asarray(cols[int(row_ptr[lo]):int(row_ptr[hi])], np.int64)
    off = c[(c < lo) | (c >= hi)]
    return np.unique(off)


def all_halos(row_ptr, cols, row_starts) -> list:
    return [halo(row_ptr, cols, row_starts, r) for r in range(len(row_starts) - 1)]


def _lists(procs, counts):
    procs = np.asarray(procs, I32)
    counts = np.asarray(counts, I32)
    displs = np.zeros(len(counts), I32)
    if len(counts):
        displs[1:] = np.cumsum(counts, dtype=np.int64)[:-1]
    return procs, counts, displs


def transpose_csr(send_idx, n_local: int):
    """Transpose of the pack map: for each local row i, the send entries k with
    send_idx[k] == i, ascending in k.  Returns (row_ptr [n_local+1], perm [E]).

    This is the structure the adjoint of the pack gather needs: the gradient of
    row i is the sum of the gradients of the entries that copied it.
    """
    idx = np.asarray(send_idx, np.int64)
    counts = np.bincount(idx, minlength=n_local) if idx.size else np.zeros(n_local, np.int64)
    row_ptr = np.zeros(n_local + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    perm = np.argsort(idx, kind="stable")
    return row_ptr.astype(I32), perm.astype(I32)


class Decomposition:
    """All ranks' halos plus the ownership/placement conventions R1-R4.

    ``placement``: "block" or "cyclic" rank-to-node placement (R2)."""

    def __init__(self, halos, row_starts, ppn: int, placement: str = "block"):
        self.halos = [np.asarray(h, np.int64) for h in halos]
        self.row_starts = np.asarray(row_starts, np.int64)
        self.R = len(self.row_starts) - 1
        self.ppn = int(ppn)
        if self.ppn < 1:
            raise ValueError("ppn must be >= 1")
        if placement not in ("block", "cyclic"):
            raise ValueError(placement)
        self.placement = placement

    # --- placement (R2) ---------------------------------------------------
    def nnodes(self) -> int:
        return (self.R + self.ppn - 1) // self.ppn

    def node(self, p: int) -> int:
        return p % self.nnodes() if self.placement == "cyclic" else p // self.ppn

    def lrank(self, p: int) -> int:
        return p // self.nnodes() if self.placement == "cyclic" else p % self.ppn

    def cnt(self, m: int) -> int:
        if self.placement == "cyclic":
            return (self.R - 1 - m) // self.nnodes() + 1
        return min(self.ppn, self.R - m * self.ppn)

    def rank_at(self, m: int, l: int) -> int:
        """The rank of node m with local rank l."""
        return l * self.nnodes() + m if self.placement == "cyclic" else m * self.ppn + l

    def node_ranks(self, m: int) -> list:
        """Ranks of node m, ascending."""
        return sorted(self.rank_at(m, l) for l in range(self.cnt(m)))

    def partner(self, q: int, m: int) -> int:
        """Rank of node m that receives q's aggregated message (reading R4)."""
        return self.rank_at(m, self.lrank(q) % self.cnt(m))

    def n_local(self, p: int) -> int:
        return int(self.row_starts[p + 1] - self.row_starts[p])

    # --- segments ---------------------------------------------------------
    def seg(self, s: int, q: int) -> np.ndarray:
        """N_s restricted to the columns owned by q (ascending global ids)."""
        h = self.halos[s]
        lo, hi = np.searchsorted(h, [self.row_starts[q], self.row_starts[q + 1]])
        return h[lo:hi]

    # --- plain variant (Listings 3-4, wrapping point-to-point) -------------
    def plain_recv(self, r: int):
        """Owner segmentation of N_r: one message per owning rank, ascending."""
        h = self.halos[r]
        if h.size == 0:
            return _lists([], [])
        own = owner(h, self.row_starts)
        procs, counts = np.unique(own, return_counts=True)
        return _lists(procs, counts)

    def plain_send(self, q: int):
        """Send lists of q = transpose of the other ranks' receive lists.

        For every rank s != q (ascending) whose halo contains columns owned by
        q, one message carrying those columns, as local rows of q.
        """
        procs, counts, idx = [], [], []
        start = int(self.row_starts[q])
        for s in range(self.R):
            if s == q:
                continue
            g = self.seg(s, q)
            if g.size:
                procs.append(s)
                counts.append(g.size)
                idx.append(g - start)
        p, c, d = _lists(procs, counts)
        return p, c, d, (np.concatenate(idx).astype(I32) if idx else np.zeros(0, I32))

    def plain_plan(self, r: int) -> dict:
        """Plan of rank r for the plain variant (no stage 2; identity unpack)."""
        rp, rc, rd = self.plain_recv(r)
        sp, sc, sd, sidx = self.plain_send(r)
        H = self.halos[r].size
        bt_ptr, bt_perm = transpose_csr(sidx, self.n_local(r))
        e = np.zeros(0, I32)
        return dict(halo=self.halos[r].copy(),
                    s1_procs=sp, s1_counts=sc, s1_displs=sd, s1_idx=sidx,
                    r1_procs=rp, r1_counts=rc, r1_displs=rd,
                    s2_procs=e, s2_counts=e, s2_displs=e, s2_src=e,
                    r2_procs=e, r2_counts=e, r2_displs=e,
                    unpack_src=np.arange(H, dtype=I32),
                    bt_ptr=bt_ptr, bt_perm=bt_perm)

    # --- locality-aware 2-step variant (Sec. 2.2, last paragraph; R4) ------
    def dedup(self, q: int, m: int) -> np.ndarray:
        """D(q -> m): distinct columns of q needed by any rank of remote node m."""
        parts = [self.seg(s, q) for s in self.node_ranks(m)]
        parts = [p for p in parts if p.size]
        if not parts:
            return np.zeros(0, np.int64)
        return np.unique(np.concatenate(parts))

    def forwarded_sources(self, t: int) -> list:
        """Remote ranks q whose aggregated message to node(t) lands on t, ascending."""
        n = self.node(t)
        return [q for q in range(self.R)
                if self.node(q) != n and self.partner(q, n) == t]

    def locality_plan(self, r: int) -> dict:
        """Plan of rank r for the 2-step locality-aware variant (reading R4)."""
        n = self.node(r)
        start = int(self.row_starts[r])
        # stage 1, send side: direct to on-node ranks, aggregated to partners
        msgs = []
        for s in self.node_ranks(n):
            if s != r:
                g = self.seg(s, r)
                if g.size:
                    msgs.append((s, g - start))
        for m in range(self.nnodes()):
            if m == n:
                continue
            d = self.dedup(r, m)
            if d.size:
                msgs.append((self.partner(r, m), d - start))
        msgs.sort(key=lambda t: t[0])
        s1p, s1c, s1d = _lists([t for t, _ in msgs], [len(v) for _, v in msgs])
        s1_idx = np.concatenate([v for _, v in msgs]).astype(I32) if msgs else np.zeros(0, I32)

        # stage 1, receive side: what arrives, with the global id of every slot
        rmsgs = []
        for q in self.node_ranks(n):
            if q != r:
                g = self.seg(r, q)
                if g.size:
                    rmsgs.append((q, g))
        fwd = self.forwarded_sources(r)
        for q in fwd:
            d = self.dedup(q, n)
            if d.size:
                rmsgs.append((q, d))
        rmsgs.sort(key=lambda t: t[0])
        r1p, r1c, r1d = _lists([q for q, _ in rmsgs], [len(v) for _, v in rmsgs])
        r1_slot = {int(q): int(d) for q, d in zip(r1p, r1d)}
        r1_ids = {int(q): v for q, v in rmsgs}
        R1 = int(r1c.sum()) if r1c.size else 0

        # stage 2, send side: r forwards to each other rank s of its node
        s2 = []
        for s in self.node_ranks(n):
            if s == r:
                continue
            src = []
            for q in fwd:
                g = self.seg(s, q)
                if g.size:
                    pos = np.searchsorted(r1_ids[q], g)
                    src.append(r1_slot[q] + pos)
            if src:
                s2.append((s, np.concatenate(src)))
        s2p, s2c, s2d = _lists([s for s, _ in s2], [len(v) for _, v in s2])
        s2_src = np.concatenate([v for _, v in s2]).astype(I32) if s2 else np.zeros(0, I32)

        # stage 2, receive side: from each other rank t of the node; within t's
        # message the entries come source by source (ascending), each source's
        # columns ascending -- remember where each source's run starts
        r2 = []
        run_start = {}
        for t in self.node_ranks(n):
            if t == r:
                continue
            c = 0
            for q in self.forwarded_sources(t):
                run_start[q] = (t, c)
                c += self.seg(r, q).size
            if c:
                r2.append((t, c))
        r2p, r2c, r2d = _lists([t for t, _ in r2], [c for _, c in r2])
        r2_slot = {int(t): int(d) for t, d in zip(r2p, r2d)}

        # unpack: where each halo entry is found in [stage-1 recv | stage-2 recv]
        h = self.halos[r]
        unpack = np.empty(h.size, np.int64)
        own = owner(h, self.row_starts)
        for q in np.unique(own):
            q = int(q)
            sel = np.nonzero(own == q)[0]
            cols_q = h[sel]
            if self.node(q) == n or self.partner(q, n) == r:
                # direct message from q, or q's aggregated message landed here
                unpack[sel] = r1_slot[q] + np.searchsorted(r1_ids[q], cols_q)
            else:
                t, c0 = run_start[q]
                unpack[sel] = R1 + r2_slot[t] + c0 + np.arange(sel.size)

        bt_ptr, bt_perm = transpose_csr(s1_idx, self.n_local(r))
        return dict(halo=h.copy(),
                    s1_procs=s1p, s1_counts=s1c, s1_displs=s1d, s1_idx=s1_idx,
                    r1_procs=r1p, r1_counts=r1c, r1_displs=r1d,
                    s2_procs=s2p, s2_counts=s2c, s2_displs=s2d, s2_src=s2_src,
                    r2_procs=r2p, r2_counts=r2c, r2_displs=r2d,
                    unpack_src=unpack.astype(I32),
                    bt_ptr=bt_ptr, bt_perm=bt_perm)

    # --- locality-aware 3-step variant (Sec. 2.2, aggregation; reading R16) -
    # (block placement only: an aggregator packs its node's contiguous rows)
    def node_start(self, n: int) -> int:
        if self.placement != "block":
            raise ValueError("the 3-step variant needs block placement (a node's rows contiguous)")
        return int(self.row_starts[n * self.ppn])

    def node_rows(self, n: int) -> int:
        return int(self.row_starts[n * self.ppn + self.cnt(n)]) - self.node_start(n)

    def aggregator(self, n: int, m: int) -> int:
        """Rank of node n that sends node n's data for node m (reading R16)."""
        return n * self.ppn + (m % self.cnt(n))

    def receiver(self, n: int, m: int) -> int:
        """Rank of node m that receives node n's data (reading R16)."""
        return m * self.ppn + (n % self.cnt(m))

    def node_seg(self, s: int, n: int) -> np.ndarray:
        """N_s restricted to the columns owned by node n (ascending)."""
        h = self.halos[s]
        lo, hi = np.searchsorted(h, [self.node_start(n), self.node_start(n) + self.node_rows(n)])
        return h[lo:hi]

    def node_dedup(self, n: int, m: int) -> np.ndarray:
        """D(n -> m): distinct columns of node n needed by any rank of node m."""
        parts = [self.node_seg(s, n) for s in self.node_ranks(m)]
        parts = [p for p in parts if p.size]
        if not parts:
            return np.zeros(0, np.int64)
        return np.unique(np.concatenate(parts))

    def received_nodes(self, t: int) -> list:
        """Remote nodes whose node-pair message to node(t) lands on t, ascending."""
        n = self.node(t)
        return [m for m in range(self.nnodes()) if m != n and self.receiver(m, n) == t]

    def locality3_plan(self, r: int) -> dict:
        """Plan of rank r for the 3-step locality-aware variant (reading R16).

        Stage 1 carries the direct on-node messages and, from each node
        pair's aggregator, one message with the node's deduplicated data for
        the other node (the aggregator packs its node-mates' rows directly,
        so the on-node gather is part of its pack); stage 2 is the
        receiver's redistribution.  Pack indices are rows of the node
        (``pack_base`` = the node's first row).
        """
        n = self.node(r)
        base = self.node_start(n)
        msgs = []
        for s in self.node_ranks(n):
            if s != r:
                g = self.seg(s, r)
                if g.size:
                    msgs.append((s, g - base))
        for m in range(self.nnodes()):
            if m != n and self.aggregator(n, m) == r:
                d = self.node_dedup(n, m)
                if d.size:
                    msgs.append((self.receiver(n, m), d - base))
        msgs.sort(key=lambda t: t[0])
        s1p, s1c, s1d = _lists([t for t, _ in msgs], [len(v) for _, v in msgs])
        s1_idx = np.concatenate([v for _, v in msgs]).astype(I32) if msgs else np.zeros(0, I32)

        # stage 1, receive side: direct messages and node-pair messages (by sender)
        rmsgs = []
        for q in self.node_ranks(n):
            if q != r:
                g = self.seg(r, q)
                if g.size:
                    rmsgs.append((q, g))
        fwd = self.received_nodes(r)
        for m in fwd:
            d = self.node_dedup(m, n)
            if d.size:
                rmsgs.append((self.aggregator(m, n), d))
        rmsgs.sort(key=lambda t: t[0])
        r1p, r1c, r1d = _lists([q for q, _ in rmsgs], [len(v) for _, v in rmsgs])
        r1_slot = {int(q): int(d) for q, d in zip(r1p, r1d)}
        r1_ids = {int(q): v for q, v in rmsgs}
        R1 = int(r1c.sum()) if r1c.size else 0

        # stage 2, send side: r forwards to each other rank s of its node the
        # entries of N_s owned by the nodes whose message landed on r
        s2 = []
        for s in self.node_ranks(n):
            if s == r:
                continue
            src = []
            for m in fwd:
                g = self.node_seg(s, m)
                if g.size:
                    a = self.aggregator(m, n)
                    src.append(r1_slot[a] + np.searchsorted(r1_ids[a], g))
            if src:
                s2.append((s, np.concatenate(src)))
        s2p, s2c, s2d = _lists([s for s, _ in s2], [len(v) for _, v in s2])
        s2_src = np.concatenate([v for _, v in s2]).astype(I32) if s2 else np.zeros(0, I32)

        # stage 2, receive side: node by node (ascending) within each forwarder
        r2 = []
        run_start = {}
        for t in self.node_ranks(n):
            if t == r:
                continue
            c = 0
            for m in self.received_nodes(t):
                run_start[m] = (t, c)
                c += self.node_seg(r, m).size
            if c:
                r2.append((t, c))
        r2p, r2c, r2d = _lists([t for t, _ in r2], [c for _, c in r2])
        r2_slot = {int(t): int(d) for t, d in zip(r2p, r2d)}

        # unpack
        h = self.halos[r]
        unpack = np.empty(h.size, np.int64)
        own = owner(h, self.row_starts)
        onode = own // self.ppn
        for m in np.unique(onode):
            m = int(m)
            sel = np.nonzero(onode == m)[0]
            cols_m = h[sel]
            if m == n:
                for q in np.unique(own[sel]):
                    q = int(q)
                    sq = sel[own[sel] == q]
                    unpack[sq] = r1_slot[q] + np.searchsorted(r1_ids[q], h[sq])
            elif self.receiver(m, n) == r:
                a = self.aggregator(m, n)
                unpack[sel] = r1_slot[a] + np.searchsorted(r1_ids[a], cols_m)
            else:
                t, c0 = run_start[m]
                unpack[sel] = R1 + r2_slot[t] + c0 + np.arange(sel.size)

        bt_ptr, bt_perm = transpose_csr(s1_idx, self.node_rows(n))
        return dict(halo=h.copy(),
                    s1_procs=s1p, s1_counts=s1c, s1_displs=s1d, s1_idx=s1_idx,
                    r1_procs=r1p, r1_counts=r1c, r1_displs=r1d,
                    s2_procs=s2p, s2_counts=s2c, s2_displs=s2d, s2_src=s2_src,
                    r2_procs=r2p, r2_counts=r2c, r2_displs=r2d,
                    unpack_src=unpack.astype(I32),
                    bt_ptr=bt_ptr, bt_perm=bt_perm, pack_base=base)

    def plan(self, r: int, variant: str) -> dict:
        if variant == "plain":
            return self.plain_plan(r)
        if variant == "locality":
            return self.locality_plan(r)
        if variant == "locality3":
            return self.locality3_plan(r)
        raise ValueError(variant)


PLAN_KEYS = ("halo", "s1_procs", "s1_counts", "s1_displs", "s1_idx",
             "r1_procs", "r1_counts", "r1_displs",
             "s2_procs", "s2_counts", "s2_displs", "s2_src",
             "r2_procs", "r2_counts", "r2_displs",
             "unpack_src", "bt_ptr", "bt_perm")
