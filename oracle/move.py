"""Data movement of the exchange, and the plain definitions it must reproduce.

TEST INFRASTRUCTURE (see the package docstring).

Source passages (MPI Advance, 2023): Listings 3 and 4 (all-to-all-v buffers
described by counts and displacements; Start / Wait of the persistent
request), Sec. 2.2 (locality-aware aggregation with forwarding inside a node)
and Sec. 2.4 (the same calls accept device memory, so the pack of a send
buffer from a vector and the unpack into the halo are device-side gathers).

The message transfer between ranks is simulated here by copying each
message's segment from the sender's buffer into the receiver's buffer.
"""
from __future__ import annotations

import numpy as np


def pack(x_local: np.ndarray, idx) -> np.ndarray:
    """Pack (Start): send[k, :] = x_local[idx[k], :]."""
    return np.take(x_local, np.asarray(idx, np.int64), axis=0)


def gather_rows(src: np.ndarray, idx) -> np.ndarray:
    """Redistribution pack and unpack: out[k, :] = src[idx[k], :]."""
    return np.take(src, np.asarray(idx, np.int64), axis=0)


def transfer(send_bufs: list, send_lists: list, recv_lists: list) -> list:
    """Simulated message transfer for every rank at once.

    ``send_lists[q]`` / ``recv_lists[r]`` are (procs, counts, displs).  The
    message r receives from q is the segment of q's send buffer addressed to r.
    """
    R = len(send_bufs)
    out = []
    for r in range(R):
        rp, rc, rd = recv_lists[r]
        tail = send_bufs[0].shape[1:] if R else ()
        dt = send_bufs[0].dtype if R else np.float64
        buf = np.empty((int(np.sum(rc, dtype=np.int64)),) + tail, dt)
        for q, c, d in zip(rp, rc, rd):
            sp, sc, sd = send_lists[q]
            pos = np.nonzero(np.asarray(sp) == r)[0]
            if pos.size != 1 or int(sc[pos[0]]) != int(c):
                raise AssertionError(f"message {q}->{r} not matched")
            s0 = int(sd[pos[0]])
            buf[int(d):int(d) + int(c)] = send_bufs[q][s0:s0 + int(c)]
        out.append(buf)
    return out


def forward_all(plans: list, x_global: np.ndarray, row_starts) -> dict:
    """Run Start and Wait for every rank with simulated transfers.

    Start: pack the stage-1 send buffer.  Wait: receive stage 1, pack the
    stage-2 (redistribution) buffer from the stage-1 receive buffer, receive
    stage 2, unpack [stage-1 recv | stage-2 recv] into the halo.
    Returns every intermediate buffer (per rank lists).
    """
    R = len(plans)
    rs = np.asarray(row_starts, np.int64)
    # pack indices are rows from the rank's first row, or from its node's
    # first row for the 3-step plan (``pack_base``)
    send1 = [pack(x_global[int(plans[p].get("pack_base", rs[p])):], plans[p]["s1_idx"]) for p in range(R)]
    recv1 = transfer(send1, [(p["s1_procs"], p["s1_counts"], p["s1_displs"]) for p in plans],
                     [(p["r1_procs"], p["r1_counts"], p["r1_displs"]) for p in plans])
    send2 = [gather_rows(recv1[p], plans[p]["s2_src"]) for p in range(R)]
    recv2 = transfer(send2, [(p["s2_procs"], p["s2_counts"], p["s2_displs"]) for p in plans],
                     [(p["r2_procs"], p["r2_counts"], p["r2_displs"]) for p in plans])
    arena = [np.concatenate([recv1[p], recv2[p]], axis=0) for p in range(R)]
    halo = [gather_rows(arena[p], plans[p]["unpack_src"]) for p in range(R)]
    return dict(send1=send1, recv1=recv1, send2=send2, recv2=recv2, arena=arena, halo=halo)


def halo_reference(x_global: np.ndarray, halo_cols) -> np.ndarray:
    """Plain definition of the exchange result: the direct global gather x[N_r]."""
    return np.take(x_global, np.asarray(halo_cols, np.int64), axis=0)


def segmented_sum_fixed_order(vals: np.ndarray, seg_ptr, order) -> np.ndarray:
    """out[i] = vals[order[seg_ptr[i]]] + vals[order[seg_ptr[i]+1]] + ... in that order.

    Sequential additions in the dtype of ``vals`` (no pairwise or tree
    reduction), the accumulator starting from the first term (so a lone -0.0
    stays -0.0); an empty segment yields +0.0.  Vectorised over segments by
    depth: step d adds the d-th term of every segment longer than d.
    """
    seg_ptr = np.asarray(seg_ptr, np.int64)
    order = np.asarray(order, np.int64)
    nseg = seg_ptr.size - 1
    out = np.zeros((nseg,) + vals.shape[1:], vals.dtype)
    lens = np.diff(seg_ptr)
    if nseg == 0 or lens.size == 0 or lens.max(initial=0) == 0:
        return out
    rows = np.nonzero(lens > 0)[0]
    out[rows] = vals[order[seg_ptr[rows]]]
    for d in range(1, int(lens.max())):
        rows = np.nonzero(lens > d)[0]
        out[rows] = out[rows] + vals[order[seg_ptr[rows] + d]]
    return out


def pack_transpose(g_send: np.ndarray, bt_ptr, bt_perm) -> np.ndarray:
    """Backward of the pack: gX[i] = sum of g_send[k] over k with idx[k] == i,
    in ascending k (the transpose CSR of the pack map)."""
    return segmented_sum_fixed_order(g_send, bt_ptr, bt_perm)


def exchange_adjoint_reference(halos: list, g_halos: list, n: int) -> np.ndarray:
    """Plain definition of the backward of the whole exchange (closed form G^T).

    gX[c] = sum over ranks s (ascending) whose halo holds column c of the
    gradient of that halo entry.  Rows referenced by no halo get +0.0.
    """
    cols = np.concatenate([np.asarray(h, np.int64) for h in halos]) if halos else np.zeros(0, np.int64)
    vals = np.concatenate(g_halos, axis=0)
    order = np.argsort(cols, kind="stable")   # concatenation is in ascending s
    counts = np.bincount(cols, minlength=n)
    ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    return segmented_sum_fixed_order(vals, ptr, order)


def reverse_transfer(recv_bufs: list, send_lists: list, recv_lists: list) -> list:
    """Adjoint of ``transfer``: every message travels back from its receiver's
    slots to its sender's slots (the same segments, the roles swapped)."""
    return transfer(recv_bufs, recv_lists, send_lists)


def staged_adjoint_reference(plans: list, g_halos: list, row_starts) -> dict:
    """Backward of the exchange taken through its stages in reverse (reading
    R15; the forward is Listing 4's Start/Wait with the locality-aware
    forwarding of Sec. 2.2):

    1. unpack, reversed: a receive slot read by the rank's own halo takes
       that entry's gradient (each slot is read by at most one halo entry);
    2. the stage-2 messages travel back (forwarder's redistribution slots);
    3. forwarder sums: a stage-1 receive slot k of rank q gets its own-halo
       term first (when q's halo reads k), then the gradients of the
       redistribution entries e with s2_src[e] == k in ascending e
       (= ascending destination rank);
    4. the stage-1 messages travel back;
    5. owner sums: gX_r[i] = sum of the stage-1 send-slot gradients packed
       from row i, in ascending slot (the pack transpose).

    Sums are sequential in the gradient dtype (``segmented_sum_fixed_order``).
    For the plain plan stages 2 and 3 are empty and the result is the
    closed-form adjoint of ``exchange_adjoint_reference``.
    """
    from .plan import transpose_csr
    R = len(plans)
    rs = np.asarray(row_starts, np.int64)
    tail = g_halos[0].shape[1:] if R else ()
    dt = g_halos[0].dtype if R else np.float64
    own, g_recv2 = [], []
    for r in range(R):
        p = plans[r]
        R1 = int(np.sum(p["r1_counts"], dtype=np.int64))
        R2 = int(np.sum(p["r2_counts"], dtype=np.int64))
        us = np.asarray(p["unpack_src"], np.int64)
        o = np.full(R1 + R2, -1, np.int64)
        if np.any(np.bincount(us, minlength=R1 + R2) > 1):
            raise AssertionError(f"rank {r}: a receive slot is read twice by the halo")
        o[us] = np.arange(us.size)
        if np.any(o[R1:] < 0):
            raise AssertionError(f"rank {r}: a stage-2 slot is not read by the halo")
        own.append(o)
        g_recv2.append(np.asarray(g_halos[r])[o[R1:]] if R2 else np.zeros((0,) + tail, dt))
    g_send2 = reverse_transfer(g_recv2, [(p["s2_procs"], p["s2_counts"], p["s2_displs"]) for p in plans],
                               [(p["r2_procs"], p["r2_counts"], p["r2_displs"]) for p in plans])
    g_recv1 = []
    for r in range(R):
        p = plans[r]
        R1 = int(np.sum(p["r1_counts"], dtype=np.int64))
        H = np.asarray(g_halos[r]).shape[0]
        vals = np.concatenate([np.asarray(g_halos[r]).reshape((H,) + tail), g_send2[r]], axis=0)
        src = np.asarray(p["s2_src"], np.int64)
        order, ptr = [], [0]
        for k in range(R1):
            terms = ([int(own[r][k])] if own[r][k] >= 0 else []) + [H + int(e) for e in np.nonzero(src == k)[0]]
            order.extend(terms)
            ptr.append(len(order))
        g_recv1.append(segmented_sum_fixed_order(vals, np.asarray(ptr, np.int64), np.asarray(order, np.int64)))
    g_send1 = reverse_transfer(g_recv1, [(p["s1_procs"], p["s1_counts"], p["s1_displs"]) for p in plans],
                               [(p["r1_procs"], p["r1_counts"], p["r1_displs"]) for p in plans])
    # owner sums over every rank's stage-1 send slots, keyed by global row,
    # ascending (rank, slot): per rank the pack transpose when only the owner
    # packs its rows (plain, 2-step), the node's senders in rank order (3-step)
    n = int(rs[-1]) if R else 0
    keys = [int(plans[r].get("pack_base", rs[r])) + np.asarray(plans[r]["s1_idx"], np.int64) for r in range(R)]
    keys = np.concatenate(keys) if R else np.zeros(0, np.int64)
    vals = np.concatenate(g_send1, axis=0) if R else np.zeros((0,) + tail, dt)
    ptr, perm = transpose_csr(keys, n)
    g_x = pack_transpose(vals, ptr, perm)
    return dict(g_x=g_x, g_recv2=g_recv2, g_send2=g_send2, g_recv1=g_recv1, g_send1=g_send1)
