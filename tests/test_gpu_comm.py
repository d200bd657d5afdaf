"""The per-rank locality-aware init (collective over a simulated
communicator): every rank joins with its own neighbor lists and global
indices, in a shuffled order and with shuffled receive orders; once the set
is complete each rank's Start/Wait moves exactly what the oracle's plan
moves (stage buffers bit for bit) and its halo holds x at its own receive
indices, in its own order."""
import numpy as np
import pytest

import paper_2309_07337_amd as P
from oracle import move as OM
from oracle import plan as OP
from tests.conftest import cached_grid2d, cached_grid3d
from tests.gpu_util import bits_equal, dev, host, need_gpu, say
from tests.test_oracle_brute import CASES
from workloads import random_small_csr, uniform_pm1

pytestmark = pytest.mark.gpu


def rank_lists(halos, rs, seed, shuffle):
    """Plain neighbor lists of every rank from the halos: receive messages
    (owner, indices) and the matching send messages; with shuffle, the
    receive neighbors and the indices inside each message come in a random
    order (the send side follows)."""
    rng = np.random.default_rng(seed)
    R = len(rs) - 1
    recv = []
    for r in range(R):
        own = OP.owner(halos[r], rs)
        msgs = [(int(q), np.asarray(halos[r])[own == q].astype(np.int64)) for q in np.unique(own)]
        if shuffle:
            msgs = [(q, rng.permutation(v)) for q, v in msgs]
            msgs = [msgs[i] for i in rng.permutation(len(msgs))]
        recv.append(msgs)
    send = [[] for _ in range(R)]
    for s in range(R):
        for q, v in recv[s]:
            send[q].append((s, v))
    return recv, send


def run_collective(rs, halos, ppn, variant, node_map, C, seed, shuffle):
    import torch
    R = len(rs) - 1
    n = int(rs[-1])
    xh = uniform_pm1(seed, n * C).reshape(n, C)
    D = OP.Decomposition(halos, rs, ppn, node_map)
    out = OM.forward_all([D.plan(r, variant) for r in range(R)], xh, rs)
    recv, send = rank_lists(halos, rs, seed, shuffle)
    var_id = {"plain": P.HX_PLAIN, "locality": P.HX_LOCALITY_2STEP, "locality3": P.HX_LOCALITY_3STEP}[variant]
    comm = P.hx_comm_create(R, rs, ppn, var_id, node_map)
    order = np.random.default_rng(seed + 1).permutation(R)
    reqs, keep = {}, []
    for k, r in enumerate(order):
        r = int(r)
        topo = P.hx_topo_create(r, R, [q for q, _ in recv[r]], [s for s, _ in send[r]])
        rind = np.concatenate([v for _, v in recv[r]]) if recv[r] else np.zeros(0, np.int64)
        sind = np.concatenate([v for _, v in send[r]]) if send[r] else np.zeros(0, np.int64)
        if variant == "locality3":   # an aggregator packs its node-mates' rows: the node's rows
            nd = r // ppn
            x_local = dev(xh[rs[nd * ppn]:rs[min(R, (nd + 1) * ppn)]])
        else:
            x_local = dev(xh[rs[r]:rs[r + 1]])
        halo = torch.full((rind.size, C), float("nan"), dtype=torch.float64, device="cuda")
        req = P.hx_neighbor_locality_alltoallv_init(x_local, [v.size for _, v in send[r]], None, sind, halo,
                                                    [v.size for _, v in recv[r]], None, rind, topo, comm)
        reqs[r] = (req, halo, rind)
        keep.append((topo, x_local))
        if k == 0 and R > 1:
            with pytest.raises(P.HXError) as e:
                P.hx_start(req)
            assert e.value.code == P.HX_ERR_STATE
    for r in range(R):
        req, halo, rind = reqs[r]
        P.req_arena_view(req, P.HX_ARENA_RECV, C, torch.float64).copy_(dev(out["arena"][r]))
        P.hx_start(req)
        P.hx_wait(req)
        send_arena = host(P.req_arena_view(req, P.HX_ARENA_SEND, C, torch.float64))
        assert bits_equal(send_arena, np.concatenate([out["send1"][r], out["send2"][r]])), r
        assert bits_equal(host(halo), xh[rind]), r
        req.free()      # requests freed before their communicator: it must not touch them
    comm.free()


@pytest.mark.parametrize("variant,node_map", [("plain", "block"), ("locality", "block"), ("locality", "cyclic"),
                                              ("locality3", "block")])
@pytest.mark.parametrize("case", CASES)
def test_tiny_decompositions(case, variant, node_map):
    need_gpu()
    n, R, mx, pf, seed, uneven, ppn = case
    rs, rp, cols = random_small_csr(n, R, mx, pf, seed, uneven)
    halos = OP.all_halos(rp, cols, rs)
    for shuffle in (False, True):
        say("collective init tiny", case, variant, node_map, shuffle)
        run_collective(rs, halos, ppn, variant, node_map, 3, seed + 7, shuffle)


@pytest.mark.parametrize("node_map", ["block", "cyclic"])
def test_grid2d(node_map):
    need_gpu()
    rs, rp, cols = cached_grid2d()
    halos = OP.all_halos(rp, cols, rs)
    say("collective init grid2d", node_map)
    run_collective(rs, halos, 4, "locality", node_map, 1, 31, True)


@pytest.mark.parametrize("variant", ["locality", "locality3"])
def test_grid3d(variant):
    """27-point 128^3, 512 ranks joining in a random order, receive orders shuffled."""
    need_gpu()
    rs, rp, cols = cached_grid3d()
    halos = OP.all_halos(rp, cols, rs)
    say("collective init grid3d", variant)
    run_collective(rs, halos, 64, variant, "block", 2, 41, True)
