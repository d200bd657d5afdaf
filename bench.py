#!/usr/bin/env python3
"""Benchmark of the halo-exchange buffer engine on one MI355X.

Headline workload ("batched256"): 256 independent persistent exchange plans,
halo sizes log-uniform in [1e3, 1e6) rows, 1..4096 neighbors, 16 FP64
columns per row.  One step = Start + Wait of all plans (pack, unpack) plus
the backward of the pack (fixed-order transpose sum), each phase one
multi-job kernel replayed from a hipGraph (or launched directly, as tuned).
The same work as one launch per plan per phase ("plain") is timed beside it.

With the headline workload the line also carries ``configs``: every other
workload measured the same way (tuned, warm back-to-back steps, a cold
median with the caches flushed before each step, each kernel alone, the
dominant kernel against the HBM roofline):

* random_rows / random_rows_f32 / random_rows_3step: 2^22 x 32 random
  matrix, 4096 ranks, 128 per node, 2-step or 3-step locality-aware plan,
  every rank batched, one FP64 / FP32 column (forward step; the staged
  backward reported aside);
* rank1511: the random matrix's rank with the most neighbors alone (one
  persistent request from the locality plan; warm, microseconds);
* diff64: the random matrix's plain plan with 64 FP32 features, forward +
  backward, as batch calls and through the autograd Function;
* grid3d_diff64: the 27-point 128^3 decomposition's plain plan with 64 FP32
  features, forward + backward;
* grid3d, grid2d: the two stencils' locality plans, one FP64 column.

``--workload`` runs one of them alone as the headline (``copy`` is the 1 GiB
calibration copy for the PMC scale factors).  ``--sched-json`` applies
recorded schedules instead of tuning (per phase, as hx_batch_get_sched
reports them), ``--replay`` fixes the replay mode.

Prints one JSON line (rank 0, one GPU).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_2309_07337_amd", "csrc", f)
               for f in ("move_kernels.h", "move_launch.h", "move_gather.hip", "move_scatter.hip",
                         "move_segsum.hip", "move.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_src_hash() -> str:
    """Hash of the data-movement kernel sources (a PMC summary is only valid
    for the kernels it was taken on)."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}__pmc.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("src_hash") != kernel_src_hash():
        return None
    return d.get("hbm_bytes_per_launch")


# ---------------------------------------------------------------------------
# Workloads: each setup returns a dict with the batch ("batch"), the phases
# of its timed step ("phases"), its configuration ("cfg"), the arithmetic
# dtype and whatever must stay alive ("keep").
# ---------------------------------------------------------------------------
def setup_batched(args, torch, P):
    import numpy as np
    from workloads import batched_plan, batched_plan_sizes, uniform_pm1
    C = 16
    dt = torch.float64
    h, k = batched_plan_sizes()
    nplans = args.plans
    members, host_keep = [], []
    t0 = time.time()
    for b in range(nplans):
        hb, kb = int(h[b]), int(k[b])
        lists = batched_plan(b, hb, kb)
        xh = uniform_pm1(50_000 + b, hb * C).reshape(hb, C)
        rh = uniform_pm1(60_000 + b, hb * C).reshape(hb, C)
        x = torch.from_numpy(xh).cuda()
        halo = torch.empty(hb, C, dtype=dt, device="cuda")
        topo = P.hx_topo_create(0, 4096, lists["procs"], lists["procs"])
        req = P.hx_neighbor_alltoallv_init(x, lists["counts"], lists["displs"], lists["send_idx"], halo,
                                           lists["counts"], lists["displs"], topo)
        P.req_arena_view(req, P.HX_ARENA_RECV, C, dt).copy_(torch.from_numpy(rh))
        g_send = torch.from_numpy(uniform_pm1(70_000 + b, hb * C).reshape(hb, C)).cuda()
        g_x = torch.empty_like(x)
        P.hx_req_bind_grad(req, g_send, g_x)
        members.append(dict(req=req, x=x, halo=halo, g_send=g_send, g_x=g_x, h=hb, k=kb))
        if len(host_keep) < args.cpu_plans:
            host_keep.append(dict(x=xh, recv=rh, idx=lists["send_idx"], g_send=None, b=b, h=hb))
    torch.cuda.synchronize()
    log(f"setup: {nplans} plans, sum h = {sum(m['h'] for m in members)}, {time.time() - t0:.1f}s")
    batch = P.hx_batch_init([m["req"] for m in members])
    tune(args, torch, P, batch, "batched256")
    # correctness of sampled members against the oracle before timing
    P.hx_batch_start(batch)
    P.hx_batch_wait(batch)
    P.hx_batch_backward(batch)
    torch.cuda.synchronize()
    from oracle import move as OM
    from oracle import plan as OP
    for hk in host_keep[:2]:
        m = members[hk["b"]]
        send = P.req_arena_view(m["req"], P.HX_ARENA_SEND, C, dt).cpu().numpy()
        assert np.array_equal(send, OM.pack(hk["x"], hk["idx"])), "pack mismatch"
        assert np.array_equal(m["halo"].cpu().numpy(), hk["recv"]), "unpack mismatch"
        ptr, perm = OP.transpose_csr(hk["idx"], hk["h"])
        gx = OM.pack_transpose(m["g_send"].cpu().numpy(), ptr, perm)
        assert np.array_equal(m["g_x"].cpu().numpy().view(np.uint64), gx.view(np.uint64)), "backward mismatch"
    log("parity: sampled members equal the oracle (pack, unpack, backward)")
    cfg = {"workload": "batched256: 256 independent plans, halo 1e3..1e6 rows (log-uniform), "
                       "1..4096 neighbors, 16 x FP64 columns (128 B rows); pack+unpack+backward",
           "plans": nplans, "ncols": C, "rows_total": int(sum(m["h"] for m in members))}
    return dict(batch=batch, host=host_keep, dtype="f64", cfg=cfg, phases=(0, 2, 3), keep=members)


def setup_copy(args, torch, P):
    """Calibration: one request whose only work is the identity unpack of a
    1 GiB receive arena (a plain device copy of known size)."""
    C, dt = 16, torch.float64
    rows = (1 << 30) // (C * 8)
    topo = P.hx_topo_create(0, 2, [1], [])
    x = torch.zeros(1, C, dtype=dt, device="cuda")
    halo = torch.empty(rows, C, dtype=dt, device="cuda")
    req = P.hx_neighbor_alltoallv_init(x, [], [], [], halo, [rows], [0], topo)
    P.req_arena_view(req, P.HX_ARENA_RECV, C, dt).copy_(torch.arange(rows * C, dtype=dt, device="cuda").view(rows, C))
    g_x = torch.empty_like(x)
    P.hx_req_bind_grad(req, None, g_x)
    batch = P.hx_batch_init([req])
    P.hx_batch_start(batch)
    P.hx_batch_wait(batch)
    torch.cuda.synchronize()
    assert torch.equal(halo, P.req_arena_view(req, P.HX_ARENA_RECV, C, dt))
    cfg = {"workload": "copy calibration: identity unpack of a 1 GiB arena (128 B rows)", "bytes_copied": rows * C * 8}
    return dict(batch=batch, host=[], dtype="f64", cfg=cfg, phases=(0, 2, 3), keep=(req, x, halo, g_x, topo))


WORLD_DESC = {
    "random_rows": "random 2^22 x 32 (70% in-block), 4096 ranks, 128/node, locality 2-step, all ranks batched, "
                   "1 x FP64",
    "random_rows_f32": "random 2^22 x 32 (70% in-block), 4096 ranks, 128/node, locality 2-step, all ranks "
                       "batched, 1 x FP32",
    "random_rows_3step": "random 2^22 x 32 (70% in-block), 4096 ranks, 128/node, locality 3-step (one message per "
                         "node pair), all ranks batched, 1 x FP64",
    "grid3d": "27-point 128^3, 512 ranks, 64/node, locality 2-step, all ranks, 1 x FP64",
    "grid2d": "5-point 512^2, 16 ranks, 4/node, locality 2-step, all ranks, 1 x FP64",
    "diff64": "random 2^22 x 32, 4096 ranks, plain plan, 64 x FP32 features, forward halo gather + fixed-order "
              "transpose-sum backward",
    "grid3d_diff64": "27-point 128^3, 512 ranks, plain plan, 64 x FP32 features, forward halo gather + "
                     "fixed-order transpose-sum backward",
}


def world_structure(name):
    from workloads import equal_row_starts, grid2d_5pt, grid3d_27pt, random_rows
    if name.startswith("random_rows") or name in ("diff64", "rank1511"):
        rp, cols = random_rows()
        return equal_row_starts(1 << 22, 4096), 128, rp, cols
    if name.startswith("grid3d"):
        rp, cols = grid3d_27pt()
        return equal_row_starts(128 ** 3, 512), 64, rp, cols
    rp, cols = grid2d_5pt()
    return equal_row_starts(512 * 512, 16), 4, rp, cols


def setup_world(args, torch, P, name):
    import numpy as np
    from workloads import uniform_pm1, uniform_pm1_f32
    t0 = time.time()
    rs, ppn, rp, cols = world_structure(name)
    log(f"generated {name} structure in {time.time() - t0:.1f}s")
    plain = name in ("diff64", "grid3d_diff64")
    variant = P.HX_PLAIN if plain else (P.HX_LOCALITY_3STEP if name.endswith("3step") else P.HX_LOCALITY_2STEP)
    rp_d, cols_d = torch.from_numpy(rp).cuda(), torch.from_numpy(cols).cuda()
    torch.cuda.synchronize()
    t0 = time.time()
    plan = P.hx_plan_from_csr(len(rs) - 1, rs, ppn, variant, rp_d, cols_d)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    del rp_d, cols_d
    R = len(rs) - 1
    n = int(rs[-1])
    H = sum(int(P.hx_plan_field(plan, r, "halo").size) for r in range(R))
    if plain:
        C, dt = 64, torch.float32
        x = torch.from_numpy(uniform_pm1_f32(7337, n * C).reshape(n, C)).cuda()
    elif name == "random_rows_f32":
        C, dt = 1, torch.float32
        x = torch.from_numpy(uniform_pm1_f32(7337, n).reshape(n, 1)).cuda()
    else:
        C, dt = 1, torch.float64
        x = torch.from_numpy(uniform_pm1(7337, n).reshape(n, 1)).cuda()
    # correctness pass with the simulated transfer (separate arenas)
    halo_chk = torch.empty(H, C, dtype=dt, device="cuda")
    chk = P.hx_batch_from_plan(plan, x, halo_chk, flags=P.HX_WORLD_SIM_TRANSFER)
    P.hx_batch_start(chk)
    P.hx_batch_wait(chk)
    torch.cuda.synchronize()
    cols_all = torch.from_numpy(np.concatenate([P.hx_plan_field(plan, r, "halo") for r in range(R)]).astype(np.int64)).cuda()
    assert torch.equal(halo_chk, x[cols_all]), "world forward mismatch"
    del chk, halo_chk, cols_all
    log("parity: every rank's halo equals the direct gather x[N_r]")
    halo = torch.empty(H, C, dtype=dt, device="cuda")
    g_halo = torch.ones_like(halo)
    g_x = torch.empty_like(x)
    # locality plans take the backward through the plan's stages (each rank-local)
    batch = P.hx_batch_from_plan(plan, x, halo, flags=0 if plain else P.HX_WORLD_STAGED_BACKWARD)
    P.hx_batch_bind_grad(batch, g_halo, g_x)
    tune(args, torch, P, batch, name)
    cfg = {"workload": WORLD_DESC[name], "ranks": R, "halo_rows": H, "ncols": C, "plan_init_s": round(plan_s, 4),
           "internode_messages": int(sum(int(np.sum(P.hx_plan_field(plan, r, "s1_procs") // ppn != r // ppn))
                                         for r in range(R))),
           "internode_rows": int(sum(int(np.sum(P.hx_plan_field(plan, r, "s1_counts")[
               P.hx_plan_field(plan, r, "s1_procs") // ppn != r // ppn])) for r in range(R)))}
    # the differentiation workloads time forward + backward; the others are
    # forward (pack / redistribution / unpack) workloads, backward reported aside
    phases = (0, 1, 2, 3) if plain else (0, 1, 2)
    cfg["step"] = "pack + redistribution + unpack" + (" + backward" if 3 in phases else "")
    return dict(batch=batch, host=[], dtype="f64" if dt == torch.float64 else "f32", cfg=cfg, phases=phases,
                keep=(plan, x, halo, g_halo, g_x), plan=plan, n=n, H=H, C=C, torch_dtype=dt)


def setup_rank(args, torch, P, rank=1511):
    """One rank's share alone: the persistent request of the random matrix's
    rank with the most receive neighbors, from the 2-step locality plan; its
    receive arena holds what its peers would send (random values)."""
    from workloads import uniform_pm1
    rs, ppn, rp, cols = world_structure("rank1511")
    plan = P.hx_plan_from_csr(len(rs) - 1, rs, ppn, P.HX_LOCALITY_2STEP, torch.from_numpy(rp).cuda(),
                              torch.from_numpy(cols).cuda())
    n_local = int(rs[rank + 1] - rs[rank])
    H = int(P.hx_plan_field(plan, rank, "halo").size)
    x = torch.from_numpy(uniform_pm1(7337, n_local).reshape(n_local, 1)).cuda()
    halo = torch.empty(H, 1, dtype=torch.float64, device="cuda")
    req = P.hx_req_from_plan(plan, rank, x, halo)
    recv = P.req_arena_view(req, P.HX_ARENA_RECV, 1, torch.float64)
    recv.copy_(torch.from_numpy(uniform_pm1(99, recv.shape[0]).reshape(-1, 1)).cuda())
    # the backward of its pack: gradients of its stage-1 send slots summed into its rows
    E1 = int(P.hx_plan_field(plan, rank, "s1_idx").size)
    g_send = torch.from_numpy(uniform_pm1(101, E1).reshape(E1, 1)).cuda()
    g_x = torch.empty_like(x)
    P.hx_req_bind_grad(req, g_send, g_x)
    batch = P.hx_batch_init([req])
    tune(args, torch, P, batch, "rank1511")
    cfg = {"workload": f"random 2^22 x 32, locality 2-step plan, rank {rank} alone (its own request: "
                       f"{n_local} rows, halo {H}, 1 x FP64); warm, not an HBM figure",
           "rank": rank, "halo_rows": H, "recv_neighbors": int(P.hx_plan_field(plan, rank, "r1_procs").size)}
    return dict(batch=batch, host=[], dtype="f64", cfg=cfg, phases=(0, 1, 2),
                keep=(plan, x, halo, req, recv, g_send, g_x))


def tune(args, torch, P, batch, name):
    """Applies recorded schedules (--sched-json) or tunes the batch."""
    if args.sched_json:
        sj = json.loads(open(args.sched_json).read() if os.path.exists(args.sched_json) else args.sched_json)
        for ph, sc in sj.items():
            P.hx_batch_set_sched(batch, int(ph), sc)
    elif not args.no_tune:
        t0 = time.time()
        P.hx_batch_tune(batch)
        torch.cuda.synchronize()
        log(f"{name}: tuned in {time.time() - t0:.1f}s")
    if args.replay:
        P.hx_batch_set_replay(batch, P.HX_REPLAY_DIRECT if args.replay == "direct" else P.HX_REPLAY_GRAPH)


# ---------------------------------------------------------------------------
# Timing
# ---------------------------------------------------------------------------
def step_fns(P, plain, sp):
    fns = {0: P.hx_batch_start_plain if plain else P.hx_batch_start,
           2: P.hx_batch_wait_plain if plain else P.hx_batch_wait,
           3: P.hx_batch_backward_plain if plain else P.hx_batch_backward}
    return {k: (lambda b, f=f: f(b, sp)) for k, f in fns.items()}


def time_steps(torch, P, batch, steps, warmup, plain, phases):
    """Warm steps (Start + Wait [+ backward when 3 is in phases]): `steps`
    steps back to back between two synchronisations (wall clock, nothing
    else in the loop), then the same steps with events around each phase for
    the breakdown; a backward outside the step is timed afterwards for the
    report only."""
    sp = torch.cuda.current_stream().cuda_stream   # passed explicitly: no stream lookup per call
    run = step_fns(P, plain, sp)
    with_bwd = 3 in phases
    for _ in range(warmup):
        run[0](batch)
        run[2](batch)
        if with_bwd:
            run[3](batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run[0](batch)
        run[2](batch)
        if with_bwd:
            run[3](batch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for i in range(steps):
        ev[i][0].record()
        run[0](batch)
        ev[i][1].record()
        run[2](batch)
        ev[i][2].record()
        if with_bwd:
            run[3](batch)
        ev[i][3].record()
    torch.cuda.synchronize()
    ph = {"start": sum(e[0].elapsed_time(e[1]) for e in ev) / steps,
          "wait": sum(e[1].elapsed_time(e[2]) for e in ev) / steps,
          "backward": sum(e[2].elapsed_time(e[3]) for e in ev) / steps}
    if not with_bwd:
        run[3](batch)
        torch.cuda.synchronize()
        eb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in eb:
            a.record()
            run[3](batch)
            b.record()
        torch.cuda.synchronize()
        ph["backward"] = sum(a.elapsed_time(b) for a, b in eb) / steps
    return wall / steps * 1e3, ph


def time_cold(torch, P, batch, phases, flush, runs=20):
    """Median step time with the L2 and Infinity Cache flushed before each
    step (a 1 GiB write outside the timed range), events on the stream."""
    sp = torch.cuda.current_stream().cuda_stream
    run = step_fns(P, False, sp)
    ts = []
    for i in range(runs):
        flush.fill_(i)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run[0](batch)
        run[2](batch)
        if 3 in phases:
            run[3](batch)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def time_kernels(torch, P, batch, reps, phases):
    """Average duration of each phase's kernel, launched alone (the same
    launch table the step replays): per phase, `reps` launches back to back
    between two HIP events on the launch stream, queued behind a bounded
    spin kernel so that no host launch gap falls between them (as in a
    profiler's kernel trace)."""
    P.hx_batch_wait(batch)
    for p in phases:
        P.hx_batch_launch_phase(batch, p)
    torch.cuda.synchronize()
    out = {}
    for p in phases:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(20_000_000)
        e0.record()
        for _ in range(reps):
            P.hx_batch_launch_phase(batch, p)
        e1.record()
        torch.cuda.synchronize()
        out[p] = e0.elapsed_time(e1) / reps
    return out


NAMES = {0: "pack", 1: "redist", 2: "unpack", 3: "backward"}


def kernel_symbol(P, b, phase, row_bytes, staged):
    """Symbol of a phase's kernel (as profiles name it) under the batch's schedule."""
    sch = P.hx_batch_get_sched(b, phase)
    if phase == 3:
        sfx = "_vec" if sch["pair_rows"] == 1 and row_bytes in (4, 8) else ""
        return f"k_segsum_fwd{sfx} + k_segsum{sfx}" if staged else f"k_segsum{sfx}"
    base = {0: "k_pack", 1: "k_redist", 2: "k_unpack"}[phase]
    if phase == 0 and sch["push_pack"] == 1:
        return "k_pack_push"
    if sch["pair_rows"] == 1 and row_bytes in (4, 8):
        return base + "_vec"
    return base


def measure(name, S, args, torch, P, flush, plain=True):
    """One workload's figures: warm step throughput, cold median, phase
    breakdown, plain one-launch-per-plan form, each kernel alone and the
    dominant kernel against the HBM roofline."""
    b = S["batch"]
    nbytes = {ph: P.hx_batch_bytes(b, ph) for ph in range(4)}
    ms, ph = time_steps(torch, P, b, args.steps, args.warmup, False, S["phases"])
    log(f"{name}: {ms:.4f} ms/step; phases (ms) {json.dumps({k: round(v, 4) for k, v in ph.items()})}")
    cold = time_cold(torch, P, b, S["phases"], flush) if flush is not None else None
    plain_ms = None
    if plain:
        plain_ms, pph = time_steps(torch, P, b, max(3, args.steps // 4), 1, True, S["phases"])
        log(f"{name} plain: {plain_ms:.3f} ms/step; phases (ms) {json.dumps({k: round(v, 4) for k, v in pph.items()})}")
    step_bytes = sum(v for ph_id, v in nbytes.items() if ph_id != 3 or 3 in S["phases"])
    value = step_bytes / (ms * 1e-3) / 1e9
    kms = time_kernels(torch, P, b, max(10, args.steps // 2), [p for p in (0, 1, 2, 3) if nbytes[p] > 0])
    log(f"{name} kernels alone (ms): {json.dumps({NAMES[p]: round(t, 4) for p, t in kms.items()})}")
    step_k = {p: t for p, t in kms.items() if p != 3 or 3 in S["phases"]}
    dom_p = max(step_k, key=lambda p: step_k[p])
    achieved = nbytes[dom_p] / (kms[dom_p] * 1e-3) / 1e9
    row_bytes = S["cfg"].get("ncols", 16) * (8 if S["dtype"] == "f64" else 4)
    # (a locality world's staged backward is reported aside, never the step's dominant kernel)
    kname = kernel_symbol(P, b, dom_p, row_bytes, staged=False)
    traffic = read_traffic(kname, name)
    replay = P.hx_batch_get_replay(b)
    # steps that move a few MB last less than the launches they take: their
    # bandwidth measures launch cost, not memory, and is not set against the peak
    launch_bound = step_bytes < 64e6
    out = {
        "workload": S["cfg"], "value": round(value, 2), "unit": "GB/s",
        "pct_of_hbm_peak": None if launch_bound else round(100 * value / HBM_PEAK_GBPS, 2),
        "ms_per_step": round(ms, 4),
        "cold_ms_median": round(cold, 4) if cold is not None else None,
        "cold_gbps": round(step_bytes / (cold * 1e-3) / 1e9, 2) if cold else None,
        "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "kernel_ms": {NAMES[p]: round(t, 4) for p, t in kms.items()},
        "kernel_gbps": {NAMES[p]: round(nbytes[p] / (t * 1e-3) / 1e9, 1) for p, t in kms.items()},
        "phase_bytes": {NAMES[p]: nbytes[p] for p in range(4)},
        "bwd_in_step": 3 in S["phases"],
        "plain_ms_per_step": round(plain_ms, 4) if plain_ms else None,
        "speedup_batched_vs_plain": round(plain_ms / ms, 3) if plain_ms else None,
        "roofline": {"bound": "launch" if launch_bound else "hbm", "kernel": f"{kname} ({NAMES[dom_p]})",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": None if launch_bound else round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic},
        "replay": "direct" if replay == P.HX_REPLAY_DIRECT else "graph",
        "note": (f"launch-bound: one step moves {step_bytes / 1e6:.2f} MB ({step_bytes / HBM_PEAK_GBPS / 1e3:.2f} us "
                 f"at 8 TB/s), less than the cost of its launches; not an HBM figure") if launch_bound else None,
        "sched": {NAMES[p]: P.hx_batch_get_sched(b, p) for p in range(4) if nbytes[p] > 0},
    }
    return out, step_bytes


def time_halo_gather(S, args, torch, P):
    """diff64 through the autograd Function: zero-copy input (the exchange's
    own vector), aliased output, gradient handed over in the exchange's
    gradient buffer; the backward's returned gradient is a fresh tensor (a
    copy, inside the timed step)."""
    from paper_2309_07337_amd.autograd import HaloExchange, halo_gather
    ex = HaloExchange(S["plan"], S["n"], S["H"], S["C"], dtype=S["torch_dtype"], sim_transfer=False)
    if args.sched_json or not args.no_tune:
        for p in (0, 2, 3):   # the schedules tuned for the batch of the same plan
            P.hx_batch_set_sched(ex.batch, p, P.hx_batch_get_sched(S["batch"], p))
        P.hx_batch_set_replay(ex.batch, P.hx_batch_get_replay(S["batch"]))
    ex.x.copy_(S["keep"][1])
    ex.g_halo.fill_(1.0)
    x = ex.x.detach().requires_grad_(True)

    def step():
        x.grad = None
        y = halo_gather(x, ex, copy_out=False)
        y.backward(ex.g_halo)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    del ex, x
    return ms


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def _plan_bytes(U, E, h, rb):
    """Algorithmic bytes of one plan step: pack, identity unpack, backward."""
    return (E + U) * rb + 4 * E + 2 * h * rb + (E + h) * rb + 4 * (E + h + 1)


def cpu_baseline(setup, budget_s, c_runs=20, c_sample_bytes=6e9):
    """The oracle as it stands on the host's cores, same plans and byte
    accounting as the GPU step (pack, identity unpack, fixed-order backward;
    the transpose of the pack map is init work, built untimed):

    * all cores: the plain OpenMP loops of oracle/cpu_move.c over the first
      plans (about c_sample_bytes of algorithmic bytes per step), median of
      c_runs timed steps after two untimed ones;
    * one core: the numpy oracle, passes over the plans until about
      budget_s of CPU time (reported beside it)."""
    import numpy as np
    from oracle import cpu as OC
    from oracle import move as OM
    from oracle import plan as OP
    plans = []
    for hk in setup["host"]:
        h, C = hk["x"].shape
        E = hk["idx"].size
        ptr, perm = OP.transpose_csr(hk["idx"], h)
        plans.append((hk, ptr, perm, np.arange(h, dtype=np.int32), np.unique(hk["idx"]).size, E, h,
                      C * hk["x"].dtype.itemsize))
    model, ncpu, usable = host_cpu()
    # all cores: C loops, preallocated outputs
    sample, sbytes = [], 0
    for pl in plans:
        if sbytes >= c_sample_bytes:
            break
        hk, ptr, perm, ident, U, E, h, rb = pl
        outs = (np.empty((E,) + hk["x"].shape[1:], hk["x"].dtype), np.empty_like(hk["recv"]),
                np.empty_like(hk["x"]))
        sample.append((pl, outs))
        sbytes += _plan_bytes(U, E, h, rb)
    times = []
    for it in range(c_runs + 2):
        t0 = time.perf_counter()
        for (hk, ptr, perm, ident, U, E, h, rb), (send, halo, gx) in sample:
            OC.gather(hk["x"], hk["idx"], out=send)
            OC.gather(hk["recv"], None, out=halo)
            OC.transpose_sum(send, ptr, perm, out=gx)   # any [E, C] gradient of this shape
        if it >= 2:
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    # one core: the numpy oracle
    done_bytes, t, passes, nplans = 0, 0.0, 0, 0
    while t < budget_s and plans:
        for hk, ptr, perm, ident, U, E, h, rb in plans:
            t0 = time.perf_counter()
            OM.pack(hk["x"], hk["idx"])
            OM.gather_rows(hk["recv"], ident)
            OM.pack_transpose(hk["x"][:E], ptr, perm)
            t += time.perf_counter() - t0
            done_bytes += _plan_bytes(U, E, h, rb)
            nplans += 1
            if t >= budget_s:
                break
        passes += 1
    return {"value": round(sbytes / med / 1e9, 3), "unit": "GB/s", "cores": OC.threads(), "kind": "oracle",
            "sample": f"first {len(sample)} of 256 plans ({sbytes / 1e9:.2f} GB algorithmic per step): pack, "
                      f"identity unpack and fixed-order transpose sum as plain OpenMP C loops, median of "
                      f"{c_runs} steps ({med * 1e3:.1f} ms)",
            "cpu_model": model, "nproc": ncpu, "cpus_usable": usable,
            "numpy_1core": {"value": round(done_bytes / t / 1e9, 3) if t > 0 else None, "unit": "GB/s", "cores": 1,
                            "kind": "oracle",
                            "sample": f"{nplans} plan steps over the first {len(plans)} of 256 plans ({passes} "
                                      f"pass(es), {done_bytes / 1e9:.2f} GB algorithmic in {t:.1f} s): numpy "
                                      "pack (np.take), identity unpack, fixed-order transpose sum"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    workloads = ["batched256", "random_rows", "random_rows_f32", "random_rows_3step", "rank1511", "diff64",
                 "grid3d_diff64", "grid3d", "grid2d", "copy"]
    ap.add_argument("--workload", default="batched256", choices=workloads)
    ap.add_argument("--plans", type=int, default=256)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="headline workload only")
    ap.add_argument("--no-cold", action="store_true", help="skip the flushed-cache median")
    ap.add_argument("--sched-json", default="", help="per-phase schedules to apply instead of tuning "
                                                     "(JSON text or file: {\"0\": {...}, ...})")
    ap.add_argument("--replay", choices=["graph", "direct"], default="")
    ap.add_argument("--cpu-plans", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "hx runs on one GPU only: one rank's share (or a batch of "
                                   "ranks) per GPU; no collectives between GPUs. Use --gpus 1."}))
        sys.exit(2)
    import gc
    import torch
    import paper_2309_07337_amd as P
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    flush = None if args.no_cold else torch.empty(1 << 28, dtype=torch.int32, device="cuda")  # 1 GiB

    def setup(name):
        if name == "batched256":
            return setup_batched(args, torch, P)
        args.cpu_plans = 0
        if name == "copy":
            return setup_copy(args, torch, P)
        if name == "rank1511":
            return setup_rank(args, torch, P)
        return setup_world(args, torch, P, name)

    with torch.cuda.stream(stream):
        cpu_plans = args.cpu_plans
        S = setup(args.workload)
        head, step_bytes = measure(args.workload, S, args, torch, P, flush, plain=not args.no_plain)
        if args.workload in ("diff64", "grid3d_diff64"):
            head["through_autograd_ms_per_step"] = round(time_halo_gather(S, args, torch, P), 4)
    args.cpu_plans = cpu_plans
    cpu = cpu_baseline(S, args.cpu_seconds) if S["host"] else None
    head_dtype = S["dtype"]
    del S
    configs = {}
    if args.workload == "batched256" and not args.no_configs:
        for name in ("random_rows", "random_rows_f32", "random_rows_3step", "rank1511", "diff64",
                     "grid3d_diff64", "grid3d", "grid2d"):
            gc.collect()
            torch.cuda.empty_cache()
            with torch.cuda.stream(stream):
                Sc = setup(name)
                res, sb = measure(name, Sc, args, torch, P, None if name == "rank1511" else flush,
                                  plain=name not in ("rank1511",) and not args.no_plain)
                if name in ("diff64", "grid3d_diff64"):
                    ams = time_halo_gather(Sc, args, torch, P)
                    res["through_autograd_ms_per_step"] = round(ams, 4)
                    res["through_autograd_gbps"] = round(sb / (ams * 1e-3) / 1e9, 2)
            configs[name] = res
            del Sc
    out = {
        "metric": "effective HBM GB/s (fwd pack+unpack, bwd) and % of peak; batched vs plain",
        "value": head["value"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": head_dtype, "data": "synthetic (seeded SplitMix64)",
        "config": head.pop("workload"),
    }
    head.pop("value")
    head.pop("unit")
    head.pop("ms_per_step")
    out.update(head)
    out["cpu_baseline"] = cpu
    if configs:
        out["configs"] = configs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
