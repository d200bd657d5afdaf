#!/usr/bin/env python3
"""Benchmark of the halo-exchange buffer engine on one MI355X.

Default workload ("batched256"): 256 independent persistent exchange plans,
halo sizes log-uniform in [1e3, 1e6) rows, 1..4096 neighbors, 16 FP64
columns per row.  One step = Start + Wait of all plans (pack, unpack) plus
the backward of the pack (fixed-order transpose sum), each phase one
multi-job kernel replayed from a hipGraph.  The same work as one launch per
plan per phase ("plain") is timed beside it.

Other workloads (``--workload``): random_rows / random_rows_f32 /
random_rows_3step (2^22 x 32 random matrix, 4096 ranks, 2-step or 3-step
locality-aware plan, every rank batched, one FP64 / FP32 column; forward
step, the staged backward reported aside), grid3d
(27-point 128^3, 512 ranks), grid2d (5-point 512^2, 16 ranks), diff64
(random-matrix plain plan, 64 FP32 features, forward + backward), copy (the
1 GiB calibration copy for the PMC scale factors).

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
# Workloads
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
    if not args.no_tune:
        t0 = time.time()
        P.hx_batch_tune(batch)
        torch.cuda.synchronize()
        log(f"tuned in {time.time() - t0:.1f}s: " + json.dumps([P.hx_batch_get_sched(batch, ph) for ph in range(4)]))
    # correctness of a sampled member against the oracle before timing
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
    return dict(batch=batch, members=members, host=host_keep, dtype="f64", cfg=cfg, phases=(0, 2, 3),
                keep=members)


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
    return dict(batch=batch, members=[req], host=[], dtype="f64", cfg=cfg, phases=(0, 2, 3),
                keep=(req, x, halo, g_x, topo))


def setup_world(args, torch, P, name):
    import numpy as np
    from workloads import equal_row_starts, grid2d_5pt, grid3d_27pt, random_rows, uniform_pm1, uniform_pm1_f32
    t0 = time.time()
    if name in ("random_rows", "random_rows_f32", "random_rows_3step", "diff64"):
        rp, cols = random_rows()
        rs, ppn = equal_row_starts(1 << 22, 4096), 128
    elif name == "grid3d":
        rp, cols = grid3d_27pt()
        rs, ppn = equal_row_starts(128 ** 3, 512), 64
    else:
        rp, cols = grid2d_5pt()
        rs, ppn = equal_row_starts(512 * 512, 16), 4
    log(f"generated {name} structure in {time.time() - t0:.1f}s")
    variant = P.HX_PLAIN if name == "diff64" else (P.HX_LOCALITY_3STEP if name.endswith("3step")
                                                    else P.HX_LOCALITY_2STEP)
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
    if name == "diff64":
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
    batch = P.hx_batch_from_plan(plan, x, halo, flags=0 if variant == P.HX_PLAIN else P.HX_WORLD_STAGED_BACKWARD)
    P.hx_batch_bind_grad(batch, g_halo, g_x)
    if not args.no_tune:
        P.hx_batch_tune(batch)
    cfg = {"workload": {"random_rows": "random 2^22 x 32 (70% in-block), 4096 ranks, 128/node, locality "
                                       "2-step, all ranks batched, 1 x FP64",
                        "random_rows_f32": "random 2^22 x 32 (70% in-block), 4096 ranks, 128/node, locality "
                                           "2-step, all ranks batched, 1 x FP32",
                        "random_rows_3step": "random 2^22 x 32 (70% in-block), 4096 ranks, 128/node, locality "
                                             "3-step (one message per node pair), all ranks batched, 1 x FP64",
                        "grid3d": "27-point 128^3, 512 ranks, 64/node, locality 2-step, all ranks, 1 x FP64",
                        "grid2d": "5-point 512^2, 16 ranks, 4/node, locality 2-step, all ranks, 1 x FP64",
                        "diff64": "random 2^22 x 32, 4096 ranks, plain plan, 64 x FP32 features, forward "
                                  "halo gather + fixed-order transpose-sum backward"}[name],
           "ranks": R, "halo_rows": H, "ncols": C, "plan_init_s": round(plan_s, 4),
           "internode_messages": int(sum(int(np.sum(P.hx_plan_field(plan, r, "s1_procs") // ppn != r // ppn))
                                         for r in range(R))),
           "internode_rows": int(sum(int(np.sum(P.hx_plan_field(plan, r, "s1_counts")[
               P.hx_plan_field(plan, r, "s1_procs") // ppn != r // ppn])) for r in range(R)))}
    # the differentiation workload times forward + backward; the others are
    # forward (pack / redistribution / unpack) workloads, backward reported aside
    phases = (0, 1, 2, 3) if name == "diff64" else (0, 1, 2)
    cfg["step"] = "pack + redistribution + unpack" + (" + backward" if 3 in phases else "")
    return dict(batch=batch, members=None, host=[], dtype="f64" if dt == torch.float64 else "f32", cfg=cfg,
                phases=phases, keep=(plan, x, halo, g_halo, g_x))


# ---------------------------------------------------------------------------
def time_steps(torch, P, batch, steps, warmup, plain, phases):
    """Times `steps` steps (Start + Wait [+ backward when 3 is in phases]);
    a backward outside the step is timed afterwards for the report only."""
    sp = torch.cuda.current_stream().cuda_stream   # passed explicitly: no stream lookup per call
    fns = {0: P.hx_batch_start_plain if plain else P.hx_batch_start,
           2: P.hx_batch_wait_plain if plain else P.hx_batch_wait,
           3: P.hx_batch_backward_plain if plain else P.hx_batch_backward}
    run = {k: (lambda b, f=f: f(b, sp)) for k, f in fns.items()}
    with_bwd = 3 in phases
    for _ in range(warmup):
        run[0](batch)
        run[2](batch)
        if with_bwd:
            run[3](batch)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
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
    wall = time.perf_counter() - t0
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


def time_kernels(torch, P, batch, reps, phases):
    """Average duration of each phase's kernel launched alone: events on the
    current stream around `reps` back-to-back launches (queued faster than
    they run, so the host's launch cost stays hidden)."""
    P.hx_batch_wait(batch)
    out = {}
    for p in phases:
        P.hx_batch_launch_phase(batch, p)
        torch.cuda.synchronize()
        a, c = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            P.hx_batch_launch_phase(batch, p)
        c.record()
        torch.cuda.synchronize()
        out[p] = a.elapsed_time(c) / reps
    return out


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
    ap.add_argument("--workload", default="batched256",
                    choices=["batched256", "random_rows", "random_rows_f32", "random_rows_3step", "grid3d", "grid2d",
                             "diff64", "copy"])
    ap.add_argument("--plans", type=int, default=256)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-plans", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "hx runs on one GPU only: one rank's share (or a batch of "
                                   "ranks) per GPU; no collectives between GPUs. Use --gpus 1."}))
        sys.exit(2)
    import torch
    import paper_2309_07337_amd as P
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        if args.workload == "batched256":
            S = setup_batched(args, torch, P)
        elif args.workload == "copy":
            args.cpu_plans = 0
            S = setup_copy(args, torch, P)
        else:
            args.cpu_plans = 0
            S = setup_world(args, torch, P, args.workload)
        b = S["batch"]
        nbytes = {ph: P.hx_batch_bytes(b, ph) for ph in range(4)}
        ms, ph = time_steps(torch, P, b, args.steps, args.warmup, False, S["phases"])
        log(f"batched: {ms:.3f} ms/step; phases (ms) {json.dumps({k: round(v, 4) for k, v in ph.items()})}")
        plain_ms = None
        if not args.no_plain:
            plain_ms, pph = time_steps(torch, P, b, max(3, args.steps // 4), 1, True, S["phases"])
            log(f"plain:   {plain_ms:.3f} ms/step; phases (ms) {json.dumps({k: round(v, 4) for k, v in pph.items()})}")
    step_bytes = sum(v for ph_id, v in nbytes.items() if ph_id != 3 or 3 in S["phases"])
    value = step_bytes / (ms * 1e-3) / 1e9
    # dominant kernel: each phase's kernel timed alone (same launch
    # table as the graphs, same stream), the longest one of the step
    names = {0: "pack", 1: "redist", 2: "unpack", 3: "backward"}
    with torch.cuda.stream(stream):
        kms = time_kernels(torch, P, b, max(5, args.steps // 2), [p for p in (0, 1, 2, 3) if nbytes[p] > 0])
    step_k = {p: t for p, t in kms.items() if p != 3 or 3 in S["phases"]}
    dom_p = max(step_k, key=lambda p: step_k[p])
    dom = names[dom_p]
    achieved = nbytes[dom_p] / (kms[dom_p] * 1e-3) / 1e9
    kname = {"pack": "k_pack", "redist": "k_redist", "unpack": "k_unpack", "backward": "k_segsum"}[dom]
    sch = P.hx_batch_get_sched(b, dom_p)
    row_bytes = S["cfg"].get("ncols", 16) * (8 if S["dtype"] == "f64" else 4)
    if dom == "pack" and sch["push_pack"] == 1:
        kname = "k_pack_push"
    elif dom != "backward" and sch["pair_rows"] == 1 and row_bytes == 8:
        kname += "_pair"   # 8-byte rows two per lane
    log(f"kernels alone (ms): {json.dumps({names[p]: round(t, 4) for p, t in kms.items()})}")
    traffic = read_traffic(kname, args.workload)
    cpu = cpu_baseline(S, args.cpu_seconds) if S["host"] else None
    out = {
        "metric": "effective HBM GB/s (fwd pack+unpack, bwd) and % of peak; batched vs plain",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": S["dtype"], "data": "synthetic (seeded SplitMix64)",
        "config": S["cfg"],
        "pct_of_hbm_peak": round(100 * value / HBM_PEAK_GBPS, 2),
        "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "kernel_ms": {names[p]: round(t, 4) for p, t in kms.items()},
        "phase_bytes": {"pack": nbytes[0], "redist": nbytes[1], "unpack": nbytes[2], "backward": nbytes[3]},
        "fwd_gbps": round((nbytes[0] + nbytes[1] + nbytes[2]) / ((ph["start"] + ph["wait"]) * 1e-3) / 1e9, 2),
        "bwd_gbps": round(nbytes[3] / (ph["backward"] * 1e-3) / 1e9, 2) if ph["backward"] > 0 else None,
        "bwd_in_step": 3 in S["phases"],
        "plain_ms_per_step": round(plain_ms, 4) if plain_ms else None,
        "plain_gbps": round(step_bytes / (plain_ms * 1e-3) / 1e9, 2) if plain_ms else None,
        "speedup_batched_vs_plain": round(plain_ms / ms, 3) if plain_ms else None,
        "roofline": {"bound": "hbm", "kernel": f"{kname} ({dom})", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
