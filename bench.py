#!/usr/bin/env python3
"""Benchmark of the sparse-to-dense interpolation on one MI355X.

Headline: interpolated Mpix/s on the 1024x436 large-displacement scene with
8000 matches, K=100, a=1, LA (synthetic stand-in for an MPI-Sintel pair).
One step = one whole interpolation (seed, geodesic transform, graph,
per-match K-NN + fit, assignment) of that pair, inputs resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes per unit of work of each stage: every stage reads its
# inputs once and writes its outputs once (no re-reads, no sweeps counted).
#   geodesic:    read C (4 B/px), write the (D, L) state (8 B/px)
#   graph_emit:  read C and the (D, L) state (12 B/px)
#   assign:      read L (4 B/px), write flow (8 B/px)
#   knn_fit:     per match: CSR row (8 B/edge, ~6 edges) + row offsets (8 B)
#                + lightest edge (4 B) + match (16 B) + model (24 B)
STAGE_BYTES_PER_PX = {"geodesic": 12.0, "graph_emit": 12.0, "assign": 12.0}
KNN_BYTES_PER_MATCH = 6 * 8 + 8 + 4 + 16 + 24


def stage_bytes(stage, HW, N, E, precision=0):
    if stage in STAGE_BYTES_PER_PX:
        # FP64 everywhere: D is 8 bytes and L a separate 4 bytes
        extra = 4.0 if precision == 1 and stage in ("geodesic", "graph_emit") else 0.0
        return (STAGE_BYTES_PER_PX[stage] + extra) * HW
    if stage == "knn_fit":
        return (2 * E * 8 + N * (8 + 4 + 16 + 24))
    if stage == "csr_scatter":
        return E * 12 + 2 * E * 8
    if stage == "clear":
        return 8 * HW
    if stage == "seed":
        return 16 * N + 8 * N
    return 0.0


def measured_traffic(stage):
    """HBM bytes per call of `stage` from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "epic_1024x436_n8000_k100_hbm_counters.txt")
    csrc = os.path.join(ROOT, "paper_1501_02565_amd", "csrc")
    try:
        # the kernel's source and the device header it includes
        h = hashlib.sha1()
        for f in ("k_geodesic.hip", "epic_dev.h"):
            h.update(open(os.path.join(csrc, f), "rb").read())
        cur = h.hexdigest()[:12]
        for line in open(prof):
            if line.startswith("TRAFFIC " + stage + " "):
                kv = dict(t.split("=") for t in line.split()[2:])
                if kv.get("source_sha1") == cur:
                    return float(kv["bytes_per_call"])
    except OSError:
        pass
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, seconds):
    """The FP64 oracle on the host cores, on the same scene, repeated for a
    bounded time: once with all its OpenMP threads (the reported value) and
    once on one core (the paper's setting)."""
    from oracle import epic_ref
    epic_ref.lib()
    cores = epic_ref.max_threads()

    def timed(threads, budget):
        epic_ref.set_threads(threads)
        reps, t0 = 0, time.perf_counter()
        while True:
            epic_ref.interp(sc.cost, sc.matches, sc.K, sc.a, sc.mode)
            reps += 1
            el = time.perf_counter() - t0
            if (el >= budget and reps >= 2) or reps >= 200:
                break
        return reps, el

    reps, el = timed(cores, seconds)
    reps1, el1 = timed(1, seconds)
    epic_ref.set_threads(cores)
    px = sc.H * sc.W
    return {"value": round(reps * px / el / 1e6, 4), "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} full interpolations of the {sc.W}x{sc.H} scene "
                      f"({sc.N} matches, K={sc.K}) in {el:.1f} s on {cores} threads",
            "single_core": {"value": round(reps1 * px / el1 / 1e6, 4), "unit": "Mpix/s", "cores": 1,
                            "ms_per_call": round(el1 / reps1 * 1e3, 1),
                            "sample": f"{reps1} full interpolations in {el1:.1f} s on 1 thread"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            # context only: the paper's one timing of this path (another
            # machine, about 5000 matches of a real pair, precision not stated)
            "paper_context": {"interp_s": 0.25, "mpix_s": round(px / 0.25 / 1e6, 3), "cores": 1,
                              "clock_ghz": 3.6, "workload": "1024x436 Sintel pair, ~5000 matches, LA"}}


def copy_bandwidth(torch, nbytes=256 << 20, reps=20):
    """A plain device-to-device copy of `nbytes`, timed with HIP events:
    the bandwidth HBM actually gives a streaming kernel on this GPU."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_per_copy": 2 * nbytes, "ms": round(ms, 4), "gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def error_vs_oracle(ctx, sc, np, torch):
    """Every result's error against the FP64 oracle: relative D error where
    labels agree, label disagreement, endpoint error of the flow."""
    from oracle import epic_ref
    dev = torch.device("cuda:0")
    g = ctx.debug_stages(torch.from_numpy(sc.cost).to(dev), torch.from_numpy(sc.matches).to(dev),
                         sc.K, sc.a, sc.mode)
    r = epic_ref.stages(sc.cost, sc.matches, sc.K, sc.a, sc.mode)
    D, L, f = g["D"].cpu().numpy().astype(np.float64), g["L"].cpu().numpy(), g["flow"].cpu().numpy()
    same = L == r["L"]
    drel = np.abs(D[same] - r["D"][same]) / np.maximum(r["D"][same], 1e-30)
    epe = np.linalg.norm(f.astype(np.float64) - r["flow"], axis=2)
    return {"max_rel_D_err": float(drel.max()), "mean_rel_D_err": float(drel.mean()),
            "label_disagreement_pct": float(100.0 * (~same).mean()),
            "mean_epe_px": float(epe.mean()), "max_epe_px": float(epe.max())}


def latency(ctx, sc, torch, mode, reps=20, warm=3):
    """Median wall latency of one call (enqueue to completion) on the plain
    single-pair path."""
    dev = torch.device("cuda:0")
    c = torch.from_numpy(sc.cost).to(dev)
    m = torch.from_numpy(sc.matches).to(dev)
    out = torch.empty((sc.H, sc.W, 2), dtype=torch.float32, device=dev)
    ts = []
    for i in range(warm + reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.interp(c, m, sc.K, sc.a, mode, out=out)
        torch.cuda.synchronize()
        if i >= warm:
            ts.append(time.perf_counter() - t0)
    ms = sorted(ts)[len(ts) // 2] * 1e3
    return {"workload": sc.name, "mode": "LA" if mode == 1 else "NW", "K": sc.K, "a": sc.a,
            "p50_ms": round(ms, 4), "mpix_s": round(sc.H * sc.W / ms / 1e3, 1)}


def pruned_leg(args, np, torch, epic, sc, steps=50):
    """The headline call with the consistency check of the matches (Sec.
    5.1, threshold 5 px): an NW pass, the compaction of the kept matches,
    then the interpolation of those; its error against the oracle's pruned
    interpolation."""
    from oracle import epic_ref
    dev = torch.device("cuda:0")
    c = torch.from_numpy(sc.cost).to(dev)
    m = torch.from_numpy(sc.matches).to(dev)
    out = torch.empty((sc.H, sc.W, 2), dtype=torch.float32, device=dev)
    with epic.Context(0, epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K), prune_px=5.0) as ctx:
        for _ in range(5):
            ctx.interp(c, m, sc.K, sc.a, sc.mode, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.interp(c, m, sc.K, sc.a, sc.mode, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        st = ctx.stats(0)
    ref, rc, _, kept = epic_ref.interp_pruned(sc.cost, sc.matches, sc.K, sc.a, sc.mode, 5.0)
    epe = np.linalg.norm(out.cpu().numpy().astype(np.float64) - ref, axis=2)
    res = {"workload": sc.name + "_pruned5px", "ms_per_step": round(ms, 5),
           "mpix_s": round(sc.H * sc.W / ms / 1e3, 1), "kept": st["n_used"], "pruned": st["n_pruned"],
           "oracle_kept": int(len(kept)), "mean_epe_vs_oracle_px": float(epe.mean()),
           "max_epe_vs_oracle_px": float(epe.max())}
    log(f"bench: pruned {res}")
    return res


def image_cost_leg(np, torch, epic, reps=20):
    """The cost maps of the 64-pair batch's RGB images from their gradient
    (Table 2, norm-of-gradient row): an HBM-bound stencil, 12 B read and
    4 B written per pixel, timed with HIP events on the current stream."""
    from scenes import batch_scenes
    scs = batch_scenes(64, with_image=True)
    imgs = [torch.from_numpy(s.image).cuda() for s in scs]
    outs = [torch.empty((s.H, s.W), dtype=torch.float32, device="cuda") for s in scs]
    plan = epic.ImageCostPlan(imgs, outs)      # descriptors marshalled once
    for _ in range(3):
        plan.run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    px = sum(s.H * s.W for s in scs)
    nbytes = 16.0 * px
    gbs = nbytes / (ms * 1e-3) / 1e9
    res = {"workload": f"gradient cost of 64 RGB images, {px / 1e6:.2f} Mpx", "ms": round(ms, 4),
           "launches": 1, "algorithmic_bytes": nbytes, "achieved_gbs": round(gbs, 1),
           "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "mpix_s": round(px / ms / 1e3, 1)}
    log(f"bench: image cost {res}")
    return res


def exact_leg(np, torch, epic, full_size=True):
    """The exact per-pixel geodesic interpolation (Table 2, "Geodesic
    (exact)"): its time, its error against the oracle (all pixels of the
    small scene, 48 sampled pixels of the large one), and -- as Table 2
    compares -- the average endpoint error of the approximated and the exact
    flow against the scene's generating motion."""
    from oracle import epic_ref
    from scenes import config_scene
    out = []
    for i in ((1, 2) if full_size else (1,)):
        sc = config_scene(i)
        c = torch.from_numpy(sc.cost).cuda()
        m = torch.from_numpy(sc.matches).cuda()
        ws = 8 * sc.K * sc.H * sc.W + sc.N + 4096 + min(1024, sc.N) * epic.workspace_bytes(sc.H, sc.W, 1, 1) \
            + (64 << 20)
        with epic.Context(0, ws) as ctx:
            ts = []
            for rep in range(3 if i == 2 else 6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fe = ctx.interp_exact(c, m, sc.K, sc.a, sc.mode)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            fa = ctx.interp(c, m, sc.K, sc.a, sc.mode).cpu().numpy().astype(np.float64)
        fe = fe.cpu().numpy().astype(np.float64)
        ms = sorted(ts[1:])[len(ts[1:]) // 2] * 1e3
        HW = sc.H * sc.W
        pix = np.arange(HW) if i == 1 else np.linspace(0, HW - 1, 48).astype(np.int64)
        rf = epic_ref.exact(sc.cost, sc.matches, sc.K, sc.a, sc.mode, pixels=pix)[0]
        e = np.linalg.norm(fe.reshape(-1, 2)[pix] - rf, axis=1)
        gt = sc.gt_flow.astype(np.float64)
        res = {"workload": sc.name, "ms": round(ms, 3), "mpix_s": round(HW / ms / 1e3, 3),
               "vs_oracle": {"pixels": int(len(pix)), "mean_epe_px": float(e.mean()), "max_epe_px": float(e.max())},
               "aee_vs_generating_motion": {"approximated": float(np.linalg.norm(fa - gt, axis=2).mean()),
                                            "exact": float(np.linalg.norm(fe - gt, axis=2).mean())},
               "mean_diff_approx_exact_px": float(np.linalg.norm(fa - fe, axis=2).mean())}
        log(f"bench: exact {res}")
        out.append(res)
    return out


def refine_leg(np, torch, epic, reps=10):
    """The one-level variational refinement (Sec. 4) of the interpolated
    field of each single-pair scene with an image pair: its time alone and
    after the interpolation (both on one stream, HIP events), the average
    endpoint error against the scene's generating motion before and after,
    and its difference from the oracle (both refining the oracle's own
    interpolation).  The sweeps run blocked in time, 12 half-sweeps per
    launch of the sweep kernel; its algorithmic bytes per launch are, per
    pixel, 36 B of the fixed-point step's system and 8 B of (du, dv) read
    and 8 B written (52 B)."""
    from oracle import epic_ref
    from oracle import variational as va
    from scenes import config_scene
    out = []
    p = epic.refine_params()
    for i in (1, 2):
        sc = config_scene(i, with_pair=True)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
        c, m, I1, I2 = t(sc.cost), t(sc.matches), t(sc.image), t(sc.image2)
        HW = sc.H * sc.W
        ws = epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K) + epic.refine_bytes(sc.H, sc.W, 3) + (1 << 20)
        with epic.Context(0, ws) as ctx:
            flow = ctx.interp(c, m, sc.K, sc.a, sc.mode)
            ref_out = ctx.refine(I1, I2, flow)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for _ in range(3):
                ctx.refine(I1, I2, flow, out=ref_out)
            e0.record()
            for _ in range(reps):
                ctx.refine(I1, I2, flow, out=ref_out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            e0.record()
            for _ in range(reps):
                ctx.interp(c, m, sc.K, sc.a, sc.mode, out=flow)
                ctx.refine(I1, I2, flow, out=ref_out)
            e1.record()
            torch.cuda.synchronize()
            ms_both = e0.elapsed_time(e1) / reps
            f0 = flow.cpu().numpy().astype(np.float64)
            f1 = ref_out.cpu().numpy().astype(np.float64)
            u0 = epic_ref.interp(sc.cost, sc.matches, sc.K, sc.a, sc.mode)[0].astype(np.float32)
            g = ctx.refine(I1, I2, t(u0)).cpu().numpy().astype(np.float64)
        r = va.refine(sc.image, sc.image2, u0)
        d = np.linalg.norm(g - r, axis=2)
        gt = sc.gt_flow.astype(np.float64)
        sweep_launches = p.fixed_point * -(-2 * p.sor // 12)
        res = {"workload": sc.name + "_pair", "ms": round(ms, 4), "interp_plus_refine_ms": round(ms_both, 4),
               "mpix_s": round(HW / ms / 1e3, 2), "fixed_point": p.fixed_point, "sor": p.sor,
               "launches": 4 + p.fixed_point + sweep_launches, "sweep_launches": sweep_launches,
               "sweep_algorithmic_bytes_per_launch": 52.0 * HW,
               "aee_vs_generating_motion": {"interpolated": float(np.linalg.norm(f0 - gt, axis=2).mean()),
                                            "refined": float(np.linalg.norm(f1 - gt, axis=2).mean())},
               "vs_oracle": {"mean_epe_px": float(d.mean()), "max_epe_px": float(d.max())}}
        log(f"bench: refine {res}")
        out.append(res)
    return out


def batched_form(args, np, torch, epic):
    """The 64-pair mixed-size batch: one fused launch sequence per batch,
    captured as a HIP graph with the autotuned configuration, against the
    plain single-pair form (one epic_interp call per pair) on the same GPU."""
    from oracle import epic_ref
    from paper_1501_02565_amd import tune
    from scenes import batch_scenes
    t0 = time.perf_counter()
    scs = batch_scenes(64)
    log(f"bench: batch scenes generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    probs = [(torch.from_numpy(sc.cost).to(dev), torch.from_numpy(sc.matches).to(dev), sc.K, sc.a, sc.mode)
             for sc in scs]
    px = sum(sc.H * sc.W for sc in scs)
    need = sum(epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K) for sc in scs)
    if args.batch_config:
        # WxH/passes[/threads]
        vals = [int(v) for v in args.batch_config.replace("/", "x").split("x")]
        best = {"tile": (vals[0], vals[1]), "passes": vals[2], "threads": vals[3] if len(vals) > 3 else 0,
                "ms": float("nan"), "trials": []}
        log(f"bench: batch configuration {best['tile']} passes {best['passes']} threads {best['threads']} "
            "(not tuned)")
    else:
        best = tune.tune(probs, need, reps=5, use_cache=False)
        log(f"bench: tuned {best['tile']} passes {best['passes']} threads {best['threads']} "
            f"({best['ms']:.3f} ms); trials "
            + ", ".join(f"{t['tile']}/{t['passes']}/{t['threads']}: {t['ms']:.3f}" for t in best["trials"]))
    with epic.Context(0, need, tile=best["tile"], passes=best["passes"], geo_threads=best["threads"]) as ctx:
        g = ctx.capture(probs)
        for _ in range(3):
            g.launch()
        torch.cuda.synchronize()
        reps = max(3, args.batch_reps)
        t0 = time.perf_counter()
        for _ in range(reps):
            g.launch()
        torch.cuda.synchronize()
        ms_batch = (time.perf_counter() - t0) / reps * 1e3
        flows = [f.cpu().numpy() for f in g.flows]
        stats = [ctx.stats(i) for i in range(len(scs))]
        g.close()
        # the plain single-pair form on the same pairs and GPU
        ms_plain = float("nan")
        if not args.no_plain:
            for c, m, K, a, mode in probs[:4]:
                ctx.interp(c, m, K, a, mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c, m, K, a, mode in probs:
                ctx.interp(c, m, K, a, mode)
            torch.cuda.synchronize()
            ms_plain = (time.perf_counter() - t0) * 1e3
    assert all(st["status"] == 0 for st in stats), stats
    epes = []
    for i in (0, 21, 42, 63):
        ref = epic_ref.interp(scs[i].cost, scs[i].matches, scs[i].K, scs[i].a, scs[i].mode)[0]
        epes.append(float(np.linalg.norm(flows[i].astype(np.float64) - ref, axis=2).mean()))
    nm = sum(sc.N for sc in scs)
    path_gbs = (36.0 * px + 150.0 * nm) / (ms_batch * 1e-3) / 1e9
    out = {"workload": f"batch of 64 mixed pairs, {px / 1e6:.2f} Mpx, {nm} matches",
           "mpix_s": round(px / ms_batch / 1e3, 2), "ms_per_batch": round(ms_batch, 4),
           "path_roofline": {"achieved": round(path_gbs, 2), "frac": round(path_gbs / HBM_PEAK_GBS, 6)},
           "plain_mpix_s": None if args.no_plain else round(px / ms_plain / 1e3, 2),
           "plain_ms": None if args.no_plain else round(ms_plain, 4),
           "speedup_vs_plain": None if args.no_plain else round(ms_plain / ms_batch, 3),
           "tuned": {"tile": list(best["tile"]), "passes": best["passes"], "threads": best["threads"]},
           "sampled_mean_epe_vs_oracle_px": epes}
    log(f"bench: batched {out}")
    return out


def served_form(args, np, torch, epic, precision, reqs_in, samples):
    """Poisson stream (mean 5 ms between arrivals) of mixed-size pairs, each
    with its own match count, through the continuous-batching server;
    latency = completion - arrival.  Then the same requests all queued at
    once (the server saturated): pixels over that wall time is the served
    capacity.  `samples` (request ids) keep their flows for the oracle."""
    from paper_1501_02565_amd.serve import GpuExecutor, Server, percentile_ms

    def fresh(r, arrival):
        return dataclasses.replace(r, arrival=arrival, admitted=None, done=None, status="waiting",
                                   batch=-1, flow=None)
    ex = GpuExecutor(slots=2, slot_workspace=args.served_budget // 2, precision=precision)
    # the loop polls without sleeping and wakes 0.3 ms before each arrival
    srv = Server(ex, args.served_budget, max_batch=64, idle_s=0.0, wake_early_s=3e-4)
    # warm up every kernel variant once
    Server(ex, args.served_budget, max_batch=64).run([fresh(reqs_in[0], 0.0)])
    reqs = [fresh(r, r.arrival) for r in reqs_in]
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    ok = [r for r in done if r.status == "done"]
    assert all(r.stats["status"] == 0 for r in ok), [r.stats for r in ok if r.stats["status"]][:3]
    # each result alone equals its result in the mix
    ident, max_epe = 0, 0.0
    sample = ok[:: max(1, len(ok) // 16)][:16]
    for r in sample:
        c = torch.from_numpy(r.cost).cuda()
        m = torch.from_numpy(r.matches).cuda()
        alone = ex.ctx[0].interp(c, m, r.K, r.a, r.mode).cpu().numpy()
        mixed = r.flow.cpu().numpy()
        ident += int(np.array_equal(alone, mixed))
        max_epe = max(max_epe, float(np.linalg.norm(alone.astype(np.float64) - mixed, axis=2).mean()))
    kept = {r.rid: r.flow.cpu().numpy() for r in ok if r.rid in samples}
    px = sum(r.pixels for r in ok)
    # saturation: every request waiting at t = 0
    srv_sat = Server(ex, args.served_budget, max_batch=64, idle_s=0.0)
    sat = [fresh(r, 0.0) for r in reqs_in]
    t0 = time.perf_counter()
    srv_sat.run(sat)
    wall_sat = time.perf_counter() - t0
    ex.close()
    span = max(r.arrival for r in reqs_in)
    out = {"precision": "fp64-everywhere" if precision else "fp32",
           "requests": len(done), "served": len(ok), "rejected": len(done) - len(ok),
           "p50_ms": round(percentile_ms([r.latency for r in ok], 50), 3),
           "p99_ms": round(percentile_ms([r.latency for r in ok], 99), 3),
           "capacity_mpix_s": round(sum(r.pixels for r in sat) / wall_sat / 1e6, 2),
           "capacity_wall_s": round(wall_sat, 3), "capacity_batches": srv_sat.batches,
           "offered_load_mpix_s": round(px / span / 1e6, 2), "wall_s": round(wall, 3),
           "batches": srv.batches, "overlapped_batches": srv.overlap_events,
           "alone_vs_mix": {"checked": len(sample), "bitwise_identical": ident,
                            "max_mean_epe_px": max_epe}}
    log(f"bench: served {out}")
    return out, kept


def served_pair(args, np, torch, epic):
    """Both served paths (FP32 and FP64-everywhere) on one stream, with each
    path's error against the oracle on 16 sampled requests."""
    from oracle import epic_ref
    from paper_1501_02565_amd.serve import Request
    from scenes import serve_bases, serve_stream
    t0 = time.perf_counter()
    stream = serve_stream(args.served_requests)
    bases = serve_bases()
    pinned_cost = {}

    def pinned(a):
        # request inputs arrive in page-locked host memory (a DMA-able receive
        # buffer), so their upload runs on the slot's stream
        t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
        t.numpy()[...] = a
        return t
    reqs, scenes = [], {}
    for i, r in enumerate(stream):
        key = (r["H"], r["W"])
        if key not in pinned_cost:
            pinned_cost[key] = pinned(bases[key].cost)
        sc = bases[key].request(r)
        pm = pinned(sc.matches)
        reqs.append(Request(i, r["arrival"], sc.H, sc.W, sc.N, sc.K, sc.a, sc.mode,
                            pinned_cost[key].numpy(), pm.numpy()))
        scenes[i] = sc
    log(f"bench: {len(reqs)} served requests drawn in {time.perf_counter() - t0:.1f} s "
        f"(N {min(r.N for r in reqs)}..{max(r.N for r in reqs)})")
    samples = set(range(0, len(reqs), max(1, len(reqs) // 16)))
    out, flows = {}, {}
    for name, prec in (("fp32", 0), ("fp64", 1)):
        out[name], flows[name] = served_form(args, np, torch, epic, prec, reqs, samples)
    t0 = time.perf_counter()
    epes = {"fp32": [], "fp64": []}
    for rid in sorted(samples):
        sc = scenes[rid]
        ref = epic_ref.interp(sc.cost, sc.matches, sc.K, sc.a, sc.mode)[0]
        for name in epes:
            if rid in flows[name]:
                e = np.linalg.norm(flows[name][rid].astype(np.float64) - ref, axis=2)
                epes[name].append((float(e.mean()), float(e.max())))
    for name in epes:
        v = epes[name]
        out[name]["error_vs_oracle"] = {"sampled": len(v),
                                        "mean_epe_px": float(np.mean([a for a, _ in v])) if v else None,
                                        "worst_mean_epe_px": max(a for a, _ in v) if v else None,
                                        "max_epe_px": max(b for _, b in v) if v else None}
    log(f"bench: served oracle check of {len(samples)} requests in {time.perf_counter() - t0:.1f} s: "
        + ", ".join(f"{k} {out[k]['error_vs_oracle']}" for k in epes))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default="32x16", help="geodesic tile WxH")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 1],
                    help="headline leg: 0 = FP32 path (default), 1 = FP64 everywhere")
    ap.add_argument("--passes", type=int, default=0,
                    help="geodesic passes per call (0 = automatic budget)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--batch-config", default="",
                    help="batched form: fixed WxH/passes[/threads] (e.g. 32x16/12) instead of autotuning")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched form: skip the single-pair comparison loop")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact per-pixel interpolation leg")
    ap.add_argument("--no-refine", action="store_true", help="skip the variational refinement leg")
    ap.add_argument("--served-requests", type=int, default=2000)
    ap.add_argument("--served-budget", type=int, default=8 << 30)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--only-headline", action="store_true",
                    help="only the single-pair measurement and the device copy (profiling runs)")
    ap.add_argument("--only-batched", action="store_true",
                    help="skip the single-pair measurement (profiling the batched form)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py: the library runs on one GPU (--gpus 1); sharding over "
            "several GPUs is not implemented")
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1501_02565_amd as epic
    from scenes import config_scene

    if args.only_batched:
        print(json.dumps({"batched": batched_form(args, np, torch, epic)}), flush=True)
        return
    sc = config_scene(2)
    HW = sc.H * sc.W
    dev = torch.device("cuda:0")
    cost = torch.from_numpy(sc.cost).to(dev)
    matches = torch.from_numpy(sc.matches).to(dev)
    flow = torch.empty((sc.H, sc.W, 2), dtype=torch.float32, device=dev)
    tile = tuple(int(v) for v in args.tile.split("x"))
    ctx = epic.Context(0, epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K, precision=args.precision), tile=tile,
                       passes=args.passes, precision=args.precision)
    stream = torch.cuda.current_stream()

    log(f"bench: {sc.name} warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.interp(cost, matches, sc.K, sc.a, sc.mode, out=flow)
    torch.cuda.synchronize()
    st = ctx.stats(0)
    if st["status"] != 0:
        raise SystemExit(f"bench: device status {st}")

    # ---------------------------------------------------------- timed region
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.interp(cost, matches, sc.K, sc.a, sc.mode, out=flow)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el / args.steps * 1e3
    mpix = args.steps * HW / el / 1e6
    log(f"bench: {ms_step:.4f} ms/step, {mpix:.1f} Mpix/s")

    # the same call replayed as a captured HIP graph (launch sequence
    # recorded once; inputs resident, identical work per step)
    g = ctx.capture([(cost, matches, sc.K, sc.a, sc.mode)], outs=[flow])
    for _ in range(args.warmup):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.launch()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) / args.steps * 1e3
    g.close()
    log(f"bench: graph replay {graph_ms:.4f} ms/step, {HW / graph_ms / 1e3:.1f} Mpix/s")

    # ------------------------------------- per-stage HIP events (same stream)
    ctx.profile(True)
    nprof = min(64, args.steps)
    for _ in range(nprof):
        ctx.interp(cost, matches, sc.K, sc.a, sc.mode, out=flow)
    stages = ctx.stage_times(nprof)
    pass_visits = ctx.pass_visits()        # of the last profiled call
    ctx.profile(False)
    E = st["n_edges"]
    log(f"bench: stats {st}")
    log("bench: stage ms " + ", ".join(f"{k}={v:.4f}" for k, v in stages.items()))
    log(f"bench: transform tile visits per pass {pass_visits}")
    dom = max(stages, key=lambda k: stages[k])
    dom_ms = stages[dom]
    nbytes = stage_bytes(dom, HW, sc.N, E, args.precision)
    achieved = nbytes / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": measured_traffic(dom) if args.precision == 0 else None,
                "kernel": dom, "kernel_ms": round(dom_ms, 5),
                "algorithmic_bytes": nbytes}

    # the path as a whole against the HBM roofline: 36 B per pixel plus
    # ~150 B per match of algorithmic traffic per step
    path_bytes = 36.0 * HW + 150.0 * sc.N
    path_gbs = path_bytes / (ms_step * 1e-3) / 1e9
    roofline["path"] = {"algorithmic_bytes": path_bytes, "achieved": round(path_gbs, 2),
                        "frac": round(path_gbs / HBM_PEAK_GBS, 6)}

    # error of the timed result against the oracle (every stage)
    err = error_vs_oracle(ctx, sc, np, torch)
    log(f"bench: error vs oracle {err}")
    ctx.close()

    lat = pruned = imcost = exact = refine = batched = served = cpu = None
    if args.only_headline:
        copy = copy_bandwidth(torch)
        roofline["copy_kernel_gbs"] = copy["gbs"]
        log(f"bench: device copy {copy}")
    else:
        # latency of the other single-pair workloads (NW and LA on the road scene)
        lat = []
        with epic.Context(0, epic.workspace_bytes(436, 1242, 10000, 100)) as c2:
            for i, mode in ((1, 1), (3, 1), (3, 0)):
                s_i = config_scene(i, mode=mode)
                lat.append(latency(c2, s_i, torch, mode))
        log(f"bench: latency {lat}")
        # the consistency check of the matches (Sec. 5.1) before the same call
        pruned = pruned_leg(args, np, torch, epic, sc)
        copy = copy_bandwidth(torch)
        roofline["copy_kernel_gbs"] = copy["gbs"]
        imcost = image_cost_leg(np, torch, epic)
        exact = None if args.no_exact else exact_leg(np, torch, epic)
        refine = None if args.no_refine else refine_leg(np, torch, epic)
        imcost["frac_of_copy"] = round(imcost["achieved_gbs"] / copy["gbs"], 4)
        log(f"bench: device copy {copy}")
        if args.calibrate_copy:
            log("bench: calibration copy of 256 MiB done")
        batched = None if args.no_batched else batched_form(args, np, torch, epic)
        served = None if args.no_served else served_pair(args, np, torch, epic)
        if not args.no_cpu_baseline:
            log("bench: timing the oracle on the host")
            cpu = cpu_baseline(sc, args.cpu_seconds)
            log(f"bench: oracle {cpu}")

    out = {
        "metric": "interpolated Mpix/s (1024x436, 8k matches, K=100); served p50/p99 latency",
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 1 else "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "H": sc.H, "W": sc.W, "N": sc.N, "K": sc.K,
                   "a": sc.a, "mode": "LA", "error_vs_oracle": err,
                   "stage_ms": {k: round(v, 5) for k, v in stages.items()},
                   "graph_replay_ms_per_step": round(graph_ms, 5),
                   "transform_tiles": -(-sc.W // tile[0]) * -(-sc.H // tile[1]),
                   "transform_visits_per_pass": pass_visits,
                   "latency_other_configs": lat},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
        "pruned": pruned,
        "image_cost": imcost,
        "exact": exact,
        "refine": refine,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
