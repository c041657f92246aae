"""Autotuner for the batched form.

For a batch of pairs, tries the launch configurations the library exposes
(geodesic tile shape, number of bulk-synchronous passes launched per call
and threads per tile of the later passes), times each as a captured HIP graph replay on the GPU, and keeps the
fastest.  Results are cached in a JSON file keyed by a shape bucket (the
multiset of (W, H, N rounded, K) of the batch), so a served or batched
workload tunes once.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

# (tile, passes) or (tile, passes, threads per tile of the later passes; 0 =
# the library's default)
DEFAULT_CANDIDATES = [((32, 16), 12), ((32, 16), 16), ((32, 16), 24),
                      ((32, 16), 12, 128), ((32, 16), 16, 128),
                      ((32, 32), 12), ((32, 32), 16), ((32, 64), 12)]


def bucket_key(shapes) -> str:
    """shapes: iterable of (H, W, N, K).  N is rounded to 1000s."""
    norm = sorted((int(H), int(W), int(round(N / 1000.0)), int(K)) for H, W, N, K in shapes)
    return hashlib.sha1(json.dumps(norm).encode()).hexdigest()[:16]


def cache_path() -> str:
    base = os.environ.get("EPIC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1501_02565_amd"))
    return os.path.join(base, "tune.json")


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, p)
    except OSError:
        pass


def time_graph(ctx, problems, reps=10, warmup=2):
    """Mean milliseconds of one replay of the captured batch."""
    import torch
    g = ctx.capture(problems)
    try:
        for _ in range(warmup):
            g.launch()
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            g.launch()
        end.record()
        torch.cuda.synchronize()
        return start.elapsed_time(end) / reps
    finally:
        g.close()


def tune(problems, workspace, candidates=None, reps=10, use_cache=True, device=0, **ctx_opts):
    """problems: list of (cost, matches, K, a, mode) CUDA tensors.
    Returns dict(tile=(w, h), passes=p, threads=t, ms=best_ms, trials=[...])."""
    import paper_1501_02565_amd as epic
    shapes = [(c.shape[0], c.shape[1], m.shape[0], K) for c, m, K, _, _ in problems]
    key = bucket_key(shapes)
    cache = load_cache() if use_cache else {}
    if key in cache:
        r = cache[key]
        return dict(tile=tuple(r["tile"]), passes=r["passes"], threads=r.get("threads", 0), ms=r["ms"],
                    trials=r.get("trials", []), cached=True)
    trials = []
    t0 = time.perf_counter()
    for cand in (candidates or DEFAULT_CANDIDATES):
        tile, passes = cand[0], cand[1]
        threads = cand[2] if len(cand) > 2 else 0
        with epic.Context(device, workspace, tile=tile, passes=passes, geo_threads=threads, **ctx_opts) as ctx:
            ms = time_graph(ctx, problems, reps=reps)
        trials.append(dict(tile=list(tile), passes=passes, threads=threads, ms=ms))
    best = min(trials, key=lambda t: t["ms"])
    out = dict(tile=tuple(best["tile"]), passes=best["passes"], threads=best["threads"], ms=best["ms"],
               trials=trials, cached=False, tune_s=time.perf_counter() - t0)
    if use_cache:
        cache[key] = dict(tile=best["tile"], passes=best["passes"], threads=best["threads"], ms=best["ms"],
                          trials=trials)
        save_cache(cache)
    return out
