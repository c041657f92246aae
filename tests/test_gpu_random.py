"""GPU: a seeded random sweep over the option space.  Each case draws an
image size, a match count, K (around the 64/128 boundaries of the K-NN's
register and LDS sorts), NW or LA, 4- or 8-connectivity, the LA weight
power, FP32 or FP64-everywhere, and some matches outside the image or on
shared pixels; every stage of the HIP path is checked against the oracle
(FP32 with the parity tolerances, FP64 bit-exact for D, L and the K-NN
lists), and the device's own invariant checks (debug_validate: transform
fixpoint, seeds, labels, graph symmetry) report nothing.  Needs an MI355X."""
from __future__ import annotations

import numpy as np
import pytest

import parity
from scenes import random_case

pytestmark = pytest.mark.gpu

KS = [1, 2, 3, 5, 8, 16, 32, 50, 64, 65, 100, 128, 129, 200, 256]


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    for i in range(n):
        H = int(rng.integers(8, 300))
        W = int(rng.integers(8, 300))
        N = int(rng.integers(2, min(3000, H * W // 3) + 2))
        yield dict(i=i, H=H, W=W, N=N, K=int(rng.choice(KS)), mode=int(rng.integers(0, 2)),
                   conn=int(rng.choice([8, 8, 8, 4])), wpow=int(rng.choice([2, 2, 1])),
                   prec=int(rng.choice([0, 0, 0, 1])), outside=int(rng.integers(0, 4)),
                   dup=int(rng.integers(0, 6)), seed=int(rng.integers(0, 1 << 30)))


def test_random_sweep():
    import paper_1501_02565_amd as epic
    ctxs = {}
    try:
        for c in _cases(80, 2024):
            key = (c["conn"], c["wpow"], c["prec"])
            if key not in ctxs:
                ctxs[key] = epic.Context(0, 2 * epic.workspace_bytes(400, 400, 4000, 256, 1, c["prec"]),
                                         connectivity=c["conn"], la_weight_power=c["wpow"],
                                         precision=c["prec"], debug_validate=1)
            ctx = ctxs[key]
            print(f"[case] {c}", flush=True)
            sc = random_case(c["H"], c["W"], c["N"], seed=c["seed"], K=c["K"], mode=c["mode"],
                             outside=min(c["outside"], c["N"] - 1), duplicates=min(c["dup"], c["N"] // 3))
            if c["prec"] == 0:
                parity.full_check(ctx, sc, conn=c["conn"], wpow=c["wpow"])
                assert ctx.stats(0)["n_invariant"] == 0, ctx.stats(0)
                continue
            g = parity.gpu_stages(ctx, sc)
            assert ctx.stats(0)["n_invariant"] == 0, ctx.stats(0)
            r = parity.ref_stages(sc, conn=c["conn"], wpow=c["wpow"])
            np.testing.assert_array_equal(g["D"], r["D"])
            np.testing.assert_array_equal(g["L"], r["L"])
            K = r["K"]
            np.testing.assert_array_equal(g["knn_idx"][:, :K], r["knn_idx"])
            if np.isfinite(r["flow"]).all():
                epe = np.linalg.norm(g["flow"].astype(np.float64) - r["flow"], axis=2)
                assert epe.mean() <= 1e-5, epe.mean()
    finally:
        for ctx in ctxs.values():
            ctx.close()
