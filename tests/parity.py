"""Stage-by-stage comparison of the GPU library with the FP64 oracle.

Tolerances (stated once, used by every parity test):
  * geodesic distance D: relative 1e-5 wherever the labels agree;
  * labels L: at most 0.1% of pixels may differ, and every differing pixel
    must be a near-tie -- the oracle's distance from the GPU's match to the
    pixel is within 1e-5 (relative) of the oracle's minimum;
  * graph weights and K-NN distances: relative 1e-5 (edges and neighbours
    that differ must be explained by label near-ties / distance near-ties);
  * dense flow: mean endpoint difference to the oracle flow <= 1e-3 px.
"""
from __future__ import annotations

import numpy as np

from oracle import epic_ref

REL = 1e-5
LABEL_FRAC = 1e-3
EPE_MEAN = 1e-3


def gpu_stages(ctx, sc, K=None, a=None, mode=None):
    import torch
    dev = torch.device("cuda:0")
    cost = torch.from_numpy(np.ascontiguousarray(sc.cost)).to(dev)
    m = torch.from_numpy(np.ascontiguousarray(sc.matches)).to(dev)
    out = ctx.debug_stages(cost, m, sc.K if K is None else K,
                           sc.a if a is None else a,
                           sc.mode if mode is None else mode)
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    return res


def ref_stages(sc, K=None, a=None, mode=None, conn=8, wpow=2):
    return epic_ref.stages(sc.cost, sc.matches, sc.K if K is None else K,
                           sc.a if a is None else a,
                           sc.mode if mode is None else mode, conn=conn, wpow=wpow)


def check_labels(sc, g, r, conn=8, frac=LABEL_FRAC):
    """D within REL where labels agree; disagreements are rare near-ties."""
    Dg, Lg = g["D"].astype(np.float64), g["L"]
    Dr, Lr = r["D"], r["L"]
    same = Lg == Lr
    np.testing.assert_allclose(Dg[same], Dr[same], rtol=REL, atol=1e-30)
    diff = np.argwhere(~same)
    assert len(diff) <= frac * Lg.size, f"{len(diff)} label differences"
    if len(diff):
        H, W = sc.cost.shape
        for lab in np.unique(Lg[~same]):
            src = int(r["seed_pix"][lab])
            assert src >= 0
            Ds = epic_ref.geodesic_from(sc.cost, src, conn)
            pts = (Lg == lab) & ~same
            np.testing.assert_allclose(Ds[pts], Dr[pts], rtol=REL)
            np.testing.assert_allclose(Dg[pts], Dr[pts], rtol=REL)
    return int((~same).sum())


def check_graph(g, r, n_label_diff):
    ge = {(int(m), int(n)): float(w) for m, n, w in zip(g["em"], g["en"], g["ew"])}
    re_ = {(int(m), int(n)): float(w) for m, n, w in zip(r["em"], r["en"], r["ew"])}
    common = ge.keys() & re_.keys()
    sym = (ge.keys() - re_.keys()) | (re_.keys() - ge.keys())
    if n_label_diff == 0:
        assert not sym, f"edge sets differ: {sorted(sym)[:10]}"
    else:
        assert len(sym) <= max(4, 0.005 * len(re_)), len(sym)
    bad = [e for e in common if abs(ge[e] - re_[e]) > REL * re_[e]]
    if n_label_diff == 0:
        assert not bad, f"edge weights differ: {[(e, ge[e], re_[e]) for e in bad[:5]]}"
    else:
        assert len(bad) <= max(4, 0.005 * len(common)), len(bad)
    return len(sym), len(bad)


def check_knn(g, r, K, tol_frac=0.0):
    """Neighbour lists: the same set with distances within REL, except where
    the K-th distance is a near-tie or the graph differs (tol_frac)."""
    gi, gd = g["knn_idx"][:, :K], g["knn_d"][:, :K].astype(np.float64)
    ri, rd = r["knn_idx"][:, :K], r["knn_d"][:, :K]
    N = ri.shape[0]
    mismatched = 0
    for s in range(N):
        if ri[s, 0] < 0:
            assert gi[s, 0] == -1
            continue
        if set(gi[s].tolist()) == set(ri[s].tolist()) and \
                np.allclose(gd[s], rd[s], rtol=REL, atol=1e-30):
            continue
        # a near-tie at the K-th neighbour swaps members of equal distance
        kth = rd[s][rd[s] < np.inf].max()
        only = set(gi[s].tolist()) ^ set(ri[s].tolist())
        dmap = dict(zip(ri[s].tolist(), rd[s].tolist()))
        dmap.update({k: v for k, v in zip(gi[s].tolist(), gd[s].tolist()) if k not in dmap})
        if all(abs(dmap[n] - kth) <= 10 * REL * kth for n in only):
            continue
        mismatched += 1
    assert mismatched <= tol_frac * N, f"{mismatched} K-NN lists differ"
    return mismatched


def check_flow(g, r, epe_mean=EPE_MEAN):
    fg = g["flow"].astype(np.float64)
    fr = r["flow"]
    if np.isnan(fr).all():
        assert np.isnan(fg).all()
        return 0.0
    epe = np.linalg.norm(fg - fr, axis=2)
    assert np.isfinite(epe).all()
    assert epe.mean() <= epe_mean, f"mean EPE {epe.mean():.3e}"
    return float(epe.mean())


def full_check(ctx, sc, K=None, a=None, mode=None, conn=8, wpow=2, knn_tol=0.0):
    K = sc.K if K is None else K
    g = gpu_stages(ctx, sc, K, a, mode)
    r = ref_stages(sc, K, a, mode, conn, wpow)
    st = g["stats"]
    assert st["n_outside"] == r["n_outside"]
    assert st["n_duplicate"] == r["n_duplicate"]
    assert st["n_used"] == r["used"]
    if r["used"] == 0:
        assert st["status"] == -3
        assert np.isnan(g["flow"]).all()
        return dict(label_diff=0, epe=0.0)
    assert st["status"] == 0, st
    nd = check_labels(sc, g, r, conn)
    check_graph(g, r, nd)
    Keff = r["K"]
    check_knn(g, r, Keff, tol_frac=knn_tol if nd == 0 else max(knn_tol, 0.01))
    epe = check_flow(g, r)
    return dict(label_diff=nd, epe=epe, stats=st)
