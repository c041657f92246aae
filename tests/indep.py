"""Independent brute-force implementations used to pin the oracle.

Nothing here is shared with the oracle or with the GPU library: shortest
paths come from scipy.sparse.csgraph, least squares from numpy.linalg.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import dijkstra, floyd_warshall

OFFS8 = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, 1), (1, -1), (-1, -1)]
OFFS4 = OFFS8[:4]


def pixel_graph(cost, conn=8):
    """Sparse pixel graph; a step between adjacent pixels costs the step
    length times the mean cost of its two end pixels."""
    H, W = cost.shape
    c = cost.astype(np.float64)
    rows, cols, vals = [], [], []
    idx = np.arange(H * W).reshape(H, W)
    for dx, dy in (OFFS8 if conn == 8 else OFFS4):
        ys0, ys1 = max(0, -dy), min(H, H - dy)
        xs0, xs1 = max(0, -dx), min(W, W - dx)
        p = idx[ys0:ys1, xs0:xs1]
        q = idx[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
        ln = math.sqrt(2.0) if dx and dy else 1.0
        w = ln * 0.5 * (c[ys0:ys1, xs0:xs1] + c[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx])
        rows.append(p.ravel())
        cols.append(q.ravel())
        vals.append(w.ravel())
    g = coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                   shape=(H * W, H * W)).tocsr()
    return g


def seed_pixels(H, W, matches):
    """Round half up; outside -> -1; first (lowest index) match keeps a pixel."""
    out = np.full(len(matches), -1, np.int64)
    taken = set()
    for m, (x, y) in enumerate(np.asarray(matches, np.float64)[:, :2]):
        if not (math.isfinite(x) and math.isfinite(y)):
            continue
        ix, iy = math.floor(x + 0.5), math.floor(y + 0.5)
        if 0 <= ix < W and 0 <= iy < H and (iy * W + ix) not in taken:
            taken.add(iy * W + ix)
            out[m] = iy * W + ix
    return out


def all_source_distances(cost, seed_pix, conn=8):
    """(N_used, HW) matrix of single-source distances and the match ids."""
    g = pixel_graph(cost, conn)
    ids = np.nonzero(seed_pix >= 0)[0]
    return dijkstra(g, indices=seed_pix[ids]), ids


def floyd_all_pairs(cost, conn=8):
    return floyd_warshall(pixel_graph(cost, conn))


def restricted_distance(cost, L, m, n, sm, sn, conn=8):
    """Shortest path from pixel sm to pixel sn using only pixels whose label
    is m or n."""
    H, W = cost.shape
    keep = np.nonzero((L.ravel() == m) | (L.ravel() == n))[0]
    g = pixel_graph(cost, conn)[keep][:, keep]
    pos = {int(p): i for i, p in enumerate(keep)}
    d = dijkstra(g, indices=pos[int(sm)])
    return d[pos[int(sn)]]


def graph_dist_matrix(N, em, en, ew):
    g = coo_matrix((np.concatenate([ew, ew]),
                    (np.concatenate([em, en]), np.concatenate([en, em]))),
                   shape=(N, N)).tocsr()
    return dijkstra(g)


def knn_from_matrix(Dg, s, K, valid):
    d = Dg[s].copy()
    d[~valid] = np.inf
    order = np.lexsort((np.arange(len(d)), d))
    order = order[np.isfinite(d[order])]
    return order[:K], d[order[:K]]


def nw_fit(disp, k):
    return np.average(disp, axis=0, weights=k)


def la_fit_absolute(pos, tgt, k):
    """Eq. (2) literally: rows k * [x, y, 1] for the affine map p' = A p + t,
    solved by numpy least squares.  Returns (A, t)."""
    A = np.column_stack([pos, np.ones(len(pos))]) * k[:, None]
    sol, *_ = np.linalg.lstsq(A, tgt * k[:, None], rcond=None)
    return sol[:2].T, sol[2]


def octile(dx, dy):
    a, b = np.maximum(abs(dx), abs(dy)), np.minimum(abs(dx), abs(dy))
    return (a - b) + math.sqrt(2.0) * b
