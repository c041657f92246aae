"""Pins for the FP64 oracle: each stage is checked against something other
than itself -- scipy shortest paths, Floyd-Warshall, closed forms, brute
force on tiny inputs, numpy least squares, and the paper's own identities
(the per-pixel approximated distance of Eq. (4) and the piecewise claim of
Sec. 3.4).  CPU only."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import indep
from scenes import random_case

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(seed, H=14, W=17, N=9, conn=8):
    rng = np.random.default_rng(seed)
    cost = (rng.uniform(0.01, 1.0, (H, W))).astype(np.float32)
    pix = rng.choice(H * W, N, replace=False)
    m = np.zeros((N, 4), np.float32)
    m[:, 0] = pix % W
    m[:, 1] = pix // W
    m[:, 2:] = m[:, :2] + rng.normal(0, 3, (N, 2)).astype(np.float32)
    return cost, m


# ---------------------------------------------------------------- seeds --

def test_seed_rounding_and_drops(ref):
    H, W = 4, 5
    m = np.array([[2.5, 1.0, 0, 0],      # -> (3, 1)
                  [2.49, 1.0, 0, 0],     # -> (2, 1)
                  [-0.5, 0.0, 0, 0],     # -> (0, 0)
                  [-0.51, 0.0, 0, 0],    # outside
                  [4.5, 0.0, 0, 0],      # x -> 5 == W: outside
                  [3.4, 0.6, 0, 0],      # -> (3, 1): duplicate of match 0
                  [0.0, 3.49, 0, 0],     # -> (0, 3)
                  [np.nan, 1, 0, 0]],    # not finite
                 np.float32)
    sp, no, nd = ref.seeds(H, W, m)
    assert sp.tolist() == [1 * W + 3, 1 * W + 2, 0, -1, -1, -1, 3 * W, -1]
    assert (no, nd) == (3, 1)
    assert sp.tolist() == indep.seed_pixels(H, W, m).tolist()


# -------------------------------------------------------------- voronoi --

@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_voronoi_matches_scipy_dijkstra(ref, seed, conn):
    cost, m = _rand_problem(seed, H=23, W=31, N=15)
    sp, _, _ = ref.seeds(*cost.shape, m)
    D, L = ref.voronoi(cost, sp, conn)
    Dall, ids = indep.all_source_distances(cost, sp, conn)
    Dmin = Dall.min(0)
    np.testing.assert_allclose(D.ravel(), Dmin, rtol=1e-12, atol=0)
    # the label is a minimiser; among (near-)equal minimisers the lowest id
    Lr = L.ravel()
    for p in range(cost.size):
        tied = ids[Dall[:, p] <= Dmin[p] * (1 + 1e-12)]
        assert Lr[p] == tied.min()


@pytest.mark.parametrize("seed", [3, 4])
def test_voronoi_floyd_warshall(ref, seed):
    cost, m = _rand_problem(seed, H=11, W=12, N=5)
    sp, _, _ = ref.seeds(*cost.shape, m)
    D, L = ref.voronoi(cost, sp, 8)
    FW = indep.floyd_all_pairs(cost, 8)
    want = FW[sp[sp >= 0]].min(0)
    np.testing.assert_allclose(D.ravel(), want, rtol=1e-12)
    lab = np.nonzero(sp >= 0)[0][FW[sp[sp >= 0]].argmin(0)]
    assert (L.ravel() == lab).all()


def test_constant_cost_octile_closed_form(ref):
    """Constant cost c: the 8-connected geodesic is c times the octile
    distance; 4-connected it is c times the Manhattan distance."""
    H, W, c = 19, 23, 0.75
    cost = np.full((H, W), c, np.float32)
    sx, sy = 7, 11
    D8 = ref.geodesic_from(cost, sy * W + sx, 8)
    D4 = ref.geodesic_from(cost, sy * W + sx, 4)
    ys, xs = np.mgrid[0:H, 0:W]
    np.testing.assert_allclose(D8, c * indep.octile(xs - sx, ys - sy), rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(D4, c * (abs(xs - sx) + abs(ys - sy)))


def test_constant_cost_manhattan_voronoi_ties(ref):
    """Manhattan distances are exact integers, so ties are exact: the lowest
    match index must win them."""
    H, W = 9, 13
    cost = np.ones((H, W), np.float32)
    m = np.array([[10, 4, 0, 0], [2, 4, 0, 0], [6, 0, 0, 0]], np.float32)
    sp, _, _ = ref.seeds(H, W, m)
    D, L = ref.voronoi(cost, sp, 4)
    ys, xs = np.mgrid[0:H, 0:W]
    d = np.stack([abs(xs - x) + abs(ys - y) for x, y in m[:, :2]])
    np.testing.assert_array_equal(D, d.min(0))
    np.testing.assert_array_equal(L, d.argmin(0))     # argmin = first = lowest id


@pytest.mark.parametrize("conn", [8, 4])
def test_cost_scaling(ref, conn):
    """C -> 2^k C scales D exactly and keeps L; a general factor keeps L
    except at near-ties and scales D to rounding."""
    cost, m = _rand_problem(7, H=30, W=40, N=25)
    sp, _, _ = ref.seeds(*cost.shape, m)
    D, L = ref.voronoi(cost, sp, conn)
    D2, L2 = ref.voronoi(cost * np.float32(4.0), sp, conn)
    np.testing.assert_array_equal(D2, 4.0 * D)
    np.testing.assert_array_equal(L2, L)
    s = np.float32(1.7)
    D3, L3 = ref.voronoi(cost * s, sp, conn)
    np.testing.assert_allclose(D3, D * float(s), rtol=1e-6)
    assert (L3 != L).mean() < 0.01


def test_golden_strip(ref):
    """Hand-worked 1 x 6 strip (tests/golden/strip_1x6.txt)."""
    g = {}
    with open(os.path.join(GOLDEN, "strip_1x6.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split("=")
                g[k.strip()] = [float(t) for t in v.split()]
    cost = np.array([g["cost"]], np.float32)
    m = np.array([[x, 0, x + 1, 0] for x in g["seeds_x"]], np.float32)
    sp, _, _ = ref.seeds(1, 6, m)
    for conn in (4, 8):
        D, L = ref.voronoi(cost, sp, conn)
        np.testing.assert_array_equal(D[0], g["D"])
        np.testing.assert_array_equal(L[0], g["L"])
        em, en, ew = ref.graph(cost, D, L, conn)
        assert em.tolist() == [0] and en.tolist() == [1]
        assert ew.tolist() == g["W01"]


def test_golden_cross(ref):
    """Hand-worked 3 x 3 grid, unit cost, seed in the centre: axial
    neighbours at 1, corners at sqrt(2) (8-connected) or 2 (4-connected)."""
    cost = np.ones((3, 3), np.float32)
    D8 = ref.geodesic_from(cost, 4, 8)
    D4 = ref.geodesic_from(cost, 4, 4)
    r2 = math.sqrt(2.0)
    assert D8.tolist() == [[r2, 1, r2], [1, 0, 1], [r2, 1, r2]]
    assert D4.tolist() == [[2, 1, 2], [1, 0, 1], [2, 1, 2]]


# ---------------------------------------------------------------- graph --

@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("seed", [0, 5])
def test_graph_weight_is_restricted_geodesic(ref, seed, conn):
    """Edge weight == shortest path between the two matches through their
    two Voronoi cells only (brute force on the restricted pixel graph); an
    edge exists exactly when the cells touch."""
    cost, m = _rand_problem(seed, H=18, W=22, N=12)
    sp, _, _ = ref.seeds(*cost.shape, m)
    D, L = ref.voronoi(cost, sp, conn)
    em, en, ew = ref.graph(cost, D, L, conn)
    assert (em < en).all()
    for a, b, w in zip(em, en, ew):
        want = indep.restricted_distance(cost, L, a, b, sp[a], sp[b], conn)
        assert abs(w - want) <= 1e-12 * want
    # adjacency: touching cells <-> edge
    H, W = cost.shape
    touch = set()
    for dx, dy in (indep.OFFS8 if conn == 8 else indep.OFFS4):
        for y in range(H):
            for x in range(W):
                if 0 <= x + dx < W and 0 <= y + dy < H:
                    a, b = L[y, x], L[y + dy, x + dx]
                    if a != b:
                        touch.add((min(a, b), max(a, b)))
    assert touch == set(zip(em.tolist(), en.tolist()))


# ------------------------------------------------------------------ knn --

@pytest.mark.parametrize("seed", [0, 1])
def test_knn_matches_scipy(ref, seed):
    sc = random_case(40, 50, 60, seed=seed, outside=3, duplicates=2)
    st = ref.stages(sc.cost, sc.matches, 12, 1.0, 1)
    N = sc.N
    Dg = indep.graph_dist_matrix(N, st["em"], st["en"], st["ew"])
    valid = st["seed_pix"] >= 0
    for s in range(N):
        if not valid[s]:
            assert (st["knn_idx"][s] == -1).all()
            continue
        idx, d = indep.knn_from_matrix(Dg, s, 12, valid)
        assert idx[0] == s and d[0] == 0
        np.testing.assert_allclose(st["knn_d"][s], d, rtol=1e-12)
        assert st["knn_idx"][s].tolist() == idx.tolist()


def test_knn_clamps_k_to_used(ref):
    sc = random_case(20, 20, 7, seed=3, outside=2)
    st = ref.stages(sc.cost, sc.matches, 50, 1.0, 1)
    assert st["K"] == 5
    v = st["seed_pix"] >= 0
    assert (np.sort(st["knn_idx"][v], 1) == np.nonzero(v)[0][None, :]).all()


# ------------------------------------------------------------------ fit --

@pytest.mark.parametrize("wpow", [1, 2])
def test_fit_vs_numpy(ref, wpow):
    rng = np.random.default_rng(11)
    N, K = 30, 10
    m = np.zeros((N, 4), np.float32)
    m[:, :2] = rng.uniform(0, 50, (N, 2))
    m[:, 2:] = m[:, :2] + rng.normal(0, 4, (N, 2))
    sp = np.arange(N, dtype=np.int32)
    ki = np.stack([np.concatenate([[s], rng.choice(np.delete(np.arange(N), s), K - 1, replace=False)])
                   for s in range(N)]).astype(np.int32)
    kd = np.sort(rng.uniform(0, 3, (N, K)), 1)
    kd[:, 0] = 0
    a = 0.7
    P, stt = ref.fit(m, sp, ki, kd, a, 1, wpow)
    Pn, sn = ref.fit(m, sp, ki, kd, a, 0, wpow)
    assert (stt == 0).all() and (sn == 1).all()
    pos = m[:, :2].astype(np.float64)
    disp = (m[:, 2:].astype(np.float64) - pos)
    for s in range(N):
        k = np.exp(-a * kd[s])
        nw = indep.nw_fit(disp[ki[s]], k)
        np.testing.assert_allclose(Pn[s, 4:], nw, rtol=1e-12, atol=1e-12)
        # LA: Eq. (2) scales each equation by k (power 2 in the normal
        # equations); power 1 scales by sqrt(k)
        row_scale = k if wpow == 2 else np.sqrt(k)
        A, t = indep.la_fit_absolute(pos[ki[s]], m[ki[s], 2:].astype(np.float64), row_scale)
        B = A - np.eye(2)
        c = A @ pos[s] + t - pos[s]
        np.testing.assert_allclose(P[s, [0, 1, 2, 3]], B.ravel(), rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(P[s, 4:], c, rtol=1e-9, atol=1e-9)


def test_fit_collinear_falls_back_to_nw(ref):
    N = 6
    m = np.zeros((N, 4), np.float32)
    m[:, 0] = np.arange(N) * 3.0
    m[:, 1] = 5.0                                   # all on one row
    m[:, 2] = m[:, 0] + np.arange(N)
    m[:, 3] = m[:, 1] - 1
    sp = np.arange(N, dtype=np.int32)
    ki = np.tile(np.arange(N, dtype=np.int32), (N, 1))
    kd = np.abs(np.arange(N)[None, :] - np.arange(N)[:, None]).astype(np.float64)
    ki = np.argsort(kd, 1, kind="stable").astype(np.int32)
    kd = np.take_along_axis(kd, ki, 1)
    P, st = ref.fit(m, sp, ki, kd, 1.0, 1)
    assert (st == 2).all()
    Pn, _ = ref.fit(m, sp, ki, kd, 1.0, 0)
    np.testing.assert_array_equal(P, Pn)
    # two neighbours (K < 3) are degenerate as well
    P2, st2 = ref.fit(m, sp, ki[:, :2], kd[:, :2], 1.0, 1)
    assert (st2 == 2).all()


def _ratio(pos, w):
    """Smallest over largest eigenvalue of the weighted covariance of the
    positions, from numpy's symmetric eigensolver."""
    c = pos - (w[:, None] * pos).sum(0) / w.sum()
    ev = np.linalg.eigvalsh((w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0) / w.sum())
    return ev[0] / ev[1]


def _line_plus_one(spacing, delta, n=10):
    """n matches on a horizontal line and one just off it (float32 positions);
    displacements follow one affine motion exactly."""
    m = np.zeros((n + 1, 4), np.float32)
    m[:n, 0] = np.arange(n) * spacing
    m[n, 0] = (n // 2 - 0.5) * spacing
    m[n, 1] = delta
    B = np.array([[0.02, -0.01], [0.015, 0.03]])
    c = np.array([1.5, -2.0])
    p = m[:, :2].astype(np.float64)
    m[:, 2:] = p + p @ B.T + c
    return m


def _fit_all_neighbours(ref, m, d_of, a, wpow):
    """Every match's neighbourhood is all matches, at distances d_of(n)."""
    N = len(m)
    sp = np.arange(N, dtype=np.int32)
    ki = np.tile(np.arange(N, dtype=np.int32), (N, 1))
    kd = np.tile(np.array([d_of(j) for j in range(N)], np.float64), (N, 1))
    return ref.fit(m, sp, ki, kd, a, 1, wpow)


@pytest.mark.parametrize("spacing", [0.01, 1.0, 100.0])
def test_fit_degeneracy_boundary_is_relative(ref, spacing):
    """The near-collinear test compares the covariance eigenvalues with each
    other (ratio 1e-9), not with an absolute threshold: at every position
    scale, a ratio of 1e-8 stays LA and a ratio of 1e-10 falls back to NW.
    Ratios come from numpy's eigensolver on the float32 positions."""
    for target, want in ((1e-8, 0), (1e-10, 2)):
        # ratio ~ delta^2 / (11 spacing^2 * 8.25 * 11/10): solve for delta
        delta = spacing * math.sqrt(target * 8.25 * 11.0) * 1.1
        for _ in range(60):
            m = _line_plus_one(spacing, delta)
            r = _ratio(m[:, :2].astype(np.float64), np.ones(len(m)))
            if abs(math.log10(r / target)) < 0.05:
                break
            delta *= math.sqrt(target / r)
        assert abs(math.log10(r / target)) < 0.05, (r, target)
        P, st = _fit_all_neighbours(ref, m, lambda j: 0.0, 0.0, 2)
        assert (st == want).all(), (spacing, target, r, st)
        if want == 0:
            # the (ill-conditioned) LA system still matches numpy's solver
            pos = m[:, :2].astype(np.float64)
            A, t = indep.la_fit_absolute(pos, m[:, 2:].astype(np.float64), np.ones(len(m)))
            np.testing.assert_allclose(P[0, :4], (A - np.eye(2)).ravel(), rtol=1e-5, atol=1e-9)


def test_fit_degeneracy_uses_the_fit_weights(ref):
    """The covariance is weighted like the fit: k^2 for the literal Eq. (2)
    (power 2), k for power 1.  One neighbourhood whose off-line match has a
    small weight sits below the threshold with k^2 weights and above it
    with k weights (and unweighted)."""
    spacing, a, d_off = 1.0, 1.0, 4.0
    d_of = lambda j: d_off if j == 10 else 0.1 * j
    k = lambda m: np.exp(-a * np.array([d_of(j) for j in range(len(m))]))
    delta = 1e-4
    for _ in range(60):
        m = _line_plus_one(spacing, delta)
        r2 = _ratio(m[:, :2].astype(np.float64), k(m) ** 2)
        if abs(math.log10(r2 / 2e-10)) < 0.05:
            break
        delta *= math.sqrt(2e-10 / r2)
    pos = m[:, :2].astype(np.float64)
    r1 = _ratio(pos, k(m))
    r0 = _ratio(pos, np.ones(len(m)))
    assert r2 < 0.3e-9 and r1 > 3e-9 and r0 > 3e-9, (r2, r1, r0)
    _, st2 = _fit_all_neighbours(ref, m, d_of, a, 2)
    _, st1 = _fit_all_neighbours(ref, m, d_of, a, 1)
    assert (st2 == 2).all() and (st1 == 0).all(), (st2, st1)


# ------------------------------------------------- whole interpolation --

def _flow(ref, sc, K=None, a=None, mode=None, **kw):
    f, rc, stats = ref.interp(sc.cost, sc.matches, sc.K if K is None else K,
                              sc.a if a is None else a,
                              sc.mode if mode is None else mode, **kw)
    assert rc == 0
    return f


def test_per_pixel_literal_eq4_equals_per_match(ref):
    """Algorithm 1 shortcut: fitting at every pixel with the approximated
    distance of Eq. (4) -- D(p, L(p)) + graph distance -- and its own K
    nearest matches gives the per-match model propagated to the cell
    (Sec. 3.4).  LA is fitted literally as p' = A p + t (Eq. 2); NW on
    displacements."""
    sc = random_case(16, 19, 14, seed=21)
    K, a = 5, 0.9
    st = ref.stages(sc.cost, sc.matches, K, a, 1)
    stn = ref.stages(sc.cost, sc.matches, K, a, 0)
    N = sc.N
    valid = st["seed_pix"] >= 0
    Dg = indep.graph_dist_matrix(N, st["em"], st["en"], st["ew"])
    pos = sc.matches[:, :2].astype(np.float64)
    tgt = sc.matches[:, 2:].astype(np.float64)
    H, W = sc.cost.shape
    for y in range(H):
        for x in range(W):
            lp = st["L"][y, x]
            dt = st["D"][y, x] + Dg[lp]
            dt[~valid] = np.inf
            order = np.lexsort((np.arange(N), dt))[:K]
            k = np.exp(-a * dt[order])
            A, t = indep.la_fit_absolute(pos[order], tgt[order], k)
            want = A @ np.array([x, y]) + t - np.array([x, y])
            np.testing.assert_allclose(st["flow"][y, x], want, rtol=1e-7, atol=1e-7)
            nw = indep.nw_fit(tgt[order] - pos[order], k)
            np.testing.assert_allclose(stn["flow"][y, x], nw, rtol=1e-9, atol=1e-9)


def _exact_affine_matches(rng, H, W, N, A, t):
    pix = rng.choice(H * W, N, replace=False)
    m = np.zeros((N, 4), np.float32)
    m[:, 0] = pix % W
    m[:, 1] = pix // W
    pt = m[:, :2].astype(np.float64) @ A.T + t
    m[:, 2:] = pt
    assert (m[:, 2:].astype(np.float64) == pt).all()   # exactly representable
    return m


@pytest.mark.parametrize("a", [0.0, 0.5, 3.0])
def test_global_affine_is_recovered_exactly(ref, a):
    rng = np.random.default_rng(5)
    H, W = 31, 37
    A = np.array([[1.0625, -0.03125], [0.046875, 0.9375]])
    t = np.array([2.25, -3.5])
    sc = random_case(H, W, 40, seed=8)
    m = _exact_affine_matches(rng, H, W, 40, A, t)
    f = ref.interp(sc.cost, m, 6, a, 1)[0]
    ys, xs = np.mgrid[0:H, 0:W]
    want_u = (A[0, 0] - 1) * xs + A[0, 1] * ys + t[0]
    want_v = A[1, 0] * xs + (A[1, 1] - 1) * ys + t[1]
    np.testing.assert_allclose(f[..., 0], want_u, atol=1e-9)
    np.testing.assert_allclose(f[..., 1], want_v, atol=1e-9)


def test_constant_translation_exact(ref):
    sc = random_case(25, 30, 20, seed=9)
    m = sc.matches.copy()
    m[:, :2] = np.round(m[:, :2] * 16) / 16        # so that x + t is exact
    m[:, 2] = m[:, 0] + np.float32(3.25)
    m[:, 3] = m[:, 1] - np.float32(1.5)
    for mode in (0, 1):
        for K in (1, 4, 20):
            f = ref.interp(sc.cost, m, K, 1.3, mode)[0]
            np.testing.assert_allclose(f[..., 0], 3.25, atol=1e-9)
            np.testing.assert_allclose(f[..., 1], -1.5, atol=1e-9)


def test_k_equals_n_a_zero_is_global_fit(ref):
    sc = random_case(22, 26, 15, seed=10, subpixel=True)
    N = sc.N
    pos = sc.matches[:, :2].astype(np.float64)
    tgt = sc.matches[:, 2:].astype(np.float64)
    f = _flow(ref, sc, K=N, a=0.0, mode=1)
    A, t = indep.la_fit_absolute(pos, tgt, np.ones(N))
    H, W = sc.cost.shape
    ys, xs = np.mgrid[0:H, 0:W]
    P = np.stack([xs, ys], -1).astype(np.float64)
    want = P @ A.T + t - P
    np.testing.assert_allclose(f, want, atol=1e-8)
    fn = _flow(ref, sc, K=N, a=0.0, mode=0)
    np.testing.assert_allclose(fn, np.broadcast_to((tgt - pos).mean(0), fn.shape), atol=1e-10)


def test_k1_copies_the_cell_match(ref):
    sc = random_case(20, 24, 18, seed=12)
    st = ref.stages(sc.cost, sc.matches, 1, 1.0, 1)
    disp = (sc.matches[:, 2:].astype(np.float64) - sc.matches[:, :2])
    np.testing.assert_allclose(st["flow"], disp[st["L"]], atol=1e-12)


def test_linear_in_displacements(ref):
    sc = random_case(24, 28, 25, seed=13)
    rng = np.random.default_rng(0)
    u1 = rng.integers(-40, 40, (sc.N, 2)) / 8.0
    u2 = rng.integers(-40, 40, (sc.N, 2)) / 8.0

    def run(u, mode):
        m = sc.matches.copy()
        m[:, :2] = np.round(m[:, :2])
        m[:, 2:] = m[:, :2] + u
        return ref.interp(sc.cost, m, 7, 0.8, mode)[0]
    for mode in (0, 1):
        np.testing.assert_allclose(run(u1 + 2 * u2, mode), run(u1, mode) + 2 * run(u2, mode),
                                   atol=1e-9)


def test_cost_and_a_equivariance(ref):
    sc = random_case(24, 28, 25, seed=14)
    f1 = _flow(ref, sc, K=8, a=1.0)
    sc2 = random_case(24, 28, 25, seed=14)
    sc2.cost = sc2.cost * np.float32(8.0)
    f2 = _flow(ref, sc2, K=8, a=1.0 / 8.0)
    np.testing.assert_array_equal(f1, f2)


def test_no_match_in_image(ref):
    cost = np.ones((5, 6), np.float32)
    m = np.array([[-5, 1, 0, 0], [9, 1, 0, 0]], np.float32)
    f, rc, stats = ref.interp(cost, m, 3, 1.0, 1)
    assert rc == -3 and np.isnan(f).all() and stats["outside"] == 2


# --------------------------------------------------------- properties --

@settings(max_examples=25, deadline=None)
@given(st.integers(2, 9), st.integers(2, 9), st.integers(1, 6),
       st.integers(0, 2**31 - 1), st.sampled_from([4, 8]))
def test_property_voronoi_bruteforce(H, W, N, seed, conn):
    from oracle import epic_ref as ref
    rng = np.random.default_rng(seed)
    N = min(N, H * W)
    cost = rng.uniform(0.05, 2.0, (H, W)).astype(np.float32)
    pix = rng.choice(H * W, N, replace=False)
    m = np.zeros((N, 4), np.float32)
    m[:, 0], m[:, 1] = pix % W, pix // W
    sp, _, _ = ref.seeds(H, W, m)
    D, L = ref.voronoi(cost, sp, conn)
    FW = indep.floyd_all_pairs(cost, conn)[sp]
    np.testing.assert_allclose(D.ravel(), FW.min(0), rtol=1e-12)
    assert (FW[L.ravel(), np.arange(H * W)] <= FW.min(0) * (1 + 1e-12)).all()


@settings(max_examples=20, deadline=None)
@given(st.integers(0, 2**31 - 1), st.integers(1, 8))
def test_property_knn_bruteforce(seed, K):
    from oracle import epic_ref as ref
    sc = random_case(12, 15, 10, seed=seed)
    s = ref.stages(sc.cost, sc.matches, K, 1.0, 1)
    Dg = indep.graph_dist_matrix(sc.N, s["em"], s["en"], s["ew"])
    valid = s["seed_pix"] >= 0
    for src in np.nonzero(valid)[0]:
        idx, d = indep.knn_from_matrix(Dg, src, s["K"], valid)
        np.testing.assert_allclose(s["knn_d"][src], d, rtol=1e-12)
        # members may differ only where brute force and the oracle order
        # distances equal to rounding differently; every such member lies
        # at the K-th distance
        only = set(s["knn_idx"][src].tolist()) ^ set(idx.tolist())
        dist = dict(zip(idx.tolist(), d.tolist()))
        dist.update(zip(s["knn_idx"][src].tolist(), s["knn_d"][src].tolist()))
        assert all(math.isclose(dist[n], d[-1], rel_tol=1e-12) for n in only), (src, only)


# ------------------------------------------------------- match pruning --

def _grid_translation(outlier_at=None, outlier_u=(30.0, 30.0)):
    """11 x 11 matches 5 px apart on a 60 x 60 image of constant cost 0.01,
    all moving by (3, -2) except one planted outlier."""
    g = 5 + 5 * np.arange(11)
    ys, xs = np.meshgrid(g, g, indexing="ij")
    m = np.zeros((121, 4), np.float32)
    m[:, 0], m[:, 1] = xs.ravel(), ys.ravel()
    u = np.tile([3.0, -2.0], (121, 1))
    if outlier_at is not None:
        u[outlier_at] = outlier_u
    m[:, 2:] = m[:, :2] + u
    return np.full((60, 60), 0.01, np.float32), m


def test_prune_drops_a_planted_outlier(ref):
    """Sec. 5.1: with graph distances of ~0.05 per grid step (weights near
    1), the outlier's NW estimate is dominated by its 31 consistent
    neighbours (about (4, -0.9), 40 px from its own displacement), while
    each neighbour's estimate moves by at most ~1/27 of the outlier's
    deviation (< 2 px): exactly the outlier goes."""
    cost, m = _grid_translation(outlier_at=60)
    kept = ref.prune(cost, m, 32, 1.0, 5.0)
    assert kept.tolist() == [i for i in range(121) if i != 60]
    # with no outlier nothing goes, even at a threshold of 1e-9 px: the NW
    # estimate of a constant field is that constant, to rounding
    cost, m = _grid_translation()
    assert ref.prune(cost, m, 32, 1.0, 5.0).tolist() == list(range(121))
    assert len(ref.prune(cost, m, 32, 1.0, 1e-9)) == 121


def test_prune_compares_with_the_nw_field_at_the_match_pixel(ref):
    """The decision is |u_m - F_NW(pixel of m)| <= threshold, F_NW being the
    dense NW interpolation; matches outside the image or on a pixel held
    by a lower index are never kept."""
    sc = random_case(70, 90, 140, seed=9, K=20, outside=4, duplicates=5)
    f, rc, _ = ref.interp(sc.cost, sc.matches, 20, sc.a, 0)
    sp, _, _ = ref.seeds(sc.H, sc.W, sc.matches)
    for thr in (0.5, 2.0, 5.0):
        kept = ref.prune(sc.cost, sc.matches, 20, sc.a, thr)
        want = []
        for i in np.nonzero(sp >= 0)[0]:
            y, x = divmod(int(sp[i]), sc.W)
            u = sc.matches[i, 2:].astype(np.float64) - sc.matches[i, :2]
            if np.linalg.norm(u - f[y, x]) <= thr:
                want.append(int(i))
        assert kept.tolist() == want


# --------------------------------------------- cost from image gradient --

def test_grad_cost_closed_forms(ref):
    """A linear ramp I = alpha x + beta y in every channel has gradient
    (alpha, beta) inside the image (exact for central differences) and half
    of the normal component on a border (one-sided over the repeated border
    pixel); a flat image costs eps; a unit step costs 1/2 on both sides of
    the edge and nothing elsewhere."""
    H, W, ch = 7, 9, 3
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    al, be = 0.25, -0.125
    ramp = np.repeat((al * xs + be * ys)[:, :, None], ch, 2).astype(np.float32)
    C = ref.grad_norm_cost(ramp, eps=0.0)
    np.testing.assert_allclose(C[1:-1, 1:-1], math.sqrt(ch * (al ** 2 + be ** 2)), rtol=1e-12)
    np.testing.assert_allclose(C[1:-1, 0], math.sqrt(ch * ((al / 2) ** 2 + be ** 2)), rtol=1e-12)
    np.testing.assert_allclose(C[0, 1:-1], math.sqrt(ch * (al ** 2 + (be / 2) ** 2)), rtol=1e-12)
    np.testing.assert_allclose(C[0, 0], math.sqrt(ch * ((al / 2) ** 2 + (be / 2) ** 2)), rtol=1e-12)
    np.testing.assert_array_equal(ref.grad_norm_cost(np.full((5, 6), 0.7, np.float32)), 1e-3)
    step = np.zeros((4, 10), np.float32)
    step[:, 5:] = 1.0
    C = ref.grad_norm_cost(step, eps=0.0)
    want = np.zeros((4, 10))
    want[:, 4:6] = 0.5
    np.testing.assert_array_equal(C, want)


def test_grad_cost_scales_and_matches_numpy_gradient(ref):
    """Scaling the image scales the cost above eps; the interior equals the
    norm of numpy.gradient (second-order central differences)."""
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (12, 15, 3)).astype(np.float32)
    C = ref.grad_norm_cost(img, eps=0.0)
    np.testing.assert_allclose(ref.grad_norm_cost(img * np.float32(4), eps=0.0), 4 * C, rtol=1e-12)
    gy, gx = np.gradient(img.astype(np.float64), axis=(0, 1))
    want = np.sqrt((gx ** 2 + gy ** 2).sum(2))
    np.testing.assert_allclose(C[1:-1, 1:-1], want[1:-1, 1:-1], rtol=1e-12)


# ------------------------------------- exact per-pixel interpolation --

@pytest.mark.parametrize("mode,wpow", [(1, 2), (1, 1), (0, 2)])
def test_exact_matches_brute_force(ref, mode, wpow):
    """Table 2's exact variant from scratch: scipy distances from every
    match, each pixel's K nearest by (distance, index), and numpy's
    weighted mean or least squares at the pixel (Eq. 1, Eq. 2 with rows
    scaled by k for power 2 and sqrt(k) for power 1)."""
    cost, m = _rand_problem(21, H=13, W=16, N=10)
    K, a = 5, 0.8
    f, ki, kd, rc = ref.exact(cost, m, K, a, mode, wpow=wpow)
    assert rc == 0
    sp = indep.seed_pixels(*cost.shape, m)
    Dall, ids = indep.all_source_distances(cost, sp)
    H, W = cost.shape
    pos = m[:, :2].astype(np.float64)
    disp = m[:, 2:].astype(np.float64) - pos
    for p in range(H * W):
        d = Dall[:, p]
        order = np.lexsort((ids, d))[:K]
        nb, dn = ids[order], d[order]
        np.testing.assert_array_equal(ki[p], nb)
        np.testing.assert_allclose(kd[p], dn, rtol=1e-12)
        k = np.exp(-a * dn)
        if mode == 0:
            want = indep.nw_fit(disp[nb], k)
        else:
            A, t = indep.la_fit_absolute(pos[nb] - [p % W, p // W], disp[nb], k if wpow == 2 else np.sqrt(k))
            want = t
        np.testing.assert_allclose(f[p], want, rtol=1e-9, atol=1e-9)


def test_exact_k1_equals_the_approximation(ref):
    """With K = 1 the nearest match is the geodesic Voronoi label, so the
    exact and the approximated interpolation agree at every pixel (to the
    rounding of k u / k: the one weight is exp(-a D) here and 1 there)."""
    sc = random_case(30, 41, 25, seed=23, K=1)
    for mode in (0, 1):
        fe, ki, _, _ = ref.exact(sc.cost, sc.matches, 1, 1.0, mode)
        st = ref.stages(sc.cost, sc.matches, 1, 1.0, mode)
        np.testing.assert_array_equal(ki[:, 0], st["L"].ravel())
        fa = st["flow"].reshape(-1, 2)
        np.testing.assert_allclose(fe, fa, rtol=1e-15, atol=1e-14)


def test_exact_closed_forms(ref):
    """A single global affine motion is recovered at every pixel (LA, any
    cost map); a constant translation by NW and LA; K = N with a = 0 gives
    the global least-squares affine map and the global mean."""
    rng = np.random.default_rng(24)
    H, W, N = 20, 26, 30
    cost = rng.uniform(0.01, 2.0, (H, W)).astype(np.float32)
    A = np.array([[1.0625, -0.03125], [0.046875, 0.9375]])
    t = np.array([2.25, -3.5])
    m = _exact_affine_matches(rng, H, W, N, A, t)
    ys, xs = np.mgrid[0:H, 0:W]
    f = ref.exact(cost, m, 6, 1.0, 1)[0]
    np.testing.assert_allclose(f[:, 0], ((A[0, 0] - 1) * xs + A[0, 1] * ys + t[0]).ravel(), atol=1e-9)
    np.testing.assert_allclose(f[:, 1], (A[1, 0] * xs + (A[1, 1] - 1) * ys + t[1]).ravel(), atol=1e-9)
    m2 = m.copy()
    m2[:, 2:] = m2[:, :2] + np.array([3.25, -1.5], np.float32)
    for mode in (0, 1):
        f = ref.exact(cost, m2, 7, 0.5, mode)[0]
        np.testing.assert_allclose(f, np.tile([3.25, -1.5], (H * W, 1)), atol=1e-9)
    rnd = m.copy()
    rnd[:, 2:] = rnd[:, :2] + rng.normal(0, 2, (N, 2)).astype(np.float32)
    pos = rnd[:, :2].astype(np.float64)
    disp = rnd[:, 2:].astype(np.float64) - pos
    fn = ref.exact(cost, rnd, N, 0.0, 0)[0]
    np.testing.assert_allclose(fn, np.tile(disp.mean(0), (H * W, 1)), atol=1e-9)
    fl = ref.exact(cost, rnd, N, 0.0, 1)[0]
    Ag, tg = indep.la_fit_absolute(pos, rnd[:, 2:].astype(np.float64), np.ones(N))
    g = np.stack([xs.ravel(), ys.ravel()], 1) @ Ag.T + tg - np.stack([xs.ravel(), ys.ravel()], 1)
    np.testing.assert_allclose(fl, g, atol=1e-8)
