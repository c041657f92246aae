"""ctypes wrapper around the FP64 CPU oracle (``oracle/epic_ref.c``).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library.
Only tests, the smoke check and the benchmark's CPU-baseline leg use it.

Every function takes and returns numpy arrays; all floating point results
are float64.  Citations refer to the EpicFlow paper (Revaud et al. 2015).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epic_ref.c")
_LIB = os.path.join(_HERE, "libepic_ref.so")

# Near-collinear test for the LA fit: the weighted covariance of the
# neighbour positions has eigenvalues l1 >= l2; LA falls back to NW when
# l2 <= DEG_TAU * l1.  Eq. (2) is under-determined for collinear neighbours.
DEG_TAU = 1e-9

NW, LA = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.epic_ref_seeds.argtypes = [i32, i32, P, i32, P, P, P]
        L.epic_ref_seeds.restype = i32
        L.epic_ref_voronoi.argtypes = [P, i32, i32, P, i32, i32, P, P]
        L.epic_ref_voronoi.restype = None
        L.epic_ref_geodesic_from.argtypes = [P, i32, i32, i32, i32, P]
        L.epic_ref_geodesic_from.restype = None
        L.epic_ref_graph.argtypes = [P, i32, i32, P, P, i32, P, P, P, i64]
        L.epic_ref_graph.restype = i64
        L.epic_ref_knn.argtypes = [i32, P, i64, P, P, P, i32, P, P]
        L.epic_ref_knn.restype = None
        L.epic_ref_fit.argtypes = [P, i32, P, P, P, i32, f64, i32, i32, f64,
                                   P, P]
        L.epic_ref_fit.restype = None
        L.epic_ref_assign.argtypes = [i32, i32, P, P, P, P]
        L.epic_ref_assign.restype = None
        L.epic_ref_interp.argtypes = [P, i32, i32, P, i32, i32, f64, i32, i32,
                                      i32, f64, P, P]
        L.epic_ref_interp.restype = i32
        L.epic_ref_prune.argtypes = [P, i32, i32, P, i32, i32, f64, i32, f64, P]
        L.epic_ref_prune.restype = i32
        L.epic_ref_grad_cost.argtypes = [P, i32, i32, i32, f64, P]
        L.epic_ref_grad_cost.restype = None
        L.epic_ref_exact.argtypes = [P, i32, i32, P, i32, i32, f64, i32, i32, i32, f64, P, i64,
                                     P, P, P]
        L.epic_ref_exact.restype = i32
        L.epic_ref_set_threads.argtypes = [i32]
        L.epic_ref_set_threads.restype = None
        L.epic_ref_max_threads.argtypes = []
        L.epic_ref_max_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().epic_ref_set_threads(int(n))


def max_threads() -> int:
    return int(lib().epic_ref_max_threads())


def seeds(H, W, matches):
    """Match -> seed pixel index (y*W + x), -1 when outside the image or when
    a lower-indexed match already holds the pixel (matches are pixels,
    Sec. 3.1).  Returns (seed_pix, n_outside, n_duplicate)."""
    m = _f32(matches).reshape(-1, 4)
    N = m.shape[0]
    out = np.empty(max(N, 1), np.int32)
    no, nd = ctypes.c_int(0), ctypes.c_int(0)
    lib().epic_ref_seeds(H, W, _p(m), N, _p(out), ctypes.byref(no),
                         ctypes.byref(nd))
    return out[:N], no.value, nd.value


def voronoi(cost, seed_pix, conn=8):
    """Geodesic distance to the nearest match, Eq. (3), and the geodesic
    Voronoi label L(p) (Sec. 3.4), lowest match index on ties."""
    c = _f32(cost)
    H, W = c.shape
    s = _i32(seed_pix)
    D = np.empty((H, W), np.float64)
    L = np.empty((H, W), np.int32)
    lib().epic_ref_voronoi(_p(c), H, W, _p(s), s.shape[0], conn, _p(D), _p(L))
    return D, L


def geodesic_from(cost, src_pix, conn=8):
    """Single-source geodesic distance from one pixel to every pixel."""
    c = _f32(cost)
    H, W = c.shape
    D = np.empty((H, W), np.float64)
    lib().epic_ref_geodesic_from(_p(c), H, W, int(src_pix), conn, _p(D))
    return D


def graph(cost, D, L, conn=8):
    """Match graph: edges (m < n) between adjacent Voronoi cells, weight =
    geodesic distance restricted to the two cells (Sec. 3.4)."""
    c = _f32(cost)
    H, W = c.shape
    D = _f64(D)
    L = _i32(L)
    cap = 4 * H * W + 1
    em = np.empty(cap, np.int32)
    en = np.empty(cap, np.int32)
    ew = np.empty(cap, np.float64)
    E = lib().epic_ref_graph(_p(c), H, W, _p(D), _p(L), conn, _p(em), _p(en),
                             _p(ew), cap)
    assert E >= 0
    return em[:E].copy(), en[:E].copy(), ew[:E].copy()


def knn(N, seed_pix, em, en, ew, K):
    """K nearest matches of each match by Dijkstra on the graph (Algorithm 1),
    ordered by (distance, index).  Rows of dropped matches are -1."""
    s = _i32(seed_pix)
    em, en, ew = _i32(em), _i32(en), _f64(ew)
    idx = np.empty((max(N, 1), K), np.int32)
    d = np.empty((max(N, 1), K), np.float64)
    lib().epic_ref_knn(N, _p(s), em.shape[0], _p(em), _p(en), _p(ew), K,
                       _p(idx), _p(d))
    return idx[:N], d[:N]


def fit(matches, seed_pix, knn_idx, knn_d, a, mode, wpow=2, deg_tau=DEG_TAU):
    """One NW (Eq. 1) or LA (Eq. 2) model per match.  Returns params (N, 6):
    b00 b01 b10 b11 c0 c1 of u = B (p - p_m) + c, and status (N,): 0 LA,
    1 NW, 2 LA degenerate -> NW, -1 unused."""
    m = _f32(matches).reshape(-1, 4)
    N = m.shape[0]
    ki = _i32(knn_idx)
    kd = _f64(knn_d)
    K = ki.shape[1]
    P = np.empty((max(N, 1), 6), np.float64)
    st = np.empty(max(N, 1), np.int32)
    lib().epic_ref_fit(_p(m), N, _p(_i32(seed_pix)), _p(ki), _p(kd), K,
                       float(a), int(mode), int(wpow), float(deg_tau), _p(P),
                       _p(st))
    return P[:N], st[:N]


def assign(H, W, L, matches, params):
    """Dense field: every pixel takes its cell's model (Algorithm 1)."""
    flow = np.empty((H, W, 2), np.float64)
    lib().epic_ref_assign(H, W, _p(_i32(L)), _p(_f32(matches)),
                          _p(_f64(params)), _p(flow))
    return flow


def interp(cost, matches, K, a, mode, conn=8, wpow=2, deg_tau=DEG_TAU):
    """Whole interpolation in one C call.  Returns (flow (H, W, 2) float64,
    status, stats dict)."""
    c = _f32(cost)
    H, W = c.shape
    m = _f32(matches).reshape(-1, 4)
    flow = np.empty((H, W, 2), np.float64)
    st = np.zeros(6, np.int64)
    rc = lib().epic_ref_interp(_p(c), H, W, _p(m), m.shape[0], int(K),
                               float(a), int(mode), conn, wpow, float(deg_tau),
                               _p(flow), _p(st))
    keys = ["used", "outside", "duplicate", "degenerate", "edges", "K"]
    return flow, rc, dict(zip(keys, st.tolist()))


def stages(cost, matches, K, a, mode, conn=8, wpow=2, deg_tau=DEG_TAU):
    """Every intermediate of the pipeline, stage by stage."""
    c = _f32(cost)
    H, W = c.shape
    m = _f32(matches).reshape(-1, 4)
    N = m.shape[0]
    sp, no, nd = seeds(H, W, m)
    used = int((sp >= 0).sum())
    out = dict(seed_pix=sp, n_outside=no, n_duplicate=nd, used=used)
    if used == 0:
        return out
    D, L = voronoi(c, sp, conn)
    em, en, ew = graph(c, D, L, conn)
    Kc = min(K, used)
    ki, kd = knn(N, sp, em, en, ew, Kc)
    P, st = fit(m, sp, ki, kd, a, mode, wpow, deg_tau)
    flow = assign(H, W, L, m, P)
    out.update(D=D, L=L, em=em, en=en, ew=ew, K=Kc, knn_idx=ki, knn_d=kd,
               params=P, status=st, flow=flow)
    return out


def prune(cost, matches, K, a, prune_px, conn=8):
    """Consistency check of the matches (Sec. 5.1, "Pruning of matches"):
    one NW interpolation, then the matches whose displacement differs from
    that estimate at their own pixel by more than prune_px are removed.
    Returns the original indices of the kept matches (increasing)."""
    c = _f32(cost)
    H, W = c.shape
    m = _f32(matches).reshape(-1, 4)
    kept = np.empty(max(m.shape[0], 1), np.int32)
    n = lib().epic_ref_prune(_p(c), H, W, _p(m), m.shape[0], int(K), float(a),
                             conn, float(prune_px), _p(kept))
    return kept[:n].copy()


def interp_pruned(cost, matches, K, a, mode, prune_px, conn=8, wpow=2, deg_tau=DEG_TAU):
    """The interpolation of the matches that pass the consistency check
    (Sec. 5.1).  Returns (flow, status, stats, kept indices)."""
    kept = prune(cost, matches, K, a, prune_px, conn)
    m = _f32(matches).reshape(-1, 4)[kept]
    if len(kept) == 0:
        H, W = np.shape(cost)
        return np.full((H, W, 2), np.nan), -3, {}, kept
    flow, rc, st = interp(cost, m, K, a, mode, conn, wpow, deg_tau)
    return flow, rc, st, kept


# --------------------------------------------------------------------------
# cost map from the image gradient (Table 2, contour row "norm of the image
# gradient"; the same gradient norm sets the smoothness weight of Sec. 4)
# --------------------------------------------------------------------------
GRAD_EPS = 1e-3


def grad_norm_cost(image, eps=GRAD_EPS):
    """C(p) = ||grad I(p)||_2 + eps in float64.  image: (H, W) or (H, W, ch).
    The gradient is taken by central differences, (I(x+1) - I(x-1)) / 2 and
    (I(y+1) - I(y-1)) / 2, with the border pixel repeated outside the image;
    the norm runs over both directions and all channels.  eps keeps the
    cost positive where the image is flat."""
    I = _f32(image)
    if I.ndim == 2:
        I = I[:, :, None]
    I = np.ascontiguousarray(I)
    H, W, ch = I.shape
    out = np.empty((H, W), np.float64)
    lib().epic_ref_grad_cost(_p(I), H, W, ch, float(eps), _p(out))
    return out


def exact(cost, matches, K, a, mode, pixels=None, conn=8, wpow=2, deg_tau=DEG_TAU):
    """The exact per-pixel geodesic interpolation (Table 2, "Geodesic
    (exact)"): every pixel's own K nearest matches under the geodesic
    distance of Eq. (3) (one Dijkstra from the pixel), its own NW or LA fit
    evaluated at the pixel.  pixels: flat indices y*W + x (default: all).
    Returns (flow (npix, 2), knn_idx (npix, K), knn_d (npix, K), status)."""
    c = _f32(cost)
    H, W = c.shape
    m = _f32(matches).reshape(-1, 4)
    pix = np.arange(H * W, dtype=np.int64) if pixels is None else np.ascontiguousarray(pixels, np.int64)
    n = len(pix)
    flow = np.empty((max(n, 1), 2), np.float64)
    ki = np.empty((max(n, 1), K), np.int32)
    kd = np.empty((max(n, 1), K), np.float64)
    rc = lib().epic_ref_exact(_p(c), H, W, _p(m), m.shape[0], int(K), float(a), int(mode), conn, wpow,
                              float(deg_tau), _p(pix), n, _p(flow), _p(ki), _p(kd))
    return flow[:n], ki[:n], kd[:n], rc
