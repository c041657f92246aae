"""Seeded synthetic inputs for the sparse-to-dense interpolation.

This module only *draws inputs*: an edge cost map C (H x W, float32, C > 0)
and a sparse match set (N x 4 float32 rows ``x, y, x', y'``).  It contains
none of the interpolation arithmetic, so both the FP64 oracle and the GPU
library may consume what it produces.

The scenes stand in for the benchmarks the paper measures on (MPI-Sintel,
KITTI, Middlebury; Sec. 5.1): piecewise-affine motion layers bounded by
polygons, a cost map built from the layer boundaries (the paper uses an edge
detector's response, Sec. 3.3), and matches on a regular grid thinned the way
the paper's matchers are (occlusions, low-saliency pruning, outliers; Sec. 5.1
and Sec. 5.3).  No dataset content is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage

__all__ = [
    "Scene",
    "config_scene",
    "layered_scene",
    "road_scene",
    "random_case",
    "batch_scenes",
    "serve_stream",
    "serve_bases",
    "ServeBase",
    "CONFIG_PARAMS",
]


@dataclasses.dataclass
class Scene:
    """One interpolation problem: cost map, matches and parameters."""

    cost: np.ndarray          # (H, W) float32, > 0
    matches: np.ndarray       # (N, 4) float32: x, y, x', y'
    K: int
    a: float
    mode: int                 # 0 = NW, 1 = LA
    name: str = ""
    gt_flow: np.ndarray | None = None   # (H, W, 2) float32, generator's motion
    image: np.ndarray | None = None     # (H, W, 3) float32 in [0, 1] (on request)
    image2: np.ndarray | None = None    # (H, W, 3) the second frame (on request)

    @property
    def H(self) -> int:
        return int(self.cost.shape[0])

    @property
    def W(self) -> int:
        return int(self.cost.shape[1])

    @property
    def N(self) -> int:
        return int(self.matches.shape[0])


# --------------------------------------------------------------------------
# geometry helpers (input generation only)
# --------------------------------------------------------------------------

def _star_polygon(rng, H, W, nv_lo=5, nv_hi=8, r_lo=0.1, r_hi=0.3):
    nv = int(rng.integers(nv_lo, nv_hi + 1))
    cx = rng.uniform(0.15 * W, 0.85 * W)
    cy = rng.uniform(0.15 * H, 0.85 * H)
    ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, nv))
    rad = rng.uniform(r_lo, r_hi, nv) * min(H, W)
    return np.stack([cx + rad * np.cos(ang), cy + rad * np.sin(ang)], 1), (cx, cy)


def _fill_polygon(poly, H, W):
    """Even-odd point-in-polygon test at every pixel centre."""
    ys, xs = np.mgrid[0:H, 0:W]
    px = xs.astype(np.float64)
    py = ys.astype(np.float64)
    inside = np.zeros((H, W), bool)
    n = len(poly)
    for i in range(n):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % n]
        if y0 == y1:
            continue
        crosses = (y0 > py) != (y1 > py)
        xint = (x1 - x0) * (py - y0) / (y1 - y0) + x0
        inside ^= crosses & (px < xint)
    return inside


def _boundary(layer):
    b = np.zeros(layer.shape, bool)
    b[:, 1:] |= layer[:, 1:] != layer[:, :-1]
    b[:, :-1] |= layer[:, 1:] != layer[:, :-1]
    b[1:, :] |= layer[1:, :] != layer[:-1, :]
    b[:-1, :] |= layer[1:, :] != layer[:-1, :]
    return b


def _cost_from_layers(rng, layer, sigma=1.0, noise=0.05, floor=1e-3):
    b = _boundary(layer).astype(np.float64)
    c = ndimage.gaussian_filter(b, sigma=sigma, mode="reflect")
    c = c + rng.uniform(0.0, noise, layer.shape) + floor
    return c.astype(np.float32)


def _layer_texture(H, W, n, seed):
    """The per-layer colours and the shared texture fields of the scene's
    images: each layer a random base colour in [0.15, 0.85]^3, plus per
    channel a smooth texture (sigma-2 blurred normal noise, amplitude 0.08).
    Its own generator, so drawing it leaves the rest of the scene
    unchanged; returns the generator for the pixel noise."""
    rng = np.random.default_rng(seed + 7919)
    base = rng.uniform(0.15, 0.85, (n, 3))
    tex = [0.08 * ndimage.gaussian_filter(rng.standard_normal((H, W)), 2.0) for _ in range(3)]
    return base, tex, rng


def _layer_image(layer, seed):
    """An RGB image of the layer map (for the cost-from-gradient path): the
    layer's base colour plus the texture at the pixel and a little pixel
    noise (U[0, 0.01]), clipped to [0, 1]."""
    H, W = layer.shape
    base, tex, rng = _layer_texture(H, W, int(layer.max()) + 1, seed)
    img = base[layer]
    for c in range(3):
        img[:, :, c] += tex[c]
    img += rng.uniform(0.0, 0.01, img.shape)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def _second_image(masks, params, seed, H, W):
    """The second frame of a layered scene: every layer moved by its affine
    motion, painted in the same order as the first frame (later layers on
    top).  A pixel y of the second frame shows layer l when the point
    p = c + (I + B)^-1 (y - c - t) that moves onto it lies inside the
    layer's polygon (the background covers everything); it takes the layer's
    colour plus the texture sampled at p (bilinear, the texture carried
    along with the layer) and fresh pixel noise.  So I2(p + u(p)) matches
    I1(p) wherever p stays visible."""
    n = len(masks)
    base, tex, rng = _layer_texture(H, W, n, seed)
    rng.uniform(0.0, 0.01, (H, W, 3))          # the first frame's pixel noise
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    top = np.zeros((H, W), np.int64)
    src = np.zeros((2, H, W))
    for li, (B, t, ctr) in enumerate(params):
        M = np.linalg.inv(np.eye(2) + B)
        rx, ry = xs - ctr[0] - t[0], ys - ctr[1] - t[1]
        px = ctr[0] + M[0, 0] * rx + M[0, 1] * ry
        py = ctr[1] + M[1, 0] * rx + M[1, 1] * ry
        if li == 0:
            cover = np.ones((H, W), bool)
        else:
            ix, iy = np.rint(px).astype(np.int64), np.rint(py).astype(np.int64)
            inside = (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H)
            cover = np.zeros((H, W), bool)
            cover[inside] = masks[li][iy[inside], ix[inside]]
        top[cover] = li
        src[0][cover], src[1][cover] = py[cover], px[cover]
    img = base[top]
    for c in range(3):
        img[:, :, c] += ndimage.map_coordinates(tex[c], src, order=1, mode="nearest")
    img += rng.uniform(0.0, 0.01, img.shape)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def _motion(layer, params):
    H, W = layer.shape
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    flow = np.zeros((H, W, 2))
    for li, (B, t, ctr) in enumerate(params):
        m = layer == li
        dx = xs[m] - ctr[0]
        dy = ys[m] - ctr[1]
        flow[m, 0] = B[0, 0] * dx + B[0, 1] * dy + t[0]
        flow[m, 1] = B[1, 0] * dx + B[1, 1] * dy + t[1]
    return flow


def _grid(H, W, stride, offset=None):
    off = stride // 2 if offset is None else offset
    xs = np.arange(off, W, stride)
    ys = np.arange(off, H, stride)
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    return gx.ravel(), gy.ravel()


def _finish_matches(rng, gx, gy, flow, n_target, drop_frac, outlier_frac,
                    outlier_r, H, W, saliency_sigma=8.0):
    """Low-saliency pruning, subsampling, targets and outliers."""
    if drop_frac > 0 and len(gx) > 0:
        sal = ndimage.gaussian_filter(rng.standard_normal((H, W)), saliency_sigma)
        s = sal[gy, gx]
        keep = np.argsort(s, kind="stable")[int(round(drop_frac * len(gx))):]
        keep.sort()
        gx, gy = gx[keep], gy[keep]
    if n_target is not None and len(gx) > n_target:
        sel = np.sort(rng.choice(len(gx), n_target, replace=False))
        gx, gy = gx[sel], gy[sel]
    u = flow[gy, gx].copy()
    n = len(gx)
    n_out = int(round(outlier_frac * n))
    if n_out:
        idx = rng.choice(n, n_out, replace=False)
        u[idx] = rng.uniform(-outlier_r, outlier_r, (n_out, 2))
    m = np.empty((n, 4), np.float32)
    m[:, 0] = gx
    m[:, 1] = gy
    m[:, 2] = gx + u[:, 0]
    m[:, 3] = gy + u[:, 1]
    return m


# --------------------------------------------------------------------------
# scene families
# --------------------------------------------------------------------------

def layered_scene(H, W, n_layers, t_range, n_matches, stride, *, seed,
                  occl_frac=0.0, drop_frac=0.0, outlier_frac=0.0,
                  outlier_r=20.0, offset=None, K=100, a=1.0, mode=1,
                  name="layered", with_image=False, with_pair=False):
    """Background plus random star-shaped polygon layers, painted in order.

    Each layer moves by its own affine field u(p) = B (p - centre) + t with
    B entries ~ U[-0.05, 0.05] and t ~ U[-t_range, t_range].
    """
    rng = np.random.default_rng(seed)
    layer = np.zeros((H, W), np.int32)
    params = [(rng.uniform(-0.05, 0.05, (2, 2)),
               rng.uniform(-t_range, t_range, 2), ((W - 1) / 2, (H - 1) / 2))]
    masks = [None]
    for li in range(1, n_layers):
        poly, ctr = _star_polygon(rng, H, W)
        masks.append(_fill_polygon(poly, H, W))
        layer[masks[-1]] = li
        params.append((rng.uniform(-0.05, 0.05, (2, 2)),
                       rng.uniform(-t_range, t_range, 2), ctr))
    cost = _cost_from_layers(rng, layer)
    flow = _motion(layer, params)
    gx, gy = _grid(H, W, stride, offset)
    if occl_frac > 0:
        band = _boundary(layer)
        while band.mean() < occl_frac:
            band = ndimage.binary_dilation(band)
        keep = ~band[gy, gx]
        gx, gy = gx[keep], gy[keep]
    m = _finish_matches(rng, gx, gy, flow, n_matches, drop_frac, outlier_frac,
                        outlier_r, H, W)
    img = _layer_image(layer, seed) if (with_image or with_pair) else None
    img2 = _second_image(masks, params, seed, H, W) if with_pair else None
    return Scene(cost, m, K, a, mode, name, flow.astype(np.float32), img, img2)


def road_scene(H=375, W=1242, n_matches=10000, *, seed, horizon=150, K=100,
               a=0.8, mode=1, name="road"):
    """Ground plane below a horizon with an affine field diverging from the
    vanishing point, a slowly moving sky, and 4 rigid rectangular objects."""
    rng = np.random.default_rng(seed)
    layer = np.zeros((H, W), np.int32)           # 0 = sky
    layer[horizon:, :] = 1                        # 1 = ground
    e = (W / 2.0, float(horizon))
    Bg = np.diag([rng.uniform(0.03, 0.08), rng.uniform(0.05, 0.12)])
    params = [(np.zeros((2, 2)), rng.uniform(-2, 2, 2), e), (Bg, np.zeros(2), e)]
    for li in range(2, 6):
        w = int(rng.integers(60, 201))
        h = int(rng.integers(40, 101))
        x0 = int(rng.integers(0, W - w))
        y0 = int(rng.integers(max(0, horizon - h // 2), H - h))
        layer[y0:y0 + h, x0:x0 + w] = li
        params.append((rng.uniform(-0.01, 0.01, (2, 2)),
                       rng.uniform(-30, 30, 2), (x0 + w / 2, y0 + h / 2)))
    cost = _cost_from_layers(rng, layer)
    flow = _motion(layer, params)
    gx1, gy1 = _grid(H, W, 5)
    low = gy1 >= horizon
    gx2, gy2 = _grid(H, W, 15)
    high = gy2 < horizon
    gx = np.concatenate([gx1[low], gx2[high]])
    gy = np.concatenate([gy1[low], gy2[high]])
    order = np.lexsort((gx, gy))
    gx, gy = gx[order], gy[order]
    m = _finish_matches(rng, gx, gy, flow, n_matches, 0.0, 0.05, 20.0, H, W)
    return Scene(cost, m, K, a, mode, name, flow.astype(np.float32))


CONFIG_PARAMS = {
    # 128x96, 3 layers, t ~ U[-8, 8], stride 6 (21 x 16 = 336 grid points),
    # ~300 matches, 10% outliers with U[-20, 20] px flow, K=32, a=1, LA.
    1: dict(H=96, W=128, n_layers=3, t_range=8.0, n_matches=300, stride=6,
            outlier_frac=0.10, outlier_r=20.0, K=32, a=1.0, mode=1, seed=1),
    # 1024x436, 6 layers, t up to +-100 px, 15% occluded at layer borders,
    # stride 5, 20% low-saliency drop, 5% outliers, exactly 8000 matches,
    # K=100, a=1, LA.
    2: dict(H=436, W=1024, n_layers=6, t_range=100.0, n_matches=8000,
            stride=5, offset=2, occl_frac=0.15, drop_frac=0.20,
            outlier_frac=0.05, outlier_r=100.0, K=100, a=1.0, mode=1, seed=2),
}


def config_scene(i: int, mode: int | None = None, with_image: bool = False,
                 with_pair: bool = False) -> Scene:
    """The single-pair workloads: 1 = 128x96 small scene, 2 = 1024x436
    large-displacement scene, 3 = 1242x375 road scene (NW or LA)."""
    if i == 3:
        return road_scene(seed=3, mode=1 if mode is None else mode,
                          name="road_1242x375_n10000_k100")
    p = dict(CONFIG_PARAMS[i])
    if mode is not None:
        p["mode"] = mode
    H, W = p.pop("H"), p.pop("W")
    name = {1: "layered_128x96_n300_k32", 2: "layered_1024x436_n8000_k100"}[i]
    return layered_scene(H, W, name=name, with_image=with_image, with_pair=with_pair, **p)


def random_case(H, W, N, *, seed, K=8, a=1.0, mode=1, subpixel=True,
                n_layers=3, cost_scale=1.0, outside=0, duplicates=0):
    """Small random problem for parity tests: random layered scene with
    random (optionally sub-pixel) match positions; optionally some matches
    outside the image and some sharing a seed pixel."""
    rng = np.random.default_rng(seed)
    layer = np.zeros((H, W), np.int32)
    params = [(rng.uniform(-0.05, 0.05, (2, 2)), rng.uniform(-8, 8, 2),
               ((W - 1) / 2, (H - 1) / 2))]
    for li in range(1, n_layers):
        poly, ctr = _star_polygon(rng, H, W)
        layer[_fill_polygon(poly, H, W)] = li
        params.append((rng.uniform(-0.05, 0.05, (2, 2)),
                       rng.uniform(-8, 8, 2), ctr))
    cost = (_cost_from_layers(rng, layer).astype(np.float64) * cost_scale)
    cost = cost.astype(np.float32)
    flow = _motion(layer, params)
    n_in = N - outside
    pix = rng.choice(H * W, size=min(n_in, H * W), replace=False)
    xs = (pix % W).astype(np.float64)
    ys = (pix // W).astype(np.float64)
    if subpixel:
        xs = xs + rng.uniform(-0.49, 0.49, xs.shape)
        ys = ys + rng.uniform(-0.49, 0.49, ys.shape)
    u = flow[pix // W, pix % W] + rng.normal(0, 0.5, (len(pix), 2))
    m = np.zeros((N, 4), np.float32)
    m[:len(pix), 0] = xs
    m[:len(pix), 1] = ys
    m[:len(pix), 2] = xs + u[:, 0]
    m[:len(pix), 3] = ys + u[:, 1]
    for j in range(len(pix), N):       # outside the image
        m[j] = [rng.choice([-3.0, W + 2.0]), rng.uniform(0, H), 0.0, 0.0]
    if duplicates and len(pix) > 1:
        src = rng.choice(len(pix), duplicates, replace=True)
        dst = rng.choice(len(pix), duplicates, replace=False)
        for s_, d_ in zip(src, dst):
            if s_ != d_:
                m[d_, 0:2] = m[s_, 0:2] + np.float32(0.1)
    return Scene(cost, m, K, a, mode, f"random_{H}x{W}_n{N}_s{seed}",
                 flow.astype(np.float32))


BATCH_SIZES = [(192, 256), (480, 640), (436, 1024), (375, 1242)]


def _stride_for(H, W, n, drop=0.0):
    """Largest grid stride that yields at least n candidates after a drop."""
    s = max(1, int(math.sqrt(H * W * (1 - drop) / max(n, 1))))
    while s > 1:
        gx, _ = _grid(H, W, s)
        if len(gx) * (1 - drop) >= n:
            break
        s -= 1
    return s


def batch_scenes(n_pairs=64, seed0=4000, K=100, a=1.0, mode=1, with_image=False):
    """Mixed-size batch: each pair uniform over 4 sizes, 500..15000 matches,
    3-6 layers with t ~ U[-32, 32], per-pair seeds seed0 + i."""
    out = []
    for i in range(n_pairs):
        rng = np.random.default_rng(seed0 + i)
        H, W = BATCH_SIZES[int(rng.integers(0, 4))]
        n = int(rng.integers(500, 15001))
        nl = int(rng.integers(3, 7))
        s = _stride_for(H, W, n, 0.1)
        out.append(layered_scene(H, W, nl, 32.0, n, s, seed=seed0 + i,
                                 drop_frac=0.1, outlier_frac=0.05,
                                 outlier_r=32.0, K=K, a=a, mode=mode,
                                 name=f"batch{i}_{W}x{H}_n{n}", with_image=with_image))
    return out


SERVE_SIZES = [(240, 320), (480, 640), (436, 1024), (375, 1242), (720, 1280),
               (1080, 1920), (1080, 2048)]


def serve_stream(n_requests=2000, seed=5000, mean_gap_s=0.005):
    """Poisson request stream: (arrival_s, size, N, K) tuples.  Scenes are
    built lazily by ``serve_scene`` so that a long stream stays cheap."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(mean_gap_s, n_requests))
    reqs = []
    for i in range(n_requests):
        H, W = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
        n_hi = min(40000, (H * W) // 40)
        n = int(rng.integers(500, n_hi + 1))
        K = int(rng.choice([50, 100]))
        reqs.append(dict(arrival=float(t[i]), H=H, W=W, N=n, K=K,
                         seed=seed + 1 + i))
    return reqs


class ServeBase:
    """One image of the served stream's size class: 4 layers (t ~ U[-32, 32])
    with their cost map, motion and saliency field.  Requests of this size
    draw their own matches from it (``ServeBase.request``)."""

    def __init__(self, H, W, seed):
        rng = np.random.default_rng(seed)
        layer = np.zeros((H, W), np.int32)
        params = [(rng.uniform(-0.05, 0.05, (2, 2)), rng.uniform(-32, 32, 2), ((W - 1) / 2, (H - 1) / 2))]
        for li in range(1, 4):
            poly, ctr = _star_polygon(rng, H, W)
            layer[_fill_polygon(poly, H, W)] = li
            params.append((rng.uniform(-0.05, 0.05, (2, 2)), rng.uniform(-32, 32, 2), ctr))
        self.H, self.W = H, W
        self.cost = _cost_from_layers(rng, layer)
        self.flow = _motion(layer, params)
        self.saliency = ndimage.gaussian_filter(rng.standard_normal((H, W)), 8.0)

    def request(self, req) -> Scene:
        """The request's own match set: grid at the stride its N needs, the
        10% lowest-saliency points dropped, subsampled to exactly N, 5%
        outliers with U[-32, 32] px displacements, all from its own seed."""
        H, W, n = self.H, self.W, req["N"]
        rng = np.random.default_rng(req["seed"])
        gx, gy = _grid(H, W, _stride_for(H, W, n, 0.1))
        keep = np.sort(np.argsort(self.saliency[gy, gx], kind="stable")[int(round(0.1 * len(gx))):])
        gx, gy = gx[keep], gy[keep]
        if len(gx) > n:
            sel = np.sort(rng.choice(len(gx), n, replace=False))
            gx, gy = gx[sel], gy[sel]
        u = self.flow[gy, gx].copy()
        n_out = int(round(0.05 * len(gx)))
        if n_out:
            idx = rng.choice(len(gx), n_out, replace=False)
            u[idx] = rng.uniform(-32.0, 32.0, (n_out, 2))
        m = np.empty((len(gx), 4), np.float32)
        m[:, 0], m[:, 1] = gx, gy
        m[:, 2], m[:, 3] = gx + u[:, 0], gy + u[:, 1]
        return Scene(self.cost, m, req["K"], 1.0, 1, f"serve_{W}x{H}_n{len(gx)}_k{req['K']}")


def serve_bases(seed=5000):
    """One ServeBase per size of the served stream."""
    return {(H, W): ServeBase(H, W, seed + 100000 + i) for i, (H, W) in enumerate(SERVE_SIZES)}


def serve_scene(req) -> Scene:
    H, W, n = req["H"], req["W"], req["N"]
    s = _stride_for(H, W, n, 0.1)
    return layered_scene(H, W, 4, 32.0, n, s, seed=req["seed"], drop_frac=0.1,
                         outlier_frac=0.05, outlier_r=32.0, K=req["K"], a=1.0,
                         mode=1, name=f"serve_{W}x{H}_n{n}_k{req['K']}")
