"""MI355X-native sparse-to-dense, edge-preserving interpolation (EpicFlow,
Revaud et al. 2015, Sec. 3), as a HIP library with a thin Python binding.

All computation runs in the HIP kernels of ``libepic.so``; this module only
marshals torch tensors (device memory) and streams into the C ABI of
``include/epic.h``.

    import torch, paper_1501_02565_amd as epic
    ctx = epic.Context()
    flow = ctx.interp(cost, matches, K=100, a=1.0, mode=epic.LA)   # (H, W, 2)
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (LA, NW, OK, EpicError, ERR_ARG, ERR_BUDGET, ERR_CAPACITY,  # noqa: F401
                   ERR_CONVERGENCE, ERR_COST, ERR_HIP, ERR_INVARIANT, ERR_NO_MATCHES, ERR_WORKSPACE)

__all__ = ["Context", "workspace_bytes", "image_cost", "ImageCostPlan", "LA", "NW", "EpicError"]

GRAD_EPS = 1e-3      # default floor of the gradient cost


def _torch():
    import torch
    return torch


def workspace_bytes(H: int, W: int, N: int, K: int, mode: int = LA,
                    precision: int = 0) -> int:
    """Device workspace one call of this size needs (host-only query)."""
    return int(_lib.load().epic_workspace_bytes(H, W, N, K, mode, precision))


class ImageCostPlan:
    """Descriptors of a fixed set of images and cost buffers, marshalled once
    (for repeated calls: run() is then a single C call)."""

    def __init__(self, images, outs=None, eps: float = GRAD_EPS):
        torch = _torch()
        self.images = list(images)
        self.eps = float(eps)
        self.descs = (_lib.Image * len(self.images))()
        self.costs = []
        for i, im in enumerate(self.images):
            _check_tensor(im, "image", torch.float32)
            H, W = im.shape[:2]
            ch = 1 if im.dim() == 2 else int(im.shape[2])
            c = outs[i] if outs is not None else torch.empty((H, W), dtype=torch.float32, device=im.device)
            _check_tensor(c, "cost", torch.float32)
            self.costs.append(c)
            self.descs[i] = _lib.Image(im.data_ptr(), H, W, ch, c.data_ptr())

    def run(self, stream=None):
        rc = _lib.load().epic_image_cost(self.descs, len(self.images), self.eps, _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_image_cost")
        return self.costs


def image_cost(images, eps: float = GRAD_EPS, outs=None, stream=None):
    """Cost maps from images (Table 2, norm of the image gradient): for each
    float32 CUDA tensor of shape (H, W) or (H, W, channels <= 4), C =
    ||grad I|| + eps as an (H, W) float32 tensor.  One launch per run of up
    to 64 images with equal channel counts."""
    torch = _torch()
    single = isinstance(images, torch.Tensor)
    costs = ImageCostPlan([images] if single else images, outs, eps).run(stream)
    return costs[0] if single else costs


def refine_params(**overrides):
    """epic_refine_params: the library defaults with `overrides` applied."""
    p = _lib.RefineParams()
    _lib.load().epic_refine_defaults(ctypes.byref(p))
    for k, v in overrides.items():
        if not any(k == f[0] for f in _lib.RefineParams._fields_):
            raise TypeError(f"unknown refinement parameter {k!r}")
        setattr(p, k, v)
    return p


def refine_bytes(H: int, W: int, channels: int = 3) -> int:
    """Workspace bytes epic_refine takes at the end of the workspace."""
    return int(_lib.load().epic_refine_bytes(H, W, channels))


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_tensor(t, name, dtype, shape_tail=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[-len(shape_tail):]) != shape_tail:
        raise ValueError(f"{name} must end in shape {shape_tail}")


class Context:
    """Owns one epic_ctx: a device workspace allocated once (``workspace``
    bytes, default enough for a 2048 x 1080 image with 40000 matches).
    ``passes`` is the geodesic pass budget per call (0 = automatic, from the
    passes the recent calls needed); it never changes results.
    ``geo_threads`` sets the threads per tile of the transform's later passes
    (0 = default; 128 or 256 with 32 x 16 tiles); like ``passes`` it only
    changes the speed.
    ``debug_validate`` makes every call check the cost map on the device
    (finite and > 0; a pair that fails reports ERR_COST in its stats) and
    the invariants of its transform and match graph (violations:
    n_invariant, ERR_INVARIANT); 2 plants a violation first (a self-test of
    the checks).
    ``prune_px`` > 0 runs the consistency check of the matches (Sec. 5.1)
    before every interpolation: matches further than prune_px from a first
    NW estimate at their pixel are removed (the paper uses 5)."""

    def __init__(self, device: int = 0, workspace: int | None = None, *,
                 connectivity: int = 8, la_weight_power: int = 2,
                 precision: int = 0, fp64_route: float = 1e-3,
                 degenerate_tau: float = 1e-9, tile: tuple[int, int] = (32, 16),
                 passes: int = 0, geo_threads: int = 0, debug_validate: int = 0,
                 prune_px: float = 0.0):
        torch = _torch()
        L = _lib.load()
        self.device = int(device)
        if workspace is None:
            workspace = workspace_bytes(1080, 2048, 40000, 256, precision=precision)
        self.workspace = int(workspace)
        self.options = _lib.Options(connectivity, la_weight_power, precision,
                                    fp64_route, degenerate_tau, tile[0], tile[1],
                                    passes, int(geo_threads), int(debug_validate),
                                    float(prune_px))
        torch.cuda.init()
        with torch.cuda.device(self.device):
            self._ctx = L.epic_create(self.device, self.workspace,
                                      ctypes.byref(self.options))
        if not self._ctx:
            raise RuntimeError("epic_create failed: " + L.epic_last_error().decode())

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.load().epic_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def interp(self, cost, matches, K: int, a: float, mode: int = LA, out=None,
               stream=None):
        """Dense flow (H, W, 2) float32 for one pair.  cost (H, W) and
        matches (N, 4) are float32 CUDA tensors.  Asynchronous on `stream`
        (default: torch's current stream)."""
        torch = _torch()
        _check_tensor(cost, "cost", torch.float32)
        _check_tensor(matches, "matches", torch.float32, (4,))
        H, W = cost.shape
        N = matches.shape[0]
        if out is None:
            out = torch.empty((H, W, 2), dtype=torch.float32, device=cost.device)
        _check_tensor(out, "out", torch.float32, (H, W, 2))
        rc = _lib.load().epic_interp(self._ctx, cost.data_ptr(), H, W,
                                     matches.data_ptr(), N, int(K), float(a),
                                     int(mode), out.data_ptr(),
                                     _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_interp")
        return out

    def interp_image(self, image, matches, K: int, a: float, mode: int = LA, eps: float = GRAD_EPS,
                     out=None, stream=None):
        """As interp, with an image (H, W[, channels]) in place of the cost
        map: the cost is its gradient norm plus eps, computed on the GPU."""
        torch = _torch()
        _check_tensor(image, "image", torch.float32)
        _check_tensor(matches, "matches", torch.float32, (4,))
        H, W = image.shape[:2]
        ch = 1 if image.dim() == 2 else int(image.shape[2])
        if out is None:
            out = torch.empty((H, W, 2), dtype=torch.float32, device=image.device)
        _check_tensor(out, "out", torch.float32, (H, W, 2))
        rc = _lib.load().epic_interp_image(self._ctx, image.data_ptr(), H, W, ch, float(eps),
                                           matches.data_ptr(), matches.shape[0], int(K), float(a),
                                           int(mode), out.data_ptr(), _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_interp_image")
        return out

    def interp_exact(self, cost, matches, K: int, a: float, mode: int = LA, out=None, stream=None):
        """The exact per-pixel geodesic interpolation (Table 2, "Geodesic
        (exact)"): each pixel's own K nearest matches under the geodesic
        distance and its own fit.  Needs a workspace of about
        8*K*H*W + N + 512 bytes plus, per match processed at once,
        workspace_bytes(H, W, 1, 1)."""
        torch = _torch()
        _check_tensor(cost, "cost", torch.float32)
        _check_tensor(matches, "matches", torch.float32, (4,))
        H, W = cost.shape
        if out is None:
            out = torch.empty((H, W, 2), dtype=torch.float32, device=cost.device)
        _check_tensor(out, "out", torch.float32, (H, W, 2))
        rc = _lib.load().epic_interp_exact(self._ctx, cost.data_ptr(), H, W, matches.data_ptr(),
                                           matches.shape[0], int(K), float(a), int(mode), out.data_ptr(),
                                           _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_interp_exact")
        return out

    def refine(self, I1, I2, flow, out=None, stream=None, **params):
        """One-level variational refinement (Sec. 4) of a dense field
        `flow` (H, W, 2) between images I1 and I2 (H, W[, channels <= 4]),
        all float32 CUDA tensors.  Keyword parameters override the defaults
        (lam, delta, gamma, kappa, eps, zeta, omega, fixed_point, sor);
        `out` may be `flow` itself.  Needs refine_bytes(H, W, channels)
        bytes at the end of the workspace beyond its fixed head."""
        torch = _torch()
        _check_tensor(I1, "I1", torch.float32)
        _check_tensor(I2, "I2", torch.float32)
        if I1.shape != I2.shape:
            raise ValueError("I1 and I2 must have the same shape")
        H, W = I1.shape[:2]
        ch = 1 if I1.dim() == 2 else int(I1.shape[2])
        _check_tensor(flow, "flow", torch.float32, (H, W, 2))
        if out is None:
            out = torch.empty((H, W, 2), dtype=torch.float32, device=flow.device)
        _check_tensor(out, "out", torch.float32, (H, W, 2))
        p = refine_params(**params)
        rc = _lib.load().epic_refine(self._ctx, I1.data_ptr(), I2.data_ptr(), H, W, ch,
                                     flow.data_ptr(), out.data_ptr(), ctypes.byref(p),
                                     _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_refine")
        return out

    def interp_batch(self, problems, outs=None, stream=None):
        """problems: list of (cost, matches, K, a, mode).  One fused launch
        sequence for all of them; returns the list of flows."""
        reqs, flows = self._requests(problems, outs)
        rc = _lib.load().epic_interp_batch(self._ctx, reqs, len(problems),
                                           _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_interp_batch")
        return flows

    def _requests(self, problems, outs):
        torch = _torch()
        n = len(problems)
        reqs = (_lib.Request * n)()
        flows = []
        for i, (cost, matches, K, a, mode) in enumerate(problems):
            _check_tensor(cost, "cost", torch.float32)
            _check_tensor(matches, "matches", torch.float32, (4,))
            H, W = cost.shape
            f = outs[i] if outs is not None else torch.empty(
                (H, W, 2), dtype=torch.float32, device=cost.device)
            _check_tensor(f, "out", torch.float32, (H, W, 2))
            flows.append(f)
            reqs[i] = _lib.Request(cost.data_ptr(), H, W, matches.data_ptr(),
                                   matches.shape[0], int(K), float(a), int(mode),
                                   f.data_ptr())
        return reqs, flows

    def capture(self, problems, outs=None):
        """Captures the launch sequence of interp_batch(problems) as a HIP
        graph bound to these tensors; returns a Graph whose launch() replays
        it (the tensors' contents may change between launches)."""
        reqs, flows = self._requests(problems, outs)
        g = _lib.load().epic_graph_capture(self._ctx, reqs, len(problems))
        if not g:
            raise RuntimeError("epic_graph_capture failed")
        return Graph(self, g, flows, problems)

    def debug_stages(self, cost, matches, K: int, a: float, mode: int = LA,
                     max_edges: int | None = None, stream=None):
        """Every stage output of one call (synchronises): D, L, edges, K-NN
        lists, per-match parameters, flow, stats."""
        torch = _torch()
        _check_tensor(cost, "cost", torch.float32)
        _check_tensor(matches, "matches", torch.float32, (4,))
        H, W = cost.shape
        N = matches.shape[0]
        dev = cost.device
        if max_edges is None:
            max_edges = 16 * N + 1024
        # the FP64-everywhere path reports D in double precision
        ddt = torch.float64 if self.options.precision == 1 else torch.float32
        D = torch.empty((H, W), dtype=ddt, device=dev)
        L = torch.empty((H, W), dtype=torch.int32, device=dev)
        em = torch.empty(max_edges, dtype=torch.int32, device=dev)
        en = torch.empty(max_edges, dtype=torch.int32, device=dev)
        ew = torch.empty(max_edges, dtype=torch.float32, device=dev)
        ne = torch.zeros(1, dtype=torch.int32, device=dev)
        ki = torch.empty((N, K), dtype=torch.int32, device=dev)
        kd = torch.empty((N, K), dtype=torch.float32, device=dev)
        P = torch.empty((N, 6), dtype=torch.float32, device=dev)
        flow = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
        rc = _lib.load().epic_debug_stages(
            self._ctx, cost.data_ptr(), H, W, matches.data_ptr(), N, int(K),
            float(a), int(mode), D.data_ptr(), L.data_ptr(), em.data_ptr(),
            en.data_ptr(), ew.data_ptr(), max_edges, ne.data_ptr(),
            ki.data_ptr(), kd.data_ptr(), P.data_ptr(), flow.data_ptr(),
            _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_debug_stages")
        st = self.stats(0)
        E = min(int(ne.item()), max_edges)
        return dict(D=D, L=L, em=em[:E], en=en[:E], ew=ew[:E], knn_idx=ki,
                    knn_d=kd, params=P, flow=flow, stats=st)

    def prune(self, cost, matches, K: int, a: float, prune_px: float = 5.0, stream=None):
        """The consistency check alone (synchronises): original indices of
        the matches whose displacement is within prune_px of the NW
        estimate at their pixel, as an int32 CUDA tensor."""
        torch = _torch()
        _check_tensor(cost, "cost", torch.float32)
        _check_tensor(matches, "matches", torch.float32, (4,))
        H, W = cost.shape
        N = matches.shape[0]
        kept = torch.empty(N, dtype=torch.int32, device=cost.device)
        nk = torch.zeros(1, dtype=torch.int32, device=cost.device)
        rc = _lib.load().epic_prune(self._ctx, cost.data_ptr(), H, W, matches.data_ptr(), N, int(K),
                                    float(a), float(prune_px), kept.data_ptr(), nk.data_ptr(),
                                    _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_prune")
        return kept[: int(nk.item())]

    def profile(self, enable: bool = True) -> None:
        """Turns per-stage HIP-event timing of every call on or off."""
        rc = _lib.load().epic_profile(self._ctx, int(bool(enable)))
        if rc != OK:
            raise EpicError(rc, "epic_profile")

    def stage_times(self, calls: int = 64) -> dict:
        """Mean milliseconds per stage over the last `calls` profiled calls
        (synchronises them)."""
        L = _lib.load()
        buf = (ctypes.c_float * 16)()
        n = L.epic_stage_times(self._ctx, buf, 16, int(calls))
        if n < 0:
            raise EpicError(n, "epic_stage_times")
        return {L.epic_stage_name(i).decode(): float(buf[i]) for i in range(n)}

    def pass_visits(self) -> list:
        """Tile visits per pass of the last call's transform (FP32 calls made
        while profiling; empty otherwise)."""
        buf = (ctypes.c_int * 256)()
        n = _lib.load().epic_pass_visits(self._ctx, buf, 256)
        if n < 0:
            raise EpicError(n, "epic_pass_visits")
        return list(buf[:n])

    def stats(self, pair: int = 0) -> dict:
        """Device counters of the last call (synchronises its stream)."""
        s = _lib.Stats()
        rc = _lib.load().epic_get_stats(self._ctx, int(pair), ctypes.byref(s))
        if rc != OK:
            raise EpicError(rc, "epic_get_stats")
        return {k: getattr(s, k) for k, _ in _lib.Stats._fields_}


class Graph:
    """A captured batch (see Context.capture)."""

    def __init__(self, ctx: Context, handle, flows, problems):
        self.ctx = ctx
        self._g = handle
        self.flows = flows
        self.problems = problems      # keeps the bound tensors alive

    def launch(self, stream=None):
        rc = _lib.load().epic_graph_launch(self._g, _stream_handle(stream))
        if rc != OK:
            raise EpicError(rc, "epic_graph_launch")
        return self.flows

    def close(self):
        if getattr(self, "_g", None):
            _lib.load().epic_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
