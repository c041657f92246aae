"""GPU: the one-level variational refinement (Sec. 4) against the FP64
oracle in oracle/variational.py, on the scenes' image pairs with the
oracle's interpolation as the initial field.

Tolerance.  The refinement is an iteration (5 x 30 relaxation sweeps whose
weights psi'(s^2) = 1 / (2 sqrt(s^2 + eps^2)) change by a large factor where
a residual s is near eps = 1e-3), so FP32 rounding is amplified where the
weights are steep.  Running the oracle's own steps in float32 on these
scenes moves the result by a mean of 1.2e-6 (128 x 96) and 8.3e-6 px
(1024 x 436), at most 1.0e-3 px at one pixel; the bars below keep a factor
of ten over that: mean end-point difference 1e-4 px, largest 1e-2 px.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import epic_ref
from oracle import variational as va
from scenes import config_scene

pytestmark = pytest.mark.gpu

MEAN_TOL = 1e-4
MAX_TOL = 1e-2


def _epe(a, b):
    return np.sqrt(((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2).sum(-1))


def _case(i):
    s = config_scene(i, with_pair=True)
    u0 = epic_ref.interp(s.cost, s.matches, s.K, s.a, s.mode)[0].astype(np.float32)
    return s, u0


def _gpu(ctx, I1, I2, u0, **kw):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    out = ctx.refine(t(I1), t(I2), t(u0), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    import paper_1501_02565_amd as epic
    with epic.Context(workspace=256 << 20) as c:
        yield c


@pytest.mark.parametrize("i", [1, 2])
def test_refine_matches_oracle(ctx, i):
    s, u0 = _case(i)
    print(f"[case] refine config scene {i} {s.H}x{s.W}", flush=True)
    got = _gpu(ctx, s.image, s.image2, u0)
    ref = va.refine(s.image, s.image2, u0)
    d = _epe(got, ref)
    assert np.isfinite(got).all()
    assert d.mean() <= MEAN_TOL, d.mean()
    assert d.max() <= MAX_TOL, d.max()
    # and the refinement does what it is for: closer to the generating motion
    assert _epe(got, s.gt_flow).mean() < _epe(u0, s.gt_flow).mean()


@pytest.mark.parametrize("H,W,ch,kw", [
    (1, 1, 3, {}), (1, 37, 1, {}), (29, 1, 3, {}), (5, 7, 1, {"fixed_point": 2, "sor": 3}),
    (63, 65, 4, {"lam": 0.5, "omega": 1.2}), (40, 300, 2, {"delta": 0.0, "gamma": 1.0}),
    (97, 131, 3, {"kappa": 0.0, "eps": 1e-2, "zeta": 0.3})])
def test_refine_shapes_and_parameters(ctx, H, W, ch, kw):
    rng = np.random.default_rng(H * 131 + W * 7 + ch)
    from scipy import ndimage
    I1 = np.stack([ndimage.gaussian_filter(rng.uniform(0, 1, (H, W)), 1.5) for _ in range(ch)], -1)
    I2 = np.roll(I1, (1, 2), (0, 1)) + rng.uniform(0, 0.01, I1.shape)
    if ch == 1:
        I1, I2 = I1[..., 0], I2[..., 0]
    u0 = np.stack([ndimage.gaussian_filter(rng.normal(0, 2, (H, W)), 4) + 2,
                   ndimage.gaussian_filter(rng.normal(0, 2, (H, W)), 4) + 1], -1)
    print(f"[case] refine {H}x{W}x{ch} {kw}", flush=True)
    got = _gpu(ctx, I1, I2, u0, **kw)
    ref = va.refine(I1, I2, u0, va.Params(**kw))
    d = _epe(got, ref)
    assert d.mean() <= MEAN_TOL, d.mean()
    assert d.max() <= MAX_TOL, d.max()


def test_refine_identity_cases(ctx):
    """No iterations (or no sweeps) return the input field itself; the
    output may be the input buffer."""
    import torch
    s, u0 = _case(1)
    for kw in ({"fixed_point": 0}, {"sor": 0}):
        got = _gpu(ctx, s.image, s.image2, u0, **kw)
        assert np.array_equal(got, u0), kw
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    I1, I2, f = t(s.image), t(s.image2), t(u0)
    sep = ctx.refine(I1, I2, f)
    ctx.refine(I1, I2, f, out=f)
    torch.cuda.synchronize()
    assert torch.equal(sep, f)


def test_refine_deterministic_and_keeps_stats(ctx):
    """Two calls give the same bits; the interpolation's statistics survive
    a refinement when the workspace holds both."""
    import torch
    s, u0 = _case(1)
    a = _gpu(ctx, s.image, s.image2, u0)
    b = _gpu(ctx, s.image, s.image2, u0)
    assert np.array_equal(a, b)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    flow = ctx.interp(t(s.cost), t(s.matches), s.K, s.a, s.mode)
    before = ctx.stats()
    ctx.refine(t(s.image), t(s.image2), flow)
    torch.cuda.synchronize()
    assert ctx.stats() == before


def test_refine_argument_errors(ctx):
    import torch
    import paper_1501_02565_amd as epic
    s, u0 = _case(1)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    I1, I2, f = t(s.image), t(s.image2), t(u0)
    for kw in ({"omega": 2.0}, {"omega": 0.0}, {"eps": 0.0}, {"zeta": -1.0}, {"lam": float("nan")},
               {"fixed_point": -1}, {"sor": 10001}, {"kappa": -1.0}):
        with pytest.raises(epic.EpicError) as e:
            ctx.refine(I1, I2, f, **kw)
        assert e.value.status == epic.ERR_ARG, kw
    # a shifted view of the input as output
    big = torch.zeros(u0.size + 2, dtype=torch.float32, device="cuda")
    big[: u0.size] = f.reshape(-1)
    with pytest.raises(epic.EpicError):
        ctx.refine(I1, I2, big[: u0.size].view(u0.shape), out=big[2:].view(u0.shape))
    # a workspace without room
    with epic.Context(workspace=1 << 20) as small:
        with pytest.raises(epic.EpicError) as e:
            small.refine(I1, I2, f)
        assert e.value.status == epic.ERR_WORKSPACE
