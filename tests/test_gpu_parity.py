"""GPU parity: every stage of the HIP path against the FP64 oracle on the
same seeded inputs (tolerances in tests/parity.py).  Runs through the C ABI
(ctypes binding).  Needs an MI355X."""
from __future__ import annotations

import numpy as np
import pytest

import parity
from scenes import config_scene, random_case, serve_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1501_02565_amd as epic
    c = epic.Context(0)
    yield c
    c.close()


def _announce(name):
    print(f"\n[case] {name}", flush=True)


@pytest.mark.parametrize("H,W,N,seed", [(45, 70, 40, 0), (130, 100, 200, 1),
                                        (33, 97, 120, 2), (64, 64, 64, 3),
                                        (200, 45, 150, 4)])
def test_random_cases(ctx, H, W, N, seed):
    """Several tiles with ragged right/bottom tails, sub-pixel matches,
    matches outside the image and on shared pixels."""
    sc = random_case(H, W, N, seed=seed, K=12, outside=3, duplicates=4)
    _announce(sc.name)
    for mode in (1, 0):
        res = parity.full_check(ctx, sc, mode=mode)
        print(res, flush=True)


@pytest.mark.parametrize("i,mode", [(1, 1), (2, 1), (3, 1), (3, 0)])
def test_config_scenes(ctx, i, mode):
    """The small scene, the 1024x436 large-displacement scene and the
    1242x375 road scene (NW and LA)."""
    sc = config_scene(i, mode=mode)
    _announce(f"{sc.name} mode={mode}")
    res = parity.full_check(ctx, sc)
    print(res, flush=True)


@pytest.mark.parametrize("K", [100, 50])
def test_largest_served_size(ctx, K):
    """The largest request of the served stream: 2048 x 1080 pixels with
    40000 matches, every stage against the oracle."""
    sc = serve_scene(dict(H=1080, W=2048, N=40000, K=K, seed=7001 + K))
    _announce(sc.name)
    res = parity.full_check(ctx, sc)
    print(res, flush=True)


def test_large_call_output_alignment(ctx):
    """A 2048 x 1080 call has more pixels than the chip holds single-pixel
    wavefronts, so its assignment takes four pixels per thread and stores
    16-byte pairs; into an output that is only 8-byte aligned it stores pixel
    by pixel.  Both outputs hold the same bits."""
    import torch
    sc = serve_scene(dict(H=1080, W=2048, N=20000, K=50, seed=7201))
    _announce(sc.name + " 8-byte aligned output")
    cost = torch.from_numpy(sc.cost).cuda()
    matches = torch.from_numpy(sc.matches).cuda()
    aligned = ctx.interp(cost, matches, sc.K, sc.a, sc.mode)
    buf = torch.full((sc.H * sc.W * 2 + 2,), 7.0, dtype=torch.float32, device="cuda")
    out = buf[2:].view(sc.H, sc.W, 2)
    assert out.data_ptr() % 16 == 8
    ctx.interp(cost, matches, sc.K, sc.a, sc.mode, out=out)
    torch.cuda.synchronize()
    assert ctx.stats()["status"] == 0
    np.testing.assert_array_equal(out.cpu().numpy(), aligned.cpu().numpy())
    assert buf[:2].cpu().tolist() == [7.0, 7.0]      # nothing written before the output


@pytest.mark.parametrize("K", [1, 2, 3, 7, 128, 256])
def test_k_values(ctx, K):
    sc = random_case(60, 80, 300, seed=11, K=K)
    _announce(f"{sc.name} K={K}")
    parity.full_check(ctx, sc, K=K)


def test_k_larger_than_matches(ctx):
    sc = random_case(40, 50, 9, seed=12, K=50)
    _announce(sc.name)
    res = parity.full_check(ctx, sc)
    assert res["stats"]["n_used"] == 9


def test_single_and_two_matches(ctx):
    for N in (1, 2):
        sc = random_case(37, 41, N, seed=13 + N, K=5)
        _announce(sc.name)
        parity.full_check(ctx, sc)


def test_no_match_in_image(ctx):
    sc = random_case(20, 30, 4, seed=15, K=3, outside=4)
    _announce(sc.name)
    res = parity.full_check(ctx, sc)
    assert res["epe"] == 0.0


@pytest.mark.parametrize("H,W", [(1, 1), (1, 77), (90, 1), (2, 2)])
def test_degenerate_shapes(ctx, H, W):
    rng = np.random.default_rng(H * 100 + W)
    sc = random_case(max(H, 3), max(W, 3), 3, seed=16, K=3)
    sc.cost = rng.uniform(0.01, 1, (H, W)).astype(np.float32)
    N = min(3, H * W)
    m = np.zeros((N, 4), np.float32)
    pix = rng.choice(H * W, N, replace=False)
    m[:, 0], m[:, 1] = pix % W, pix // W
    m[:, 2:] = m[:, :2] + rng.normal(0, 2, (N, 2))
    sc.matches = m
    _announce(f"shape {H}x{W}")
    parity.full_check(ctx, sc, K=3)


def test_a_zero_and_large(ctx):
    sc = random_case(50, 60, 80, seed=17, K=10)
    for a in (0.0, 5.0):
        _announce(f"{sc.name} a={a}")
        parity.full_check(ctx, sc, a=a)


def test_global_affine_recovered(ctx):
    """A single global affine motion is reproduced at every pixel by LA,
    for any cost map (exactly in the oracle; to FP32 rounding here)."""
    import torch
    H, W, N = 96, 128, 300
    rng = np.random.default_rng(18)
    A = np.array([[1.0625, -0.03125], [0.046875, 0.9375]])
    t = np.array([2.25, -3.5])
    sc = random_case(H, W, N, seed=18, K=32)
    pix = rng.choice(H * W, N, replace=False)
    m = np.zeros((N, 4), np.float32)
    m[:, 0], m[:, 1] = pix % W, pix // W
    m[:, 2:] = m[:, :2].astype(np.float64) @ A.T + t
    t_cost = torch.from_numpy(sc.cost).cuda()
    flow = ctx.interp(t_cost, torch.from_numpy(m).cuda(), 32, 1.0, 1).cpu().numpy()
    ys, xs = np.mgrid[0:H, 0:W]
    # FP32 rounding: centred sums of 32 terms (relative ~2e-6) move B by
    # ~1e-7 and c by ~1e-6 px, i.e. ~1e-5 px at 30 px from the match
    err = np.maximum(np.abs(flow[..., 0] - ((A[0, 0] - 1) * xs + A[0, 1] * ys + t[0])),
                     np.abs(flow[..., 1] - (A[1, 0] * xs + (A[1, 1] - 1) * ys + t[1])))
    print(f"global affine: max error {err.max():.2e} px", flush=True)
    assert err.max() <= 1e-4


def test_label_invariance_under_cost_scaling(ctx):
    """C -> 4 C keeps every label and scales D exactly (powers of two)."""
    sc = random_case(100, 120, 150, seed=19, K=10)
    g1 = parity.gpu_stages(ctx, sc)
    sc2 = random_case(100, 120, 150, seed=19, K=10)
    sc2.cost = sc2.cost * np.float32(4.0)
    g2 = parity.gpu_stages(ctx, sc2, a=sc.a / 4.0)
    np.testing.assert_array_equal(g1["L"], g2["L"])
    np.testing.assert_array_equal(g1["D"] * 4, g2["D"])
    np.testing.assert_array_equal(g1["flow"], g2["flow"])


def test_repeatable(ctx):
    """Two runs give bitwise identical flows."""
    import torch
    sc = config_scene(1)
    c = torch.from_numpy(sc.cost).cuda()
    m = torch.from_numpy(sc.matches).cuda()
    f1 = ctx.interp(c, m, sc.K, sc.a, sc.mode).clone()
    f2 = ctx.interp(c, m, sc.K, sc.a, sc.mode)
    torch.cuda.synchronize()
    assert torch.equal(f1, f2)


@pytest.mark.parametrize("opts", [dict(connectivity=4), dict(la_weight_power=1),
                                  dict(tile=(32, 16)), dict(tile=(32, 64))])
def test_options(opts):
    import paper_1501_02565_amd as epic
    sc = random_case(150, 170, 250, seed=20, K=16)
    conn = opts.get("connectivity", 8)
    wpow = opts.get("la_weight_power", 2)
    _announce(f"{sc.name} {opts}")
    with epic.Context(0, epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K), **opts) as c:
        parity.full_check(c, sc, conn=conn, wpow=wpow)


def test_workspace_too_small():
    import torch
    import paper_1501_02565_amd as epic
    sc = random_case(64, 64, 50, seed=21, K=8)
    with epic.Context(0, epic.workspace_bytes(32, 32, 10, 8)) as c:
        with pytest.raises(epic.EpicError) as ei:
            c.interp(torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda(), 8, 1.0, 1)
        assert ei.value.status == epic.ERR_WORKSPACE


def test_pass_budget_does_not_change_results():
    """The geodesic pass budget (fixed small, fixed large, automatic over
    repeated calls) and the threads per tile of the later passes only change
    how the work is done: flows are bitwise identical."""
    import torch
    import paper_1501_02565_amd as epic
    sc = random_case(180, 230, 400, seed=22, K=16)
    _announce(f"{sc.name} pass budgets")
    c = torch.from_numpy(sc.cost).cuda()
    m = torch.from_numpy(sc.matches).cuda()
    ws = epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K)
    flows = []
    for passes, calls, threads in ((1, 1, 0), (3, 1, 0), (16, 1, 0), (0, 4, 0), (3, 1, 128), (0, 2, 128),
                                   (2, 1, 256)):
        with epic.Context(0, ws, passes=passes, geo_threads=threads) as ctx:
            for _ in range(calls):
                f = ctx.interp(c, m, sc.K, sc.a, sc.mode).clone()
                torch.cuda.synchronize()
                flows.append(f)
    for f in flows[1:]:
        assert torch.equal(flows[0], f)
    # the FP64 transform: budgets per phase, its finisher doing most of the
    # work when the budget is 1 pass
    ws64 = epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K, precision=1)
    flows64 = []
    for passes, calls in ((1, 1), (3, 1), (0, 3)):
        with epic.Context(0, ws64, passes=passes, precision=1) as ctx:
            for _ in range(calls):
                flows64.append(ctx.interp(c, m, sc.K, sc.a, sc.mode).clone())
                torch.cuda.synchronize()
    for f in flows64[1:]:
        assert torch.equal(flows64[0], f)


def test_pass_budget_bitwise_on_large_scene():
    """On the 1024 x 436 scene: 2 passes (the finisher does the rest), 5, 12
    and the automatic budget over repeated calls give bitwise identical D,
    L and flow -- the transform reaches the same fixpoint whatever the
    schedule."""
    import torch
    import paper_1501_02565_amd as epic
    sc = config_scene(2)
    _announce(f"{sc.name} pass budgets")
    ws = epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K)
    outs = []
    for passes, calls in ((2, 1), (5, 1), (12, 1), (0, 4)):
        with epic.Context(0, ws, passes=passes) as c:
            for _ in range(calls):
                g = parity.gpu_stages(c, sc)
            outs.append(g)
    for g in outs[1:]:
        for k in ("D", "L", "flow"):
            np.testing.assert_array_equal(outs[0][k], g[k])
