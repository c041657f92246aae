"""GPU: the batched form.  Many pairs in one fused launch sequence (and its
captured HIP graph) give each pair the result it gets alone, and match the
oracle on sampled pairs at full size."""
from __future__ import annotations

import numpy as np
import pytest

import parity
from oracle import epic_ref
from scenes import batch_scenes, random_case

pytestmark = pytest.mark.gpu


def _dev(sc):
    import torch
    return (torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda(),
            sc.K, sc.a, sc.mode)


def _mixed(n=8):
    out = []
    for i in range(n):
        sc = random_case(40 + 23 * i, 70 + 31 * (i % 3), 30 + 40 * i, seed=100 + i,
                         K=[4, 16, 100, 33][i % 4], mode=i % 2, outside=i % 2, duplicates=i % 3)
        out.append(sc)
    return out


def _epe(a, b):
    return np.linalg.norm(a.astype(np.float64) - b.astype(np.float64), axis=2)


@pytest.fixture(scope="module")
def ctx():
    import paper_1501_02565_amd as epic
    c = epic.Context(0, 512 << 20)
    yield c
    c.close()


# up to 8 pairs the descriptor table travels in the first kernel's
# arguments; 9 takes the upload path
@pytest.mark.parametrize("n", [8, 9])
def test_batch_equals_single(ctx, n):
    import torch
    scs = _mixed(n)
    probs = [_dev(sc) for sc in scs]
    flows = [f.cpu().numpy() for f in ctx.interp_batch(probs)]
    stats = [ctx.stats(i) for i in range(len(scs))]
    identical = 0
    for sc, p, f, st in zip(scs, probs, flows, stats):
        alone = ctx.interp(*p).cpu().numpy()
        assert st["status"] == 0
        identical += int(np.array_equal(alone, f))
        assert _epe(alone, f).mean() <= parity.EPE_MEAN
        ref = epic_ref.interp(sc.cost, sc.matches, sc.K, sc.a, sc.mode)[0]
        assert _epe(f, ref).mean() <= parity.EPE_MEAN
    print(f"bitwise identical alone vs batched: {identical}/{len(scs)}")
    # a unique fixpoint, sorted neighbour lists and fixed-order sums: the
    # batch changes nothing
    assert identical == len(scs)


@pytest.mark.parametrize("n", [5, 9])
def test_graph_replay_matches_eager(ctx, n):
    """Replays of the captured graph, with eager work and synchronisation in
    between, reproduce the eager batch every time."""
    import torch
    scs = _mixed(n)
    probs = [_dev(sc) for sc in scs]
    eager = [f.clone() for f in ctx.interp_batch(probs)]
    torch.cuda.synchronize()
    g = ctx.capture(probs)
    try:
        for rep in range(3):
            for f in g.flows:
                f.fill_(float("nan"))
            g.launch()
            torch.cuda.synchronize()
            for a, b in zip(eager, g.flows):
                assert _epe(a.cpu().numpy(), b.cpu().numpy()).mean() <= 1e-6
            # unrelated eager work between replays
            ctx.interp(*probs[0])
            torch.cuda.synchronize()
    finally:
        g.close()


def test_graph_sees_new_inputs(ctx):
    """The graph is bound to buffers, not to their contents."""
    import torch
    sc = random_case(60, 80, 120, seed=7, K=12)
    c, m, K, a, mode = _dev(sc)
    g = ctx.capture([(c, m, K, a, mode)])
    try:
        g.launch()
        torch.cuda.synchronize()
        sc2 = random_case(60, 80, 120, seed=8, K=12)
        c.copy_(torch.from_numpy(sc2.cost))
        m.copy_(torch.from_numpy(sc2.matches))
        g.launch()
        torch.cuda.synchronize()
        ref = epic_ref.interp(sc2.cost, sc2.matches, K, a, mode)[0]
        assert _epe(g.flows[0].cpu().numpy(), ref).mean() <= parity.EPE_MEAN
    finally:
        g.close()


def _shape_case(H, W, seed):
    """A pair of any shape (down to one row or column) with three matches."""
    rng = np.random.default_rng(seed)
    sc = random_case(max(H, 3), max(W, 3), 3, seed=seed, K=3)
    sc.cost = rng.uniform(0.01, 1, (H, W)).astype(np.float32)
    N = min(3, H * W)
    m = np.zeros((N, 4), np.float32)
    pix = rng.choice(H * W, N, replace=False)
    m[:, 0], m[:, 1] = pix % W, pix // W
    m[:, 2:] = m[:, :2] + rng.normal(0, 2, (N, 2))
    sc.matches = m
    return sc


def test_large_batch_with_odd_shapes_equals_single():
    """A batch above 2.1 Mpx assigns four pixels per thread, whose runs wrap
    rows (every pixel of a one-column image) and end short (pixel counts not
    a multiple of four); each pair equals its single call, bitwise."""
    import torch
    import paper_1501_02565_amd as epic
    from scenes import serve_scene
    scs = [serve_scene(dict(H=1080, W=2048, N=5000, K=16, seed=7401))]
    scs += [_shape_case(H, W, 7402 + i) for i, (H, W) in enumerate([(1, 77), (90, 1), (3, 5), (1, 1), (7, 3)])]
    print(f"[case] batch of {len(scs)}, {sum(s.H * s.W for s in scs)} px", flush=True)
    need = sum(epic.workspace_bytes(s.H, s.W, s.N, s.K) for s in scs)
    with epic.Context(0, need) as c:
        probs = [_dev(sc) for sc in scs]
        flows = [f.cpu().numpy() for f in c.interp_batch(probs)]
        st = [c.stats(i) for i in range(len(scs))]
        for i, sc in enumerate(scs):
            assert st[i]["status"] == 0, (i, st[i])
            alone = c.interp(*probs[i]).cpu().numpy()
            assert np.array_equal(alone, flows[i]), (i, sc.H, sc.W)
        ref = epic_ref.interp(scs[1].cost, scs[1].matches, scs[1].K, scs[1].a, scs[1].mode)[0]
        assert _epe(flows[1], ref).mean() <= parity.EPE_MEAN


@pytest.mark.parametrize("seed", [11, 12])
def test_random_large_batch(seed):
    """A random pair above 2.1 Mpx beside five small random pairs: the
    large-call forms (two-pixel emit, four-pixel assignment) give each pair
    its single call's flow, bitwise, and the large pair matches the oracle
    at every stage."""
    import torch
    import paper_1501_02565_amd as epic
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1450, 1500)), int(rng.integers(1500, 2048))
    big = random_case(H, W, int(rng.integers(3000, 18000)), seed=int(rng.integers(1 << 30)),
                      K=int(rng.choice([16, 50, 100])), mode=int(rng.integers(0, 2)))
    smalls = []
    for _ in range(5):
        h, w = int(rng.integers(3, 200)), int(rng.integers(3, 200))
        smalls.append(random_case(h, w, int(rng.integers(2, max(3, h * w // 4))), seed=int(rng.integers(1 << 30)),
                                  K=int(rng.choice([3, 8, 32, 100])), mode=int(rng.integers(0, 2)),
                                  outside=int(rng.integers(0, 3))))
    scs = [big] + smalls
    assert sum(s.H * s.W for s in scs) >= 4 * 256 * 32 * 64
    print(f"[case] seed {seed}: {big.name} with 5 small pairs", flush=True)
    need = sum(epic.workspace_bytes(s.H, s.W, s.N, s.K) for s in scs)
    with epic.Context(0, need) as c:
        probs = [_dev(sc) for sc in scs]
        flows = [f.cpu().numpy() for f in c.interp_batch(probs)]
        st = [c.stats(i) for i in range(len(scs))]
        assert all(x["status"] == 0 for x in st), st
        for i in range(len(scs)):
            alone = c.interp(*probs[i]).cpu().numpy()
            assert np.array_equal(alone, flows[i]), i
        parity.full_check(c, big)


def test_full_size_batch_sampled_parity():
    """The 64-pair mixed-size batch at full size (the batched benchmark's
    launch configuration); every 8th pair is checked against the oracle and
    against its own single call, bitwise (the batch assigns four pixels per
    thread, a call of one such pair one)."""
    import torch
    import paper_1501_02565_amd as epic
    scs = batch_scenes(64)
    print(f"[case] batch of 64, {sum(s.H * s.W for s in scs) / 1e6:.1f} Mpx, "
          f"{sum(s.N for s in scs)} matches", flush=True)
    need = sum(epic.workspace_bytes(s.H, s.W, s.N, s.K) for s in scs)
    with epic.Context(0, need) as c:
        probs = [_dev(sc) for sc in scs]
        flows = c.interp_batch(probs)
        torch.cuda.synchronize()
        for i in range(0, 64, 8):
            st = c.stats(i)
            assert st["status"] == 0, st
            ref = epic_ref.interp(scs[i].cost, scs[i].matches, scs[i].K, scs[i].a, scs[i].mode)[0]
            e = _epe(flows[i].cpu().numpy(), ref).mean()
            print(f"pair {i} {scs[i].name}: mean EPE {e:.2e}", flush=True)
            assert e <= parity.EPE_MEAN
        # (after the batch's stats: a single call becomes the context's last call)
        for i in range(0, 64, 8):
            alone = c.interp(*probs[i]).cpu().numpy()
            assert np.array_equal(alone, flows[i].cpu().numpy()), i
