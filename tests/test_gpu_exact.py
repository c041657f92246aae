"""GPU: the exact per-pixel geodesic interpolation (Table 2, "Geodesic
(exact)") against the oracle's own per-pixel definition."""
from __future__ import annotations

import numpy as np
import pytest

import parity
from oracle import epic_ref
from scenes import config_scene, random_case

pytestmark = pytest.mark.gpu

@pytest.mark.parametrize("case", ["config1", "random_la", "random_nw", "k1", "k128", "seed_on_border_a",
                                  "seed_on_border_b", "dense_k2"])
def test_exact_matches_oracle(case):
    """Mean EPE within the tolerance; every pixel within MAX_EPE except
    where the oracle's K-th and (K+1)-th distances are a near-tie (FP32
    distances against FP64 may then swap the K-th neighbour)."""
    import torch
    import paper_1501_02565_amd as epic
    sc = {"config1": lambda: config_scene(1),
          "random_la": lambda: random_case(45, 70, 60, seed=81, K=9, outside=3, duplicates=4),
          "random_nw": lambda: random_case(33, 90, 80, seed=82, K=16, mode=0),
          "k1": lambda: random_case(40, 50, 30, seed=83, K=1),
          # the largest K: the selection's LDS lists exceed 64 KB
          "k128": lambda: random_case(30, 40, 200, seed=86, K=128),
          # dense matches and small K (tight bounds): sources seeded on a
          # tile's border must still reach the tile behind it
          "seed_on_border_a": lambda: random_case(60, 46, 249, seed=993076779, K=1, mode=0),
          "seed_on_border_b": lambda: random_case(8, 66, 154, seed=512832132, K=1, mode=0, outside=2),
          "dense_k2": lambda: random_case(19, 51, 270, seed=177738499, K=2, mode=0)}[case]()
    print(f"[case] exact {sc.name} K={sc.K} mode={sc.mode}", flush=True)
    with epic.Context(0, 256 << 20) as c:
        f = c.interp_exact(torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda(),
                           sc.K, sc.a, sc.mode).cpu().numpy()
    rf, ri, rd, rc = epic_ref.exact(sc.cost, sc.matches, sc.K, sc.a, sc.mode)
    assert rc == 0
    epe = np.linalg.norm(f.reshape(-1, 2).astype(np.float64) - rf, axis=1)
    assert np.isfinite(epe).all()
    used = int((epic_ref.seeds(sc.H, sc.W, sc.matches)[0] >= 0).sum())
    Kc = min(sc.K, used)
    tie = np.zeros(len(rf), bool)
    if Kc < used:
        d2 = epic_ref.exact(sc.cost, sc.matches, Kc + 1, sc.a, sc.mode)[2]
        tie = np.abs(d2[:, Kc] - d2[:, Kc - 1]) <= 1e-4 * d2[:, Kc - 1]
    print(f"mean EPE {epe.mean():.2e}, max {epe.max():.2e}, max away from ties "
          f"{epe[~tie].max():.2e}, {int(tie.sum())} tie pixels", flush=True)
    assert epe.mean() <= parity.EPE_MEAN
    assert epe[~tie].max() <= parity.MAX_EPE


def test_exact_k1_equals_approximation():
    """K = 1: the nearest match is the Voronoi label, so the exact path and
    epic_interp agree (to the rounding of k u / k)."""
    import torch
    import paper_1501_02565_amd as epic
    sc = random_case(60, 80, 70, seed=84, K=1)
    with epic.Context(0, 256 << 20) as c:
        cost, m = torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda()
        fe = c.interp_exact(cost, m, 1, 1.0, 1).cpu().numpy()
        fa = c.interp(cost, m, 1, 1.0, 1).cpu().numpy()
    np.testing.assert_allclose(fe, fa, rtol=1e-6, atol=1e-6)


def test_exact_in_chunks_equals_one_chunk():
    """A workspace that holds only a few single-source transforms at a time
    gives bitwise the result of one chunk."""
    import torch
    import paper_1501_02565_amd as epic
    sc = random_case(50, 64, 90, seed=85, K=12)
    cost, m = torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda()
    HW = sc.H * sc.W
    # the lists, bounds, approximated lists and boxes at the workspace's end, the
    # approximated pass, then room for about 20 single-source transforms at
    # a time (a pair's bytes: a one-match workspace less the fixed head,
    # which is what a 1 x 1 workspace nearly is)
    tail = 8 * sc.K * HW + 4 * HW + sc.N + 8 * sc.N * sc.K + (36 << 10)
    per = epic.workspace_bytes(sc.H, sc.W, 1, 1) - epic.workspace_bytes(1, 1, 1, 1) + 4096
    small = max(epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K), epic.workspace_bytes(1, 1, 1, 1) + 20 * per) + tail
    assert 20 * per < sc.N * per                       # several chunks
    outs = []
    for ws in (256 << 20, small):
        with epic.Context(0, ws) as c:
            outs.append(c.interp_exact(cost, m, sc.K, sc.a, sc.mode).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_exact_full_size_sampled():
    """The 1024 x 436 scene (8000 matches, K = 100) in the configuration the
    benchmark times (chunks of 1024 single-source transforms): sampled
    pixels -- a spread over the image, its corners and random ones --
    against the oracle's per-pixel definition, to the bar of the other
    cases (near-ties of the K-th neighbour excused)."""
    import torch
    import paper_1501_02565_amd as epic
    sc = config_scene(2)
    HW = sc.H * sc.W
    rng = np.random.default_rng(87)
    pix = np.unique(np.concatenate([np.linspace(0, HW - 1, 40).astype(np.int64),
                                    [0, sc.W - 1, HW - sc.W, HW - 1], rng.integers(0, HW, 20)]))
    print(f"[case] exact full size {sc.name}, {len(pix)} sampled pixels", flush=True)
    ws = 8 * sc.K * HW + 4 * HW + sc.N + 8 * sc.N * sc.K + 1024 * epic.workspace_bytes(sc.H, sc.W, 1, 1) \
        + (64 << 20)
    with epic.Context(0, ws) as c:
        f = c.interp_exact(torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda(),
                           sc.K, sc.a, sc.mode).cpu().numpy().reshape(-1, 2).astype(np.float64)
    rf = epic_ref.exact(sc.cost, sc.matches, sc.K, sc.a, sc.mode, pixels=pix)[0]
    d2 = epic_ref.exact(sc.cost, sc.matches, sc.K + 1, sc.a, sc.mode, pixels=pix)[2]
    tie = np.abs(d2[:, sc.K] - d2[:, sc.K - 1]) <= 1e-4 * d2[:, sc.K - 1]
    epe = np.linalg.norm(f[pix] - rf, axis=1)
    print(f"mean EPE {epe.mean():.2e}, max {epe.max():.2e}, {int(tie.sum())} tie pixels", flush=True)
    assert np.isfinite(f).all()
    assert epe.mean() <= parity.EPE_MEAN
    assert epe[~tie].max() <= parity.MAX_EPE
