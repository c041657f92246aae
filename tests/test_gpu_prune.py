"""GPU: the consistency check of the matches (Sec. 5.1, "Pruning of
matches") -- one NW interpolation, removal of the matches further than 5 px
from it at their own pixel, then the interpolation of the kept matches --
against the oracle, stage by stage."""
from __future__ import annotations

import numpy as np
import pytest

import parity
from oracle import epic_ref
from scenes import config_scene, random_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1501_02565_amd as epic
    c = epic.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_pruned():
    import paper_1501_02565_amd as epic
    c = epic.Context(0, prune_px=5.0)
    yield c
    c.close()


CASES = [lambda: config_scene(1), lambda: config_scene(2), lambda: config_scene(3, mode=0),
         lambda: random_case(90, 130, 260, seed=51, K=24, outside=5, duplicates=6),
         lambda: random_case(33, 200, 150, seed=52, K=8, mode=0)]


@pytest.mark.parametrize("i", range(len(CASES)))
def test_kept_set_matches_oracle(ctx, i):
    sc = CASES[i]()
    print(f"[case] {sc.name}", flush=True)
    kg, kr, near = parity.prune_check(ctx, sc, 5.0)
    print(f"kept {len(kg)} of {sc.N} (oracle {len(kr)}), {near} within 1e-3 px of the threshold", flush=True)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_pruned_interpolation_matches_oracle(ctx_pruned, i):
    sc = CASES[i]()
    print(f"[case] {sc.name} pruned", flush=True)
    print(parity.full_check_pruned(ctx_pruned, sc, 5.0), flush=True)


def test_everything_pruned_gives_nan(ctx):
    """A threshold no match meets leaves no match: NaN flow, NO_MATCHES."""
    import torch
    import paper_1501_02565_amd as epic
    sc = random_case(40, 60, 50, seed=53, K=8)
    sc.matches[:, 2:] = sc.matches[:, :2] + np.where(np.arange(50)[:, None] % 2 == 0, 40.0, -40.0)
    with epic.Context(0, prune_px=1e-3) as c:
        flow = c.interp(torch.from_numpy(sc.cost).cuda(), torch.from_numpy(sc.matches).cuda(), 8, 1.0, 1)
        st = c.stats(0)
    ref, rc, _, kept = epic_ref.interp_pruned(sc.cost, sc.matches, 8, 1.0, 1, 1e-3)
    print(st, len(kept), flush=True)
    assert len(kept) == 0 and rc == -3
    assert st["status"] == epic.ERR_NO_MATCHES and np.isnan(flow.cpu().numpy()).all()


def test_batch_with_pruning_equals_alone(ctx_pruned):
    """Each pair of a pruned batch is bitwise what it is alone."""
    import torch
    scs = [random_case(50 + 17 * i, 80 + 9 * i, 60 + 30 * i, seed=60 + i, K=[8, 16, 32][i % 3],
                       mode=i % 2, outside=i % 3) for i in range(10)]
    probs = [(torch.from_numpy(s.cost).cuda(), torch.from_numpy(s.matches).cuda(), s.K, s.a, s.mode)
             for s in scs]
    flows = [f.cpu().numpy() for f in ctx_pruned.interp_batch(probs)]
    stats = [ctx_pruned.stats(i) for i in range(len(scs))]
    for sc, p, f, st in zip(scs, probs, flows, stats):
        alone = ctx_pruned.interp(*p).cpu().numpy()
        st1 = ctx_pruned.stats(0)
        assert np.array_equal(alone, f, equal_nan=True)
        # every count but the transform's tile visits (which depend on the
        # schedule, not the result) is the same alone and in the batch
        assert {k: v for k, v in st.items() if k != "tile_visits"} == \
            {k: v for k, v in st1.items() if k != "tile_visits"}
        ref, rc, _, kept = epic_ref.interp_pruned(sc.cost, sc.matches, sc.K, sc.a, sc.mode, 5.0)
        assert st["n_used"] == len(kept)
        if rc == 0:
            assert np.linalg.norm(f.astype(np.float64) - ref, axis=2).mean() <= parity.EPE_MEAN
