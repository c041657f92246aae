"""GPU: the debug_validate option.  A context created with it checks every
cost map on the device (finite and > 0).  A valid map gives exactly the
result of a context without the check; a map with bad values reports
ERR_COST with their count and a NaN flow, leaves the other pairs of a batch
untouched, and leaves the context usable.  Needs an MI355X."""
from __future__ import annotations

import numpy as np
import pytest

from scenes import random_case

pytestmark = pytest.mark.gpu


def _announce(name):
    print(f"\n[case] {name}", flush=True)


def _dev(sc):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(sc.cost)).cuda(),
            torch.from_numpy(np.ascontiguousarray(sc.matches)).cuda())


def _spoil(cost):
    """A copy of `cost` with a zero, a negative, a NaN and both infinities."""
    bad = cost.copy()
    H, W = bad.shape
    spots = [(0, 0), (H // 2, W // 3), (H - 1, W - 1), (1, W - 2), (H // 3, 1)]
    for (y, x), v in zip(spots, [0.0, -0.25, np.nan, np.inf, -np.inf]):
        bad[y, x] = v
    return bad, len(set(spots))


@pytest.mark.parametrize("precision", [0, 1])
def test_validation_flags_bad_costs(precision):
    import torch
    import paper_1501_02565_amd as epic
    sc = random_case(70, 90, 60, seed=41, K=8)
    bad_np, n_bad = _spoil(sc.cost)
    cost, matches = _dev(sc)
    bad = torch.from_numpy(bad_np).cuda()
    with epic.Context(0, precision=precision) as plain, \
            epic.Context(0, precision=precision, debug_validate=True) as chk:
        _announce(f"{sc.name} precision={precision} valid cost")
        ref = plain.interp(cost, matches, K=8, a=1.0, mode=epic.LA).cpu().numpy()
        out = chk.interp(cost, matches, K=8, a=1.0, mode=epic.LA).cpu().numpy()
        st = chk.stats(0)
        assert st["status"] == 0 and st["n_bad_cost"] == 0, st
        np.testing.assert_array_equal(out, ref)

        _announce(f"{sc.name} precision={precision} {n_bad} bad cost values")
        out = chk.interp(bad, matches, K=8, a=1.0, mode=epic.LA).cpu().numpy()
        st = chk.stats(0)
        print(st, flush=True)
        assert st["status"] == epic.ERR_COST and st["n_bad_cost"] == n_bad, st
        assert st["n_used"] == 0 and st["n_outside"] == 0 and st["n_duplicate"] == 0, st
        assert np.isnan(out).all()

        _announce(f"{sc.name} precision={precision} valid cost after a rejected one")
        out = chk.interp(cost, matches, K=8, a=1.0, mode=epic.LA).cpu().numpy()
        assert chk.stats(0)["status"] == 0
        np.testing.assert_array_equal(out, ref)


def test_validation_in_a_batch():
    """One pair of a batch with a bad map: only that pair is rejected."""
    import torch
    import paper_1501_02565_amd as epic
    scs = [random_case(40 + 9 * i, 50 + 13 * i, 30 + 10 * i, seed=50 + i, K=6) for i in range(3)]
    bad_np, n_bad = _spoil(scs[1].cost)
    probs = []
    for i, sc in enumerate(scs):
        cost, matches = _dev(sc)
        if i == 1:
            cost = torch.from_numpy(bad_np).cuda()
        probs.append((cost, matches, 6, 1.0, epic.LA))
    _announce("batch of 3, pair 1 with bad cost values")
    with epic.Context(0) as plain, epic.Context(0, debug_validate=True) as chk:
        flows = [f.cpu().numpy() for f in chk.interp_batch(probs)]
        stats = [chk.stats(i) for i in range(3)]
        print(stats, flush=True)
        assert stats[1]["status"] == epic.ERR_COST and stats[1]["n_bad_cost"] == n_bad
        assert np.isnan(flows[1]).all()
        for i in (0, 2):
            assert stats[i]["status"] == 0 and stats[i]["n_bad_cost"] == 0, stats[i]
            cost, matches, K, a, mode = probs[i]
            ref = plain.interp(cost, matches, K=K, a=a, mode=mode).cpu().numpy()
            np.testing.assert_array_equal(flows[i], ref)


def test_knn_table_overflow_is_reported():
    """A match whose cell touches more than the largest K-NN table holds
    (a cheap row shared by one match, 2 x 2200 matches along it): every
    search reaches it and overflows.  The pair reports EPIC_ERR_CAPACITY
    instead of a silently zero model."""
    import torch
    import paper_1501_02565_amd as epic
    H, W = 3, 2200
    cost = np.ones((H, W), np.float32)
    cost[1, :] = 1e-4
    m = np.zeros((2 * W + 1, 4), np.float32)
    m[0, :2] = (0, 1)                               # the hub: all of row 1 is its cell
    m[1:W + 1, 0], m[1:W + 1, 1] = np.arange(W), 0
    m[W + 1:, 0], m[W + 1:, 1] = np.arange(W), 2
    m[:, 2:] = m[:, :2] + 1.0
    print(f"[case] hub {H}x{W}, {len(m)} matches, K=100", flush=True)
    with epic.Context(0, epic.workspace_bytes(H, W, len(m), 100)) as c:
        flow = c.interp(torch.from_numpy(cost).cuda(), torch.from_numpy(m).cuda(), 100, 1.0, 1)
        st = c.stats(0)
    print(st, flush=True)
    assert st["status"] == epic.ERR_CAPACITY
    assert np.isfinite(flow.cpu().numpy()).all()


@pytest.mark.parametrize("precision,conn", [(0, 8), (0, 4), (1, 8)])
def test_invariants_hold_and_change_nothing(precision, conn):
    """With debug_validate the device checks the transform's fixpoint, the
    seeds, the labels and the graph's symmetry: none is violated on scenes
    with sub-pixel, outside and shared matches, a batch and the consistency
    check, and the flow is bitwise that of a context without the checks."""
    import torch
    import paper_1501_02565_amd as epic
    from scenes import config_scene
    cases = [random_case(70, 90, 140, seed=9, K=20, outside=4, duplicates=5),
             random_case(33, 257, 300, seed=12, K=8), config_scene(1)]
    kw = dict(precision=precision, connectivity=conn)
    with epic.Context(0, **kw) as plain, epic.Context(0, debug_validate=1, **kw) as chk:
        for sc in cases:
            _announce(f"{sc.name} precision={precision} conn={conn}")
            cost, matches = _dev(sc)
            ref = plain.interp(cost, matches, sc.K, sc.a, sc.mode).cpu().numpy()
            out = chk.interp(cost, matches, sc.K, sc.a, sc.mode).cpu().numpy()
            st = chk.stats(0)
            assert st["status"] == 0 and st["n_invariant"] == 0, st
            np.testing.assert_array_equal(out, ref)
        _announce(f"batch of 3 precision={precision} conn={conn}")
        probs = [(*_dev(sc), sc.K, sc.a, sc.mode) for sc in cases]
        flows = [f.cpu().numpy() for f in chk.interp_batch(probs)]
        for i, (cost, matches, K, a, mode) in enumerate(probs):
            assert chk.stats(i)["n_invariant"] == 0, chk.stats(i)
            np.testing.assert_array_equal(flows[i], plain.interp(cost, matches, K, a, mode).cpu().numpy())
    with epic.Context(0, debug_validate=1, prune_px=5.0, **kw) as chk:
        sc = cases[0]
        _announce(f"{sc.name} with the consistency check precision={precision}")
        cost, matches = _dev(sc)
        chk.interp(cost, matches, sc.K, sc.a, sc.mode)
        st = chk.stats(0)
        assert st["status"] == 0 and st["n_invariant"] == 0, st


@pytest.mark.parametrize("precision", [0, 1])
def test_planted_violation_is_reported(precision):
    """debug_validate = 2 raises pixel 0's distance before the checks (a
    planted violation of the fixpoint): the pair reports ERR_INVARIANT."""
    import paper_1501_02565_amd as epic
    sc = random_case(70, 90, 140, seed=9, K=20)
    cost, matches = _dev(sc)
    _announce(f"{sc.name} planted violation precision={precision}")
    with epic.Context(0, precision=precision, debug_validate=2) as chk:
        chk.interp(cost, matches, sc.K, sc.a, sc.mode)
        st = chk.stats(0)
    print(st, flush=True)
    assert st["status"] == epic.ERR_INVARIANT and st["n_invariant"] >= 1, st


def test_pass_visits_are_counted_while_profiling():
    """epic_pass_visits: the first pass visits every tile, the counts add up
    to the call's tile visits, and nothing is counted without profiling."""
    import paper_1501_02565_amd as epic
    from scenes import config_scene
    sc = config_scene(1)
    cost, matches = _dev(sc)
    _announce(f"{sc.name} pass visits")
    with epic.Context(0) as ctx:
        ctx.interp(cost, matches, sc.K, sc.a, sc.mode)
        assert ctx.pass_visits() == []
        ctx.profile(True)
        ctx.interp(cost, matches, sc.K, sc.a, sc.mode)
        v = ctx.pass_visits()
        st = ctx.stats(0)
        ctx.profile(False)
    tiles = -(-sc.W // 32) * -(-sc.H // 16)
    print(v, st["tile_visits"], tiles, flush=True)
    assert v[0] == tiles and sum(v) == st["tile_visits"] and all(x > 0 for x in v)
