"""GPU: the cost map from the image gradient (Table 2, norm-of-gradient
contour row) against the oracle, its batched launches, and the
interpolation from an image."""
from __future__ import annotations

import numpy as np
import pytest

import parity
from oracle import epic_ref
from scenes import batch_scenes, config_scene

pytestmark = pytest.mark.gpu

# FP32 arithmetic with one rounding per operation: the difference of two
# floats is rounded relative to itself, then halved (exact), squared, summed
# over 2*ch terms and square-rooted -- at most ~(4 + 4 ch) * 2^-24 relative
# to the gradient norm, below 1e-6 for ch <= 4; eps is added last.
RTOL = 1e-6


def _rand_image(rng, H, W, ch):
    img = rng.uniform(0, 1, (H, W, ch)).astype(np.float32)
    # smooth regions and sharp edges, as images have
    img[: H // 2] = img[: H // 2].mean()
    return img[:, :, 0] if ch == 1 and rng.integers(0, 2) else img


@pytest.mark.parametrize("H,W,ch", [(1, 1, 3), (1, 300, 1), (300, 1, 2), (17, 257, 3), (250, 513, 4),
                                    (16, 256, 3), (33, 1000, 1), (436, 1024, 3)])
def test_cost_matches_oracle(H, W, ch):
    import torch
    import paper_1501_02565_amd as epic
    rng = np.random.default_rng(H * 7 + W + ch)
    img = _rand_image(rng, H, W, ch)
    print(f"[case] image {img.shape}", flush=True)
    got = epic.image_cost(torch.from_numpy(img).cuda(), eps=1e-3).cpu().numpy()
    ref = epic_ref.grad_norm_cost(img, 1e-3)
    np.testing.assert_allclose(got, ref, rtol=RTOL, atol=0)


def test_batched_launches_equal_single_calls():
    """40 images with mixed channel counts (several launches) give each
    image what it gets alone, bitwise."""
    import torch
    import paper_1501_02565_amd as epic
    rng = np.random.default_rng(5)
    imgs = [torch.from_numpy(_rand_image(rng, int(rng.integers(1, 90)), int(rng.integers(1, 600)),
                                         [1, 3, 3, 4][i % 4])).cuda() for i in range(40)]
    print("[case] 40 mixed images", flush=True)
    many = [c.cpu().numpy() for c in epic.image_cost(imgs)]
    for im, c in zip(imgs, many):
        assert np.array_equal(epic.image_cost(im).cpu().numpy(), c)


def test_full_size_batch_images():
    """The images of the 64-pair batch (the bench's workload), every pixel
    against the oracle."""
    import torch
    import paper_1501_02565_amd as epic
    scs = batch_scenes(64, with_image=True)
    print(f"[case] 64 batch images, {sum(s.H * s.W for s in scs) / 1e6:.1f} Mpx", flush=True)
    costs = epic.image_cost([torch.from_numpy(s.image).cuda() for s in scs])
    for s, c in zip(scs, costs):
        np.testing.assert_allclose(c.cpu().numpy(), epic_ref.grad_norm_cost(s.image), rtol=RTOL, atol=0)


def test_interp_from_image():
    """interp_image equals the image cost followed by interp, bitwise, and
    matches the oracle run on the oracle's own gradient cost."""
    import torch
    import paper_1501_02565_amd as epic
    sc = config_scene(2, with_image=True)
    print(f"[case] {sc.name} from its image", flush=True)
    img = torch.from_numpy(sc.image).cuda()
    m = torch.from_numpy(sc.matches).cuda()
    ws = epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K) + 4 * sc.H * sc.W + 512
    with epic.Context(0, ws) as c:
        f1 = c.interp_image(img, m, sc.K, sc.a, sc.mode).cpu().numpy()
        cost = epic.image_cost(img)
        f2 = c.interp(cost, m, sc.K, sc.a, sc.mode).cpu().numpy()
        st = c.stats(0)
    assert np.array_equal(f1, f2) and st["status"] == 0
    ref_cost = epic_ref.grad_norm_cost(sc.image)
    ref = epic_ref.interp(ref_cost.astype(np.float32), sc.matches, sc.K, sc.a, sc.mode)[0]
    epe = np.linalg.norm(f1.astype(np.float64) - ref, axis=2)
    print(f"mean EPE {epe.mean():.2e}, max {epe.max():.2e}", flush=True)
    assert epe.mean() <= parity.EPE_MEAN
    # too small a workspace is refused before anything runs
    with epic.Context(0, epic.workspace_bytes(sc.H, sc.W, sc.N, sc.K)) as c:
        with pytest.raises(epic.EpicError) as ei:
            c.interp_image(img, m, sc.K, sc.a, sc.mode)
        assert ei.value.status == epic.ERR_WORKSPACE
