"""The seeded scene generator: determinism and the shape of what it renders."""
import numpy as np
import pytest

from paper_1807_02044_amd import scenes


@pytest.mark.parametrize("key", ["tiny", "mid"])
def test_deterministic_and_in_range(key):
    wl = scenes.workload(key)
    a = scenes.make_pair(wl)
    b = scenes.make_pair(wl)
    assert a.left.dtype == np.uint8 and a.left.shape == (wl.height, wl.width)
    np.testing.assert_array_equal(a.left, b.left)
    np.testing.assert_array_equal(a.right, b.right)
    # visible surfaces sit strictly inside the search range
    assert a.gt_disp.min() >= wl.d_min + 1 and a.gt_disp.max() <= wl.d_max - 1
    assert 0.0 < a.occluded.mean() < 0.35
    c = scenes.make_pair(wl, seed=wl.seed + 1)
    assert not np.array_equal(a.left, c.left)


def test_tiny_scene_has_integer_fronto_planes():
    wl = scenes.workload("tiny")
    p = scenes.make_pair(wl)
    vals = np.unique(p.gt_disp)
    assert np.all(vals == np.round(vals)) and 1 <= vals.size <= 3
    assert vals.min() >= 2 and vals.max() <= 14


def test_mid_scene_slant_bound():
    wl = scenes.workload("mid")
    p = scenes.make_pair(wl)
    gx = np.abs(np.diff(p.gt_disp, axis=1))
    # inside planes the disparity gradient is at most 0.1 px/px
    assert np.median(gx) <= 0.1 + 1e-9


def test_warp_is_consistent_without_noise():
    wl = scenes.workload("tiny").with_(noise_sigma=0.0)
    p = scenes.make_pair(wl)
    H, W = p.left.shape
    ys, xs = np.nonzero(~p.occluded)
    u = xs - p.gt_disp[ys, xs].astype(int)
    np.testing.assert_array_equal(p.left[ys, xs], p.right[ys, u])


def test_fronto_pair_relation():
    L, R = scenes.textured_fronto_pair(30, 5, 4, seed=3)
    np.testing.assert_array_equal(R[:, :26], L[:, 4:])


def test_batched_mix():
    b = scenes.batched_workloads()
    assert len(b) == 64
    assert {w.n_disp for w in b} <= {32, 64, 96, 128}
    assert {w.radius for w in b} <= {5, 7, 10}
    assert len({(w.width, w.height) for w in b}) >= 4


# ------------------------------------------------ e_PEP of Eqs. 11-12 (sweeps)

def test_pep_hand_worked():
    from paper_1807_02044_amd import sweeps
    est = np.array([[1.0, 5.0], [3.0, -1.0]])
    gt = np.array([[1.0, 2.0], [0.5, 3.0]])
    # |1-1|=0 ok; |5-2|=3 > 2 error; |3-0.5|=2.5 error; -1 = no estimate, error
    assert sweeps.pep(est, gt, np.ones((2, 2), bool)) == 75.0
    # only the first row: one error of two
    assert sweeps.pep(est, gt, np.array([[1, 1], [0, 0]], bool)) == 50.0
    # delta is 0 at exactly eps_d (Eq. 12: d <= eps_d)
    assert sweeps.pep(np.array([4.0]), np.array([2.0]), np.array([True])) == 0.0
    assert sweeps.pep(np.array([4.0 + 1e-9]), np.array([2.0]), np.array([True])) == 100.0
    assert sweeps.pep(est, gt, np.zeros((2, 2), bool)) == 0.0


def test_region_masks_hand_worked():
    from paper_1807_02044_amd import sweeps
    flat = np.full((6, 8), 77, dtype=np.uint8)
    assert sweeps.textureless(flat).all()
    ramp = np.tile((np.arange(8) * 10).astype(np.uint8), (6, 1))  # gradient 10 per px
    tl = sweeps.textureless(ramp)
    assert not tl[:, 2:-2].any()
    gt = np.zeros((5, 12))
    gt[:, 6:] = 10.0                     # a jump between columns 5 and 6
    m = sweeps.discontinuities(gt)
    # columns 5 and 6 touch the jump; 2 px either side are inside the band
    assert m[:, 3:9].all() and not m[:, :3].any() and not m[:, 9:].any()
    small = gt.copy()
    small[:, 6:] = 2.0                   # a jump of exactly 2 is not a discontinuity
    assert not sweeps.discontinuities(small).any()
