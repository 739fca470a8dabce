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
