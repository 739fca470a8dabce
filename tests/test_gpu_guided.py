"""Search ranges suggested by reliable pixels (Section V, future work)
through the C ABI, against the FP64 oracle.

* fbs_guided_ranges is integer work: equal to oracle.guided_ranges.
* fbs_run_ranged with whole ranges equals fbs_run bit for bit (same kernel,
  same arithmetic); with arbitrary ranges (narrow, empty, excluding the true
  match) it follows oracle.fbs_ranged under the parity rules.
* the guided pipeline (cheap left-right run -> seeds -> ranges -> ranged
  full run) is measured against the plain full run (bad-1px), a property of
  the method rather than parity.
"""
import numpy as np
import pytest

import oracle
from oracle import Problem
from paper_1807_02044_amd import _lib as L
from paper_1807_02044_amd import scenes
import paper_1807_02044_amd as fbs

from parity import compare_maps, weight_floor

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _h(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("halo,margin", [(0, 0), (7, 2), (20, 5)])
def test_guided_ranges_equal_oracle(halo, margin):
    wl = scenes.workload("mid")
    p = fbs.params_for(wl)
    rng = np.random.default_rng(halo * 10 + margin)
    disp = rng.integers(-3, 70, (wl.height, wl.width)).astype(np.int32)
    valid = (rng.random((wl.height, wl.width)) < 0.3).astype(np.uint8)
    valid[:40, :60] = 0                                   # tiles without seeds
    got = _h(fbs.guided_ranges(p, _d(disp), _d(valid), halo, margin))
    tw, th = L.fbs_range_tile(p)
    want = oracle.guided_ranges(Problem.from_workload(wl), disp, valid, tw, th, halo, margin)
    np.testing.assert_array_equal(got, want)


def _random_ranges(shape, pb, seed):
    rng = np.random.default_rng(seed)
    lo = rng.integers(pb.d_min, pb.d_max + 1, shape)
    width = rng.integers(0, 20, shape)
    rg = np.stack([lo, np.minimum(lo + width, pb.d_max)], axis=-1).astype(np.int32)
    rg[0, 0] = [pb.d_max, pb.d_min]                       # empty: the whole range
    rg[-1, -1] = [pb.d_min, pb.d_max]
    rg[0, -1] = [pb.d_min - 5, pb.d_max + 9]              # clipped
    return rg


@pytest.mark.parametrize("name", ["tiny", "mid", "tiny_rgb"])
def test_run_ranged_vs_oracle(name):
    wl = scenes.workload("tiny" if name.startswith("tiny") else name)
    if name == "tiny_rgb":
        wl = wl.with_(channels=3)
    pr = scenes.make_pair(wl)
    p = fbs.params_for(wl)
    pb = Problem.from_workload(wl)
    tw, th = L.fbs_range_tile(p)
    shape = ((wl.height + th - 1) // th, (wl.width + tw - 1) // tw)
    Ld, Rd = _d(pr.left), _d(pr.right)
    # whole ranges: fbs_run bit for bit
    full = np.zeros(shape + (2,), np.int32)
    full[..., 0], full[..., 1] = pb.d_min, pb.d_max
    d0, s0 = fbs.run(p, Ld, Rd)
    d1, s1 = fbs.run_ranged(p, Ld, Rd, _d(full))
    np.testing.assert_array_equal(_h(d1), _h(d0))
    np.testing.assert_array_equal(_h(s1).view(np.uint32), _h(s0).view(np.uint32))
    # arbitrary ranges against the oracle
    rg = _random_ranges(shape, pb, 3)
    d2, s2 = fbs.run_ranged(p, Ld, Rd, _d(rg))
    d2, s2 = _h(d2), _h(s2)
    rg_o = rg.copy()
    rg_o[..., 0] = np.maximum(rg_o[..., 0], pb.d_min)
    rg_o[..., 1] = np.minimum(rg_o[..., 1], pb.d_max)
    empty = rg_o[..., 0] > rg_o[..., 1]
    rg_o[empty] = [pb.d_min, pb.d_max]
    do, so = oracle.fbs_ranged(pb, pr.left, pr.right, tw, th, rg_o)
    _, _, ao = oracle.fbs(pb, pr.left, pr.right, want_agg=True)
    rep = compare_maps(d2, s2, do, so, ao.reshape(ao.shape[0], -1), pb.d_min,
                       floor=weight_floor((2 * pb.radius + 1) ** 2, pb.tau))
    print(name, rep, flush=True)
    assert rep.ok, str(rep)
    # every pixel's disparity lies in its tile's range
    ys, xs = np.mgrid[0:wl.height, 0:wl.width]
    lo = rg_o[ys // th, xs // tw, 0]
    hi = rg_o[ys // th, xs // tw, 1]
    assert np.all((d2 >= lo) & (d2 <= hi))


def test_guided_pipeline_against_plain_full_run():
    """Seeds from a cheap radius-3 left-right run, ranges with a halo of the
    full radius, then the full-radius run over the ranges only."""
    wl = scenes.Workload("g640", 640, 480, 1, 0, 95, 10, 10.0, 10.0, 40.0, scene="slanted",
                         seed=200005, n_planes=8)
    pr = scenes.make_pair(wl)
    pf = fbs.params_for(wl)
    pc = fbs.params_for(wl.with_(radius=3, sigma_s=3.0))
    Ld, Rd = _d(pr.left), _d(pr.right)
    dl, dr, valid, _ = fbs.run_lr(pc, Ld, Rd, 0)
    rg = fbs.guided_ranges(pf, dl, valid, 10, 3)
    dg, sg = fbs.run_ranged(pf, Ld, Rd, rg)
    dp, sp = fbs.run(pf, Ld, Rd)
    bad = float(((sg - sp).abs() > 1.0).float().mean().item())
    width = (rg[..., 1] - rg[..., 0] + 1).float().mean().item()
    print(f"guided: mean range {width:.1f} of {wl.n_disp}, bad-1px vs plain {bad:.4f}", flush=True)
    # a measurement of the method, not parity: the ranges narrow the search
    # and the result stays close to the full search (about 5 % of the pixels
    # differ by more than 1 px on these scenes)
    assert width < wl.n_disp / 2
    assert bad < 0.10
    # pixels whose full-search disparity lies inside their tile's range and
    # away from its ends get the full search's value (same costs, same WTA)
    tw, th = L.fbs_range_tile(pf)
    rg_h, dp_h, dg_h = _h(rg), _h(dp), _h(dg)
    ys, xs = np.mgrid[0:wl.height, 0:wl.width]
    lo = rg_h[ys // th, xs // tw, 0]
    hi = rg_h[ys // th, xs // tw, 1]
    inside = (dp_h > lo) & (dp_h < hi)
    np.testing.assert_array_equal(dg_h[inside], dp_h[inside])
