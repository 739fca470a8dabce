"""Both views and the left-right check (Sections II-A, II-C, II-D, Eq. 9)
through the C ABI, against the FP64 oracle.

* fbs_cost_lr (dual storage): both volumes equal the oracle's left and right
  volumes (TAD bit for bit, NCC within the cost test's 2e-6).
* right maps (staged: fbs_cost_lr -> fbs_aggregate with the right image ->
  fbs_wta_subpixel; fused: fbs_run_lr) follow the parity rules of
  tests/parity.py against oracle.fbs_right.
* the check itself is integer work: the GPU mask equals Eq. 9 evaluated in
  numpy on the GPU's own maps, bit for bit, and equals the oracle's mask on
  every pixel whose left disparity and right partner disparity agree with
  the oracle's (the others follow accepted 1e-5 ties and are counted).
* the refined map equals fbs_run's subpixel map where the check holds and is
  -1 where it fails.
"""
import sys
import zlib

import numpy as np
import pytest

import oracle
from oracle import NCC, TAD, Problem
from paper_1807_02044_amd import _lib as L
from paper_1807_02044_amd import scenes
import paper_1807_02044_amd as fbs

from parity import Report, compare_maps, weight_floor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _h(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(left, pb: Problem, flags=0):
    H, W = left.shape[:2]
    C = 1 if left.ndim == 2 else left.shape[2]
    return L.make_params(W, H, C, pb.d_min, pb.d_max, pb.radius, pb.gamma_d, pb.gamma_r,
                         pb.tau, pb.cost_type, pb.ncc_radius, flags)


def _floor(pb: Problem) -> float:
    return weight_floor((2 * pb.radius + 1) ** 2, pb.tau if pb.cost_type == TAD else 2.0)


def _lrc_numpy(dl, dr, max_diff):
    """Eq. 9 written out on integer maps (independent of both libraries)."""
    H, W = dl.shape
    valid = np.zeros((H, W), dtype=np.uint8)
    for y in range(H):
        for x in range(W):
            u = x - int(dl[y, x])
            if 0 <= u < W and abs(int(dr[y, u]) - int(dl[y, x])) <= max_diff:
                valid[y, x] = 1
    return valid


def _check_lr(pb, Lh, Rh, dl, dr, valid, sub, sub_ref, max_diff):
    """Full-frame comparison of one left-right result with the oracle."""
    do, so, ao = oracle.fbs(pb, Lh, Rh, want_agg=True)
    dro, sro, aro = oracle.fbs_right(pb, Lh, Rh, want_agg=True)
    fl = _floor(pb)
    rep_l = compare_maps(dl, sub_ref, do, so, ao.reshape(ao.shape[0], -1), pb.d_min, floor=fl)
    rep_r = compare_maps(dr, dr.astype(np.float64), dro, dro.astype(np.float64),
                         aro.reshape(aro.shape[0], -1), pb.d_min, floor=fl)
    _say("left", rep_l)
    _say("right", rep_r)
    assert rep_l.ok, f"left map: {rep_l}"
    assert rep_r.ok, f"right map: {rep_r}"
    # Eq. 9 on the GPU's own maps: exact
    np.testing.assert_array_equal(valid, _lrc_numpy(dl, dr, max_diff))
    # against the oracle's check, wherever the inputs of the check agree
    vo = oracle.lrc(pb, do, dro, max_diff)
    H, W = dl.shape
    xs = np.arange(W)[None, :].repeat(H, 0)
    u = xs - dl
    inside = (u >= 0) & (u < W)
    uc = np.clip(u, 0, W - 1)
    same_inputs = (dl == do) & (~inside | (np.take_along_axis(dr, uc, 1) ==
                                            np.take_along_axis(dro, uc, 1)))
    mism = (valid != vo) & same_inputs
    assert not mism.any(), f"{int(mism.sum())} check results differ with equal inputs"
    _say(f"lrc: valid={int(valid.sum())}/{valid.size} oracle={int(vo.sum())} "
         f"pixels following a tie={int((~same_inputs).sum())}")
    # refined map: Eq. 10 where the check holds, -1 where it fails
    np.testing.assert_array_equal(sub[valid == 1].view(np.uint32),
                                  sub_ref[valid == 1].view(np.uint32))
    assert np.all(sub[valid == 0] == -1.0)


def _tiny(channels=1):
    wl = scenes.workload("tiny")
    if channels == 3:
        wl = wl.with_(channels=3)
    pr = scenes.make_pair(wl)
    return wl, pr.left, pr.right


# ------------------------------------------------------------- dual storage


@pytest.mark.parametrize("channels,d_min", [(1, 0), (3, 0), (1, 4), (3, 2)])
def test_cost_lr_dual_storage_bit_exact(channels, d_min):
    wl, Lh, Rh = _tiny(channels)
    pb = Problem(d_min, 15, wl.radius, wl.sigma_s, wl.sigma_r, wl.cost_cap)
    _say("cost_lr", channels, d_min)
    p = _params(Lh, pb)
    cl, cr = fbs.cost_lr(p, _d(Lh), _d(Rh))
    cl, cr = _h(cl), _h(cr)
    np.testing.assert_array_equal(cl, oracle.cost(pb, Lh, Rh).astype(np.float32))
    np.testing.assert_array_equal(cr, oracle.cost_right(pb, Lh, Rh).astype(np.float32))
    # the plain cost step writes the same left volume
    np.testing.assert_array_equal(_h(fbs.cost(p, _d(Lh), _d(Rh))), cl)


def test_cost_lr_ncc():
    wl, Lh, Rh = _tiny(1)
    pb = Problem(1, 15, wl.radius, wl.sigma_s, wl.sigma_r, cost_type=NCC, ncc_radius=1)
    p = _params(Lh, pb)
    _say("cost_lr ncc")
    cl, cr = fbs.cost_lr(p, _d(Lh), _d(Rh))
    np.testing.assert_allclose(_h(cl), oracle.cost(pb, Lh, Rh), rtol=0, atol=2e-6)
    np.testing.assert_allclose(_h(cr), oracle.cost_right(pb, Lh, Rh), rtol=0, atol=2e-6)


# ---------------------------------------------------------- staged pipeline


@pytest.mark.parametrize("channels,ct", [(1, TAD), (3, TAD), (1, NCC)])
def test_staged_lr_pipeline(channels, ct):
    """Paper's staged path: dual storage, both aggregations, both WTAs, Eq. 9."""
    wl, Lh, Rh = _tiny(channels)
    pb = Problem.from_workload(wl, cost_type=ct)
    p = _params(Lh, pb)
    _say("staged lr", channels, ct)
    Ld, Rd = _d(Lh), _d(Rh)
    cl, cr = fbs.cost_lr(p, Ld, Rd)
    al = fbs.aggregate(p, Ld, cl)
    ar = fbs.aggregate(p, Rd, cr)
    dl, sl = fbs.wta_subpixel(p, al)
    dr, _ = fbs.wta_subpixel(p, ar)
    sub = sl.clone()
    valid = fbs.lrc(p, dl, dr, 0, disp_sub=sub)
    _check_lr(pb, Lh, Rh, _h(dl), _h(dr), _h(valid), _h(sub), _h(sl), 0)


# ------------------------------------------------------------ fused path


FUSED = {
    "tiny_gray": (1, TAD, 0, 0),
    "tiny_rgb": (3, TAD, 0, 0),
    "tiny_gray_ncc": (1, NCC, 0, 0),
    "tiny_gray_valu": (1, TAD, L.FBS_F_FORCE_VALU, 0),
    "tiny_gray_maxdiff1": (1, TAD, 0, 1),
}


@pytest.mark.parametrize("name", list(FUSED))
def test_run_lr_tiny_vs_oracle(name):
    channels, ct, flags, max_diff = FUSED[name]
    wl, Lh, Rh = _tiny(channels)
    pb = Problem.from_workload(wl, cost_type=ct)
    p = _params(Lh, pb, flags)
    _say("run_lr", name, "variant", L.fbs_run_variant(p))
    Ld, Rd = _d(Lh), _d(Rh)
    dl, dr, valid, sub = fbs.run_lr(p, Ld, Rd, max_diff)
    _, s_ref = fbs.run(p, Ld, Rd)
    _check_lr(pb, Lh, Rh, _h(dl), _h(dr), _h(valid), _h(sub), _h(s_ref), max_diff)


def test_run_lr_mid_full_frame_vs_oracle():
    wl = scenes.workload("mid")
    pr = scenes.make_pair(wl)
    pb = Problem.from_workload(wl)
    p = _params(pr.left, pb)
    _say("run_lr mid", wl.name)
    Ld, Rd = _d(pr.left), _d(pr.right)
    dl, dr, valid, sub = fbs.run_lr(p, Ld, Rd, 0)
    d_ref, s_ref = fbs.run(p, Ld, Rd)
    np.testing.assert_array_equal(_h(dl), _h(d_ref))
    _check_lr(pb, pr.left, pr.right, _h(dl), _h(dr), _h(valid), _h(sub), _h(s_ref), 0)
    # the check removes the half-occluded pixels of the synthetic scene (a
    # sanity trend of Section II-D, not parity): most removed pixels are
    # occluded or within a pixel of a depth edge
    v = _h(valid).astype(bool)
    assert pr.occluded[~v].mean() > pr.occluded[v].mean()


def test_run_lr_large_rgb_sampled():
    wl = scenes.workload("large")
    pr = scenes.make_pair(wl)
    pb = Problem.from_workload(wl)
    p = _params(pr.left, pb)
    _say("run_lr large", wl.name)
    dl, dr, valid, sub = fbs.run_lr(p, _d(pr.left), _d(pr.right), 0)
    dl, dr, valid, sub = _h(dl), _h(dr), _h(valid), _h(sub)
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.integers(0, wl.width, 600), [0, 1, wl.width - 2, wl.width - 1]])
    ys = np.concatenate([rng.integers(0, wl.height, 600), [0, wl.height - 1, 1, wl.height - 2]])
    xs, ys = xs.astype(np.int32), ys.astype(np.int32)
    aro, dro, sro = oracle.fbs_right_pixels(pb, pr.left, pr.right, xs, ys)
    rep = compare_maps(dr[ys, xs], dr[ys, xs].astype(np.float64), dro, dro.astype(np.float64),
                       aro.T, pb.d_min, floor=_floor(pb))
    _say("right sampled", rep)
    assert rep.ok, str(rep)
    np.testing.assert_array_equal(valid, _lrc_numpy_fast(dl, dr, 0))
    assert np.all(sub[valid == 0] == -1.0)


def _lrc_numpy_fast(dl, dr, max_diff):
    H, W = dl.shape
    xs = np.arange(W)[None, :].repeat(H, 0)
    u = xs - dl
    inside = (u >= 0) & (u < W)
    partner = np.take_along_axis(dr, np.clip(u, 0, W - 1), 1)
    return (inside & (np.abs(partner - dl) <= max_diff)).astype(np.uint8)


EDGE = {
    "ragged_37x23": dict(W=37, H=23, C=1, dmin=2, dmax=6, r=3),
    "one_disparity": dict(W=30, H=20, C=1, dmin=4, dmax=4, r=2),
    "full_width_range": dict(W=12, H=9, C=1, dmin=0, dmax=11, r=2),
    "radius0": dict(W=33, H=17, C=1, dmin=0, dmax=9, r=0),
    "rgb_ragged": dict(W=41, H=19, C=3, dmin=1, dmax=9, r=2),
    "two_pixels": dict(W=2, H=1, C=1, dmin=0, dmax=1, r=1),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_run_lr_edge_cases(name):
    e = EDGE[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 1000)
    shape = (e["H"], e["W"]) if e["C"] == 1 else (e["H"], e["W"], 3)
    Lh = rng.integers(0, 256, shape, dtype=np.uint8)
    Rh = np.roll(Lh, -min(3, e["W"] - 1), axis=1)
    Rh = np.clip(Rh.astype(int) + rng.integers(-6, 7, shape), 0, 255).astype(np.uint8)
    pb = Problem(e["dmin"], e["dmax"], e["r"], 3.0, 9.0, 40.0)
    for flags in (0, L.FBS_F_FORCE_VALU):
        p = _params(Lh, pb, flags)
        _say("run_lr edge", name, "flags", flags)
        Ld, Rd = _d(Lh), _d(Rh)
        dl, dr, valid, sub = fbs.run_lr(p, Ld, Rd, 0)
        _, s_ref = fbs.run(p, Ld, Rd)
        _check_lr(pb, Lh, Rh, _h(dl), _h(dr), _h(valid), _h(sub), _h(s_ref), 0)


def test_run_lr_partial_outputs_and_errors():
    wl, Lh, Rh = _tiny(1)
    pb = Problem.from_workload(wl)
    p = _params(Lh, pb)
    Ld, Rd = _d(Lh), _d(Rh)
    dl, dr, valid, sub = fbs.run_lr(p, Ld, Rd, 0)
    ws = torch.empty(L.fbs_lr_workspace_bytes(p), dtype=torch.uint8, device="cuda")
    only_valid = torch.zeros((wl.height, wl.width), dtype=torch.uint8, device="cuda")
    L.fbs_run_lr(p, Ld, Rd, 0, None, None, only_valid, None, ws)
    np.testing.assert_array_equal(_h(only_valid), _h(valid))
    only_right = torch.zeros((wl.height, wl.width), dtype=torch.int32, device="cuda")
    L.fbs_run_lr(p, Ld, Rd, 0, None, only_right, None, None, ws)
    np.testing.assert_array_equal(_h(only_right), _h(dr))
    with pytest.raises(L.FbsError) as e:
        L.fbs_run_lr(p, Ld, Rd, 0, dl, dr, valid, sub, None)
    assert e.value.status == L.FBS_E_WORKSPACE
    with pytest.raises(L.FbsError) as e:
        L.fbs_run_lr(p, Ld, Rd, -1, dl, dr, valid, sub, ws)
    assert e.value.status == L.FBS_E_INVALID
