"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Rules (tests/parity.py): TAD cost bit-exact; aggregated costs within 1e-4
relative; integer disparities equal outside the oracle's 1e-5 tie zone;
subpixel within 1e-3 px outside flat parabolas.  Inputs are the seeded
synthetic scenes; sizes span several 16x16 tiles with ragged tails.
"""
import math
import sys
import zlib

import numpy as np
import pytest

import oracle
from oracle import NCC, TAD, Problem
from paper_1807_02044_amd import _lib as L
from paper_1807_02044_amd import scenes
import paper_1807_02044_amd as fbs

from parity import Report, compare_agg, compare_maps, weight_floor

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


def _params(left, pb: Problem, flags=0, row_stride=None):
    H, W = left.shape[:2]
    C = 1 if left.ndim == 2 else left.shape[2]
    return L.make_params(W, H, C, pb.d_min, pb.d_max, pb.radius, pb.gamma_d, pb.gamma_r,
                         pb.tau, pb.cost_type, pb.ncc_radius, flags, row_stride)


def _staged(p, Ld, Rd):
    c = fbs.cost(p, Ld, Rd)
    a = fbs.aggregate(p, Ld, c)
    d, s = fbs.wta_subpixel(p, a)
    return c, a, d, s


def _floor(pb: Problem) -> float:
    return weight_floor((2 * pb.radius + 1) ** 2, pb.tau if pb.cost_type == TAD else 2.0)


def _full_compare(pb, left, right, disp, sub, agg=None):
    do, so, ao = oracle.fbs(pb, left, right, want_agg=True)
    fl = _floor(pb)
    rep = compare_maps(disp, sub, do, so, ao.reshape(ao.shape[0], -1), pb.d_min, floor=fl)
    if agg is not None:
        compare_agg(agg, ao, rep, floor=fl)
    return rep


def _tiny(channels=1, seed=None):
    wl = scenes.workload("tiny")
    if channels == 3:
        wl = wl.with_(channels=3)
    p = scenes.make_pair(wl, seed=seed)
    return wl, p.left, p.right


# ------------------------------------------------------------------ staged steps


@pytest.mark.parametrize("channels,d_min", [(1, 0), (3, 0), (1, 3), (3, 5)])
def test_cost_tad_bit_exact(channels, d_min):
    wl, Lh, Rh = _tiny(channels)
    pb = Problem(d_min, 15, wl.radius, wl.sigma_s, wl.sigma_r, wl.cost_cap)
    _say("cost_tad", channels, d_min)
    c = _h(fbs.cost(_params(Lh, pb), _d(Lh), _d(Rh)))
    want = oracle.cost(pb, Lh, Rh).astype(np.float32)
    np.testing.assert_array_equal(c, want)


@pytest.mark.parametrize("ncc_r", [0, 1, 3])
def test_cost_ncc(ncc_r):
    wl, Lh, Rh = _tiny(1)
    pb = Problem(0, 15, wl.radius, wl.sigma_s, wl.sigma_r, cost_type=NCC, ncc_radius=ncc_r)
    _say("cost_ncc", ncc_r)
    c = _h(fbs.cost(_params(Lh, pb), _d(Lh), _d(Rh)))
    want = oracle.cost(pb, Lh, Rh)
    np.testing.assert_allclose(c, want, rtol=0, atol=2e-6)


def test_wta_subpixel_quadratic_profiles():
    D, W = 24, 40
    d = np.arange(D, dtype=np.float64)
    deltas = np.linspace(1.6, 21.4, W)
    vol = 0.37 * (d[:, None] - deltas[None, :]) ** 2 + 5.0          # [D][W]
    vol = vol[:, None, :].astype(np.float32)                         # H = 1
    p = L.make_params(W, 1, 1, 0, D - 1, 0, 1.0, 1.0)
    _say("wta quadratic")
    disp, sub = fbs.wta_subpixel(p, _d(vol))
    disp, sub = _h(disp), _h(sub)
    np.testing.assert_array_equal(disp[0], np.rint(deltas).astype(np.int32))
    np.testing.assert_allclose(sub[0], deltas, atol=2e-4)


def test_wta_ties_and_edges():
    prof = np.array([[5, 2, 7, 2, 9, 9], [1, 2, 3, 4, 5, 6], [6, 5, 4, 3, 2, 1], [4, 4, 4, 4, 4, 4]],
                    dtype=np.float32).T                                # [D=6][W=4]
    p = L.make_params(8, 1, 1, 3, 8, 0, 1.0, 1.0)
    vol = np.zeros((6, 1, 8), dtype=np.float32)
    vol[:, 0, :4] = prof
    vol[:, 0, 4:] = prof
    disp, sub = fbs.wta_subpixel(p, _d(vol))
    disp, sub = _h(disp)[0], _h(sub)[0]
    assert list(disp[:4]) == [4, 3, 8, 3]
    assert sub[0] == pytest.approx(4 + (5 - 7) / 16.0, abs=1e-6)
    assert list(sub[1:4]) == [3.0, 8.0, 3.0]


# --------------------------------------------------- staged and fused pipelines

CASES = {
    "tiny_gray_tad": (1, TAD, {}),
    "tiny_rgb_tad": (3, TAD, {}),
    "tiny_gray_ncc": (1, NCC, {}),
    "tiny_gray_tad_d3": (1, TAD, {"d_min": 3}),
}


def _case(name):
    channels, ct, over = CASES[name]
    wl, Lh, Rh = _tiny(channels)
    pb = Problem.from_workload(wl, cost_type=ct)
    if over:
        pb = Problem(over.get("d_min", pb.d_min), pb.d_max, pb.radius, pb.gamma_d, pb.gamma_r,
                     pb.tau, pb.cost_type, pb.ncc_radius)
    return pb, Lh, Rh


@pytest.mark.parametrize("name", list(CASES))
def test_staged_vs_oracle(name):
    pb, Lh, Rh = _case(name)
    _say("staged", name)
    p = _params(Lh, pb)
    c, a, d, s = _staged(p, _d(Lh), _d(Rh))
    rep = _full_compare(pb, Lh, Rh, _h(d), _h(s), _h(a))
    _say(rep)
    assert rep.ok, str(rep)


@pytest.mark.parametrize("name", list(CASES))
def test_fused_valu_equals_staged_bitwise(name):
    pb, Lh, Rh = _case(name)
    _say("fused==staged", name)
    p = _params(Lh, pb, flags=L.FBS_F_FORCE_VALU)
    Ld, Rd = _d(Lh), _d(Rh)
    _, a, d, s = _staged(p, Ld, Rd)
    d2, s2, a2 = fbs.run(p, Ld, Rd, want_agg=True)
    np.testing.assert_array_equal(_h(d2), _h(d))
    np.testing.assert_array_equal(_h(s2).view(np.uint32), _h(s).view(np.uint32))
    np.testing.assert_array_equal(_h(a2).view(np.uint32), _h(a).view(np.uint32))


@pytest.mark.parametrize("name", list(CASES))
def test_fused_default_vs_oracle(name):
    pb, Lh, Rh = _case(name)
    p = _params(Lh, pb)
    _say("fused", name, "variant", L.fbs_run_variant(p))
    d, s, a = fbs.run(p, _d(Lh), _d(Rh), want_agg=True)
    rep = _full_compare(pb, Lh, Rh, _h(d), _h(s), _h(a))
    _say(rep)
    assert rep.ok, str(rep)


@pytest.mark.parametrize("force_valu", [False, True])
def test_mid_full_frame_vs_oracle(force_valu):
    wl = scenes.workload("mid")
    pr = scenes.make_pair(wl)
    pb = Problem.from_workload(wl)
    p = _params(pr.left, pb, flags=L.FBS_F_FORCE_VALU if force_valu else 0)
    _say("mid", wl.name, "variant", L.fbs_run_variant(p))
    d, s, a = fbs.run(p, _d(pr.left), _d(pr.right), want_agg=True)
    rep = _full_compare(pb, pr.left, pr.right, _h(d), _h(s), _h(a))
    _say(rep)
    assert rep.ok, str(rep)
    # bad-2px against the synthetic ground truth stays a sanity trend (not parity)
    ok = ~pr.occluded
    bad2 = float(np.mean(np.abs(_h(s)[ok] - pr.gt_disp[ok]) > 2.0))
    assert bad2 < 0.2


def _sample_pixels(W, H, n, seed):
    rng = np.random.default_rng(seed)
    xs = list(rng.integers(0, W, n))
    ys = list(rng.integers(0, H, n))
    # corners, borders and the last tile
    for x in (0, 1, W // 2, W - 2, W - 1):
        for y in (0, 1, H // 2, H - 2, H - 1):
            xs.append(x)
            ys.append(y)
    return np.array(xs, dtype=np.int32), np.array(ys, dtype=np.int32)


@pytest.mark.parametrize("force_valu", [False, True])
def test_large_rgb_sampled_vs_oracle(force_valu):
    wl = scenes.workload("large")
    pr = scenes.make_pair(wl)
    pb = Problem.from_workload(wl)
    p = _params(pr.left, pb, flags=L.FBS_F_FORCE_VALU if force_valu else 0)
    _say("large", wl.name, "variant", L.fbs_run_variant(p))
    d, s, a = fbs.run(p, _d(pr.left), _d(pr.right), want_agg=True)
    d, s = _h(d), _h(s)
    xs, ys = _sample_pixels(wl.width, wl.height, 1500, 7)
    a_smp = a[:, torch.from_numpy(ys).long().cuda(), torch.from_numpy(xs).long().cuda()]
    a_smp = _h(a_smp)
    del a
    ao, do, so = oracle.fbs_pixels(pb, pr.left, pr.right, xs, ys)
    rep = compare_maps(d[ys, xs], s[ys, xs], do, so, ao.T, pb.d_min, floor=_floor(pb))
    compare_agg(a_smp, ao.T, rep, floor=_floor(pb))
    _say(rep)
    assert rep.ok, str(rep)


# ----------------------------------------------------------------- edge cases

EDGE = {
    "ragged_37x23": dict(W=37, H=23, C=1, dmin=2, dmax=6, r=3),
    "one_disparity": dict(W=30, H=20, C=1, dmin=4, dmax=4, r=2),
    "radius0": dict(W=33, H=17, C=1, dmin=0, dmax=9, r=0),
    "radius16": dict(W=45, H=38, C=1, dmin=0, dmax=7, r=16),
    "two_pixels": dict(W=2, H=1, C=1, dmin=0, dmax=1, r=1),
    "one_row": dict(W=50, H=1, C=1, dmin=0, dmax=12, r=2),
    "one_column_band": dict(W=3, H=40, C=1, dmin=0, dmax=2, r=4),
    "uniform_weights": dict(W=40, H=21, C=1, dmin=0, dmax=10, r=3, sig=math.inf),
    "rgb_ragged": dict(W=41, H=19, C=3, dmin=1, dmax=9, r=2),
    "rgb_radius16": dict(W=40, H=34, C=3, dmin=0, dmax=5, r=16),
    "padded_stride": dict(W=29, H=18, C=1, dmin=0, dmax=8, r=2, pad=11),
    "padded_stride_rgb": dict(W=26, H=18, C=3, dmin=0, dmax=8, r=2, pad=5),
    "ncc_r0": dict(W=35, H=22, C=1, dmin=0, dmax=9, r=2, ncc=0),
    "ncc_r3": dict(W=35, H=22, C=1, dmin=1, dmax=9, r=2, ncc=3),
    "ncc_radius16": dict(W=40, H=36, C=1, dmin=0, dmax=6, r=16, ncc=1),
    "many_disparities": dict(W=1100, H=3, C=1, dmin=0, dmax=1023, r=1),
    "small_cap": dict(W=40, H=20, C=1, dmin=0, dmax=10, r=2, tau=3.5),
}


def _edge_inputs(e, seed):
    rng = np.random.default_rng(seed)
    shape = (e["H"], e["W"]) if e["C"] == 1 else (e["H"], e["W"], 3)
    Lh = rng.integers(0, 256, shape, dtype=np.uint8)
    shift = min(3, e["W"] - 1)
    Rh = np.roll(Lh, -shift, axis=1)
    Rh = np.clip(Rh.astype(int) + rng.integers(-6, 7, shape), 0, 255).astype(np.uint8)
    return Lh, Rh


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_case_vs_oracle(name):
    e = EDGE[name]
    Lh, Rh = _edge_inputs(e, seed=zlib.crc32(name.encode()) % 1000)
    sig = e.get("sig", 3.0)
    ct = NCC if "ncc" in e else TAD
    pb = Problem(e["dmin"], e["dmax"], e["r"], sig, sig * 3 if sig != math.inf else sig,
                 e.get("tau", 40.0), ct, e.get("ncc", 1))
    W, H, C = e["W"], e["H"], e["C"]
    pad = e.get("pad", 0)
    if pad:
        buf_l = np.zeros((H, W * C + pad), dtype=np.uint8)
        buf_r = np.zeros((H, W * C + pad), dtype=np.uint8)
        buf_l[:, :W * C] = Lh.reshape(H, W * C)
        buf_r[:, :W * C] = Rh.reshape(H, W * C)
        Ld, Rd = _d(buf_l), _d(buf_r)
        stride = W * C + pad
    else:
        Ld, Rd = _d(Lh), _d(Rh)
        stride = None
    for flags in (0, L.FBS_F_FORCE_VALU):
        p = _params(Lh, pb, flags=flags, row_stride=stride)
        _say("edge", name, "flags", flags, "variant", L.fbs_run_variant(p))
        d, s, a = fbs.run(p, Ld, Rd, want_agg=True)
        rep = _full_compare(pb, Lh, Rh, _h(d), _h(s), _h(a))
        _say(rep)
        assert rep.ok, f"{name} flags={flags}: {rep}"
    # the staged path on the same inputs
    p = _params(Lh, pb, row_stride=stride)
    c, a, d, s = _staged(p, Ld, Rd)
    rep = _full_compare(pb, Lh, Rh, _h(d), _h(s), _h(a))
    assert rep.ok, f"{name} staged: {rep}"


# ---------------------------------------------------------- runtime behaviour


def test_deterministic_repeat():
    wl = scenes.workload("mid")
    pr = scenes.make_pair(wl)
    p = fbs.params_for(wl)
    Ld, Rd = _d(pr.left), _d(pr.right)
    d1, s1 = fbs.run(p, Ld, Rd)
    d2, s2 = fbs.run(p, Ld, Rd)
    np.testing.assert_array_equal(_h(d1), _h(d2))
    np.testing.assert_array_equal(_h(s1).view(np.uint32), _h(s2).view(np.uint32))


def test_partial_outputs_and_side_stream():
    wl, Lh, Rh = _tiny(1)
    p = fbs.params_for(wl)
    Ld, Rd = _d(Lh), _d(Rh)
    d_ref, s_ref = fbs.run(p, Ld, Rd)
    st = torch.cuda.Stream()
    disp = torch.full((wl.height, wl.width), -7, dtype=torch.int32, device="cuda")
    sub = torch.full((wl.height, wl.width), -7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        L.fbs_run(p, Ld, Rd, disp, None, None, None, st)
    st.synchronize()
    np.testing.assert_array_equal(_h(disp), _h(d_ref))
    L.fbs_run(p, Ld, Rd, None, sub, None, None, None)
    np.testing.assert_array_equal(_h(sub), _h(s_ref))


def test_invalid_call_enqueues_nothing():
    wl, Lh, Rh = _tiny(1)
    p = fbs.params_for(wl)
    p.radius = 99
    disp = torch.full((wl.height, wl.width), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(L.FbsError) as e:
        L.fbs_run(p, _d(Lh), _d(Rh), disp, None)
    assert e.value.status == L.FBS_E_UNSUPPORTED
    assert int(_h(disp).max()) == -7
    p = fbs.params_for(wl, cost_type=L.FBS_COST_NCC)
    with pytest.raises(L.FbsError) as e:
        L.fbs_run(p, _d(Lh), _d(Rh), disp, None, None, None)
    assert e.value.status == L.FBS_E_WORKSPACE
    assert int(_h(disp).max()) == -7
