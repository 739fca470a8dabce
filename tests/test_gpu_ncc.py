"""The NCC cost (Eqs. 1-3, block radius 0 or 1) on the matrix-core kernel,
through fbs_run and the C ABI, against the FP64 oracle (rules of
tests/parity.py: disparities outside the 1e-5 tie zone, subpixel within 1e-3
px, aggregated costs within 1e-4 relative, no tie decided by the weight
floor alone) and against the vector-ALU kernel on the same inputs.
Sizes span several 8-row tiles with ragged tails; the radii cover both tile
group shapes and the 4-wave tiles of r = 10.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import NCC, Problem
from paper_1807_02044_amd import _lib as L
from paper_1807_02044_amd import scenes
import paper_1807_02044_amd as fbs

from parity import compare_agg, compare_maps, weight_floor

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


def _params(left, pb, flags=0):
    H, W = left.shape[:2]
    return L.make_params(W, H, 1, pb.d_min, pb.d_max, pb.radius, pb.gamma_d, pb.gamma_r,
                         pb.tau, pb.cost_type, pb.ncc_radius, flags)


def _compare(pb, left, right, d, s, a):
    do, so, ao = oracle.fbs(pb, left, right, want_agg=True)
    fl = weight_floor((2 * pb.radius + 1) ** 2, 2.0)
    rep = compare_maps(d, s, do, so, ao.reshape(ao.shape[0], -1), pb.d_min, floor=fl)
    compare_agg(a, ao, rep, floor=fl)
    return rep


def _pair(W, H, d_max, seed):
    # scenes need a disparity range of some width; a narrower search is fine
    wl = scenes.Workload(f"ncc_{W}x{H}", W, H, 1, 0, max(d_max, 12), 3, 5.0, 10.0, 40.0,
                         scene="slanted", seed=seed, n_planes=4)
    pr = scenes.make_pair(wl)
    return pr.left, pr.right


# (W, H, d_min, d_max, radius, ncc_radius, seed)
CASES = {
    "r3_rho1": (70, 37, 0, 20, 3, 1, 11),
    "r1_rho1_dmin": (45, 19, 4, 27, 1, 1, 12),
    "r5_rho0": (60, 29, 0, 16, 5, 0, 13),
    "r7_rho1_tail": (83, 41, 2, 40, 7, 1, 14),
    "r10_rho1_four_waves": (50, 27, 0, 33, 10, 1, 15),
    "r2_rho1_one_block": (33, 10, 0, 5, 2, 1, 16),
}


@pytest.mark.parametrize("name", list(CASES))
def test_ncc_matrix_core_vs_oracle(name):
    W, H, dmin, dmax, r, nr, seed = CASES[name]
    Lh, Rh = _pair(W, H, dmax, seed)
    pb = Problem(dmin, dmax, r, 5.0, 10.0, 40.0, NCC, nr)
    p = _params(Lh, pb)
    assert L.fbs_run_variant(p) == 1, "NCC with block radius <= 1 takes the matrix-core kernel"
    _say("ncc", name)
    d, s, a = fbs.run(p, _d(Lh), _d(Rh), want_agg=True)
    rep = _compare(pb, Lh, Rh, _h(d), _h(s), _h(a))
    _say(rep)
    assert rep.ok, str(rep)


def test_ncc_matrix_core_agrees_with_vector_kernel():
    Lh, Rh = _pair(96, 40, 31, 21)
    pb = Problem(0, 31, 4, 5.0, 10.0, 40.0, NCC, 1)
    Ld, Rd = _d(Lh), _d(Rh)
    _say("ncc mfma vs valu")
    d1, s1, a1 = fbs.run(_params(Lh, pb), Ld, Rd, want_agg=True)
    d2, s2, a2 = fbs.run(_params(Lh, pb, flags=L.FBS_F_FORCE_VALU), Ld, Rd, want_agg=True)
    a1, a2 = _h(a1), _h(a2)
    # both aggregate the same costs within float rounding of their sums
    np.testing.assert_allclose(a1, a2, rtol=2e-5, atol=1e-6)
    d1, d2 = _h(d1), _h(d2)
    assert float((d1 == d2).mean()) > 0.999


def test_ncc_mid_frame_vs_oracle():
    """The 450x375 pair (D = 64, r = 7) with the paper's block radius 1."""
    wl = scenes.workload("mid")
    pr = scenes.make_pair(wl)
    pb = Problem.from_workload(wl, cost_type=NCC)
    assert pb.ncc_radius == 1
    p = _params(pr.left, pb)
    assert L.fbs_run_variant(p) == 1
    _say("ncc mid", wl.name)
    d, s, a = fbs.run(p, _d(pr.left), _d(pr.right), want_agg=True)
    rep = _compare(pb, pr.left, pr.right, _h(d), _h(s), _h(a))
    _say(rep)
    assert rep.ok, str(rep)


def test_ncc_block_radius_above_one_stays_on_vector_kernel():
    Lh, Rh = _pair(40, 20, 9, 31)
    pb = Problem(0, 9, 2, 5.0, 10.0, 40.0, NCC, 2)
    assert L.fbs_run_variant(_params(Lh, pb)) == 0
