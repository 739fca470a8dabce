"""The parameter sweep's measurements (Eqs. 11-12 on synthetic ground truth)
from the library's left-right path against the same measurement on the FP64
oracle's maps, at small sizes and a few parameter points."""
import numpy as np
import pytest

import oracle
from oracle import Problem
from paper_1807_02044_amd import scenes, sweeps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("rho,gd,gr", [(2, 2.0, 10.0), (4, 4.0, 5.0), (6, 25.0, 50.0)])
def test_point_matches_oracle_measurement(rho, gd, gr):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = scenes.Workload("sw", 96, 64, 1, 0, 23, rho, gd, gr, 40.0, scene="slanted", seed=77,
                         n_planes=5)
    pr = scenes.make_pair(wl)
    res = sweeps.run_point(wl, pr, torch.device("cuda:0"), rho, gd, gr)
    pb = Problem(wl.d_min, wl.d_max, rho, gd, gr, wl.cost_cap)
    dl, dr, valid, sub = oracle.fbs_lrc(pb, pr.left, pr.right)
    want = sweeps.evaluate(sub, pr)
    # the GPU maps follow the oracle's up to accepted 1e-5 ties, each of which
    # can move one pixel's verdict; there are none on this scene
    for k, v in want.items():
        n = int(sweeps.regions(pr)[k].sum())
        assert abs(res["e_pep"][k] - v) <= 100.0 * 2 / n, (k, res["e_pep"][k], v)
    assert res["lrc_kept"] == pytest.approx(float(valid.mean()), abs=4.0 / valid.size)
    _, sub_left = oracle.fbs(pb, pr.left, pr.right)
    want_left = sweeps.evaluate(sub_left, pr)
    for k, v in want_left.items():
        n = int(sweeps.regions(pr)[k].sum())
        assert abs(res["e_pep_left"][k] - v) <= 100.0 * 2 / n, (k, res["e_pep_left"][k], v)


def test_runtime_grows_with_rho():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = scenes.workload("mid")
    pr = scenes.make_pair(wl)
    dev = torch.device("cuda:0")
    t = [sweeps.run_point(wl, pr, dev, r, 7.0, 10.0, timed_steps=20)["fbs_run_ms"]
         for r in (2, 6, 10)]
    print("fbs_run ms at rho 2, 6, 10:", t, flush=True)
    assert t[0] < t[1] < t[2]
