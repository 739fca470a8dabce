"""Batched plans: one graph launch over many pairs of uneven sizes.

The plan runs each pair through the same per-pixel arithmetic as fbs_run
(the accumulation order depends on the radius only, never on the tuned
waves-per-workgroup or slab depth), so its outputs must equal per-pair
fbs_run bit for bit.
"""
import json
import os
import sys

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


def _say(*a):
    print(*a, flush=True)


# a small uneven batch: sizes, ranges and radii differ; one RGB pair and one
# pair the matrix cores do not take (radius 12 -> vector-ALU kernel)
def _batch():
    specs = [
        (96, 72, 1, 0, 31, 5), (150, 97, 1, 3, 66, 7), (64, 48, 1, 0, 15, 10),
        (200, 40, 3, 0, 47, 7), (77, 61, 1, 0, 20, 12), (130, 90, 1, 0, 95, 5),
    ]
    out = []
    for i, (W, H, C, d0, d1, r) in enumerate(specs):
        wl = scenes.Workload(f"b{i}", W, H, C, d0, d1, r, float(r), 10.0, 40.0,
                             scene="slanted", seed=500 + i, n_planes=4)
        out.append((wl, scenes.make_pair(wl)))
    return out


def _run_plan(plan, pairs):
    dev = torch.device("cuda:0")
    Ls = [torch.from_numpy(p.left).to(dev) for _, p in pairs]
    Rs = [torch.from_numpy(p.right).to(dev) for _, p in pairs]
    Ds = [torch.full((wl.height, wl.width), -1, dtype=torch.int32, device=dev) for wl, _ in pairs]
    Ss = [torch.full((wl.height, wl.width), -1.0, dtype=torch.float32, device=dev) for wl, _ in pairs]
    plan.launch(Ls, Rs, Ds, Ss)
    torch.cuda.synchronize()
    return Ls, Rs, [d.cpu().numpy() for d in Ds], [s.cpu().numpy() for s in Ss]


def test_plan_equals_per_pair_run_bitwise():
    pairs = _batch()
    params = [fbs.params_for(wl) for wl, _ in pairs]
    plan = L.FbsPlan(params)
    cfgs = [plan.pair_config(i) for i in range(len(pairs))]
    _say("configs", cfgs, "launches", plan.num_launches())
    assert cfgs[4][0] == 0 and all(c[0] == 1 for i, c in enumerate(cfgs) if i != 4)
    assert plan.num_launches() == 2
    Ls, Rs, Ds, Ss = _run_plan(plan, pairs)
    for i, (wl, _) in enumerate(pairs):
        d, s = fbs.run(params[i], Ls[i], Rs[i])
        np.testing.assert_array_equal(Ds[i], d.cpu().numpy(), err_msg=wl.name)
        np.testing.assert_array_equal(Ss[i].view(np.uint32), s.cpu().numpy().view(np.uint32),
                                      err_msg=wl.name)
    plan.close()


def test_per_tile_plan_equals_per_pair_run_bitwise():
    """FBS_PLAN_PER_TILE: one workgroup per (pair, tile) item, same bits."""
    pairs = _batch()
    params = [fbs.params_for(wl) for wl, _ in pairs]
    plan = L.FbsPlan(params, per_tile=True)
    assert plan.num_launches() == 2
    Ls, Rs, Ds, Ss = _run_plan(plan, pairs)
    _run_plan(plan, pairs)                      # replay with fresh buffers
    Ls, Rs, Ds, Ss = _run_plan(plan, pairs)
    for i, (wl, _) in enumerate(pairs):
        d, s = fbs.run(params[i], Ls[i], Rs[i])
        np.testing.assert_array_equal(Ds[i], d.cpu().numpy(), err_msg=wl.name)
        np.testing.assert_array_equal(Ss[i].view(np.uint32), s.cpu().numpy().view(np.uint32),
                                      err_msg=wl.name)
    plan.close()


def test_plan_tuning_cache_roundtrip(tmp_path):
    pairs = _batch()[:3]
    params = [fbs.params_for(wl) for wl, _ in pairs]
    cache = str(tmp_path / "tune.json")
    plan = L.FbsPlan(params, tune_cache=cache, tune=True)
    tuned = [plan.pair_config(i) for i in range(3)]
    _, _, Ds, Ss = _run_plan(plan, pairs)
    plan.close()
    data = json.load(open(cache))
    assert data["arch"] == "gfx950" and len(data["entries"]) == 3
    for key, (nw, nb, us, path) in data["entries"].items():
        assert nw in (4, 8, 12) and nb >= 1 and us > 0
        # the loop order the depth implies: chunk-outer when one slab holds every block
        nblk = (int(key.split(",")[3]) + 15) // 16
        assert path == ("chunk-outer" if nb == nblk and nblk <= 6 else "slab")
    # a plan built from the cache alone picks the same configurations
    plan2 = L.FbsPlan(params, tune_cache=cache, tune=False)
    assert [plan2.pair_config(i) for i in range(3)] == tuned
    _, _, Ds2, Ss2 = _run_plan(plan2, pairs)
    for a, b in zip(Ds, Ds2):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(Ss, Ss2):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    plan2.close()


def test_plan_relaunch_with_new_buffers_and_oracle():
    pairs = _batch()
    params = [fbs.params_for(wl) for wl, _ in pairs]
    plan = L.FbsPlan(params)
    _run_plan(plan, pairs)                       # first launch, then fresh buffers
    Ls, Rs, Ds, Ss = _run_plan(plan, pairs)
    wl, pr = pairs[1]
    pb = Problem.from_workload(wl)
    do, so, ao = oracle.fbs(pb, pr.left, pr.right, want_agg=True)
    rep = compare_maps(Ds[1], Ss[1], do, so, ao.reshape(ao.shape[0], -1), pb.d_min,
                       floor=weight_floor((2 * pb.radius + 1) ** 2, pb.tau))
    _say(rep)
    assert rep.ok, str(rep)
    plan.close()


def test_plan_rejects_bad_input():
    wl = scenes.workload("tiny")
    p = fbs.params_for(wl)
    plan = L.FbsPlan([p])
    with pytest.raises(L.FbsError):
        plan.launch([None], [None], [None], [None])
    plan.close()


def _max_nb(params, wl, tmp_path, nw):
    """Deepest slab the library accepts for one pair at `nw` waves (probed
    through single-pair plans built from a cache entry)."""
    best = 0
    for nb in range(1, 17):
        cache = tmp_path / f"probe_{wl.name}_{nb}.json"
        key = f"{wl.width},{wl.height},1,{wl.n_disp},{wl.radius}"
        cache.write_text(json.dumps({"arch": "gfx950", "entries": {key: [nw, nb, 1.0]}}))
        plan = L.FbsPlan([params], tune_cache=str(cache), tune=False)
        if plan.pair_config(0) == (1, nw, nb):
            best = nb
        plan.close()
    return best


def test_plan_class_mixing_slab_depths(tmp_path):
    """One class (r = 10, 8 waves) holding a 64-disparity pair at its deepest
    slab and two wider-range pairs at theirs (shallower, found by probing):
    the launch must size LDS for the largest per-pair layout, not for
    (largest D) x (deepest slab), and every pair keeps fbs_run's bits."""
    def wl_of(i, W, H, d0, D):
        return scenes.Workload(f"m{i}", W, H, 1, d0, d0 + D - 1, 10, 10.0, 10.0, 40.0,
                               scene="slanted", seed=700 + i, n_planes=3)
    small = wl_of(0, 80, 40, 0, 64)
    nb_small = _max_nb(fbs.params_for(small), small, tmp_path, 8)
    big_D = None
    for D in (256, 512, 768, 1000):
        w = wl_of(9, D + 40, 8, 0, D)
        if _max_nb(fbs.params_for(w), w, tmp_path, 8) < nb_small:
            big_D = D
            break
    assert big_D is not None, "no disparity range with a shallower deepest slab"
    pairs = [(small, scenes.make_pair(small))]
    for i, (extra_w, H, d0) in enumerate([(40, 24, 0), (50, 17, 2)], start=1):
        wl = wl_of(i, big_D + extra_w + d0, H, d0, big_D)
        pairs.append((wl, scenes.make_pair(wl)))
    params = [fbs.params_for(wl) for wl, _ in pairs]
    nbs = [_max_nb(p, wl, tmp_path, 8) for p, (wl, _) in zip(params, pairs)]
    _say("deepest slabs at 8 waves", nbs, "big D", big_D)
    assert nbs[0] > nbs[1] >= 1 and nbs[2] >= 1
    cache = tmp_path / "tune.json"
    entries = {f"{wl.width},{wl.height},1,{wl.n_disp},10": [8, nb, 1.0]
               for (wl, _), nb in zip(pairs, nbs)}
    cache.write_text(json.dumps({"arch": "gfx950", "entries": entries}))
    for per_tile in (False, True):
        plan = L.FbsPlan(params, tune_cache=str(cache), tune=False, per_tile=per_tile)
        cfgs = [plan.pair_config(i) for i in range(len(pairs))]
        _say("configs", cfgs)
        assert cfgs == [(1, 8, nb) for nb in nbs]
        Ls, Rs, Ds, Ss = _run_plan(plan, pairs)
        for i, (wl, _) in enumerate(pairs):
            d, s = fbs.run(params[i], Ls[i], Rs[i])
            np.testing.assert_array_equal(Ds[i], d.cpu().numpy(), err_msg=wl.name)
            np.testing.assert_array_equal(Ss[i].view(np.uint32), s.cpu().numpy().view(np.uint32))
        plan.close()


def test_one_plan_launched_on_two_streams():
    """Two launches of one plan on two streams, with different buffers: the
    second waits for the first on the device, so both equal fbs_run."""
    pairs = _batch()
    params = [fbs.params_for(wl) for wl, _ in pairs]
    plan = L.FbsPlan(params)
    dev = torch.device("cuda:0")
    Ls = [torch.from_numpy(p.left).to(dev) for _, p in pairs]
    Rs = [torch.from_numpy(p.right).to(dev) for _, p in pairs]
    outs = []
    for _ in range(2):
        outs.append(([torch.full((wl.height, wl.width), -1, dtype=torch.int32, device=dev)
                      for wl, _ in pairs],
                     [torch.full((wl.height, wl.width), -1.0, dtype=torch.float32, device=dev)
                      for wl, _ in pairs]))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(3):
        for k in range(2):
            plan.launch(Ls, Rs, outs[k][0], outs[k][1], streams[k])
    torch.cuda.synchronize()
    for i, (wl, pr) in enumerate(pairs):
        d_ref, s_ref = fbs.run(params[i], Ls[i], Rs[i])
        d_ref, s_ref = d_ref.cpu().numpy(), s_ref.cpu().numpy()
        for k in range(2):
            np.testing.assert_array_equal(outs[k][0][i].cpu().numpy(), d_ref)
            np.testing.assert_array_equal(outs[k][1][i].cpu().numpy().view(np.uint32),
                                          s_ref.view(np.uint32))
    plan.close()


# pair shapes of the 64-pair batch at their real sizes: the largest frame with
# the largest range and radius, a mid one, and a small one
BIG = [(1280, 960, 0, 127, 10), (960, 720, 0, 95, 5), (320, 240, 0, 31, 7)]


@pytest.mark.parametrize("per_tile", [False, True])
def test_batch_sized_pairs_vs_oracle_sampled(per_tile):
    pairs = []
    for i, (W, H, d0, d1, r) in enumerate(BIG):
        wl = scenes.Workload(f"big{i}", W, H, 1, d0, d1, r, float(r), 10.0, 40.0,
                             scene="slanted", seed=1000 + 7 * i, n_planes=8)
        pairs.append((wl, scenes.make_pair(wl)))
    params = [fbs.params_for(wl) for wl, _ in pairs]
    plan = L.FbsPlan(params, per_tile=per_tile)
    _say("batch-sized pairs, per_tile", per_tile,
         [plan.pair_config(i) for i in range(len(pairs))])
    Ls, Rs, Ds, Ss = _run_plan(plan, pairs)
    plan.close()
    for i, (wl, pr) in enumerate(pairs):
        d_ref, s_ref = fbs.run(params[i], Ls[i], Rs[i])
        np.testing.assert_array_equal(Ds[i], d_ref.cpu().numpy())
        np.testing.assert_array_equal(Ss[i].view(np.uint32), s_ref.cpu().numpy().view(np.uint32))
        rng = np.random.default_rng(40 + i)
        xs = np.concatenate([rng.integers(0, wl.width, 300), [0, wl.width - 1, wl.width // 2]])
        ys = np.concatenate([rng.integers(0, wl.height, 300), [wl.height - 1, 0, wl.height // 2]])
        xs, ys = xs.astype(np.int32), ys.astype(np.int32)
        pb = Problem.from_workload(wl)
        ao, do, so = oracle.fbs_pixels(pb, pr.left, pr.right, xs, ys)
        rep = compare_maps(Ds[i][ys, xs], Ss[i][ys, xs], do, so, ao.T, pb.d_min,
                           floor=weight_floor((2 * pb.radius + 1) ** 2, pb.tau))
        _say(wl.name, wl.width, wl.height, wl.n_disp, wl.radius, rep)
        assert rep.ok, f"{wl.name}: {rep}"
