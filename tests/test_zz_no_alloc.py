"""fbs_run_lr_noalloc (static per-GPU scratch, no allocation) against
fbs_run_lr (caller's workspace) through the C ABI: two calls in a row, the
second on a smaller input, each bit for bit equal to the workspace entry
point; sizes past the scratch are rejected before anything runs."""
import numpy as np
import pytest

from paper_1807_02044_amd import _lib as L
from paper_1807_02044_amd import scenes
import paper_1807_02044_amd as fbs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pair(wl):
    pr = scenes.make_pair(wl)
    return (torch.from_numpy(pr.left).cuda(), torch.from_numpy(pr.right).cuda())


def _outs(wl):
    H, W = wl.height, wl.width
    return (torch.full((H, W), -5, dtype=torch.int32, device="cuda"),
            torch.full((H, W), -5, dtype=torch.int32, device="cuda"),
            torch.full((H, W), 7, dtype=torch.uint8, device="cuda"),
            torch.full((H, W), -5.0, dtype=torch.float32, device="cuda"))


def _same(a, b):
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        xa, ya = x.cpu().numpy(), y.cpu().numpy()
        if xa.dtype == np.float32:
            xa, ya = xa.view(np.uint32), ya.view(np.uint32)
        np.testing.assert_array_equal(xa, ya)


def test_noalloc_equals_workspace_entry_point_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # first call: the 450x375 gray pair; second call: a smaller RGB pair
    for wl in (scenes.workload("mid"), scenes.workload("tiny").with_(channels=3)):
        p = fbs.params_for(wl)
        assert L.fbs_lr_workspace_bytes(p) <= L.FBS_NOALLOC_SCRATCH_BYTES
        Ld, Rd = _pair(wl)
        ref = fbs.run_lr(p, Ld, Rd, 0)
        got = _outs(wl)
        L.fbs_run_lr_noalloc(p, Ld, Rd, 0, *got)
        print(wl.name, "valid", int(got[2].sum().item()), "of", wl.width * wl.height, flush=True)
        _same(got, ref)


def test_noalloc_on_a_side_stream_and_max_diff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = scenes.workload("tiny")
    p = fbs.params_for(wl)
    Ld, Rd = _pair(wl)
    ref = fbs.run_lr(p, Ld, Rd, 1)
    got = _outs(wl)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    L.fbs_run_lr_noalloc(p, Ld, Rd, 1, *got, st)
    st.synchronize()
    _same(got, ref)


def test_noalloc_rejects_sizes_past_the_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = L.make_params(4000, 3000, 3, 0, 63, 3, 3.0, 10.0, 40.0)
    assert L.fbs_lr_workspace_bytes(p) > L.FBS_NOALLOC_SCRATCH_BYTES
    d = torch.full((4, 4), -5, dtype=torch.int32, device="cuda")
    with pytest.raises(L.FbsError) as e:
        L.fbs_run_lr_noalloc(p, d, d, 0, d, None, None, None)
    assert e.value.status == L.FBS_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert int(d.min().item()) == -5
