"""Pins of the surrogate oracle (features, conv net, loss, Adam) on the CPU.

Each check reaches its expected value by another route: torch's bfloat16
cast, scipy's 2-D correlation, central finite differences, a stable sort,
and the closed form of Adam's first step.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import surrogate as S


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.uniform(-1e-3, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.4e38]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x), want)


def test_conv3x3_is_scipy_correlation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, 9, 3))
    w = rng.normal(size=(3, 3, 2, 3)).astype(np.float32)
    b = np.array([0.5, -1.0], dtype=np.float32)
    y = S.conv3x3(x, w, b)
    for co in range(2):
        want = np.full((7, 9), float(b[co]))
        for ci in range(3):
            want += signal.correlate2d(x[..., ci], w[:, :, co, ci].astype(np.float64), mode="same",
                                       boundary="fill", fillvalue=0.0)
        np.testing.assert_allclose(y[..., co], want, rtol=1e-12, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    H, W = 6, 7
    feat = rng.uniform(0, 1, size=(H, W, 17))
    params = {k: v.astype(np.float64) for k, v in S.init_params(3).items()}
    for l in range(4):
        params[f"b{l}"] = rng.normal(0, 0.1, params[f"b{l}"].shape)
    r = rng.normal(size=(H, W))                      # L = sum(pred * r)

    def loss(p):
        out, _, _ = S.forward(feat, p, bf16_points=False)
        return float(np.sum(out * r))

    out, acts, _ = S.forward(feat, params, bf16_points=False)
    grads = S.backward(r, acts, params, bf16_points=False)
    h = 1e-6
    for key in ["w0", "w1", "w2", "w3", "b0", "b1", "b2", "b3"]:
        flat = params[key].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            save = flat[idx]
            flat[idx] = save + h
            lp = loss(params)
            flat[idx] = save - h
            lm = loss(params)
            flat[idx] = save
            fd = (lp - lm) / (2 * h)
            an = grads[key].reshape(-1)[idx]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-7), (key, idx)


def test_features_sorted_with_ties_to_lower_d():
    agg = np.array([[[5.0]], [[2.0]], [[7.0]], [[2.0]], [[9.0]], [[1.0]], [[2.0]], [[8.0]],
                    [[3.0]], [[6.0]]])                      # D = 10, 1x1 image
    left = np.array([[51]], dtype=np.uint8)
    f = S.features(agg, left, d_min=4, tau=10.0)
    # ascending costs 1, 2, 2, 2, 3, 5, 6, 7 at indices 5, 1, 3, 6, 8, 0, 9, 2
    np.testing.assert_allclose(f[0, 0, :8], np.float32([1, 2, 2, 2, 3, 5, 6, 7]) / np.float32(10))
    np.testing.assert_allclose(f[0, 0, 8:16], np.array([5, 1, 3, 6, 8, 0, 9, 2]) / 9.0)
    assert f[0, 0, 16] == pytest.approx(51 / 255.0)


def test_features_near_ties_at_key_resolution():
    """Costs that differ only in the low kbits of their float32 pattern (kbits =
    bit width of D - 1 = 4 here) are equal for the selection: the lower
    disparity goes first and the truncated cost is reported."""
    base = np.float32(3.0)
    near = (base.view(np.uint32) + np.uint32(5)).view(np.float32)   # 3.0 plus 5 ulp
    far = (base.view(np.uint32) + np.uint32(16)).view(np.float32)   # 3.0 plus 16 ulp
    agg = np.full((10, 1, 1), 50.0)
    agg[7, 0, 0] = base
    agg[2, 0, 0] = near          # lower d than 7, slightly larger cost: a tie at key resolution
    agg[0, 0, 0] = far           # a real difference: stays after both
    f = S.features(agg, np.zeros((1, 1), dtype=np.uint8), d_min=0, tau=1.0)
    np.testing.assert_array_equal(f[0, 0, 8:11], np.array([2, 7, 0]) / 9.0)
    assert f[0, 0, 0] == f[0, 0, 1] == 3.0
    assert f[0, 0, 2] == float(far)


def test_l1_gradient_closed_form():
    pred = np.array([[1.0, 2.0], [3.0, 4.0]])
    label = np.array([[0.5, 2.0], [3.5, 1.0]])
    loss, g = S.l1_loss_grad(pred, label)
    assert loss == pytest.approx((0.5 + 0 + 0.5 + 3.0) / 4)
    np.testing.assert_array_equal(g, np.array([[0.25, 0.0], [-0.25, 0.25]]))


def test_adam_first_step_is_lr_times_sign():
    p = {"w": np.array([1.0, -2.0, 0.5], dtype=np.float32)}
    g = {"w": np.array([3.0, -0.01, 1e-3])}
    new, st = S.adam_step(p, g, {}, lr=0.01)
    # m_hat = g, v_hat = g^2 on the first step: the move is lr * g / (|g| + eps)
    want = p["w"].astype(np.float64) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    np.testing.assert_allclose(new["w"], want.astype(np.float32), rtol=0, atol=1e-7)
    assert st["t"] == 1
    new2, st2 = S.adam_step(new, g, st, lr=0.01)
    assert st2["t"] == 2 and np.all(np.abs(new2["w"] - new["w"]) <= 0.0100001)


def test_bf16_forward_close_to_exact():
    rng = np.random.default_rng(4)
    feat = rng.uniform(0, 1, size=(8, 8, 17))
    params = S.init_params(5)
    a, _, _ = S.forward(feat, params, bf16_points=True)
    b, _, _ = S.forward(feat, params, bf16_points=False)
    assert np.max(np.abs(a - b)) < 0.05 * (np.max(np.abs(b)) + 1e-3)
