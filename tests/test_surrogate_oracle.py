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
    np.testing.assert_allclose(f[0, 0, :8], np.array([1, 2, 2, 2, 3, 5, 6, 7]) / 10.0,
                               rtol=0, atol=0)
    np.testing.assert_allclose(f[0, 0, 8:16], np.array([5, 1, 3, 6, 8, 0, 9, 2]) / 9.0)
    assert f[0, 0, 16] == pytest.approx(51 / 255.0)


def test_features_order_is_exact_at_ulp_level():
    """Costs one float32 ulp apart are ordered by value, not by disparity:
    the definition is the exact ascending order (only exactly equal costs go
    to the lower disparity)."""
    base = np.float32(3.0)
    up1 = (base.view(np.uint32) + np.uint32(1)).view(np.float32)    # 3.0 plus 1 ulp
    up5 = (base.view(np.uint32) + np.uint32(5)).view(np.float32)    # 3.0 plus 5 ulp
    agg = np.full((10, 1, 1), 50.0)
    agg[7, 0, 0] = base
    agg[2, 0, 0] = up5           # lower d than 7, larger cost: goes after it
    agg[0, 0, 0] = up1           # lowest d, between the two
    agg[9, 0, 0] = base          # exact tie with d = 7: after it (higher d)
    f = S.features(agg, np.zeros((1, 1), dtype=np.uint8), d_min=0, tau=1.0)
    np.testing.assert_array_equal(f[0, 0, 8:12], np.array([7, 9, 0, 2]) / 9.0)
    np.testing.assert_array_equal(f[0, 0, :4], [3.0, 3.0, float(up1), float(up5)])


def test_features_against_brute_force_selection():
    """Top-8 by repeated extraction of the minimum (first index on ties) on
    random volumes with many exact ties: an independent route to the order."""
    rng = np.random.default_rng(11)
    D, H, W = 19, 3, 4
    agg = rng.integers(0, 6, size=(D, H, W)) * 0.5 + rng.integers(0, 2, size=(D, H, W)) * 1e-9
    f = S.features(agg, np.zeros((H, W), dtype=np.uint8), d_min=3, tau=2.0)
    for y in range(H):
        for x in range(W):
            col = list(agg[:, y, x])
            taken = []
            for _ in range(8):
                best = None
                for k in range(D):
                    if k in taken:
                        continue
                    if best is None or col[k] < col[best]:
                        best = k
                taken.append(best)
            assert list(np.rint(f[y, x, 8:16] * (D - 1)).astype(int)) == taken
            assert list(f[y, x, :8]) == [col[k] / 2.0 for k in taken]


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


def test_adam_two_steps_hand_worked():
    """Two Adam steps with beta1 != beta2, worked by hand, where the bias
    corrections of step 2 matter (Kingma and Ba, Algorithm 1):
      beta1 = 1/2, beta2 = 3/4, lr = 1/10, g1 = 1/2, g2 = 1/4, p0 = 1.
      step 1: m = 1/4, v = 1/16, m^ = 1/2, v^ = 1/4      -> p1 = 1 - 0.1 = 0.9
      step 2: m = 1/4, v = 1/16, m^ = (1/4)/(3/4) = 1/3,
              v^ = (1/16)/(7/16) = 1/7                   -> p2 = 0.9 - 0.1 * sqrt(7) / 3
    Dropping either bias correction, using t = 1 at step 2, or swapping the
    betas gives 0.8 or a value further off."""
    p = {"w": np.array([1.0], dtype=np.float32)}
    p1, st = S.adam_step(p, {"w": np.array([0.5])}, {}, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    assert float(p1["w"][0]) == pytest.approx(0.9, abs=1e-7)
    p2, st2 = S.adam_step(p1, {"w": np.array([0.25])}, st, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    want = 0.9 - 0.1 * np.sqrt(7.0) / 3.0                 # 0.81180829...
    assert float(p2["w"][0]) == pytest.approx(want, abs=2e-7)
    assert abs(want - 0.8) > 0.01
    # the moments are kept uncorrected between steps
    assert st2["m_w"][0] == pytest.approx(0.25) and st2["v_w"][0] == pytest.approx(0.0625)


# ---- BF16 rounding points (reading S5), worked in exact rationals ----------

from fractions import Fraction as Fr  # noqa: E402


def _round_sig(x: Fr, bits: int) -> Fr:
    """x rounded to `bits` significant bits, ties to even (exact rationals)."""
    if x == 0:
        return Fr(0)
    sgn = -1 if x < 0 else 1
    a = abs(x)
    e = 0
    while a >= 2:
        a /= 2
        e += 1
    while a < 1:
        a *= 2
        e -= 1
    q = a * 2 ** (bits - 1)                     # in [2^(bits-1), 2^bits)
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and n % 2 == 1):
        n += 1
    return sgn * Fr(n) * Fr(2) ** (e - (bits - 1))


def _bf(x: Fr) -> Fr:
    """Stored as BF16: the float32 value of x rounded to 8 significant bits."""
    return _round_sig(_round_sig(x, 24), 8)


# A 1x1 image: with 'same' padding only the centre tap of each 3x3 kernel sees
# data, and only channels 0 and 1 of every layer are non-zero, so the net is
# the 2-channel chain below, small enough to follow by hand.
_F = [Fr(1, 3), Fr(7, 10)]                                    # features 0, 1
_W = [[[Fr(3, 10), Fr(7, 10)], [Fr(11, 20), Fr(-1, 5)]],      # w0[co][ci]
      [[Fr(13, 20), Fr(1, 5)], [Fr(2, 5), Fr(17, 20)]],       # w1
      [[Fr(-9, 20), Fr(7, 10)], [Fr(3, 5), Fr(1, 3)]],        # w2
      [[Fr(5, 7), Fr(-2, 3)]]]                                # w3 (one output)
_B = [[Fr(1, 8), Fr(3, 16)], [Fr(-1, 16), Fr(1, 32)], [Fr(1, 4), Fr(-1, 8)], [Fr(1, 2)]]
_GOUT = Fr(3, 10)                                             # dL/d(output)
_POINTS = ("feat", "w", "act1", "act2", "act3", "g3", "g2", "g1", "g0")


def _chain(skip=None):
    """Forward and backward of the 2-channel chain; `skip` names one rounding
    point left out.  Returns (output, {grad name: values})."""
    def q(x, pt):
        return x if pt == skip else _bf(x)

    f32 = lambda v: Fr(float(np.float32(float(v))))            # noqa: E731 (float32 master)
    w = [[[q(f32(v), "w") for v in row] for row in layer] for layer in _W]
    b = [[f32(v) for v in layer] for layer in _B]
    acts = [[q(v, "feat") for v in _F]]
    for l in range(3):
        z = [sum(w[l][co][ci] * acts[l][ci] for ci in range(2)) + b[l][co] for co in range(2)]
        acts.append([q(max(v, Fr(0)), f"act{l + 1}") for v in z])
    out = sum(w[3][0][ci] * acts[3][ci] for ci in range(2)) + b[3][0]
    grads = {}
    g = [_GOUT]
    for l in (3, 2, 1, 0):
        gq = [q(v, f"g{l}") for v in g]
        grads[f"w{l}"] = [gq[co] * acts[l][ci] for co in range(len(gq)) for ci in range(2)]
        grads[f"b{l}"] = list(gq)
        if l > 0:
            gx = [sum(gq[co] * w[l][co][ci] for co in range(len(gq))) for ci in range(2)]
            g = [gx[ci] if acts[l][ci] > 0 else Fr(0) for ci in range(2)]
    return out, grads


def _oracle_chain():
    feat = np.zeros((1, 1, 17))
    feat[0, 0, :2] = [float(v) for v in _F]
    params = {}
    for l, (cin, cout) in enumerate(zip(S.CH[:-1], S.CH[1:])):
        w = np.zeros((3, 3, cout, cin), dtype=np.float32)
        for co, row in enumerate(_W[l]):
            for ci, v in enumerate(row):
                w[1, 1, co, ci] = float(v)
        bias = np.zeros(cout, dtype=np.float32)
        bias[:len(_B[l])] = [float(v) for v in _B[l]]
        params[f"w{l}"], params[f"b{l}"] = w, bias
    out, acts, _ = S.forward(feat, params, bf16_points=True)
    grads = S.backward(np.full((1, 1), float(_GOUT)), acts, params, bf16_points=True)
    g = {}
    for l in range(4):
        cout = 1 if l == 3 else 2
        g[f"w{l}"] = [grads[f"w{l}"][1, 1, co, ci] for co in range(cout) for ci in range(2)]
        g[f"b{l}"] = list(grads[f"b{l}"][:cout])
    return float(out[0, 0]), g


def test_bf16_rounding_points_hand_worked():
    """The oracle's BF16 forward and backward equal the exact-rational chain
    with every rounding point of reading S5, to the last bit."""
    want_out, want_g = _chain()
    out, g = _oracle_chain()
    assert out == float(want_out)
    for k, vals in want_g.items():
        assert g[k] == [float(v) for v in vals], k


@pytest.mark.parametrize("point", _POINTS)
def test_bf16_rounding_point_is_observable(point):
    """Dropping any single rounding point changes the chain's output or a
    gradient, so the hand-worked pin above fails for an oracle that misses it."""
    full_out, full_g = _chain()
    out, g = _chain(skip=point)
    changed = float(out) != float(full_out) or any(
        [float(v) for v in g[k]] != [float(v) for v in full_g[k]] for k in full_g)
    assert changed, point
