"""Pins of the oracle's network (oracle/cnn.py) against facts it does not compute itself:
library convolutions, finite differences, adjointness, closed forms of special weights,
and hand-rounded BF16 values."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def rand_weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(cnn.NUM_WEIGHTS) * scale / 3.0


def test_weight_count_matches_layers():
    assert cnn.NUM_WEIGHTS == 9 * (32 + 3 * 32 * 32 + 32) == 28224


def test_bf16_rounding_hand_values():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                          # halfway, tie to the even neighbour 1.0
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,          # halfway between 1+2^-7 (odd) and 1+2^-6 (even)
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,  # just above halfway
        -3.0: -3.0,
        0.0: 0.0,
        1.0e-3: 0.0009994506835937500,                 # 0x3A83 -> 2^-10 * (1 + 3/128)
    }
    for x, want in cases.items():
        assert cnn.bf16_round(np.array([x]))[0] == want, x


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-5, 5, 10000)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(x), ref)


def test_single_channel_conv_is_correlate2d():
    rng = np.random.default_rng(2)
    img = rng.standard_normal((7, 11))
    k = rng.standard_normal((3, 3))
    got = cnn.conv3(img[None, None], k[None, None])[0, 0]
    assert np.allclose(got, correlate2d(img, k, mode="same", boundary="fill"), rtol=0, atol=1e-13)


def test_multi_channel_conv_is_sum_of_correlations():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, 3, 6, 5))
    k = rng.standard_normal((4, 3, 3, 3))
    got = cnn.conv3(a, k)
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(a[n, c], k[o, c], mode="same") for c in range(3))
            assert np.allclose(got[n, o], ref, rtol=0, atol=1e-12)


def test_conv_adjoint_dot_product():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 3, 5, 7))
    g = rng.standard_normal((2, 4, 5, 7))
    k = rng.standard_normal((4, 3, 3, 3))
    lhs = np.sum(cnn.conv3(a, k) * g)
    rhs = np.sum(a * cnn.conv3_adjoint(g, k))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_zero_last_layer_is_identity():
    w = rand_weights(5)
    w[-9 * 32:] = 0.0
    y = np.random.default_rng(6).standard_normal((2, 5, 9))
    assert np.array_equal(cnn.forward(w, y)[0], y)


def test_positive_homogeneity():
    w = rand_weights(7)
    y = np.random.default_rng(8).standard_normal((2, 6, 6))
    a = 3.7
    out1 = cnn.forward(w, a * y)[0]
    out2 = a * cnn.forward(w, y)[0]
    assert np.allclose(out1, out2, rtol=1e-13, atol=1e-13)


def test_linear_network_superposition_and_composite_stencil():
    """With the identity activation f is linear and equals one 11x11 correlation (the five 3x3
    kernels composed), here checked on a single channel path against scipy."""
    w = rand_weights(24)
    rng = np.random.default_rng(25)
    y1, y2 = rng.standard_normal((2, 1, 13, 12))
    f = lambda y: cnn.forward(w, y, linear=True)[0] - y
    assert np.allclose(f(2.0 * y1 - 0.5 * y2), 2.0 * f(y1) - 0.5 * f(y2), rtol=0, atol=1e-12)
    # impulse response = the composite stencil; away from the edges f(y) = correlate2d(y, stencil)
    e = np.zeros((1, 31, 31))
    e[0, 15, 15] = 1.0
    stencil = f(e)[0, 10:21, 10:21][::-1, ::-1]
    big = rng.standard_normal((1, 40, 40))
    ref = correlate2d(big[0], stencil, mode="same")
    assert np.allclose(f(big)[0, 5:-5, 5:-5], ref[5:-5, 5:-5], rtol=0, atol=1e-11)


@pytest.mark.parametrize("linear", [False, True])
def test_gradient_matches_central_differences(linear):
    w = rand_weights(9, scale=0.6)
    rng = np.random.default_rng(10)
    y = rng.standard_normal((2, 5, 6))
    x = rng.standard_normal((2, 5, 6))
    loss, g = cnn.loss_grad(w, y, x, linear)
    assert loss == pytest.approx(np.sum((cnn.forward(w, y, linear)[0] - x) ** 2) / (2 * x.size), rel=1e-14)
    offs = np.cumsum([0] + [9 * ci * co for ci, co in cnn.LAYERS])
    idx = np.concatenate([rng.choice(np.arange(offs[l], offs[l + 1]), 8, replace=False) for l in range(5)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (cnn.loss_grad(wp, y, x, linear)[0] - cnn.loss_grad(wm, y, x, linear)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), (i, fd, g[i])
