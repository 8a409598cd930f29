"""Pins for oracle.cnn: convolution against a library routine, gradients by finite differences."""
import numpy as np
from scipy import ndimage, special

from oracle import cnn


def test_conv_single_channel_equals_ndimage_correlate():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((6, 6, 6, 1))
    W = rng.standard_normal((27, 1, 1))
    z = cnn.conv(a, W, np.zeros(1))[..., 0]
    k = np.zeros((3, 3, 3))
    for t, (dx, dy, dz) in enumerate(cnn.TAPS):
        k[dx + 1, dy + 1, dz + 1] = W[t, 0, 0]
    ref = ndimage.correlate(a[..., 0], k, mode="constant", cval=0.0)
    assert np.max(np.abs(z - ref)) < 1e-12


def test_centre_tap_is_pointwise_linear_map():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 4, 4, 3))
    W = np.zeros((27, 3, 5))
    W[13] = rng.standard_normal((3, 5))
    b = rng.standard_normal(5)
    assert np.allclose(cnn.conv(a, W, b), a @ W[13] + b)


def test_gelu_definition():
    z = np.linspace(-4, 4, 33)
    assert np.allclose(cnn.gelu(z), 0.5 * z * (1 + special.erf(z / np.sqrt(2))))
    h = 1e-6
    assert np.allclose(cnn.gelu_grad(z), (cnn.gelu(z + h) - cnn.gelu(z - h)) / (2 * h), atol=1e-8)


def test_bf16_rounding():
    assert cnn.bf16(1.0 + 2 ** -9) == 1.0            # tie -> even
    assert cnn.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7
    assert cnn.bf16(-3.140625) == -3.140625


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    n = 5
    x = rng.standard_normal((n, n, n, 3))
    target = rng.standard_normal((n, n, n))
    params = cnn.init_params(3)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    mu, s, cache = cnn.forward(params, x)
    grads = cnn.backward(params, cache, mu, s, target)

    def L(ps):
        m, sv, _ = cnn.forward(ps, x)
        return cnn.loss(m, sv, target)

    h = 1e-6
    for l in range(4):
        W, b = params[l]
        for idx in [(0, 0, 0), (13, W.shape[1] - 1, W.shape[2] - 1), (26, 1, 0)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = [p if i != l else (Wp, b) for i, p in enumerate(params)]
            pm = [p if i != l else (Wm, b) for i, p in enumerate(params)]
            fd = (L(pp) - L(pm)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) < 1e-6 * max(1.0, abs(fd)), (l, idx)
        bp, bm = b.copy(), b.copy()
        bp[0] += h
        bm[0] -= h
        fd = (L([p if i != l else (W, bp) for i, p in enumerate(params)])
              - L([p if i != l else (W, bm) for i, p in enumerate(params)])) / (2 * h)
        assert abs(fd - grads[l][1][0]) < 1e-6 * max(1.0, abs(fd))


def test_loss_minimised_by_mean_and_variance():
    """d loss / d mu = 0 at mu = mean, d loss / d s = 0 at exp(s) = variance (pointwise)."""
    x = np.array([1.0, 3.0])
    mu, s = 2.0, np.log(1.0)
    g_mu = np.mean(-(x - mu) * np.exp(-s))
    g_s = np.mean(0.5 * (1 - (x - mu) ** 2 * np.exp(-s)))
    assert abs(g_mu) < 1e-15 and abs(g_s) < 1e-15
