"""GPU parity of the MFMA CNN (forward, gradients) with the float64 oracle at bf16 rounding points."""
import numpy as np
import pytest
from scipy import special

from oracle import cnn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1821_amd.binding import CNN, cnn_flatten, cnn_unflatten  # noqa: E402


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def case(n, seed):
    rng = np.random.default_rng(seed)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in cnn.init_params(seed)]
    x = rng.standard_normal((n, n, n, 3))
    target = rng.standard_normal((n, n, n))
    # the device takes float32 parameters: round them first so both sides start equal
    params = cnn_unflatten(cnn_flatten(params).astype(np.float64))
    return params, x, target


# End to end the two sides differ by more than float32 accumulation error: where
# a sum lands within its float32 error of a bf16 rounding tie, the two sides round
# it to neighbouring bf16 values (a relative jump of 2^-8 to 2^-7), and the next
# layer sees that jump and rounds near other ties differently in turn.  An upstream
# relative deviation s flips a fraction ~ s / 2^-8 of the next layer's roundings,
# so the deviation grows from ~1e-7 (one float32 sum) through the three activation
# layers to ~1e-4 at the outputs (measured 0.9e-6 - 2.2e-4 at 8^3 - 128^3), and
# through the further rounding points of the backward pass to ~1e-3 in the
# smallest grids' weight gradients (measured up to 2.0e-3 at 8^3, where a gradient
# sums few voxels; 1.7e-4 at 64^3).  The bounds below are about 4 and 2.5 times
# the largest measured; test_layers_match_oracle_from_their_own_inputs checks
# each layer from its own inputs, where the float32 sums agree to ~1e-7.
FWD_TOL, GRAD_TOL = 1e-3, 5e-3


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_forward_matches_oracle(n):
    params, x, target = case(n, n)
    net = CNN(params)
    mu, lv = net.forward(np.moveaxis(x, -1, 0))
    rmu, rs, _ = cnn.forward(params, x.astype(np.float32).astype(np.float64), bf=True)
    e1, e2 = rel(mu.cpu().numpy(), rmu), rel(lv.cpu().numpy(), rs)
    print(f"N={n}: forward rel-L2 mu {e1:.2e} logvar {e2:.2e}")
    assert e1 < FWD_TOL and e2 < FWD_TOL
    net.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [8, 16, 32, 64])     # 64^3: more bricks than weight-gradient blocks
def test_gradients_match_oracle(n):
    params, x, target = case(n, 100 + n)
    net = CNN(params)
    g, loss = net.gradient(np.moveaxis(x, -1, 0), target)
    xx = x.astype(np.float32).astype(np.float64)
    tt = target.astype(np.float32).astype(np.float64)
    mu, s, cache = cnn.forward(params, xx, bf=True)
    ref = cnn_flatten(cnn.backward(params, cache, mu, s, tt, bf=True)).astype(np.float64)
    assert abs(loss - cnn.loss(mu, s, tt)) < 1e-4 * abs(loss)
    gl = cnn_unflatten(g)
    rl = cnn_unflatten(ref)
    for l in range(4):
        eW, eb = rel(gl[l][0], rl[l][0]), rel(gl[l][1], rl[l][1])
        print(f"N={n} layer {l}: dW rel-L2 {eW:.2e} db {eb:.2e}")
        assert eW < GRAD_TOL and eb < GRAD_TOL
    net.close()


def bf16_ulp(x):
    """Spacing of bfloat16 values at |x| (8 significant bits)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    e = np.floor(np.log2(np.where(x > 0, x, 1.0)))
    return np.where(x > 0, 2.0 ** (e - 7), 2.0 ** -133)


def rounding_flips(got, want, slack=0.0):
    """Fraction of entries where two bf16-rounded arrays differ.  Each difference
    must be what rounding the same value computed two ways can give: at most one
    bf16 step plus `slack`, a bound on the difference of the two unrounded values
    (float32 against float64 arithmetic)."""
    d = np.abs(got - want)
    bad = d > 0
    lim = 1.0001 * bf16_ulp(np.maximum(np.abs(got), np.abs(want))) + slack
    over = bad & (d > np.broadcast_to(lim, d.shape))
    i = np.argmax(np.where(over, d / np.maximum(np.broadcast_to(lim, d.shape), 1e-300), 0))
    assert not over.any(), (int(over.sum()), float(got.flat[i]), float(want.flat[i]),
                            float(np.broadcast_to(lim, d.shape).flat[i]))
    return float(bad.mean())


# float32 accumulation of the 27 x 16 products of one output: at most
# gamma_432 = 432 u / (1 - 432 u) < 3e-5 of the sum of their magnitudes
ACC_BOUND = 3e-5


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_layers_match_oracle_from_their_own_inputs(n):
    """Each layer against the oracle fed with that layer's own device inputs.

    The network's rounding points are its bf16 weights, activations and output
    gradients; in between both sides sum exactly the same bf16 products, the
    device in float32 and the oracle in float64.  Fed with the device's own
    inputs, each float32 quantity (pre-activations z, weight and bias gradients)
    must agree to float32 accumulation error, and each bf16 quantity must be the
    bf16 rounding of the oracle's value except where the two sums fall on either
    side of a rounding tie (a one-step flip, in a small fraction of entries).
    Gradients at 64^3 walk more bricks than the weight-gradient kernel has blocks."""
    params, x, target = case(n, 200 + n)
    net = CNN(params)
    g, loss = net.gradient(np.moveaxis(x, -1, 0), target)
    gl = cnn_unflatten(g)
    nv = n ** 3
    st = [net.layer_state(l, n) for l in range(4)]
    a_in = cnn.bf16(x.astype(np.float32).astype(np.float64))
    for l, (W, b) in enumerate(params):
        z, a, dz = st[l]
        zr = cnn.conv(a_in, cnn.bf16(W), b).reshape(nv, -1)
        ez = rel(z, zr)
        if a is not None:
            # GELU of the device's own z: its float32 evaluation, a few units of u
            fa = rounding_flips(a, cnn.bf16(cnn.gelu(z)), 1e-6 * np.abs(cnn.gelu(z)))
        else:
            fa = 0.0
        # weight and bias gradients from the device's activations and output gradient
        dWr, dbr = cnn.conv_weight_grad(a_in, dz.reshape(n, n, n, -1))
        eW, eb = rel(gl[l][0], dWr), rel(gl[l][1], dbr)
        print(f"N={n} layer {l}: z rel-L2 {ez:.2e}, activation flips {fa:.1e}, "
              f"dW rel-L2 {eW:.2e}, db rel-L2 {eb:.2e}", flush=True)
        assert ez < 1e-5 and eW < 1e-4 and eb < 1e-4
        assert fa < 2e-3
        if l > 0:
            # the output gradient of the layer below, from this layer's
            zp = st[l - 1][0].reshape(n, n, n, -1)
            dz4 = dz.reshape(n, n, n, -1)
            da = cnn.conv_input_grad(dz4, cnn.bf16(W))
            exact = da * cnn.gelu_grad(zp)
            # a sum that cancels keeps its absolute float32 error: bound it by the sum
            # of magnitudes; the GELU derivative Phi(z) + z phi(z) cancels too (it
            # vanishes near z = -0.75), so its float32 error is a few units of u of
            # |Phi(z)| + |z phi(z)|, not of its value
            terms = np.abs(special.ndtr(zp)) + np.abs(zp) * np.exp(-0.5 * zp * zp) / np.sqrt(2 * np.pi)
            slack = (ACC_BOUND * cnn.conv_input_grad(np.abs(dz4), np.abs(cnn.bf16(W)))
                     * np.abs(cnn.gelu_grad(zp)) + 1e-6 * np.abs(da) * terms)
            fd = rounding_flips(st[l - 1][2], cnn.bf16(exact).reshape(nv, -1), slack.reshape(nv, -1))
            print(f"N={n} layer {l - 1}: output-gradient flips {fd:.1e}", flush=True)
            assert fd < 2e-3
        if a is not None:
            a_in = a.reshape(n, n, n, -1)
    # the loss gradient at the output, from the device's outputs
    z3 = st[3][0]
    tt = target.astype(np.float32).astype(np.float64).ravel()
    e = np.exp(-z3[:, 1])
    d = tt - z3[:, 0]
    g3 = np.stack([-d * e / nv, 0.5 * (1.0 - d * d * e) / nv], axis=1)
    # float32 arithmetic: a few units of u of the magnitudes that enter, including
    # those of t - mu and 1 - d^2 e, which cancel
    big = np.abs(tt) + np.abs(z3[:, 0])
    slack3 = 1e-6 * np.stack([(np.abs(d) + big) * e,
                              0.5 * (1.0 + d * d * e + 2.0 * np.abs(d) * big * e)], axis=1) / nv
    f3 = rounding_flips(st[3][2], cnn.bf16(g3), slack3)
    print(f"N={n} output gradient flips {f3:.1e}", flush=True)
    assert f3 < 2e-3
    net.close()


def test_training_lowers_the_loss():
    """Fit mu, s to draws x = m + sqrt(v) eps with known smooth m and v."""
    n = 16
    rng = np.random.default_rng(9)
    c = np.linspace(-1, 1, n)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    inputs = np.stack([X, Y, Z]).astype(np.float32)
    m = 0.5 * X - 0.3 * Y
    v = np.exp(-1.0 + 0.5 * Z)
    net = CNN(cnn.init_params(1))
    losses = []
    for step in range(300):
        draw = (m + np.sqrt(v) * rng.standard_normal(m.shape)).astype(np.float32)
        losses.append(net.train_step(inputs, draw, 3e-3))
    print("loss", losses[0], "->", np.mean(losses[-20:]))
    assert np.mean(losses[-20:]) < losses[0] - 0.2
    mu, lv = net.forward(inputs)
    assert rel(mu.cpu().numpy(), m) < 0.3
    net.close()
