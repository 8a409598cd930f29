"""GPU parity of the MFMA CNN (forward, gradients) with the float64 oracle at bf16 rounding points."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_forward_matches_oracle(n):
    params, x, target = case(n, n)
    net = CNN(params)
    mu, lv = net.forward(np.moveaxis(x, -1, 0))
    rmu, rs, _ = cnn.forward(params, x.astype(np.float32).astype(np.float64), bf=True)
    e1, e2 = rel(mu.cpu().numpy(), rmu), rel(lv.cpu().numpy(), rs)
    print(f"N={n}: forward rel-L2 mu {e1:.2e} logvar {e2:.2e}")
    assert e1 < 2e-3 and e2 < 2e-3
    net.close()


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
        assert eW < 2e-2 and eb < 2e-2
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
