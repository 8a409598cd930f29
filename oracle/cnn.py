"""Oracle: the small 3-D CNN of the learned warm start and mass (test infrastructure only).

Four 3x3x3 convolutions with zero padding, 16 hidden channels and GELU,
mapping 3 input channels (normalised data, angular mask, radial selection)
to 2 outputs per voxel: the posterior mean mu and log-variance s of the
density.  The loss is the heteroscedastic Gaussian negative log-likelihood
mean_i 1/2 [(x_i - mu_i)^2 exp(-s_i) + s_i], minimised by the posterior mean
and variance of the training draws x.

Tap t = 9 (dx+1) + 3 (dy+1) + (dz+1), (dx, dy, dz) in {-1, 0, 1}^3; a layer is
z[v, o] = b[o] + sum_t sum_c a[v + d_t, c] W[t, c, o] (correlation, zero
outside the grid).  GELU(z) = z Phi(z) with the exact normal CDF.

With bf16=True the weights and every convolution input (activations on the
forward path, output gradients on the backward path) are rounded to bfloat16
(round to nearest even) where the device kernels round them; sums stay float64.
"""
import numpy as np
from scipy import special

CH = [3, 16, 16, 16, 2]
TAPS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]


def bf16(x):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shifted(a, d):
    """b[v] = a[v + d] with zeros outside (a: [N, N, N, C])."""
    n = a.shape[0]
    out = np.zeros_like(a)
    src = [slice(max(0, k), n + min(0, k)) for k in d]
    dst = [slice(max(0, -k), n + min(0, -k)) for k in d]
    out[dst[0], dst[1], dst[2]] = a[src[0], src[1], src[2]]
    return out


def conv(a, W, b):
    z = np.broadcast_to(b, a.shape[:3] + (W.shape[2],)).astype(np.float64).copy()
    for t, d in enumerate(TAPS):
        z += shifted(a, d) @ W[t]
    return z


def conv_input_grad(dz, W):
    """d/da of sum(dz * conv(a)): correlation of dz with the mirrored taps."""
    da = np.zeros(dz.shape[:3] + (W.shape[1],))
    for t, d in enumerate(TAPS):
        da += shifted(dz, tuple(-k for k in d)) @ W[t].T
    return da


def conv_weight_grad(a, dz):
    dW = np.zeros((27, a.shape[3], dz.shape[3]))
    for t, d in enumerate(TAPS):
        s = shifted(a, d)
        dW[t] = s.reshape(-1, a.shape[3]).T @ dz.reshape(-1, dz.shape[3])
    return dW, dz.reshape(-1, dz.shape[3]).sum(axis=0)


def gelu(z):
    return z * special.ndtr(z)


def gelu_grad(z):
    return special.ndtr(z) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def init_params(seed=0):
    """He-style uniform initialisation (fan-in 27 C_in); biases zero."""
    rng = np.random.default_rng(seed)
    params = []
    for ci, co in zip(CH[:-1], CH[1:]):
        lim = np.sqrt(6.0 / (27 * ci))
        params.append((rng.uniform(-lim, lim, (27, ci, co)), np.zeros(co)))
    return params


def forward(params, x, bf=False):
    """x: [N, N, N, 3].  Returns (mu, s, cache)."""
    r = bf16 if bf else (lambda v: v)
    a = r(x)
    cache = []
    for l, (W, b) in enumerate(params):
        z = conv(a, r(W), b)
        cache.append((a, z))
        a = r(gelu(z)) if l < len(params) - 1 else z
    return a[..., 0], a[..., 1], cache


def loss(mu, s, target):
    return float(np.mean(0.5 * ((target - mu) ** 2 * np.exp(-s) + s)))


def backward(params, cache, mu, s, target, bf=False):
    """Gradients of loss() w.r.t. every (W, b)."""
    r = bf16 if bf else (lambda v: v)
    nv = target.size
    e = np.exp(-s)
    dz = np.zeros(mu.shape + (2,))
    dz[..., 0] = -(target - mu) * e / nv
    dz[..., 1] = 0.5 * (1.0 - (target - mu) ** 2 * e) / nv
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        a_in, _ = cache[l]
        W, _ = params[l]
        dzr = r(dz)
        dW, db = conv_weight_grad(a_in, dzr)
        grads[l] = (dW, db)
        if l > 0:
            da = conv_input_grad(dzr, r(W))
            dz = da * gelu_grad(cache[l - 1][1])
    return grads
