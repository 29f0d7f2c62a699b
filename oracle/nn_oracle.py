"""CPU oracle for the learned proposal network (float64 NumPy).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU library neither imports nor links it.

The proposal network is not part of the paper: it is the production extension
that predicts an initial plane per pixel so that the PatchMatch iterations
(Sec. 3) start from a good hypothesis instead of a random one.  The paper's
pieces it reuses are the matching cost (Eq. 8, through ``oracle.matching_cost``)
and the confidence mapping C(m) = exp(-m^2 / (2 beta^2)) (Eq. 3), which turns a
final matching cost into the confidence target.

What this module computes, in plain float64 with no blocking or fusion:
  * 3x3 convolution with zero padding (and 1x1 for the head), bias, ReLU;
  * 2x2 average pooling, nearest 2x upsampling, channel concatenation;
  * the 4-level encoder-decoder built from them (channels 16/32/48/64);
  * the decoded outputs: depth as a bounded correction of the plane sweep's
    winning inverse depth (a refinement head over the sweep, in [d_min, d_max]),
    unit normal, confidence;
  * the training loss: L1 on normalised depth + (1 - n_hat . n) + binary
    cross-entropy of the confidence, its gradient, the backward pass of every
    layer, and one Adam step (Kingma and Ba, 2015) on float64 master weights.

Pins (tests/test_oracle_nn.py): convolution, pooling and upsampling against
torch's float64 CPU routines; every backward against torch autograd and central
finite differences; the loss against finite differences and closed forms; Adam
against its closed-form first step and torch.optim.Adam.  The network's
*trained result* is parity unpinned: it is checked against ground-truth depth.

Layout: activations are NHWC float64 arrays (n, h, w, c); a 3x3 weight is
(c_out, 3, 3, c_in) with tap (ky, kx) reading input pixel (y + ky - 1,
x + kx - 1); the 1x1 head weight is (c_out, 1, 1, c_in).  The canonical flat
parameter order is, layer by layer, the weight in that layout then the bias.
"""
from __future__ import annotations

import numpy as np

# (name, c_in, c_out, kernel size), in canonical parameter order.  The
# decoder's input is the concatenation [upsampled deeper features, skip].
LAYERS = (
    ("enc0a", 16, 16, 3), ("enc0b", 16, 16, 3),
    ("enc1a", 16, 32, 3), ("enc1b", 32, 32, 3),
    ("enc2a", 32, 48, 3), ("enc2b", 48, 48, 3),
    ("enc3a", 48, 64, 3), ("enc3b", 64, 64, 3),
    ("dec2", 112, 48, 3), ("dec1", 80, 32, 3), ("dec0", 48, 16, 3),
    ("head", 16, 5, 1),
)
IN_CHANNELS = 16
OUT_CHANNELS = 5


def param_count() -> int:
    return sum(co * k * k * ci + co for _, ci, co, k in LAYERS)


def unflatten(theta):
    """Flat canonical vector -> {name: (W, b)} (views into a float64 copy)."""
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for name, ci, co, k in LAYERS:
        nw = co * k * k * ci
        out[name] = (theta[o:o + nw].reshape(co, k, k, ci), theta[o + nw:o + nw + co])
        o += nw + co
    assert o == theta.size, "parameter vector has the wrong length"
    return out


def flatten(params) -> np.ndarray:
    parts = []
    for name, _, _, _ in LAYERS:
        W, b = params[name]
        parts += [np.ravel(W), np.ravel(b)]
    return np.concatenate(parts).astype(np.float64)


# --------------------------------------------------------------------------------------
# layers
# --------------------------------------------------------------------------------------

def conv(x, W, b):
    """y[n, i, j, o] = b[o] + sum_{ky, kx, c} x[n, i + ky - r, j + kx - r, c] W[o, ky, kx, c],
    with x = 0 outside the image and r = k // 2 (same-size output)."""
    k = W.shape[1]
    r = k // 2
    n, h, w, _ = x.shape
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    y = np.broadcast_to(b, (n, h, w, W.shape[0])).copy()
    for ky in range(k):
        for kx in range(k):
            y += xp[:, ky:ky + h, kx:kx + w, :] @ W[:, ky, kx, :].T
    return y


def conv_backward(x, W, g):
    """Gradients of sum(g * conv(x, W, b)) with respect to x, W and b."""
    k = W.shape[1]
    r = k // 2
    n, h, w, _ = x.shape
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            win = xp[:, ky:ky + h, kx:kx + w, :]
            dW[:, ky, kx, :] = np.einsum("nijo,nijc->oc", g, win)
            dxp[:, ky:ky + h, kx:kx + w, :] += g @ W[:, ky, kx, :]
    db = g.sum(axis=(0, 1, 2))
    return dxp[:, r:r + h, r:r + w, :], dW, db


def relu(x):
    return np.maximum(x, 0.0)


def pool(x):
    """2x2 average pooling (h and w even)."""
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) * 0.25


def up(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(g):
    n, h, w, c = g.shape
    return g.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


# --------------------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------------------

def forward(params, x):
    """Returns (z, cache): z is the head output (n, h, w, 5) before decoding."""
    a = {"x": x}

    def cr(name, inp):
        W, b = params[name]
        return relu(conv(inp, W, b))

    a["e0a"] = cr("enc0a", x)
    a["e0"] = cr("enc0b", a["e0a"])
    a["e1a"] = cr("enc1a", pool(a["e0"]))
    a["e1"] = cr("enc1b", a["e1a"])
    a["e2a"] = cr("enc2a", pool(a["e1"]))
    a["e2"] = cr("enc2b", a["e2a"])
    a["e3a"] = cr("enc3a", pool(a["e2"]))
    a["e3"] = cr("enc3b", a["e3a"])
    a["c2"] = np.concatenate([up(a["e3"]), a["e2"]], axis=3)
    a["d2"] = cr("dec2", a["c2"])
    a["c1"] = np.concatenate([up(a["d2"]), a["e1"]], axis=3)
    a["d1"] = cr("dec1", a["c1"])
    a["c0"] = np.concatenate([up(a["d1"]), a["e0"]], axis=3)
    a["d0"] = cr("dec0", a["c0"])
    W, b = params["head"]
    z = conv(a["d0"], W, b)
    return z, a


def backward(params, a, dz):
    """Gradients {name: (dW, db)} of sum(dz * z) for the forward pass that made cache ``a``."""
    grads = {}

    def back(name, inp, out, g_out):
        # g_out: gradient w.r.t. the post-ReLU output ``out``
        g = g_out * (out > 0)
        dx, dW, db = conv_backward(inp, params[name][0], g)
        grads[name] = (dW, db)
        return dx

    dx, dW, db = conv_backward(a["d0"], params["head"][0], dz)
    grads["head"] = (dW, db)
    dc0 = back("dec0", a["c0"], a["d0"], dx)
    d1c = a["d1"].shape[3]
    dd1, de0 = up_backward(dc0[..., :d1c]), dc0[..., d1c:]
    dc1 = back("dec1", a["c1"], a["d1"], dd1)
    d2c = a["d2"].shape[3]
    dd2, de1 = up_backward(dc1[..., :d2c]), dc1[..., d2c:]
    dc2 = back("dec2", a["c2"], a["d2"], dd2)
    e3c = a["e3"].shape[3]
    de3, de2 = up_backward(dc2[..., :e3c]), dc2[..., e3c:]
    g = back("enc3b", a["e3a"], a["e3"], de3)
    g = back("enc3a", pool(a["e2"]), a["e3a"], g)
    de2 = de2 + pool_backward(g)
    g = back("enc2b", a["e2a"], a["e2"], de2)
    g = back("enc2a", pool(a["e1"]), a["e2a"], g)
    de1 = de1 + pool_backward(g)
    g = back("enc1b", a["e1a"], a["e1"], de1)
    g = back("enc1a", pool(a["e0"]), a["e1a"], g)
    de0 = de0 + pool_backward(g)
    g = back("enc0b", a["e0a"], a["e0"], de0)
    back("enc0a", a["x"], a["e0a"], g)
    return grads


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def inverse_depth(z0, q_ref, d_min: float, d_max: float):
    """Depth head: the sweep's winning inverse depth q_ref moved by at most one twelfth of
    the inverse-depth range, q = clamp(q_ref + R tanh(z0), 1/d_max, 1/d_min), R = (1/d_min
    - 1/d_max) / 12.  Returns (q, dq/dz0) with the derivative 0 where the clamp binds."""
    qf, qn = 1.0 / d_max, 1.0 / d_min
    R = (qn - qf) / 12.0
    th = np.tanh(z0)
    u = q_ref + R * th
    q = np.clip(u, qf, qn)
    dq = np.where((u > qf) & (u < qn), R * (1.0 - th * th), 0.0)
    return q, dq


def decode(z, q_ref, d_min: float, d_max: float):
    """(depth, unit normal, confidence) from the head output and the sweep's inverse depth."""
    q, _ = inverse_depth(z[..., 0], q_ref, d_min, d_max)
    nv = z[..., 1:4]
    normal = nv / np.linalg.norm(nv, axis=-1, keepdims=True)
    return 1.0 / q, normal, sigmoid(z[..., 4])


def confidence_target(cost, beta: float = 0.3):
    """C(m) of Eq. (3) applied to a final matching cost."""
    return np.exp(-np.asarray(cost, np.float64) ** 2 / (2.0 * beta * beta))


def loss(z, q_ref, target, d_min: float, d_max: float):
    """Mean over pixels of  w (|s - t_d| + 1 - n_hat . n_t) + BCE(sigmoid(z4), t_c).

    target (n, h, w, 6): depth, normal (3), confidence target, weight w of the
    depth and normal terms.  s = (depth - d_min) / (d_max - d_min) of the decoded
    depth, t_d the same of the target depth.  Returns (loss, dL/dz); the gradient
    of |.| at 0 is taken as 0."""
    P = z.shape[0] * z.shape[1] * z.shape[2]
    q, dq = inverse_depth(z[..., 0], q_ref, d_min, d_max)
    span = d_max - d_min
    s = (1.0 / q - d_min) / span
    td = (target[..., 0] - d_min) / span
    w = target[..., 5]
    nv = z[..., 1:4]
    nn = np.linalg.norm(nv, axis=-1)
    nh = nv / nn[..., None]
    nt = target[..., 1:4]
    cosang = (nh * nt).sum(-1)
    z4, tc = z[..., 4], target[..., 4]
    bce = np.logaddexp(0.0, z4) - tc * z4
    L = (w * (np.abs(s - td) + 1.0 - cosang) + bce).sum() / P
    dz = np.zeros_like(z)
    dz[..., 0] = w * np.sign(s - td) * (-1.0 / (q * q * span)) * dq
    dz[..., 1:4] = -(w / nn)[..., None] * (nt - cosang[..., None] * nh)
    dz[..., 4] = sigmoid(z4) - tc
    return L, dz / P


def loss_and_grads(theta, x, q_ref, target, d_min: float, d_max: float):
    """Loss and flat canonical gradient of the whole network at parameters ``theta``."""
    params = unflatten(theta)
    z, a = forward(params, x)
    L, dz = loss(z, q_ref, target, d_min, d_max)
    return L, flatten(backward(params, a, dz))


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1).  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even), returned as float64.
    Used to describe what the GPU's bf16 storage keeps of a value."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)
