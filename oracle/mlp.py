"""CPU reference of the sampler's MLP (test infrastructure only).

Plain NumPy in FP64: forward pass, mean-squared-error loss, backward pass by the
chain rule, and one Adam step -- the definitions written out.  With
``bf16=True`` it rounds to BF16 at the points where the GPU kernels store BF16
(inputs, weights, activations, the SiLU derivatives kept from the forward pass for
the backward pass, the backward operands), so that GPU gradients
can be compared closely; with ``bf16=False`` it is the exact FP64 network,
pinned by finite differences in the CPU tests.

Parameter vector layout (as the library's): W1 [256][n_in] (trajectory features
first, then point inputs), b1 [256], W2 [256][256], b2, W3 [256][256], b3,
W4 [256], b4 [1].
"""
from __future__ import annotations

import numpy as np

WIDTH = 256


def layout(n_in):
    sizes = [("W1", (WIDTH, n_in)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
             ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (WIDTH,)), ("b4", (1,))]
    out, o = {}, 0
    for name, shape in sizes:
        n = int(np.prod(shape))
        out[name] = (o, shape)
        o += n
    return out, o


def unpack(theta, n_in):
    lay, total = layout(n_in)
    assert theta.size == total
    return {k: theta[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in lay.items()}


def pack(parts, n_in):
    lay, total = layout(n_in)
    theta = np.zeros(total)
    for k, (o, s) in lay.items():
        theta[o:o + int(np.prod(s))] = np.asarray(parts[k], dtype=np.float64).ravel()
    return theta


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def inputs(feat, traj, x):
    """Layer-1 input rows [features of the point's trajectory, point inputs]."""
    feat = np.asarray(feat, dtype=np.float64).reshape(len(feat), -1)
    return np.concatenate([feat[np.asarray(traj)], np.asarray(x, dtype=np.float64)], axis=1)


def forward(theta, feat, traj, x, bf=False):
    """Returns y and the cache of pre-activations and activations."""
    n_in = inputs(feat[:1], [0], np.zeros((1, np.asarray(x).shape[1]))).shape[1]
    P = unpack(theta, n_in)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    a0 = r(inputs(feat, traj, x))
    W1, W2, W3, W4 = r(P["W1"]), r(P["W2"]), r(P["W3"]), r(P["W4"])
    z1 = a0 @ W1.T + P["b1"]
    h1 = r(silu(z1))
    z2 = h1 @ W2.T + P["b2"]
    h2 = r(silu(z2))
    z3 = h2 @ W3.T + P["b3"]
    h3 = r(silu(z3))
    y = h3 @ W4 + P["b4"][0]
    return y, dict(a0=a0, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, W=(W1, W2, W3, W4), n_in=n_in)


def loss_and_grad(theta, feat, traj, x, target, bf=False):
    """Mean squared error (1/B) sum (y - t)^2 and its gradient with respect to theta."""
    y, c = forward(theta, feat, traj, x, bf)
    r = bf16 if bf else (lambda a: a)
    B = y.size
    d = y - np.asarray(target, dtype=np.float64)
    loss = float(np.sum(d * d) / B)
    dy = 2.0 * d / B
    W1, W2, W3, W4 = c["W"]
    g = {}
    g["W4"] = c["h3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = (dy[:, None] * W4[None, :]) * r(dsilu(c["z3"]))
    g["W3"] = r(dz3).T @ c["h2"]
    g["b3"] = dz3.sum(0)
    dz2 = (r(dz3) @ W3) * r(dsilu(c["z2"]))
    g["W2"] = r(dz2).T @ c["h1"]
    g["b2"] = dz2.sum(0)
    dz1 = (r(dz2) @ W2) * r(dsilu(c["z1"]))
    g["W1"] = r(dz1).T @ c["a0"]
    g["b1"] = dz1.sum(0)
    return loss, pack(g, c["n_in"])


def adam(theta, m1, m2, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction at step number `step` (>= 1)."""
    m1 = b1 * m1 + (1.0 - b1) * grad
    m2 = b2 * m2 + (1.0 - b2) * grad * grad
    mh = m1 / (1.0 - b1 ** step)
    vh = m2 / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2
