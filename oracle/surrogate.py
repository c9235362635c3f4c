"""FP64 residual CNN surrogate (oracle; test infrastructure only).

The paper has no learned component; this is the reference for the
surrogate the library trains on the GPU: a map u(t) -> u(t + M tau) on a
2-D grid, gated at run time by the plain stepper.

Network (C = 48 channels, 3x3 kernels, zero padding, pixel p = i1 + n1 i2):
    x   = [Re u, Im u, five standardised coefficient planes]     (7 channels)
    h0  = silu(conv_in(x))                                        (7 -> C)
    h_k = h_{k-1} + silu(conv_k(h_{k-1})),  k = 1..4               (C -> C)
    d   = conv_out(h_4)                                           (C -> 2)
    y   = (Re b, Im b) + s d,  b = u, or a base state the caller gives; s the
          output scale (1 unless given)
The base b is where the network's correction starts from: the input itself,
or a cheap propagation of it (the exact linear flow e^{M tau K} u of the
Lawson change of variables, Section 2.2, or one Strang step of size M tau);
it does not depend on the parameters, so the gradients do not involve it.
silu(a) = a sigmoid(a).  Loss "mse": mean over samples, channels and pixels
of (y - target)^2; loss "rel": mean over samples of the squared relative L2
error sum (y - target)^2 / sum target^2 (sums over channels and pixels).  Parameters are packed in the order W_in, b_in, W_1, b_1,
..., W_4, b_4, W_out, b_out with W[co, ci, ky, kx] (ky along i2, kx along i1).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

CIN = 7


def layer_shapes(C: int = 48, blocks: int = 4) -> List[Tuple[int, int]]:
    return [(C, CIN)] + [(C, C)] * blocks + [(2, C)]


def param_count(C: int = 48, blocks: int = 4) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(C, blocks))


def unpack(params: np.ndarray, C: int = 48, blocks: int = 4):
    out = []
    o = 0
    for co, ci in layer_shapes(C, blocks):
        W = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out.append((W, b))
    assert o == params.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed: int, C: int = 48, blocks: int = 4) -> np.ndarray:
    """He-uniform weights scaled down in the residual and output layers, zero biases."""
    rng = np.random.default_rng(seed)
    layers = []
    shapes = layer_shapes(C, blocks)
    for k, (co, ci) in enumerate(shapes):
        bound = np.sqrt(6.0 / (ci * 9))
        scale = 1.0 if k == 0 else 0.1
        W = scale * rng.uniform(-bound, bound, size=(co, ci, 3, 3))
        layers.append((W, np.zeros(co)))
    return pack(layers)


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[s, co, i2, i1] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] x[s, ci, i2+ky-1, i1+kx-1],
    zero outside the grid.  x: (S, ci, n2, n1)."""
    S, ci, n2, n1 = x.shape
    xp = np.zeros((S, ci, n2 + 2, n1 + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((S, W.shape[0], n2, n1))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,scyx->soyx", W[:, :, ky, kx], xp[:, :, ky:ky + n2, kx:kx + n1])
    return out + b[None, :, None, None]


def conv3x3_grads(x: np.ndarray, W: np.ndarray, dout: np.ndarray):
    """Gradients of sum(dout * conv3x3(x, W, b)) with respect to x, W and b."""
    S, ci, n2, n1 = x.shape
    xp = np.zeros((S, ci, n2 + 2, n1 + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.einsum("soyx,scyx->oc", dout, xp[:, :, ky:ky + n2, kx:kx + n1])
            dxp[:, :, ky:ky + n2, kx:kx + n1] += np.einsum("oc,soyx->scyx", W[:, :, ky, kx], dout)
    db = dout.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dW, db


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def silu(a):
    return a * sigmoid(a)


def silu_grad(a):
    s = sigmoid(a)
    return s * (1.0 + a * (1.0 - s))


def forward(params: np.ndarray, x: np.ndarray, C: int = 48, blocks: int = 4, base=None,
            oscale: float = 1.0):
    """x: (S, 7, n2, n1); base: None (the input's planes 0, 1) or (S, 2, n2, n1).
    Returns y (S, 2, n2, n1) and the cache for backward."""
    layers = unpack(params, C, blocks)
    cache: Dict[str, list] = {"a": [], "h": [x]}
    W, b = layers[0]
    a = conv3x3(x, W, b)
    h = silu(a)
    cache["a"].append(a)
    cache["h"].append(h)
    for k in range(1, blocks + 1):
        W, b = layers[k]
        a = conv3x3(h, W, b)
        h = h + silu(a)
        cache["a"].append(a)
        cache["h"].append(h)
    W, b = layers[-1]
    d = conv3x3(h, W, b)
    y = (x[:, 0:2] if base is None else base) + oscale * d
    return y, cache


def loss(y: np.ndarray, target: np.ndarray, kind: str = "mse") -> float:
    if kind == "mse":
        return float(np.mean((y - target) ** 2))
    num = np.sum((y - target) ** 2, axis=(1, 2, 3))
    den = np.sum(target ** 2, axis=(1, 2, 3))
    return float(np.mean(num / den))


def loss_grad(y: np.ndarray, target: np.ndarray, kind: str = "mse") -> np.ndarray:
    """d loss / d y."""
    if kind == "mse":
        return 2.0 * (y - target) / y.size
    den = np.sum(target ** 2, axis=(1, 2, 3))
    return 2.0 * (y - target) / (y.shape[0] * den[:, None, None, None])


def backward(params: np.ndarray, cache, y: np.ndarray, target: np.ndarray, C: int = 48,
             blocks: int = 4, kind: str = "mse", oscale: float = 1.0) -> np.ndarray:
    """Gradient of loss(y, target, kind) with respect to the packed parameters
    (y = base + oscale d: the output conv receives oscale dloss/dy)."""
    layers = unpack(params, C, blocks)
    grads = [None] * len(layers)
    dy = oscale * loss_grad(y, target, kind)
    hs, As = cache["h"], cache["a"]
    # output conv: d = conv_out(h_last)
    dh, dW, db = conv3x3_grads(hs[-1], layers[-1][0], dy)
    grads[-1] = (dW, db)
    for k in range(blocks, 0, -1):  # h_k = h_{k-1} + silu(a_k), a_k = conv_k(h_{k-1})
        da = dh * silu_grad(As[k])
        dprev, dW, db = conv3x3_grads(hs[k], layers[k][0], da)
        grads[k] = (dW, db)
        dh = dh + dprev
    da = dh * silu_grad(As[0])  # h_0 = silu(a_0), a_0 = conv_in(x)
    _, dW, db = conv3x3_grads(hs[0], layers[0][0], da)
    grads[0] = (dW, db)
    return pack(grads)


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of FP64 arrays; returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def standardise_coeffs(c, ranges) -> np.ndarray:
    """Map (a1, b1, a2, a3, b3) to [-1, 1] using the sweep's ranges."""
    keys = ["a1", "b1", "a2", "a3", "b3"]
    vals = [c.a1, c.b1, c.a2, c.a3, c.b3]
    return np.array([2.0 * (v - ranges[k][0]) / (ranges[k][1] - ranges[k][0]) - 1.0
                     for k, v in zip(keys, vals)])


def make_input(u: np.ndarray, coeff_std: np.ndarray) -> np.ndarray:
    """x for one state u (n1, n2): planes (2 + 5, n2, n1)."""
    n1, n2 = u.shape
    x = np.zeros((CIN, n2, n1))
    x[0] = u.real.T
    x[1] = u.imag.T
    for k in range(5):
        x[2 + k] = coeff_std[k]
    return x
