"""The oracle's network evaluated with the surrogate kernels' roundings: every
convolution input (activations, output gradients) and every weight is
rounded to bf16 (round to nearest even, through float32), everything else
in FP64.  Composes the oracle's conv3x3 / conv3x3_grads; used to check the
device kernels to tight tolerances (their remaining differences are FP32
accumulation and epilogue arithmetic)."""
from __future__ import annotations

import numpy as np

from oracle import surrogate as osur


def bf16(a: np.ndarray) -> np.ndarray:
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x, base=None, oscale=1.0):
    layers = [(bf16(W), b) for W, b in osur.unpack(params)]
    cache = {"a": [], "h": [x]}
    W, b = layers[0]
    a = osur.conv3x3(bf16(x), W, b)
    h = osur.silu(a)
    cache["a"].append(a)
    cache["h"].append(h)
    for k in range(1, len(layers) - 1):
        W, b = layers[k]
        a = osur.conv3x3(bf16(h), W, b)
        h = h + osur.silu(a)
        cache["a"].append(a)
        cache["h"].append(h)
    W, b = layers[-1]
    y = (x[:, 0:2] if base is None else base) + oscale * osur.conv3x3(bf16(h), W, b)
    return y, cache, layers


def grad(params, x, target, kind="mse", base=None, oscale=1.0):
    y, cache, layers = forward(params, x, base, oscale)
    nb = len(layers) - 2
    grads = [None] * len(layers)
    dy = oscale * osur.loss_grad(y, target, kind)
    hs, As = cache["h"], cache["a"]
    _, dW, db = osur.conv3x3_grads(bf16(hs[-1]), layers[-1][0], bf16(dy))
    grads[-1] = (dW, db)
    dh, _, _ = osur.conv3x3_grads(hs[-1], layers[-1][0], bf16(dy))
    for k in range(nb, 0, -1):
        da = dh * osur.silu_grad(As[k])
        _, dW, db = osur.conv3x3_grads(bf16(hs[k]), layers[k][0], bf16(da))  # hs[k] = h_{k-1}
        grads[k] = (dW, db)
        dprev, _, _ = osur.conv3x3_grads(hs[k], layers[k][0], bf16(da))
        dh = dh + dprev
    da = dh * osur.silu_grad(As[0])
    _, dW, db = osur.conv3x3_grads(bf16(hs[0]), layers[0][0], bf16(da))
    grads[0] = (dW, db)
    return y, osur.pack(grads), osur.loss(y, target, kind)


def inputs_from_states(u: np.ndarray, cstd: np.ndarray, n1: int, n2: int) -> np.ndarray:
    """u complex (S, P) sample-major with p = i1 + n1 i2; cstd (S, 5)."""
    S = u.shape[0]
    x = np.zeros((S, osur.CIN, n2, n1))
    for s in range(S):
        x[s] = osur.make_input(u[s].reshape(n1, n2, order="F"), cstd[s])
    return x


def planes_to_states(y: np.ndarray) -> np.ndarray:
    """y (S, 2, n2, n1) -> complex (S, P) with p = i1 + n1 i2."""
    S = y.shape[0]
    return (y[:, 0] + 1j * y[:, 1]).reshape(S, -1)
