"""Pins of the FP64 surrogate oracle: the 3x3 convolution against an
independent library correlation, gradients against central finite
differences, the SiLU derivative, Adam's first step, and the parameter count."""
import numpy as np
import pytest
import scipy.signal

from oracle import surrogate as S


def test_param_count_of_the_48_channel_6_layer_net():
    assert S.param_count(48, 4) == 87074


def test_conv3x3_equals_scipy_correlate2d_with_zero_padding():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 6, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = S.conv3x3(x, W, b)
    for s in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(x[s, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.abs(out[s, o] - ref).max() < 1e-12


def test_silu_derivative():
    a = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (S.silu(a + h) - S.silu(a - h)) / (2 * h)
    assert np.abs(S.silu_grad(a) - fd).max() < 1e-8


@pytest.mark.parametrize("kind", ["mse", "rel"])
def test_backward_matches_central_finite_differences(kind):
    C, blocks = 3, 2
    rng = np.random.default_rng(1)
    params = S.init_params(2, C, blocks) + 0.05 * rng.standard_normal(S.param_count(C, blocks))
    x = rng.standard_normal((2, 7, 5, 6))
    target = rng.standard_normal((2, 2, 5, 6)) * np.array([1.0, 0.01])[:, None, None, None]
    y, cache = S.forward(params, x, C, blocks)
    g = S.backward(params, cache, y, target, C, blocks, kind=kind)
    h = 1e-6
    fd = np.zeros_like(params)
    for i in range(params.size):
        e = np.zeros_like(params)
        e[i] = h
        fd[i] = (S.loss(S.forward(params + e, x, C, blocks)[0], target, kind)
                 - S.loss(S.forward(params - e, x, C, blocks)[0], target, kind)) / (2 * h)
    assert np.abs(g - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())


def test_backward_with_a_base_and_an_output_scale_matches_finite_differences():
    """y = base + s d: the gradient carries the factor s and no dependence on
    the base (checked against central differences of the loss itself)."""
    C, blocks, s = 3, 1, 0.03
    rng = np.random.default_rng(5)
    params = S.init_params(6, C, blocks) + 0.05 * rng.standard_normal(S.param_count(C, blocks))
    x = rng.standard_normal((2, 7, 4, 5))
    base = rng.standard_normal((2, 2, 4, 5))
    target = base + 0.02 * rng.standard_normal((2, 2, 4, 5))
    y, cache = S.forward(params, x, C, blocks, base=base, oscale=s)
    g = S.backward(params, cache, y, target, C, blocks, oscale=s)
    h = 1e-6
    fd = np.zeros_like(params)
    for i in range(params.size):
        e = np.zeros_like(params)
        e[i] = h
        fd[i] = (S.loss(S.forward(params + e, x, C, blocks, base=base, oscale=s)[0], target)
                 - S.loss(S.forward(params - e, x, C, blocks, base=base, oscale=s)[0], target)) / (2 * h)
    assert np.abs(g - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())
    # the base enters additively: a shifted base shifts y and nothing else
    y2, _ = S.forward(params, x, C, blocks, base=base + 1.5, oscale=s)
    assert np.allclose(y2 - y, 1.5, atol=1e-12)


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    q, m, v = S.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(q, p - 0.01 * g / (np.abs(g) + 1e-8))


def test_identity_net_returns_its_input_state():
    """With zero output weights and biases the network is the identity on u."""
    C, blocks = 4, 1
    params = S.init_params(3, C, blocks)
    layers = S.unpack(params, C, blocks)
    layers[-1] = (np.zeros_like(layers[-1][0]), np.zeros(2))
    x = np.random.default_rng(4).standard_normal((1, 7, 4, 5))
    y, _ = S.forward(S.pack(layers), x, C, blocks)
    assert np.array_equal(y, x[:, 0:2])


def test_relative_loss_closed_forms():
    """y = (1 + e_s) t per sample gives the mean of e_s^2, whatever the scale
    of t; with equal target norms it is the mean square divided by the mean
    square of the target."""
    rng = np.random.default_rng(5)
    t = rng.standard_normal((3, 2, 4, 6)) * np.array([1e-3, 1.0, 50.0])[:, None, None, None]
    e = np.array([0.1, -0.02, 0.3])
    y = t * (1.0 + e)[:, None, None, None]
    assert abs(S.loss(y, t, "rel") - np.mean(e ** 2)) < 1e-14
    t2 = rng.standard_normal((2, 2, 4, 6))
    t2[1] *= np.sqrt(np.sum(t2[0] ** 2) / np.sum(t2[1] ** 2))
    y2 = t2 + 0.1 * rng.standard_normal(t2.shape)
    assert abs(S.loss(y2, t2, "rel") - S.loss(y2, t2) / np.mean(t2 ** 2)) < 1e-12
