"""Pins for the score-network oracle: library convolution, finite differences, Adam."""
import numpy as np
import torch

import workloads
from oracle import cnn


def test_conv_matches_library_routine():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 16, 16))
    w = rng.standard_normal((7, 5, 3, 3))
    b = rng.standard_normal(7)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), padding=1)
    assert np.allclose(cnn.conv3x3(x, w, b), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_conv_grads_match_library_autograd():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 16, 16))
    w = rng.standard_normal((6, 4, 3, 3))
    gz = rng.standard_normal((2, 6, 16, 16))
    xt = torch.from_numpy(x).requires_grad_()
    wt = torch.from_numpy(w).requires_grad_()
    torch.nn.functional.conv2d(xt, wt, padding=1).backward(torch.from_numpy(gz))
    assert np.allclose(cnn.conv3x3_input_grad(gz, w), xt.grad.numpy(), rtol=1e-12, atol=1e-11)
    assert np.allclose(cnn.conv3x3_weight_grad(gz, x), wt.grad.numpy(), rtol=1e-12, atol=1e-10)


def test_backward_matches_finite_differences():
    p = workloads.cnn_params(3)
    x, lab = workloads.cnn_batch(3, 4)
    y, cache = cnn.forward(p, x)
    g = cnn.backward(p, cache, y, lab)
    rng = np.random.default_rng(5)
    h = 1e-6
    for name in cnn.NAMES:
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in p[name].shape)
            q = {k: v.copy() for k, v in p.items()}
            q[name] = np.array(q[name], dtype=np.float64)
            q[name][idx] += h
            lp = cnn.loss(cnn.forward(q, x)[0], lab)
            q[name][idx] -= 2 * h
            lm = cnn.loss(cnn.forward(q, x)[0], lab)
            fd = (lp - lm) / (2 * h)
            an = float(np.asarray(g[name])[idx])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)


def test_zero_network_outputs_bias():
    p = {k: np.zeros_like(v) for k, v in workloads.cnn_params(0).items()}
    p["b4"] = np.array(0.37)
    x, _ = workloads.cnn_batch(5, 1)
    y, _ = cnn.forward(p, x)
    assert np.allclose(y, 0.37, rtol=0, atol=0)


def test_adam_first_step_is_lr_times_sign():
    p = {k: np.ones_like(v) for k, v in workloads.cnn_params(0).items()}
    rng = np.random.default_rng(2)
    # gradients bounded away from 0 so that eps/|g| stays negligible
    g = {k: np.sign(rng.standard_normal(np.shape(v))) * (0.5 + rng.random(np.shape(v))) for k, v in p.items()}
    opt = cnn.Adam(lr=0.01)
    q = {k: v.copy() for k, v in p.items()}
    opt.step(q, g)
    for k in cnn.NAMES:
        assert np.allclose(q[k] - p[k], -0.01 * np.sign(g[k]), rtol=0, atol=1e-6)


def test_adam_fits_a_tiny_regression():
    p = workloads.cnn_params(7)
    x, _ = workloads.cnn_batch(6, 8)
    lab = 10 * x[:, 0].mean(axis=(1, 2))  # a learnable function of the input
    opt = cnn.Adam(lr=1e-3)
    first = None
    for _ in range(25):
        y, cache = cnn.forward(p, x)
        if first is None:
            first = cnn.loss(y, lab)
        opt.step(p, cnn.backward(p, cache, y, lab))
    assert cnn.loss(cnn.forward(p, x)[0], lab) < 0.5 * first


def test_layer_input_hook_touches_exactly_the_three_convolution_inputs():
    """With zero biases the network is positively homogeneous layer by layer, so doubling the
    input of each of the three convolutions (and nothing else) multiplies y - b4 by exactly 8;
    the cache holds the doubled inputs.  The identity hook changes nothing."""
    import workloads
    p = {k: np.asarray(v, dtype=np.float64) for k, v in workloads.cnn_params(4).items()}
    for k in ("b1", "b2", "b3"):
        p[k] = np.zeros_like(p[k])
    x, _ = workloads.cnn_batch(3, 5)
    y0, c0 = cnn.forward(p, x)
    y1, c1 = cnn.forward(p, x, layer_input=lambda a: a)
    assert np.array_equal(y0, y1)
    y2, c2 = cnn.forward(p, x, layer_input=lambda a: 2.0 * a)
    assert np.allclose(y2 - p["b4"], 8.0 * (y0 - p["b4"]), rtol=1e-13, atol=0)
    assert np.array_equal(c2["x"], 2.0 * x)
    assert np.allclose(c2["a1"], 4.0 * c0["a1"], rtol=1e-14) and np.allclose(c2["a2"], 8.0 * c0["a2"], rtol=1e-14)
