"""Pins of the corrector network's FP64 reference."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import cnn
from paper_0710_5912_amd import inputs


def test_nparams_matches_layer_shapes():
    assert cnn.nparams() == 2 * 32 * 9 + 32 * 32 * 9 * 2 + 32 * 2 * 9 + 32 * 3 + 2
    assert inputs.cnn_init_params(0).size == cnn.nparams()
    assert inputs.CNN_LAYERS == cnn.LAYERS


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3, 5, 6))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    z = cnn.conv3x3(a, W, b)
    H, Wd = 5, 6
    for co in range(2):
        for i in range(H):
            for j in range(Wd):
                s = b[co]
                for ci in range(3):
                    for ky in range(3):
                        for kx in range(3):
                            s += W[co, ci, ky, kx] * a[ci, (i + ky - 1) % H, (j + kx - 1) % Wd]
                assert abs(z[co, i, j] - s) <= 1e-12


def test_conv_matches_library_wrap_correlation():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 8, 8))
    W = rng.standard_normal((3, 4, 3, 3))
    z = cnn.conv3x3(a, W, np.zeros(3))
    for co in range(3):
        ref = sum(ndi.correlate(a[ci], W[co, ci], mode="wrap") for ci in range(4))
        assert np.max(np.abs(z[co] - ref)) <= 1e-12


def test_conv_adjoints():
    """<conv(a), dz> = <a, conv_dx(dz)> and the weight gradient by linearity."""
    rng = np.random.default_rng(2)
    a = rng.standard_normal((4, 6, 7))
    dz = rng.standard_normal((5, 6, 7))
    W = rng.standard_normal((5, 4, 3, 3))
    lhs = np.sum(cnn.conv3x3(a, W, np.zeros(5)) * dz)
    assert abs(lhs - np.sum(a * cnn.conv3x3_dx(dz, W))) <= 1e-10 * abs(lhs)
    dW, db = cnn.conv3x3_dw(dz, a)
    assert abs(lhs - np.sum(W * dW)) <= 1e-10 * abs(lhs)
    assert np.allclose(db, dz.sum(axis=(1, 2)))


def test_silu_and_grad():
    z = np.linspace(-8, 8, 101)
    assert np.allclose(cnn.silu(z), z * torch.sigmoid(torch.tensor(z)).numpy(), atol=1e-15)
    h = 1e-6
    fd = (cnn.silu(z + h) - cnn.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - cnn.silu_grad(z))) <= 1e-8


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(x), ref)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    params = inputs.cnn_init_params(5) + rng.uniform(-0.05, 0.05, cnn.nparams())
    xs = [rng.standard_normal((2, 6, 5)) for _ in range(2)]
    ts = [rng.standard_normal((2, 6, 5)) * 0.1 for _ in range(2)]
    scales = (1.0, 3.0, 0.5, 0.2)
    L, g = cnn.loss_and_grad(params, xs, ts, scales)
    idx = rng.choice(cnn.nparams(), 60, replace=False)
    # every bias and a sample of weights, in every layer
    idx = np.unique(np.concatenate([idx, [576, 576 + 32 + 9216, cnn.nparams() - 1]]))
    h = 1e-6
    for k in idx:
        p1 = params.copy(); p1[k] += h
        p0 = params.copy(); p0[k] -= h
        fd = (cnn.loss_and_grad(p1, xs, ts, scales)[0] - cnn.loss_and_grad(p0, xs, ts, scales)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_restriction_conserves_mean():
    a = np.random.default_rng(6).standard_normal((32, 16))
    c = cnn.restrict4(a)
    assert c.shape == (8, 4)
    assert abs(c.mean() - a.mean()) <= 1e-15
    assert abs(c[1, 2] - a[4:8, 8:12].mean()) <= 1e-15
