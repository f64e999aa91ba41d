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


def test_tile_mean_field_constant_total_and_subtile_content():
    """A constant plane is reproduced; the total is kept (so the corrected phi
    keeps its mean); content that averages to zero over every 16 x 16 tile
    (a period-16 cosine along x, a period-8 one along y) gives zero."""
    assert np.allclose(cnn.tile_mean_field(np.full((32, 48), 0.37)), 0.37, atol=1e-15, rtol=0)
    a = np.random.default_rng(7).standard_normal((48, 32))
    assert abs(cnn.tile_mean_field(a).sum() - a.sum()) <= 1e-11
    y, x = np.mgrid[0:32, 0:64]
    sub = np.cos(2 * np.pi * x / 16) + np.sin(2 * np.pi * y / 8 + 0.3)
    assert np.max(np.abs(cnn.tile_mean_field(sub))) <= 1e-13


def test_tile_mean_field_hat_is_centred_and_oriented():
    """One tile at 1, the rest at 0 (48 x 32, so rows and columns differ): the
    result is the product of two hats centred on the tile's centre 7.5 in
    both axes, symmetric about it, reaching the neighbouring tiles' centres
    (23.5) at zero, with the tile's own pixels 7 and 8 at (1 - 1/32)^2."""
    a = np.zeros((48, 32))
    a[16:32, 0:16] = 1.0                       # tile row 1, tile column 0
    f = cnn.tile_mean_field(a)
    assert abs(f[23, 7] - (1 - 1 / 32) ** 2) <= 1e-15
    assert abs(f[24, 8] - (1 - 1 / 32) ** 2) <= 1e-15
    for d in range(8):
        assert abs(f[23 - d, 7] - f[24 + d, 7]) <= 1e-15
        assert abs(f[23, 7 - d] - f[23, 8 + d]) <= 1e-15
    assert np.all(f[40:48, :] == 0.0) and np.all(f[0:8, :] == 0.0)   # rows beyond the hat
    # periodic in x (two tiles wide): column 31 lies 8.5 from the centre across
    # the wrap, as column 16 does on the other side
    assert abs(f[23, 31] - f[23, 16]) <= 1e-15 and f[23, 31] > 0.0


def test_tile_mean_field_second_order_on_smooth_planes():
    """On a smooth periodic plane the field converges to the plane itself at
    second order in the tile size over the wavelength (a midpoint mean plus
    linear interpolation)."""
    errs = []
    for n in (256, 512, 1024):
        y, x = np.mgrid[0:n // 4, 0:n]
        a = np.sin(2 * np.pi * x / n + 0.4) + 0.5 * np.cos(2 * np.pi * y / (n // 4))
        errs.append(np.max(np.abs(cnn.tile_mean_field(a) - a)))
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 <= e0 / e1 <= 4.5, errs
