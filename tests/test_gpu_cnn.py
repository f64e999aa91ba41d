"""Corrector network on the GPU against the FP64 oracle (oracle.cnn).

Per-layer parity: the GPU layer is fed BF16 inputs (and BF16-exact
gradients), the oracle evaluates the same convolution in FP64 on the same
values with the BF16-rounded weights; the only difference left is FP32
accumulation order, held to 1e-5 relative to the result's max norm.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import cnn
from paper_0710_5912_amd import inputs

pytestmark = pytest.mark.gpu

le = pytest.importorskip("paper_0710_5912_amd.le")
torch = pytest.importorskip("torch")

H, W = 32, 64
P = H * W


def bf16_bits(x):
    """BF16 bit patterns (RNE) of float values, and the rounded values."""
    r = cnn.bf16_round(x)
    bits = (np.asarray(r, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return bits, r


def dev(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def params_bf16_layers(params):
    """The oracle's layers with weights rounded to BF16 (biases stay FP32)."""
    out = []
    for Wl, b in cnn.unpack(params):
        out.append((cnn.bf16_round(Wl), np.asarray(b, dtype=np.float32).astype(np.float64)))
    return out


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def test_mfma_lane_layout():
    rng = np.random.default_rng(0)
    ab, a = bf16_bits(rng.standard_normal((32, 16)))
    bb, b = bf16_bits(rng.standard_normal((16, 32)))
    c = le.mfma_probe(ab, bb)
    assert rel(c, a @ b) <= 1e-6


@pytest.fixture(scope="module")
def net():
    n = le.Net(H, W)
    params = inputs.cnn_init_params(3) + np.random.default_rng(1).uniform(-0.02, 0.02,
                                                                            cnn.nparams())
    params[576:608] = np.random.default_rng(2).uniform(-0.1, 0.1, 32)   # nonzero biases
    n.set_params(params.astype(np.float32), [1.0, 1.0, 1.0, 1.0])
    n._params = params.astype(np.float32).astype(np.float64)
    yield n
    n.close()


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_forward(net, layer):
    cin, cout = cnn.LAYERS[layer]
    rng = np.random.default_rng(10 + layer)
    bits, a = bf16_bits(rng.standard_normal((P, cin)))
    z = torch.empty((P, cout), dtype=torch.float32, device="cuda")
    ao = torch.empty((P, cout), dtype=torch.int16, device="cuda")
    net.layer_fwd(layer, dev(bits.view(np.int16), torch.int16), z, ao if layer < 3 else None)
    Wl, b = params_bf16_layers(net._params)[layer]
    ref = cnn.conv3x3(a.T.reshape(cin, H, W), Wl, b)          # (cout, H, W)
    got = z.cpu().numpy().astype(np.float64).T.reshape(cout, H, W)
    assert rel(got, ref) <= 1e-5
    if layer < 3:   # the BF16 activation is silu(z) rounded once
        act = ao.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        act = act.view(np.float32).astype(np.float64).T.reshape(cout, H, W)
        want = cnn.bf16_round(cnn.silu(got))
        assert np.max(np.abs(act - want)) <= 2.0 ** -7 * np.max(np.abs(want))


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_backward(net, layer):
    cin, cout = cnn.LAYERS[layer]
    rng = np.random.default_rng(20 + layer)
    abits, a = bf16_bits(rng.standard_normal((P, cin)))
    _, dz = bf16_bits(rng.standard_normal((P, cout)))         # BF16-exact gradients
    zprev = rng.standard_normal((P, cin))
    nw = 9 * cin * cout + cout
    dw = torch.empty(nw, dtype=torch.float32, device="cuda")
    dzp = torch.empty((P, cin), dtype=torch.float32, device="cuda") if layer > 0 else None
    net.layer_bwd(layer, dev(dz), dev(abits.view(np.int16), torch.int16),
                  dev(zprev) if layer > 0 else None, dzp, dw)
    dz_c = dz.T.reshape(cout, H, W)
    a_c = a.T.reshape(cin, H, W)
    dW_ref, db_ref = cnn.conv3x3_dw(dz_c, a_c)
    got = dw.cpu().numpy().astype(np.float64)
    assert rel(got[:9 * cin * cout], dW_ref.ravel()) <= 1e-5
    assert rel(got[9 * cin * cout:], db_ref) <= 1e-5
    if layer > 0:
        Wl, _ = params_bf16_layers(net._params)[layer]
        da = cnn.conv3x3_dx(dz_c, Wl)
        zp = np.asarray(zprev, dtype=np.float32).astype(np.float64).T.reshape(cin, H, W)
        ref = da * cnn.silu_grad(zp)
        gotp = dzp.cpu().numpy().astype(np.float64).T.reshape(cin, H, W)
        assert rel(gotp, ref) <= 1e-5


def test_full_gradient_agrees_with_oracle(net):
    """End to end the GPU keeps activations and MFMA operands in BF16, so
    the gradient agrees with the FP64 oracle to BF16 accuracy (2%)."""
    rng = np.random.default_rng(30)
    xs = rng.standard_normal((2, 2, H, W)) * np.array([0.8, 0.05])[None, :, None, None]
    ts = rng.standard_normal((2, 2, H, W)) * 0.01
    scales = [1.0, 20.0, 0.05, 0.002]
    net.set_params(net._params.astype(np.float32), scales)
    loss, g = net.grad(dev(xs), dev(ts), 2, want_grad=True)
    rparams = np.concatenate([np.concatenate([Wl.ravel(), b]) for Wl, b in
                              params_bf16_layers(net._params)])
    L_ref, g_ref = cnn.loss_and_grad(rparams, list(xs), list(ts), scales)
    assert abs(loss - L_ref) <= 0.02 * L_ref
    cos = float(np.dot(g, g_ref) / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    assert cos >= 0.999
    assert np.linalg.norm(g - g_ref) <= 0.03 * np.linalg.norm(g_ref)
    net.set_params(net._params.astype(np.float32), [1.0, 1.0, 1.0, 1.0])


def test_training_lowers_the_loss():
    """Fit a fixed smooth residual map: the loss keeps falling under Adam."""
    n = le.Net(H, W)
    n.set_params(inputs.cnn_init_params(7).astype(np.float32), [1.0, 1.0, 1.0, 1.0])
    rng = np.random.default_rng(40)
    xs = rng.uniform(-1, 1, (8, 2, H, W))
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    ts = np.stack([0.3 * np.tanh(xs[:, 0]) * np.cos(2 * np.pi * xx / W)[None],
                   0.2 * xs[:, 1] * xs[:, 0]], axis=1)
    X, T = dev(xs), dev(ts)
    first = None
    for it in range(150):
        loss, _ = n.grad(X, T, 8)
        first = loss if first is None else first
        n.adam(3e-3)
    last, _ = n.grad(X, T, 8)
    assert np.isfinite(last) and last <= 0.7 * first, (first, last)
    n.close()


def test_gpu_forward_planes_match_layers(net):
    """The fused forward on planes equals chaining the per-layer kernels."""
    rng = np.random.default_rng(50)
    x = rng.standard_normal((2, H, W)) * np.array([0.7, 0.03])[:, None, None]
    r = torch.empty((2, H, W), dtype=torch.float32, device="cuda")
    net.forward(dev(x), r)
    # chain through the oracle with BF16 rounding of the layer inputs
    rparams = np.concatenate([np.concatenate([Wl.ravel(), b]) for Wl, b in
                              params_bf16_layers(net._params)])
    ref = cnn.forward(rparams, x, (1.0, 1.0, 1.0, 1.0), round_act=cnn.bf16_round)
    assert rel(r.cpu().numpy(), ref) <= 2e-2
