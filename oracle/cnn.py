"""FP64 reference of the learned coarse-step corrector's network.

TEST INFRASTRUCTURE ONLY (see the header of oracle.model_h).

The corrector is not in the paper: it is a small convolutional network that
maps a coarse state u* = (phi*, omega*), already advanced by one plain coarse
step, to a residual r that is added to it.  Layers: four 3x3 convolutions
2 -> 32 -> 32 -> 32 -> 2 with SiLU between them, circular (periodic) padding,
which is the cosheared frame's boundary condition.  Inputs and outputs carry
fixed per-channel scales: a0 = (phi* s_in0, omega* s_in1), r = (z4_0 s_out0,
z4_1 s_out1).

Parameter vector layout (float): for each layer, W[co][ci][ky][kx] then b[co].
Convolution convention (cross-correlation):
    z[co][i][j] = b[co] + sum_{ci,ky,kx} W[co][ci][ky][kx] a[ci][i+ky-1][j+kx-1]
with indices taken modulo the grid.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((2, 32), (32, 32), (32, 32), (32, 2))


def nparams() -> int:
    return sum(9 * ci * co + co for ci, co in LAYERS)


def unpack(params):
    out, k = [], 0
    for ci, co in LAYERS:
        W = np.asarray(params[k:k + 9 * ci * co], dtype=np.float64).reshape(co, ci, 3, 3)
        k += 9 * ci * co
        b = np.asarray(params[k:k + co], dtype=np.float64)
        k += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def shifted(a, dy, dx):
    """shifted(a, dy, dx)[..., i, j] = a[..., i+dy, j+dx] (periodic)."""
    return np.roll(a, (-dy, -dx), axis=(-2, -1))


def conv3x3(a, W, b):
    """a: (Cin, H, Wd) -> (Cout, H, Wd)."""
    co = W.shape[0]
    z = np.broadcast_to(b[:, None, None], (co,) + a.shape[1:]).copy()
    for ky in range(3):
        for kx in range(3):
            z += np.tensordot(W[:, :, ky, kx], shifted(a, ky - 1, kx - 1), axes=(1, 0))
    return z


def conv3x3_dx(dz, W):
    """Gradient of conv3x3 w.r.t. its input a, given dz = dL/dz."""
    ci = W.shape[1]
    da = np.zeros((ci,) + dz.shape[1:])
    for ky in range(3):
        for kx in range(3):
            da += shifted(np.tensordot(W[:, :, ky, kx], dz, axes=(0, 0)), 1 - ky, 1 - kx)
    return da


def conv3x3_dw(dz, a):
    """Gradients w.r.t. W and b."""
    co, ci = dz.shape[0], a.shape[0]
    dW = np.zeros((co, ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.tensordot(dz, shifted(a, ky - 1, kx - 1), axes=((1, 2), (1, 2)))
    return dW, dz.sum(axis=(1, 2))


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, scales, keep=False, round_act=None):
    """x: (2, H, W) coarse state u*; returns r (2, H, W) [and the saved tensors].

    round_act: optional rounding applied to every layer input (the GPU keeps
    activations in BF16); None keeps FP64 throughout.
    """
    rnd = (lambda t: t) if round_act is None else round_act
    layers = unpack(params)
    a = rnd(np.stack([x[0] * scales[0], x[1] * scales[1]]))
    saved = []
    for li, (W, b) in enumerate(layers):
        z = conv3x3(a, W, b)
        saved.append((a, z))
        a = rnd(silu(z)) if li < len(layers) - 1 else z
    r = np.stack([a[0] * scales[2], a[1] * scales[3]])
    return (r, saved) if keep else r


def loss_and_grad(params, xs, targets, scales):
    """Mean squared residual error over a batch and its gradient.

    L = sum_b sum_{c,i,j} (r_b - t_b)^2 / (B * 2 * H * W).
    """
    layers = unpack(params)
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    B = len(xs)
    total = 0.0
    for x, t in zip(xs, targets):
        r, saved = forward(params, x, scales, keep=True)
        n = r.size
        e = r - t
        total += float(np.sum(e * e))
        dr = 2.0 * e / (B * n)
        dz = np.stack([dr[0] * scales[2], dr[1] * scales[3]])
        for li in range(len(layers) - 1, -1, -1):
            a, z = saved[li]
            if li < len(layers) - 1:
                dz = dz * silu_grad(z)
            dW, db = conv3x3_dw(dz, a)
            grads[li] = (grads[li][0] + dW, grads[li][1] + db)
            if li > 0:
                dz = conv3x3_dx(dz, layers[li][0])
    return total / (B * xs[0].size), pack(grads)


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def restrict4(a):
    """4 x 4 block mean (fine grid -> coarse grid); conserves the mean."""
    H, W = a.shape
    return a.reshape(H // 4, 4, W // 4, 4).mean(axis=(1, 3))


def tile_mean_field(a, ft=16):
    """The tile-mean field of a periodic plane a (H x W, both multiples of ft):
    the means of its ft x ft tiles, placed at the tile centres
    (ft t + (ft - 1) / 2 in pixel units) and interpolated bilinearly between
    neighbouring centres, periodically.  The corrector subtracts this field from
    its phi residual in projection mode 1 (in mode 0 it subtracts the plain
    mean): the field has the same total as a, so the corrected phi keeps its
    mean, and it carries a's content at scales beyond a tile."""
    H, W = a.shape
    ty, tx = H // ft, W // ft
    tm = a.reshape(ty, ft, tx, ft).mean(axis=(1, 3))
    out = np.empty((H, W))
    for y in range(H):
        v = (y + 0.5) / ft - 0.5
        j0 = int(np.floor(v))
        fy = v - j0
        ja, jb = j0 % ty, (j0 + 1) % ty
        for x in range(W):
            u = (x + 0.5) / ft - 0.5
            i0 = int(np.floor(u))
            fx = u - i0
            ia, ib = i0 % tx, (i0 + 1) % tx
            out[y, x] = ((1 - fy) * ((1 - fx) * tm[ja, ia] + fx * tm[ja, ib])
                         + fy * ((1 - fx) * tm[jb, ia] + fx * tm[jb, ib]))
    return out
