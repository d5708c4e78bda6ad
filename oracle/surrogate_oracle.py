"""Plain FP64 oracle of the CNN surrogate (numpy).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only callers; it shares no code with the HIP
surrogate kernels.

The network maps per-cavity parameters plus grid coordinates to a steady
field.  Tensors are channels-last: activations x[b, y, x, c]; a 3x3 layer has
weights w[co, tap, ci] with tap = (dy + 1) * 3 + (dx + 1) addressing the input
pixel (y + dy, x + dx) (zero outside the image) and bias b[co]:

    z[b, y, x, co] = b[co] + sum_{tap, ci} w[co, tap, ci] x[b, y + dy, x + dx, ci]

Hidden layers apply SiLU(z) = z / (1 + exp(-z)); the last layer is linear.
Loss: mean squared error over the real output channels.  Optimiser: Adam
(Kingma & Ba 2015) with bias correction.

``bf16`` rounds float64 values to bfloat16 (round to nearest, ties to even on
the float32 bit pattern), the storage precision of the GPU weights and
activations; the oracle applies it where the GPU stores bfloat16, so both
sides compute from identical operands.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) and return float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x, dy, dx):
    """out[b, y, x, :] = x[b, y + dy, x + dx, :], zero outside the image."""
    out = np.zeros_like(x)
    B, H, W, C = x.shape
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    yt = slice(max(0, dy), min(H, H + dy))
    xt = slice(max(0, dx), min(W, W + dx))
    out[:, ys, xs, :] = x[:, yt, xt, :]
    return out


N_FEATURES = 15


def features(params, H, W):
    """Network input [B, H, W, 15]: the B x 5 normalised cavity parameters
    broadcast over the grid, the cell-centre coordinates xc = (i + 1/2)/W,
    yc = (j + 1/2)/H, and sin/cos of pi xc, 2 pi xc, pi yc, 2 pi yc."""
    params = np.asarray(params, dtype=np.float64)
    B = params.shape[0]
    xc = (np.arange(W) + 0.5) / W
    yc = (np.arange(H) + 0.5) / H
    X, Y = np.meshgrid(xc, yc)
    coord = [X, Y]
    for v in (X, Y):
        for k in (1.0, 2.0):
            coord += [np.sin(k * np.pi * v), np.cos(k * np.pi * v)]
    out = np.empty((B, H, W, N_FEATURES))
    for bi in range(B):
        for c in range(5):
            out[bi, :, :, c] = params[bi, c]
        for c, plane in enumerate(coord):
            out[bi, :, :, 5 + c] = plane
    return out


def conv_forward(x, w, b):
    """z = b + sum over taps of shift(x, tap) @ w[:, tap, :]^T."""
    z = np.broadcast_to(b, x.shape[:3] + (w.shape[0],)).astype(np.float64).copy()
    for t, (dy, dx) in enumerate(TAPS):
        z += shift(x, dy, dx) @ w[:, t, :].T
    return z


def conv_backward(x, w, dz):
    """Gradients of sum(dz * conv_forward(x, w, b)) w.r.t. x, w, b."""
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for t, (dy, dxs) in enumerate(TAPS):
        xs = shift(x, dy, dxs)
        dw[:, t, :] = np.einsum("byxo,byxi->oi", dz, xs)
        dx += shift(dz @ w[:, t, :], -dy, -dxs)
    db = dz.sum(axis=(0, 1, 2))
    return dx, dw, db


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mse(pred, target):
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def forward(layers, x, bf16_storage=False):
    """layers: list of (w, b).  Returns (zs, acts): zs[l] pre-activations,
    acts[l] the input of layer l (acts[0] = x).  With bf16_storage the inputs
    of every layer and the weights are rounded to bfloat16 as the GPU stores them."""
    acts, zs = [bf16(x) if bf16_storage else x], []
    for l, (w, b) in enumerate(layers):
        wl = bf16(w) if bf16_storage else w
        z = conv_forward(acts[-1], wl, b)
        zs.append(z)
        if l + 1 < len(layers):
            a = silu(z)
            acts.append(bf16(a) if bf16_storage else a)
    return zs, acts


def backward(layers, zs, acts, dz_out, bf16_storage=False):
    """Gradients (dw, db) of every layer given dL/dz of the last layer."""
    grads = [None] * len(layers)
    dz = bf16(dz_out) if bf16_storage else dz_out
    for l in range(len(layers) - 1, -1, -1):
        w, _ = layers[l]
        wl = bf16(w) if bf16_storage else w
        dx, dw, db = conv_backward(acts[l], wl, dz)
        grads[l] = (dw, db)
        if l > 0:
            dz = dx * silu_grad(zs[l - 1])
            if bf16_storage:
                dz = bf16(dz)
    return grads


def loss_and_grads(layers, x, target, out_channels):
    zs, acts = forward(layers, x)
    pred = zs[-1][..., :out_channels]
    loss, dpred = mse(pred, target)
    dz = np.zeros_like(zs[-1])
    dz[..., :out_channels] = dpred
    return loss, backward(layers, zs, acts, dz)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---- warm-start preparation ---------------------------------------------------
def smooth(planes):
    """Separable [1 2 1]/4 filter of every [..., H, W] plane, edge values replicated."""
    a = np.asarray(planes, dtype=np.float64)
    p = np.pad(a, [(0, 0)] * (a.ndim - 2) + [(1, 1), (1, 1)], mode="edge")
    out = np.zeros_like(a)
    wts = (0.25, 0.5, 0.25)
    H, W = a.shape[-2:]
    for dy in range(3):
        for dx in range(3):
            out += wts[dy] * wts[dx] * p[..., dy:dy + H, dx:dx + W]
    return out


def destagger(fields):
    """fields [n, 4, H, W] = (u, v, T, C): remove <u (-1)^x> (-1)^x from u and
    <v (-1)^y> (-1)^y from v (means over the plane); T and C unchanged."""
    f = np.array(fields, dtype=np.float64, copy=True)
    H, W = f.shape[-2:]
    sx = np.tile((-1.0) ** np.arange(W), (H, 1))
    sy = np.tile(((-1.0) ** np.arange(H))[:, None], (1, W))
    for k in range(f.shape[0]):
        f[k, 0] -= np.mean(f[k, 0] * sx) * sx
        f[k, 1] -= np.mean(f[k, 1] * sy) * sy
    return f
