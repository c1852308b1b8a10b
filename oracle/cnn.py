"""Plain FP64 reference of the learned preconditioner's network (numpy).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark may use this module.  The product path never imports it.

The network is not part of the paper; it answers the observation of Sec. 5
that diagonally preconditioned Krylov solves become costly for fine meshes
and higher degrees.  It acts per patch on the (2^m+p) x (2^m+p) coefficient
grid of the spline space (Sec. 2.2):

    M(r) = y + f(y),  y = D^-1 r,

f = five 3x3 convolutions (channels 1 -> 32 -> 32 -> 32 -> 32 -> 1), ReLU (or
the identity, a linear network) after the first four, no biases, zero padding at the grid edges.  Weights
are given layer after layer, each as [c_out][c_in][dy][dx]; tap (dy, dx)
reads pixel (y + dy - 1, x + dx - 1) (a cross-correlation).  The loss of a
batch of pairs (y, x) is L = sum (y + f(y) - x)^2 / (2 N), N the number of
values.  Everything here is FP64; the weights are used exactly as given (the
caller rounds them to BF16 with `bf16_round` to match the device passes).

Pins (tests/test_oracle_cnn.py): single- and multi-channel convolution
against scipy.signal.correlate2d; the gradient against central differences
of the loss; the data gradient as the adjoint of the convolution; identity
for a zero last layer; positive homogeneity; BF16 rounding against
hand-computed values and torch's conversion.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 1)]
NUM_WEIGHTS = sum(9 * ci * co for ci, co in LAYERS)


def split(w):
    """Flat weight vector -> list of [c_out][c_in][3][3] arrays (views)."""
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    assert w.size == NUM_WEIGHTS
    out, o = [], 0
    for ci, co in LAYERS:
        out.append(w[o:o + 9 * ci * co].reshape(co, ci, 3, 3))
        o += 9 * ci * co
    return out


def bf16_round(w):
    """Round to the nearest bfloat16 value (ties to even) after rounding to float32; returns float64."""
    u = np.asarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3(a, k):
    """out[n, o, y, x] = sum_c sum_{dy,dx} k[o, c, dy, dx] a[n, c, y+dy-1, x+dx-1], zero outside."""
    n, c, H, W = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, k.shape[0], H, W))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,nchw->nohw", k[:, :, dy, dx], ap[:, :, dy:dy + H, dx:dx + W])
    return out


def conv3_adjoint(g, k):
    """Adjoint of conv3 in its input: a[n, c, y, x] = sum_o sum_{dy,dx} k[o, c, dy, dx] g[n, o, y-dy+1, x-dx+1]."""
    n, o, H, W = g.shape
    gp = np.pad(g, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, k.shape[1], H, W))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,nohw->nchw", k[:, :, dy, dx], gp[:, :, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W])
    return out


def relu(z):
    return np.maximum(z, 0.0)


def forward(w, y, linear=False):
    """(y + f(y), pre-activations z_0..z_3) for images y of shape (n, H, W); linear=True takes the
    identity for the activation."""
    ks = split(w)
    a = np.asarray(y, dtype=np.float64)[:, None]
    zs = []
    for l, k in enumerate(ks):
        z = conv3(a, k)
        if l < len(ks) - 1:
            zs.append(z)
            a = z if linear else relu(z)
        else:
            f = z[:, 0]
    return np.asarray(y, dtype=np.float64) + f, zs


def loss_grad(w, y, x, linear=False):
    """(L, dL/dw) for images y, targets x of shape (n, H, W)."""
    ks = split(w)
    y = np.asarray(y, dtype=np.float64)
    out, zs = forward(w, y, linear)
    d = out - np.asarray(x, dtype=np.float64)
    N = d.size
    loss = float(np.sum(d * d) / (2 * N))
    g = (d / N)[:, None]                      # dL / d(output of the last layer)
    grads = [None] * len(ks)
    for l in range(len(ks) - 1, -1, -1):
        a = y[:, None] if l == 0 else (zs[l - 1] if linear else relu(zs[l - 1]))
        ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
        H, W = a.shape[2], a.shape[3]
        gw = np.zeros_like(ks[l])
        for dy in range(3):
            for dx in range(3):
                gw[:, :, dy, dx] = np.einsum("nohw,nchw->oc", g, ap[:, :, dy:dy + H, dx:dx + W])
        grads[l] = gw
        if l > 0:
            g = conv3_adjoint(g, ks[l])
            if not linear:
                g = g * (zs[l - 1] > 0)
    return loss, np.concatenate([gw.reshape(-1) for gw in grads])


def precondition(w, r, D, n_img, side, linear=False):
    """M(r) = y + f(y), y = r / D, for a vector of n_img grids of side x side (FP64)."""
    y = (np.asarray(r) / np.asarray(D)).reshape(n_img, side, side)
    return forward(w, y, linear)[0].reshape(-1)
