"""Plain numpy oracle of the learned initial guess / preconditioner network.

TEST INFRASTRUCTURE ONLY (used by the tests and the smoke check).  It shares
no code with the GPU kernels.

The network is a 3-level convolutional encoder-decoder with skip
concatenation: channels 16 / 32 / 64, 3x3 (2D) or 3x3x3 (3D) "same"
convolutions with zero padding, ReLU, 2x average pooling and 2x nearest
upsampling:

    e0 = relu(conv(x,              W0, b0))    C_in -> 16, full resolution
    e1 = relu(conv(pool(e0),       W1, b1))    16 -> 32, 1/2
    e2 = relu(conv(pool(e1),       W2, b2))    32 -> 64, 1/4
    d1 = relu(conv([up(e2), e1],   W3, b3))    96 -> 32, 1/2
    d0 = relu(conv([up(d1), e0],   W4, b4))    48 -> 16, full
    y  =       conv(d0,             W5, b5)     16 -> 1

Tensors are channels-last: shape spatial + (C,), spatial = (nz, nx) in 2D or
(nz, ny, nx) in 3D, matching the cell index i + nx*(j + ny*k).  A weight
tensor has shape (C_out, taps, C_in); tap t is the offset (dz, dx) (2D) or
(dz, dy, dx) (3D) in lexicographic order over {-1, 0, 1}; y[p] uses
x[p + offset].

Everything is FP64 unless ``bf16=True``: then weights and every stored
activation (the output of each convolution, pooling and concatenation) are
rounded to bfloat16 (round to nearest even), products are accumulated in
float32, gradients are kept in float32 and rounded to bfloat16 where they
enter a convolution -- the arithmetic of the GPU kernels, for parity.  The
network output stays float32.  The loss is L = sum((y - t)^2) / (2 * npix).
"""
from __future__ import annotations

import itertools

import numpy as np

CH = (16, 32, 64)


def taps(ndim: int):
    return list(itertools.product((-1, 0, 1), repeat=ndim))


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(f.shape)


def shift(x: np.ndarray, off) -> np.ndarray:
    """s[p] = x[p + off] with zeros outside (spatial axes = all but the last)."""
    nd = x.ndim - 1
    out = np.zeros_like(x)
    src = []
    dst = []
    for a in range(nd):
        n = x.shape[a]
        o = off[a]
        if o >= 0:
            dst.append(slice(0, n - o))
            src.append(slice(o, n))
        else:
            dst.append(slice(-o, n))
            src.append(slice(0, n + o))
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv(x, W, b, bf16=False):
    """y[p, co] = b[co] + sum_t sum_ci x[p + off_t, ci] W[co, t, ci]"""
    nd = x.ndim - 1
    if bf16:
        x = round_bf16(x)
        W = round_bf16(W)
        acc = np.zeros(x.shape[:-1] + (W.shape[0],), dtype=np.float32)
    else:
        acc = np.zeros(x.shape[:-1] + (W.shape[0],), dtype=np.float64)
    for t, off in enumerate(taps(nd)):
        acc = acc + shift(x, off) @ W[:, t, :].T.astype(acc.dtype)
    return acc + b.astype(acc.dtype)


def conv_backward(x, W, dy, bf16=False):
    """gradients of conv with respect to x, W and b"""
    nd = x.ndim - 1
    if bf16:
        x = round_bf16(x)
        W = round_bf16(W)
        dy = round_bf16(dy)
        dt = np.float32
    else:
        dt = np.float64
    dx = np.zeros(x.shape, dtype=dt)
    dW = np.zeros(W.shape, dtype=dt)
    C_in = x.shape[-1]
    C_out = dy.shape[-1]
    X2 = None
    for t, off in enumerate(taps(nd)):
        neg = tuple(-o for o in off)
        dx = dx + shift(dy, neg) @ W[:, t, :].astype(dt)
        X2 = shift(x, off).reshape(-1, C_in)
        dW[:, t, :] = dy.reshape(-1, C_out).T.astype(dt) @ X2.astype(dt)
    db = dy.reshape(-1, C_out).sum(axis=0)
    return dx, dW, db


def relu(a):
    return np.maximum(a, 0)


def pool(x):
    """2x average pooling in every spatial direction"""
    nd = x.ndim - 1
    s = x.shape
    if nd == 2:
        return x.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2]).mean(axis=(1, 3))
    return x.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2, s[3]).mean(axis=(1, 3, 5))


def pool_backward(dy):
    nd = dy.ndim - 1
    return up(dy) / (2 ** nd)


def up(x):
    """2x nearest upsampling"""
    nd = x.ndim - 1
    for a in range(nd):
        x = np.repeat(x, 2, axis=a)
    return x


def up_backward(dy):
    nd = dy.ndim - 1
    s = dy.shape
    if nd == 2:
        return dy.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2]).sum(axis=(1, 3))
    return dy.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2, s[3]).sum(axis=(1, 3, 5))


def layer_shapes(ndim: int, c_in: int):
    """(C_out, C_in) of the six convolutions"""
    c0, c1, c2 = CH
    return [(c0, c_in), (c1, c0), (c2, c1), (c1, c2 + c1), (c0, c1 + c0), (1, c0)]


def init_params(ndim: int, c_in: int, seed: int = 0):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    nt = 3 ** ndim
    params = []
    for co, ci in layer_shapes(ndim, c_in):
        std = np.sqrt(2.0 / (nt * ci))
        params.append((rng.normal(0.0, std, size=(co, nt, ci)), np.zeros(co)))
    return params


def forward(params, x, bf16=False):
    """returns (y, cache of activations)"""
    (W0, b0), (W1, b1), (W2, b2), (W3, b3), (W4, b4), (W5, b5) = params
    st = round_bf16 if bf16 else (lambda a: a)   # storage of an activation
    c = {}
    c["x"] = st(x)
    c["e0"] = st(relu(conv(c["x"], W0, b0, bf16)))
    c["p0"] = st(pool(c["e0"]))
    c["e1"] = st(relu(conv(c["p0"], W1, b1, bf16)))
    c["p1"] = st(pool(c["e1"]))
    c["e2"] = st(relu(conv(c["p1"], W2, b2, bf16)))
    c["c1"] = np.concatenate([up(c["e2"]), c["e1"]], axis=-1)
    c["d1"] = st(relu(conv(c["c1"], W3, b3, bf16)))
    c["c0"] = np.concatenate([up(c["d1"]), c["e0"]], axis=-1)
    c["d0"] = st(relu(conv(c["c0"], W4, b4, bf16)))
    y = conv(c["d0"], W5, b5, bf16)
    return y, c


def loss(y, t):
    npix = y.size // y.shape[-1]
    return float(np.sum((np.asarray(y, np.float64) - t) ** 2) / (2 * npix))


def backward(params, cache, y, t, bf16=False):
    """gradients of loss(forward(params, x), t) with respect to every (W, b)"""
    (W0, b0), (W1, b1), (W2, b2), (W3, b3), (W4, b4), (W5, b5) = params
    c = cache
    npix = y.size // y.shape[-1]
    dy = (np.asarray(y, np.float64) - t) / npix
    g = [None] * 6
    dd0, dW5, db5 = conv_backward(c["d0"], W5, dy, bf16)
    g[5] = (dW5, db5)
    dpre = dd0 * (c["d0"] > 0)
    dc0, dW4, db4 = conv_backward(c["c0"], W4, dpre, bf16)
    g[4] = (dW4, db4)
    k1 = c["d1"].shape[-1]
    dd1 = up_backward(dc0[..., :k1])
    de0 = dc0[..., k1:]
    dpre = dd1 * (c["d1"] > 0)
    dc1, dW3, db3 = conv_backward(c["c1"], W3, dpre, bf16)
    g[3] = (dW3, db3)
    k2 = c["e2"].shape[-1]
    de2 = up_backward(dc1[..., :k2])
    de1 = dc1[..., k2:]
    dpre = de2 * (c["e2"] > 0)
    dp1, dW2, db2 = conv_backward(c["p1"], W2, dpre, bf16)
    g[2] = (dW2, db2)
    de1 = de1 + pool_backward(dp1)
    dpre = de1 * (c["e1"] > 0)
    dp0, dW1, db1 = conv_backward(c["p0"], W1, dpre, bf16)
    g[1] = (dW1, db1)
    de0 = de0 + pool_backward(dp0)
    dpre = de0 * (c["e0"] > 0)
    _, dW0, db0 = conv_backward(c["x"], W0, dpre, bf16)
    g[0] = (dW0, db0)
    return g


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """one Adam step (Kingma & Ba, Algorithm 1) on every tensor; t >= 1"""
    out = []
    for k, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, gp) in enumerate(((W, gW), (b, gb))):
            m[k][j] = b1 * m[k][j] + (1 - b1) * gp
            v[k][j] = b2 * v[k][j] + (1 - b2) * gp * gp
            mh = m[k][j] / (1 - b1 ** t)
            vh = v[k][j] / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out
