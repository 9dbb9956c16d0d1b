"""Pins of the CNN oracle (oracle/cnn.py): the convolution against brute-force
loops, adjoint identities of every linear piece, the hand-written backward
pass against central finite differences, bfloat16 rounding against torch's
conversion, and the first Adam step against its closed form."""
import itertools

import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, W, b):
    nd = x.ndim - 1
    sp = x.shape[:-1]
    out = np.zeros(sp + (W.shape[0],))
    offs = cnn.taps(nd)
    for p in itertools.product(*[range(n) for n in sp]):
        for co in range(W.shape[0]):
            s = b[co]
            for t, off in enumerate(offs):
                q = tuple(pi + oi for pi, oi in zip(p, off))
                if all(0 <= qi < n for qi, n in zip(q, sp)):
                    s += float(np.dot(x[q], W[co, t]))
            out[p + (co,)] = s
    return out


@pytest.mark.parametrize("shape", [(5, 6), (3, 4, 5)])
def test_conv_matches_brute_force_loops(shape):
    rng = np.random.default_rng(0)
    nd = len(shape)
    x = rng.normal(size=shape + (3,))
    W = rng.normal(size=(2, 3 ** nd, 3))
    b = rng.normal(size=2)
    np.testing.assert_allclose(cnn.conv(x, W, b), brute_conv(x, W, b), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape", [(8, 4), (4, 8, 4)])
def test_adjoint_identities(shape):
    rng = np.random.default_rng(1)
    nd = len(shape)
    x = rng.normal(size=shape + (3,))
    W = rng.normal(size=(5, 3 ** nd, 3))
    y = rng.normal(size=shape + (5,))
    lhs = np.sum(cnn.conv(x, W, np.zeros(5)) * y)
    rhs = np.sum(x * cnn.conv_backward(x, W, y)[0])
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    # dW: d/dW <conv(x,W), y> = conv_backward(...)[1]
    dW = cnn.conv_backward(x, W, y)[1]
    assert abs(np.sum(dW * W) - lhs) < 1e-10 * abs(lhs)
    c = rng.normal(size=tuple(n // 2 for n in shape) + (3,))
    assert abs(np.sum(cnn.pool(x) * c) - np.sum(x * cnn.pool_backward(c))) < 1e-12
    f = rng.normal(size=shape + (3,))
    assert abs(np.sum(cnn.up(c) * f) - np.sum(c * cnn.up_backward(f))) < 1e-12


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4)])
def test_network_gradient_matches_finite_differences(shape):
    rng = np.random.default_rng(2)
    nd = len(shape)
    c_in = 2
    params = cnn.init_params(nd, c_in, seed=3)
    params = [(W, rng.normal(0, 0.1, size=b.shape)) for W, b in params]
    x = rng.normal(size=shape + (c_in,))
    t = rng.normal(size=shape + (1,))
    y, cache = cnn.forward(params, x)
    g = cnn.backward(params, cache, y, t)
    h = 1e-6
    checked = 0
    for k, (W, b) in enumerate(params):
        for arr, garr in ((W, g[k][0]), (b, g[k][1])):
            flat = arr.reshape(-1)
            gflat = garr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = cnn.loss(cnn.forward(params, x)[0], t)
                flat[idx] = old - h
                lm = cnn.loss(cnn.forward(params, x)[0], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, idx, fd, gflat[idx])
                checked += 1
    assert checked >= 40


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    a = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-8, 8, size=1000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0]])
    want = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(cnn.round_bf16(a), want)


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(5)
    params = [(rng.normal(size=(2, 9, 3)), rng.normal(size=2))]
    grads = [(rng.normal(size=(2, 9, 3)), rng.normal(size=2))]
    m = [[np.zeros((2, 9, 3)), np.zeros(2)]]
    v = [[np.zeros((2, 9, 3)), np.zeros(2)]]
    out = cnn.adam_step(params, grads, m, v, 1, lr=1e-2, eps=0.0)
    np.testing.assert_allclose(out[0][0], params[0][0] - 1e-2 * np.sign(grads[0][0]), rtol=1e-12)
    np.testing.assert_allclose(out[0][1], params[0][1] - 1e-2 * np.sign(grads[0][1]), rtol=1e-12)
