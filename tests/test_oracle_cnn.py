"""Pins for the CNN oracle: direct nested-loop convolution, finite-difference
gradients of the whole network, GELU special values, hand-computed bfloat16
roundings and one Adam step written out by hand."""
import math

import numpy as np

from oracle import cnn as N


def test_bf16_round_hand_values():
    one = 1.0
    assert N.bf16_round(np.array([one]))[0] == 1.0
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert N.bf16_round(np.array([1 + 2.0 ** -8]))[0] == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6 ... rounds to even (1 + 2^-6)
    assert N.bf16_round(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert N.bf16_round(np.array([1 + 2.0 ** -8 + 2.0 ** -12]))[0] == 1 + 2.0 ** -7
    assert N.bf16_round(np.array([-3.0]))[0] == -3.0
    assert N.bf16_round(np.array([0.1]))[0] == 0.10009765625


def test_conv_equals_nested_loop_direct_sum():
    rng = np.random.default_rng(0)
    n, C, O = 4, 2, 3
    x = rng.standard_normal((C, n, n, n))
    w = rng.standard_normal((O, C, 3, 3, 3))
    b = rng.standard_normal(O)
    y = N.conv3d(x, w, b)
    for o in range(O):
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    acc = b[o]
                    for c in range(C):
                        for a in range(3):
                            for bb in range(3):
                                for cc in range(3):
                                    acc += w[o, c, a, bb, cc] * x[c, (i + a - 1) % n, (j + bb - 1) % n, (k + cc - 1) % n]
                    assert abs(acc - y[o, i, j, k]) < 1e-12


def test_adjoint_identity():
    # <conv(x), dy> = <x, conv^T(dy)> and <conv(x), dy> = <w, dW(x, dy)>
    rng = np.random.default_rng(1)
    n, C, O = 5, 3, 2
    x = rng.standard_normal((C, n, n, n))
    w = rng.standard_normal((O, C, 3, 3, 3))
    dy = rng.standard_normal((O, n, n, n))
    lhs = np.sum(N.conv3d(x, w, None) * dy)
    assert abs(lhs - np.sum(x * N.conv3d_adjoint_input(dy, w))) < 1e-10
    assert abs(lhs - np.sum(w * N.conv3d_weight_grad(x, dy))) < 1e-10


def test_gelu_values_and_derivative():
    assert N.gelu(np.array([0.0]))[0] == 0.0
    assert abs(N.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # Phi(1)
    assert abs(N.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15
    u = np.linspace(-4, 4, 17)
    e = 1e-6
    fd = (N.gelu(u + e) - N.gelu(u - e)) / (2 * e)
    np.testing.assert_allclose(N.gelu_grad(u), fd, atol=1e-9)


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    n = 4
    params = N.init_params(channels=3, layers=3, seed=5)
    params = [(w, rng.standard_normal(b.shape) * 0.1) for w, b in params]
    x = rng.standard_normal((n, n, n))
    t = rng.standard_normal((n, n, n))

    def loss(ps, xx):
        y, _ = N.forward(xx, ps)
        return N.loss_mse(y, t)[0]

    y, cache = N.forward(x, params)
    _, dy = N.loss_mse(y, t)
    grads, dx = N.backward(dy, params, cache)
    e = 1e-6
    for l, (w, b) in enumerate(params):
        for idx in [(0, 0, 1, 1, 1), (w.shape[0] - 1, w.shape[1] - 1, 0, 2, 1), (0, w.shape[1] - 1, 2, 0, 2)]:
            wp = w.copy(); wp[idx] += e
            wm = w.copy(); wm[idx] -= e
            pp = list(params); pp[l] = (wp, b)
            pm = list(params); pm[l] = (wm, b)
            fd = (loss(pp, x) - loss(pm, x)) / (2 * e)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx)
        bp = b.copy(); bp[0] += e
        bm = b.copy(); bm[0] -= e
        pp = list(params); pp[l] = (w, bp)
        pm = list(params); pm[l] = (w, bm)
        fd = (loss(pp, x) - loss(pm, x)) / (2 * e)
        assert abs(fd - grads[l][1][0]) <= 1e-6 * max(1.0, abs(fd))
    for p in [(0, 0, 0), (1, 2, 3), (3, 3, 0)]:
        xp = x.copy(); xp[p] += e
        xm = x.copy(); xm[p] -= e
        fd = (loss(params, xp) - loss(params, xm)) / (2 * e)
        assert abs(fd - dx[p]) <= 1e-6 * max(1.0, abs(fd))


def test_quantized_forward_rounds_at_storage_points():
    rng = np.random.default_rng(3)
    params = N.init_params(channels=4, layers=3, seed=1)
    x = rng.standard_normal((4, 4, 4))
    y, cache = N.forward(x, params, quantize=True)
    for a, z in cache:
        np.testing.assert_array_equal(a, N.bf16_round(a))
        if z is not None:
            np.testing.assert_array_equal(z, N.bf16_round(z))
    y64, _ = N.forward(x, params, quantize=False)
    assert np.linalg.norm(y - y64) / np.linalg.norm(y64) < 3e-2


def test_adam_step_by_hand():
    p, g = np.array([1.0]), np.array([0.5])
    m, v = np.zeros(1), np.zeros(1)
    p1, m1, v1 = N.adam_step(p, g, m, v, t=1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2  ->  p - lr * g / (|g| + eps)
    assert abs(p1[0] - (1.0 - 0.1 * 0.5 / (0.5 + 1e-8))) < 1e-15
    assert abs(m1[0] - 0.05) < 1e-15 and abs(v1[0] - 0.00025) < 1e-15
    assert math.isclose(p1[0], 0.9, rel_tol=1e-7)
