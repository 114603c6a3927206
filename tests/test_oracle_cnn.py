"""Pins of the proposer's FP64 network reference and of the counter-based generator.

- conv / conv_backward against a direct loop over the convolution sum;
- the full backward pass against central finite differences of the loss;
- Philox4x32-10 against its published known-answer vectors;
- the Exp(1) noise built on it has the Exp(1) mean, variance and tail.
"""
import math

import numpy as np

import oracle
from oracle import cnn


def test_conv_matches_direct_sum():
    r = np.random.default_rng(0)
    x = r.normal(size=(2, 3, 9))
    W = r.normal(size=(4, 3, 5))
    b = r.normal(size=4)
    y = cnn.conv(x, W, b)
    for bb in range(2):
        for o in range(4):
            for l in range(9):
                acc = b[o]
                for c in range(3):
                    for t in range(5):
                        li = l + t - 2
                        if 0 <= li < 9:
                            acc += W[o, c, t] * x[bb, c, li]
                assert abs(y[bb, o, l] - acc) < 1e-12


def test_backward_matches_finite_differences():
    c_in, c_out, L, B = 3, 4, 7, 2
    r = np.random.default_rng(1)
    params = cnn.init_params(c_in, c_out, 2).astype(np.float64)
    params += r.normal(scale=0.05, size=params.size)   # nonzero biases too
    x = r.normal(size=(B, c_in, L))
    target = np.array([5, 17])

    def loss_of(p):
        z, _ = cnn.forward(p, x, c_in, c_out)
        return cnn.softmax_xent(z, target)[0]

    z, cache = cnn.forward(params, x, c_in, c_out)
    loss, dz = cnn.softmax_xent(z, target)
    g = cnn.backward(params, cache, dz, c_in, c_out)
    assert g.size == cnn.n_params(c_in, c_out)
    idx = r.choice(params.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(params)
        e[i] = h
        fd = (loss_of(params + e) - loss_of(params - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_softmax_xent_closed_form():
    z = np.zeros((2, 3, 4))                  # uniform logits over 12 cells
    loss, dz = cnn.softmax_xent(z, np.array([3, -1]))
    assert abs(loss - math.log(12.0)) < 1e-15
    assert np.allclose(dz[1], 0.0)
    assert abs(dz[0].ravel()[3] - (1 / 12 - 1)) < 1e-15


def test_philox_known_answers():
    assert [int(v) for v in oracle.philox4x32_10([0, 0, 0, 0], [0, 0])] == \
        [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert [int(v) for v in oracle.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2)] == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert [int(v) for v in oracle.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                                                  [0xa4093822, 0x299f31d0])] == \
        [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_exp_noise_moments():
    x = oracle.exp_noise(seed=12345, stream=0, r=3, n=400000).astype(np.float64)
    assert np.all(x > 0)
    assert abs(x.mean() - 1.0) < 0.01 and abs(x.var() - 1.0) < 0.02
    assert abs((x > 1.6).mean() - math.exp(-1.6)) < 0.003
    y = oracle.exp_noise(seed=12345, stream=0, r=4, n=1000)
    assert not np.array_equal(x[:1000], y)   # realisations differ
