"""FP64 reference of the learned proposer's network (test infrastructure only).

The proposer ranks fine-grid cells from a coarse statistic map: input
x[B][C_in][L] (C_in coarse-map channels along L coarse f0 positions), four
1-D convolutions with zero padding,
    h1 = relu(conv5(x;  W1, b1))    C_in -> 32
    h2 = relu(conv5(h1; W2, b2))    32   -> 32
    h3 = relu(conv5(h2; W3, b3))    32   -> 32
    z  = conv1(h3; W4, b4)          32   -> C_out   (logits of the fine cells)
    conv_k(x; W, b)[o][l] = b[o] + sum_c sum_t W[o][c][t] x[c][l + t - (k-1)/2]
and a softmax cross-entropy over the C_out*L logits of a sample against one
target cell (target -1: no target, no loss).  The parameters are one flat
vector in the order W1, b1, W2, b2, W3, b3, W4, b4 with W[o][c][t] row-major.
Plain numpy in FP64, written from these definitions; pinned by central
finite differences in tests/test_oracle_cnn.py.

With rnd=bf16_operands every product takes both operands rounded to FP32
and then to bfloat16 (round to nearest even), the sums staying exact: the
arithmetic of BF16 matrix units.  Forward: weights and layer inputs;
backward: weights and upstream gradients (input gradients), upstream
gradients and layer inputs (weight gradients).  Bias gradients and the loss
take no rounding.
"""
import numpy as np

from oracle import bf16_rne


def bf16_operands(a):
    """a rounded to FP32, then to bfloat16 (RNE), returned as FP64."""
    codes = bf16_rne(np.asarray(a, dtype=np.float32)).astype(np.uint32) << 16
    return codes.view(np.float32).astype(np.float64)


def _id(a):
    return a

WIDTH = 32
K = 5


def layer_shapes(c_in, c_out):
    return [(WIDTH, c_in, K), (WIDTH,), (WIDTH, WIDTH, K), (WIDTH,), (WIDTH, WIDTH, K), (WIDTH,),
            (c_out, WIDTH, 1), (c_out,)]


def n_params(c_in, c_out):
    return sum(int(np.prod(s)) for s in layer_shapes(c_in, c_out))


def unpack(params, c_in, c_out):
    out, o = [], 0
    for s in layer_shapes(c_in, c_out):
        n = int(np.prod(s))
        out.append(np.asarray(params[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def init_params(c_in, c_out, seed):
    """He-uniform weights and zero biases (seeded)."""
    r = np.random.default_rng(seed)
    parts = []
    for s in layer_shapes(c_in, c_out):
        if len(s) == 3:
            fan_in = s[1] * s[2]
            lim = np.sqrt(6.0 / fan_in)
            parts.append(r.uniform(-lim, lim, s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def conv(x, W, b, rnd=None):
    """x [B][C][L], W [O][C][k], b [O] -> [B][O][L], zero padding (k-1)/2."""
    rnd = rnd or _id
    x, W = rnd(x), rnd(W)
    B, C, L = x.shape
    O, _, k = W.shape
    p = (k - 1) // 2
    xp = np.zeros((B, C, L + 2 * p))
    xp[:, :, p:p + L] = x
    y = np.zeros((B, O, L)) + b[None, :, None]
    for t in range(k):
        y += np.einsum("oc,bcl->bol", W[:, :, t], xp[:, :, t:t + L])
    return y


def conv_backward(x, W, dy, rnd=None):
    """Gradients of conv(x, W, b) for upstream dy: (dx, dW, db)."""
    db = dy.sum(axis=(0, 2))
    rnd = rnd or _id
    x, W, dy = rnd(x), rnd(W), rnd(dy)
    B, C, L = x.shape
    O, _, k = W.shape
    p = (k - 1) // 2
    xp = np.zeros((B, C, L + 2 * p))
    xp[:, :, p:p + L] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for t in range(k):
        dW[:, :, t] = np.einsum("bol,bcl->oc", dy, xp[:, :, t:t + L])
        dxp[:, :, t:t + L] += np.einsum("oc,bol->bcl", W[:, :, t], dy)
    return dxp[:, :, p:p + L], dW, db


def forward(params, x, c_in, c_out, rnd=None):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(params, c_in, c_out)
    x = np.asarray(x, np.float64)
    a1 = conv(x, W1, b1, rnd)
    h1 = np.maximum(a1, 0.0)
    a2 = conv(h1, W2, b2, rnd)
    h2 = np.maximum(a2, 0.0)
    a3 = conv(h2, W3, b3, rnd)
    h3 = np.maximum(a3, 0.0)
    z = conv(h3, W4, b4, rnd)
    return z, (x, a1, h1, a2, h2, a3, h3)


def backward(params, cache, dz, c_in, c_out, rnd=None):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(params, c_in, c_out)
    x, a1, h1, a2, h2, a3, h3 = cache
    dh3, dW4, db4 = conv_backward(h3, W4, dz, rnd)
    da3 = dh3 * (a3 > 0)
    dh2, dW3, db3 = conv_backward(h2, W3, da3, rnd)
    da2 = dh2 * (a2 > 0)
    dh1, dW2, db2 = conv_backward(h1, W2, da2, rnd)
    da1 = dh1 * (a1 > 0)
    _, dW1, db1 = conv_backward(x, W1, da1, rnd)
    return np.concatenate([g.ravel() for g in (dW1, db1, dW2, db2, dW3, db3, dW4, db4)])


def softmax_xent(z, target):
    """Mean cross-entropy of softmax over each sample's flattened logits against
    one target cell (target < 0: excluded); returns (loss, dz)."""
    B = z.shape[0]
    flat = z.reshape(B, -1)
    m = flat.max(axis=1, keepdims=True)
    e = np.exp(flat - m)
    p = e / e.sum(axis=1, keepdims=True)
    target = np.asarray(target)
    valid = target >= 0
    n = max(int(valid.sum()), 1)
    loss = 0.0
    d = np.zeros_like(flat)
    for i in np.nonzero(valid)[0]:
        loss -= np.log(p[i, target[i]])
        d[i] = p[i]
        d[i, target[i]] -= 1.0
    return loss / n, (d / n).reshape(z.shape)


def adam(p, g, m, v, lr, beta1, beta2, eps, step):
    """One Adam step (Kingma and Ba, Algorithm 1) in FP64: returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
