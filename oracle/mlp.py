"""Warm-start network: forward pass, loss, gradients and Adam (oracle; test use only).

The network maps a geometry coordinate R to the ansatz parameters:
  h1 = tanh(W1 R + b1)        (hidden, 1 input)
  h2 = tanh(W2 h1 + b2)       (hidden x hidden)
  y  = W3 h2 + b3             (n_out x hidden)
trained with the mean squared error L = mean over samples and outputs of
(y - t)^2 and Adam (beta1 0.9, beta2 0.999, eps 1e-8).  Parameters are one
flat float array packed as [W1 (H), b1 (H), W2 (H*H, row j = output j),
b2 (H), W3 (O*H), b3 (O)].

With ``bf16=True`` every operand of a product is first rounded to bfloat16
(round to nearest, ties to even), at the points where a BF16-input /
FP32-accumulate implementation rounds: R and W1 in the first layer; h1, W2
in the second; h2, W3 in the third; and in the backward pass the output
error dL/dy and the hidden errors dL/d(pre-activation) of the second layer
together with the weights and activations they multiply.  Biases, tanh
derivatives, the first layer's weight gradient and all bias gradients use
the unrounded values.  Everything else is float64, so the oracle stands for
exact arithmetic on the rounded operands.
"""

import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def bf16(v):
    """Round float64 values to the nearest bfloat16 (8 significant bits), ties
    to even; bfloat16 subnormals are not modelled (|v| >= 2^-126 assumed or 0)."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)                       # v = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)  # rint rounds half to even


def param_count(hidden, n_out):
    return 3 * hidden + hidden * hidden + n_out * hidden + n_out


def unpack(p, hidden, n_out):
    H, O = hidden, n_out
    p = np.asarray(p, dtype=np.float64)
    i = 0
    W1 = p[i:i + H]; i += H
    b1 = p[i:i + H]; i += H
    W2 = p[i:i + H * H].reshape(H, H); i += H * H
    b2 = p[i:i + H]; i += H
    W3 = p[i:i + O * H].reshape(O, H); i += O * H
    b3 = p[i:i + O]; i += O
    assert i == p.size
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def forward(p, x, hidden, n_out, bf16_inputs=True):
    """Returns y [n, O] and the activations the backward pass needs."""
    r = bf16 if bf16_inputs else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p, hidden, n_out)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    h1 = np.tanh(np.outer(r(x), r(W1)) + b1)
    h2 = np.tanh(r(h1) @ r(W2).T + b2)
    y = r(h2) @ r(W3).T + b3
    return y, (x, h1, h2)


def loss_grad(p, x, t, hidden, n_out, bf16_inputs=True):
    """Mean squared error and its gradient with respect to the packed parameters."""
    r = bf16 if bf16_inputs else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p, hidden, n_out)
    y, (x, h1, h2) = forward(p, x, hidden, n_out, bf16_inputs)
    t = np.asarray(t, dtype=np.float64).reshape(y.shape)
    n = y.shape[0]
    d = y - t
    loss = np.sum(d * d) / (n * n_out)
    dy = 2.0 * d / (n * n_out)                      # dL/dy
    gW3 = r(dy).T @ r(h2)
    gb3 = dy.sum(axis=0)
    dz2 = (r(dy) @ r(W3)) * (1.0 - h2 * h2)         # dL/d(W2 h1 + b2)
    gW2 = r(dz2).T @ r(h1)
    gb2 = dz2.sum(axis=0)
    dz1 = (r(dz2) @ r(W2)) * (1.0 - h1 * h1)        # dL/d(W1 x + b1)
    gW1 = dz1.T @ r(x)
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(p, g, m, v, step, lr):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mhat = m / (1.0 - BETA1 ** step)
    vhat = v / (1.0 - BETA2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + EPS), m, v


def train(p, x, t, hidden, n_out, n_steps, lr, bf16_inputs=True, state=None):
    """Full-batch Adam; ``state`` = (m, v, step) to continue a run.  Returns
    (p, losses, state)."""
    p = np.asarray(p, dtype=np.float64).copy()
    m, v, step = state if state is not None else (np.zeros_like(p), np.zeros_like(p), 0)
    losses = []
    for _ in range(n_steps):
        loss, g = loss_grad(p, x, t, hidden, n_out, bf16_inputs)
        step += 1
        p, m, v = adam_step(p, g, m, v, step, lr)
        losses.append(loss)
    return p, np.array(losses), (m, v, step)
