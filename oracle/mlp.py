"""Plain FP64 reference of the initial-guess network (test infrastructure:
only tests and the entry point's smoke check call it).

Three linear layers with ReLU after the first two, masked mean-square error
loss, and its gradients by the chain rule written out.  Used to check the
GPU's BF16 matrix-core forward and backward passes; it shares no code with
them.  With `bf16=True` the values that the GPU stores in BF16 (inputs,
weights, hidden activations, the output gradient and the back-propagated
gradients) are rounded to BF16 here too, round-to-nearest-even, so that the
two sides decide the same roundings; all arithmetic stays FP64."""

import numpy as np


def round_bf16(x):
    """Nearest BF16 value (ties to even) of each entry, as FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def forward(X, W, b, bf16=False):
    """X: (n, in); W: three (fan_in, fan_out) matrices; b: three vectors.
    Returns the pre-activations, the layer inputs and the output."""
    rd = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    acts = [rd(X)]
    pre = []
    h = acts[0]
    for k in range(3):
        z = h @ rd(W[k]) + b[k]
        pre.append(z)
        if k < 2:
            h = rd(np.maximum(z, 0.0))
            acts.append(h)
    return pre, acts, pre[2]


def loss_and_grads(X, T, mask, W, b, bf16=False):
    """loss = sum mask (Y - T)^2 / count, count = sum(mask); gradients of
    loss with respect to W and b."""
    rd = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    pre, acts, Y = forward(X, W, b, bf16)
    count = float(np.sum(mask))
    d = (Y - T) * mask
    loss = float(np.sum(d * d) / count)
    g = 2.0 * d / count
    dW, db = [None] * 3, [None] * 3
    for k in (2, 1, 0):
        gr = rd(g)
        dW[k] = acts[k].T @ gr
        db[k] = g.sum(axis=0)
        if k > 0:
            g = (gr @ rd(W[k]).T) * (pre[k - 1] > 0)
    return loss, dW, db
