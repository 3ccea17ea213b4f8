"""FP64 reference for the learned cost model -- TEST INFRASTRUCTURE ONLY.

A fully connected network: hidden layers h_{l+1} = max(0, h_l W_l + b_l),
last layer linear; loss = mean over the batch of (y - t)^2; Adam with
bias-corrected moments (Kingma & Ba, 2015).  Parameters are laid out layer by
layer, W_l (dims[l] x dims[l+1], row-major) then b_l.  Backpropagation is the
chain rule written out per layer.  Pinned in tests by central finite
differences and a hand-computed two-unit network.
"""
import numpy as np


def unpack(params, dims):
    out, off = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        w = np.asarray(params[off:off + a * b], dtype=np.float64).reshape(a, b)
        off += a * b
        bias = np.asarray(params[off:off + b], dtype=np.float64)
        off += b
        out.append((w, bias))
    if off != len(params):
        raise ValueError("parameter count does not match the layer widths")
    return out


def forward(params, dims, x):
    """Returns the list of layer outputs (post-activation), input first."""
    acts = [np.asarray(x, dtype=np.float64)]
    layers = unpack(params, dims)
    for i, (w, b) in enumerate(layers):
        z = acts[-1] @ w + b
        acts.append(np.maximum(z, 0.0) if i + 1 < len(layers) else z)
    return acts


def loss_and_grad(params, dims, x, t):
    """MSE of the single output against t and its gradient (flat, same layout)."""
    acts = forward(params, dims, x)
    layers = unpack(params, dims)
    y = acts[-1][:, 0]
    n = len(y)
    loss = float(np.mean((y - t) ** 2))
    dz = (2.0 * (y - t) / n)[:, None]
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        w, _ = layers[l]
        grads[l] = (acts[l].T @ dz, dz.sum(axis=0))
        if l > 0:
            dz = (dz @ w.T) * (acts[l] > 0)
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss, flat


def adam(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
