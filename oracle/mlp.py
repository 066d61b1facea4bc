"""Oracle: the small regression network of the learned window (test infrastructure only).

The learned extension predicts the spectral bound and the central density of states from
coupling statistics, so that the filter degree and the window (Sec. II.A, Sec. III
parameter settings) can be set without the Lanczos / kernel-polynomial estimates.  The
network is a multilayer perceptron: `layers` hidden layers of width `hidden` with tanh,
then a linear output layer; the loss is the mean over samples of 0.5 * |y - t|^2.

Parameters are one flat vector, layer by layer, each layer as W (n_out x n_in, row-major)
followed by its bias b (n_out).  Everything here is FP64 and written for clarity: forward
pass, then the backward pass of the chain rule, layer by layer.
"""
import numpy as np


def layer_dims(n_in, hidden, layers, n_out):
    """[(n_out_l, n_in_l)] for every layer, input to output."""
    dims = []
    prev = n_in
    for _ in range(layers):
        dims.append((hidden, prev))
        prev = hidden
    dims.append((n_out, prev))
    return dims


def n_params(n_in, hidden, layers, n_out):
    return sum(o * i + o for o, i in layer_dims(n_in, hidden, layers, n_out))


def unpack(theta, n_in, hidden, layers, n_out):
    """Views (W, b) of every layer in the flat parameter vector."""
    out = []
    pos = 0
    for o, i in layer_dims(n_in, hidden, layers, n_out):
        W = theta[pos:pos + o * i].reshape(o, i)
        pos += o * i
        b = theta[pos:pos + o]
        pos += o
        out.append((W, b))
    assert pos == theta.size
    return out


def forward(theta, X, n_in, hidden, layers, n_out):
    """Returns (Y, activations); activations[0] = X, activations[l] = tanh(z_l)."""
    acts = [np.asarray(X, dtype=np.float64)]
    params = unpack(np.asarray(theta, dtype=np.float64), n_in, hidden, layers, n_out)
    for li, (W, b) in enumerate(params):
        z = acts[-1] @ W.T + b
        if li < len(params) - 1:
            acts.append(np.tanh(z))
        else:
            return z, acts
    raise AssertionError("unreachable")


def loss_and_grad(theta, X, T, n_in, hidden, layers, n_out):
    """Mean-squared loss 0.5 mean_s |y_s - t_s|^2 and its gradient (flat, same layout)."""
    theta = np.asarray(theta, dtype=np.float64)
    Y, acts = forward(theta, X, n_in, hidden, layers, n_out)
    ns = Y.shape[0]
    R = Y - np.asarray(T, dtype=np.float64)
    loss = 0.5 * np.sum(R * R) / ns
    params = unpack(theta, n_in, hidden, layers, n_out)
    grads = [None] * len(params)
    delta = R / ns  # dloss / dz of the output layer
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        a_prev = acts[li]
        grads[li] = (delta.T @ a_prev, delta.sum(axis=0))
        if li > 0:
            delta = (delta @ W) * (1.0 - a_prev * a_prev)  # through tanh of layer li - 1
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), t counted from 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
