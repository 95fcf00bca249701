"""FP64 reference of the per-rank-column warm-start network.

The paper has no learned component; this is the reference for the network the
library adds on top of the paper's "optimal guess" (warm start from the
previous converged CPD, Section "An improved initial guess strategy").

Network: L linear layers with ReLU between them,
    h_0 = x,  h_l = relu(h_{l-1} W_l^T + b_l)  (l < L),  y = h_{L-1} W_L^T + b_L,
loss = mean over all output elements of (y - target)^2, and Adam
(Kingma & Ba, arXiv:1412.6980, Algorithm 1) with bias correction.

Parameter order everywhere: W_1, b_1, W_2, b_2, ..., W_L, b_L, each W_l of
shape (fan_out, fan_in), row-major.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def forward(params, x):
    """Returns (output, list of layer inputs, list of pre-activations)."""
    n_layers = len(params) // 2
    h = x
    inputs, pre = [], []
    for layer in range(n_layers):
        w, b = params[2 * layer], params[2 * layer + 1]
        inputs.append(h)
        z = h @ w.T + b
        pre.append(z)
        h = np.maximum(z, 0.0) if layer < n_layers - 1 else z
    return h, inputs, pre


def loss_and_grads(params, x, target):
    """MSE loss and its gradient with respect to every parameter (backpropagation)."""
    y, inputs, pre = forward(params, x)
    diff = y - target
    loss = float(np.mean(diff * diff))
    n_layers = len(params) // 2
    grads = [None] * len(params)
    g = 2.0 * diff / diff.size
    for layer in reversed(range(n_layers)):
        if layer < n_layers - 1:
            g = g * (pre[layer] > 0.0)
        grads[2 * layer] = g.T @ inputs[layer]
        grads[2 * layer + 1] = g.sum(axis=0)
        g = g @ params[2 * layer]
    return loss, grads


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; ``step`` counts from 1."""
    for k in range(len(params)):
        m[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] * grads[k]
        mhat = m[k] / (1.0 - beta1 ** step)
        vhat = v[k] / (1.0 - beta2 ** step)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params, m, v


def train(params, x, target, epochs, lr=1e-3, batch=None):
    """Full-batch (or in-order mini-batch) Adam training; returns (params, loss history)."""
    params = [p.astype(np.float64).copy() for p in params]
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    n = x.shape[0]
    batch = n if batch is None else batch
    step = 0
    hist = []
    for _ in range(epochs):
        for s in range(0, n, batch):
            step += 1
            loss, g = loss_and_grads(params, x[s:s + batch], target[s:s + batch])
            params, m, v = adam_step(params, g, m, v, step, lr)
        hist.append(loss_and_grads(params, x, target)[0])
    return params, hist
