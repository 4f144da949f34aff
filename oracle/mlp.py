"""FP64 reference of the learned warm start's network: a multilayer
perceptron with exact-erf GELU, mean-squared-error loss and Adam.

This part is not in the paper.  The paper leaves the Schwarz initial guess
psi^(0) free (Section 4.1: "a given function"); the learned warm start
predicts it.  The network here is the plain textbook definition, written
out layer by layer:
  h_0 = x;  h_l = GELU(h_{l-1} W_l^T + b_l) for the hidden layers;
  y = h_L W_out^T + b_out;  GELU(z) = z/2 (1 + erf(z/sqrt 2));
  loss = mean over all entries of (y - t)^2;
  Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  p -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
Parameters are one flat vector, layer by layer, each layer its weight
matrix (out x in, row-major) followed by its bias.

Pinned by: central finite differences of the loss (gradient), the GELU
closed form at reference points, and a one-step Adam update written from
its definition in the test.
"""
import numpy as np
from scipy.special import erf


def layer_shapes(n_in, n_hidden, n_layers, n_out):
    dims = [n_in] + [n_hidden] * n_layers + [n_out]
    return [(dims[l + 1], dims[l]) for l in range(len(dims) - 1)]


def param_count(n_in, n_hidden, n_layers, n_out):
    return sum(o * i + o for o, i in layer_shapes(n_in, n_hidden, n_layers, n_out))


def unpack(params, shapes):
    out, off = [], 0
    for o, i in shapes:
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(params, x, shapes):
    layers = unpack(params, shapes)
    h = x
    cache = []
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if l < len(layers) - 1 else z
    return h, cache


def loss_and_grad(params, x, t, shapes):
    y, cache = forward(params, x, shapes)
    layers = unpack(params, shapes)
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / y.size
    grads = []
    d = dy
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h_in, z = cache[l]
        if l < len(layers) - 1:
            d = d * gelu_grad(z)
        gW = d.T @ h_in
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        d = d @ W
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
