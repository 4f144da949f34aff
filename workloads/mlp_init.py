"""Seeded initial parameters of the warm-start network (plain random draws).

Weights of a layer with fan-in n are uniform in [-sqrt(6/n)/2, sqrt(6/n)/2]
(a scaled Kaiming-uniform draw), biases are zero.  The layout is one flat
vector, layer by layer, weight matrix (out x in, row-major) then bias.
"""
import numpy as np

# network of the learned warm start of the two-electron workload
N_IN, N_HIDDEN, N_LAYERS, N_OUT = 552, 256, 3, 16384


def initial_params(n_in=N_IN, n_hidden=N_HIDDEN, n_layers=N_LAYERS, n_out=N_OUT, seed=2401):
    rng = np.random.default_rng(seed)
    dims = [n_in] + [n_hidden] * n_layers + [n_out]
    parts = []
    for l in range(len(dims) - 1):
        fan_in, fan_out = dims[l], dims[l + 1]
        a = 0.5 * np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-a, a, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
