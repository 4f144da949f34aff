"""Pins of the FP64 network oracle: central finite differences of the loss,
the GELU closed form, and one Adam step from its definition."""
import math

import numpy as np
import pytest

from oracle import mlp
from workloads import mlp_init


def test_gelu_reference_values():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    ref = np.array([0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))) for v in z])
    assert np.allclose(mlp.gelu(z), ref, rtol=0, atol=1e-15)
    # derivative against a central difference
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-9)


def test_gradient_matches_central_differences():
    n_in, n_h, n_l, n_out = 7, 5, 3, 4
    shapes = mlp.layer_shapes(n_in, n_h, n_l, n_out)
    p = mlp_init.initial_params(n_in, n_h, n_l, n_out, seed=3)
    p = p + np.random.default_rng(4).normal(scale=0.1, size=p.size)  # non-zero biases
    rng = np.random.default_rng(5)
    x = rng.normal(size=(6, n_in))
    t = rng.normal(size=(6, n_out))
    loss, g = mlp.loss_and_grad(p, x, t, shapes)
    h = 1e-6
    for k in rng.choice(p.size, size=40, replace=False):
        e = np.zeros(p.size)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, x, t, shapes)[0] - mlp.loss_and_grad(p - e, x, t, shapes)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    assert mlp.param_count(n_in, n_h, n_l, n_out) == p.size


def test_adam_first_step_is_signed_learning_rate():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_network_size_of_warm_start():
    n = mlp.param_count(mlp_init.N_IN, mlp_init.N_HIDDEN, mlp_init.N_LAYERS, mlp_init.N_OUT)
    assert n == 552 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 16384 + 16384
