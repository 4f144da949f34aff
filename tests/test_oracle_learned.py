"""Pins of the warm-start plumbing: the interpolation reproduces polynomials
of degree <= 7 and is the identity at the time nodes."""
import numpy as np
import pytest

from oracle import learned


def test_time_nodes_span_the_window():
    n = learned.time_nodes(1000)
    assert n[0] == 0 and n[-1] == 1000 and all(a < b for a, b in zip(n, n[1:]))
    assert learned.time_nodes(11)[1] == 1
    with pytest.raises(ValueError):
        learned.time_nodes(10)
    n32 = learned.time_nodes(1000, 32)
    assert len(n32) == 32 and n32[0] == 0 and n32[-1] == 1000
    with pytest.raises(ValueError):
        learned.time_nodes(190, 32)


def test_interpolation_with_32_nodes_reproduces_degree_31_polynomials():
    n_T, dt = 1000, 0.005
    ts = np.array(learned.time_nodes(n_T, 32)) * dt
    w = learned.bary_weights(ts)
    coef = np.random.default_rng(3).normal(size=32) / np.arange(1, 33) ** 2
    x = lambda t: (t - 2.5) / 2.5                      # Chebyshev-friendly variable
    poly = lambda t: np.polynomial.chebyshev.chebval(x(t), coef)
    for k in (0, 1, 17, 333, 500, 999, 1000):
        row = learned.lagrange_row(k * dt, ts, w)
        assert row @ poly(ts) == pytest.approx(poly(k * dt), rel=1e-9, abs=1e-11)


def test_interpolation_reproduces_degree_seven_polynomials():
    n_T, dt = 1000, 0.005
    nodes = learned.time_nodes(n_T)
    ts = np.array(nodes) * dt
    w = learned.bary_weights(ts)
    coef = np.random.default_rng(0).normal(size=8)
    poly = lambda t: sum(c * t ** k for k, c in enumerate(coef))
    for k in (0, 1, 37, 500, 999, 1000):
        row = learned.lagrange_row(k * dt, ts, w)
        assert row @ poly(ts) == pytest.approx(poly(k * dt), rel=1e-10, abs=1e-10)


def test_apply_of_targets_recovers_node_values():
    n_T, dt = 200, 0.01
    rng = np.random.default_rng(1)
    g0 = [rng.normal(size=5) + 1j * rng.normal(size=5), np.zeros(3, dtype=complex)]
    nodes = learned.time_nodes(n_T)
    gn = [np.vstack([g0[0]] + [rng.normal(size=5) + 1j * rng.normal(size=5) for _ in range(7)]),
          np.zeros((8, 3), dtype=complex)]
    X, s = learned.features(g0, np.ones(8) * 0.05, 2 * 5 + learned.tail_len(), np.zeros((2, 4)))
    assert np.all(s == learned.item_rms(g0[0])) and np.allclose(X[0, -16:-8], 0.5)
    assert X[0, -4] == 1.0 and X[1, -4] == 0.0 and not X[1, :-16].any()
    Y = learned.targets(gn, s, 8 * 2 * 5)
    out = learned.apply(Y, s, g0, n_T, dt)
    for m, n in enumerate(nodes):
        assert np.allclose(out[0][n], gn[0][m], atol=1e-12)


def test_window_scale_of_vanishing_data_is_one():
    assert learned.window_scale([np.zeros(3, dtype=complex), np.zeros(0, dtype=complex)]) == 1.0


def test_item_positions_of_a_symmetric_grid():
    """Box centres of a 3 x 2 grid on a box symmetric about 0 are symmetric
    and lie inside (-1, 1)."""
    import workloads
    from oracle import swr
    cfg = dict(workloads.tiny_configs()[1], box_lo=[-6.0, -5.0], box_hi=[6.0, 5.0])
    pos = learned.item_positions(swr.Problem(cfg))
    assert pos.shape == (6, 4) and np.all(np.abs(pos) < 1) and not pos[:, 2:].any()
    assert np.allclose(np.sort(pos[:, 0]), -np.sort(pos[:, 0])[::-1])
    assert np.allclose(pos[:, 0].reshape(2, 3)[:, 1], 0.0)
