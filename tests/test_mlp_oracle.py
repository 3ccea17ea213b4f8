"""Pins for the FP64 reference of the learned cost model (CPU only)."""
import numpy as np

from oracle import mlp as M


def test_hand_computed_two_unit_network():
    # x = [1, 2]; W1 = [[1, -1], [2, 1]], b1 = [0, 0.5] -> z1 = [5, 1.5] (both
    # positive, so h = z1); W2 = [[1], [-2]], b2 = 0.25 -> y = 5 - 3 + 0.25 = 2.25.
    # t = 1: loss = 1.25^2 = 1.5625, dL/dy = 2.5; dW2 = h^T 2.5 = [12.5, 3.75],
    # db2 = 2.5; dh = 2.5 W2^T = [2.5, -5]; dW1 = x^T dh = [[2.5, -5], [5, -10]],
    # db1 = [2.5, -5].
    dims = [2, 2, 1]
    p = np.array([1, -1, 2, 1, 0, 0.5, 1, -2, 0.25])
    acts = M.forward(p, dims, np.array([[1.0, 2.0]]))
    assert acts[-1][0, 0] == 2.25
    loss, g = M.loss_and_grad(p, dims, np.array([[1.0, 2.0]]), np.array([1.0]))
    assert loss == 1.5625
    np.testing.assert_array_equal(g, [2.5, -5, 5, -10, 2.5, -5, 12.5, 3.75, 2.5])


def test_relu_blocks_gradient():
    dims = [1, 1, 1]
    p = np.array([-1.0, 0.0, 3.0, 0.0])   # z1 = -x < 0 for x > 0: output constant 0
    loss, g = M.loss_and_grad(p, dims, np.array([[2.0]]), np.array([1.0]))
    assert loss == 1.0
    np.testing.assert_array_equal(g[:2], [0.0, 0.0])
    np.testing.assert_array_equal(g[2:], [0.0, -2.0])


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    dims = [6, 5, 4, 1]
    n = sum(a * b + b for a, b in zip(dims[:-1], dims[1:]))
    p = rng.normal(size=n) * 0.5
    x = rng.normal(size=(9, 6))
    t = rng.normal(size=9)
    _, g = M.loss_and_grad(p, dims, x, t)
    num = np.zeros(n)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        num[i] = (M.loss_and_grad(p + e, dims, x, t)[0] - M.loss_and_grad(p - e, dims, x, t)[0]) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-9)


def test_adam_first_step():
    # step 1 from zero moments: m_hat = g, v_hat = g^2, so the update is
    # lr * g / (|g| + eps) = lr * sign(g) for |g| >> eps.
    p, m, v = M.adam(np.array([1.0, 1.0]), np.array([0.5, -4.0]), np.zeros(2), np.zeros(2), 1, 0.01)
    np.testing.assert_allclose(p, [0.99, 1.01], rtol=0, atol=1e-9)
    np.testing.assert_allclose(m, [0.05, -0.4])
    np.testing.assert_allclose(v, [0.00025, 0.016])


def test_adam_constant_gradient_steps_unbiased():
    # With the same gradient g at every step the moments are
    # m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias-corrected
    # estimates are exactly g and g^2 at every step t and each step moves
    # the parameter by lr * g / (|g| + eps).  A correction by b1 (instead of
    # b1^t) would move step 2 by lr * 1.9 / sqrt(1.999) = 1.3439 lr instead.
    g = np.array([0.5, -4.0])
    p, m, v = np.array([1.0, 1.0]), np.zeros(2), np.zeros(2)
    for step in (1, 2, 3):
        p, m, v = M.adam(p, g, m, v, step, 0.01)
        np.testing.assert_allclose(m, (1 - 0.9 ** step) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** step) * g * g, rtol=1e-12)
        np.testing.assert_allclose(p, 1.0 - step * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_adam_second_and_third_step_by_hand():
    # gradient 1 at step 1, then 0 at steps 2 and 3, lr = 1, eps = 0:
    #   step 1: m = 0.1, v = 0.001; m^ = 1, v^ = 1 -> p = 1 - 1 = 0
    #   step 2: m = 0.09, v = 0.000999; m^ = 0.09 / 0.19 = 9/19,
    #           v^ = 0.000999 / 0.001999 = 999/1999 -> p = -(9/19) / sqrt(999/1999)
    #   step 3: m = 0.081, v = 0.000998001; m^ = 0.081 / 0.271 = 81/271,
    #           v^ = 0.000998001 / 0.002997001 = 998001/2997001
    p, m, v = M.adam(np.array([1.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, 1.0, eps=0.0)
    np.testing.assert_allclose(p, [0.0], atol=1e-15)
    p, m, v = M.adam(p, np.array([0.0]), m, v, 2, 1.0, eps=0.0)
    p2 = -(9 / 19) / np.sqrt(999 / 1999)
    np.testing.assert_allclose(p, [p2], rtol=1e-12)
    p, m, v = M.adam(p, np.array([0.0]), m, v, 3, 1.0, eps=0.0)
    np.testing.assert_allclose(m, [0.081], rtol=1e-12)
    np.testing.assert_allclose(v, [0.000998001], rtol=1e-12)
    np.testing.assert_allclose(p, [p2 - (81 / 271) / np.sqrt(998001 / 2997001)], rtol=1e-12)
