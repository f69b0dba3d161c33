"""Pins of the FP64 surrogate reference: finite differences, closed forms."""
import math

import numpy as np

from oracle import mlp_ref as R


def small_net(rng, sizes):
    Ws = [rng.normal(0, 1 / math.sqrt(a), (b, a)) for a, b in zip(sizes[:-1], sizes[1:])]
    bs = [rng.normal(0, 0.1, b) for b in sizes[1:]]
    return Ws, bs


def test_gelu_and_derivative():
    # GELU(0) = 0, GELU(z) -> z for large z, -> 0 for very negative z
    assert R.gelu(np.array(0.0)) == 0.0
    assert abs(R.gelu(np.array(8.0)) - 8.0) < 1e-12
    assert abs(R.gelu(np.array(-8.0))) < 1e-12
    # Phi(1) from the normal CDF: 0.841344746...
    assert abs(R.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    z = np.linspace(-4, 4, 41)
    fd = (R.gelu(z + 1e-6) - R.gelu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(R.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [32, 16, 12, 10]
    Ws, bs = small_net(rng, sizes)
    x = rng.normal(size=(7, 32))
    t = rng.normal(size=(7, 10))
    mask = (rng.random((7, 10)) > 0.3).astype(float)
    loss, gW, gb = R.loss_and_grads(x, t, mask, Ws, bs)
    eps = 1e-6
    for l in range(len(Ws)):
        for (i, j) in [(0, 0), (1, 3), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += eps
            Wm[l][i, j] -= eps
            fd = (R.loss_and_grads(x, t, mask, Wp, bs)[0] - R.loss_and_grads(x, t, mask, Wm, bs)[0]) / (2 * eps)
            assert abs(gW[l][i, j] - fd) <= 1e-6 * max(abs(fd), 1e-3), (l, i, j)
        k = bs[l].size // 2
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][k] += eps
        bm[l][k] -= eps
        fd = (R.loss_and_grads(x, t, mask, Ws, bp)[0] - R.loss_and_grads(x, t, mask, Ws, bm)[0]) / (2 * eps)
        assert abs(gb[l][k] - fd) <= 1e-6 * max(abs(fd), 1e-3)


def test_linear_network_closed_form():
    """No hidden layer: the output is x W^T + b exactly."""
    rng = np.random.default_rng(1)
    W, b = rng.normal(size=(4, 32)), rng.normal(size=4)
    x = rng.normal(size=(3, 32))
    y, _ = R.forward(x, [W], [b])
    np.testing.assert_allclose(y, x @ W.T + b, rtol=1e-15)


def test_encode():
    lo = np.array([0, 0, 0, 5, -50, 50, 1, 20, 1, 0.5, 1, 1], dtype=float)
    hi = np.array([10, 20, 360, 85, 50, 300, 5, 100, 3, 2, 1, 1], dtype=float)
    p = np.array([[10, 5, 90, 45, 0, 175, 3, 60, 2, 0.5, 1, 1]], dtype=float)
    x = R.encode(p, lo, hi)
    np.testing.assert_allclose(x[0, :11], [1.0, -0.5, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0],
                               atol=1e-15)
    assert x.shape == (1, 32) and np.all(x[0, 11:] == 0)


def test_adam_first_step_is_sign_lr():
    """After one step from zero moments Adam moves each weight by lr * sign(g)
    (up to eps)."""
    w, g = np.array([1.0, -2.0, 3.0]), np.array([0.5, -4.0, 1e-3])
    w2, m, v = R.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(w - w2, 0.01 * np.sign(g), rtol=1e-4)


def test_masked_mse_hand_computed():
    """A 2-input linear network (no hidden layer), 2 rows x 4 outputs, a partial
    mask: y = x W^T + b worked out by hand.  Row 0 gives y = (1, 1, 0, 2.5)
    against t = (0, 1, 1, 2) with mask (1, 1, 0, 1): masked residuals
    (1, 0, -, 0.5); row 1 gives y = (2, 2, 0, 0.5) against t = (2, 0, 0, 1)
    with mask (0, 1, 1, 1): residuals (-, 2, 0, -0.5).  Sum of squares
    1 + 0.25 + 4 + 0.25 = 5.5 over 6 unmasked entries: loss 11/12 (not
    5.5/8, the mean over every entry).  d loss / d y = 2 r / 6, so the bias
    gradient is the column sum (1/3, 2/3, 0, 0) and d loss / d W[0][0] =
    (1/3) x[0][0] = 1/3, d loss / d W[3][1] = (1/6)(0) + (-1/6)(1) = -1/6."""
    x = np.array([[1.0, 0.0], [0.0, 1.0]])
    W = np.array([[1.0, 2.0], [0.0, 1.0], [1.0, 1.0], [2.0, 0.0]])
    b = np.array([0.0, 1.0, -1.0, 0.5])
    t = np.array([[0.0, 1.0, 1.0, 2.0], [2.0, 0.0, 0.0, 1.0]])
    mask = np.array([[1.0, 1.0, 0.0, 1.0], [0.0, 1.0, 1.0, 1.0]])
    loss, gW, gb = R.loss_and_grads(x, t, mask, [W], [b])
    assert abs(loss - 11.0 / 12.0) < 1e-15
    np.testing.assert_allclose(gb[0], [1.0 / 3.0, 2.0 / 3.0, 0.0, 0.0], atol=1e-15)
    assert abs(gW[0][0, 0] - 1.0 / 3.0) < 1e-15
    assert abs(gW[0][3, 1] - (-1.0 / 6.0)) < 1e-15
    # a fully masked batch has zero loss and zero gradients
    loss0, gW0, gb0 = R.loss_and_grads(x, t, np.zeros_like(mask), [W], [b])
    assert loss0 == 0.0 and not gW0[0].any() and not gb0[0].any()


def test_adam_three_steps_closed_forms():
    """Bias-corrected Adam over three steps, in closed form.
    Constant gradient g: m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    corrected moments are g and g^2 and every step moves by lr g / (|g| + eps).
    Alternating +g, -g, +g: m_2 = -(1 - b1)^2 g, corrected -(1 - b1)/(1 + b1) g
    = -g/19, and v_2 corrected = g^2, so step 2 is -lr/19 sign g;
    m_3 = (1 - b1)(1 - b1 (1 - b1)) g = 0.091 g, corrected 0.091/0.271 g, so
    step 3 is (91/271) lr sign g.  A bias correction with the wrong power of t
    moves steps 2 and 3."""
    lr, g = 0.01, np.array([0.5, -4.0, 2.0])
    w, m, v = np.array([1.0, -2.0, 3.0]), np.zeros(3), np.zeros(3)
    for t in (1, 2, 3):
        w2, m, v = R.adam_step(w, g, m, v, t, lr=lr)
        np.testing.assert_allclose(w - w2, lr * g / (np.abs(g) + 1e-8), rtol=1e-13)
        w = w2
    w, m, v = np.array([1.0, -2.0, 3.0]), np.zeros(3), np.zeros(3)
    expect = (1.0, -1.0 / 19.0, 91.0 / 271.0)
    for t, sgn in zip((1, 2, 3), (1.0, -1.0, 1.0)):
        w2, m, v = R.adam_step(w, sgn * g, m, v, t, lr=lr)
        np.testing.assert_allclose(w - w2, expect[t - 1] * lr * np.sign(g), rtol=1e-7)
        w = w2
