"""Pins of the learned-guess oracle against facts that do not use its own
formulas: finite differences of the loss, exact PCA of data with a known
covariance, and the closed form of a first Adam step."""
import numpy as np

from oracle import learned as L


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    nin, nh, nout, B = 5, 7, 4, 6
    p = rng.normal(0, 0.4, L.nparams(nin, nh, nout))
    X = rng.normal(size=(B, nin))
    T = rng.normal(size=(B, nout))
    _, g = L.loss_and_grad(p, X, T, nin, nh, nout)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (L.loss_and_grad(p + e, X, T, nin, nh, nout)[0] - L.loss_and_grad(p - e, X, T, nin, nh, nout)[0]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-8 * max(1.0, np.abs(g).max())


def test_forward_reduces_to_affine_map_for_small_weights():
    """tanh(z) = z + O(z^3): with tiny hidden weights the network is the
    product of its three affine maps to third order."""
    rng = np.random.default_rng(1)
    nin, nh, nout = 3, 5, 2
    p = rng.normal(0, 1e-3, L.nparams(nin, nh, nout))
    W1, b1, W2, b2, W3, b3 = L.unpack(p, nin, nh, nout)
    X = rng.normal(size=(4, nin))
    lin = ((X @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    Y, _ = L.forward(p, X, nin, nh, nout)
    assert np.abs(Y - lin).max() < 1e-12


def test_pca_recovers_known_axes_and_variances():
    """Data on k orthonormal axes with distinct, exactly known second
    moments (balanced +-1 patterns): PCA returns those axes, variances and
    reconstructs the data exactly."""
    rng = np.random.default_rng(2)
    d, k = 40, 3
    Q, _ = np.linalg.qr(rng.normal(size=(d, k)))
    scales = np.array([3.0, 2.0, 0.5])
    # 8 samples, columns of a Hadamard-type sign pattern: zero mean, orthogonal
    S = np.array([[1, 1, 1], [1, 1, -1], [1, -1, 1], [1, -1, -1],
                  [-1, 1, 1], [-1, 1, -1], [-1, -1, 1], [-1, -1, -1]], dtype=float)
    mean = rng.normal(size=d)
    X = mean + (S * scales) @ Q.T
    m, U, C, w = L.pca_fit(X, k)
    assert np.abs(m - mean).max() < 1e-12
    assert np.abs(w - 8 * scales ** 2).max() < 1e-10
    assert np.abs(np.abs(U @ Q) - np.eye(k)).max() < 1e-10
    assert np.abs(U @ U.T - np.eye(k)).max() < 1e-12
    assert np.abs(m + C @ U - X).max() < 1e-12
    for i in range(k):
        assert U[i, np.argmax(np.abs(U[i]))] > 0


def test_first_adam_step_is_signed_learning_rate():
    """At step 1 the bias-corrected moments are g and g^2, so every
    parameter moves by -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    p1, m, v = L.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_decreases_loss_on_a_smooth_map():
    rng = np.random.default_rng(3)
    nin, nh, nout = 2, 16, 3
    X = rng.normal(size=(64, nin))
    T = np.stack([np.sin(X[:, 0]), X[:, 0] * X[:, 1], np.cos(X[:, 1])], axis=1)
    p = rng.normal(0, 0.3, L.nparams(nin, nh, nout))
    order = [rng.permutation(64)[:16] for _ in range(300)]
    _, losses = L.train(p, X, T, nin, nh, nout, order, 16, lr=1e-2)
    assert losses[-20:].mean() < 0.2 * losses[:5].mean()
