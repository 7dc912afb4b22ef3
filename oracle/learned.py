"""FP64 reference of the learned initial-guess model: principal component
analysis of solution vectors and a two-hidden-layer tanh perceptron that maps
geometry coordinates to principal-component coefficients, trained by Adam on
the mean squared error.

Test infrastructure only (the GPU path does not use it).  The model is the
learned part that predicts starting vectors for the iterative solves; the
method's own residual decides whether a prediction is used.

Conventions shared with the device implementation
  - PCA of X [n][d]: mean m = column mean; basis U [k][d] = the k leading
    eigenvectors of the covariance (X - m)^T (X - m), orthonormal rows, sign
    fixed so that the largest-magnitude element of each row is positive;
    coefficients C = (X - m) U^T.
  - Perceptron with layer sizes (nin, nh, nh, nout):
        h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3,
    W_l [out][in] row-major; the parameter vector is
    [W1 | b1 | W2 | b2 | W3 | b3].
  - Loss over a batch of B samples: (1 / (2 B)) sum_b sum_j (y_bj - t_bj)^2.
  - Adam: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    p -= lr * (m / (1 - b1^s)) / (sqrt(v / (1 - b2^s)) + eps), step s >= 1.
"""
import numpy as np


def pca_fit(X, k):
    X = np.asarray(X, dtype=np.float64)
    m = X.mean(axis=0)
    Xc = X - m
    # leading eigenvectors of Xc^T Xc from those of the Gram matrix Xc Xc^T
    w, V = np.linalg.eigh(Xc @ Xc.T)
    order = np.argsort(w)[::-1][:k]
    w, V = w[order], V[:, order]
    U = (Xc.T @ V) / np.sqrt(np.maximum(w, 1e-300))
    U = U.T
    for i in range(U.shape[0]):
        j = np.argmax(np.abs(U[i]))
        if U[i, j] < 0:
            U[i] = -U[i]
    return m, U, Xc @ U.T, w


def layer_shapes(nin, nh, nout):
    return [(nh, nin), (nh,), (nh, nh), (nh,), (nout, nh), (nout,)]


def unpack(p, nin, nh, nout):
    out, off = [], 0
    for s in layer_shapes(nin, nh, nout):
        n = int(np.prod(s))
        out.append(p[off:off + n].reshape(s))
        off += n
    return out


def nparams(nin, nh, nout):
    return sum(int(np.prod(s)) for s in layer_shapes(nin, nh, nout))


def forward(p, X, nin, nh, nout):
    W1, b1, W2, b2, W3, b3 = unpack(p, nin, nh, nout)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3, (h1, h2)


def loss_and_grad(p, X, T, nin, nh, nout):
    """Loss and its gradient by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(p, nin, nh, nout)
    B = X.shape[0]
    Y, (h1, h2) = forward(p, X, nin, nh, nout)
    E = Y - T
    loss = 0.5 * np.sum(E * E) / B
    dY = E / B
    gW3 = dY.T @ h2
    gb3 = dY.sum(axis=0)
    d2 = (dY @ W3) * (1.0 - h2 * h2)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def train(p, X, T, nin, nh, nout, order, batch, lr=1e-3):
    """Adam over the minibatches given by `order` (a list of index arrays);
    returns the parameters and the loss of every step."""
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for s, idx in enumerate(order, start=1):
        loss, g = loss_and_grad(p, X[idx], T[idx], nin, nh, nout)
        p, m, v = adam_step(p, g, m, v, s, lr)
        losses.append(loss)
    return p, np.array(losses)
