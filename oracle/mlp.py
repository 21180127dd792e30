"""Learned correction to the diagonal Davidson preconditioner (oracle).

Test infrastructure: imported only by tests.

The paper solves each two-site problem with an iterative eigensolver and
leaves the preconditioner open (Sec. 2.1, "solving").  The library offers,
besides the diagonal preconditioner t_i = r_i / (theta - H_ii), a learned
per-element correction: a small multilayer perceptron maps features of
element i to g_i and the correction becomes

    t_i = d_i r_i exp(clamp(g_i, -3, 3)),    d_i = 1 / (theta - H_ii)

(with |theta - H_ii| clamped to >= 1e-12 as in the diagonal case).  None of
this is in the paper; the definitions below are this project's and the
library implements them independently.

Network: F=12 inputs -> 64 tanh -> 64 tanh -> 1 linear.  Parameters are one
flat vector in the order W1 (64 x F, row-major), b1 (64), W2 (64 x 64), b2
(64), w3 (64), b3 (1).  Loss: mean over the batch of (g - target)^2.
Training: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).

Features of element i of the two-site vector (sector (Q_l, s, t, Q_r)):
  0  (theta - H_ii) / max(1, |theta|)
  1  log(max(|theta - H_ii|, 1e-12)) / 10
  2  r_i sqrt(n) / ||r||          (0 when ||r|| = 0)
  3  u_i sqrt(n)                  (u: current Ritz vector, unit norm)
  4  N(Q_l) / max(1, N)           5  2S_z(Q_l) / max(1, N)
  6  n(s) / 2                     7  n(t) / 2
  8  2s_z(s)                      9  2s_z(t)
  10 log(1 + m(Q_l)) / 8          11 (j + 0.5) / K for the pair (j, j+1)
Features 4..11 depend only on the layout ("static features").

Training target of element i at Davidson iteration k (u = u_k, r = r_k):
the ideal correction t* = psi - (psi . u) u, psi the converged vector of the
step; alpha = (t* . dr) / (t* . t*) over the sampled elements with dr = d r
(the least-squares scale of t* onto the diagonal correction); then
rho_i = alpha t*_i / dr_i and target_i = clamp(log rho_i, -3, 3) if rho_i > 0,
-3 if rho_i <= 0 and 0 where dr_i = 0.

Parity: forward is pinned by closed forms (zero second layer; a single
active unit), the gradient by central finite differences in FP64, the first
Adam step by its closed form lr * sign(g); features and targets by direct
element-wise definitions checked on hand-made cases.
"""

from __future__ import annotations

import numpy as np

N_FEATURES = 12
HIDDEN = 64


def n_params(F=N_FEATURES, H=HIDDEN):
    return H * F + H + H * H + H + H + 1


def unpack(p, F=N_FEATURES, H=HIDDEN):
    """Views of the flat parameter vector: W1, b1, W2, b2, w3, b3."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n_params(F, H)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, X):
    """g for each row of X (B x F); also returns the activations."""
    W1, b1, W2, b2, w3, b3 = unpack(p, X.shape[1])
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    g = h2 @ w3 + b3
    return g, (h1, h2)


def loss_and_grad(p, X, y):
    """Mean squared error over the batch and its gradient (flat, same order
    as the parameters), by the chain rule through the three layers."""
    W1, b1, W2, b2, w3, b3 = unpack(p, X.shape[1])
    B = X.shape[0]
    g, (h1, h2) = forward(p, X)
    e = g - y
    loss = float(np.mean(e * e))
    dg = 2.0 * e / B                      # dL/dg
    dw3 = h2.T @ dg
    db3 = dg.sum()
    dz2 = (dg[:, None] * w3[None, :]) * (1.0 - h2 * h2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
    return loss, grad


def adam_step(p, m, v, t, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update; t is the 1-based step number."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def clamp_den(theta, diag):
    """theta - H_ii with magnitudes below 1e-12 replaced by +-1e-12."""
    den = theta - np.asarray(diag, dtype=np.float64)
    small = np.abs(den) < 1e-12
    return np.where(small, np.where(den < 0, -1e-12, 1e-12), den)


def features(theta, diag, r, u, static):
    """Feature matrix (n x 12) from the dynamic quantities and the static
    features (n x 8, columns 4..11 above)."""
    diag = np.asarray(diag, dtype=np.float64)
    n = diag.size
    den = theta - diag
    rn = np.linalg.norm(r)
    X = np.zeros((n, N_FEATURES))
    X[:, 0] = den / max(1.0, abs(theta))
    X[:, 1] = np.log(np.maximum(np.abs(den), 1e-12)) / 10.0
    X[:, 2] = r * np.sqrt(n) / rn if rn > 0 else 0.0
    X[:, 3] = u * np.sqrt(n)
    X[:, 4:] = static
    return X


def static_features(N_l, sz_l, n_s, n_t, sz_s, sz_t, m_l, j, K, N):
    """Columns 4..11 of the features for arrays of per-element labels."""
    return np.stack([np.asarray(N_l) / max(1, N), np.asarray(sz_l) / max(1, N),
                     np.asarray(n_s) / 2.0, np.asarray(n_t) / 2.0,
                     np.asarray(sz_s, dtype=np.float64), np.asarray(sz_t, dtype=np.float64),
                     np.log1p(np.asarray(m_l, dtype=np.float64)) / 8.0,
                     np.full(len(N_l), (j + 0.5) / K)], axis=1)


def correction(theta, diag, r, g):
    """Learned correction t = d r exp(clamp(g, -3, 3))."""
    return r / clamp_den(theta, diag) * np.exp(np.clip(g, -3.0, 3.0))


def targets(psi_s, u_s, c, dr_s):
    """Targets at the sampled elements of one iteration: psi_s, u_s, dr_s
    are the sampled entries of the converged vector, the Ritz vector and
    the diagonal correction d r; c = psi . u over the whole vector."""
    ts = psi_s - c * u_s
    tt = float(ts @ ts)
    alpha = float(ts @ dr_s) / tt if tt > 0 else 0.0
    out = np.zeros_like(dr_s)
    nz = dr_s != 0
    rho = np.zeros_like(dr_s)
    rho[nz] = alpha * ts[nz] / dr_s[nz]
    pos = nz & (rho > 0)
    out[pos] = np.clip(np.log(rho[pos]), -3.0, 3.0)
    out[nz & ~pos] = -3.0
    return out
