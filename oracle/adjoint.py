"""Adjoint of the reweighted fit with the reweighting set held fixed
(test infrastructure; see the package docstring).

Sec. 4 steps 9-10 define the end of the fit: with W the rows whose squared
distance under the raw fit does not exceed the cutoff,

    mu    = (1/n_w) sum_{j in W} x_j
    Sigma = c / (n_w - 1) sum_{j in W} (x_j - mu)(x_j - mu)^T     (c = 1, or
            the consistency factor when it is applied)
    d_i   = sqrt((x_i - mu)^T Sigma^{-1} (x_i - mu))   for every row i
            (eq. statdist).

W (like the h-subsets before it) is a step function of X, constant away from
ties at the cutoff, so wherever the fit is differentiable its derivative is
that of the three formulas above with W fixed.  ``fixed_set_forward`` writes
them out; ``adjoint`` is their reverse-mode derivative, derived by hand:

    r_i = x_i - mu,  P = Sigma^{-1},  w_i = v_i / d_i  (v = cotangent of d)
    direct:   g_i  = w_i P r_i                                  (every row)
    g_mu   = gbar_mu - P sum_i w_i r_i
    G      = Gbar_Sigma - 1/2 P (sum_i w_i r_i r_i^T) P
    W rows:   g_j += g_mu / n_w + c / (n_w - 1) (G + G^T) (x_j - mu)

The closed form is pinned by central finite differences of
``fixed_set_forward`` (a separate computation) in the tests.
"""
from __future__ import annotations

import numpy as np


def fixed_set_forward(X: np.ndarray, W: np.ndarray, c: float = 1.0):
    """(mu, Sigma, d) of Sec. 4 steps 9-10 for a fixed reweighting set W."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=bool)
    XW = X[W]
    n_w = XW.shape[0]
    mu = XW.mean(axis=0)
    R = XW - mu
    Sigma = c * (R.T @ R) / (n_w - 1)
    Rall = X - mu
    y = np.linalg.solve(Sigma, Rall.T).T
    d = np.sqrt(np.maximum(np.einsum("ij,ij->i", Rall, y), 0.0))
    return mu, Sigma, d


def adjoint(X: np.ndarray, W: np.ndarray, c: float, g_d=None, g_mu=None, g_sigma=None):
    """Gradient of <g_d, d> + <g_mu, mu> + <g_sigma, Sigma> with respect to X
    (n x p, float64), W held fixed.  Rows with d_i = 0 get no direct term."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=bool)
    n, p = X.shape
    mu, Sigma, d = fixed_set_forward(X, W, c)
    n_w = int(W.sum())
    P = np.linalg.inv(Sigma)
    P = 0.5 * (P + P.T)
    R = X - mu
    v = np.zeros(n) if g_d is None else np.asarray(g_d, dtype=np.float64)
    w = np.where(d > 0.0, v / np.where(d > 0.0, d, 1.0), 0.0)
    PR = R @ P                                  # rows: P r_i
    G_X = w[:, None] * PR                       # direct term
    gmu = (np.zeros(p) if g_mu is None else np.asarray(g_mu, float)) - P @ (w @ R)
    B = (R * w[:, None]).T @ R                  # sum_i w_i r_i r_i^T
    G = (np.zeros((p, p)) if g_sigma is None else np.asarray(g_sigma, float)) - 0.5 * P @ B @ P
    K = c / (n_w - 1) * (G + G.T)
    G_X[W] += gmu / n_w + R[W] @ K.T
    return G_X
