"""From-scratch quantities that pin the oracle walker -- TEST INFRASTRUCTURE ONLY.

Nothing here tracks state: each function rebuilds products of propagators
from the field configuration X alone.

  * log_weight: Pi_s det(P_s^+ B_M ... B_1 P_s), the determinant part of the
    configuration weight W(X) (Eq. (8)); the product is re-orthonormalised
    every few slices and the dropped triangular factors' determinants are
    accumulated, so it stays accurate for M in the hundreds.
  * green_at: G_l = 1 - R (L R)^{-1} L with R = B_l ... B_1 P and
    L = P^+ B_M ... B_{l+1} (Eq. (12)), both re-orthonormalised on the way.
"""
from __future__ import annotations

import numpy as np

SPIN_SIGN = (+1.0, -1.0)


def b_diag(alpha, s, xrow):
    return np.exp(alpha * SPIN_SIGN[s] * np.asarray(xrow, np.float64))


def det_factor(P, K, alpha, s, X, every=4):
    """(phase, log|det|) of P^+ B_M ... B_1 P for spin s."""
    R = P.astype(np.result_type(P, alpha, np.float64))
    logabs, phase = 0.0, 1.0 + 0j
    for li in range(X.shape[0]):
        R = b_diag(alpha, s, X[li])[:, None] * (K @ R)
        if (li + 1) % every == 0 or li == X.shape[0] - 1:
            Q, Rf = np.linalg.qr(R)
            dg = np.diag(Rf)
            logabs += float(np.sum(np.log(np.abs(dg))))
            phase *= np.prod(dg / np.abs(dg))
            R = Q
    det = np.linalg.det(P.conj().T @ R)
    return phase * det / abs(det), logabs + float(np.log(abs(det)))


def log_weight(P2, K, alpha, X):
    """Sum over spins of det_factor: returns (phase, log|W|) up to P(X)."""
    ph, la = 1.0 + 0j, 0.0
    for s in range(2):
        p, l_ = det_factor(P2[s], K, alpha, s, X)
        ph *= p
        la += l_
    return ph, la


def weight_ratio(P2, K, alpha, X, Xp):
    """W(X')/W(X) as a complex number (P(X) is constant for the discrete field)."""
    p1, l1 = log_weight(P2, K, alpha, X)
    p2, l2 = log_weight(P2, K, alpha, Xp)
    return (p2 / p1) * np.exp(l2 - l1)


def spin_ratio(P, K, alpha, s, X, Xp):
    p1, l1 = det_factor(P, K, alpha, s, X)
    p2, l2 = det_factor(P, K, alpha, s, Xp)
    return (p2 / p1) * np.exp(l2 - l1)


def green_at(P, K, alpha, s, X, l, every=4):
    """G_l for spin s at position l (0..M) from scratch."""
    M = X.shape[0]
    dt = np.result_type(P, alpha, np.float64)
    R = P.astype(dt)
    for li in range(l):
        R = b_diag(alpha, s, X[li])[:, None] * (K @ R)
        if (li + 1) % every == 0:
            R = np.linalg.qr(R)[0]
    Lm = P.conj().T.astype(dt)
    for li in range(M - 1, l - 1, -1):
        Lm = (Lm * b_diag(alpha, s, X[li])[None, :]) @ K
        if (M - li) % every == 0:
            Lm = np.linalg.qr(Lm.conj().T)[0].conj().T
    N = P.shape[0]
    return np.eye(N) - R @ np.linalg.solve(Lm @ R, Lm)
