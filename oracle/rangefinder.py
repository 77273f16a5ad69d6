"""Range finder of the snapshots (oracle side).

RanLocalSolu returns the snapshot matrix Y = G~ Omega; the paper adds a QR
factorization at its end to return an orthonormal basis (Section 3), and the
randomized SVD it recalls (Section 2.3, Theorem average_spectral, after
Halko-Martinsson-Tropp) projects onto span(Y).  Here: Householder QR of Y,
SVD of the triangular factor, and truncation to the k leading left singular
vectors.  With k = s this is the paper's QR basis up to a rotation.
"""
from __future__ import annotations

import numpy as np


def sign_fix(Q: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (first index on ties)."""
    Q = Q.copy()
    idx = np.argmax(np.abs(Q), axis=0)
    sgn = np.sign(Q[idx, np.arange(Q.shape[1])])
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :]


def range_finder(Y: np.ndarray, k: int):
    """Y (n x s) -> (Q_k (n x k) orthonormal, singular values of Y (s,))."""
    Qh, R = np.linalg.qr(Y, mode="reduced")
    U, S, _ = np.linalg.svd(R)
    Qk = Qh @ U[:, :k]
    return sign_fix(Qk), S


def numerical_rank(sv: np.ndarray, tau: float) -> int:
    """Numerical tau-rank (Def. num_rank): the smallest rank of a matrix within
    spectral-norm distance tau.  By Eckart-Young the best rank-r approximation
    is at distance sigma_{r+1}, so this is the number of singular values above
    tau."""
    return int(np.count_nonzero(np.asarray(sv) > tau))


def adaptive_rank(sv: np.ndarray, k: int, rank_tol: float) -> int:
    """Rank kept for a sampled patch: k when rank_tol is 0, else the numerical
    rank of the snapshots at tau = rank_tol sigma_1, clamped to [1, k]."""
    if rank_tol <= 0.0:
        return k
    return max(1, min(k, numerical_rank(sv, rank_tol * sv[0])))


def projection_error(G: np.ndarray, Q: np.ndarray) -> float:
    """||G - Q Q^T G||_2 / ||G||_2, the local error of the elliptic and kinetic local tests."""
    E = G - Q @ (Q.T @ G)
    return float(np.linalg.norm(E, 2) / np.linalg.norm(G, 2))


def sin_max_angle(Qa: np.ndarray, Qb: np.ndarray) -> float:
    """sin of the largest principal angle between span(Qa) and span(Qb) (orthonormal inputs)."""
    E = Qb - Qa @ (Qa.T @ Qb)
    return float(np.linalg.norm(E, 2))
