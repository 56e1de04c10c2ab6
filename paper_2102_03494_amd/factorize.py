"""Low-rank factorisation of a convolution's weights (Eq. 2, Section 4.1).

A d x d convolution with weights W (d x d x I_c x O_c, read as the K x O_c
matrix of Eq. 1, K = d^2 I_c) is replaced by a d x d convolution with
O'_c = r filters, W1 (K x r), followed by a 1 x 1 convolution W2 (r x O_c).
The pair minimising ||W - W1 W2||_F over rank-r products is the truncated
singular value decomposition (Eckart-Young-Mirsky).

Computed here through the eigendecomposition of the O_c x O_c Gram matrix
W^T W = V diag(s^2) V^T: with V_r the eigenvectors of the r largest
eigenvalues, W2 = V_r^T (orthonormal rows) and W1 = W V_r, so W1 W2 is the
projection of W's rows onto its top-r right singular subspace -- the same
product as the truncated SVD.  This is host-side weight preparation (the
server runs it once per model), not part of the encrypted evaluation.
"""
from __future__ import annotations

import numpy as np


def as_matrix(w: np.ndarray) -> np.ndarray:
    """d x d x I_c x O_c filters -> K x O_c (row (kh d + kw) I_c + c, as Eq. 1)."""
    d1, d2, c, o = w.shape
    return np.asarray(w, dtype=np.float64).reshape(d1 * d2 * c, o)


def singular_values(w: np.ndarray) -> np.ndarray:
    """Singular values of W's K x O_c matrix, largest first."""
    evals = np.linalg.eigvalsh(as_matrix(w).T @ as_matrix(w))
    return np.sqrt(np.clip(evals[::-1], 0.0, None))


def factorize(w: np.ndarray, rank: int):
    """(W1 as d x d x I_c x r filters, W2 as r x O_c) minimising ||W - W1 W2||_F."""
    d1, d2, c, o = w.shape
    wm = as_matrix(w)
    if not 1 <= rank <= min(wm.shape):
        raise ValueError(f"rank {rank} outside 1..{min(wm.shape)}")
    evals, evecs = np.linalg.eigh(wm.T @ wm)
    top = np.argsort(evals)[::-1][:rank]
    v = evecs[:, top]
    w1 = (wm @ v).reshape(d1, d2, c, rank)
    return w1, np.ascontiguousarray(v.T)


def relative_error(w: np.ndarray, w1: np.ndarray, w2: np.ndarray) -> float:
    """||W - W1 W2||_F / ||W||_F."""
    wm = as_matrix(w)
    return float(np.linalg.norm(wm - as_matrix(w1) @ w2) / np.linalg.norm(wm))


def with_spectrum(left: np.ndarray, right: np.ndarray, sigma: np.ndarray, shape) -> np.ndarray:
    """Weights of the given shape (d x d x I_c x O_c) whose K x O_c matrix has
    singular values `sigma`, from two Gaussian matrices (K x m and O_c x m,
    m = len(sigma)) orthonormalised by QR: Q_left diag(sigma) Q_right^T."""
    m = len(sigma)
    ql, _ = np.linalg.qr(left)
    qr, _ = np.linalg.qr(right)
    return ((ql[:, :m] * sigma) @ qr[:, :m].T).reshape(shape)
