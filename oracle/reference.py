"""FP64 plaintext reference convolutions (test infrastructure; see package doc).

Eq. 1 of Section 3.1: a convolution is the matrix product Z = I x W, where
row p = i*O_w + j of I (S x K, S = O_w*O_h, K = d^2*I_c) is the input patch
under output location (i, j), flattened, and column o of W (K x O_c) is filter
o flattened the same way.  Out-of-image pixels read as zero.  Tensors are laid
out as X[h][w][c], filters as Y[kh][kw][c][o] (d x d x I_c x O_c).

Eq. 2 of Section 4.1: W is approximated by W1 W2 (K x O'_c times O'_c x O_c);
W1 is a d x d conv with O'_c filters and W2 a 1x1 conv.  The best rank-O'_c
approximation in Frobenius norm is the truncated SVD (Eckart-Young-Mirsky).
"""
from __future__ import annotations

import numpy as np


def im2col(x: np.ndarray, d: int, stride: int, pad: int) -> np.ndarray:
    h, w, c = x.shape
    oh = (h + 2 * pad - d) // stride + 1
    ow = (w + 2 * pad - d) // stride + 1
    xp = np.zeros((h + 2 * pad, w + 2 * pad, c))
    xp[pad:pad + h, pad:pad + w, :] = x
    rows = np.empty((oh * ow, d * d * c))
    for i in range(oh):
        for j in range(ow):
            patch = xp[stride * i: stride * i + d, stride * j: stride * j + d, :]
            rows[i * ow + j] = patch.reshape(-1)  # order (kh, kw, c)
    return rows


def filters_as_matrix(weights: np.ndarray) -> np.ndarray:
    d1, d2, c, o = weights.shape
    return weights.reshape(d1 * d2 * c, o)  # row index (kh*d + kw)*c + ch


def conv2d(x: np.ndarray, weights: np.ndarray, stride: int = 1, pad: int = 0) -> np.ndarray:
    """Z[i][j][o] by Eq. 1 (im2col then one matrix product), float64."""
    d = weights.shape[0]
    h, w, _ = x.shape
    oh = (h + 2 * pad - d) // stride + 1
    ow = (w + 2 * pad - d) // stride + 1
    z = im2col(x, d, stride, pad) @ filters_as_matrix(weights)
    return z.reshape(oh, ow, weights.shape[3])


def compose_factors(w1: np.ndarray, w2: np.ndarray) -> np.ndarray:
    """d x d x I_c x O_c filters of the product W1 W2 (W2 given as O'_c x O_c)."""
    d1, d2, c, r = w1.shape
    return (filters_as_matrix(w1) @ w2).reshape(d1, d2, c, w2.shape[1])


def ffconv_reference(x, w1, w2, stride=1, pad=0, square=False):
    y = conv2d(x, w1, stride, pad)
    z = y @ w2  # 1x1 conv: per-pixel product over channels
    return z * z if square else z


def truncated_svd_factors(w_mat: np.ndarray, rank: int):
    """W (K x O_c) -> (W1 K x r, W2 r x O_c) minimising ||W - W1 W2||_F (Eq. 2)."""
    u, s, vt = np.linalg.svd(w_mat, full_matrices=False)
    w1 = u[:, :rank] * s[:rank]
    w2 = vt[:rank]
    return w1, w2
