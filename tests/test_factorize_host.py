"""The product's low-rank factorisation (Eq. 2) against the oracle (no GPU).

The product computes the truncated SVD through the eigendecomposition of
W^T W; the oracle through numpy's SVD.  Pins: both give the same product
W1 W2; its squared error is the sum of the discarded squared singular values
(Eckart-Young-Mirsky, singular values from the oracle's SVD); W2's rows are
orthonormal; full rank reproduces W; a W built with a given spectrum has
exactly that spectrum.
"""
import numpy as np
import pytest

import synth
from oracle import reference as R
from paper_2102_03494_amd import factorize as F


@pytest.mark.parametrize("shape", [(5, 5, 1, 5), (3, 3, 3, 64), (3, 3, 8, 16), (1, 1, 12, 4)])
def test_factorize_matches_oracle_svd(shape):
    w = synth.weights("unit", 77, shape, 0.1)
    wm = R.filters_as_matrix(w)
    s = np.linalg.svd(wm, compute_uv=False)
    for r in range(1, min(wm.shape) + 1):
        w1, w2 = F.factorize(w, r)
        assert w1.shape == shape[:3] + (r,) and w2.shape == (r, shape[3])
        a, b = R.truncated_svd_factors(wm, r)
        prod = R.filters_as_matrix(w1) @ w2
        assert np.abs(prod - a @ b).max() <= 1e-9 * np.abs(wm).max()
        err2 = np.linalg.norm(wm - prod) ** 2
        assert err2 == pytest.approx(float((s[r:] ** 2).sum()), rel=1e-8, abs=1e-20)
        assert np.allclose(w2 @ w2.T, np.eye(r), atol=1e-12)
    assert F.relative_error(w, *F.factorize(w, min(wm.shape))) < 1e-12
    assert np.allclose(F.singular_values(w)[: min(wm.shape)], s, rtol=1e-9)


def test_rank_out_of_range():
    w = synth.weights("unit", 78, (3, 3, 1, 4), 0.1)
    with pytest.raises(ValueError):
        F.factorize(w, 5)
    with pytest.raises(ValueError):
        F.factorize(w, 0)


def test_with_spectrum():
    sigma = 0.5 * 0.6 ** np.arange(27)
    rng = synth.rng("unit", "test", 31)
    w = F.with_spectrum(rng.normal(size=(27, 27)), rng.normal(size=(64, 27)), sigma, (3, 3, 3, 64))
    s = np.linalg.svd(R.filters_as_matrix(w), compute_uv=False)
    assert np.allclose(s, sigma, rtol=1e-10)
    # the rank-r relative error is the tail of the spectrum
    w1, w2 = F.factorize(w, 8)
    assert F.relative_error(w, w1, w2) == pytest.approx(np.sqrt((sigma[8:] ** 2).sum() / (sigma ** 2).sum()), rel=1e-8)
