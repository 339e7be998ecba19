"""Pins for the oracle's completion loop (Sec. 5, Example 3), CPU only."""
import numpy as np
import pytest

from oracle import tsvd_oracle as O
from paper_2504_04989_amd import inputs


def test_full_observation_returns_the_data():
    M = inputs.random_tensor((12, 10, 3), 61)
    T = np.ones_like(M)
    Om = inputs.omega(10, 4, 3, 61)
    assert np.array_equal(O.complete(M, T, Om, 2, 4, 1, 3), M)


@pytest.mark.parametrize("alg", [1, 2])
def test_observed_entries_equal_the_data(alg):
    M = inputs.random_tensor((14, 12, 4), 62)
    T = inputs.bernoulli_mask(M.shape, 0.6, 62)
    Om = inputs.omega(12, 3, 4, 62)
    C = O.complete(M, T, Om, 2, 3, 1, 4, alg=alg)
    assert np.array_equal(C[T == 1], M[T == 1])


def test_objective_non_increasing_with_exact_rank_step():
    # b (q + 1) = n1: every slice's basis spans everything, so L is the exact
    # truncated T-SVD (Eckart-Young per slice); both half-steps then minimise
    # ||X - C||_F exactly (over the rank-k set, then over the data-consistent
    # set), so the objective never rises.
    n1, n2, n3 = 12, 15, 4
    M = inputs.exact_lowrank_tensor(n1, n2, n3, 3, seed=63) + 0.05 * inputs.random_tensor((n1, n2, n3), 63)
    T = inputs.bernoulli_mask(M.shape, 0.5, 63)
    Om = inputs.omega(n2, 6, n3, 63)
    _, hist = O.complete(M, T, Om, 3, 6, 1, 15, history=True)
    assert all(h2 <= h1 * (1 + 1e-12) + 1e-12 for h1, h2 in zip(hist, hist[1:]))
    assert hist[-1] < hist[0]


def test_low_tubal_rank_recovery():
    n1, n2, n3, r = 20, 24, 3, 2
    M = inputs.exact_lowrank_tensor(n1, n2, n3, r, seed=64)
    T = inputs.bernoulli_mask(M.shape, 0.6, 64)
    Om = inputs.omega(n2, 4, n3, 64)
    C = O.complete(M, T, Om, r, 4, 1, 150)
    assert O.relative_error(M, C) < 1e-3 * O.relative_error(M, T * M)


def test_image_recipe_and_masks():
    X = inputs.image_tensor(64, 96, 3, 65)
    assert X.min() == 0.0 and X.max() == 255.0
    m = inputs.bernoulli_mask(X.shape, 0.3, 65)
    assert abs(m.mean() - 0.3) < 0.02 and np.array_equal(m[:, :, 0], m[:, :, 2])
    L = inputs.line_mask(X.shape, 8, 65)
    assert 0.85 < L.mean() < 0.98 and L[:, :, 0].min(axis=1).max() == 1.0
    assert L[:, :, 0].max(axis=1).min() == 1.0 and L[:, :, 0].max(axis=0).min() == 1.0   # no empty row / column


def test_circle_mask():
    m = inputs.circle_mask((128, 160, 3), 12, 66)
    assert 0.5 < m.mean() < 0.99 and np.array_equal(m[:, :, 0], m[:, :, 1])
    assert set(np.unique(m)) <= {0.0, 1.0}
