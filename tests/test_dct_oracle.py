"""Pins of the DCT-basis FOFSE oracle (the DCT variant the paper names in
Section 2, after eq. 9) against what the mathematics fixes: the same iteration
by direct spatial sums, the orthogonal special case (greedy best-K-term
approximation in the orthonormal DCT, computed with scipy's DCT), closed-form
coefficient decay, the exact weighted energy, the residual-spectrum invariant,
direct synthesis, scaling, the tie rule, and the product-to-sum identity that
lets the transform-domain update read four entries of the cosine transform of
w."""

import numpy as np
import pytest
import scipy.fft

from oracle.fofse_dct import (basis_function, dct_basis_1d, fofse_dct, fofse_dct_spatial,
                              synthesize_dct)
from oracle.fofse_dft import isotropic_weight


def _dctn(x):
    return scipy.fft.dctn(x, type=2, norm="ortho")


def _area(M, N, seed, hole=None):
    rng = np.random.default_rng(seed)
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    f = 100 + 40 * np.cos(2 * np.pi * (0.09 * m + 0.21 * n)) + 8 * rng.normal(size=(M, N))
    known = np.ones((M, N), np.uint8)
    if hole is not None:
        (a, b), (c, d) = hole
        known[a:b, c:d] = 0
    return f, known


@pytest.mark.parametrize("T,M,N,K,hole", [(8, 6, 7, 12, ((2, 4), (2, 5))),
                                          (16, 12, 12, 20, ((4, 8), (4, 8))),
                                          (16, 16, 11, 15, ((0, 3), (5, 9)))])
def test_transform_domain_matches_spatial_twin(T, M, N, K, hole):
    f, known = _area(M, N, T + M + N, hole)
    res = fofse_dct(f, known, T, 0.8, 0.5, K)
    g_s, keys_s, coef_s = fofse_dct_spatial(f, known, T, 0.8, 0.5, K)
    assert np.array_equal(res.keys, keys_s)
    np.testing.assert_allclose(res.coef, coef_s, rtol=1e-9, atol=1e-9 * np.abs(coef_s).max())
    np.testing.assert_allclose(res.g, g_s, rtol=0, atol=1e-9 * np.abs(g_s).max())


def test_orthogonal_weighting_is_best_k_term_dct_approximation():
    """M = N = T, every sample known, rho_hat = 1 (w = 1): the basis is
    orthonormal under the weighting, so with gamma = 1 every step removes one
    DCT coefficient and the model after K steps keeps the K largest."""
    T, K = 16, 30
    f = np.random.default_rng(4).normal(size=(T, T)) * 20
    res = fofse_dct(f, np.ones((T, T), np.uint8), T, 1.0, 1.0, K)
    X = _dctn(f)
    order = np.argsort(-np.abs(X).reshape(-1), kind="stable")[:K]
    assert np.array_equal(res.keys, order)
    np.testing.assert_allclose(res.coef, X.reshape(-1)[order], rtol=1e-12)
    kept = np.zeros(T * T)
    kept[order] = X.reshape(-1)[order]
    np.testing.assert_allclose(res.g, scipy.fft.idctn(kept.reshape(T, T), norm="ortho"),
                               atol=1e-11 * np.abs(f).max())
    rest = np.delete(X.reshape(-1), order)
    np.testing.assert_allclose(res.energy[-1], np.sum(rest ** 2), rtol=1e-10)


def test_orthogonal_weighting_coefficient_decay():
    """f = 5 phi_a + 2 phi_b with w = 1: phi_a is selected while
    5 (1 - gamma)^n > 2 and its coefficients are gamma 5 (1 - gamma)^n."""
    T, gamma = 8, 0.3
    a, b = 2 * T + 3, 5 * T + 1
    f = 5.0 * basis_function(a, T, T, T) + 2.0 * basis_function(b, T, T, T)
    res = fofse_dct(f, np.ones((T, T), np.uint8), T, 1.0, gamma, 4)
    assert list(res.keys) == [a, a, a, b]            # 5 * 0.7^2 = 2.45 > 2 > 5 * 0.7^3
    np.testing.assert_allclose(res.coef, [gamma * 5.0 * (1 - gamma) ** n for n in range(3)] + [gamma * 2.0],
                               rtol=1e-12)


def test_tie_goes_to_smallest_key():
    T = 8
    a, b = 6 * T + 2, 1 * T + 7            # equal |R|, b has the smaller key
    f = 3.0 * basis_function(a, T, T, T) - 3.0 * basis_function(b, T, T, T)
    res = fofse_dct(f, np.ones((T, T), np.uint8), T, 1.0, 1.0, 2)
    assert list(res.keys) == [b, a]


@pytest.mark.parametrize("gamma", [0.2, 0.5, 1.0])
def test_energy_is_exact_and_never_increases(gamma):
    T, M, N, K = 16, 12, 14, 25
    f, known = _area(M, N, 11, ((3, 9), (4, 10)))
    res = fofse_dct(f, known, T, 0.85, gamma, K)
    w = isotropic_weight(known, 0.85)
    direct = np.sum(w * (f - res.g) ** 2)
    np.testing.assert_allclose(res.energy[-1], direct, rtol=1e-9)
    assert np.all(np.diff(res.energy) <= 1e-9 * res.energy[0])


def test_residual_spectrum_invariant():
    """After K steps R_w = T{w (f - g)} on the support area."""
    T, M, N = 16, 13, 10
    f, known = _area(M, N, 3, ((5, 9), (2, 6)))
    res = fofse_dct(f, known, T, 0.75, 0.6, 18)
    w = isotropic_weight(known, 0.75)
    grid = np.zeros((T, T))
    grid[:M, :N] = w * (f - res.g)
    np.testing.assert_allclose(res.R, _dctn(grid), atol=1e-10 * np.abs(res.R).max())


def test_direct_synthesis_equals_inverse_transform():
    T, M, N = 16, 12, 12
    f, known = _area(M, N, 8, ((4, 8), (4, 8)))
    res = fofse_dct(f, known, T, 0.8, 0.5, 30)
    np.testing.assert_allclose(synthesize_dct(res.keys, res.coef, T, M, N), res.g,
                               atol=1e-11 * np.abs(res.g).max())


def test_scaling_keeps_the_selection():
    T, M, N = 16, 12, 12
    f, known = _area(M, N, 9, ((4, 8), (4, 8)))
    r1 = fofse_dct(f, known, T, 0.8, 0.5, 20)
    r3 = fofse_dct(3.0 * f, known, T, 0.8, 0.5, 20)
    assert np.array_equal(r1.keys, r3.keys)
    np.testing.assert_allclose(r3.g, 3.0 * r1.g, rtol=1e-10, atol=1e-10 * np.abs(r3.g).max())


def test_basis_is_orthonormal_on_the_grid():
    T = 16
    A = dct_basis_1d(T, T)
    np.testing.assert_allclose(A @ A.T, np.eye(T), atol=1e-13)


def test_product_to_sum_identity():
    """T{w phi_u}[k] = a_k1 a_k2 a_u1 a_u2 / 4 * sum over the four sign pairs of
    Wc[k1 +- u1, k2 +- u2], with Wc[a, b] = sum w cos(pi a (2m+1)/2T)
    cos(pi b (2n+1)/2T) extended by Wc[-a] = Wc[a] and Wc[2T - a] = -Wc[a] in
    each index (so Wc[T] = 0).  This is how a transform-domain update reads
    the Gram entries <w phi_u, phi_k> from one table."""
    T, M, N = 16, 12, 13
    rng = np.random.default_rng(2)
    w = rng.uniform(0.1, 1.0, size=(M, N)) * (rng.uniform(size=(M, N)) > 0.2)
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    a_idx = np.arange(2 * T)
    Cm = np.cos(np.pi * a_idx[:, None] * (2 * m.T + 1) / (2 * T))   # (2T, M)
    Cn = np.cos(np.pi * a_idx[:, None] * (2 * n + 1) / (2 * T))     # (2T, N)
    Wc = Cm @ w @ Cn.T                                              # (2T, 2T), indices 0..2T-1

    def ext(i):
        i = abs(i)
        return (i, 1.0) if i <= T else (2 * T - i, -1.0)

    alpha = np.where(np.arange(T) == 0, np.sqrt(1.0 / T), np.sqrt(2.0 / T))
    for (u1, u2) in [(0, 0), (3, 7), (15, 15), (8, 0), (11, 2)]:
        phi = np.outer(dct_basis_1d(T, M)[u1], dct_basis_1d(T, N)[u2])
        grid = np.zeros((T, T))
        grid[:M, :N] = w * phi
        ref = _dctn(grid)
        got = np.zeros((T, T))
        for k1 in range(T):
            for k2 in range(T):
                s = 0.0
                for r in (k1 - u1, k1 + u1):
                    for c in (k2 - u2, k2 + u2):
                        (ri, rs), (ci, cs) = ext(r), ext(c)
                        s += rs * cs * Wc[ri, ci]
                got[k1, k2] = alpha[k1] * alpha[k2] * alpha[u1] * alpha[u2] / 4.0 * s
        np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())
    # the extension is exact: Wc at 2T - a equals -Wc at a, and Wc at T is 0
    np.testing.assert_allclose(Wc[T], 0.0, atol=1e-12 * np.abs(Wc).max())
    np.testing.assert_allclose(Wc[2 * T - 5], -Wc[5], atol=1e-12 * np.abs(Wc).max())


def test_batch_equals_single_calls():
    T, M, N = 16, 12, 11
    f1, k1 = _area(M, N, 21, ((3, 7), (2, 6)))
    f2, k2 = _area(M, N, 22, ((5, 9), (4, 8)))
    both = fofse_dct(np.stack([f1, f2]), np.stack([k1, k2]), T, 0.8, 0.5, 15)
    for i, (f, k) in enumerate(((f1, k1), (f2, k2))):
        one = fofse_dct(f, k, T, 0.8, 0.5, 15)
        assert np.array_equal(both.keys[i], one.keys)
        np.testing.assert_allclose(both.g[i], one.g, rtol=0, atol=1e-12 * np.abs(one.g).max())
