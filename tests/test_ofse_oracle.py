"""Pins of the full-compensation (OFSE, eqs. 10-13) oracle in the DFT domain,
CPU only: the explicit-matrix spatial twin, and the orthogonal case where the
compensation factor is exactly 1."""

import numpy as np
import pytest

from oracle.fofse_dft import fofse
from oracle.ofse_dft import ofse_full
from oracle.ofse_spatial import ofse_spatial


@pytest.mark.parametrize("seed,M,N,T", [(0, 6, 6, 8), (1, 7, 5, 8), (2, 8, 8, 8)])
def test_full_compensation_matches_explicit_matrix(seed, M, N, T):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 255, (M, N))
    known = (rng.random((M, N)) > 0.35).astype(np.uint8)
    known[0, 0] = 1
    K = 8
    ref = ofse_spatial(f, known, T, 0.8, 0.0, K, mode="full")
    got = ofse_full(f, known, T, 0.8, K)
    np.testing.assert_array_equal(got["keys"], ref["keys"])
    np.testing.assert_allclose(got["gamma"], ref["gamma"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(got["coef"], ref["coef"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(got["g"], ref["g"], atol=1e-8 * np.abs(ref["g"]).max())


def test_orthogonal_weighting_gives_unit_compensation():
    # M = N = T, all known, rho_hat = 1: W = T^2 delta, Khat = I, gamma_u = 1,
    # so OFSE equals FOFSE with gamma = 1 (plain frequency selective extrapolation)
    T, K = 8, 12
    rng = np.random.default_rng(4)
    f = rng.normal(size=(T, T)) * 30 + 100
    known = np.ones((T, T), np.uint8)
    got = ofse_full(f, known, T, 1.0, K)
    np.testing.assert_allclose(got["gamma"], np.ones(K), atol=1e-12)
    ref = fofse(f, known, T, 1.0, 1.0, K)
    np.testing.assert_array_equal(got["keys"], ref.keys)
    np.testing.assert_allclose(got["g"], ref.g, atol=1e-9)


def test_selection_margin_matches_fofse_before_the_first_update():
    """Both oracles select on the same spectrum in the first iteration, so the
    reported margin and largest magnitude agree there (and so does the key)."""
    from oracle.fofse_dft import fofse
    rng = np.random.default_rng(17)
    M, N, T = 12, 10, 16
    f = 100 + 30 * rng.normal(size=(M, N))
    known = np.ones((M, N), np.uint8)
    known[4:8, 3:7] = 0
    a = ofse_full(f, known, T, 0.8, 3)
    b = fofse(f, known, T, 0.8, 0.5, 3)
    assert a["keys"][0] == b.keys[0]
    np.testing.assert_allclose(a["margin"][0], b.margin[0], rtol=1e-12)
    np.testing.assert_allclose(a["top"][0], b.top[0], rtol=1e-12)
    assert np.all(a["margin"] >= 0) and np.all(a["top"] > 0)
