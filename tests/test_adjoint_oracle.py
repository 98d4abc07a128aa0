"""Pins of the FP64 adjoint oracle (oracle/fofse_adjoint.py), CPU only.

The adjoint is checked against things it does not compute itself: central
finite differences of the fixed-selection forward (``replay``), the exact
linearity of f -> g with the selection fixed (dot-product test), and closed
forms for a constant signal and for one frequency pair under orthogonal
weighting."""

import numpy as np
import pytest

from oracle.fofse_adjoint import fofse_adjoint
from oracle.fofse_dft import fofse, isotropic_weight, replay, self_conjugate


def _case(seed, M=10, N=9, T=16, K=14, hole=True):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(M, N)) * 25 + 110
    f += 30 * np.cos(2 * np.pi * (0.13 * np.arange(M)[:, None] + 0.07 * np.arange(N)[None, :]))
    known = (rng.random((M, N)) > 0.25).astype(np.uint8)
    if hole:
        known[3:7, 3:6] = 0
    g_bar = rng.normal(size=(M, N))
    return rng, f, known, g_bar


def _loss(f, known, T, rho, gamma, keys, g_bar, weight=None):
    return float(np.sum(replay(f, known, T, rho, gamma, keys, weight=weight)[0] * g_bar))


@pytest.mark.parametrize("seed,T,gamma", [(0, 16, 0.5), (1, 16, 0.2), (2, 10, 0.9), (3, 16, 1.0)])
def test_adjoint_matches_central_differences(seed, T, gamma):
    rng, f, known, g_bar = _case(seed, T=T)
    rho = 0.8
    K = 14
    keys = fofse(f, known, T, rho, gamma, K).keys
    adj = fofse_adjoint(f, known, T, rho, gamma, keys, g_bar)
    h = 1e-4
    v = rng.normal(size=f.shape)
    fd_f = (_loss(f + h * v, known, T, rho, gamma, keys, g_bar)
            - _loss(f - h * v, known, T, rho, gamma, keys, g_bar)) / (2 * h)
    assert np.sum(adj.f_bar * v) == pytest.approx(fd_f, rel=1e-7, abs=1e-9)
    fd_rho = (_loss(f, known, T, rho + h, gamma, keys, g_bar)
              - _loss(f, known, T, rho - h, gamma, keys, g_bar)) / (2 * h)
    assert adj.rho_bar == pytest.approx(fd_rho, rel=1e-6, abs=1e-6)
    if gamma < 1.0:
        fd_g = (_loss(f, known, T, rho, gamma + h, keys, g_bar)
                - _loss(f, known, T, rho, gamma - h, keys, g_bar)) / (2 * h)
    else:   # one-sided second-order difference at the end of the range
        fd_g = (3 * _loss(f, known, T, rho, gamma, keys, g_bar)
                - 4 * _loss(f, known, T, rho, gamma - h, keys, g_bar)
                + _loss(f, known, T, rho, gamma - 2 * h, keys, g_bar)) / (2 * h)
    assert adj.gamma_bar == pytest.approx(fd_g, rel=1e-5, abs=1e-6)


def test_adjoint_covers_self_conjugate_steps():
    # DC and (-1)^m plus one cosine: about half the selections are self-conjugate
    rng = np.random.default_rng(7)
    M, N, T, K = 8, 8, 8, 16
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    f = 90 + 20 * (-1.0) ** m + 25 * np.cos(2 * np.pi * (0.2 * m + 0.3 * n)) + 3 * rng.normal(size=(M, N))
    known = np.ones((M, N), np.uint8)
    known[2:5, 3:6] = 0
    g_bar = rng.normal(size=(M, N))
    keys = fofse(f, known, T, 0.7, 0.6, K).keys
    n_self = sum(bool(self_conjugate(k // T, k % T, T)) for k in keys)
    assert 3 <= n_self < K
    adj = fofse_adjoint(f, known, T, 0.7, 0.6, keys, g_bar)
    h = 1e-4
    for name, dp in (("rho", (h, 0.0)), ("gamma", (0.0, h))):
        lp = _loss(f, known, T, 0.7 + dp[0], 0.6 + dp[1], keys, g_bar)
        lm = _loss(f, known, T, 0.7 - dp[0], 0.6 - dp[1], keys, g_bar)
        got = adj.rho_bar if name == "rho" else adj.gamma_bar
        assert got == pytest.approx((lp - lm) / (2 * h), rel=1e-6)
    # every sample's derivative, by differences of the linear map
    J = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            e = np.zeros((M, N))
            e[i, j] = 1.0
            J[i, j] = _loss(e, known, T, 0.7, 0.6, keys, g_bar)
    np.testing.assert_allclose(adj.f_bar, J, rtol=1e-9, atol=1e-12)


def test_adjoint_dot_product_identity():
    # with the selection fixed f -> g is linear: <J v, gbar> = <v, J^T gbar>
    rng, f, known, g_bar = _case(11, M=12, N=12, T=16)
    keys = fofse(f, known, 16, 0.85, 0.3, 20).keys
    adj = fofse_adjoint(f, known, 16, 0.85, 0.3, keys, g_bar)
    for _ in range(3):
        v = rng.normal(size=f.shape)
        Jv = replay(v, known, 16, 0.85, 0.3, keys)[0]
        assert np.sum(Jv * g_bar) == pytest.approx(np.sum(v * adj.f_bar), rel=1e-10)
    # f_bar vanishes off the support area
    assert np.all(adj.f_bar[known == 0] == 0.0)


def test_adjoint_constant_signal_closed_form():
    # f = c selects DC in every iteration: g = c (1 - (1-gamma)^K) independent
    # of w, so rho_bar = 0, gamma_bar = sum(gbar) c K (1-gamma)^(K-1) and
    # f_bar = sum(gbar) (1 - (1-gamma)^K) w / W0
    M, N, T, K, c, gamma, rho = 12, 12, 16, 9, 37.0, 0.35, 0.75
    known = np.ones((M, N), np.uint8)
    known[4:8, 4:8] = 0
    f = np.full((M, N), c)
    rng = np.random.default_rng(5)
    g_bar = np.zeros((M, N))
    g_bar[4:8, 4:8] = rng.normal(size=(4, 4))
    res = fofse(f, known, T, rho, gamma, K)
    assert np.all(res.keys == 0)
    adj = fofse_adjoint(f, known, T, rho, gamma, res.keys, g_bar)
    S = g_bar.sum()
    assert adj.gamma_bar == pytest.approx(S * c * K * (1 - gamma) ** (K - 1), rel=1e-10)
    assert abs(adj.rho_bar) < 1e-9 * abs(S * c)
    w = isotropic_weight(known, rho)
    np.testing.assert_allclose(adj.f_bar, S * (1 - (1 - gamma) ** K) * w / w.sum(),
                               rtol=1e-10, atol=1e-14)


def test_adjoint_orthogonal_pair_closed_form():
    # M = N = T, everything known, rho_hat = 1: W = T^2 delta, so a pure pair
    # A cos(2 pi <u, x>/T + theta) is selected K times and g = (1-(1-gamma)^K) f.
    # Then f_bar = (1-(1-gamma)^K) P_u gbar (P_u the projection on the pair)
    # and gamma_bar = K (1-gamma)^(K-1) <gbar, f>.
    T, K, gamma = 8, 6, 0.45
    u, v = 1, 2
    m = np.arange(T)[:, None]
    n = np.arange(T)[None, :]
    f = 25.0 * np.cos(2 * np.pi * (u * m + v * n) / T + 0.6)
    known = np.ones((T, T), np.uint8)
    res = fofse(f, known, T, 1.0, gamma, K)
    assert np.all(res.keys == u * T + v)
    g_bar = np.random.default_rng(9).normal(size=(T, T))
    adj = fofse_adjoint(f, known, T, 1.0, gamma, res.keys, g_bar)
    phi = np.exp(2j * np.pi * (u * m + v * n) / T)
    proj = 2.0 / T ** 2 * (np.sum(g_bar * np.conj(phi)) * phi).real
    np.testing.assert_allclose(adj.f_bar, (1 - (1 - gamma) ** K) * proj, atol=1e-12)
    assert adj.gamma_bar == pytest.approx(K * (1 - gamma) ** (K - 1) * np.sum(g_bar * f), rel=1e-10)


def test_adjoint_weight_input_matches_differences():
    # arbitrary rho (eq. 4 allows any weighting): w_bar against differences
    rng, f, known, g_bar = _case(21, M=7, N=8, T=8, hole=False)
    known[2:4, 3:5] = 0
    weight = rng.uniform(0.2, 1.0, size=f.shape)
    keys = fofse(f, known, 8, 0.0, 0.5, 9, weight=weight).keys
    adj = fofse_adjoint(f, known, 8, 0.0, 0.5, keys, g_bar, weight=weight)
    assert adj.rho_bar == 0.0
    h = 1e-5
    for (i, j) in [(0, 0), (1, 5), (6, 7), (2, 3)]:
        e = np.zeros_like(weight)
        e[i, j] = h
        d = (_loss(f, known, 8, 0.0, 0.5, keys, g_bar, weight=weight + e)
             - _loss(f, known, 8, 0.0, 0.5, keys, g_bar, weight=weight - e)) / (2 * h)
        assert adj.w_bar[i, j] == pytest.approx(d, rel=1e-5, abs=1e-7)
