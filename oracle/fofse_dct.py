"""FP64 reference of FOFSE with the two-dimensional DCT as its set of basis
functions.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with the
HIP path and imports nothing from it.

The paper remarks (Section 2, after eq. 9) that besides the 2-D DFT the 2-D
DCT also lets the whole iteration run in the transform domain.  This module is
that variant, with every step of the DFT oracle kept and only the basis
changed:

* basis phi_{k,l}[m,n] = a_k a_l cos(pi k (2m+1) / (2T)) cos(pi l (2n+1) / (2T)),
  k, l in [0, T): the orthonormal DCT-II basis of a T x T grid, with
  a_0 = sqrt(1/T) and a_k = sqrt(2/T) otherwise; the M x N area occupies rows
  0..M-1 and columns 0..N-1 of the grid (for the DCT the placement matters);
* the decomposition operator of eq. 8 is the orthonormal 2-D DCT-II of its
  argument zero-padded to T x T, so R_w[k] = sum r w phi_k, the numerator of
  eq. 5;
* selection (eq. 9): the basis function with the largest |R_w| over all T*T of
  them; ties go to the smallest key k*T + l;
* projection coefficient p_u = R_w[u] / sum_A w phi_u^2 (eq. 5; unlike the DFT
  case the denominator depends on u);
* constant compensation c_u = gamma p_u (eq. 14); model g += c_u phi_u (eq. 2);
  residual r -= c_u phi_u on A (eq. 3);
* the residual update in the transform domain: the transform of w (r - c phi_u)
  is R_w - c T{w phi_u}, so the spatial residual is never formed.

Every basis function is real: there are no conjugate pairs and every
coefficient is real.  The model spectrum G holds the coefficients on the
orthonormal basis, and g is its inverse DCT restricted to the area.
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.fft

from oracle.fofse_dft import isotropic_weight


def dct_basis_1d(T: int, L: int) -> np.ndarray:
    """A[k, m] = a_k cos(pi k (2m+1) / (2T)) for k < T, m < L: one factor of
    the separable orthonormal DCT-II basis, evaluated on the first L samples."""
    k = np.arange(T, dtype=np.float64)[:, None]
    m = np.arange(L, dtype=np.float64)[None, :]
    a = np.where(k == 0, np.sqrt(1.0 / T), np.sqrt(2.0 / T))
    return a * np.cos(np.pi * k * (2.0 * m + 1.0) / (2.0 * T))


def basis_function(key: int, T: int, M: int, N: int) -> np.ndarray:
    """phi_{k,l} on the M x N area for key = k*T + l."""
    k, l = divmod(int(key), T)
    return np.outer(dct_basis_1d(T, M)[k], dct_basis_1d(T, N)[l])


@dataclasses.dataclass
class DctResult:
    """Output of :func:`fofse_dct`.

    g        (B, M, N) float64 model over the whole area.
    keys     (B, K) int64 key k*T + l of the basis function of each iteration.
    coef     (B, K) float64 coefficient c added for it.
    margin   (B, K) float64 (|R|_(1) - |R|_(2)) / |R|_(1) over distinct basis
             functions at selection time (0 when the largest magnitude is 0).
    top      (B, K) float64 |R|_(1), the largest magnitude at selection time.
    energy   (B, K + 1) float64 weighted residual energy sum_A w r^2 before the
             first and after every iteration, tracked by the exact drop per step.
    R        (B, T, T) float64 weighted residual spectrum after the last step.
    """
    g: np.ndarray
    keys: np.ndarray
    coef: np.ndarray
    margin: np.ndarray
    top: np.ndarray
    energy: np.ndarray
    R: np.ndarray


def _pad(x: np.ndarray, T: int) -> np.ndarray:
    B, M, N = x.shape
    out = np.zeros((B, T, T))
    out[:, :M, :N] = x
    return out


def _dct2(x: np.ndarray) -> np.ndarray:
    return scipy.fft.dctn(x, type=2, norm="ortho", axes=(1, 2))


def fofse_dct(f, known, T: int, rho_hat: float, gamma: float, K: int,
              weight: np.ndarray | None = None) -> DctResult:
    """Run K iterations of FOFSE with DCT basis functions on a batch of areas.

    f, known: (B, M, N) or (M, N).  Samples of f outside the support area are
    ignored.  ``weight`` overrides the isotropic model with an arbitrary rho
    (multiplied by ``known``)."""
    f = np.asarray(f, dtype=np.float64)
    known = np.asarray(known)
    single = f.ndim == 2
    if single:
        f = f[None]
        known = known[None]
        if weight is not None and np.ndim(weight) == 2:
            weight = np.asarray(weight)[None]
    B, M, N = f.shape
    if T < max(M, N):
        raise ValueError("T must be at least the area size")
    if K < 0:
        raise ValueError("K must be >= 0")
    if not (0.0 < gamma <= 1.0):
        raise ValueError("gamma must lie in (0, 1]")

    # eq. 4 / eq. 15: weighting function
    if weight is None:
        w = isotropic_weight(known, rho_hat)
    else:
        w = np.asarray(weight, dtype=np.float64) * known
    if np.any(w.sum(axis=(1, 2)) <= 0.0):
        raise ValueError("no known sample with positive weight")
    # eq. 7 / eq. 8: transform of the weighted signal (r^(0) = f on A)
    R = _dct2(_pad(w * f, T))
    A_m = dct_basis_1d(T, M)
    A_n = dct_basis_1d(T, N)
    bidx = np.arange(B)
    G = np.zeros((B, T, T))
    keys = np.zeros((B, K), np.int64)
    coef = np.zeros((B, K))
    margin = np.zeros((B, K))
    top = np.zeros((B, K))
    energy = np.zeros((B, K + 1))
    energy[:, 0] = np.sum(w * f * f, axis=(1, 2))

    for nu in range(K):
        # eq. 9: basis function with the largest |R_w| (first maximum = smallest key)
        score = np.abs(R).reshape(B, -1)
        best = np.argmax(score, axis=1)
        a1 = score[bidx, best]
        rest = score.copy()
        rest[bidx, best] = -1.0
        a2 = rest.max(axis=1)
        margin[:, nu] = np.where(a1 > 0.0, (a1 - a2) / np.where(a1 > 0.0, a1, 1.0), 0.0)
        top[:, nu] = a1
        keys[:, nu] = best
        u, v = np.divmod(best, T)
        Ru = R[bidx, u, v]
        # eq. 5: p = <r, phi_u>_w / <phi_u, phi_u>_w; eq. 14: c = gamma p
        phi = A_m[u][:, :, None] * A_n[v][:, None, :]            # (B, M, N)
        S = np.sum(w * phi * phi, axis=(1, 2))
        c = gamma * Ru / S
        coef[:, nu] = c
        # eq. 2: model spectrum
        G[bidx, u, v] += c
        # eq. 3 in the transform domain: T{w (r - c phi_u)} = R_w - c T{w phi_u}
        R = R - c[:, None, None] * _dct2(_pad(w * phi, T))
        # exact drop of sum_A w r^2: 2 c <r, phi>_w - c^2 <phi, phi>_w
        energy[:, nu + 1] = energy[:, nu] - (2.0 * c * Ru - c * c * S)

    # eq. 1: g = sum of c_k phi_k = inverse orthonormal DCT of the model spectrum
    g = scipy.fft.idctn(G, type=2, norm="ortho", axes=(1, 2))[:, :M, :N]
    res = DctResult(g, keys, coef, margin, top, energy, R)
    if single:
        res = DctResult(g[0], keys[0], coef[0], margin[0], top[0], energy[0], R[0])
    return res


def fofse_dct_spatial(f, known, T: int, rho_hat: float, gamma: float, K: int):
    """The same iteration computed in the spatial domain by direct sums (eqs. 2,
    3, 5, 9, 14): every iteration forms all T*T weighted inner products of the
    residual with explicit basis functions.  O(T^2 M N) per iteration: tiny
    areas only.  One area (f, known are (M, N)); returns (g, keys, coef)."""
    f = np.asarray(f, dtype=np.float64)
    M, N = f.shape
    a = (np.asarray(known) != 0).astype(np.float64)
    w = isotropic_weight(known, rho_hat)
    A_m = dct_basis_1d(T, M)
    A_n = dct_basis_1d(T, N)
    phis = A_m[:, None, :, None] * A_n[None, :, None, :]         # (T, T, M, N)
    r = a * f
    g = np.zeros((M, N))
    keys, coefs = [], []
    for _ in range(K):
        num = np.einsum("klmn,mn->kl", phis, r * w)              # eq. 8 by direct sums
        key = int(np.argmax(np.abs(num).reshape(-1)))            # eq. 9
        k, l = divmod(key, T)
        phi = phis[k, l]
        p = num[k, l] / np.sum(w * phi * phi)                    # eq. 5
        c = gamma * p                                            # eq. 14
        g = g + c * phi                                          # eq. 2
        r = (r - c * phi) * a                                    # eq. 3
        keys.append(key)
        coefs.append(c)
    return g, np.array(keys, np.int64), np.array(coefs)


def synthesize_dct(keys, coef, T: int, M: int, N: int) -> np.ndarray:
    """Direct synthesis of the model from a selection record:
    g = sum_nu c_nu phi_{u_nu} (eqs. 1, 2)."""
    A_m = dct_basis_1d(T, M)
    A_n = dct_basis_1d(T, N)
    g = np.zeros((M, N))
    for key, c in zip(np.asarray(keys).tolist(), np.asarray(coef).tolist()):
        k, l = divmod(int(key), T)
        g += c * np.outer(A_m[k], A_n[l])
    return g
