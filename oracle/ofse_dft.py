"""FP64 reference of OFSE, the full orthogonality deficiency compensation
(eqs. 10-13), carried out in the DFT domain.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with the
HIP path and imports nothing from it.

Eq. 10 sets c_u = p_u / sum_l (p_l / p_u) Khat_{u,l}, with Khat = diag(diag K)^-1 K
(eq. 11) and K the matrix of weighted scalar products of the basis functions
(eq. 12).  With the complex DFT basis and the conjugate inner product taken
throughout (the same reading as for eq. 5):

    K_{u,l} = sum_x w[x] phi_l[x] conj(phi_u[x]) = W[u - l],   K_{u,u} = W0,

so sum_l p_l Khat_{u,l} = (p (*) W)[u] / W0, the cyclic convolution of the
projection spectrum p = R_w / W0 with W.  The compensation factor of eq. 13 is

    gamma_u = p_u W0 / (p (*) W)[u],

and no |L| x |L| matrix is formed.  Selection (eq. 6 = eq. 9), the conjugate
pair, the real coefficient of a self-conjugate class and the residual update
are those of the FOFSE oracle; only the coefficient differs (c = gamma_u p_u
instead of gamma p_u).  gamma_u is complex in this reading; the paper's Fig. 2
shows real factors, so histograms report Re gamma_u (parity unpinned against
the paper: its images are not available).
"""

from __future__ import annotations

import numpy as np

from .fofse_dft import _embed, canonical_mask, isotropic_weight, self_conjugate


def ofse_full(f, known, T: int, rho_hat: float, K: int, weight=None):
    """K OFSE iterations on one (M, N) area in the DFT domain.

    Returns dict with g (M, N), keys (K,), coef (K,) complex, gamma (K,)
    complex (eq. 13 factor of the selected class in every iteration; NaN when
    the residual is exactly zero and eq. 10 is 0 / 0, the iteration then adds
    nothing), and margin (K,) / top (K,): the selection margin
    (|R|_(1) - |R|_(2)) / |R|_(1) over distinct classes and |R|_(1), as in the
    FOFSE oracle."""
    f = np.asarray(f, dtype=np.float64)
    M, N = f.shape
    a = (np.asarray(known) != 0).astype(np.float64)
    w = isotropic_weight(a, rho_hat) if weight is None else np.asarray(weight, np.float64) * a
    R = np.fft.fft2(_embed((w * f)[None], T))[0]          # eqs. 7, 8
    W = np.fft.fft2(_embed(w[None], T))[0]
    W0 = W[0, 0].real
    if W0 <= 0.0:
        raise ValueError("no known sample with positive weight (W0 <= 0)")
    FW = np.fft.fft2(W)
    canon = canonical_mask(T).reshape(-1)
    G = np.zeros((T, T), np.complex128)
    keys = np.zeros(K, np.int64)
    coef = np.zeros(K, np.complex128)
    gam = np.zeros(K, np.complex128)
    margin = np.zeros(K)
    top = np.zeros(K)
    for nu in range(K):
        score = np.where(canon, (R.real ** 2 + R.imag ** 2).reshape(-1), -1.0)
        best = int(np.argmax(score))                        # eq. 9, smallest key on ties
        a1 = np.sqrt(score[best])
        a2 = np.sqrt(max(np.delete(score, best).max(), 0.0))
        margin[nu] = (a1 - a2) / a1 if a1 > 0.0 else 0.0
        top[nu] = a1
        u, v = divmod(best, T)
        keys[nu] = best
        p = R / W0                                          # eq. 5 for every bin
        conv = np.fft.ifft2(np.fft.fft2(p) * FW)            # (p (*) W)[k] = sum_l p_l W[k - l]
        if p[u, v] == 0 or conv[u, v] == 0:
            # residual exactly zero (eq. 10 reads 0 / 0): no update, factor undefined
            gu, c = complex(np.nan, np.nan), 0j
        else:
            gu = p[u, v] * W0 / conv[u, v]                  # eq. 13
            c = gu * p[u, v]                                # eq. 10
        gam[nu] = gu
        sc = bool(self_conjugate(u, v, T))
        if sc:
            c = complex(c.real)
        coef[nu] = c
        G[u, v] += c
        R = R - c * np.roll(W, (u, v), axis=(0, 1))         # eq. 3 in the DFT domain
        if not sc:
            G[-u % T, -v % T] += np.conj(c)
            R = R - np.conj(c) * np.roll(W, (-u, -v), axis=(0, 1))
    g = (T * T * np.fft.ifft2(G)).real[:M, :N]              # eqs. 1, 2
    return {"g": g, "keys": keys, "coef": coef, "gamma": gam, "margin": margin, "top": top}
