"""FP64 spatial-domain twin of FOFSE, with the projections of eq. 5 recomputed
by explicit sums over the area in every iteration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It imports nothing from
the HIP path and nothing from the DFT-domain oracle.

This is the plain definition of the iteration (Section 2): residual r^(0) = f on
the support area A (0 on the missing area B), model g^(0) = 0; per iteration

* projection coefficient of every basis function (eq. 5)
      p_k = sum_L r w conj(phi_k) / sum_L w |phi_k|^2 ;
* selection by the distance criterion of eq. 6,
      u = argmax_k |p_k|^2 sum_L w |phi_k|^2 ,
  over the conjugate classes (same candidate set and tie rule as the DFT
  oracle: smallest key k*T + l);
* coefficient estimate
      - "constant": c_u = gamma p_u (eq. 14, FOFSE), or
      - "full": c_u = p_u / sum_l (p_l / p_u) Khat_{u,l} (eq. 10), with
        Khat = diag(diag K)^-1 K (eq. 11) and K the matrix of weighted scalar
        products of the basis functions (eq. 12), K_{u,l} = sum w phi_l conj(phi_u);
* model update g += delta and residual update r = (r - delta) on A, 0 on B
  (eqs. 2 and 3), with delta = c phi_u + conj(c) phi_{-u} for a pair and
  delta = c phi_u (c real) for a self-conjugate class.

Cost O(T^2 M N) per iteration (and O(T^4) for "full"), so it is run on tiny
areas only.  The "full" mode is the paper's OFSE compensation in the complex
reading taken here; no printed value exists to pin it (parity unpinned beyond
its agreement with the transform-domain identity in the tests).
"""

from __future__ import annotations

import numpy as np


def _basis(T: int, M: int, N: int) -> np.ndarray:
    """phi[k, l, m, n] = exp(+j 2 pi (k m + l n) / T) on the M x N area."""
    k = np.arange(T)[:, None, None, None]
    l = np.arange(T)[None, :, None, None]
    m = np.arange(M)[None, None, :, None]
    n = np.arange(N)[None, None, None, :]
    return np.exp(2j * np.pi * (k * m + l * n) / T)


def _is_rep(k: int, l: int, T: int) -> bool:
    h = T // 2
    if l > h:
        return False
    if l in (0, h):
        return k <= h
    return True


def _is_self_conj(k: int, l: int, T: int) -> bool:
    h = T // 2
    return k in (0, h) and l in (0, h)


def ofse_spatial(f, known, T: int, rho_hat: float, gamma: float, K: int,
                 weight=None, mode: str = "constant"):
    """Run K iterations on one M x N area by direct sums.

    Returns dict with g (M, N) float64, keys (K,), coef (K,) complex,
    energy (K+1,) = sum_A w r^2 before/after every iteration, and for
    mode="full" the compensation factors gamma_u (K,) complex of eq. 13.
    """
    f = np.asarray(f, dtype=np.float64)
    a = np.asarray(known).astype(np.float64)
    M, N = f.shape
    if weight is None:
        m = np.arange(M)[:, None]
        n = np.arange(N)[None, :]
        d = np.sqrt((m - (M - 1) / 2.0) ** 2 + (n - (N - 1) / 2.0) ** 2)
        w = a * float(rho_hat) ** d                        # eqs. 4 and 15
    else:
        w = a * np.asarray(weight, dtype=np.float64)
    phi = _basis(T, M, N)
    norm = np.einsum("mn,klmn->kl", w, np.abs(phi) ** 2)   # sum_L w |phi_k|^2
    r = f * a                                               # r^(0): f on A, 0 on B
    g = np.zeros((M, N))
    keys = np.zeros(K, np.int64)
    coef = np.zeros(K, np.complex128)
    gam = np.zeros(K, np.complex128)
    energy = np.zeros(K + 1)
    energy[0] = np.sum(w * r * r)
    if mode == "full":
        # eq. 12: K_{u,l} = sum_L w phi_l conj(phi_u), flattened over (k, l)
        flat = phi.reshape(T * T, M * N)
        Kmat = (flat.conj() * w.reshape(1, -1)) @ flat.T   # [u, l]
        Khat = Kmat / np.diag(Kmat)[:, None]               # eq. 11
    for nu in range(K):
        # eq. 5: weighted projection of the residual onto every basis function
        p = np.einsum("mn,klmn->kl", r * w, phi.conj()) / norm
        # eq. 6: distance criterion, over the class representatives
        crit = np.abs(p) ** 2 * norm
        best, bk, bl = -1.0, 0, 0
        for k in range(T):
            for l in range(T):
                if _is_rep(k, l, T) and crit[k, l] > best:
                    best, bk, bl = crit[k, l], k, l
        keys[nu] = bk * T + bl
        pu = p[bk, bl]
        if mode == "constant":
            c = gamma * pu                                  # eq. 14
        elif mode == "full":
            # eq. 10 / eq. 13: gamma_u = 1 / sum_l (p_l / p_u) Khat_{u,l}
            s = np.sum(p.reshape(-1) * Khat[bk * T + bl, :]) / pu
            gam[nu] = 1.0 / s
            c = pu * gam[nu]
        else:
            raise ValueError(mode)
        if _is_self_conj(bk, bl, T):
            c = complex(c.real)
            delta = (c * phi[bk, bl]).real
        else:
            delta = 2.0 * (c * phi[bk, bl]).real            # c phi_u + conj(c) phi_-u
        coef[nu] = c
        g = g + delta                                       # eq. 2
        r = (r - delta) * a                                 # eq. 3
        energy[nu + 1] = np.sum(w * r * r)
    out = {"g": g, "keys": keys, "coef": coef, "energy": energy}
    if mode == "full":
        out["gamma"] = gam
    return out
