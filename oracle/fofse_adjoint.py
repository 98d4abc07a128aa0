"""FP64 reference of the adjoint (reverse-mode derivative) of FOFSE with the
selection sequence held fixed.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with the
HIP path and imports nothing from it.

The paper does not differentiate the extrapolation.  With the classes u_1..u_K
of every iteration fixed (the record of a forward run), the model g on the area
is a function of the known samples f, of rho_hat (through the weighting
function of eqs. 4 and 15) and of the compensation factor gamma (eq. 14).  The
forward steps it differentiates are those of ``fofse_dft.replay``:

    w      = a * rho_hat ** d                                  (eqs. 4, 15)
    R0     = DFT(w f),  W = DFT(w),  W0 = sum w                (eqs. 7, 8)
    s_nu   = R_{nu-1}[u_nu]
    c_nu   = gamma s_nu / W0      (Re of it for a self-conjugate class; eqs. 5, 14)
    R_nu   = R_{nu-1} - c_nu W[. - u_nu] - conj(c_nu) W[. + u_nu]  (eq. 3 in the
             DFT domain; the second term is absent for a self-conjugate class)
    g      = sum_nu mult_nu Re(c_nu phi_{u_nu})                 (eqs. 1, 2)

Convention: for a complex intermediate z, zbar = dL/dRe z + j dL/dIm z.  With
that convention z = a b gives abar = zbar conj(b), and z = conj(a) b gives
abar = conj(zbar) b.  The reverse sweep below applies these rules to the steps
above in reverse order, carrying the full T x T adjoint spectra Rbar and Wbar
(no sparsity is exploited here; this is the plain form).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .fofse_dft import _embed, area_distance, isotropic_weight, replay, self_conjugate


@dataclasses.dataclass
class AdjointResult:
    """Gradients of L for one area, given gbar = dL/dg over the area.

    f_bar      (M, N) dL/df (zero off the support area, where w = 0).
    w_bar      (M, N) dL/dw for the weighting function w as an input.
    rho_bar    dL/drho_hat through the isotropic model (0 when ``weight`` is given).
    gamma_bar  dL/dgamma.
    coef       (K,) complex coefficients of the forward replay (for reference).
    """
    f_bar: np.ndarray
    w_bar: np.ndarray
    rho_bar: float
    gamma_bar: float
    coef: np.ndarray


def _shift(X: np.ndarray, u: int, v: int) -> np.ndarray:
    """Y[k, l] = X[k - u, l - v] (indices mod T)."""
    return np.roll(X, (u, v), axis=(0, 1))


def fofse_adjoint(f, known, T: int, rho_hat: float, gamma: float, keys, g_bar,
                  weight: np.ndarray | None = None) -> AdjointResult:
    """Reverse sweep through a fixed-selection FOFSE run on one (M, N) area.

    ``keys`` are the canonical keys u*T + v of the K iterations (a forward
    record); ``g_bar`` is dL/dg on the whole area (put zeros where the loss
    does not look, e.g. off the missing area).  ``weight`` replaces the
    isotropic model by an arbitrary rho (then rho_bar is 0 and w_bar is the
    gradient with respect to that rho times the known mask)."""
    f = np.asarray(f, dtype=np.float64)
    g_bar = np.asarray(g_bar, dtype=np.float64)
    M, N = f.shape
    a = (np.asarray(known) != 0).astype(np.float64)
    if weight is None:
        w = isotropic_weight(a, rho_hat)
    else:
        w = np.asarray(weight, dtype=np.float64) * a
    W = np.fft.fft2(_embed(w[None], T))[0]
    W0 = W[0, 0].real
    # forward replay: the coefficients of every iteration (needed by the sweep)
    _, coef = replay(f, a, T, rho_hat, gamma, keys, weight=weight)

    # eqs. 1, 2 reversed: g = sum mult Re(c phi_u)  =>  cbar0 = mult * Gbar[u]
    # with Gbar[k] = sum_x gbar[x] exp(-j 2 pi <k, x> / T)
    Gbar = np.fft.fft2(_embed(g_bar[None], T))[0]

    Rbar = np.zeros((T, T), np.complex128)
    Wbar = np.zeros((T, T), np.complex128)
    W0bar = 0.0
    gamma_bar = 0.0
    for nu in range(len(coef) - 1, -1, -1):
        u, v = divmod(int(keys[nu]), T)
        c = complex(coef[nu])
        sc = bool(self_conjugate(u, v, T))
        # contribution of the synthesis: Gbar[u] + conj(Gbar[-u]) for a pair
        # (g holds c phi_u + conj(c) phi_-u); Gbar[u] for a self-conjugate class
        if sc:
            cbar = Gbar[u, v]
        else:
            cbar = Gbar[u, v] + np.conj(Gbar[-u % T, -v % T])
        # residual update R_nu = R_{nu-1} - c W[. - u] - conj(c) W[. + u]
        Wm = _shift(W, u, v)              # W[k - u]
        cbar -= np.sum(np.conj(Wm) * Rbar)
        Wbar -= np.conj(c) * _shift(Rbar, -u, -v)     # Wbar[j] -= conj(c) Rbar[j + u]
        if not sc:
            Wp = _shift(W, -u, -v)        # W[k + u]
            cbar -= np.conj(np.sum(np.conj(Wp) * Rbar))
            Wbar -= c * _shift(Rbar, u, v)            # Wbar[j] -= c Rbar[j - u]
        # coefficient c = gamma s / W0 (real part for a self-conjugate class)
        if sc:
            cbar = complex(cbar.real)
        t = (cbar * np.conj(c)).real
        gamma_bar += t / gamma
        W0bar -= t / W0
        Rbar[u, v] += gamma * cbar / W0               # s = R_{nu-1}[u]

    # R0 = DFT(w f), W = DFT(w), W0 = sum w  =>  adjoints on the area
    wf_bar = (T * T * np.fft.ifft2(Rbar)).real[:M, :N]
    f_bar = w * wf_bar
    w_bar = f * wf_bar + (T * T * np.fft.ifft2(Wbar)).real[:M, :N] + W0bar
    w_bar = w_bar * a                  # w is a * rho: only samples of A carry it
    if weight is None:
        d = area_distance(M, N)
        dw = np.where(a > 0, d * float(rho_hat) ** (d - 1.0), 0.0)
        rho_bar = float(np.sum(w_bar * dw))
    else:
        rho_bar = 0.0
    return AdjointResult(f_bar, w_bar, rho_bar, float(gamma_bar), coef)
