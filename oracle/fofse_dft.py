"""FP64 reference of FOFSE run entirely in the DFT domain.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with the
HIP path and imports nothing from it.

What it computes (Seiler & Kaup, "Fast orthogonality deficiency compensation
for improved frequency selective image extrapolation"):

* weighting function w = rho on the support area A, 0 elsewhere (eq. 4), with
  the isotropic model rho[m,n] = rho_hat ** dist((m,n), area centre) (eq. 15);
* weighted residual r_w = r * w (eq. 7) and its transform R_w = T{r_w} (eq. 8)
  with the 2-D DFT of size T x T as the operator T (Section 3 and Results);
* selection of the basis function with the largest |R_w| (eq. 9);
* projection coefficient p_u = <r, phi_u>_w / <phi_u, phi_u>_w (eq. 5);
* constant compensation c_u = gamma * p_u (eq. 14);
* model update g += c_u phi_u (eq. 2) and residual update r -= c_u phi_u on A
  (eq. 3), both carried out on spectra (the paper notes that for DFT bases the
  whole iteration can stay in the transform domain, Section 2).

Readings of the paper taken here (each is listed with its reason in the design
notes of the repository):

* Basis phi_{k,l}[m,n] = exp(+j 2 pi (k m + l n) / T).  Inner products are
  conjugate-linear, so eq. 5 becomes p_k = sum r w conj(phi_k) / sum w |phi_k|^2
  = R_w[k] / W0, with W = DFT(w) and W0 = W[0,0] = sum w.
* A real model needs conjugate pairs: one iteration adds c phi_u + conj(c)
  phi_{-u}; a self-conjugate frequency (both indices in {0, T/2}) is added once
  with a real coefficient.
* Candidates are the T*T/2 + 2 conjugate classes; each class is represented by
  (k, l) with l in [0, T/2] and, when l is 0 or T/2, k in [0, T/2].  Ties go to
  the smallest key k*T + l.
* The forward DFT is unnormalised with exp(-j ...).  The area sits at the
  origin of the T x T grid (the result does not depend on the placement).
* Exactly K iterations are run; iteration nu selects on the spectrum left by
  iteration nu - 1.

Shifting the DFT of w by the selected frequency is what replaces the spatial
residual update: DFT(w * phi_u)[k] = W[k - u], so after adding the pair,
R_w[k] <- R_w[k] - c W[k - u] - conj(c) W[k + u]   (indices mod T).
"""

from __future__ import annotations

import dataclasses

import numpy as np


def area_distance(M: int, N: int) -> np.ndarray:
    """Distance of every sample of an M x N area from its centre
    ((M-1)/2, (N-1)/2), the exponent of the isotropic model (eq. 15)."""
    m = np.arange(M, dtype=np.float64)[:, None]
    n = np.arange(N, dtype=np.float64)[None, :]
    return np.sqrt((m - (M - 1) / 2.0) ** 2 + (n - (N - 1) / 2.0) ** 2)


def isotropic_weight(known: np.ndarray, rho_hat: float) -> np.ndarray:
    """w = rho_hat ** dist on the support area, 0 elsewhere (eqs. 4 and 15).

    ``known`` is (..., M, N) with 1 on A; the result has the same shape."""
    M, N = known.shape[-2:]
    return known.astype(np.float64) * float(rho_hat) ** area_distance(M, N)


def canonical_mask(T: int) -> np.ndarray:
    """Boolean T x T map of the representatives of the conjugate classes
    {(k, l), (-k, -l) mod T}: l in [0, T/2]; if l in {0, T/2} also k in [0, T/2]."""
    h = T // 2
    k = np.arange(T)[:, None]
    l = np.arange(T)[None, :]
    edge = (l == 0) | (l == h)
    return (l <= h) & (~edge | (k <= h))


def canonical_key(k, l, T: int):
    """Key k*T + l of the representative of the class of (k, l)."""
    k = np.asarray(k) % T
    l = np.asarray(l) % T
    h = T // 2
    flip = (l > h) | (((l == 0) | (l == h)) & (k > h))
    kc = np.where(flip, (-k) % T, k)
    lc = np.where(flip, (-l) % T, l)
    return kc * T + lc


def self_conjugate(k, l, T: int):
    """True where (k, l) equals (-k, -l) mod T, i.e. both indices in {0, T/2}."""
    h = T // 2
    k = np.asarray(k)
    l = np.asarray(l)
    return ((k == 0) | (k == h)) & ((l == 0) | (l == h))


@dataclasses.dataclass
class FofseResult:
    """Output of :func:`fofse`.

    g        (B, M, N) float64 model over the whole area (its values on the
             missing area are the extrapolation).
    keys     (B, K) int64 canonical key u*T + v selected in each iteration.
    coef     (B, K) complex128 coefficient c added for that class (real for a
             self-conjugate class).
    margin   (B, K) float64 (|R|_(1) - |R|_(2)) / |R|_(1) over distinct classes
             at selection time (0 when the largest magnitude is 0).
    energy   (B, K + 1) float64 weighted residual energy sum_A w r^2 before the
             first and after every iteration, tracked by the exact drop per step.
    W0       (B,) float64 sum of the weights.
    top      (B, K) float64 |R|_(1), the largest magnitude at selection time.
    """
    g: np.ndarray
    keys: np.ndarray
    coef: np.ndarray
    margin: np.ndarray
    energy: np.ndarray
    W0: np.ndarray
    top: np.ndarray = None


def _embed(x: np.ndarray, T: int) -> np.ndarray:
    """Place a (B, M, N) area at the origin of a (B, T, T) zero grid."""
    B, M, N = x.shape
    out = np.zeros((B, T, T), dtype=x.dtype)
    out[:, :M, :N] = x
    return out


def fofse(f, known, T: int, rho_hat: float, gamma: float, K: int,
          weight: np.ndarray | None = None, offset=(0, 0)) -> FofseResult:
    """Run K FOFSE iterations on a batch of areas (all of one size).

    f, known: (B, M, N) or (M, N).  Samples of f outside the support area are
    ignored (their weight is 0).  ``weight`` overrides the isotropic model with
    an arbitrary rho (eq. 4 allows any rho); it is multiplied by ``known``.
    ``offset`` places the area at (offset) inside the T x T grid instead of the
    origin (used to check that the placement does not matter).
    """
    f = np.asarray(f, dtype=np.float64)
    known = np.asarray(known)
    single = f.ndim == 2
    if single:
        f = f[None]
        known = known[None]
        if weight is not None and np.ndim(weight) == 2:
            weight = np.asarray(weight)[None]
    B, M, N = f.shape
    if T < max(M, N) or T % 2:
        raise ValueError("T must be even and at least the area size")
    if K < 0:
        raise ValueError("K must be >= 0")
    if not (0.0 < gamma <= 1.0):
        raise ValueError("gamma must lie in (0, 1]")

    # eq. 4 / eq. 15: weighting function
    if weight is None:
        w = isotropic_weight(known, rho_hat)
    else:
        w = np.asarray(weight, dtype=np.float64) * known
    # eq. 7 / eq. 8: transform the weighted signal (r^(0) = f on A, g^(0) = 0)
    grid_f = np.zeros((B, T, T))
    grid_w = np.zeros((B, T, T))
    oy, ox = offset
    grid_f[:, oy:oy + M, ox:ox + N] = w * f
    grid_w[:, oy:oy + M, ox:ox + N] = w
    R = np.fft.fft2(grid_f)
    W = np.fft.fft2(grid_w)
    W0 = W[:, 0, 0].real.copy()
    if np.any(W0 <= 0.0):
        raise ValueError("no known sample with positive weight (W0 <= 0)")

    canon = canonical_mask(T).reshape(-1)
    kk = np.arange(T)[None, :, None]
    ll = np.arange(T)[None, None, :]
    bidx = np.arange(B)
    bb = bidx[:, None, None]
    G = np.zeros((B, T, T), dtype=np.complex128)
    keys = np.zeros((B, K), np.int64)
    coef = np.zeros((B, K), np.complex128)
    margin = np.zeros((B, K))
    top = np.zeros((B, K))
    energy = np.zeros((B, K + 1))
    energy[:, 0] = np.sum(w * f * f, axis=(1, 2))

    for nu in range(K):
        # eq. 9: class with the largest |R_w| (squared magnitude, same order)
        score = (R.real ** 2 + R.imag ** 2).reshape(B, -1)
        score = np.where(canon[None, :], score, -1.0)
        best = np.argmax(score, axis=1)          # first maximum = smallest key
        s1 = score[bidx, best]
        rest = score.copy()
        rest[bidx, best] = -1.0
        s2 = rest.max(axis=1)
        a1 = np.sqrt(s1)
        a2 = np.sqrt(np.maximum(s2, 0.0))
        safe = np.where(a1 > 0.0, a1, 1.0)
        margin[:, nu] = np.where(a1 > 0.0, (a1 - a2) / safe, 0.0)
        top[:, nu] = a1
        u, v = np.divmod(best, T)
        keys[:, nu] = best
        Ru = R[bidx, u, v]
        # eq. 5 (p = R_w[u] / W0) and eq. 14 (c = gamma p); a self-conjugate
        # class has a real basis function and a real coefficient
        sc = self_conjugate(u, v, T)
        c = gamma * Ru / W0
        c = np.where(sc, c.real + 0j, c)
        coef[:, nu] = c
        # eq. 2: the model spectrum gets c at (u, v) and conj(c) at (-u, -v)
        pair = np.where(sc, 0.0, 1.0)
        G[bidx, u, v] += c
        G[bidx, (-u) % T, (-v) % T] += pair * np.conj(c)
        # eq. 3 carried to the DFT domain: R[k] -= c W[k - u] + conj(c) W[k + u]
        uu = u[:, None, None]
        vv = v[:, None, None]
        Wm = W[bb, (kk - uu) % T, (ll - vv) % T]
        Wp = W[bb, (kk + uu) % T, (ll + vv) % T]
        R = R - c[:, None, None] * Wm - (pair * np.conj(c))[:, None, None] * Wp
        # exact drop of the weighted residual energy sum_A w r^2 for this step
        W2u = W[bidx, (2 * u) % T, (2 * v) % T]
        d_pair = 2.0 * (2.0 * np.real(c * np.conj(Ru))
                        - np.abs(c) ** 2 * W0 - np.real(c * c * np.conj(W2u)))
        d_self = 2.0 * c.real * Ru.real - c.real ** 2 * W0
        energy[:, nu + 1] = energy[:, nu] - np.where(sc, d_self, d_pair)

    # eq. 1: g = sum over the model spectrum of c_k phi_k, phi with exp(+j)
    g = (T * T * np.fft.ifft2(G)).real[:, oy:oy + M, ox:ox + N]
    res = FofseResult(g, keys, coef, margin, energy, W0, top)
    if single:
        res = FofseResult(g[0], keys[0], coef[0], margin[0], energy[0], W0[0], top[0])
    return res


def synthesize(keys, coef, T: int, M: int, N: int) -> np.ndarray:
    """Direct synthesis of the model from a selection record (eq. 1 and 2):
    g[m, n] = sum_nu 2 Re(c_nu phi_{u_nu}[m, n]) for a pair and
    c_nu phi_{u_nu}[m, n] for a self-conjugate class."""
    keys = np.asarray(keys)
    coef = np.asarray(coef)
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    g = np.zeros((M, N))
    for key, c in zip(keys.tolist(), coef.tolist()):
        u, v = divmod(int(key), T)
        ph = np.exp(2j * np.pi * (u * m + v * n) / T)
        if self_conjugate(u, v, T):
            g += (c * ph).real
        else:
            g += 2.0 * (c * ph).real
    return g


def replay(f, known, T: int, rho_hat: float, gamma: float, keys,
           weight: np.ndarray | None = None):
    """Fixed-selection forward: the same steps as :func:`fofse` but the class of
    every iteration is taken from ``keys`` instead of the argmax.  Given the
    keys the map f -> g is linear, which the adjoint tests rely on.

    Returns (g, coef) for one area (f, known are (M, N))."""
    f = np.asarray(f, dtype=np.float64)
    M, N = f.shape
    w = isotropic_weight(known, rho_hat) if weight is None else np.asarray(weight) * known
    R = np.fft.fft2(_embed((w * f)[None], T))[0]
    W = np.fft.fft2(_embed(w[None], T))[0]
    W0 = W[0, 0].real
    G = np.zeros((T, T), np.complex128)
    coef = []
    for key in np.asarray(keys).tolist():
        u, v = divmod(int(key), T)
        c = gamma * R[u, v] / W0
        if self_conjugate(u, v, T):
            c = complex(c.real)
            G[u, v] += c
            R = R - c * np.roll(W, (u, v), axis=(0, 1))
        else:
            G[u, v] += c
            G[-u % T, -v % T] += np.conj(c)
            R = (R - c * np.roll(W, (u, v), axis=(0, 1))
                 - np.conj(c) * np.roll(W, (-u, -v), axis=(0, 1)))
        coef.append(c)
    g = (T * T * np.fft.ifft2(G)).real[:M, :N]
    return g, np.array(coef, np.complex128)


# Rounding floor of the parity rule, relative to the initial largest class
# magnitude A0 = |R^(0)|_max of the block.  Two computations of the same
# iteration in IEEE double precision differ in |R[u]| by their rounding noise
# (transform, and the accumulated updates); a selection can only swap two
# classes whose gap is below twice that difference.  Measured on the 1,024-block
# sample of the 1080p concealment workload (48 x 48 areas, T = 64, K = 200) and
# bounded again by every parity test (spectral_drift): at most 2.9e-14 A0.
FLOOR = 1e-13


def selection_parity(keys_gpu, keys_ref, margin_ref, tol: float = 1e-6,
                     top_ref=None, floor: float = FLOOR):
    """Acceptance rule for a selection sequence computed with other rounding
    (eq. 9: the class of largest |R_w| is selected).

    Iteration nu is "undecided" when the reference gap between the two largest
    class magnitudes, a1 - a2 = margin * a1, is at most tol * a1 (the relative
    rule) or, when ``top_ref`` (a1 per iteration) is given, at most
    floor * A0 with A0 = a1 of the first iteration: a gap at the level of the
    two computations' rounding noise.  nu* is the first undecided iteration;
    the sequences must agree before nu* (the whole sequence if there is none).
    Returns (ok, diverged): ok[b] is False on a mismatch before nu*;
    diverged[b] is True when they differ at or after it.
    """
    keys_gpu = np.atleast_2d(np.asarray(keys_gpu))
    keys_ref = np.atleast_2d(np.asarray(keys_ref))
    margin_ref = np.atleast_2d(np.asarray(margin_ref))
    B, K = keys_ref.shape
    nu_star = undecided_from(margin_ref, tol, top_ref, floor)
    mism = keys_gpu != keys_ref
    first = np.where(mism.any(axis=1), mism.argmax(axis=1), K)
    ok = first >= nu_star
    diverged = ok & (first < K)
    return ok, diverged


def undecided_from(margin_ref, tol: float = 1e-6, top_ref=None, floor: float = FLOOR):
    """nu* per block: the first iteration the rule of :func:`selection_parity`
    leaves undecided (K if none)."""
    margin_ref = np.atleast_2d(np.asarray(margin_ref))
    B, K = margin_ref.shape
    low = margin_ref <= tol
    if top_ref is not None and K > 0:
        top_ref = np.atleast_2d(np.asarray(top_ref))
        gap = margin_ref * top_ref
        low = low | (gap <= floor * top_ref[:, :1])
    return np.where(low.any(axis=1), low.argmax(axis=1), K)


def divergence_report(keys_gpu, keys_ref, margin_ref, top_ref, tol: float = 1e-6,
                      floor: float = FLOOR, limit: int = 50):
    """Where and why each diverging block leaves the reference sequence: its
    nu*, its first mismatching iteration, and the reference margin, gap / A0 and
    a1 / A0 there (at most ``limit`` blocks)."""
    keys_gpu = np.atleast_2d(np.asarray(keys_gpu))
    keys_ref = np.atleast_2d(np.asarray(keys_ref))
    margin_ref = np.atleast_2d(np.asarray(margin_ref))
    top_ref = np.atleast_2d(np.asarray(top_ref))
    K = keys_ref.shape[1]
    nu_star = undecided_from(margin_ref, tol, top_ref, floor)
    mism = keys_gpu != keys_ref
    first = np.where(mism.any(axis=1), mism.argmax(axis=1), K)
    rows = []
    for b in np.nonzero(first < K)[0][:limit]:
        f = int(first[b])
        a0 = float(top_ref[b, 0])
        rows.append({"block": int(b), "nu_star": int(nu_star[b]), "first_mismatch": f,
                     "oracle_margin": float(margin_ref[b, f]),
                     "gap_over_A0": float(margin_ref[b, f] * top_ref[b, f] / a0) if a0 > 0 else 0.0,
                     "top_over_A0": float(top_ref[b, f] / a0) if a0 > 0 else 0.0,
                     "within_rule": bool(f >= nu_star[b])})
    return rows


def spectral_drift(keys_gpu, coef_gpu, keys_ref, coef_ref, W0, top_ref, gamma: float):
    """Largest difference, relative to A0, between two computations of the
    selected R_w[u] over the iterations where their sequences still agree.
    With the constant compensation c = gamma R_w[u] / W0 (eqs. 5, 14), so
    |c_a - c_b| W0 / gamma is that difference.  coef_gpu is complex (B, K) or
    (B, K, 2) (re, im).  Returns the per-block maximum (0 for a block without a
    compared iteration or with A0 = 0)."""
    keys_gpu = np.atleast_2d(np.asarray(keys_gpu))
    keys_ref = np.atleast_2d(np.asarray(keys_ref))
    c = np.asarray(coef_gpu)
    if c.ndim >= 2 and c.shape[-1] == 2 and not np.iscomplexobj(c) and c.ndim == keys_ref.ndim + 1:
        c = c[..., 0] + 1j * c[..., 1]
    c = np.atleast_2d(c)
    cr = np.atleast_2d(np.asarray(coef_ref))
    top_ref = np.atleast_2d(np.asarray(top_ref))
    W0 = np.atleast_1d(np.asarray(W0, dtype=np.float64))
    B, K = keys_ref.shape
    mism = keys_gpu != keys_ref
    first = np.where(mism.any(axis=1), mism.argmax(axis=1), K)
    valid = np.arange(K)[None, :] < first[:, None]
    a0 = top_ref[:, :1] if K > 0 else np.ones((B, 1))
    d = np.abs(c - cr) * (W0[:, None] / gamma) / np.where(a0 > 0, a0, np.inf)
    return np.where(valid, d, 0.0).max(axis=1) if K > 0 else np.zeros(B)
