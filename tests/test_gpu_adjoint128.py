"""Parity of the adjoint at FFT size 128 (fofse_backward on a 128-point plan:
the Hermitian half planes of W and then D held in LDS, one workgroup per
block) with the FP64 adjoint oracle and with central differences of the
oracle's fixed-selection forward.

The selection record handed to the GPU is the oracle's own, so both sides
differentiate the same function.  Bars as for the smaller sizes: dL/df within
1e-6 of the block's largest |dL/df|, dL/drho_hat and dL/dgamma within 1e-6
relative; finite differences within 1e-5 relative.
"""

import numpy as np
import pytest

from oracle.fofse_dft import fofse, replay
from paper_2207_01205_amd import synth
from test_gpu_adjoint import _plan, _support, check, gpu_backward, oracle_adjoints

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def class128():
    """Blocks of the mixed workload's 32 x 32 class: 64 x 64 areas, B in the
    middle, frame content."""
    areas, target, _, _ = synth.mixed_blocks(synth.frame(100), 7, 32, 16, 6)
    return areas, target


def _ragged(n, M, N, seed):
    """Areas of M x N (128-point plans hold areas up to 64 x 64) with an
    off-centre rectangular B and irregular known masks."""
    rng = np.random.default_rng(seed)
    target = np.zeros((M, N), np.uint8)
    target[M // 3:M // 3 + M // 3, N // 4:N // 4 + N // 3] = 1
    m = np.arange(M)[:, None]
    nn = np.arange(N)[None, :]
    areas = (120 + 40 * np.cos(2 * np.pi * (0.031 * m + 0.017 * nn))[None]
             + 25 * np.sin(2 * np.pi * 0.09 * nn)[None] + 10 * rng.normal(size=(n, M, N))).astype(np.float32)
    known = (rng.random((n, M, N)) > 0.12).astype(np.uint8)
    return areas, known, target


def test_backward128_mixed_class(class128):
    areas, target = class128
    K = 300
    f, kn = _support(areas, None, target)
    ref = fofse(f, kn, 128, 0.8, 0.5, K)
    gbar_b = np.random.default_rng(5).normal(size=(f.shape[0], int(target.sum()))).astype(np.float32)
    plan = _plan(64, 64, 128, K, target)
    ga, grg, gb = gpu_backward(plan, areas, None, 0.8, 0.5, ref.keys, ref.coef, gbar_b, "T=128 mixed class")
    fb, rb, gmb = oracle_adjoints(f, kn, target, 128, 0.8, 0.5, ref.keys, gbar_b)
    check("T=128 mixed class", ga, gb, grg, fb, rb, gmb)
    assert np.all(ga.reshape(ga.shape[0], -1)[:, target.reshape(-1) == 1] == 0.0)


@pytest.mark.parametrize("M,N,K", [(64, 60, 150), (64, 64, 64), (37, 53, 200)])
def test_backward128_ragged_areas(M, N, K):
    """The largest area, a ragged one and odd sizes; per-block known masks;
    panels of the recurrence with a ragged last one."""
    areas, known, target = _ragged(3, M, N, seed=M + N + K)
    f, kn = _support(areas, known, target)
    ref = fofse(f, kn, 128, 0.85, 0.4, K)
    gbar_b = np.random.default_rng(K).normal(size=(3, int(target.sum()))).astype(np.float32)
    plan = _plan(M, N, 128, K, target)
    label = f"T=128 {M}x{N} K={K}"
    ga, grg, gb = gpu_backward(plan, areas, known, 0.85, 0.4, ref.keys, ref.coef, gbar_b, label)
    fb, rb, gmb = oracle_adjoints(f, kn, target, 128, 0.85, 0.4, ref.keys, gbar_b)
    check(label, ga, gb, grg, fb, rb, gmb)
    assert np.all(ga[kn == 0] == 0.0)


def test_backward128_largest_record(class128):
    """K = 512, the largest record the kernel holds; K = 513 is refused."""
    areas, target = class128
    areas = areas[:2]
    K = 512
    f, kn = _support(areas, None, target)
    ref = fofse(f, kn, 128, 0.9, 0.6, K)
    gbar_b = np.random.default_rng(9).normal(size=(2, int(target.sum()))).astype(np.float32)
    plan = _plan(64, 64, 128, K, target)
    ga, grg, gb = gpu_backward(plan, areas, None, 0.9, 0.6, ref.keys, ref.coef, gbar_b, "T=128 K=512")
    fb, rb, gmb = oracle_adjoints(f, kn, target, 128, 0.9, 0.6, ref.keys, gbar_b)
    check("T=128 K=512", ga, gb, grg, fb, rb, gmb)
    from paper_2207_01205_amd import fofse as F
    big = _plan(64, 64, 128, 513, target)
    dev = torch.device("cuda", 0)
    a = torch.from_numpy(np.ascontiguousarray(areas)).to(dev)
    rg = torch.tensor([0.9, 0.6], dtype=torch.float64, device=dev)
    sel = torch.zeros((2, 513), dtype=torch.int32, device=dev)
    cf = torch.zeros((2, 513, 2), dtype=torch.float64, device=dev)
    go = torch.zeros((2, int(target.sum())), dtype=torch.float32, device=dev)
    with pytest.raises(F.FofseError):
        big.backward(a, rg, sel, cf, go)


def test_backward128_finite_differences(class128):
    """Central differences (h = 1e-4) of the FP64 fixed-selection forward."""
    areas, target = class128
    idx = [1, 4]
    rho, gamma, K = 0.8, 0.5, 120
    f, kn = _support(areas[idx], None, target)
    ref = fofse(f, kn, 128, rho, gamma, K)
    rng = np.random.default_rng(21)
    gbar_b = rng.normal(size=(len(idx), int(target.sum()))).astype(np.float32)
    plan = _plan(64, 64, 128, K, target)
    ga, _, gb = gpu_backward(plan, areas[idx], None, rho, gamma, ref.keys, ref.coef, gbar_b,
                             "T=128 finite differences")
    tb = target.astype(bool)
    h = 1e-4
    for i in range(len(idx)):
        gbar = np.zeros(f.shape[1:])
        gbar[tb] = gbar_b[i]

        def L(ff, r, g):
            return float(np.sum(replay(ff, kn[i], 128, r, g, ref.keys[i])[0] * gbar))

        v = rng.normal(size=f.shape[1:]) * kn[i]
        fd_f = (L(f[i] + h * v, rho, gamma) - L(f[i] - h * v, rho, gamma)) / (2 * h)
        fd_r = (L(f[i], rho + h, gamma) - L(f[i], rho - h, gamma)) / (2 * h)
        fd_g = (L(f[i], rho, gamma + h) - L(f[i], rho, gamma - h)) / (2 * h)
        print(f"[gpu] T=128 block {idx[i]}: df {np.sum(ga[i] * v):.9e} vs {fd_f:.9e}; "
              f"drho {gb[i, 0]:.9e} vs {fd_r:.9e}; dgamma {gb[i, 1]:.9e} vs {fd_g:.9e}", flush=True)
        assert np.sum(ga[i] * v) == pytest.approx(fd_f, rel=1e-5)
        assert gb[i, 0] == pytest.approx(fd_r, rel=1e-5)
        assert gb[i, 1] == pytest.approx(fd_g, rel=1e-5)


def test_backward128_edge_cases():
    """Non-finite known sample and a block without support: zero gradients;
    parameters out of range: zero everywhere; repeated calls and a block's
    neighbours in the batch do not change its bits."""
    areas, known, target = _ragged(6, 60, 60, seed=3)
    K = 80
    f, kn = _support(areas, known, target)
    ref = fofse(f, kn, 128, 0.8, 0.5, K)
    keys, coef = ref.keys.copy(), ref.coef.copy()
    areas = areas.copy()
    known = known.copy()
    areas[2, 0, 0] = np.nan
    known[2, 0, 0] = 1
    known[4] = 0
    gbar_b = np.random.default_rng(2).normal(size=(6, int(target.sum()))).astype(np.float32)
    plan = _plan(60, 60, 128, K, target)
    ga, grg, gb = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "T=128 edge cases")
    assert np.all(ga[2] == 0) and np.all(gb[2] == 0)
    assert np.all(ga[4] == 0) and np.all(gb[4] == 0)
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gb))
    ok = [0, 1, 3, 5]
    fb, rb, gmb = oracle_adjoints(f[ok], kn[ok], target, 128, 0.8, 0.5, keys[ok], gbar_b[ok])
    check("T=128 edge cases (regular blocks)", ga[ok], gb[ok], np.array([rb.sum(), gmb.sum()]), fb, rb, gmb)
    np.testing.assert_allclose(grg, [gb[:, 0].sum(), gb[:, 1].sum()], rtol=1e-12)
    _, grg2, gb2 = gpu_backward(plan, areas, known, 0.8, 1.5, keys, coef, gbar_b, "T=128 gamma 1.5")
    assert np.all(gb2 == 0) and np.all(grg2 == 0)
    ga3, _, gb3 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "T=128 repeat")
    assert np.array_equal(ga3, ga) and np.array_equal(gb3, gb)
    sub = [5, 0]
    ga4, _, gb4 = gpu_backward(plan, areas[sub], known[sub], 0.8, 0.5, keys[sub], coef[sub], gbar_b[sub],
                               "T=128 sub-batch")
    assert np.array_equal(ga4, ga[sub]) and np.array_equal(gb4, gb[sub])


def test_backward128_keys_on_both_half_planes(class128):
    """Records that name a class by either of its two keys (u or -u), repeat
    classes, and hit the columns l = 0 and l = 64 whose bins the half plane
    holds twice, and the four self-conjugate classes; the coefficients are the
    oracle's fixed-selection replay of those keys."""
    areas, target = class128
    areas = areas[:3]
    T, K = 128, 160
    f, kn = _support(areas, None, target)
    ref = fofse(f, kn, T, 0.8, 0.5, K)
    rng = np.random.default_rng(31)
    keys = ref.keys.copy()
    for i in range(keys.shape[0]):
        u, v = keys[i] // T, keys[i] % T
        flip = rng.random(K) < 0.5                       # the other key of the same class
        keys[i] = np.where(flip, ((-u) % T) * T + ((-v) % T), keys[i])
        special = [0 * T + 0, 64 * T + 0, 0 * T + 64, 64 * T + 64,      # self-conjugate
                   5 * T + 0, 123 * T + 0, 7 * T + 64, 121 * T + 64]     # l = 0, 64 and their negatives
        pos = rng.choice(K, size=len(special) + 6, replace=False)
        keys[i, pos[:len(special)]] = special
        keys[i, pos[len(special):]] = keys[i, rng.choice(K, size=6)]   # repeats
    coef = np.stack([replay(f[i], kn[i], T, 0.8, 0.5, keys[i])[1] for i in range(keys.shape[0])])
    gbar_b = rng.normal(size=(keys.shape[0], int(target.sum()))).astype(np.float32)
    plan = _plan(64, 64, T, K, target)
    ga, grg, gb = gpu_backward(plan, areas, None, 0.8, 0.5, keys, coef, gbar_b, "T=128 keys on both half planes")
    fb, rb, gmb = oracle_adjoints(f, kn, target, T, 0.8, 0.5, keys, gbar_b)
    check("T=128 keys on both half planes", ga, gb, grg, fb, rb, gmb)
