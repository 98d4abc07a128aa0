"""Parity of the grouped adjoint (fofse_backward on FOFSE_PATH_GROUPED, T = 64,
K <= 256: blocks of one support mask share Z = W + j D, one wavefront per
block) with the FP64 adjoint oracle and with the per-block adjoint kernel.

Bars: against the oracle, the same as the per-block adjoint (dL/df within 1e-6
of the block's largest |dL/df|, dL/drho_hat and dL/dgamma within 1e-6
relative).  Against the per-block kernel on whole frames (both FP64, different
summation orders): dL/df within 1e-9 of the block's largest value, the
per-block parameter gradients within 1e-9 relative.
"""

import numpy as np
import pytest

from oracle.fofse_dft import fofse
from paper_2207_01205_amd import synth
from test_gpu_adjoint import _support, check, gpu_backward, oracle_adjoints

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _plan(M, N, T, K, target, path):
    from paper_2207_01205_amd.fofse import Plan
    p = Plan(M, N, T, K, target, device=0)
    p.set_path(path)
    return p


def _grouped(M, N, K, target):
    from paper_2207_01205_amd.fofse import FOFSE_PATH_GROUPED
    return _plan(M, N, 64, K, target, FOFSE_PATH_GROUPED)


def _split(M, N, K, target):
    from paper_2207_01205_amd.fofse import FOFSE_PATH_SPLIT
    return _plan(M, N, 64, K, target, FOFSE_PATH_SPLIT)


@pytest.fixture(scope="module")
def frame_areas():
    return synth.frame_concealment(0, 1)


def test_grouped_backward_frame_blocks(frame_areas):
    """24 frame blocks: mixed masks (classes of several blocks and singletons)."""
    A = frame_areas
    sub = slice(200, 224)
    f, kn = _support(A.areas[sub], A.known[sub], A.target)
    ref = fofse(f, kn, 64, 0.8, 0.5, 200)
    gbar_b = np.random.default_rng(3).normal(size=(f.shape[0], int(A.target.sum()))).astype(np.float32)
    plan = _grouped(48, 48, 200, A.target)
    ga, grg, gb = gpu_backward(plan, A.areas[sub], A.known[sub], 0.8, 0.5, ref.keys, ref.coef,
                               gbar_b, "grouped, frame blocks 200-223")
    fb, rb, gmb = oracle_adjoints(f, kn, A.target, 64, 0.8, 0.5, ref.keys, gbar_b)
    check("grouped frame blocks", ga, gb, grg, fb, rb, gmb)
    assert np.all(ga.reshape(ga.shape[0], -1)[:, A.target.reshape(-1) == 1] == 0.0)
    assert np.all(ga[kn == 0] == 0.0)


@pytest.mark.parametrize("K", [1, 63, 64, 65, 129, 256])
def test_grouped_backward_chunk_boundaries(K):
    """K around the 64-row chunks of a lane (1, ragged, exact, one over, the
    register capacity); areas without a known-mask array (every block shares
    the complement of B)."""
    f0, _, target = synth.single_block(5)
    rng = np.random.default_rng(K)
    n = 6
    areas = (f0[None] + 4.0 * rng.normal(size=(n,) + f0.shape)).astype(np.float32)
    f, kn = _support(areas, None, target)
    ref = fofse(f, kn, 64, 0.75, 0.6, K)
    gbar_b = rng.normal(size=(n, int(target.sum()))).astype(np.float32)
    plan = _grouped(32, 32, K, target)
    ga, grg, gb = gpu_backward(plan, areas, None, 0.75, 0.6, ref.keys, ref.coef, gbar_b, f"grouped K={K}")
    fb, rb, gmb = oracle_adjoints(f, kn, target, 64, 0.75, 0.6, ref.keys, gbar_b)
    check(f"grouped K={K}", ga, gb, grg, fb, rb, gmb)


def test_grouped_backward_tall_target_with_holes():
    """B's bounding box spans 22 rows (two passes of the separable Gbar) and
    has holes; 40 x 44 areas, per-block masks with a few lost samples."""
    rng = np.random.default_rng(21)
    M, N, K, n = 40, 44, 120, 10
    target = np.zeros((M, N), np.uint8)
    target[9:31, 15:27] = 1
    target[12, 18] = target[25, 20] = target[30, 15] = 0
    m = np.arange(M)[:, None]
    nn = np.arange(N)[None, :]
    areas = (90 + 50 * np.cos(2 * np.pi * (0.07 * m + 0.13 * nn))[None]
             + 6 * rng.normal(size=(n, M, N))).astype(np.float32)
    known = np.ones((n, M, N), np.uint8)
    known[3:6, rng.integers(0, M, 5), rng.integers(0, N, 5)] = 0   # three blocks share one mask
    known[8, :4, :] = 0
    f, kn = _support(areas, known, target)
    ref = fofse(f, kn, 64, 0.85, 0.45, K)
    gbar_b = rng.normal(size=(n, int(target.sum()))).astype(np.float32)
    plan = _grouped(M, N, K, target)
    ga, grg, gb = gpu_backward(plan, areas, known, 0.85, 0.45, ref.keys, ref.coef, gbar_b, "grouped tall B")
    fb, rb, gmb = oracle_adjoints(f, kn, target, 64, 0.85, 0.45, ref.keys, gbar_b)
    check("grouped tall B", ga, gb, grg, fb, rb, gmb)


def test_grouped_backward_matches_per_block_on_frames():
    """Two whole 1080p frames (about 1,600 blocks, the forward's own records):
    grouped and per-block adjoint agree to FP64 rounding-order differences."""
    A = synth.replicate_frames(2, 0, 1000)
    n = A.areas.shape[0]
    dev = torch.device("cuda", 0)
    a = torch.from_numpy(A.areas).to(dev)
    k = torch.from_numpy(A.known).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    pg = _grouped(48, 48, 200, A.target)
    ps = _split(48, 48, 200, A.target)
    print(f"[gpu] grouped vs per-block adjoint: {n} blocks", flush=True)
    _, sel, coef, st = pg.extrapolate(a, rg, known=k, record=True)
    go = torch.from_numpy(np.random.default_rng(9).normal(size=(n, pg.nB)).astype(np.float32)).to(dev)
    ga_g, grg_g, gb_g = pg.backward(a, rg, sel, coef, go, known=k, per_block=True)
    ga_s, grg_s, gb_s = ps.backward(a, rg, sel, coef, go, known=k, per_block=True)
    torch.cuda.synchronize()
    ga_g, ga_s = ga_g.cpu().numpy(), ga_s.cpu().numpy()
    gb_g, gb_s = gb_g.cpu().numpy(), gb_s.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    print(f"[gpu] per-block dL/drho: {int(np.sum(gb_s[:, 0] == 0))} zero, "
          f"{int(np.sum(~np.isfinite(gb_s)))} non-finite; grouped: {int(np.sum(gb_g[:, 0] == 0))} zero, "
          f"{int(np.sum(~np.isfinite(gb_g)))} non-finite", flush=True)
    assert np.all(np.isfinite(gb_s)) and np.all(np.isfinite(gb_g))
    scale = np.abs(ga_s).reshape(n, -1).max(axis=1)
    err = np.abs(ga_g - ga_s).reshape(n, -1).max(axis=1)
    assert np.all(err <= 1e-9 * scale + 1e-30), np.max(err / scale)
    np.testing.assert_allclose(gb_g, gb_s, rtol=1e-9, atol=1e-9 * np.abs(gb_s).max())
    np.testing.assert_allclose(grg_g.cpu().numpy(), grg_s.cpu().numpy(), rtol=1e-9)
    rel_r = np.abs(gb_g[:, 0] - gb_s[:, 0]) / np.maximum(np.abs(gb_s[:, 0]), 1e-300)
    print(f"[gpu] grouped vs per-block: max rel dL/df {np.max(err / scale):.2e}, "
          f"max rel dL/drho {np.max(rel_r):.2e}, float32 dL/df values that differ "
          f"{int(np.sum(ga_g != ga_s))}", flush=True)


def test_grouped_backward_edge_cases(frame_areas):
    A = frame_areas
    sub = slice(0, 12)
    areas = A.areas[sub].copy()
    known = A.known[sub].copy()
    f, kn = _support(areas, known, A.target)
    ref = fofse(f, kn, 64, 0.8, 0.5, 50)
    keys, coef = ref.keys.copy(), ref.coef.copy()
    areas[2, 0, 0] = np.nan            # non-finite known sample
    known[2, 0, 0] = 1
    known[5] = 0                       # no support at all
    areas[6, 20, 20] = np.inf          # on B: ignored
    gbar_b = np.random.default_rng(1).normal(size=(12, int(A.target.sum()))).astype(np.float32)
    plan = _grouped(48, 48, 50, A.target)
    ga, grg, gb = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "grouped edge cases")
    assert np.all(ga[2] == 0) and np.all(gb[2] == 0)
    assert np.all(ga[5] == 0) and np.all(gb[5] == 0)
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gb))
    ok = [0, 1, 3, 4, 6, 7, 8, 9, 10, 11]
    fb, rb, gmb = oracle_adjoints(f[ok], kn[ok], A.target, 64, 0.8, 0.5, keys[ok], gbar_b[ok])
    check("grouped edge cases (regular blocks)", ga[ok], gb[ok], np.array([rb.sum(), gmb.sum()]),
          fb, rb, gmb)
    np.testing.assert_allclose(grg, [gb[:, 0].sum(), gb[:, 1].sum()], rtol=1e-12)
    _, grg2, gb2 = gpu_backward(plan, areas, known, 0.8, 0.0, keys, coef, gbar_b, "grouped gamma 0")
    assert np.all(gb2 == 0) and np.all(grg2 == 0)
    # without dL/df, and twice in a row: the same bits (fixed-point scatter)
    _, grg3, gb3 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "grouped no dL/df",
                                grad_areas=False)
    ga4, grg4, gb4 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "grouped repeat")
    assert np.array_equal(gb3, gb) and np.array_equal(grg3, grg)
    assert np.array_equal(ga4, ga) and np.array_equal(gb4, gb)


@pytest.mark.parametrize("path", ["grouped", "split"])
def test_backward_ignores_imaginary_part_of_self_conjugate_coefficients(frame_areas, path):
    """The forward writes a real coefficient for a self-conjugate class; a record
    with a non-zero imaginary part there gives the same gradients, bit for bit."""
    A = frame_areas
    sub = slice(40, 52)
    f, kn = _support(A.areas[sub], A.known[sub], A.target)
    ref = fofse(f, kn, 64, 0.8, 0.5, 120)
    k, l = ref.keys // 64, ref.keys % 64
    sc = ((k % 32) == 0) & ((l % 32) == 0)
    assert sc.any()
    coef2 = ref.coef.copy()
    coef2[sc] += 7.0j
    gbar_b = np.random.default_rng(5).normal(size=(12, int(A.target.sum()))).astype(np.float32)
    plan = (_grouped if path == "grouped" else _split)(48, 48, 120, A.target)
    ga, grg, gb = gpu_backward(plan, A.areas[sub], A.known[sub], 0.8, 0.5, ref.keys, ref.coef, gbar_b,
                               f"{path} clean record")
    ga2, grg2, gb2 = gpu_backward(plan, A.areas[sub], A.known[sub], 0.8, 0.5, ref.keys, coef2, gbar_b,
                                  f"{path} imaginary parts on self-conjugate classes")
    assert np.array_equal(ga, ga2) and np.array_equal(gb, gb2) and np.array_equal(grg, grg2)


def test_grouped_backward_queue_many_items_per_workgroup():
    """The grouped adjoint over far more work items than resident workgroups
    (4 frames, one workgroup per CU, items from a queue): two runs and the same
    blocks in a small batch give the same bits."""
    frames = [synth.frame_concealment(30 + i, 40 + i) for i in range(4)]
    areas = np.concatenate([f.areas for f in frames])
    known = np.concatenate([f.known for f in frames])
    target = frames[0].target
    n, K = areas.shape[0], 80
    rng = np.random.default_rng(17)
    keys = rng.integers(0, 64 * 64, size=(n, K)).astype(np.int32)
    coef = rng.normal(size=(n, K)) + 1j * rng.normal(size=(n, K))
    gbar_b = rng.normal(size=(n, int(target.sum()))).astype(np.float32)
    plan = _grouped(48, 48, K, target)
    plan.set_occupancy(1)
    r1 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "queue run 1")
    r2 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "queue run 2")
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)
    lo = 1700
    part = gpu_backward(plan, areas[lo:lo + 150], known[lo:lo + 150], 0.8, 0.5, keys[lo:lo + 150],
                        coef[lo:lo + 150], gbar_b[lo:lo + 150], "queue, small batch")
    assert np.array_equal(r1[0][lo:lo + 150], part[0])
    assert np.array_equal(r1[2][lo:lo + 150], part[2])
