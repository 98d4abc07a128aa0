"""Parity of the adjoint kernel (fofse_backward, through the C ABI) with the FP64
adjoint oracle, and with central finite differences of the oracle's
fixed-selection forward.

The selection record handed to the GPU is the oracle's own forward record, so
both sides differentiate the same function.  Bar: dL/df within 1e-6 of the
largest |dL/df| of the block, dL/drho_hat and dL/dgamma within 1e-6 relative
(both sides compute in FP64; the margin covers rounding-order differences
through up to 300 coupled iterations and the float32 output of dL/df).
"""

import numpy as np
import pytest

from oracle.fofse_adjoint import fofse_adjoint
from oracle.fofse_dft import fofse, replay, selection_parity
from paper_2207_01205_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-6


def _plan(M, N, T, K, target):
    from paper_2207_01205_amd.fofse import Plan
    return Plan(M, N, T, K, target, device=0)


def _support(areas, known, target):
    f = np.asarray(areas, dtype=np.float32).astype(np.float64)
    kn = np.broadcast_to(1 - target, f.shape) if known is None else known
    return f, (kn * (1 - target)[None]).astype(np.uint8)


def gpu_backward(plan, areas, known, rho, gamma, keys, coef, gbar_b, label, grad_areas=True):
    print(f"[gpu] backward {label}: n={areas.shape[0]} M={plan.M} N={plan.N} T={plan.T} K={plan.K}",
          flush=True)
    dev = torch.device("cuda", 0)
    a = torch.from_numpy(np.ascontiguousarray(areas, dtype=np.float32)).to(dev)
    k = None if known is None else torch.from_numpy(np.ascontiguousarray(known, dtype=np.uint8)).to(dev)
    rg = torch.tensor([rho, gamma], dtype=torch.float64, device=dev)
    sel = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.int32)).to(dev)
    cf = torch.from_numpy(np.ascontiguousarray(np.stack([coef.real, coef.imag], -1))).to(dev)
    go = torch.from_numpy(np.ascontiguousarray(gbar_b, dtype=np.float32)).to(dev)
    ga, grg, gb = plan.backward(a, rg, sel, cf, go, known=k, grad_areas=grad_areas, per_block=True)
    torch.cuda.synchronize()
    return (None if ga is None else ga.cpu().numpy()), grg.cpu().numpy(), gb.cpu().numpy()


def oracle_adjoints(f, kn, target, T, rho, gamma, keys, gbar_b):
    n = f.shape[0]
    tb = target.astype(bool)
    fb = np.zeros(f.shape)
    rb = np.zeros(n)
    gmb = np.zeros(n)
    for i in range(n):
        gbar = np.zeros(f.shape[1:])
        gbar[tb] = np.asarray(gbar_b[i], dtype=np.float32)
        adj = fofse_adjoint(f[i], kn[i], T, rho, gamma, keys[i], gbar)
        fb[i], rb[i], gmb[i] = adj.f_bar, adj.rho_bar, adj.gamma_bar
    return fb, rb, gmb


def check(label, ga, gb, grg, fb, rb, gmb):
    n = fb.shape[0]
    scale_f = np.abs(fb).reshape(n, -1).max(axis=1)
    err_f = np.abs(ga - fb).reshape(n, -1).max(axis=1)
    assert np.all(err_f <= TOL * scale_f + 1e-12), f"{label}: dL/df rel err {np.max(err_f / scale_f)}"
    np.testing.assert_allclose(gb[:, 0], rb, rtol=TOL, atol=TOL * np.abs(rb).max() * 1e-3)
    np.testing.assert_allclose(gb[:, 1], gmb, rtol=TOL, atol=TOL * np.abs(gmb).max() * 1e-3)
    np.testing.assert_allclose(grg, [rb.sum(), gmb.sum()], rtol=TOL)
    print(f"[gpu] backward {label}: max rel dL/df {np.max(err_f / scale_f):.2e} "
          f"max rel rho {np.max(np.abs(gb[:, 0] - rb) / np.abs(rb)):.2e} "
          f"max rel gamma {np.max(np.abs(gb[:, 1] - gmb) / np.abs(gmb)):.2e}", flush=True)


@pytest.fixture(scope="module")
def frame_areas():
    return synth.frame_concealment(0, 1)


def test_backward_frame_blocks(frame_areas):
    A = frame_areas
    sub = slice(200, 224)
    f, kn = _support(A.areas[sub], A.known[sub], A.target)
    ref = fofse(f, kn, 64, 0.8, 0.5, 200)
    gbar_b = np.random.default_rng(3).normal(size=(f.shape[0], int(A.target.sum()))).astype(np.float32)
    plan = _plan(48, 48, 64, 200, A.target)
    ga, grg, gb = gpu_backward(plan, A.areas[sub], A.known[sub], 0.8, 0.5, ref.keys, ref.coef,
                               gbar_b, "frame blocks 200-223")
    fb, rb, gmb = oracle_adjoints(f, kn, A.target, 64, 0.8, 0.5, ref.keys, gbar_b)
    check("frame blocks", ga, gb, grg, fb, rb, gmb)
    assert np.all(ga.reshape(ga.shape[0], -1)[:, A.target.reshape(-1) == 1] == 0.0)
    assert np.all(ga[kn == 0] == 0.0)


def test_backward_single_block_32():
    f0, _, target = synth.single_block(0)
    f, kn = _support(f0[None], None, target)
    ref = fofse(f, kn, 32, 0.8, 0.5, 100)
    gbar_b = np.random.default_rng(4).normal(size=(1, int(target.sum()))).astype(np.float32)
    plan = _plan(32, 32, 32, 100, target)
    ga, grg, gb = gpu_backward(plan, f0[None], None, 0.8, 0.5, ref.keys, ref.coef, gbar_b,
                               "single block 32x32")
    fb, rb, gmb = oracle_adjoints(f, kn, target, 32, 0.8, 0.5, ref.keys, gbar_b)
    check("single block", ga, gb, grg, fb, rb, gmb)


def test_backward_long_record_and_ragged_panels():
    """K = 300: five panels of the recurrence (the last one ragged) and the
    large-record kernel; irregular masks, 24 x 20 areas in a 32-point grid."""
    rng = np.random.default_rng(12)
    n, M, N, T, K = 6, 24, 20, 32, 300
    target = np.zeros((M, N), np.uint8)
    target[8:16, 6:14] = 1
    m = np.arange(M)[:, None]
    nn = np.arange(N)[None, :]
    areas = (120 + 40 * np.cos(2 * np.pi * (0.11 * m + 0.05 * nn))[None]
             + 12 * rng.normal(size=(n, M, N))).astype(np.float32)
    known = (rng.random((n, M, N)) > 0.15).astype(np.uint8)
    f, kn = _support(areas, known, target)
    ref = fofse(f, kn, T, 0.85, 0.4, K)
    gbar_b = rng.normal(size=(n, int(target.sum()))).astype(np.float32)
    plan = _plan(M, N, T, K, target)
    ga, grg, gb = gpu_backward(plan, areas, known, 0.85, 0.4, ref.keys, ref.coef, gbar_b, "K=300")
    fb, rb, gmb = oracle_adjoints(f, kn, target, T, 0.85, 0.4, ref.keys, gbar_b)
    check("K=300", ga, gb, grg, fb, rb, gmb)


def test_backward_against_finite_differences(frame_areas):
    """Central differences (h = 1e-4) of the FP64 fixed-selection forward."""
    A = frame_areas
    idx = [5, 317, 640]
    f, kn = _support(A.areas[idx], A.known[idx], A.target)
    rho, gamma, K = 0.8, 0.5, 200
    ref = fofse(f, kn, 64, rho, gamma, K)
    rng = np.random.default_rng(8)
    gbar_b = rng.normal(size=(len(idx), int(A.target.sum()))).astype(np.float32)
    plan = _plan(48, 48, 64, K, A.target)
    ga, _, gb = gpu_backward(plan, A.areas[idx], A.known[idx], rho, gamma, ref.keys, ref.coef,
                             gbar_b, "finite differences")
    tb = A.target.astype(bool)
    h = 1e-4
    for i in range(len(idx)):
        gbar = np.zeros(f.shape[1:])
        gbar[tb] = gbar_b[i]

        def L(ff, r, g):
            return float(np.sum(replay(ff, kn[i], 64, r, g, ref.keys[i])[0] * gbar))

        v = rng.normal(size=f.shape[1:]) * kn[i]
        fd_f = (L(f[i] + h * v, rho, gamma) - L(f[i] - h * v, rho, gamma)) / (2 * h)
        fd_r = (L(f[i], rho + h, gamma) - L(f[i], rho - h, gamma)) / (2 * h)
        fd_g = (L(f[i], rho, gamma + h) - L(f[i], rho, gamma - h)) / (2 * h)
        print(f"[gpu] block {idx[i]}: df {np.sum(ga[i] * v):.9e} vs {fd_f:.9e}; "
              f"drho {gb[i, 0]:.9e} vs {fd_r:.9e}; dgamma {gb[i, 1]:.9e} vs {fd_g:.9e}", flush=True)
        assert np.sum(ga[i] * v) == pytest.approx(fd_f, rel=1e-5)
        assert gb[i, 0] == pytest.approx(fd_r, rel=1e-5)
        assert gb[i, 1] == pytest.approx(fd_g, rel=1e-5)


def test_backward_edge_cases(frame_areas):
    A = frame_areas
    sub = slice(0, 8)
    areas = A.areas[sub].copy()
    known = A.known[sub].copy()
    f, kn = _support(areas, known, A.target)
    ref = fofse(f, kn, 64, 0.8, 0.5, 50)
    keys, coef = ref.keys.copy(), ref.coef.copy()
    areas[2, 0, 0] = np.nan            # non-finite known sample
    known[2, 0, 0] = 1
    known[5] = 0                       # no support at all
    areas[6, 20, 20] = np.inf          # on B: ignored
    gbar_b = np.random.default_rng(1).normal(size=(8, int(A.target.sum()))).astype(np.float32)
    plan = _plan(48, 48, 64, 50, A.target)
    ga, grg, gb = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "edge cases")
    assert np.all(ga[2] == 0) and np.all(gb[2] == 0)
    assert np.all(ga[5] == 0) and np.all(gb[5] == 0)
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gb))
    ok = [0, 1, 3, 4, 6, 7]
    fb, rb, gmb = oracle_adjoints(f[ok], kn[ok], A.target, 64, 0.8, 0.5, keys[ok], gbar_b[ok])
    check("edge cases (regular blocks)", ga[ok], gb[ok], np.array([rb.sum(), gmb.sum()]), fb, rb, gmb)
    np.testing.assert_allclose(grg, [gb[:, 0].sum(), gb[:, 1].sum()], rtol=1e-12)
    # parameters out of range: every block gets zero gradients
    _, grg2, gb2 = gpu_backward(plan, areas, known, 1.5, 0.5, keys, coef, gbar_b, "rho 1.5")
    assert np.all(gb2 == 0) and np.all(grg2 == 0)
    # without dL/df, and twice in a row: the same bits
    _, grg3, gb3 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "no dL/df",
                                grad_areas=False)
    ga4, grg4, gb4 = gpu_backward(plan, areas, known, 0.8, 0.5, keys, coef, gbar_b, "repeat")
    assert np.array_equal(gb3, gb) and np.array_equal(grg3, grg)
    assert np.array_equal(ga4, ga) and np.array_equal(gb4, gb)
    # n = 0 is a no-op
    from paper_2207_01205_amd import fofse as F
    F.fofse_backward(plan.handle, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0)


def test_autograd_mse_loss(frame_areas):
    """torch.autograd end to end: forward kernel, MSE on B against the true
    pixels, adjoint kernel.  The adjoint is defined for any fixed selection, so
    every block is compared with the oracle adjoint of the GPU's own record and
    loss gradient, and the summed (rho_hat, gamma) gradient is always checked."""
    from paper_2207_01205_amd.autograd import fofse_extrapolate
    A = frame_areas
    sub = slice(400, 432)
    n = 32
    dev = torch.device("cuda", 0)
    plan = _plan(48, 48, 64, 200, A.target)
    tb = A.target.reshape(-1) == 1
    a = torch.from_numpy(A.areas[sub].copy()).to(dev).requires_grad_(True)
    k = torch.from_numpy(A.known[sub].copy()).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev, requires_grad=True)
    truth = torch.from_numpy(A.truth[sub].reshape(n, -1)[:, tb].copy()).to(dev)
    print("[gpu] autograd: 32 frame blocks, K=200", flush=True)
    out, status = fofse_extrapolate(a, rg, plan, k)
    loss = ((out - truth) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    assert torch.all(status == 0)
    # the record of the same forward (deterministic: the same bits as inside
    # the autograd call) and the loss gradient the backward received
    out2, sel, _, _ = plan.extrapolate(a.detach(), rg.detach(), known=k, record=True)
    assert torch.equal(out2, out.detach())
    sel = sel.cpu().numpy()
    f, kn = _support(A.areas[sub], A.known[sub], A.target)
    ref = fofse(f, kn, 64, 0.8, 0.5, 200)
    ok, div = selection_parity(sel, ref.keys, ref.margin, 1e-6, top_ref=ref.top)
    assert ok.all()
    gbar_b = (2.0 * (out.detach() - truth) / out.numel()).cpu().numpy()
    fb, rb, gmb = oracle_adjoints(f, kn, A.target, 64, 0.8, 0.5, sel, gbar_b)
    ga = a.grad.cpu().numpy()
    scale = np.abs(fb).reshape(n, -1).max(axis=1)
    err = np.abs(ga - fb).reshape(n, -1).max(axis=1)
    assert np.all(err <= 1e-5 * scale), np.max(err / scale)
    np.testing.assert_allclose(rg.grad.cpu().numpy(), [rb.sum(), gmb.sum()], rtol=1e-5)
    print(f"[gpu] autograd: {n} blocks ({int(div.sum())} diverging from the oracle's selection), "
          f"max rel dL/df {np.max(err / scale):.2e}", flush=True)


@pytest.mark.parametrize("T,side,path", [(64, 48, "grouped"), (64, 48, "split"), (32, 24, "split"),
                                         (16, 12, "split"), (128, 64, "auto")])
def test_backward_empty_record(T, side, path):
    """K = 0: the model is 0, so every gradient is 0.  The record pointers are
    valid but hold no iteration; no organisation may read them."""
    from paper_2207_01205_amd import fofse as F
    rng = np.random.default_rng(T + side)
    target = np.zeros((side, side), np.uint8)
    target[side // 3:2 * side // 3, side // 3:2 * side // 3] = 1
    n = 40
    areas = (100 + 20 * rng.normal(size=(n, side, side))).astype(np.float32)
    plan = _plan(side, side, T, 0, target)
    if path == "grouped":
        plan.set_path(F.FOFSE_PATH_GROUPED)
    elif path == "split":
        plan.set_path(F.FOFSE_PATH_SPLIT)
    print(f"[gpu] backward K = 0: T={T} {side}x{side} {path}", flush=True)
    dev = torch.device("cuda", 0)
    a = torch.from_numpy(areas).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    sel = torch.zeros(1, dtype=torch.int32, device=dev)
    cf = torch.zeros(2, dtype=torch.float64, device=dev)
    go = torch.from_numpy(rng.normal(size=(n, plan.nB)).astype(np.float32)).to(dev)
    ga = torch.full((n, side, side), 7.0, dtype=torch.float32, device=dev)
    grg = torch.zeros(2, dtype=torch.float64, device=dev)
    gb = torch.full((n, 2), 7.0, dtype=torch.float64, device=dev)
    F.fofse_backward(plan.handle, n, a.data_ptr(), 0, rg.data_ptr(), sel.data_ptr(), cf.data_ptr(), go.data_ptr(),
                     ga.data_ptr(), grg.data_ptr(), gb.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    assert np.all(ga.cpu().numpy() == 0.0)
    assert np.all(grg.cpu().numpy() == 0.0) and np.all(gb.cpu().numpy() == 0.0)
