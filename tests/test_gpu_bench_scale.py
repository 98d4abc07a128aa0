"""The bench's forward workload at its full size and in its launch
configuration, checked against the FP64 oracle on seeded samples: 16
synthetic 1080p frames with 10% of the 16 x 16 macroblocks lost (12,864
blocks, 48 x 48 areas, T = 64, K = 200, rho_hat = 0.8, gamma = 0.5), one launch
on the default organisation (the grouped kernel at this size).

Forward: the sampled blocks follow the selection rule and the output bar of
the other parity tests.  Adjoint: one launch over the whole batch with the
GPU's own record; the sampled blocks' dL/df and (rho_hat, gamma) gradients
match the oracle adjoint of the same record (the adjoint is defined for any
fixed selection) to the bars of the adjoint tests.
"""

import numpy as np
import pytest

from paper_2207_01205_amd import synth
from test_gpu_adjoint import TOL, oracle_adjoints
from test_gpu_parity import _plan, check_parity, oracle_on, run_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bench_batch():
    parts = [synth.frame_concealment(i, 1000 + i) for i in range(16)]
    areas = np.concatenate([p.areas for p in parts])
    known = np.concatenate([p.known for p in parts])
    return areas, known, parts[0].target


def test_bench_batch_forward_sampled(bench_batch):
    areas, known, target = bench_batch
    assert areas.shape == (12864, 48, 48)
    plan = _plan(48, 48, 64, 200, target)
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 0.5, "bench batch, 12,864 blocks")
    assert np.all(st == 0) and np.all(np.isfinite(out))
    idx = np.sort(np.random.default_rng(13).choice(len(areas), 40, replace=False))
    ref = oracle_on(areas[idx], known[idx], target, 64, 0.8, 0.5, 200)
    check_parity(ref, target, out[idx], sel[idx], coef[idx], st[idx], "bench batch sample")


def test_bench_batch_adjoint_sampled(bench_batch):
    areas, known, target = bench_batch
    n = areas.shape[0]
    plan = _plan(48, 48, 64, 200, target)
    dev = torch.device("cuda", 0)
    a = torch.from_numpy(areas).to(dev)
    k = torch.from_numpy(known).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    print("[gpu] bench batch adjoint, 12,864 blocks", flush=True)
    _, sel, coef, st = plan.extrapolate(a, rg, known=k, record=True)
    rng = np.random.default_rng(17)
    gbar = rng.normal(size=(n, plan.nB)).astype(np.float32)
    go = torch.from_numpy(gbar).to(dev)
    ga, grg, gb = plan.backward(a, rg, sel, coef, go, known=k, per_block=True)
    torch.cuda.synchronize()
    assert torch.all(st == 0)
    ga, gb, sel = ga.cpu().numpy(), gb.cpu().numpy(), sel.cpu().numpy()
    assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gb))
    np.testing.assert_allclose(grg.cpu().numpy(), gb.sum(axis=0), rtol=1e-12)
    idx = np.sort(rng.choice(n, 12, replace=False))
    f = areas[idx].astype(np.float64)
    kn = known[idx] * (1 - target)[None]
    fb, rb, gmb = oracle_adjoints(f, kn, target, 64, 0.8, 0.5, sel[idx], gbar[idx])
    scale = np.abs(fb).reshape(len(idx), -1).max(axis=1)
    err = np.abs(ga[idx] - fb).reshape(len(idx), -1).max(axis=1)
    assert np.all(err <= TOL * scale + 1e-12), np.max(err / scale)
    np.testing.assert_allclose(gb[idx, 0], rb, rtol=TOL, atol=TOL * np.abs(rb).max() * 1e-3)
    np.testing.assert_allclose(gb[idx, 1], gmb, rtol=TOL, atol=TOL * np.abs(gmb).max() * 1e-3)
    print(f"[gpu] bench batch adjoint sample: max rel dL/df {np.max(err / scale):.2e}", flush=True)


@pytest.fixture(scope="module")
def mixed_batch():
    """The bench's mixed-size batch at full size: 25,000 blocks of each class
    (4x4, 8x8, 16x16 and 32x32 losses at seeded positions of four synthetic
    1080p frames, seeded order within each class)."""
    imgs = [synth.frame(100 + i) for i in range(4)]
    classes = []
    for ci, (block, support, T, K) in enumerate(synth.MIXED_CLASSES):
        parts = [synth.mixed_blocks(img, 1000 * ci + j, block, support, 25000 // 4) for j, img in enumerate(imgs)]
        areas = np.concatenate([q[0] for q in parts])
        order = np.random.default_rng(ci).permutation(len(areas))
        classes.append((block, T, K, np.ascontiguousarray(areas[order]), parts[0][1]))
    return classes


def test_mixed_batch_full_size_sampled(mixed_batch):
    """Every class of the mixed batch in one launch each on its default
    organisation; two seeded blocks per class against the oracle forward and
    one against the oracle adjoint of the GPU's own record."""
    dev = torch.device("cuda", 0)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    for ci, (block, T, K, areas, target) in enumerate(mixed_batch):
        n, A = areas.shape[0], areas.shape[1]
        assert n == 25000
        plan = _plan(A, A, T, K, target)
        out, sel, coef, st = run_gpu(plan, areas, None, 0.8, 0.5, f"mixed {block}x{block} T={T} full class")
        assert np.all(st == 0) and np.all(np.isfinite(out))
        rng = np.random.default_rng(100 + ci)
        idx = np.sort(rng.choice(n, 2, replace=False))
        ref = oracle_on(areas[idx], None, target, T, 0.8, 0.5, K)
        check_parity(ref, target, out[idx], sel[idx], coef[idx], st[idx], f"mixed {block}x{block} sample")
        a = torch.from_numpy(areas).to(dev)
        gbar = rng.normal(size=(n, plan.nB)).astype(np.float32)
        s_t = torch.from_numpy(np.ascontiguousarray(sel)).to(dev)
        c_t = torch.from_numpy(np.ascontiguousarray(coef)).to(dev)
        ga, grg, gb = plan.backward(a, rg, s_t, c_t, torch.from_numpy(gbar).to(dev), per_block=True)
        torch.cuda.synchronize()
        ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
        assert np.all(np.isfinite(ga)) and np.all(np.isfinite(gb))
        j = idx[:1]
        kn = np.broadcast_to(1 - target, (1,) + target.shape).astype(np.uint8)
        fb, rb, gmb = oracle_adjoints(areas[j].astype(np.float64), kn, target, T, 0.8, 0.5, sel[j], gbar[j])
        scale = np.abs(fb).max()
        assert np.abs(ga[j] - fb).max() <= TOL * scale + 1e-12
        # a sampled block's gradient can be near 0 by cancellation: the absolute
        # bar is TOL of the largest gradient of the class
        np.testing.assert_allclose(gb[j, 0], rb, rtol=TOL, atol=TOL * np.abs(gb[:, 0]).max())
        np.testing.assert_allclose(gb[j, 1], gmb, rtol=TOL, atol=TOL * np.abs(gb[:, 1]).max())
        print(f"[gpu] mixed {block}x{block}: adjoint sample rel dL/df {np.abs(ga[j] - fb).max() / scale:.2e}",
              flush=True)


def test_bench_batch_dct_and_full_compensation_sampled(bench_batch):
    """The bench's DCT-basis and full-compensation legs: the same 12,864-block
    batch in one launch each, sampled against the DCT oracle and the OFSE
    oracle (eqs. 10-13)."""
    import test_gpu_dct as D
    import test_gpu_ofse as O
    areas, known, target = bench_batch
    rng = np.random.default_rng(19)
    plan = D._plan(48, 48, 200, target)
    out, sel, coef, st = D.run_gpu(plan, areas, known, 0.8, 0.5, "bench batch, DCT basis")
    assert np.all(st == 0) and np.all(np.isfinite(out))
    idx = np.sort(rng.choice(len(areas), 6, replace=False))
    ref = D.oracle_on(areas[idx], known[idx], target, 64, 0.8, 0.5, 200)
    D.check_parity(ref, target, out[idx], sel[idx], coef[idx], st[idx], "bench batch DCT sample")
    plan = O._plan(48, 48, 200, target)
    out, sel, coef, st = O.run_gpu(plan, areas, known, 0.8, 0.5, "bench batch, full compensation")
    assert np.all(st == 0) and np.all(np.isfinite(out))
    idx = np.sort(rng.choice(len(areas), 4, replace=False))
    ref = O.oracle_on(areas[idx], known[idx], target, 0.8, 200)
    O.check_parity(ref, target, out[idx], sel[idx], coef[idx], st[idx], "bench batch full compensation sample")
