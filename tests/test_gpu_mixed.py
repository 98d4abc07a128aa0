"""The size classes of the mixed-size workload (4x4 / 8x8 / 16x16 / 32x32 losses
with FFT sizes 16 / 32 / 64 / 128) against the FP64 oracle, forward and
adjoint, through the C ABI.  Areas lie inside a seeded synthetic frame, so every
block's support is the complement of B (known = NULL)."""

import numpy as np
import pytest

from oracle.fofse_adjoint import fofse_adjoint
from oracle.fofse_dft import fofse, selection_parity
from paper_2207_01205_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def frame_img():
    return synth.frame(11)


def _run(frame_img, cls_index, n, seed, waves=0):
    from paper_2207_01205_amd.fofse import Plan
    block, support, T, K = synth.MIXED_CLASSES[cls_index]
    areas, target, truth, _ = synth.mixed_blocks(frame_img, seed, block, support, n)
    A = areas.shape[1]
    print(f"[gpu] mixed class {block}x{block}: n={n} area={A} T={T} K={K} waves={waves}", flush=True)
    dev = torch.device("cuda", 0)
    plan = Plan(A, A, T, K, target, device=0)
    if waves == "grouped":
        from paper_2207_01205_amd.fofse import FOFSE_PATH_GROUPED
        plan.set_path(FOFSE_PATH_GROUPED)
    else:
        plan.set_waves(waves)
    a = torch.from_numpy(areas).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    out, sel, coef, st = plan.extrapolate(a, rg, record=True)
    torch.cuda.synchronize()
    f = areas.astype(np.float64)
    kn = np.broadcast_to(1 - target, f.shape).astype(np.uint8)
    ref = fofse(f, kn, T, 0.8, 0.5, K)
    return plan, areas, target, truth, out.cpu().numpy(), sel.cpu().numpy(), coef.cpu().numpy(), st.cpu().numpy(), ref, f, kn


@pytest.mark.parametrize("cls_index", [0, 1])
def test_mixed_class_forward_and_adjoint(frame_img, cls_index):
    plan, areas, target, truth, out, sel, coef, st, ref, f, kn = _run(frame_img, cls_index, 48, 100 + cls_index)
    T, K = plan.T, plan.K
    assert np.all(st == 0)
    ok, div = selection_parity(sel, ref.keys, ref.margin, 1e-6, top_ref=ref.top)
    assert ok.all(), np.nonzero(~ok)[0]
    same = np.all(sel == ref.keys, axis=1)
    tb = target.reshape(-1) == 1
    err = np.abs(out - ref.g.reshape(len(f), -1)[:, tb]).max(axis=1)
    assert np.all(err[same] <= 1e-3), err[same].max()
    print(f"[gpu] forward: diverging {int(div.sum())}/{len(f)}, max|dg| {err[same].max():.2e}", flush=True)
    # adjoint with the oracle's record
    dev = torch.device("cuda", 0)
    gbar_b = np.random.default_rng(cls_index).normal(size=(len(f), plan.nB)).astype(np.float32)
    cf = np.stack([ref.coef.real, ref.coef.imag], -1)
    ga, grg, gb = plan.backward(torch.from_numpy(areas).to(dev),
                                torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev),
                                torch.from_numpy(ref.keys.astype(np.int32)).to(dev),
                                torch.from_numpy(np.ascontiguousarray(cf)).to(dev),
                                torch.from_numpy(gbar_b).to(dev), per_block=True)
    torch.cuda.synchronize()
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    tbm = target.astype(bool)
    for i in range(0, len(f), 6):
        gbar = np.zeros(f.shape[1:])
        gbar[tbm] = gbar_b[i]
        adj = fofse_adjoint(f[i], kn[i], T, 0.8, 0.5, ref.keys[i], gbar)
        scale = np.abs(adj.f_bar).max()
        assert np.abs(ga[i] - adj.f_bar).max() <= 1e-6 * scale
        assert gb[i, 0] == pytest.approx(adj.rho_bar, rel=1e-6, abs=1e-9 * scale)
        assert gb[i, 1] == pytest.approx(adj.gamma_bar, rel=1e-6, abs=1e-9 * scale)


@pytest.mark.parametrize("waves", [8, 16, "grouped"])
def test_mixed_class_128_forward(frame_img, waves):
    """32 x 32 losses in 64 x 64 areas, 128-point DFT, K = 300 (row-half
    spectra; 8 or 16 wavefronts per block, or two blocks of four wavefronts
    sharing W)."""
    plan, areas, target, truth, out, sel, coef, st, ref, f, kn = _run(frame_img, 3, 8, 103, waves)
    assert np.all(st == 0)
    ok, div = selection_parity(sel, ref.keys, ref.margin, 1e-6, top_ref=ref.top)
    assert ok.all(), np.nonzero(~ok)[0]
    same = np.all(sel == ref.keys, axis=1)
    tb = target.reshape(-1) == 1
    err = np.abs(out - ref.g.reshape(len(f), -1)[:, tb]).max(axis=1)
    assert same.sum() >= 6 and np.all(err[same] <= 1e-3), (same, err)
    c_ref = np.stack([ref.coef.real, ref.coef.imag], -1)
    print(f"[gpu] T=128: diverging {int(div.sum())}/{len(f)}, max|dg| {err[same].max():.2e}, "
          f"max|dc| {np.abs(coef - c_ref)[same].max():.2e}", flush=True)


@pytest.mark.parametrize("path", ["split", "grouped"])
def test_128_irregular_masks_and_flags(frame_img, path):
    """T = 128 with irregular support masks, a block without support, a NaN
    known sample, and the adjoint of the record (zero for the flagged blocks).
    Blocks 0 and 2 share a mask (on the grouped path a live block next to a flagged
    one), as do blocks 3 and 4; block 1 is alone."""
    from paper_2207_01205_amd import fofse as F
    block, support, T, K = synth.MIXED_CLASSES[3]
    areas, target, truth, _ = synth.mixed_blocks(frame_img, 77, block, support, 5)
    rng = np.random.default_rng(5)
    known = (rng.random(areas.shape) > 0.2).astype(np.uint8)
    known[1] = 0
    areas[2, 3, 3] = np.nan
    known[2, 3, 3] = 1
    known[0] = known[2]
    known[4] = known[3]
    dev = torch.device("cuda", 0)
    plan = F.Plan(64, 64, T, 60, target, device=0)
    plan.set_path(F.FOFSE_PATH_GROUPED if path == "grouped" else F.FOFSE_PATH_SPLIT)
    print(f"[gpu] T=128 irregular masks and flags, {path}", flush=True)
    out, sel, coef, st = plan.extrapolate(torch.from_numpy(areas).to(dev),
                                          torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev),
                                          known=torch.from_numpy(known).to(dev), record=True)
    torch.cuda.synchronize()
    out, sel, st = out.cpu().numpy(), sel.cpu().numpy(), st.cpu().numpy()
    assert st[1] == F.FOFSE_BLOCK_NO_SUPPORT and st[2] == F.FOFSE_BLOCK_NONFINITE
    assert np.all(out[[1, 2]] == 0) and np.all(sel[[1, 2]] == 0)
    ok_blocks = [0, 3, 4]
    f = areas[ok_blocks].astype(np.float64)
    kn = (known[ok_blocks] * (1 - target)).astype(np.uint8)
    ref = fofse(f, kn, T, 0.8, 0.5, 60)
    ok, _ = selection_parity(sel[ok_blocks], ref.keys, ref.margin, 1e-6, top_ref=ref.top)
    assert ok.all()
    same = np.all(sel[ok_blocks] == ref.keys, axis=1)
    err = np.abs(out[ok_blocks] - ref.g.reshape(3, -1)[:, target.reshape(-1) == 1]).max(axis=1)
    assert np.all(err[same] <= 1e-3)
    # the adjoint of the same record: zero for the flagged blocks, the oracle
    # adjoint's for the others
    gbar = np.random.default_rng(6).normal(size=(5, plan.nB)).astype(np.float32)
    ga, _, gb = plan.backward(torch.from_numpy(areas).to(dev),
                              torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev),
                              torch.from_numpy(sel).to(dev), coef,
                              torch.from_numpy(gbar).to(dev), known=torch.from_numpy(known).to(dev), per_block=True)
    torch.cuda.synchronize()
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    assert np.all(ga[[1, 2]] == 0) and np.all(gb[[1, 2]] == 0)
    tb = target.astype(bool)
    for j, b in enumerate(ok_blocks):
        gfull = np.zeros(target.shape)
        gfull[tb] = gbar[b]
        adj = fofse_adjoint(f[j], kn[j], T, 0.8, 0.5, sel[b], gfull)
        scale = np.abs(adj.f_bar).max()
        assert np.abs(ga[b] - adj.f_bar).max() <= 1e-6 * scale
        assert gb[b, 0] == pytest.approx(adj.rho_bar, rel=1e-6)
        assert gb[b, 1] == pytest.approx(adj.gamma_bar, rel=1e-6)


def test_mixed_batch_graph_and_autotune(frame_img):
    """All four classes in one captured graph on concurrent streams give the
    same bits as the classes run one after another; the autotuner's choice
    stays within the parity rule."""
    from paper_2207_01205_amd import fofse as F
    from paper_2207_01205_amd.autotune import autotune
    from paper_2207_01205_amd.mixed import MixedBatch
    dev = torch.device("cuda", 0)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    plans, inputs, outs, recs, data = [], [], [], [], []
    for ci, (block, support, T, K) in enumerate(synth.MIXED_CLASSES):
        areas, target, _, _ = synth.mixed_blocks(frame_img, 500 + ci, block, support, 40)
        A = areas.shape[1]
        plans.append(F.Plan(A, A, T, K, target, device=0))
        a = torch.from_numpy(areas).to(dev)
        inputs.append((a, None))
        outs.append(torch.empty((40, plans[-1].nB), dtype=torch.float32, device=dev))
        recs.append((torch.empty((40, K), dtype=torch.int32, device=dev),
                     torch.empty((40, K, 2), dtype=torch.float64, device=dev)))
        data.append((areas, target, T, K))
    print("[gpu] mixed batch: 4 classes x 40 blocks, sequential vs graph", flush=True)
    mb = MixedBatch(plans)
    mb.extrapolate(inputs, rg, outs, recs, concurrent=False)
    torch.cuda.synchronize()
    seq = [(o.cpu().numpy().copy(), r[0].cpu().numpy().copy()) for o, r in zip(outs, recs)]
    graph = torch.cuda.CUDAGraph()
    mb.extrapolate(inputs, rg, outs, recs)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        mb.extrapolate(inputs, rg, outs, recs)
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        for (o_seq, s_seq), o, r in zip(seq, outs, recs):
            assert np.array_equal(o.cpu().numpy(), o_seq) and np.array_equal(r[0].cpu().numpy(), s_seq)
    del graph
    # autotune the 16x16 class and check the chosen organisation against the oracle
    areas, target, T, K = data[2]
    times, best = autotune(plans[2], inputs[2][0], rg)
    print(f"[gpu] autotune T=64: {best} {times}", flush=True)
    out, sel, coef, st = plans[2].extrapolate(inputs[2][0], rg, record=True)
    torch.cuda.synchronize()
    f = areas[:12].astype(np.float64)
    kn = np.broadcast_to(1 - target, f.shape).astype(np.uint8)
    ref = fofse(f, kn, T, 0.8, 0.5, K)
    ok, _ = selection_parity(sel.cpu().numpy()[:12], ref.keys, ref.margin, 1e-6, top_ref=ref.top)
    assert ok.all()


@pytest.mark.parametrize("T,side,path,waves,comp", [
    (16, 12, "split", 1, "constant"), (32, 24, "split", 2, "constant"), (64, 48, "split", 4, "constant"),
    (64, 48, "grouped", 0, "constant"), (128, 64, "split", 8, "constant"), (128, 64, "grouped", 0, "constant"),
    (32, 24, "split", 0, "full"), (64, 48, "grouped", 0, "full")])
def test_bad_parameters_flag_alone_on_every_path(T, side, path, waves, comp):
    """rho_hat outside (0, 1]: every block reports FOFSE_BLOCK_BAD_PARAM and
    nothing else, also a block with a non-finite known sample or no support,
    and its record and model are zero, on every organisation."""
    from paper_2207_01205_amd.fofse import (FOFSE_BLOCK_BAD_PARAM, FOFSE_COMP_FULL, FOFSE_PATH_GROUPED,
                                            FOFSE_PATH_SPLIT, Plan)
    rng = np.random.default_rng(T)
    target = np.zeros((side, side), np.uint8)
    q = side // 4
    target[q:side - q, q:side - q] = 1
    areas = (100 + 20 * rng.normal(size=(6, side, side))).astype(np.float32)
    known = np.broadcast_to(1 - target, areas.shape).copy()
    areas[2, 0, 0] = np.nan
    known[4] = 0
    plan = Plan(side, side, T, 20, target, device=0)
    plan.set_path(FOFSE_PATH_GROUPED if path == "grouped" else FOFSE_PATH_SPLIT)
    if waves:
        plan.set_waves(waves)
    if comp == "full":
        plan.set_compensation(FOFSE_COMP_FULL)
    dev = torch.device("cuda", 0)
    print(f"[gpu] bad parameters: T={T} {path} waves={waves} {comp}", flush=True)
    a = torch.from_numpy(areas).to(dev)
    k = torch.from_numpy(known).to(dev)
    rg = torch.tensor([1.5, 0.5], dtype=torch.float64, device=dev)
    out, sel, coef, st = plan.extrapolate(a, rg, known=k, record=True)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert np.all(st == FOFSE_BLOCK_BAD_PARAM), st
    assert np.all(out.cpu().numpy() == 0) and np.all(sel.cpu().numpy() == 0) and np.all(coef.cpu().numpy() == 0)
