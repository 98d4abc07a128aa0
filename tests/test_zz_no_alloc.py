"""fofse_extrapolate_batch_noalloc (the forward for callers that cannot
allocate) against fofse_extrapolate_batch on the same inputs: the same
kernels, so the same bits, on two calls in a row, the second with a smaller
batch (the fixed scratch keeps the first call's contents), for the grouped
DFT organisation, the T = 128 grouped organisation and the DCT basis (the
paths whose grouping workspace lives in the scratch) and the split path; and
the limit and the required record rejected with their status codes."""

import numpy as np
import pytest

from paper_2207_01205_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bufs(plan, n, dev):
    return (torch.empty((n, plan.nB), dtype=torch.float32, device=dev),
            torch.empty((n, plan.K), dtype=torch.int32, device=dev),
            torch.empty((n, plan.K, 2), dtype=torch.float64, device=dev),
            torch.empty((n,), dtype=torch.int32, device=dev))


def _call(fn, plan, n, a, k, rg, bufs, stream):
    out, sel, coef, st = bufs
    fn(plan.handle, n, a.data_ptr(), k.data_ptr() if k is not None else 0, rg.data_ptr(), out.data_ptr(),
       sel.data_ptr(), coef.data_ptr(), st.data_ptr(), stream)


CASES = [("grouped T=64", 48, 64, 120, "grouped", None),
         ("grouped T=128", 48, 128, 60, "grouped", None),
         ("DCT T=64", 48, 64, 80, None, "dct"),
         ("split T=64", 48, 64, 80, "split", None)]


@pytest.mark.parametrize("label,side,T,K,path,basis", CASES)
def test_noalloc_matches_allocating_entry_point(label, side, T, K, path, basis):
    from paper_2207_01205_amd import fofse as F
    A = synth.frame_concealment(12, 13)
    dev = torch.device("cuda", 0)
    plan = F.Plan(side, side, T, K, A.target)
    if path == "grouped":
        plan.set_path(F.FOFSE_PATH_GROUPED)
    elif path == "split":
        plan.set_path(F.FOFSE_PATH_SPLIT)
    if basis == "dct":
        plan.set_basis(F.FOFSE_BASIS_DCT)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    for n, lo in ((700, 0), (213, 301)):          # second call smaller, other blocks
        print(f"[gpu] no-alloc {label}: {n} blocks from {lo}", flush=True)
        a = torch.from_numpy(A.areas[lo:lo + n].copy()).to(dev)
        k = torch.from_numpy(A.known[lo:lo + n].copy()).to(dev)
        ref = _bufs(plan, n, dev)
        got = _bufs(plan, n, dev)
        for t in got:
            t.fill_(7)
        _call(F.fofse_extrapolate_batch, plan, n, a, k, rg, ref, s)
        _call(F.fofse_extrapolate_batch_noalloc, plan, n, a, k, rg, got, s)
        torch.cuda.synchronize()
        for x, y in zip(ref, got):
            assert torch.equal(x, y), label
        assert int((ref[3] != 0).sum()) == 0


def test_noalloc_limits():
    from paper_2207_01205_amd import fofse as F
    A = synth.frame_concealment(12, 13)
    dev = torch.device("cuda", 0)
    plan = F.Plan(48, 48, 64, 10, A.target)
    n = F.NOALLOC_MAX_BLOCKS + 1
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    x = torch.zeros(16, dtype=torch.float32, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    print("[gpu] no-alloc limits", flush=True)
    # beyond the maximum: refused before anything is read or enqueued
    with pytest.raises(F.FofseError) as e:
        F.fofse_extrapolate_batch_noalloc(plan.handle, n, x.data_ptr(), 0, rg.data_ptr(), x.data_ptr(),
                                          x.data_ptr(), x.data_ptr(), 0, s)
    assert e.value.status == F.FOFSE_ERR_LIMIT
    # the record is required
    with pytest.raises(F.FofseError) as e:
        F.fofse_extrapolate_batch_noalloc(plan.handle, 1, x.data_ptr(), 0, rg.data_ptr(), x.data_ptr(),
                                          0, x.data_ptr(), 0, s)
    assert e.value.status == F.FOFSE_ERR_ARG
    F.fofse_extrapolate_batch_noalloc(plan.handle, 0, 0, 0, 0, 0, 0, 0, 0, s)    # n = 0: no-op
