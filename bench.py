#!/usr/bin/env python3
"""FOFSE forward and forward+adjoint benchmark on one MI355X.

Workload: 1080p frame concealment (the paper's block-loss concealment setting:
16x16 lost blocks, 16-pixel support frame -> 48x48 areas, 64x64 DFT, rho_hat
0.8, gamma 0.5, K = 200 iterations), on seeded synthetic 8-bit frames with 10 %
of the 120 x 67 full macroblocks lost (804 blocks per frame).  One step = one
forward pass over a batch of ``--frames`` frames, inputs resident in HBM; the
forward+adjoint step adds the MSE gradient on B against the true pixels and the
adjoint pass (gradients for the known samples, rho_hat and gamma); the DCT leg
runs the same batch with DCT basis functions, and the full-compensation leg
with the orthogonality deficiency compensation of eqs. 10-13 (OFSE).  Prints
one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--frames F]
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T, K, RHO, GAMMA, AREA = 64, 200, 0.8, 0.5, 48
FP64_VECTOR_PEAK = 78.6e12     # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
FP32_VECTOR_PEAK = 157.3e12    # published packed-FP32 vector peak


# HBM traffic of the main forward kernel per launch on the 16-frame batch,
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch)
# of ``bench.py --steps 2 --warmup 0 --no-cpu-baseline --no-single-frame
# --no-single-block --no-adjoint --mixed 0 --no-dct --no-ofse --tune 0
# --copy-calibration 256 --jobs 1``.  In those runs a plain 256 MiB device copy
# read FETCH_SIZE = 131,093 KiB and WRITE_SIZE = 262,144 KiB, so FETCH_SIZE is
# scaled by 2.0 and WRITE_SIZE by 1.0.  The figure holds only for the kernel
# sources it was taken on (hash below); otherwise the bench reports null.
KERNEL_SOURCES = ("fofse_group.hip", "iterate.hpp", "device_common.hpp", "fofse_kernel.h")
TRAFFIC = {"sources_sha256_16": "ea4327c021b01fac", "blocks": 12864,
           "fetch_kib": 67343.0, "write_kib": 67336.7, "fetch_scale": 2.0, "write_scale": 1.0}


# FP64 instruction counters of the same kernel (rocprofv3 --pmc SQ_INSTS_VALU_FMA_F64
# SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 with four more SQ counters, ``bench.py
# --steps 2 --warmup 0 --no-cpu-baseline --no-single-frame --mixed 2048 --tune 0
# --jobs 1``), per dispatch on the same batch: FMA 434,005,852, ADD 213,030,048,
# MUL 102,321,940 wave instructions.
COUNTERS = {"sources_sha256_16": "ea4327c021b01fac", "blocks": 12864, "flop": 75735276288.0}


def measured_traffic(n_blocks: int):
    """HBM bytes per launch of the main forward kernel, or None when the kernel
    sources or the batch differ from those the counters were taken on."""
    if not _sources_match(TRAFFIC, n_blocks):
        return None
    kib = TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"]
    return kib * 1024.0


def measured_counter_flop(n_blocks: int):
    """FP64 FLOP per launch of the main forward kernel from its rocprofv3
    counters (64 lanes x (ADD_F64 + MUL_F64 + 2 FMA_F64) wave instructions),
    or None when the kernel sources or the batch differ from those measured."""
    if COUNTERS.get("flop") is None or not _sources_match(COUNTERS, n_blocks):
        return None
    return COUNTERS["flop"]


def _sources_match(rec, n_blocks: int) -> bool:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2207_01205_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16] == rec["sources_sha256_16"] and n_blocks == rec["blocks"]


def flops_per_block(T: int, K: int) -> float:
    """Algorithmic FLOP of one block: per iteration 19 per conjugate class
    (|R|^2: 3, two complex multiply-adds: 16) over T^2/2 + 2 classes, plus two
    T x T real FFTs at 2.5 T^2 log2(T^2) each (forward transform, synthesis)."""
    classes = T * T // 2 + 2
    return K * 19.0 * classes + 2 * 2.5 * T * T * np.log2(T * T)


def executed_flops_per_block(T: int, K: int) -> float:
    """FP64 operations the forward kernel's iteration actually issues per block
    (the loop of the general, complex-W form): per class |R|^2 (a multiply and
    a fused multiply-add, 3 FLOP) and the update as two complex sums of the two
    W reads followed by four fused multiply-adds (4 + 8 = 12 FLOP), 15 in all
    against the 19 credited; the two transforms as credited."""
    classes = T * T // 2 + 2
    return K * 15.0 * classes + 2 * 2.5 * T * T * np.log2(T * T)


def adjoint_flops_per_block(T: int, K: int, nB: int) -> float:
    """Algorithmic FLOP of the adjoint of one block for its selection record:
    the synthesis transposed (K nB real-by-complex multiply-adds, 4 FLOP), the
    transposed coefficient recurrence over the K(K-1)/2 iteration pairs (two
    complex multiply-adds, 16, and the two rho_hat terms, 20), and two T x T
    FFTs (weights with their rho_hat derivative, and the adjoint spectrum)."""
    return 4.0 * K * nB + 36.0 * K * (K - 1) / 2 + 2 * 2.5 * T * T * np.log2(T * T)


def dct_flops_per_block(T: int, K: int) -> float:
    """Algorithmic FLOP of one block with DCT basis functions: per iteration 6
    per bin over the T^2 bins (the four-entry Gram sum: 3, the scaled
    subtraction: 2, the magnitude comparison: 1), plus two T x T transforms at
    2.5 T^2 log2(T^2) each (forward transform, synthesis)."""
    return K * 6.0 * T * T + 2 * 2.5 * T * T * np.log2(T * T)


def adjoint_kernel_name(n: int, dev) -> str:
    """The adjoint kernel the library runs for n blocks of the 48 x 48 / T = 64 /
    K = 200 workload: grouped (blocks of one mask share W) from 8 blocks per
    compute unit, as the forward."""
    import torch
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    return "fofse_bwd_group_kernel<9>" if n >= 8 * n_cu else "fofse_bwd_kernel<64,256>"


def _frame(i):
    from paper_2207_01205_amd import synth
    a = synth.frame_concealment(i, 1000 + i)
    return a.areas, a.known, a.target, a.truth


def _frame4k(i):
    from paper_2207_01205_amd import synth
    a = synth.frame_concealment(i, 5000 + i, height=2160, width=3840, fraction=0.05)
    return a.areas, a.known, a.target, a.truth


def _map(fn, items, jobs):
    """fn over items in a fork pool of ``jobs`` processes (in this process
    when jobs <= 1, e.g. under a profiler)."""
    if jobs <= 1:
        return [fn(x) for x in items]
    with mp.get_context("fork").Pool(min(jobs, len(items))) as pool:
        return pool.map(fn, items)


JOBS = 16


def make_tuning_workload(n_train: int, n_held: int):
    """3840 x 2160 frames with 5 % of the 16 x 16 blocks lost (1,620 per
    frame): n_train frames for the fit, n_held further frames for the PSNR."""
    parts = _map(_frame4k, range(n_train + n_held), JOBS)
    cat = lambda j, sl: np.concatenate([p[j] for p in parts[sl]])
    tr = slice(0, n_train)
    he = slice(n_train, n_train + n_held)
    return ((cat(0, tr), cat(1, tr), cat(3, tr)), (cat(0, he), cat(1, he), cat(3, he)), parts[0][2])


def _frame_img(i):
    from paper_2207_01205_amd import synth
    return synth.frame(100 + i)


def make_mixed_workload(per_class: int, n_frames: int = 4):
    """The mixed-size batch: per_class blocks of each size class (4x4, 8x8,
    16x16, 32x32 losses), at seeded positions of n_frames synthetic 1080p
    frames, in a seeded order within each class."""
    from paper_2207_01205_amd import synth
    imgs = _map(_frame_img, range(n_frames), JOBS)
    classes = []
    for ci, (block, support, Tc, Kc) in enumerate(synth.MIXED_CLASSES):
        parts = [synth.mixed_blocks(img, 1000 * ci + j, block, support, per_class // n_frames)
                 for j, img in enumerate(imgs)]
        areas = np.concatenate([q[0] for q in parts])
        order = np.random.default_rng(ci).permutation(len(areas))
        classes.append({"block": block, "support": support, "T": Tc, "K": Kc,
                        "areas": np.ascontiguousarray(areas[order]), "target": parts[0][1]})
    return classes


def make_workload(n_frames: int):
    parts = _map(_frame, range(n_frames), JOBS)
    areas = np.concatenate([p[0] for p in parts])
    known = np.concatenate([p[1] for p in parts])
    truth = np.concatenate([p[3] for p in parts])
    return areas, known, parts[0][2], truth


def _oracle_chunk(args):
    areas, known, target = args
    from oracle.fofse_dft import fofse
    f = areas.astype(np.float32).astype(np.float64)
    kn = known * (1 - target)[None]
    r = fofse(f, kn, T, RHO, GAMMA, K)
    return r.g.reshape(len(f), -1)[:, target.reshape(-1) == 1], r.keys, r.margin, r.top, r.coef, r.W0


def cpu_baseline(areas, known, target, n_sample: int, workers: int):
    """The FP64 oracle, unchanged, on a seeded sample of the batch's blocks,
    split over ``workers`` processes.  Runs before the GPU is touched."""
    idx = np.sort(np.random.default_rng(11).choice(len(areas), n_sample, replace=False))
    chunks = np.array_split(idx, workers)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_chunk, [(areas[c], known[c], target) for c in chunks])
    dt = time.perf_counter() - t0
    g, keys, margin, top, coef, W0 = (np.concatenate([r[i] for r in res]) for i in range(6))
    info = {
        "value": n_sample / dt, "unit": "blocks/s", "cores": workers, "kind": "oracle",
        "sample": f"{n_sample} seeded blocks of the same batch (FP64 NumPy DFT-domain oracle, "
                  f"{workers} processes, {dt:.1f} s)",
        "host": _host_info(workers),
    }
    return info, (idx, g, keys, margin, top, coef, W0)


DCT_SAMPLE = 64        # oracle-checked blocks of the DCT-basis leg


def _dct_oracle_chunk(args):
    areas, known, target = args
    from oracle.fofse_dct import fofse_dct
    f = areas.astype(np.float32).astype(np.float64)
    kn = known * (1 - target)[None]
    r = fofse_dct(np.where(kn != 0, f, 0.0), kn, T, RHO, GAMMA, K)
    return r.g.reshape(len(f), -1)[:, target.reshape(-1) == 1], r.keys, r.margin, r.top


def dct_cpu_baseline(areas, known, target, n_sample: int, workers: int):
    """The FP64 DCT-basis oracle, unchanged, on a seeded sample of the batch's
    blocks (timed, and the parity reference of the DCT leg).  Runs before the
    GPU is touched."""
    idx = np.sort(np.random.default_rng(12).choice(len(areas), n_sample, replace=False))
    chunks = [c for c in np.array_split(idx, workers) if len(c)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(chunks)) as pool:
        res = pool.map(_dct_oracle_chunk, [(areas[c], known[c], target) for c in chunks])
    dt = time.perf_counter() - t0
    info = {"value": n_sample / dt, "unit": "blocks/s", "cores": len(chunks), "kind": "oracle",
            "sample": f"{n_sample} seeded blocks of the same batch (FP64 NumPy DCT oracle, "
                      f"{len(chunks)} processes, {dt:.1f} s)"}
    ref = (idx,) + tuple(np.concatenate([r[i] for r in res]) for i in range(4))
    return info, ref


def run_dct(d_areas, d_known, target, n, args, dev, base):
    """The same batch with DCT basis functions: K steps of one forward launch."""
    import torch
    from paper_2207_01205_amd import fofse as F
    plan = F.Plan(AREA, AREA, T, K, target, device=0)
    plan.set_basis(F.FOFSE_BASIS_DCT)
    out = torch.empty((n, plan.nB), dtype=torch.float32, device=dev)
    sel = torch.empty((n, K), dtype=torch.int32, device=dev)
    coef = torch.empty((n, K, 2), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        F.fofse_extrapolate_batch(plan.handle, n, d_areas.data_ptr(), d_known.data_ptr(),
                                  rg.data_ptr(), out.data_ptr(), sel.data_ptr(),
                                  coef.data_ptr(), st.data_ptr(), stream.cuda_stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    F.fofse_set_timing(plan.handle, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(args.steps):
        step()
    ev[1].record(stream)
    torch.cuda.synchronize()
    kern = float(np.mean(F.fofse_kernel_times(plan.handle, args.steps))) * 1e-3
    F.fofse_set_timing(plan.handle, False)
    total = ev[0].elapsed_time(ev[1]) * 1e-3
    fpb = dct_flops_per_block(T, K)
    res = {"value": n * args.steps / total, "unit": "blocks/s", "ms_per_step": total / args.steps * 1e3,
           "roofline": {"bound": "alu", "kernel": "fofse_dct_kernel", "flop_per_block": fpb,
                        "avg_launch_ms": kern * 1e3, "achieved": fpb * n / kern / 1e12,
                        "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                        "frac": fpb * n / kern / FP64_VECTOR_PEAK},
           "block_status_nonzero": int(np.count_nonzero(st.cpu().numpy()))}
    print(f"[bench] DCT basis: {total / args.steps * 1e3:.3f} ms per step, kernel {kern * 1e3:.3f} ms",
          file=sys.stderr, flush=True)
    if base is not None:
        info, ref = base
        info["sample_parity"] = sample_parity(ref, out.cpu().numpy(), sel.cpu().numpy())
        res["cpu_baseline"] = info
    plan.close()
    return res


OFSE_SAMPLE = 32       # oracle-checked blocks of the full-compensation leg


def ofse_flops_per_block(T: int, K: int) -> float:
    """Algorithmic FLOP of one block with the full compensation of eqs. 10-13:
    the FOFSE iteration plus, per iteration, the convolution (R (*) W)[u] over
    the full spectrum (two complex multiply-adds, 16 FLOP, per conjugate
    class)."""
    return flops_per_block(T, K) + K * 16.0 * (T * T // 2 + 2)


def _ofse_oracle_chunk(args):
    areas, known, target = args
    from oracle.ofse_dft import ofse_full
    kn = known * (1 - target)[None]
    out = []
    for b in range(len(areas)):
        f = areas[b].astype(np.float32).astype(np.float64)
        r = ofse_full(np.where(kn[b] != 0, f, 0.0), kn[b], T, RHO, K)
        out.append((r["g"].reshape(-1)[target.reshape(-1) == 1], r["keys"], r["margin"], r["top"]))
    return out


def ofse_cpu_baseline(areas, known, target, n_sample: int, workers: int):
    """The FP64 OFSE oracle (eqs. 10-13 in the DFT domain), unchanged, on a
    seeded sample of the batch's blocks (timed, and the parity reference of the
    full-compensation leg).  Runs before the GPU is touched."""
    idx = np.sort(np.random.default_rng(13).choice(len(areas), n_sample, replace=False))
    chunks = [c for c in np.array_split(idx, workers) if len(c)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(chunks)) as pool:
        res = pool.map(_ofse_oracle_chunk, [(areas[c], known[c], target) for c in chunks])
    dt = time.perf_counter() - t0
    rows = [r for part in res for r in part]
    info = {"value": n_sample / dt, "unit": "blocks/s", "cores": len(chunks), "kind": "oracle",
            "sample": f"{n_sample} seeded blocks of the same batch (FP64 NumPy OFSE oracle, "
                      f"{len(chunks)} processes, {dt:.1f} s)"}
    ref = (idx,) + tuple(np.stack([r[i] for r in rows]) for i in range(4))
    return info, ref


def run_ofse(d_areas, d_known, target, n, args, dev, base):
    """The same batch with the full compensation of eqs. 10-13 (OFSE)."""
    import torch
    from paper_2207_01205_amd import fofse as F
    plan = F.Plan(AREA, AREA, T, K, target, device=0)
    plan.set_compensation(F.FOFSE_COMP_FULL)
    out = torch.empty((n, plan.nB), dtype=torch.float32, device=dev)
    sel = torch.empty((n, K), dtype=torch.int32, device=dev)
    coef = torch.empty((n, K, 2), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        F.fofse_extrapolate_batch(plan.handle, n, d_areas.data_ptr(), d_known.data_ptr(),
                                  rg.data_ptr(), out.data_ptr(), sel.data_ptr(),
                                  coef.data_ptr(), st.data_ptr(), stream.cuda_stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    F.fofse_set_timing(plan.handle, True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(args.steps):
        step()
    ev[1].record(stream)
    torch.cuda.synchronize()
    kern = float(np.mean(F.fofse_kernel_times(plan.handle, args.steps))) * 1e-3
    F.fofse_set_timing(plan.handle, False)
    total = ev[0].elapsed_time(ev[1]) * 1e-3
    fpb = ofse_flops_per_block(T, K)
    res = {"value": n * args.steps / total, "unit": "blocks/s", "ms_per_step": total / args.steps * 1e3,
           "roofline": {"bound": "alu", "kernel": "fofse_group_kernel<64, 9, true>", "flop_per_block": fpb,
                        "avg_launch_ms": kern * 1e3, "achieved": fpb * n / kern / 1e12,
                        "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                        "frac": fpb * n / kern / FP64_VECTOR_PEAK},
           "block_status_nonzero": int(np.count_nonzero(st.cpu().numpy()))}
    print(f"[bench] full compensation: {total / args.steps * 1e3:.3f} ms per step, kernel {kern * 1e3:.3f} ms",
          file=sys.stderr, flush=True)
    if base is not None:
        info, ref = base
        info["sample_parity"] = sample_parity(ref, out.cpu().numpy(), sel.cpu().numpy())
        res["cpu_baseline"] = info
    plan.close()
    return res


def sample_parity(ref, gpu_out, gpu_sel, gpu_coef=None):
    """Compare the GPU's outputs with the oracle sample (parity rule).  With the
    GPU record's coefficients and the oracle's (constant compensation, DFT
    basis) also the largest difference of the selected |R_w[u]| relative to
    A0, against the rule's rounding floor."""
    from oracle.fofse_dft import FLOOR, divergence_report, selection_parity, spectral_drift
    idx, g, keys, margin, top = ref[:5]
    ok, div = selection_parity(gpu_sel[idx], keys, margin, top_ref=top)
    same = np.all(gpu_sel[idx] == keys, axis=1)
    err = np.abs(gpu_out[idx] - g).max(axis=1)
    rows = divergence_report(gpu_sel[idx], keys, margin, top, limit=len(idx))
    for r in rows:
        r["block"] = int(idx[r["block"]])
    res = {"blocks": int(len(idx)), "rule_ok": bool(ok.all()), "diverging": int(div.sum()),
           "max_abs_dg": float(err[same].max()) if same.any() else None,
           "floor_over_A0": FLOOR, "diverging_blocks": rows[:20],
           "failures": [r for r in rows if not r["within_rule"]][:5]}
    if gpu_coef is not None and len(ref) >= 7:
        coef_ref, W0 = ref[5], ref[6]
        d = spectral_drift(gpu_sel[idx], gpu_coef[idx], keys, coef_ref, W0, top, GAMMA)
        res["drift_max_over_A0"] = float(d.max())
    return res


SMALL_SAMPLE = 4       # oracle-checked blocks per class and variant of the small-size leg


def _small_oracle(args):
    areas, target, T_, K_, variant = args
    kn = np.broadcast_to(1 - target, areas.shape).astype(np.uint8)
    f = areas.astype(np.float32).astype(np.float64)
    sel_b = target.reshape(-1) == 1
    if variant == "dct":
        from oracle.fofse_dct import fofse_dct
        r = fofse_dct(np.where(kn != 0, f, 0.0), kn, T_, RHO, GAMMA, K_)
        return r.g.reshape(len(f), -1)[:, sel_b], r.keys, r.margin, r.top
    from oracle.ofse_dft import ofse_full
    res = [ofse_full(np.where(kn[b] != 0, f[b], 0.0), kn[b], T_, RHO, K_) for b in range(len(f))]
    return (np.stack([x["g"].reshape(-1)[sel_b] for x in res]), np.stack([x["keys"] for x in res]),
            np.stack([x["margin"] for x in res]), np.stack([x["top"] for x in res]))


def run_small_variants(classes, args, dev):
    """The DCT basis and the full compensation at T = 16 and 32, on the 4x4 and
    8x8 classes of the mixed-size batch (canonical masks): blocks/s, the
    kernel's HIP-event mean, its rate on the algorithmic FLOPs, and parity of
    a few oracle-checked blocks."""
    import torch
    from paper_2207_01205_amd import fofse as F
    out_all = {}
    for c in classes:
        if c["T"] not in (16, 32):
            continue
        T_, K_, A = c["T"], c["K"], c["areas"].shape[1]
        n = len(c["areas"])
        d_areas = torch.from_numpy(c["areas"]).to(dev)
        for variant in ("dct", "full"):
            plan = F.Plan(A, A, T_, K_, c["target"], device=0)
            if variant == "dct":
                plan.set_basis(F.FOFSE_BASIS_DCT)
                fpb, kname = dct_flops_per_block(T_, K_), f"fofse_dct_kernel<{T_}>"
            else:
                plan.set_compensation(F.FOFSE_COMP_FULL)
                fpb, kname = ofse_flops_per_block(T_, K_), f"fofse_fwd_kernel<{T_}, 1, true>"
            out = torch.empty((n, plan.nB), dtype=torch.float32, device=dev)
            sel = torch.empty((n, K_), dtype=torch.int32, device=dev)
            coef = torch.empty((n, K_, 2), dtype=torch.float64, device=dev)
            st = torch.empty((n,), dtype=torch.int32, device=dev)
            rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
            stream = torch.cuda.current_stream(dev)

            def step():
                F.fofse_extrapolate_batch(plan.handle, n, d_areas.data_ptr(), 0, rg.data_ptr(), out.data_ptr(),
                                          sel.data_ptr(), coef.data_ptr(), st.data_ptr(), stream.cuda_stream)

            for _ in range(max(1, args.warmup)):
                step()
            torch.cuda.synchronize()
            F.fofse_set_timing(plan.handle, True)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record(stream)
            for _ in range(args.steps):
                step()
            ev[1].record(stream)
            torch.cuda.synchronize()
            kern = float(np.mean(F.fofse_kernel_times(plan.handle, args.steps))) * 1e-3
            total = ev[0].elapsed_time(ev[1]) * 1e-3
            res = {"blocks": n, "value": n * args.steps / total, "unit": "blocks/s",
                   "ms_per_step": total / args.steps * 1e3,
                   "roofline": {"bound": "alu", "kernel": kname, "flop_per_block": fpb,
                                "avg_launch_ms": kern * 1e3, "achieved": fpb * n / kern / 1e12,
                                "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                                "frac": fpb * n / kern / FP64_VECTOR_PEAK},
                   "block_status_nonzero": int(np.count_nonzero(st.cpu().numpy()))}
            if not args.no_cpu_baseline:
                idx = np.arange(SMALL_SAMPLE)
                g, keys, margin, top = _small_oracle((c["areas"][:SMALL_SAMPLE], c["target"], T_, K_, variant))
                res["sample_parity"] = sample_parity((idx, g, keys, margin, top), out.cpu().numpy(),
                                                     sel.cpu().numpy())
            print(f"[bench] {variant} T={T_}: {res['ms_per_step']:.3f} ms per step, kernel {kern * 1e3:.3f} ms",
                  file=sys.stderr, flush=True)
            out_all[f"{variant}_T{T_}"] = res
            plan.close()
    return out_all


def run_single_block(args, dev):
    """The single-block configuration: one 32 x 32 area (seed 0 of the
    single-block generator, 16 x 16 centred missing block), T = 32, K = 100,
    rho_hat 0.8, gamma 0.5.  One workgroup runs it, so the figure of merit is
    latency: the whole call (weights, iteration kernel, synthesis) by HIP events
    around each call, and the iteration kernel alone, for every wavefront count
    of the split path; the rate is put against one compute unit's share of the
    FP64 peak.  The oracle's selection and output for the block are checked."""
    import torch
    from oracle.fofse_dft import fofse, selection_parity
    from paper_2207_01205_amd import fofse as F
    from paper_2207_01205_amd import synth
    from paper_2207_01205_amd.autotune import SPLIT_WAVES
    f, known, target = synth.single_block(0)
    T1, K1 = 32, 100
    a = torch.from_numpy(f.astype(np.float32)[None]).to(dev)
    rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
    ref = fofse(f.astype(np.float32).astype(np.float64), known, T1, RHO, GAMMA, K1)
    fpb = flops_per_block(T1, K1)
    cu_peak = FP64_VECTOR_PEAK / 256
    stream = torch.cuda.current_stream(dev)
    res = {"workload": "single 32x32 block, 16x16 centred missing block, T=32, K=100, rho=0.8, gamma=0.5 "
                       "(one workgroup)", "flop_per_block": fpb, "by_waves": {}}
    reps = 50
    for w in SPLIT_WAVES[T1]:
        plan = F.Plan(32, 32, T1, K1, target, device=0)
        plan.set_path(F.FOFSE_PATH_SPLIT)
        plan.set_waves(w)
        out, sel, coef, st = plan.extrapolate(a, rg, record=True)
        torch.cuda.synchronize()
        ok, _ = selection_parity(sel.cpu().numpy(), ref.keys[None], ref.margin[None], top_ref=ref.top[None])
        err = float(np.abs(out.cpu().numpy()[0] - ref.g.reshape(-1)[target.reshape(-1) == 1]).max())
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        F.fofse_set_timing(plan.handle, True)
        for i in range(reps):
            ev[2 * i].record(stream)
            plan.extrapolate(a, rg, out=out, status=False)
            ev[2 * i + 1].record(stream)
            torch.cuda.synchronize()
        kern = F.fofse_kernel_times(plan.handle, reps)
        F.fofse_set_timing(plan.handle, False)
        call_ms = float(np.median([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps)]))
        kern_ms = float(np.median(kern))
        res["by_waves"][f"split/{w}"] = {
            "call_latency_ms": call_ms, "kernel_ms": kern_ms,
            "kernel_tflops": fpb / (kern_ms * 1e-3) / 1e12,
            "frac_of_one_cu": fpb / (kern_ms * 1e-3) / cu_peak,
            "parity_ok": bool(ok[0]), "max_abs_dg": err}
        plan.close()
    best = min(res["by_waves"], key=lambda k: res["by_waves"][k]["call_latency_ms"])
    res["best"] = best
    res["call_latency_ms"] = res["by_waves"][best]["call_latency_ms"]
    res["frac_of_one_cu"] = res["by_waves"][best]["frac_of_one_cu"]
    res["one_cu_fp64_peak_tflops"] = cu_peak / 1e12
    print(f"[bench] single block: {res['call_latency_ms']:.3f} ms per call ({best})", file=sys.stderr, flush=True)
    return res


def _host_info(workers: int):
    """The host the CPU baseline ran on: model string, logical CPUs, the CPUs
    this process may use, and the worker processes started (at most 16, the
    host share of one GPU)."""
    return {"cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "workers": workers}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


MIXED_SAMPLE = 3       # oracle-checked blocks per size class


def _mixed_oracle(args):
    areas, target, T, K = args
    from oracle.fofse_dft import fofse
    kn = np.broadcast_to(1 - target, areas.shape).astype(np.uint8)
    r = fofse(areas.astype(np.float64), kn, T, RHO, GAMMA, K)
    return r.keys, r.margin, r.top, r.g.reshape(len(areas), -1)[:, target.reshape(-1) == 1]


def mixed_oracle_sample(classes, workers):
    """FP64 oracle on the first MIXED_SAMPLE blocks of every class."""
    tasks = [(c["areas"][:MIXED_SAMPLE], c["target"], c["T"], c["K"]) for c in classes]
    with mp.get_context("fork").Pool(min(workers, len(tasks))) as pool:
        return pool.map(_mixed_oracle, tasks)


def run_mixed(classes, refs, args, dev):
    """The mixed-size batch: plain (one launch per class, in turn, default
    organisation) against batched (organisation per class picked by the
    autotuner, the whole batch one graph, classes on concurrent streams or in
    turn as measured faster)."""
    import torch
    from oracle.fofse_dft import selection_parity
    from paper_2207_01205_amd import fofse as F
    from paper_2207_01205_amd.autotune import autotune
    from paper_2207_01205_amd.mixed import MixedBatch
    rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
    plans, inputs, outs, recs, sts = [], [], [], [], []
    for c in classes:
        A = c["areas"].shape[1]
        plan = F.Plan(A, A, c["T"], c["K"], c["target"], device=0)
        a = torch.from_numpy(c["areas"]).to(dev)
        n = a.shape[0]
        plans.append(plan)
        inputs.append((a, None))
        outs.append(torch.empty((n, plan.nB), dtype=torch.float32, device=dev))
        recs.append((torch.empty((n, c["K"]), dtype=torch.int32, device=dev),
                     torch.empty((n, c["K"], 2), dtype=torch.float64, device=dev)))
        sts.append(torch.empty((n,), dtype=torch.int32, device=dev))
    mb = MixedBatch(plans)
    print("[bench] mixed batch: plain, autotune, batched", file=sys.stderr, flush=True)
    n_all = sum(int(x[0].shape[0]) for x in inputs)
    flops = sum(int(x[0].shape[0]) * flops_per_block(c["T"], c["K"]) for x, c in zip(inputs, classes))
    steps = max(3, args.steps // 4)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    # plain: default organisation, classes one after the other on one stream
    for p_ in plans:
        p_.set_path(F.FOFSE_PATH_AUTO)
        p_.set_waves(0)
    t_plain = timed(lambda: mb.extrapolate(inputs, rg, outs, recs, sts, concurrent=False), steps)
    # autotune each class on a sample of its blocks
    tuned = {}
    for c, p_, (a, _) in zip(classes, plans, inputs):
        times, best = autotune(p_, a, rg)
        tuned[f"{c['block']}x{c['block']}/T{c['T']}"] = {"choice": best,
                                                         "ms_per_class": {k: round(v, 4) for k, v in times.items()}}
    print(f"[bench] autotune: {json.dumps(tuned)}", file=sys.stderr, flush=True)
    # batched: the tuned organisation per class, the whole batch captured once
    # and replayed; the classes on concurrent streams or one after the other,
    # whichever is faster (a persistent kernel that fills every compute unit
    # gains nothing from sharing them)
    t_launch = {}
    for label, conc in (("concurrent", True), ("sequential", False)):
        mb.extrapolate(inputs, rg, outs, recs, sts, concurrent=conc)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            mb.extrapolate(inputs, rg, outs, recs, sts, concurrent=conc)
        t_launch[label] = timed(graph.replay, steps)
        torch.cuda.synchronize()
        del graph
    launch = min(t_launch, key=t_launch.get)
    t_batched = t_launch[launch]
    adjoint = None if args.no_adjoint else run_mixed_adjoint(classes, plans, inputs, recs, rg, timed, steps,
                                                             n_all, t_batched, dev)
    parity = []
    if refs is not None:
        for c, ref, o, (sel, _), st in zip(classes, refs, outs, recs, sts):
            keys, margin, top, g_ref = ref
            s_h = sel[:MIXED_SAMPLE].cpu().numpy()
            ok, div = selection_parity(s_h, keys, margin, 1e-6, top_ref=top)
            same = np.all(s_h == keys, axis=1)
            err = np.abs(o[:MIXED_SAMPLE].cpu().numpy() - g_ref).max(axis=1)
            parity.append({"class": f"{c['block']}x{c['block']}", "blocks": MIXED_SAMPLE,
                           "rule_ok": bool(ok.all()), "diverging": int(div.sum()),
                           "max_abs_dg": float(err[same].max()) if same.any() else None,
                           "status_nonzero": int((st != 0).sum().item())})
    return {"workload": "mixed-size batch: 4x4/8x8/16x16/32x32 losses, areas 12/24/48/64, "
                        "T 16/32/64/128, K 32/64/200/300, one quarter each, synthetic 1080p frames",
            "blocks": n_all, "flop_per_batch": flops,
            "plain": {"ms_per_batch": t_plain * 1e3, "blocks_per_s": n_all / t_plain,
                      "fp64_peak_frac": flops / t_plain / FP64_VECTOR_PEAK},
            "batched": {"ms_per_batch": t_batched * 1e3, "blocks_per_s": n_all / t_batched,
                        "fp64_peak_frac": flops / t_batched / FP64_VECTOR_PEAK,
                        "organisation": tuned, "launch": launch,
                        "ms_per_launch_form": {k: round(v * 1e3, 3) for k, v in t_launch.items()}},
            "fwd_adjoint": adjoint,
            "sample_parity": parity}


def run_mixed_adjoint(classes, plans, inputs, recs, rg, timed, steps, n_all, t_fwd, dev):
    """The adjoint of every class of the mixed batch for the record of the
    batched forward (dL/dg a fixed pseudo-random field on B): the classes in
    turn on one stream, each plan's default organisation.  Reports the adjoint
    time per batch, the forward+adjoint rate and each class's adjoint kernel."""
    import torch
    from paper_2207_01205_amd import fofse as F
    stream = torch.cuda.current_stream(dev).cuda_stream
    gos, gas = [], []
    for i, (p_, (a, _)) in enumerate(zip(plans, inputs)):
        n = int(a.shape[0])
        g = np.random.default_rng(70 + i).normal(size=(n, p_.nB)).astype(np.float32)
        gos.append(torch.from_numpy(g).to(dev))
        gas.append(torch.empty_like(a))
    grg = torch.zeros((len(plans), 2), dtype=torch.float64, device=dev)

    def backward_all():
        for i, (p_, (a, _), (sel, coef), go, ga) in enumerate(zip(plans, inputs, recs, gos, gas)):
            F.fofse_backward(p_.handle, int(a.shape[0]), a.data_ptr(), 0, rg.data_ptr(), sel.data_ptr(),
                             coef.data_ptr(), go.data_ptr(), ga.data_ptr(), grg[i].data_ptr(), 0, stream)

    print("[bench] mixed batch: adjoint of every class", file=sys.stderr, flush=True)
    t_bwd = timed(backward_all, steps)
    per_class = {}
    for p_ in plans:
        F.fofse_set_timing(p_.handle, True)
    for _ in range(steps):
        backward_all()
    torch.cuda.synchronize()
    for c, p_, (a, _) in zip(classes, plans, inputs):
        n = int(a.shape[0])
        ms = float(np.mean(F.fofse_kernel_times(p_.handle, steps)))
        F.fofse_set_timing(p_.handle, False)
        fl = n * adjoint_flops_per_block(c["T"], c["K"], p_.nB)
        per_class[f"{c['block']}x{c['block']}/T{c['T']}"] = {
            "kernel_ms": round(ms, 4), "fp64_peak_frac": round(fl / (ms * 1e-3) / FP64_VECTOR_PEAK, 4)}
    ok = bool(torch.isfinite(grg).all().item()) and all(bool(torch.isfinite(g).all().item()) for g in gas)
    return {"adjoint_ms_per_batch": t_bwd * 1e3, "ms_per_batch": (t_fwd + t_bwd) * 1e3,
            "blocks_per_s": n_all / (t_fwd + t_bwd), "adjoint_per_class": per_class, "finite": ok}


def run_tuning(data, args, dev):
    """Adam on theta with (rho_hat, gamma) = sigmoid(theta), loss = MSE on B
    against the true pixels over every lost block of the training frames; the
    gradient comes from one replay of the captured forward+adjoint graph."""
    import torch
    from paper_2207_01205_amd import fofse as F
    (tr_a, tr_k, tr_t), (he_a, he_k, he_t), target = data
    tb = target.reshape(-1) == 1
    plan = F.Plan(AREA, AREA, T, K, target, device=0)
    nB = plan.nB

    def put(a, k, t):
        n = len(a)
        return (n, torch.from_numpy(a).to(dev), torch.from_numpy(k).to(dev),
                torch.from_numpy(np.ascontiguousarray(t.reshape(n, -1)[:, tb])).to(dev))

    n, a, k, truth = put(tr_a, tr_k, tr_t)
    rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
    out = torch.empty((n, nB), dtype=torch.float32, device=dev)
    sel = torch.empty((n, K), dtype=torch.int32, device=dev)
    coef = torch.empty((n, K, 2), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    gout = torch.empty_like(out)
    grg = torch.empty((2,), dtype=torch.float64, device=dev)
    gblk = torch.empty((n, 2), dtype=torch.float64, device=dev)

    def step():
        s = torch.cuda.current_stream(dev).cuda_stream
        F.fofse_extrapolate_batch(plan.handle, n, a.data_ptr(), k.data_ptr(), rg.data_ptr(),
                                  out.data_ptr(), sel.data_ptr(), coef.data_ptr(), st.data_ptr(), s)
        torch.sub(out, truth, out=gout)
        gout.mul_(2.0 / gout.numel())
        F.fofse_backward(plan.handle, n, a.data_ptr(), k.data_ptr(), rg.data_ptr(), sel.data_ptr(),
                         coef.data_ptr(), gout.data_ptr(), 0, grg.data_ptr(), gblk.data_ptr(), s)

    def heldout_psnr(params):
        nh, ha, hk, ht = put(he_a, he_k, he_t)
        p = torch.tensor(params, dtype=torch.float64, device=dev)
        o, _, _, _ = plan.extrapolate(ha, p, known=hk)
        mse = ((o.clamp(0.0, 255.0) - ht) ** 2).mean().item()
        return 10.0 * np.log10(255.0 ** 2 / mse)

    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    # Adam on theta = logit(rho_hat, gamma), made monotone: every step is one
    # replay at the proposed parameters, which yields both the training loss
    # there and its gradient; a proposal whose loss is higher than the current
    # one is rejected and the step size halved.  The fixed-selection gradient is
    # exact for the selection of the evaluated point but blind to selection
    # changes, which dominate this loss, so a plain Adam step can go uphill.
    psnr0 = heldout_psnr([RHO, GAMMA])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_steps = [0.0]

    def evaluate(th):
        params = torch.sigmoid(th)
        rg.copy_(params)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        t_steps[0] += e0.elapsed_time(e1) * 1e-3
        loss = ((out - truth) ** 2).mean().item()
        return loss, grg.cpu() * params * (1.0 - params)

    theta = torch.logit(torch.tensor([RHO, GAMMA], dtype=torch.float64))
    m1 = torch.zeros(2, dtype=torch.float64)
    m2 = torch.zeros(2, dtype=torch.float64)
    b1, b2, lr = 0.9, 0.999, args.tune_lr
    loss_cur, g_cur = evaluate(theta)
    loss0, accepted, evals = loss_cur, 0, 1
    for it in range(1, args.tune + 1):
        m1 = b1 * m1 + (1 - b1) * g_cur
        m2 = b2 * m2 + (1 - b2) * g_cur * g_cur
        step = lr * (m1 / (1 - b1 ** it)) / (torch.sqrt(m2 / (1 - b2 ** it)) + 1e-8)
        prop = theta - step
        loss_p, g_p = evaluate(prop)
        evals += 1
        if loss_p <= loss_cur:
            theta, loss_cur, g_cur = prop, loss_p, g_p
            accepted += 1
        else:
            lr *= 0.5
        params = torch.sigmoid(theta)
        print(f"[tune] step {it}: rho {params[0].item():.4f} gamma {params[1].item():.4f} "
              f"loss {loss_cur:.4f} ({'accepted' if loss_cur == loss_p else 'rejected'} {loss_p:.4f})",
              file=sys.stderr, flush=True)
    final = [float(x) for x in torch.sigmoid(theta)]
    psnr1 = heldout_psnr(final)
    del graph
    return {"frames": args.tune_frames, "frame": "3840x2160", "loss_fraction": 0.05,
            "blocks_per_step": n, "steps": args.tune, "graph_replays": evals, "accepted_steps": accepted,
            "optimizer": f"monotone Adam on logit(rho_hat, gamma), lr {args.tune_lr}, halved on a rejected step",
            "lr_end": lr,
            "blocks_per_s": n * evals / t_steps[0], "ms_per_step": t_steps[0] / evals * 1e3,
            "rho_gamma_start": [RHO, GAMMA], "rho_gamma_end": final,
            "loss_start": loss0, "loss_end": loss_cur,
            "heldout_psnr_db_start": psnr0, "heldout_psnr_db_end": psnr1,
            "heldout": "8 further frames, PSNR over the lost-block pixels, output clipped to 0..255"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint leg")
    ap.add_argument("--no-dct", action="store_true", help="skip the DCT-basis leg")
    ap.add_argument("--no-ofse", action="store_true", help="skip the full-compensation (OFSE) leg")
    ap.add_argument("--small-variants", action="store_true",
                    help="also time the DCT basis and the full compensation at T = 16 and 32 on the mixed batch's "
                         "4x4 and 8x8 classes (needs --mixed > 0)")
    ap.add_argument("--mixed", type=int, default=25000, metavar="PER_CLASS",
                    help="blocks per size class of the mixed-size batch (0 = skip)")
    ap.add_argument("--tune", type=int, default=50, metavar="STEPS",
                    help="fit (rho_hat, gamma) by monotone Adam for STEPS steps on 64 synthetic "
                         "3840x2160 frames with 5%% block loss, one captured graph per step "
                         "(forward, MSE gradient, adjoint), and report held-out PSNR (0 = skip)")
    ap.add_argument("--tune-frames", type=int, default=64)
    ap.add_argument("--jobs", type=int, default=16,
                    help="processes generating the synthetic inputs (1: in this process)")
    ap.add_argument("--tune-lr", type=float, default=0.1)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the workload, copy MIB MiB once with a plain device copy, so "
                         "that a counter run can scale FETCH_SIZE / WRITE_SIZE by known bytes")
    ap.add_argument("--no-single-block", action="store_true",
                    help="skip the single-block (32x32, T=32, K=100) latency leg")
    ap.add_argument("--no-single-frame", action="store_true",
                    help="skip the one-frame latency launches (so a profiler's per-kernel "
                         "average covers only full-batch launches)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(blocks are independent: a multi-GPU run would shard the block list; it is not built).",
              file=sys.stderr)
        sys.exit(2)

    # everything that forks runs before the GPU is initialised
    global JOBS
    JOBS = args.jobs
    print(f"[bench] generating {args.frames} frames", file=sys.stderr, flush=True)
    areas, known, target, truth = make_workload(args.frames)
    tune_data = make_tuning_workload(args.tune_frames, 8) if args.tune > 0 else None
    if args.mixed > 0:
        print(f"[bench] generating the mixed-size batch", file=sys.stderr, flush=True)
    mixed_data = make_mixed_workload(args.mixed) if args.mixed > 0 else None
    mixed_ref = None
    if mixed_data is not None and not args.no_cpu_baseline:
        mixed_ref = mixed_oracle_sample(mixed_data, min(16, len(os.sched_getaffinity(0))))
    n = len(areas)
    base = None
    if not args.no_cpu_baseline:
        workers = min(16, len(os.sched_getaffinity(0)))
        base = cpu_baseline(areas, known, target, min(args.cpu_sample, n), workers)
        print(f"[bench] cpu baseline: {base[0]['value']:.2f} blocks/s on {workers} processes",
              file=sys.stderr, flush=True)
    dct_base = None
    if not args.no_cpu_baseline and not args.no_dct:
        dct_base = dct_cpu_baseline(areas, known, target, min(DCT_SAMPLE, n),
                                    min(16, len(os.sched_getaffinity(0))))
    ofse_base = None
    if not args.no_cpu_baseline and not args.no_ofse:
        ofse_base = ofse_cpu_baseline(areas, known, target, min(OFSE_SAMPLE, n),
                                      min(16, len(os.sched_getaffinity(0))))

    import torch
    from paper_2207_01205_amd.fofse import Plan

    dev = torch.device("cuda", 0)
    plan = Plan(AREA, AREA, T, K, target, device=0)
    d_areas = torch.from_numpy(areas).to(dev)
    d_known = torch.from_numpy(known).to(dev)
    rg = torch.tensor([RHO, GAMMA], dtype=torch.float64, device=dev)
    out = torch.empty((n, plan.nB), dtype=torch.float32, device=dev)
    sel = torch.empty((n, K), dtype=torch.int32, device=dev)
    coef = torch.empty((n, K, 2), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones((nbytes // 4,), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] calibration copy of {nbytes} bytes", file=sys.stderr, flush=True)

    from paper_2207_01205_amd import fofse as F

    def step():
        F.fofse_extrapolate_batch(plan.handle, n, d_areas.data_ptr(), d_known.data_ptr(),
                                  rg.data_ptr(), out.data_ptr(), sel.data_ptr(),
                                  coef.data_ptr(), st.data_ptr(), stream.cuda_stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    F.fofse_set_timing(plan.handle, True)      # events around the main kernel of each step
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = np.array([ev[i].elapsed_time(ev[i + 1]) * 1e-3 for i in range(args.steps)])
    kern_ms = F.fofse_kernel_times(plan.handle, args.steps)
    F.fofse_set_timing(plan.handle, False)
    total = ev[0].elapsed_time(ev[-1]) * 1e-3
    print(f"[bench] {n} blocks x {args.steps} steps: {total * 1e3:.2f} ms (host wall {wall * 1e3:.2f} ms)",
          file=sys.stderr, flush=True)

    # one frame alone (804 blocks): the single-frame latency and rate
    n1 = int(np.count_nonzero(np.arange(n) < 804))
    t_frame = None
    if not args.no_single_frame:
        def step1():
            F.fofse_extrapolate_batch(plan.handle, n1, d_areas.data_ptr(), d_known.data_ptr(),
                                      rg.data_ptr(), out.data_ptr(), sel.data_ptr(),
                                      coef.data_ptr(), st.data_ptr(), stream.cuda_stream)
        step1()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            step1()
        e1.record(stream)
        torch.cuda.synchronize()
        t_frame = e0.elapsed_time(e1) * 1e-3 / 5

    # forward + adjoint: MSE on B against the true pixels, gradients for the
    # known samples, rho_hat and gamma (the forward's record feeds the adjoint)
    adj = None
    if not args.no_adjoint:
        tb = target.reshape(-1) == 1
        d_truth = torch.from_numpy(np.ascontiguousarray(truth.reshape(n, -1)[:, tb])).to(dev)
        gout = torch.empty_like(out)
        gareas = torch.empty_like(d_areas)
        grg = torch.empty((2,), dtype=torch.float64, device=dev)
        gblk = torch.empty((n, 2), dtype=torch.float64, device=dev)

        def step_adj(s=None):
            s = stream.cuda_stream if s is None else s
            F.fofse_extrapolate_batch(plan.handle, n, d_areas.data_ptr(), d_known.data_ptr(),
                                      rg.data_ptr(), out.data_ptr(), sel.data_ptr(),
                                      coef.data_ptr(), st.data_ptr(), s)
            torch.sub(out, d_truth, out=gout)
            gout.mul_(2.0 / gout.numel())
            F.fofse_backward(plan.handle, n, d_areas.data_ptr(), d_known.data_ptr(), rg.data_ptr(),
                             sel.data_ptr(), coef.data_ptr(), gout.data_ptr(), gareas.data_ptr(),
                             grg.data_ptr(), gblk.data_ptr(), s)

        def step_graphable():
            step_adj(torch.cuda.current_stream(dev).cuda_stream)

        for _ in range(args.warmup):
            step_adj()
        torch.cuda.synchronize()
        F.fofse_set_timing(plan.handle, True)   # forward and adjoint kernels alternate in the ring
        ea = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ea[0].record(stream)
        for _ in range(args.steps):
            step_adj()
        ea[1].record(stream)
        torch.cuda.synchronize()
        times = F.fofse_kernel_times(plan.handle, 2 * args.steps)
        F.fofse_set_timing(plan.handle, False)
        t_adj = ea[0].elapsed_time(ea[1]) * 1e-3
        bwd_k = float(np.mean(times[1::2])) * 1e-3
        fab = adjoint_flops_per_block(T, K, plan.nB)
        fpb_all = flops_per_block(T, K) + fab
        adj = {"value": n * args.steps / t_adj, "unit": "blocks/s",
               "ms_per_step": t_adj / args.steps * 1e3,
               "fp32_vector_peak_frac": fpb_all * n * args.steps / t_adj / FP32_VECTOR_PEAK,
               "adjoint_kernel": {"kernel": adjoint_kernel_name(n, dev), "flop_per_block": fab,
                                  "avg_launch_ms": bwd_k * 1e3,
                                  "achieved": fab * n / bwd_k / 1e12, "unit": "TFLOP/s",
                                  "peak": FP64_VECTOR_PEAK / 1e12,
                                  "frac": fab * n / bwd_k / FP64_VECTOR_PEAK},
               "grad_rho_gamma": [float(x) for x in grg.cpu().numpy()]}
        print(f"[bench] fwd+adjoint: {t_adj / args.steps * 1e3:.3f} ms per step, adjoint kernel "
              f"{bwd_k * 1e3:.3f} ms", file=sys.stderr, flush=True)

    # the same forward+adjoint step captured in one HIP graph and replayed
    if adj is not None:
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step_graphable()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step_graphable()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            graph.replay()
        eg = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        eg[0].record(stream)
        for _ in range(args.steps):
            graph.replay()
        eg[1].record(stream)
        torch.cuda.synchronize()
        t_g = eg[0].elapsed_time(eg[1]) * 1e-3
        adj["graph_value"] = n * args.steps / t_g
        adj["graph_ms_per_step"] = t_g / args.steps * 1e3
        del graph

    single_block = None if args.no_single_block else run_single_block(args, dev)
    dct = None if args.no_dct else run_dct(d_areas, d_known, target, n, args, dev, dct_base)
    ofse = None if args.no_ofse else run_ofse(d_areas, d_known, target, n, args, dev, ofse_base)
    tuning = run_tuning(tune_data, args, dev) if tune_data is not None else None
    mixed = run_mixed(mixed_data, mixed_ref, args, dev) if mixed_data is not None else None
    small = (run_small_variants(mixed_data, args, dev)
             if args.small_variants and mixed_data is not None else None)

    # final full-batch pass for the outputs checked below
    step()
    torch.cuda.synchronize()
    status = st.cpu().numpy()
    out_h = out.cpu().numpy()
    sel_h = sel.cpu().numpy()
    coef_h = coef.cpu().numpy()

    fpb = flops_per_block(T, K)
    kern = float(np.mean(kern_ms)) * 1e-3
    achieved = fpb * n / kern
    kname = "fofse_group_kernel<64, 9, false>" if n >= 8 * 256 else "fofse_fwd_kernel<64, 4>"
    result = {
        "metric": "blocks/s (16x16 loss, 48x48 area, K=200) fwd & fwd+adjoint; % FP32 VALU peak",
        "value": n * args.steps / total,
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"1080p frame concealment, 10% of 16x16 macroblocks lost, "
                               f"{args.frames} frames per step ({n} blocks), 48x48 areas, "
                               f"T=64, K=200, rho=0.8, gamma=0.5, forward",
                   "blocks_per_step": n, "frames_per_step": args.frames},
        "extrapolated_px_per_s": n * args.steps / total * plan.nB,
        "fp32_vector_peak_frac": achieved / FP32_VECTOR_PEAK,
        "single_frame": (None if t_frame is None else
                         {"blocks": n1, "ms": t_frame * 1e3, "blocks_per_s": n1 / t_frame}),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK,
                     "credited_flop_note": "achieved counts the algorithmic FLOP per block (19 per conjugate "
                                           "class and iteration plus two FFTs); the kernel issues fewer (see "
                                           "executed_*)",
                     "executed_flop_per_block": executed_flops_per_block(T, K),
                     "executed_achieved": executed_flops_per_block(T, K) * n / kern / 1e12,
                     "executed_frac": executed_flops_per_block(T, K) * n / kern / FP64_VECTOR_PEAK,
                     "counter_flop_per_launch": measured_counter_flop(n),
                     "counter_achieved": (None if measured_counter_flop(n) is None
                                          else measured_counter_flop(n) / kern / 1e12),
                     "traffic": measured_traffic(n) if kname.startswith("fofse_group") else None,
                     "traffic_unit": "bytes per launch (HBM, counters scaled by a copy of known size)",
                     "kernel": kname, "flop_per_block": fpb,
                     "avg_launch_ms": kern * 1e3, "avg_step_ms": float(np.mean(per_step)) * 1e3},
        "block_status_nonzero": int(np.count_nonzero(status)),
        "single_block": single_block,
        "fwd_adjoint": adj,
        "dct_basis": dct,
        "full_compensation": ofse,
    }
    if tuning is not None:
        result["tuning"] = tuning
    if mixed is not None:
        result["mixed"] = mixed
    if small is not None:
        result["small_variants"] = small
    if base is not None:
        info, ref = base
        info["sample_parity"] = sample_parity(ref, out_h, sel_h, coef_h)
        result["cpu_baseline"] = info
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
