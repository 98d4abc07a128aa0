"""Distribution of the OFSE compensation factors of eq. 13 on synthetic frames.

Test infrastructure (oracle side, CPU only).  Runs the full-compensation
oracle (``ofse_dft.ofse_full``) on lost 16 x 16 blocks of the seeded synthetic
1080p concealment workload (48 x 48 areas, 64-point DFT, rho_hat = 0.8, as in
the setting of Fig. 2) and prints a text histogram of Re gamma_u over all
iterations of all blocks, with its mode, median and quartiles.

    python -m oracle.gamma_histogram [--blocks 81] [--iterations 200] [--workers 8]
"""

from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.ofse_dft import ofse_full  # noqa: E402


def _one(args):
    f, known, K = args
    return ofse_full(f, known, 64, 0.8, K)["gamma"]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=81)
    ap.add_argument("--iterations", type=int, default=200)
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    from paper_2207_01205_amd import synth
    A = synth.frame_concealment(args.seed, args.seed + 1)
    idx = np.sort(np.random.default_rng(args.seed).choice(len(A), args.blocks, replace=False))
    tasks = []
    for i in idx:
        kn = A.known[i] * (1 - A.target)
        tasks.append((A.areas[i].astype(np.float64), kn, args.iterations))
    with mp.get_context("fork").Pool(args.workers) as pool:
        gams = pool.map(_one, tasks)
    allg = np.concatenate(gams)
    undefined = int(np.isnan(allg.real).sum())
    allg = allg[~np.isnan(allg.real)]
    g = allg.real
    edges = np.arange(-0.5, 1.55, 0.05)
    hist, _ = np.histogram(np.clip(g, edges[0], edges[-1] - 1e-12), edges)
    print(f"Re gamma_u over {len(g)} iterations of {args.blocks} blocks ({undefined} iterations "
          f"with a zero residual left out) "
          f"(K = {args.iterations}, T = 64, rho_hat = 0.8, 48 x 48 areas, frame seed {args.seed})")
    top = hist.max()
    for lo, c in zip(edges[:-1], hist):
        print(f"  [{lo:+.2f}, {lo + 0.05:+.2f})  {c:6d}  " + "#" * int(round(60 * c / top)))
    q = np.percentile(g, [25, 50, 75])
    mode = edges[np.argmax(hist)] + 0.025
    print(f"mode {mode:.3f}  median {q[1]:.3f}  quartiles {q[0]:.3f} .. {q[2]:.3f}  "
          f"mean {g.mean():.3f}  |Im gamma| median {np.median(np.abs(allg.imag)):.3g}")


if __name__ == "__main__":
    main()
