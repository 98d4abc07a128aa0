"""Per-geometry choice of the kernel organisation by measurement.

For one plan and a sample batch, every organisation built for the plan's FFT
size is timed on the device (HIP events on the caller's stream, after one
warm-up call): the split path with each built number of wavefronts per block
and, for T = 64 and 128, the grouped path.  The fastest is set on the plan.  The
arithmetic is the same for every candidate (the selections and outputs agree
up to the rounding of the initial transform), so the choice only affects time.
"""

from __future__ import annotations

from . import fofse as F

# wavefronts per block built for the split path, per FFT size
SPLIT_WAVES = {16: (1, 2), 32: (1, 2, 4), 64: (2, 4, 8), 128: (8, 16)}


def candidates(T: int):
    """(label, path, waves) of every organisation built for FFT size T."""
    out = [(f"split/{w}", F.FOFSE_PATH_SPLIT, w) for w in SPLIT_WAVES[T]]
    if T in (64, 128):
        out.append(("grouped", F.FOFSE_PATH_GROUPED, 0))
    return out


def autotune(plan: F.Plan, areas, rho_gamma, known=None, repeats: int = 3):
    """Time every candidate on (areas, known) and keep the fastest on ``plan``.

    Returns {label: mean milliseconds per call} and the chosen label."""
    import torch
    dev = torch.device("cuda", plan.device)
    stream = torch.cuda.current_stream(dev)
    times = {}
    for label, path, waves in candidates(plan.T):
        try:
            plan.set_path(path)
            plan.set_waves(waves)
        except F.FofseError:
            continue                      # not available for this geometry
        plan.extrapolate(areas, rho_gamma, known=known, status=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(repeats):
            plan.extrapolate(areas, rho_gamma, known=known, status=False)
        e1.record(stream)
        torch.cuda.synchronize(dev)
        times[label] = e0.elapsed_time(e1) / repeats
    best = min(times, key=times.get)
    for label, path, waves in candidates(plan.T):
        if label == best:
            plan.set_path(path)
            plan.set_waves(waves)
    return times, best
