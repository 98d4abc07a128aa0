"""Per-geometry choice of the kernel organisation by measurement.

For one plan and a sample batch, every organisation built for the plan's FFT
size is timed on the device (HIP events on the caller's stream, after one
warm-up call):

* the split path with each built number of wavefronts per block;
* for T = 64 and 128 the grouped path, with each built number of resident
  workgroups per compute unit (the persistent grid's size).

The number of blocks sharing one W per workgroup is not a dimension: it is
fixed by the registers and LDS of the grouped kernels (four blocks of one
wavefront each at T = 64, two blocks of four wavefronts at T = 128).

The fastest candidate is set on the plan.  The arithmetic is the same for every
candidate (the selections and outputs agree up to the rounding of the initial
transform), so the choice only affects time.  With a cache file the choice is
stored per device architecture, geometry, FFT size, K and batch size (rounded
to a power of two) and reused without timing.
"""

from __future__ import annotations

import json
import os

from . import fofse as F

# wavefronts per block built for the split path, per FFT size
SPLIT_WAVES = {16: (1, 2), 32: (1, 2, 4), 64: (2, 4, 8), 128: (8, 16)}
# resident workgroups per compute unit built for the grouped path, per FFT size
GROUPED_OCCUPANCY = {64: (1, 2), 128: (1,)}


def candidates(T: int):
    """(label, path, waves, workgroups per CU) of every organisation built for
    FFT size T."""
    out = [(f"split/{w}", F.FOFSE_PATH_SPLIT, w, 0) for w in SPLIT_WAVES[T]]
    for occ in GROUPED_OCCUPANCY.get(T, ()):
        out.append((f"grouped/{occ}", F.FOFSE_PATH_GROUPED, 0, occ))
    return out


def _apply(plan: F.Plan, path: int, waves: int, occ: int) -> None:
    plan.set_path(path)
    plan.set_waves(waves)
    plan.set_occupancy(occ)


def cache_key(plan: F.Plan, n_blocks: int, arch: str) -> str:
    bucket = 1 << max(0, int(n_blocks) - 1).bit_length()
    return f"{arch}/M{plan.M}xN{plan.N}/T{plan.T}/K{plan.K}/n{bucket}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune(plan: F.Plan, areas, rho_gamma, known=None, repeats: int = 3, cache: str | None = None):
    """Time every candidate on (areas, known) and keep the fastest on ``plan``.

    With ``cache`` (a JSON file path) an earlier choice for the same key is
    applied without timing, and a new one is stored.  Returns
    ({label: mean milliseconds per call}, chosen label); the times are empty
    when the choice came from the cache."""
    import torch
    dev = torch.device("cuda", plan.device)
    n = int(areas.shape[0])
    key = cache_key(plan, n, torch.cuda.get_device_properties(dev).gcnArchName)
    cands = {c[0]: c for c in candidates(plan.T)}
    if cache is not None:
        hit = _load(cache).get(key)
        if hit in cands:
            _apply(plan, *cands[hit][1:])
            return {}, hit
    stream = torch.cuda.current_stream(dev)
    times = {}
    for label, path, waves, occ in cands.values():
        try:
            _apply(plan, path, waves, occ)
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
    _apply(plan, *cands[best][1:])
    if cache is not None:
        entries = _load(cache)
        entries[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(entries, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return times, best
