"""Seeded synthetic workloads shaped like the paper's block-loss concealment runs.

The paper conceals 16x16 blocks cut out of natural test images, with a 16-pixel
support frame around each block and a 64x64 FFT (Section 4, Results).  Those
images are not available, so this module draws stand-in frames and loss maps.

This module holds none of the extrapolation method's arithmetic: no weighting
function, no transform, no iteration.  It only produces pixels and geometry
(which samples of an area are known, which are to be extrapolated), and it is
the one module that both the FP64 oracle tests and the HIP path are fed from.

Every generator takes an integer seed and derives independent streams for its
components with ``numpy.random.SeedSequence.spawn``, so a component's values do
not change when another component's draw count changes.
"""

from __future__ import annotations

import dataclasses

import numpy as np

# Macroblock size and support width of the paper's concealment experiment.
MB = 16
SUPPORT = 16


# ---------------------------------------------------------------------------
# Single block (32x32 area, 16x16 centred loss)
# ---------------------------------------------------------------------------

def single_block(seed: int = 0, size: int = 32, block: int = 16):
    """One smooth-plus-oscillation test area with a centred missing block.

    f[m, n] = 40 + 0.5 m + 0.3 n + sum_{i=1,2} 30 cos(2 pi (a_i m + b_i n) + t_i)
              + N(0, 2^2),
    a_i, b_i ~ U[0, 0.25] cycles/px, t_i ~ U[0, 2 pi).  Draw order: a1, b1, t1,
    a2, b2, t2, then size*size Gaussian samples in row-major order.

    Returns (f, known, target): f float64 (size, size); known and target uint8
    masks (1 = sample in the support area A / in the missing area B).
    """
    rng = np.random.default_rng(seed)
    params = []
    for _ in range(2):
        a = rng.uniform(0.0, 0.25)
        b = rng.uniform(0.0, 0.25)
        t = rng.uniform(0.0, 2.0 * np.pi)
        params.append((a, b, t))
    noise = rng.normal(0.0, 2.0, size=(size, size))
    m = np.arange(size, dtype=np.float64)[:, None]
    n = np.arange(size, dtype=np.float64)[None, :]
    f = 40.0 + 0.5 * m + 0.3 * n
    for a, b, t in params:
        f = f + 30.0 * np.cos(2.0 * np.pi * (a * m + b * n) + t)
    f = f + noise
    target = np.zeros((size, size), np.uint8)
    lo = (size - block) // 2
    target[lo:lo + block, lo:lo + block] = 1
    known = (1 - target).astype(np.uint8)
    return f, known, target


# ---------------------------------------------------------------------------
# Frames
# ---------------------------------------------------------------------------

def _gaussian_blur(x: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur with periodic borders (radius 4 sigma)."""
    r = int(np.ceil(4.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (t / sigma) ** 2)
    k /= k.sum()
    out = np.zeros_like(x)
    for i, ki in enumerate(k):
        out += ki * np.roll(x, i - r, axis=0)
    x = out
    out = np.zeros_like(x)
    for i, ki in enumerate(k):
        out += ki * np.roll(x, i - r, axis=1)
    return out


def frame(seed: int, height: int = 1080, width: int = 1920,
          n_cells: int = 24, n_edges: int = 200) -> np.ndarray:
    """8-bit luma frame: piecewise-smooth ramps + straight edges + texture.

    (i)   Voronoi partition with ``n_cells`` uniform seeds; each cell carries an
          affine ramp with intercept ~U[40, 215] and slopes ~U[-0.08, 0.08]/px.
    (ii)  ``n_edges`` straight edges: segment centre uniform over the frame,
          angle ~U[0, pi), length ~U[32, 480] px; s*C with C ~U[20, 120] and
          s = +-1 is added over a band of width ~U[16, 128] px on the left-hand
          side of the segment (only where the projection falls on the segment).
    (iii) Gaussian white noise blurred with sigma = 1 px, rescaled to std 8.
    The sum is clipped to [0, 255] and rounded to uint8.
    """
    s_cells, s_edges, s_tex = np.random.SeedSequence(seed).spawn(3)
    rc = np.random.default_rng(s_cells)
    cy = rc.uniform(0, height, n_cells)
    cx = rc.uniform(0, width, n_cells)
    icpt = rc.uniform(40.0, 215.0, n_cells)
    gy = rc.uniform(-0.08, 0.08, n_cells)
    gx = rc.uniform(-0.08, 0.08, n_cells)

    yy = np.arange(height, dtype=np.float64)[:, None]
    xx = np.arange(width, dtype=np.float64)[None, :]
    best = np.full((height, width), np.inf)
    owner = np.zeros((height, width), np.int32)
    for i in range(n_cells):
        d = (yy - cy[i]) ** 2 + (xx - cx[i]) ** 2
        closer = d < best
        best = np.where(closer, d, best)
        owner = np.where(closer, i, owner)
    img = icpt[owner] + gy[owner] * (yy - cy[owner]) + gx[owner] * (xx - cx[owner])

    re = np.random.default_rng(s_edges)
    for _ in range(n_edges):
        ey = re.uniform(0, height)
        ex = re.uniform(0, width)
        ang = re.uniform(0.0, np.pi)
        length = re.uniform(32.0, 480.0)
        contrast = re.uniform(20.0, 120.0)
        sign = 1.0 if re.uniform() < 0.5 else -1.0
        band = re.uniform(16.0, 128.0)
        dy, dx = np.sin(ang), np.cos(ang)          # unit direction
        ny, nx = -dx, dy                            # left-hand normal
        reach = length / 2.0 + band
        y0 = max(int(np.floor(ey - reach)), 0)
        y1 = min(int(np.ceil(ey + reach)) + 1, height)
        x0 = max(int(np.floor(ex - reach)), 0)
        x1 = min(int(np.ceil(ex + reach)) + 1, width)
        if y0 >= y1 or x0 >= x1:
            continue
        py = np.arange(y0, y1, dtype=np.float64)[:, None] - ey
        px = np.arange(x0, x1, dtype=np.float64)[None, :] - ex
        along = py * dy + px * dx
        across = py * ny + px * nx
        sel = (np.abs(along) <= length / 2.0) & (across > 0.0) & (across <= band)
        img[y0:y1, x0:x1] += sign * contrast * sel

    rt = np.random.default_rng(s_tex)
    tex = _gaussian_blur(rt.normal(0.0, 1.0, (height, width)), 1.0)
    tex *= 8.0 / tex.std()
    img = img + tex
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


# ---------------------------------------------------------------------------
# Loss maps and concealment areas
# ---------------------------------------------------------------------------

def loss_map(seed: int, mb_rows: int, mb_cols: int, fraction: float) -> np.ndarray:
    """Boolean (mb_rows, mb_cols) map with round(fraction * total) macroblocks
    lost, drawn uniformly without replacement."""
    total = mb_rows * mb_cols
    n_lost = int(round(fraction * total))
    rng = np.random.default_rng(seed)
    idx = rng.choice(total, size=n_lost, replace=False)
    lost = np.zeros(total, bool)
    lost[idx] = True
    return lost.reshape(mb_rows, mb_cols)


@dataclasses.dataclass
class Areas:
    """Concealment areas cut from a frame around lost macroblocks.

    areas[i]  float32 (A, A): frame pixels of area i; 0 where not known.
    known[i]  uint8   (A, A): 1 where the pixel is in the support area
              (inside the frame, not in any lost macroblock).
    target    uint8   (A, A): 1 on the missing block B (the centre block).
    truth[i]  float32 (A, A): frame pixels before the loss (0 outside the frame).
    origin[i] (row, col) of the area's top-left pixel in the frame.
    """
    areas: np.ndarray
    known: np.ndarray
    target: np.ndarray
    truth: np.ndarray
    origin: np.ndarray

    def __len__(self):
        return self.areas.shape[0]


def extract_areas(img: np.ndarray, lost: np.ndarray, block: int = MB,
                  support: int = SUPPORT) -> Areas:
    """Cut an area of side block + 2*support around every lost macroblock.

    Macroblock (r, c) covers frame rows block*r .. block*r+block-1 and the same
    for columns.  Pixels outside the frame and inside any lost macroblock are
    not known; the target block of each area is its centre macroblock.
    Areas are listed in row-major macroblock order.
    """
    height, width = img.shape
    side = block + 2 * support
    lost_px = np.zeros((height, width), bool)
    rows, cols = np.nonzero(lost)
    for r, c in zip(rows, cols):
        lost_px[block * r:block * r + block, block * c:block * c + block] = True
    n = len(rows)
    areas = np.zeros((n, side, side), np.float32)
    truth = np.zeros((n, side, side), np.float32)
    known = np.zeros((n, side, side), np.uint8)
    origin = np.zeros((n, 2), np.int64)
    for i, (r, c) in enumerate(zip(rows, cols)):
        y0 = block * r - support
        x0 = block * c - support
        origin[i] = (y0, x0)
        ys0, ys1 = max(y0, 0), min(y0 + side, height)
        xs0, xs1 = max(x0, 0), min(x0 + side, width)
        sub = img[ys0:ys1, xs0:xs1].astype(np.float32)
        lp = lost_px[ys0:ys1, xs0:xs1]
        oy, ox = ys0 - y0, xs0 - x0
        truth[i, oy:oy + sub.shape[0], ox:ox + sub.shape[1]] = sub
        kn = ~lp
        known[i, oy:oy + sub.shape[0], ox:ox + sub.shape[1]] = kn
        areas[i, oy:oy + sub.shape[0], ox:ox + sub.shape[1]] = np.where(kn, sub, 0.0)
    target = np.zeros((side, side), np.uint8)
    target[support:support + block, support:support + block] = 1
    return Areas(areas, known, target, truth, origin)


def frame_concealment(frame_seed: int = 0, loss_seed: int = 1,
                      height: int = 1080, width: int = 1920,
                      fraction: float = 0.10) -> Areas:
    """1080p frame with 10 % of its full 16x16 macroblocks lost.

    1080/16 = 67.5, so the grid is 120 x 67 full macroblocks; the last 8 pixel
    rows are never lost and serve only as support.  round(0.1 * 8040) = 804
    blocks are lost.
    """
    img = frame(frame_seed, height, width)
    lost = loss_map(loss_seed, height // MB, width // MB, fraction)
    return extract_areas(img, lost)


def replicate_frames(n_frames: int, frame_seed0: int = 0, loss_seed0: int = 1000,
                     height: int = 1080, width: int = 1920,
                     fraction: float = 0.10) -> Areas:
    """Concatenate the areas of ``n_frames`` independently seeded frames."""
    parts = [frame_concealment(frame_seed0 + i, loss_seed0 + i, height, width, fraction)
             for i in range(n_frames)]
    return Areas(np.concatenate([p.areas for p in parts]),
                 np.concatenate([p.known for p in parts]),
                 parts[0].target,
                 np.concatenate([p.truth for p in parts]),
                 np.concatenate([p.origin for p in parts]))


def random_tiny(seed: int, m: int, n: int, p_known: float = 0.7):
    """Tiny random area for brute-force checks: f ~ U[0, 255), a random known
    mask (at least one known sample) and its complement as the target."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 255.0, (m, n))
    known = (rng.uniform(size=(m, n)) < p_known).astype(np.uint8)
    if known.sum() == 0:
        known[0, 0] = 1
    target = (1 - known).astype(np.uint8)
    return f, known, target


# block (lost B side), support width, FFT size, iterations of the four classes
# of the mixed-size workload: 4x4 / 8x8 / 16x16 / 32x32 losses
MIXED_CLASSES = ((4, 4, 16, 32), (8, 8, 32, 64), (16, 16, 64, 200), (32, 16, 128, 300))


def mixed_blocks(frame_img: np.ndarray, pos_seed: int, block: int, support: int, n: int):
    """n lost blocks of size ``block`` at seeded positions of the frame's block
    grid, each with an area of side block + 2 * support lying fully inside the
    frame (so every area has the complement of B as support).

    Returns (areas float32 (n, A, A), target uint8 (A, A), truth float32 (n, A, A),
    origin int64 (n, 2)); areas hold the frame pixels with B zeroed."""
    height, width = frame_img.shape
    side = block + 2 * support
    rng = np.random.default_rng(pos_seed)
    # block-grid cells whose area stays inside the frame
    r_lo = -(-support // block)
    r_hi = (height - block - support) // block
    c_lo = r_lo
    c_hi = (width - block - support) // block
    rows = rng.integers(r_lo, r_hi + 1, n)
    cols = rng.integers(c_lo, c_hi + 1, n)
    target = np.zeros((side, side), np.uint8)
    target[support:support + block, support:support + block] = 1
    areas = np.zeros((n, side, side), np.float32)
    truth = np.zeros((n, side, side), np.float32)
    origin = np.zeros((n, 2), np.int64)
    for i, (r, c) in enumerate(zip(rows, cols)):
        y0, x0 = block * r - support, block * c - support
        origin[i] = (y0, x0)
        sub = frame_img[y0:y0 + side, x0:x0 + side].astype(np.float32)
        truth[i] = sub
        areas[i] = np.where(target == 1, 0.0, sub)
    return areas, target, truth, origin
