"""Oracle parity on every kernel organisation that the C ABI and the autotuner
can select, and on the FSE end point gamma = 1 (eq. 14 with the compensation
factor at 1: the uncompensated frequency selective extrapolation).

* every wavefront count of the split path the autotuner may pick, per FFT
  size (its candidate list is imported, so a new candidate is tested here);
* T = 64 areas above 48 x 48 samples (56 x 60 and 64 x 64), which the grouped
  forward, the full compensation and the grouped adjoint run with their
  larger-area instantiations, with per-block support masks;
* gamma = 1 on the DFT basis (every organisation) and on the DCT basis,
  including the nearest case to orthogonal weighting that the interface
  admits (rho_hat = 1 on a T x T area with a one-sample missing area: B
  cannot be empty, so W is T^2 delta minus one sample's spectrum).

Bars are those of the other parity tests: selections equal wherever the
oracle decides them (margin rule and rounding floor of selection_parity),
max |g_gpu - g_oracle| <= 1e-3 on matching blocks, coefficients within 1e-9
of the block's largest |c|; the adjoint within 1e-6 of the oracle adjoint.
"""

import numpy as np
import pytest

from oracle.fofse_adjoint import fofse_adjoint
from oracle.fofse_dct import fofse_dct
from oracle.fofse_dft import FLOOR, divergence_report, fofse, selection_parity, spectral_drift
from oracle.ofse_dft import ofse_full
from paper_2207_01205_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_G = 1e-3
MARGIN = 1e-6


def _put(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(torch.device("cuda", 0))


def _plan(M, N, T, K, target, path=None, waves=None, comp=None, basis=None):
    from paper_2207_01205_amd import fofse as F
    plan = F.Plan(M, N, T, K, target, device=0)
    if path is not None:
        plan.set_path({"split": F.FOFSE_PATH_SPLIT, "grouped": F.FOFSE_PATH_GROUPED}[path])
    if waves is not None:
        plan.set_waves(waves)
    if comp == "full":
        plan.set_compensation(F.FOFSE_COMP_FULL)
    if basis == "dct":
        plan.set_basis(F.FOFSE_BASIS_DCT)
    return plan


def run_gpu(plan, areas, known, rho, gamma, label):
    print(f"[gpu] {label}: n={areas.shape[0]} M={plan.M} N={plan.N} T={plan.T} K={plan.K} "
          f"rho={rho} gamma={gamma}", flush=True)
    a = _put(areas, np.float32)
    k = None if known is None else _put(known, np.uint8)
    rg = torch.tensor([rho, gamma], dtype=torch.float64, device=a.device)
    out, sel, coef, st = plan.extrapolate(a, rg, known=k, record=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), sel.cpu().numpy(), coef.cpu().numpy(), st.cpu().numpy()


def _support(areas, known, target):
    f = np.asarray(areas, dtype=np.float32).astype(np.float64)   # the exact inputs the GPU sees
    kn = (np.broadcast_to(1 - target, f.shape) if known is None else known).astype(np.uint8)
    return f, (kn * (1 - target)[None]).astype(np.uint8)


def oracle_dft(areas, known, target, T, rho, gamma, K):
    f, kn = _support(areas, known, target)
    r = fofse(f, kn, T, rho, gamma, K)
    return {"g": r.g, "keys": r.keys, "coef": r.coef, "margin": r.margin, "top": r.top, "W0": r.W0,
            "gamma": gamma}


def oracle_ofse(areas, known, target, T, rho, K, scale=1.0):
    """The OFSE oracle on the float32 inputs the GPU sees, times ``scale``."""
    f, kn = _support(areas, known, target)
    f = f * scale
    res = [ofse_full(np.where(kn[b] != 0, f[b], 0.0), kn[b], T, rho, K) for b in range(len(f))]
    return {key: np.stack([r[key] for r in res]) for key in ("g", "keys", "coef", "margin", "top")}


def ofse_rounding_spread(areas, known, target, T, rho, K, ref):
    """Per-block spread of the FP64 OFSE oracle under a rounding-level change
    of its arithmetic: the inputs scaled by alpha = 1 + 2^-30 and 1 - 3 2^-31
    (exactly homogeneous in exact arithmetic: c and g scale by alpha), results
    scaled back.  The full compensation divides by the convolution (R (*) W)[u],
    which can cancel, so on some blocks the iteration amplifies rounding far
    above FP64 resolution; two FP64 computations of such a block (the oracle and
    the GPU) can then differ by as much as this spread.  Returns (spread of c
    relative to the block's largest |c|, spread of g) per block, the larger of
    the two scalings."""
    sc = np.zeros(len(areas))
    sg = np.zeros(len(areas))
    for alpha in (1.0 + 2.0 ** -30, 1.0 - 3.0 * 2.0 ** -31):
        r = oracle_ofse(areas, known, target, T, rho, K, scale=alpha)
        same = np.all(r["keys"] == ref["keys"], axis=1)
        dc = np.abs(r["coef"] / alpha - ref["coef"]).max(axis=1) / np.abs(ref["coef"]).max(axis=1)
        dg = np.abs(r["g"] / alpha - ref["g"]).reshape(len(areas), -1).max(axis=1)
        sc = np.maximum(sc, np.where(same, dc, np.inf))
        sg = np.maximum(sg, np.where(same, dg, np.inf))
    return sc, sg


def oracle_dct(areas, known, target, T, rho, gamma, K):
    f, kn = _support(areas, known, target)
    r = fofse_dct(np.where(kn != 0, f, 0.0), kn, T, rho, gamma, K)
    return {"g": r.g, "keys": r.keys, "coef": r.coef + 0j, "margin": r.margin, "top": r.top}


def check(ref, target, out, sel, coef, st, label, min_same=None, tol_c=1e-9, tol_g=TOL_G):
    """Parity rule; returns the mask of blocks whose whole sequence matches.
    tol_c (coefficients, relative to the block's largest |c|) and tol_g may be
    per-block arrays."""
    assert np.all(st == 0), f"{label}: unexpected block status {np.unique(st)}"
    ok, div = selection_parity(sel, ref["keys"], ref["margin"], MARGIN, top_ref=ref["top"])
    bad = np.nonzero(~ok)[0]
    assert len(bad) == 0, f"{label}: selection differs before the rule allows, blocks {bad[:10]}"
    same = np.all(sel == ref["keys"], axis=1)
    tb = target.reshape(-1) == 1
    g_ref = ref["g"].reshape(ref["g"].shape[0], -1)[:, tb]
    err = np.abs(out - g_ref).max(axis=1)
    tol_g = np.broadcast_to(tol_g, err.shape)
    tol_c = np.broadcast_to(tol_c, err.shape)
    assert np.all(err[same] <= tol_g[same]), f"{label}: max |dg| {err[same].max()}"
    if same.any():
        c_gpu = coef[same][..., 0] + 1j * coef[same][..., 1]
        scale = np.maximum(np.abs(ref["coef"][same]).max(axis=1), 1e-300)
        cerr = np.abs(c_gpu - ref["coef"][same]).max(axis=1) / scale
        assert np.all(cerr <= tol_c[same]), f"{label}: coefficient error {cerr.max():.3e}"
    drift = 0.0
    if "W0" in ref:     # the constant compensation: |R_w[u]| = |c| W0 / gamma
        drift = spectral_drift(sel, coef, ref["keys"], ref["coef"], ref["W0"], ref["top"], ref["gamma"]).max()
        assert drift <= FLOOR / 2, f"{label}: |R_w[u]| differs by {drift:.3e} A0, above half the floor"
    for row in divergence_report(sel, ref["keys"], ref["margin"], ref["top"], MARGIN, limit=5):
        print(f"[gpu] {label}: diverging block {row}", flush=True)
    if min_same is not None:
        assert same.sum() >= min_same, f"{label}: only {same.sum()} of {len(same)} blocks match throughout"
    print(f"[gpu] {label}: blocks={len(same)} diverging={int(div.sum())} "
          f"max|dg|={err[same].max() if same.any() else 0:.3e} drift={drift:.2e}", flush=True)
    return same


# ---------------------------------------------------------------------------
# inputs

@pytest.fixture(scope="module")
def frame_img():
    return synth.frame(21)


def frame_blocks(img, n, side, support, seed, crop=None):
    """n lost macroblocks of a frame with areas of side 16 + 2 support, per-block
    support masks (other lost macroblocks are unknown); ``crop`` = (r0, r1, c0,
    c1) cuts a rectangular area out of each (the target moves with it)."""
    rng = np.random.default_rng(seed)
    lost = synth.loss_map(seed, img.shape[0] // 16, img.shape[1] // 16, 0.10)
    A = synth.extract_areas(img, lost, 16, support)
    idx = np.sort(rng.choice(len(A), n, replace=False))
    areas, known, target = A.areas[idx], A.known[idx], A.target
    if crop is not None:
        r0, r1, c0, c1 = crop
        areas, known, target = areas[:, r0:r1, c0:c1], known[:, r0:r1, c0:c1], target[r0:r1, c0:c1]
    return np.ascontiguousarray(areas), np.ascontiguousarray(known), np.ascontiguousarray(target)


# ---------------------------------------------------------------------------
# every split wavefront count the autotuner can pick

def _split_cases():
    from paper_2207_01205_amd.autotune import SPLIT_WAVES
    return [(T, w) for T in sorted(SPLIT_WAVES) for w in SPLIT_WAVES[T]]


# FFT size -> (lost block side, support width, K) for the split-path cases
_SPLIT_GEOM = {16: (4, 4, 32), 32: (8, 8, 64), 64: (16, 16, 200), 128: (32, 16, 300)}


@pytest.mark.parametrize("T,waves", _split_cases())
def test_split_wave_counts(frame_img, T, waves):
    """Each built wavefront count of the split path, with canonical masks on
    the mixed workload's geometry for T and with per-block masks."""
    block, support, K = _SPLIT_GEOM[T]
    n = 8 if T == 128 else 16
    areas, target, _, _ = synth.mixed_blocks(frame_img, 300 + T + waves, block, support, n)
    side = areas.shape[1]
    plan = _plan(side, side, T, K, target, path="split", waves=waves)
    out, sel, coef, st = run_gpu(plan, areas, None, 0.8, 0.5, f"split/{waves} T={T} canonical masks")
    check(oracle_dft(areas, None, target, T, 0.8, 0.5, K), target, out, sel, coef, st,
          f"split/{waves} T={T} canonical", min_same=n // 2)
    # per-block masks: random holes in the support
    rng = np.random.default_rng(T * 10 + waves)
    known = (rng.uniform(size=areas.shape) < 0.85).astype(np.uint8)
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 0.5, f"split/{waves} T={T} per-block masks")
    check(oracle_dft(areas, known, target, T, 0.8, 0.5, K), target, out, sel, coef, st,
          f"split/{waves} T={T} per-block masks", min_same=n // 2)


@pytest.mark.parametrize("K", [1, 2, 3])
def test_grouped_128_short_records(frame_img, K):
    """The grouped T = 128 forward on point-symmetric masks at K = 1, 2, 3.  Its
    block maximum goes through three 64-bit key slots in turn, each cleared one
    iteration ahead, and every work item starts from a cleared first slot; 1,200
    blocks give each workgroup two or three items, so items start after every
    residue of K mod 3."""
    block, support, _ = _SPLIT_GEOM[128]
    n = 1200
    areas, target, _, _ = synth.mixed_blocks(frame_img, 900 + K, block, support, n)
    side = areas.shape[1]
    plan = _plan(side, side, 128, K, target, path="grouped")
    plan.set_occupancy(1)
    out, sel, coef, st = run_gpu(plan, areas, None, 0.8, 0.5, f"grouped T=128 K={K}")
    check(oracle_dft(areas, None, target, 128, 0.8, 0.5, K), target, out, sel, coef, st,
          f"grouped T=128 K={K}", min_same=n // 2)


@pytest.mark.parametrize("T,occ", [(64, 1), (64, 2), (128, 1)])
def test_grouped_occupancy(frame_img, T, occ):
    """Every grouped-path grid the autotuner can pick (resident workgroups per
    compute unit) gives the oracle's result, and the same bits as the default
    grid; a count that is not built is refused."""
    from paper_2207_01205_amd import fofse as F
    block, support, K = _SPLIT_GEOM[T]
    areas, target, _, _ = synth.mixed_blocks(frame_img, 500 + T + occ, block, support, 64)
    side = areas.shape[1]
    rng = np.random.default_rng(occ)
    known = (rng.uniform(size=areas.shape) < 0.9).astype(np.uint8)
    known[::2] = 1                                   # half of the blocks share the canonical mask
    plan = _plan(side, side, T, K, target, path="grouped")
    ref_run = run_gpu(plan, areas, known, 0.8, 0.5, f"grouped T={T} default grid")
    plan.set_occupancy(occ)
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 0.5, f"grouped T={T} {occ} workgroups per CU")
    for x, y in zip(ref_run, (out, sel, coef, st)):
        assert np.array_equal(x, y)
    check(oracle_dft(areas, known, target, T, 0.8, 0.5, K), target, out, sel, coef, st,
          f"grouped T={T} occupancy {occ}", min_same=32)
    with pytest.raises(F.FofseError):
        plan.set_occupancy(3 if T == 64 else 2)


def test_autotune_cache(frame_img, tmp_path):
    """The autotuner times every candidate once, stores its choice, and a
    second call with the same key applies it without timing."""
    from paper_2207_01205_amd.autotune import autotune, candidates
    block, support, K = _SPLIT_GEOM[64]
    areas, target, _, _ = synth.mixed_blocks(frame_img, 77, block, support, 256)
    plan = _plan(48, 48, 64, 40, target)
    a = _put(areas, np.float32)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=a.device)
    cache = str(tmp_path / "autotune.json")
    print("[gpu] autotune with a cache file", flush=True)
    times, best = autotune(plan, a, rg, cache=cache)
    assert set(times) == {c[0] for c in candidates(64)} and best in times
    times2, best2 = autotune(plan, a, rg, cache=cache)
    assert times2 == {} and best2 == best
    out, sel, coef, st = run_gpu(plan, areas, None, 0.8, 0.5, f"autotuned ({best})")
    check(oracle_dft(areas, None, target, 64, 0.8, 0.5, 40), target, out, sel, coef, st,
          f"autotuned {best}", min_same=200)


# ---------------------------------------------------------------------------
# T = 64 areas larger than 48 x 48 (the larger-area kernel instantiations)

# 64 x 64: support 24 around the 16 x 16 block; 56 x 60: the same cut to an
# off-centre rectangle (B at rows 20..35, columns 22..37)
_LARGE = {"64x64": None, "56x60": (4, 60, 2, 62)}


@pytest.mark.parametrize("shape", sorted(_LARGE))
@pytest.mark.parametrize("org", ["grouped", "split", "full"])
def test_large_t64_areas_forward(frame_img, shape, org):
    areas, known, target = frame_blocks(frame_img, 40, 64, 24, 31, _LARGE[shape])
    M, N = target.shape
    K = 200 if org != "full" else 120
    tol_c, tol_g = 1e-9, TOL_G
    if org == "full":
        plan = _plan(M, N, 64, K, target, comp="full")
        ref = oracle_ofse(areas, known, target, 64, 0.8, K)
        # blocks whose full compensation amplifies rounding: the bar is ten
        # times the oracle's own rounding spread where that exceeds the default
        sc, sg = ofse_rounding_spread(areas, known, target, 64, 0.8, K, ref)
        tol_c, tol_g = np.maximum(1e-9, 10.0 * sc), np.maximum(TOL_G, 10.0 * sg)
        print(f"[gpu] full {shape}: oracle rounding spread of c up to {sc.max():.2e}, of g up to {sg.max():.2e} "
              f"({int((sc > 1e-10).sum())} blocks above 1e-10)", flush=True)
    else:
        plan = _plan(M, N, 64, K, target, path=org)
        ref = oracle_dft(areas, known, target, 64, 0.8, 0.5, K)
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 0.5, f"{org} {shape} per-block masks")
    check(ref, target, out, sel, coef, st, f"{org} {shape}", min_same=30, tol_c=tol_c, tol_g=tol_g)


@pytest.mark.parametrize("shape", sorted(_LARGE))
@pytest.mark.parametrize("path", ["grouped", "split"])
def test_large_t64_areas_adjoint(frame_img, shape, path):
    """The adjoint (grouped: the larger-area instantiation; split: one
    workgroup per block) for the GPU forward's own record, against the oracle
    adjoint of that record, on every block."""
    areas, known, target = frame_blocks(frame_img, 24, 64, 24, 37, _LARGE[shape])
    M, N = target.shape
    K = 200
    plan = _plan(M, N, 64, K, target, path=path)
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 0.5, f"{path} {shape} forward for the adjoint")
    assert np.all(st == 0)
    n, nB = len(areas), int(target.sum())
    gbar_b = np.random.default_rng(5).normal(size=(n, nB)).astype(np.float32)
    dev = torch.device("cuda", 0)
    ga, grg, gb = plan.backward(_put(areas, np.float32), torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev),
                                _put(sel, np.int32), _put(coef, np.float64), _put(gbar_b, np.float32),
                                known=_put(known, np.uint8), per_block=True)
    torch.cuda.synchronize()
    ga, grg, gb = ga.cpu().numpy(), grg.cpu().numpy(), gb.cpu().numpy()
    f, kn = _support(areas, known, target)
    tb = target.astype(bool)
    rb = np.zeros(n)
    gmb = np.zeros(n)
    for i in range(n):
        gbar = np.zeros((M, N))
        gbar[tb] = gbar_b[i]
        adj = fofse_adjoint(f[i], kn[i], 64, 0.8, 0.5, sel[i], gbar)
        scale = np.abs(adj.f_bar).max()
        assert np.abs(ga[i] - adj.f_bar).max() <= 1e-6 * scale, i
        rb[i], gmb[i] = adj.rho_bar, adj.gamma_bar
    np.testing.assert_allclose(gb[:, 0], rb, rtol=1e-6, atol=1e-9 * np.abs(rb).max())
    np.testing.assert_allclose(gb[:, 1], gmb, rtol=1e-6, atol=1e-9 * np.abs(gmb).max())
    np.testing.assert_allclose(grg, [rb.sum(), gmb.sum()], rtol=1e-6)
    print(f"[gpu] adjoint {path} {shape}: {n} blocks against the oracle adjoint of the GPU record", flush=True)


# ---------------------------------------------------------------------------
# gamma = 1: FSE (eq. 14 with the factor at its end point)

_GAMMA1_ORGS = [(16, "split", 1), (16, "split", 2), (32, "split", 2), (64, "split", 4), (64, "grouped", None),
                (128, "split", 8), (128, "grouped", None)]


@pytest.mark.parametrize("T,path,waves", _GAMMA1_ORGS)
def test_gamma_one_dft(frame_img, T, path, waves):
    block, support, K = _SPLIT_GEOM[T]
    n = 8 if T == 128 else 16
    areas, target, _, _ = synth.mixed_blocks(frame_img, 700 + T, block, support, n)
    side = areas.shape[1]
    rng = np.random.default_rng(T)
    known = (rng.uniform(size=areas.shape) < 0.9).astype(np.uint8)
    plan = _plan(side, side, T, K, target, path=path, waves=waves)
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 1.0, f"gamma 1 T={T} {path}/{waves}")
    check(oracle_dft(areas, known, target, T, 0.8, 1.0, K), target, out, sel, coef, st,
          f"gamma 1 T={T} {path}/{waves}", min_same=n // 2)


@pytest.mark.parametrize("path", ["split", "grouped"])
def test_gamma_one_frame_blocks(path):
    """FSE on the concealment workload's geometry (48 x 48, T = 64, K = 200)."""
    A = synth.frame_concealment(7, 8)
    sub = slice(0, 40)
    plan = _plan(48, 48, 64, 200, A.target, path=path)
    out, sel, coef, st = run_gpu(plan, A.areas[sub], A.known[sub], 0.8, 1.0, f"gamma 1 frame blocks {path}")
    check(oracle_dft(A.areas[sub], A.known[sub], A.target, 64, 0.8, 1.0, 200), A.target, out, sel, coef, st,
          f"gamma 1 frame blocks {path}", min_same=30)


@pytest.mark.parametrize("path", ["split", "grouped"])
def test_gamma_one_constant_areas(path):
    """A constant area at gamma = 1: the first iteration takes the DC class
    with c = the constant exactly, after which the residual is rounding noise
    (any later selection is allowed by the rule); g equals the constant on B."""
    _, _, target = synth.single_block(0, size=48, block=16)
    rng = np.random.default_rng(2)
    vals = [255.0, 3.0, 128.0, 77.5]
    f = np.stack([np.full((48, 48), v) for v in vals] * 2)
    known = (rng.uniform(size=f.shape) < 0.9).astype(np.uint8)
    plan = _plan(48, 48, 64, 50, target, path=path)
    out, sel, coef, st = run_gpu(plan, f, known, 0.8, 1.0, f"gamma 1 constant areas {path}")
    assert np.all(st == 0)
    assert np.all(sel[:, 0] == 0)
    np.testing.assert_allclose(coef[:, 0, 0], np.array(vals * 2), rtol=1e-13)
    tb = target.reshape(-1) == 1
    for i in range(len(f)):
        assert np.abs(out[i] - f[i].reshape(-1)[tb]).max() <= 1e-9 * 255
    check(oracle_dft(f, known, target, 64, 0.8, 1.0, 50), target, out, sel, coef, st,
          f"gamma 1 constant areas {path}")


@pytest.mark.parametrize("T,path", [(32, "split"), (64, "grouped"), (64, "split")])
def test_gamma_one_near_orthogonal(T, path):
    """rho_hat = 1 on a T x T area whose missing area is one sample: W is
    T^2 delta minus that sample's spectrum, so with gamma = 1 each selected
    class is removed up to the one-sample cross term, and the selections are
    those of the greedy best-K approximation of the area's DFT up to that
    perturbation.  Checked against the oracle on random areas."""
    rng = np.random.default_rng(T)
    target = np.zeros((T, T), np.uint8)
    target[T // 2, T // 2 - 1] = 1
    f = rng.uniform(0.0, 255.0, (8, T, T))
    K = 100
    plan = _plan(T, T, T, K, target, path=path)
    out, sel, coef, st = run_gpu(plan, f, None, 1.0, 1.0, f"near-orthogonal T={T} {path}")
    ref = oracle_dft(f, None, target, T, 1.0, 1.0, K)
    check(ref, target, out, sel, coef, st, f"near-orthogonal T={T} {path}", min_same=6)
    # the first selection is the largest class of the transform of f on A
    from oracle.fofse_dft import canonical_mask
    F0 = np.fft.fft2(f * (1 - target)[None])
    mag = np.where(canonical_mask(T)[None], np.abs(F0), -1.0).reshape(len(f), -1)
    assert np.array_equal(sel[:, 0], mag.argmax(axis=1))


@pytest.mark.parametrize("T", [16, 32, 64])
def test_gamma_one_dct(frame_img, T):
    """FSE with DCT basis functions: per-block masks, and the near-orthogonal
    case (rho_hat = 1 on a T x T area with one missing sample)."""
    block, support, K = _SPLIT_GEOM[T]
    n = 16
    areas, target, _, _ = synth.mixed_blocks(frame_img, 900 + T, block, support, n)
    side = areas.shape[1]
    rng = np.random.default_rng(T + 1)
    known = (rng.uniform(size=areas.shape) < 0.9).astype(np.uint8)
    plan = _plan(side, side, T, K, target, basis="dct")
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 1.0, f"DCT gamma 1 T={T}")
    check(oracle_dct(areas, known, target, T, 0.8, 1.0, K), target, out, sel, coef, st,
          f"DCT gamma 1 T={T}", min_same=n // 2)
    tgt = np.zeros((T, T), np.uint8)
    tgt[T // 2, T // 2] = 1
    f = rng.uniform(0.0, 255.0, (8, T, T))
    plan = _plan(T, T, T, 60, tgt, basis="dct")
    out, sel, coef, st = run_gpu(plan, f, None, 1.0, 1.0, f"DCT near-orthogonal T={T}")
    check(oracle_dct(f, None, tgt, T, 1.0, 1.0, 60), tgt, out, sel, coef, st,
          f"DCT near-orthogonal T={T}", min_same=6)


# ---------------------------------------------------------------------------
# the grouped T = 64 kernel's real-table iteration for point-symmetric weights

@pytest.mark.parametrize("T", [64, 128])
@pytest.mark.parametrize("M,N", [(48, 48), (49, 47), (45, 50), (64, 64), (33, 64), (50, 36)])
def test_symmetric_masks_grouped(frame_img, M, N, T):
    """Support masks symmetric about the area's centre take the grouped
    kernels' real-table iteration (its column and row wrap signs depend on the
    parities of M and N); a mask with one sample removed takes the complex
    path.  Both against the oracle, in one batch, with classes of several
    blocks, for T = 64 and T = 128."""
    rng = np.random.default_rng(M * 100 + N)
    target = np.zeros((M, N), np.uint8)
    bm, bn = (M - 16) // 2, (N - 16) // 2
    target[bm:M - bm, bn:N - bn] = 1                      # centred: symmetric
    assert np.array_equal(target, target[::-1, ::-1])
    n = 24
    y = rng.integers(0, frame_img.shape[0] - M, n)
    x = rng.integers(0, frame_img.shape[1] - N, n)
    areas = np.stack([frame_img[a:a + M, b:b + N] for a, b in zip(y, x)]).astype(np.float32)
    sym = []
    for _ in range(3):                                    # three symmetric mask classes
        kn = (rng.uniform(size=(M, N)) < 0.9).astype(np.uint8)
        sym.append(kn & kn[::-1, ::-1])
    asym = sym[0].copy()
    asym[2, 3] = 1 - asym[2, 3]                           # breaks the symmetry
    assert not np.array_equal(asym * (1 - target), (asym * (1 - target))[::-1, ::-1])
    masks = [sym[i % 3] for i in range(18)] + [asym] * 6
    known = np.stack(masks).astype(np.uint8)
    K = 150 if T == 64 else 120
    plan = _plan(M, N, T, K, target, path="grouped")
    out, sel, coef, st = run_gpu(plan, areas, known, 0.8, 0.5, f"symmetric masks {M}x{N} T={T} grouped")
    ref = oracle_dft(areas, known, target, T, 0.8, 0.5, K)
    check(ref, target, out, sel, coef, st, f"symmetric masks {M}x{N} T={T}", min_same=18)
