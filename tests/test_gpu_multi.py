"""fofse_extrapolate_multi: blocks of several geometries in one call, areas at
arbitrary offsets of one packed buffer.  Every block must get exactly the
result of its geometry's own plan (the same kernels: the same bits), g must
land on the samples of B at the block's offset and nowhere else, and a few
blocks are checked against the FP64 oracle."""

import numpy as np
import pytest

from oracle.fofse_dft import fofse, selection_parity
from paper_2207_01205_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _geometries():
    geoms = []
    for (M, N, T, K, box) in ((12, 12, 16, 32, (4, 8, 4, 8)), (24, 24, 32, 64, (8, 16, 8, 16)),
                              (48, 48, 64, 120, (16, 32, 16, 32)), (37, 53, 64, 60, (5, 17, 30, 50))):
        t = np.zeros((M, N), np.uint8)
        t[box[0]:box[1], box[2]:box[3]] = 1
        geoms.append((M, N, T, K, t))
    return geoms


def test_multi_geometry_matches_per_geometry_plans():
    from paper_2207_01205_amd import fofse as F
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    img = synth.frame(41)
    geoms = _geometries()
    per = [40, 33, 600, 25]                      # the 48 x 48 class large enough for the grouped path
    gid = np.concatenate([np.full(c, g) for g, c in enumerate(per)]).astype(np.int32)
    rng.shuffle(gid)
    n = len(gid)
    # areas cut from the frame, packed with random gaps
    offs, areas, knowns, pos = [], [], [], 0
    for b in range(n):
        M, N = geoms[gid[b]][:2]
        y, x = rng.integers(0, img.shape[0] - M), rng.integers(0, img.shape[1] - N)
        areas.append(img[y:y + M, x:x + N].astype(np.float32))
        kn = (rng.uniform(size=(M, N)) < 0.92).astype(np.uint8)
        if b % 3 == 0:
            kn[:] = 1
        knowns.append(kn)
        pos += int(rng.integers(0, 7))
        offs.append(pos)
        pos += M * N
    buf = np.full(pos + 5, -7.0, np.float32)
    kbuf = np.zeros(pos + 5, np.uint8)
    for o, a, k in zip(offs, areas, knowns):
        buf[o:o + a.size] = a.reshape(-1)
        kbuf[o:o + a.size] = k.reshape(-1)
    mp = F.fofse_create_multi(geoms, 0)
    try:
        d_gid = torch.from_numpy(gid).to(dev)
        d_buf = torch.from_numpy(buf).to(dev)
        d_off = torch.from_numpy(np.array(offs, np.int64)).to(dev)
        d_kbuf = torch.from_numpy(kbuf).to(dev)
        rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
        d_out = torch.full_like(d_buf, 1234.5)
        d_st = torch.full((n,), -1, dtype=torch.int32, device=dev)
        s = torch.cuda.current_stream(dev).cuda_stream
        print(f"[gpu] multi-geometry call: {n} blocks of {len(geoms)} geometries", flush=True)
        F.fofse_extrapolate_multi(mp, n, d_gid.data_ptr(), d_buf.data_ptr(), d_off.data_ptr(), d_kbuf.data_ptr(),
                                  rg.data_ptr(), d_out.data_ptr(), d_st.data_ptr(), s)
        torch.cuda.synchronize()
        out = d_out.cpu().numpy()
        st = d_st.cpu().numpy()
        assert np.all(st == 0)
        written = np.zeros(out.size, bool)
        for g, (M, N, T, K, t) in enumerate(geoms):
            idx = np.nonzero(gid == g)[0]
            plan = F.Plan(M, N, T, K, t, device=0)
            a = torch.from_numpy(np.stack([areas[b] for b in idx])).to(dev)
            k = torch.from_numpy(np.stack([knowns[b] for b in idx])).to(dev)
            o, sel, coef, st_g = plan.extrapolate(a, rg, known=k, record=True)
            torch.cuda.synchronize()
            o = o.cpu().numpy()
            tb = np.nonzero(t.reshape(-1))[0]
            for j, b in enumerate(idx):
                got = out[offs[b] + tb]
                assert np.array_equal(got, o[j]), (g, b)
                written[offs[b] + tb] = True
            if g == 3:                           # oracle on a few blocks of the off-centre geometry
                f = np.stack([areas[b] for b in idx[:4]]).astype(np.float64)
                kn = np.stack([knowns[b] for b in idx[:4]]) * (1 - t)[None]
                ref = fofse(f, kn, T, 0.8, 0.5, K)
                ok, _ = selection_parity(sel.cpu().numpy()[:4], ref.keys, ref.margin, top_ref=ref.top)
                assert ok.all()
                assert np.abs(o[:4] - ref.g.reshape(4, -1)[:, tb]).max() <= 1e-3
        assert np.all(out[~written] == 1234.5)      # nothing outside B is touched
        # a geometry index out of range: refused, nothing written
        d_gid[3] = len(geoms)
        d_out.fill_(0.0)
        with pytest.raises(F.FofseError) as e:
            F.fofse_extrapolate_multi(mp, n, d_gid.data_ptr(), d_buf.data_ptr(), d_off.data_ptr(), 0,
                                      rg.data_ptr(), d_out.data_ptr(), 0, s)
        assert e.value.status == F.FOFSE_ERR_ARG
        torch.cuda.synchronize()
        assert float(d_out.abs().max()) == 0.0
        assert F.fofse_multi_geometry_plan(mp, 0) != 0 and F.fofse_multi_geometry_plan(mp, 9) == 0
    finally:
        F.fofse_destroy_multi(mp)
