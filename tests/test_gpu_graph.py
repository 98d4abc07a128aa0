"""Forward + MSE gradient + adjoint captured in one HIP graph (torch.cuda
graphs over the C ABI).  Every replay, with (rho_hat, gamma) changed in device
memory between replays and eager work in between, must give the same bits as
the same step run eagerly."""

import numpy as np
import pytest

from paper_2207_01205_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("path", ["split", "grouped"])
def test_forward_adjoint_graph_replays_match_eager(path):
    from paper_2207_01205_amd import fofse as F
    A = synth.frame_concealment(3, 4)
    n = 600
    dev = torch.device("cuda", 0)
    plan = F.Plan(48, 48, 64, 200, A.target)
    plan.set_path({"split": F.FOFSE_PATH_SPLIT, "grouped": F.FOFSE_PATH_GROUPED}[path])
    tb = A.target.reshape(-1) == 1
    a = torch.from_numpy(A.areas[:n].copy()).to(dev)
    k = torch.from_numpy(A.known[:n].copy()).to(dev)
    truth = torch.from_numpy(np.ascontiguousarray(A.truth[:n].reshape(n, -1)[:, tb])).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    out = torch.empty((n, plan.nB), dtype=torch.float32, device=dev)
    sel = torch.empty((n, plan.K), dtype=torch.int32, device=dev)
    coef = torch.empty((n, plan.K, 2), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    gout = torch.empty_like(out)
    ga = torch.empty_like(a)
    grg = torch.empty((2,), dtype=torch.float64, device=dev)
    gblk = torch.empty((n, 2), dtype=torch.float64, device=dev)

    def step():
        s = torch.cuda.current_stream(dev).cuda_stream
        F.fofse_extrapolate_batch(plan.handle, n, a.data_ptr(), k.data_ptr(), rg.data_ptr(),
                                  out.data_ptr(), sel.data_ptr(), coef.data_ptr(), st.data_ptr(), s)
        torch.sub(out, truth, out=gout)
        gout.mul_(2.0 / gout.numel())
        F.fofse_backward(plan.handle, n, a.data_ptr(), k.data_ptr(), rg.data_ptr(), sel.data_ptr(),
                         coef.data_ptr(), gout.data_ptr(), ga.data_ptr(), grg.data_ptr(),
                         gblk.data_ptr(), s)

    def snapshot():
        return [t.detach().cpu().numpy().copy() for t in (out, sel, coef, st, ga, grg, gblk)]

    print(f"[gpu] graph capture: {path} path, {n} blocks", flush=True)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        step()                     # plan workspaces allocated before capture
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rho, gamma in [(0.8, 0.5), (0.7, 0.3), (0.9, 0.6), (0.8, 0.5)]:
        rg.copy_(torch.tensor([rho, gamma], dtype=torch.float64))
        graph.replay()
        torch.cuda.synchronize()
        replayed = snapshot()
        junk = torch.randn(1 << 20, device=dev).sum()       # eager work between replays
        for t in (out, ga, grg, gblk):
            t.fill_(-1)
        step()
        torch.cuda.synchronize()
        eager = snapshot()
        for x, y, name in zip(replayed, eager, ("out", "sel", "coef", "status", "dL/df", "dL/drg", "blocks")):
            assert np.array_equal(x, y), f"replay differs from eager in {name} at rho={rho} gamma={gamma}"
        assert np.all(eager[3] == 0) and np.isfinite(eager[5]).all()
        print(f"[gpu] replay rho={rho} gamma={gamma}: dL/drho={eager[5][0]:.6e} dL/dgamma={eager[5][1]:.6e}",
              flush=True)
        del junk


def test_dct_basis_graph_replays_match_eager():
    """The DCT-basis forward (grouping kernels and the DCT kernel) captured in
    one graph: every replay, with (rho_hat, gamma) changed in device memory and
    eager work in between, gives the same bits as the eager call."""
    from paper_2207_01205_amd import fofse as F
    A = synth.frame_concealment(3, 4)
    n = 400
    dev = torch.device("cuda", 0)
    plan = F.Plan(48, 48, 64, 120, A.target)
    plan.set_basis(F.FOFSE_BASIS_DCT)
    a = torch.from_numpy(A.areas[:n].copy()).to(dev)
    k = torch.from_numpy(A.known[:n].copy()).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    out = torch.empty((n, plan.nB), dtype=torch.float32, device=dev)
    sel = torch.empty((n, plan.K), dtype=torch.int32, device=dev)
    coef = torch.empty((n, plan.K, 2), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)

    def step():
        F.fofse_extrapolate_batch(plan.handle, n, a.data_ptr(), k.data_ptr(), rg.data_ptr(), out.data_ptr(),
                                  sel.data_ptr(), coef.data_ptr(), st.data_ptr(),
                                  torch.cuda.current_stream(dev).cuda_stream)

    def snapshot():
        return [t.detach().cpu().numpy().copy() for t in (out, sel, coef, st)]

    print(f"[gpu] graph capture: DCT basis, {n} blocks", flush=True)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        step()                     # plan workspaces allocated before capture
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rho, gamma in [(0.8, 0.5), (0.7, 0.3), (0.8, 0.5)]:
        rg.copy_(torch.tensor([rho, gamma], dtype=torch.float64))
        graph.replay()
        torch.cuda.synchronize()
        replayed = snapshot()
        junk = torch.randn(1 << 20, device=dev).sum()       # eager work between replays
        out.fill_(-1)
        step()
        torch.cuda.synchronize()
        eager = snapshot()
        for x, y, name in zip(replayed, eager, ("out", "sel", "coef", "status")):
            assert np.array_equal(x, y), f"replay differs from eager in {name} at rho={rho} gamma={gamma}"
        assert np.all(eager[3] == 0)
        del junk


def test_plan_buffers_survive_growth_after_capture():
    """A graph captured at one batch size keeps working after an eager call
    with a larger batch grows the plan's buffers (the replaced buffers stay
    allocated); a captured call that would have to grow a buffer is refused
    instead of allocating under capture."""
    from paper_2207_01205_amd import fofse as F
    A = synth.frame_concealment(8, 9)
    dev = torch.device("cuda", 0)
    plan = F.Plan(48, 48, 64, 60, A.target)
    plan.set_path(F.FOFSE_PATH_GROUPED)
    a = torch.from_numpy(A.areas[:600].copy()).to(dev)
    k = torch.from_numpy(A.known[:600].copy()).to(dev)
    rg = torch.tensor([0.8, 0.5], dtype=torch.float64, device=dev)
    out = torch.empty((600, plan.nB), dtype=torch.float32, device=dev)

    def call(n, s):
        # no record: the plan's own record and grouping workspace are used
        F.fofse_extrapolate_batch(plan.handle, n, a.data_ptr(), k.data_ptr(), rg.data_ptr(),
                                  out.data_ptr(), 0, 0, 0, s)

    print("[gpu] capture, then growth of the plan's buffers", flush=True)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        call(40, side.cuda_stream)
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    eager40 = out[:40].clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call(40, torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    call(600, torch.cuda.current_stream(dev).cuda_stream)      # grows record and workspace
    torch.cuda.synchronize()
    eager600 = out.clone()
    for _ in range(3):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[:40], eager40)
    assert torch.equal(eager600[:40], eager40)
    del graph
    # growth needed under capture: refused, nothing enqueued
    plan2 = F.Plan(48, 48, 64, 60, A.target)
    plan2.set_path(F.FOFSE_PATH_GROUPED)
    g2 = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g2):
        try:
            F.fofse_extrapolate_batch(plan2.handle, 40, a.data_ptr(), k.data_ptr(), rg.data_ptr(),
                                      out.data_ptr(), 0, 0, 0, torch.cuda.current_stream(dev).cuda_stream)
        except F.FofseError as e:
            err = e
    torch.cuda.synchronize()
    assert err is not None and err.status == F.FOFSE_ERR_UNSUPPORTED
    del g2
