"""Step and adjoint calls captured in a HIP graph (torch.cuda.CUDAGraph over the C ABI).

Every step call only enqueues kernels on the caller's stream and never allocates or
copies (no memset nodes either), so a loop of steps can be captured once and
replayed.  Two fused steps (I -> I2 -> I, ping-pong) are captured; each replay
must equal two eager steps bit for bit, on several replays in a row, with eager
work and synchronisations between them, in both precision forms.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import DeviceProblem
from paper_2002_08377_amd import inputs as inp
from paper_2002_08377_amd import rt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_captured_steps_replay_like_eager_steps(dtype):
    p = inp.make_problem(0, n=9, K=80, steps=6)
    a = DeviceProblem(p, dtype=dtype)  # eager reference
    g = DeviceProblem(p, dtype=dtype)  # graph replays

    def two_steps(d):
        rt.step(d.mesh, d.params, d.angles, d.I, d.I2, d.vol, d.rho, d.mom, d.etot, d.kP, d.kJ, d.ks, d.T)
        rt.step(d.mesh, d.params, d.angles, d.I2, d.I, d.vol, d.rho, d.mom, d.etot, d.kP, d.kJ, d.ks, d.T)

    init = [t.clone() for t in (g.I, g.vol, g.mom, g.etot)]
    # warm-up outside the capture (first launches load the code objects), then restore the state
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        two_steps(g)
    torch.cuda.current_stream().wait_stream(side)
    for t, t0 in zip((g.I, g.vol, g.mom, g.etot), init):
        t.copy_(t0)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        two_steps(g)
    # capture records without running: the state is still the initial one
    torch.cuda.synchronize()
    assert torch.equal(g.I, init[0]) and torch.equal(g.etot, init[3])

    for rep in range(3):
        graph.replay()
        two_steps(a)
        torch.cuda.synchronize()
        assert torch.equal(g.I, a.I), rep
        assert torch.equal(g.vol, a.vol) and torch.equal(g.mom, a.mom) and torch.equal(g.etot, a.etot), rep
        assert torch.equal(g.T, a.T), rep
        # eager work between replays
        _ = (a.I * 2.0).sum().item()


@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_captured_taped_steps_and_run_adjoint_replay_like_eager(dtype):
    """Three taped steps (each output in its own buffer, with its source tape) and the run
    adjoint over them, captured in one graph.  The adjoints are re-seeded inside the graph by
    a copy and fill kernels (no memset nodes).  Every replay continues the gas trajectory, as
    the eager twin does; gradients and states must be bitwise equal on each of three replays."""
    p = inp.make_problem(2, n=8, K=24, steps=3)
    N, K = p.state.I.shape

    def make():
        d = DeviceProblem(p, dtype=dtype, flags=rt.MESH_ADJOINT)
        td = rt.torch_dtype(dtype)
        d.outs = [torch.empty((N, K), dtype=td, device="cuda") for _ in range(3)]
        d.tapes = [torch.empty((N, rt.SRC_TAPE), dtype=torch.float64, device="cuda") for _ in range(3)]
        d.lamI = torch.empty((N, K), dtype=td, device="cuda")
        d.lamE, d.lamM = torch.empty_like(d.etot), torch.empty_like(d.mom)
        d.dk = torch.empty_like(d.kP)
        d.seed = torch.as_tensor(np.random.default_rng(3).normal(size=(N, K)), device="cuda").to(td)
        return d

    def fwd_adj(d):
        cur = d.I
        for o, t in zip(d.outs, d.tapes):
            rt.step_taped(d.mesh, d.params, d.angles, cur, o, None, d.vol, d.rho, d.mom, d.etot, d.kP, d.kJ, d.ks,
                          src_tape=t)
            cur = o
        d.lamI.copy_(d.seed)
        d.lamE.zero_()
        d.lamM.zero_()
        d.dk.zero_()
        rt.step_adjoint_run(d.mesh, d.params, d.angles, d.outs, d.tapes, d.rho, d.kP, d.kJ, d.ks, d.lamI, d.lamE,
                            d.lamM, d.dk, d.dk)

    a, g = make(), make()
    init = [t.clone() for t in (g.vol, g.mom, g.etot)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fwd_adj(g)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    for t, t0 in zip((g.vol, g.mom, g.etot), init):
        t.copy_(t0)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fwd_adj(g)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        fwd_adj(a)
        torch.cuda.synchronize()
        for name in ("lamI", "lamE", "lamM", "dk", "vol", "mom", "etot"):
            assert torch.equal(getattr(g, name), getattr(a, name)), (rep, name)
        assert all(torch.equal(x, y) for x, y in zip(g.outs, a.outs)), rep
        _ = (a.lamI * 2.0).sum().item()  # eager work between replays
