"""Independent meshes stepped concurrently on two streams give, bit for bit, what they give
one after the other: every call only enqueues on the caller's stream (the current torch
stream) and keeps its scratch with its mesh, so nothing is shared between meshes.  Four
meshes (both precision forms, first-order and PLM-VL2, paired and general lane layouts)
take 6 steps each, their launches interleaved over two streams with no synchronisation
between them; then their angle moments, on the same streams."""
import pytest
import torch

from gpu_helpers import DeviceProblem
from paper_2002_08377_amd import inputs as inp
from paper_2002_08377_amd import rt

pytestmark = pytest.mark.gpu


def _cases():
    return [DeviceProblem(inp.make_problem(0, n=10, K=80, steps=1), dtype=rt.F32),
            DeviceProblem(inp.make_problem(2, n=9, K=48, steps=1), dtype=rt.F64),
            DeviceProblem(inp.make_problem(1, n=8, K=24, steps=1), dtype=rt.F32, scheme=rt.PLM_VL2),
            DeviceProblem(inp.make_problem(0, n=8, K=24, steps=1), dtype=rt.F64, scheme=rt.PLM_VL2,
                          layout=rt.ANGLES_GENERAL)]


def _moments(d):
    m = torch.empty((d.mesh.n_cells, 10), dtype=torch.float64, device="cuda")
    rt.moments(d.mesh, d.params, d.angles, d.I, m)
    return m


def test_meshes_on_two_streams_step_like_one_after_another():
    seq, con = _cases(), _cases()
    for d in seq:
        d.run_gpu(6)
    m_seq = [_moments(d) for d in seq]
    torch.cuda.synchronize()

    streams = [torch.cuda.Stream(), torch.cuda.Stream()]  # default priority
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for _ in range(6):
        for i, d in enumerate(con):
            with torch.cuda.stream(streams[i % 2]):
                d.gpu_step()
    m_con = []
    for i, d in enumerate(con):
        with torch.cuda.stream(streams[i % 2]):
            m_con.append(_moments(d))
    for s in streams:
        torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()

    for i, (a, b) in enumerate(zip(seq, con)):
        assert torch.equal(a.I, b.I), i
        assert torch.equal(a.vol, b.vol) and torch.equal(a.mom, b.mom) and torch.equal(a.etot, b.etot), i
        assert torch.equal(a.T, b.T), i
        assert torch.equal(m_seq[i], m_con[i]), i
    for d in seq + con:
        d.angles.free()
        d.mesh.free()
