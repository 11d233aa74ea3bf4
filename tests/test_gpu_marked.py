"""Boundary and emitter cells (sections 2.4-2.5) on the GPU against the oracle.

* One application to a random mixed set of boundary and emitter cells (moving
  gas, random directions, opening cosines and temperatures): FP64 <= 1e-12 on
  I, momentum and energy; FP32 intensities <= 1e-6.
* A crossing-beams set-up after the paper's (section 3.4): two columns of
  emitters along z, beaming at 45 and 135 degrees in the x-y plane, an absorbing
  layer at the top in y, near-vacuum elsewhere; 10 full steps (transport,
  source, marked cells) agree with the oracle to 1e-12 (FP64) / 1e-5 (FP32).
* The shadow set-up (section 3.5): an emitter layer beaming along +y past an
  optically thick sphere, 24^3 cells, 80 angles, 90 full steps: agrees with the
  oracle to 1e-12 (FP64) / 1e-5 (FP32), and the GPU result shows the shadow
  (behind the sphere below half the lit band's radiation energy).
* A set uploaded for another cell count is refused.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_helpers import DeviceProblem, rel_err
from paper_2002_08377_amd import inputs as inp
from paper_2002_08377_amd import rt
from shadow_setup import radiation_energy, shadow_problem

pytestmark = pytest.mark.gpu

TOL = {rt.F64: 1e-12, rt.F32: 1e-5}


def _random_set(N, rng, n=40):
    cells = rng.choice(N, n, replace=False)
    kinds = rng.choice([rt.CELL_BOUNDARY, rt.CELL_EMITTER], n)
    T = rng.uniform(0.3, 2.0, n)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    co = rng.uniform(-0.5, 0.95, n)
    co[:4] = 2.0  # no direction of interest: an absorbing boundary / an idle emitter
    return cells, kinds, T, d, co


@pytest.mark.parametrize("K", [24, 80])
@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_marked_cells_match_oracle(dtype, K):
    p = inp.make_problem(0, n=8, K=K, steps=1)
    st = p.state
    dp = DeviceProblem(p, dtype=dtype)
    rng = np.random.default_rng(11)
    cells, kinds, T, d, co = _random_set(p.mesh.n_cells, rng)
    tau = 2.5 * p.dt  # f = 0.4
    mk = rt.MarkedCells(p.mesh.n_cells, cells, kinds, T, d, co, tau)
    rt.marked_apply(dp.mesh, dp.params, dp.angles, mk, dp.I, dp.rho, dp.mom, dp.etot, dp.kP)
    torch.cuda.synchronize()
    I_in = dp.host(torch.as_tensor(st.I).to(rt.torch_dtype(dtype)))  # the oracle starts from the stored values
    ref = orc.marked_cells(p.dirs, p.phys, p.dt, orc.OState(I_in, st.vol, st.mom, st.etot), st.rho, st.kP,
                           cells, kinds, T, d, co, tau)
    assert rel_err(dp.host(dp.I), ref.I) < (1e-14 if dtype == rt.F64 else 1e-6)
    assert rel_err(dp.mom.cpu().numpy(), ref.mom) < 1e-14
    assert rel_err(dp.etot.cpu().numpy(), ref.etot) < 1e-14
    untouched = np.setdiff1d(np.arange(p.mesh.n_cells), cells)
    assert np.array_equal(dp.host(dp.I)[untouched], I_in[untouched])
    mk.free()


def _crossing_beams(n=12, K=24):
    p = inp.make_problem(0, n=n, K=K, steps=10)
    st = p.state
    N = p.mesh.n_cells
    st.kP[:] = 1e-3
    st.kJ[:] = 1e-3
    st.ks[:] = 0.0
    st.I *= 1e-3  # a faint background, so the beams dominate
    x, y = p.mesh.gen[:, 0], p.mesh.gen[:, 1]
    h = p.mesh.h
    left = np.nonzero((np.abs(x - 0.25) < 0.6 * h) & (np.abs(y - 0.2) < 0.6 * h))[0]
    right = np.nonzero((np.abs(x - 0.75) < 0.6 * h) & (np.abs(y - 0.2) < 0.6 * h))[0]
    top = np.nonzero(np.abs(y - 0.9) < 0.6 * h)[0]
    top = np.setdiff1d(top, np.concatenate([left, right]))
    cells = np.concatenate([left, right, top])
    kinds = np.array([rt.CELL_EMITTER] * (left.size + right.size) + [rt.CELL_BOUNDARY] * top.size)
    dl = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    dr = np.array([-1.0, 1.0, 0.0]) / np.sqrt(2.0)
    d = np.concatenate([np.tile(dl, (left.size, 1)), np.tile(dr, (right.size, 1)),
                        np.tile([0.0, 1.0, 0.0], (top.size, 1))])
    T = np.concatenate([np.full(left.size + right.size, 2.0), np.zeros(top.size)])
    # 0.85 selects the 4 angles of the 24-angle set nearest each beam direction (n.d = 0.862)
    co = np.concatenate([np.full(left.size + right.size, 0.85), np.full(top.size, 2.0)])
    st.kP[left] = st.kP[right] = st.kJ[left] = st.kJ[right] = 50.0  # emitters radiate through their opacity
    return p, (cells, kinds, T, d, co)


@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_crossing_beams_steps_match_oracle(dtype):
    p, mset = _crossing_beams()
    st = p.state
    cells, kinds, T, d, co = mset
    assert (kinds == rt.CELL_EMITTER).sum() >= 8 and (kinds == rt.CELL_BOUNDARY).sum() >= 100
    assert (p.dirs @ d[0] >= co[0]).sum() == 4
    tau = p.dt
    dp = DeviceProblem(p, dtype=dtype)
    mk = rt.MarkedCells(p.mesh.n_cells, *mset, tau)
    for _ in range(p.steps):
        dp.gpu_step()
        rt.marked_apply(dp.mesh, dp.params, dp.angles, mk, dp.I, dp.rho, dp.mom, dp.etot, dp.kP)
    torch.cuda.synchronize()
    s = dp.oracle_state()
    for _ in range(p.steps):
        s, _ = orc.step(dp.om, p.dirs, p.weights, p.phys, p.dt, s, st.rho, st.kP, st.kJ, st.ks)
        s = orc.marked_cells(p.dirs, p.phys, p.dt, s, st.rho, st.kP, *mset, tau)
    assert rel_err(dp.host(dp.I), s.I) < TOL[dtype]
    if dtype == rt.F64:
        assert rel_err(dp.etot.cpu().numpy(), s.etot) < 1e-12
    # the beams carry the emitted energy: far more radiation than the faint start
    E0 = 4 * np.pi * (st.I @ p.weights)
    E = 4 * np.pi * (s.I @ p.weights)
    assert np.sum(st.vol * E) > 3 * np.sum(st.vol * E0)
    mk.free()


@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_shadow_steps_match_oracle(dtype):
    p, mset, reg = shadow_problem(24, 80, 90)
    st = p.state
    cells, kinds, T, d, co = mset
    dp = DeviceProblem(p, dtype=dtype)
    mk = rt.MarkedCells(p.mesh.n_cells, *mset, p.dt)
    for _ in range(p.steps):
        dp.gpu_step()
        rt.marked_apply(dp.mesh, dp.params, dp.angles, mk, dp.I, dp.rho, dp.mom, dp.etot, dp.kP)
    torch.cuda.synchronize()
    s = dp.oracle_state()
    for _ in range(p.steps):
        s, _ = orc.step(dp.om, p.dirs, p.weights, p.phys, p.dt, s, st.rho, st.kP, st.kJ, st.ks)
        s = orc.marked_cells(p.dirs, p.phys, p.dt, s, st.rho, st.kP, *mset, p.dt)
    Ig = dp.host(dp.I)
    assert rel_err(Ig, s.I) < TOL[dtype]
    if dtype == rt.F64:
        assert rel_err(dp.etot.cpu().numpy(), s.etot) < 1e-12
    E = radiation_energy(Ig, p.weights)
    assert E[reg["shadow"]].mean() < 0.5 * E[reg["lit"]].mean()
    mk.free()


def test_marked_set_for_another_mesh_is_refused():
    p = inp.make_problem(0, n=6, K=24, steps=1)
    dp = DeviceProblem(p)
    mk = rt.MarkedCells(p.mesh.n_cells + 1, [0], [rt.CELL_BOUNDARY], [1.0], [[1.0, 0.0, 0.0]], [0.5], 1.0)
    with pytest.raises(rt.RTError) as e:
        rt.marked_apply(dp.mesh, dp.params, dp.angles, mk, dp.I, dp.rho, dp.mom, dp.etot, dp.kP)
    assert e.value.code == rt.RT_EINVAL
    mk.free()
