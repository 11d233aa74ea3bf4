"""Multigroup source and steps (section 2.3, groups coupled through T only) on the
GPU against the oracle: FP64 <= 1e-12 (intensities, temperature, gas), FP32
transport <= 1e-5 on intensities; one group of weight 1 equals the grey update to
roundoff; bad group counts and the PLM scheme are refused."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_helpers import rel_err
from paper_2002_08377_amd import inputs as inp
from paper_2002_08377_amd import rt

pytestmark = pytest.mark.gpu

TOL = {rt.F64: 1e-12, rt.F32: 1e-5}


def _d(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _mg_problem(K, G=3, n=7, seed=5):
    p = inp.make_problem(0, n=n, K=K, steps=3)
    st = p.state
    rng = np.random.default_rng(seed)
    N = p.mesh.n_cells
    I = st.I[None, :, :] * rng.uniform(0.2, 1.0, (G, N, 1)) * (1 + 0.1 * rng.normal(size=(G, N, K)))
    kP = st.kP[None, :] * rng.uniform(0.1, 3.0, (G, N))
    kJ = kP * rng.uniform(0.5, 2.0, (G, N))
    ks = np.full((G, N), 0.1) * rng.uniform(0.5, 2.0, (G, 1))
    Wg = rng.uniform(0.2, 1.0, G)
    return p, np.ascontiguousarray(I), kP, kJ, ks, Wg


@pytest.mark.parametrize("adjacent", [False, True])
@pytest.mark.parametrize("K", [24, 80])
@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_source_mg_matches_oracle(dtype, K, adjacent):
    """adjacent: the angles reordered so that each antipodal pair sits side by side."""
    p, I, kP, kJ, ks, Wg = _mg_problem(K)
    if adjacent:
        perm = inp.adjacent_pair_order(K)
        p, I = inp.with_angle_order(p, perm), np.ascontiguousarray(I[:, :, perm])
        assert rt.angles_layout(p.dirs, p.weights) == rt.ANGLES_ANTIPODAL_ADJACENT
    st, ph = p.state, p.phys
    mesh = rt.Mesh.from_inputs(p.mesh, st.mesh_vel, k_max=K)
    ang = rt.AngleSet(p.dirs, p.weights)
    prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, dtype)
    td = rt.torch_dtype(dtype)
    Id = _d(I).to(td)
    mom, etot, T = _d(st.mom), _d(st.etot), torch.zeros(p.mesh.n_cells, dtype=torch.float64, device="cuda")
    rt.source_implicit_mg(mesh, prm, ang, _d(Wg), Id, _d(st.rho), mom, etot, _d(kP), _d(kJ), _d(ks), T)
    torch.cuda.synchronize()
    I_in = _d(I).to(td).double().cpu().numpy()
    Io, mo, eo, To = orc.source_mg(p.dirs, p.weights, Wg, ph, p.dt, I_in, st.rho, st.mom, st.etot, kP, kJ, ks)
    assert rel_err(Id.double().cpu().numpy(), Io) < TOL[dtype]
    if dtype == rt.F64:
        assert rel_err(T.cpu().numpy(), To) < 1e-12
        assert rel_err(etot.cpu().numpy(), eo) < 1e-12
        assert rel_err(mom.cpu().numpy(), mo) < 1e-12
    mesh.free()


@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_step_mg_matches_oracle(dtype):
    K, G = 48, 3
    p, I, kP, kJ, ks, Wg = _mg_problem(K, G)
    st, ph = p.state, p.phys
    mesh = rt.Mesh.from_inputs(p.mesh, st.mesh_vel, k_max=K)
    ang = rt.AngleSet(p.dirs, p.weights)
    prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, dtype)
    td = rt.torch_dtype(dtype)
    Ia, Ib = _d(I).to(td), torch.empty((G,) + st.I.shape, dtype=td, device="cuda")
    vol, mom, etot = _d(st.vol), _d(st.mom), _d(st.etot)
    T = torch.zeros(p.mesh.n_cells, dtype=torch.float64, device="cuda")
    for _ in range(p.steps):
        rt.step_mg(mesh, prm, ang, _d(Wg), Ia, Ib, vol, _d(st.rho), mom, etot, _d(kP), _d(kJ), _d(ks), T)
        Ia, Ib = Ib, Ia
    torch.cuda.synchronize()
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    Io, vo, mo, eo = I.copy(), st.vol.copy(), st.mom.copy(), st.etot.copy()
    for _ in range(p.steps):
        tr = [orc.step(om, p.dirs, p.weights, ph, p.dt, orc.OState(Io[j], vo, mo, eo), st.rho, kP[j], kJ[j], ks[j],
                       with_source=False)[0] for j in range(G)]
        Io = np.stack([t.I for t in tr])
        vo = tr[0].vol
        Io, mo, eo, To = orc.source_mg(p.dirs, p.weights, Wg, ph, p.dt, Io, st.rho, mo, eo, kP, kJ, ks)
    assert rel_err(Ia.double().cpu().numpy(), Io) < TOL[dtype]
    assert rel_err(vol.cpu().numpy(), vo) < 1e-14
    if dtype == rt.F64:
        assert rel_err(T.cpu().numpy(), To) < 1e-12
        assert rel_err(etot.cpu().numpy(), eo) < 1e-12
    mesh.free()


def test_one_group_equals_grey_source():
    K = 80
    p, I, kP, kJ, ks, Wg = _mg_problem(K, G=1)
    st, ph = p.state, p.phys
    mesh = rt.Mesh.from_inputs(p.mesh, st.mesh_vel, k_max=K)
    ang = rt.AngleSet(p.dirs, p.weights)
    prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, rt.F64)
    Ia, Ig = _d(I), _d(I[0])
    ma, ea, mg, eg = _d(st.mom), _d(st.etot), _d(st.mom), _d(st.etot)
    rt.source_implicit_mg(mesh, prm, ang, _d(np.ones(1)), Ia, _d(st.rho), ma, ea, _d(kP), _d(kJ), _d(ks))
    rt.source_implicit(mesh, prm, ang, Ig, _d(st.rho), mg, eg, _d(kP[0]), _d(kJ[0]), _d(ks[0]))
    torch.cuda.synchronize()
    assert rel_err(Ia[0].cpu().numpy(), Ig.cpu().numpy()) < 1e-14
    assert rel_err(ea.cpu().numpy(), eg.cpu().numpy()) < 1e-14
    mesh.free()


def test_multigroup_refuses_bad_arguments():
    K = 24
    p, I, kP, kJ, ks, Wg = _mg_problem(K, G=2)
    st, ph = p.state, p.phys
    mesh = rt.Mesh.from_inputs(p.mesh, st.mesh_vel, k_max=K, flags=rt.MESH_PLM)
    ang = rt.AngleSet(p.dirs, p.weights)
    prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, rt.F64)
    L = rt.lib()
    import ctypes
    nul = [None] * 10
    for G in (0, 17):
        rc = L.rt_source_implicit_mg(mesh.ptr, ctypes.byref(prm), ctypes.byref(ang.c), G, *nul)
        assert rc == rt.RT_EINVAL
    plm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, rt.F64, rt.PLM_VL2)
    with pytest.raises(rt.RTError) as e:
        rt.step_mg(mesh, plm, ang, _d(Wg), _d(I), torch.empty_like(_d(I)), _d(st.vol), _d(st.rho), _d(st.mom),
                   _d(st.etot), _d(kP), _d(kJ), _d(ks))
    assert e.value.code == rt.RT_EINVAL
    mesh.free()
