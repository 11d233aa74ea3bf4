"""Pins of the oracle's boundary and emitter cells (sections 2.4 and 2.5).

* Boundary with dt >= tau (f = 1): every intensity lands exactly on its target
  (a T_eff^4/4pi in the directions of interest, 0 elsewhere), the momentum on
  zero, and the gas loses exactly its kinetic energy (its temperature, from the
  internal energy, is unchanged).
* Boundary with f < 1 applied n times: I - I0 = (I_init - I0)(1 - f)^n and
  rho v = rho v_init (1 - f)^n (the discretised relaxation is geometric).
* Emitter at rest (Gamma = 1): I' = (I + x S)/(1 + x) with x = dt cbar rho kP;
  repeated application converges to S, and S itself is a fixed point.
* Moving emitter: the comoving equilibrium I = S / Gamma^4 is a fixed point.
* Directions outside the opening cone, unmarked cells and (for emitters) the gas
  are untouched bit for bit.
* A beam from an emitter layer past an optically thick sphere (the paper's shadow
  set-up, section 3.5) leaves a shadow: behind the sphere the radiation energy is
  below half of that in the lit band at the same height, which itself is far
  above the faint start.
"""
import numpy as np

import oracle as orc
from paper_2002_08377_amd import inputs as inp
from shadow_setup import radiation_energy, shadow_problem

PHYS = inp.Physics()


def _setup(N=6, K=24, seed=0, v=0.0):
    rng = np.random.default_rng(seed)
    dirs, W = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    mom = rho[:, None] * rng.normal(0, v, (N, 3)) if v else np.zeros((N, 3))
    T = rng.uniform(0.5, 2.0, N)
    etot = rho * PHYS.cv * T + 0.5 * np.sum(mom * mom, axis=1) / rho
    I = rng.uniform(0.01, 1.0, (N, K))
    st = orc.OState(I, np.ones(N), mom, etot)
    return dirs, rho, st, rng.uniform(0.5, 5.0, N)


def _cone(dirs, d, c):
    return dirs @ np.asarray(d) >= c


def test_boundary_full_relaxation():
    dirs, rho, st, kP = _setup(v=0.1)
    d, c, Te = np.array([0.0, 1.0, 0.0]), 0.5, 1.7
    out = orc.marked_cells(dirs, PHYS, 0.2, st, rho, kP, [1, 4], [1, 1], [Te, 0.0], [d, d], [c, c], tau=0.1)
    S = PHYS.a_rad * Te ** 4 / (4 * np.pi)
    cone = _cone(dirs, d, c)
    assert 0 < cone.sum() < dirs.shape[0]
    assert np.array_equal(out.I[1], np.where(cone, S, 0.0))
    assert np.array_equal(out.I[4], np.zeros(dirs.shape[0]))
    assert np.array_equal(out.mom[[1, 4]], np.zeros((2, 3)))
    ke = 0.5 * np.sum(st.mom ** 2, axis=1) / rho
    np.testing.assert_allclose(out.etot[[1, 4]], (st.etot - ke)[[1, 4]], rtol=1e-15)
    untouched = [0, 2, 3, 5]
    assert np.array_equal(out.I[untouched], st.I[untouched])
    assert np.array_equal(out.mom[untouched], st.mom[untouched])


def test_boundary_geometric_relaxation():
    dirs, rho, st, kP = _setup(v=0.1, seed=1)
    d, c, Te, dt, tau, n = np.array([1.0, 0.0, 0.0]), 0.3, 1.2, 0.01, 0.04, 7
    s = st
    for _ in range(n):
        s = orc.marked_cells(dirs, PHYS, dt, s, rho, kP, [2], [1], [Te], [d], [c], tau)
    f = dt / tau
    I0 = np.where(_cone(dirs, d, c), PHYS.a_rad * Te ** 4 / (4 * np.pi), 0.0)
    np.testing.assert_allclose(s.I[2] - I0, (st.I[2] - I0) * (1 - f) ** n, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(s.mom[2], st.mom[2] * (1 - f) ** n, rtol=1e-13)


def test_emitter_at_rest_closed_form_and_fixed_point():
    dirs, rho, st, kP = _setup(seed=2)
    d, c, Te, dt = np.array([0.0, 0.0, 1.0]), 0.6, 1.5, 0.003
    cone = _cone(dirs, d, c)
    assert 0 < cone.sum() < dirs.shape[0]
    out = orc.marked_cells(dirs, PHYS, dt, st, rho, kP, [3], [2], [Te], [d], [c], 1.0)
    S = PHYS.a_rad * Te ** 4 / (4 * np.pi)
    x = dt * PHYS.c_red * rho[3] * kP[3]
    np.testing.assert_allclose(out.I[3][cone], (st.I[3][cone] + x * S) / (1 + x), rtol=1e-15)
    assert np.array_equal(out.I[3][~cone], st.I[3][~cone])
    assert np.array_equal(out.etot, st.etot) and np.array_equal(out.mom, st.mom)
    s = st
    for _ in range(400):
        s = orc.marked_cells(dirs, PHYS, 0.05, s, rho, kP, [3], [2], [Te], [d], [c], 1.0)
    np.testing.assert_allclose(s.I[3][cone], S, rtol=1e-12)
    fixed = st.copy()
    fixed.I[3][cone] = S
    out = orc.marked_cells(dirs, PHYS, dt, fixed, rho, kP, [3], [2], [Te], [d], [c], 1.0)
    np.testing.assert_allclose(out.I[3], fixed.I[3], rtol=1e-15)


def test_moving_emitter_comoving_equilibrium_is_fixed_point():
    dirs, rho, st, kP = _setup(seed=3, v=3.0)
    d, c, Te = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0), 0.2, 1.1
    cone = _cone(dirs, d, c)
    v = st.mom[0] / rho[0]
    gam = 1.0 / np.sqrt(1.0 - v @ v / PHYS.c_light ** 2)
    G = gam * (1.0 - dirs @ v / PHYS.c_light)
    S = PHYS.a_rad * Te ** 4 / (4 * np.pi)
    eq = st.copy()
    eq.I[0][cone] = S / G[cone] ** 4
    out = orc.marked_cells(dirs, PHYS, 0.01, eq, rho, kP, [0], [2], [Te], [d], [c], 1.0)
    np.testing.assert_allclose(out.I[0], eq.I[0], rtol=1e-14)
    assert not np.allclose(G, 1.0)


def test_beam_casts_shadow_behind_opaque_sphere():
    p, mset, reg = shadow_problem(16, 80, 60)
    st = p.state
    cells, kinds, T, d, co = mset
    assert (p.dirs @ d[0] >= co[0]).sum() == 4
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    s = orc.OState(st.I, st.vol, st.mom, st.etot)
    for _ in range(p.steps):
        s, _ = orc.step(om, p.dirs, p.weights, p.phys, p.dt, s, st.rho, st.kP, st.kJ, st.ks)
        s = orc.marked_cells(p.dirs, p.phys, p.dt, s, st.rho, st.kP, cells, kinds, T, d, co, p.dt)
    E = radiation_energy(s.I, p.weights)
    E0 = radiation_energy(st.I, p.weights)
    shadow, lit = E[reg["shadow"]].mean(), E[reg["lit"]].mean()
    assert reg["shadow"].sum() >= 4 and reg["lit"].sum() >= 100
    assert lit > 100 * E0[reg["lit"]].mean()
    assert shadow < 0.5 * lit
