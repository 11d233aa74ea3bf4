"""Pins of the oracle's hand-written reverse mode (the adjoint of the radiation step).

* Transport is linear in the intensities: its reverse must be the exact
  transpose, <lam, J d> = <J^T lam, d> to roundoff.
* The source step's reverse must match complex-step derivatives of the same C
  forward code (compiled with complex arithmetic) to ~1e-13.
* Whole runs: the gradient of the emergent-flux loss with respect to the tied
  absorption opacity and the initial intensities matches complex-step
  derivatives of the full forward run and central finite differences, and is
  exactly zero outside the domain of dependence of first-order upwinding.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2002_08377_amd import inputs as inp


def _problem(n=6, K=24, steps=4, seed=0):
    p = inp.make_problem(2, n=n, K=K, steps=steps)
    st = p.state
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    u = inp.loss_face_weights(p.mesh, np.random.default_rng(seed))
    return p, om, u


def test_transport_vjp_is_transpose():
    p, om, u = _problem()
    rng = np.random.default_rng(1)
    N, K = p.state.I.shape
    dlt = rng.normal(size=(N, K))
    lam = rng.normal(size=(N, K))
    Jd, _ = orc.transport_upwind(om, p.dirs, p.phys.c_red, p.dt, dlt, p.state.vol)
    JTl = orc.transport_upwind_vjp(om, p.dirs, p.phys.c_red, p.dt, p.state.vol, lam)
    a, b = np.sum(lam * Jd), np.sum(JTl * dlt)
    assert abs(a - b) <= 1e-13 * (abs(a) + np.abs(lam * Jd).sum() * 1e-2)


@pytest.mark.parametrize("stiff", [False, True])
def test_source_vjp_matches_complex_step(stiff):
    rng = np.random.default_rng(2 + stiff)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    K, N = 24, 12
    d, w = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2, N)
    v = rng.normal(0, 5.0, (N, 3))
    mom = rho[:, None] * v
    etot = rho * phys.cv * T + 0.5 * rho * np.sum(v * v, 1)
    kP = 10 ** rng.uniform(2, 5, N) if stiff else 10 ** rng.uniform(-1, 1, N)
    kJ = kP * rng.uniform(0.5, 2, N)
    ks = rng.uniform(0, 1, N)
    I = (T ** 4 / (4 * np.pi))[:, None] * rng.uniform(0.5, 1.5, (N, K))
    dt = 2e-3
    # random output adjoints
    lI = rng.normal(size=(N, K)); lE = rng.normal(size=N); lM = rng.normal(size=(N, 3))
    gI, gE, gM, gkP, gkJ = orc.source_vjp(d, w, phys, dt, I, rho, mom, etot, kP, kJ, ks, lI, lE, lM)
    h = 1e-30
    # random input direction
    dI = rng.normal(size=(N, K)) * I; dE = rng.normal(size=N) * etot; dM = rng.normal(size=(N, 3))
    dkP = rng.normal(size=N) * kP; dkJ = rng.normal(size=N) * kJ
    I1, m1, e1, _ = orc.source(d, w, phys, dt, I + 1j * h * dI, rho, mom + 1j * h * dM, etot + 1j * h * dE,
                               kP + 1j * h * dkP, kJ + 1j * h * dkJ, ks, complex_step=True)
    lhs = np.sum(lI * I1.imag / h, axis=1) + lE * e1.imag / h + np.sum(lM * m1.imag / h, axis=1)
    rhs = np.sum(gI * dI, axis=1) + gE * dE + np.sum(gM * dM, axis=1) + gkP * dkP + gkJ * dkJ
    scale = np.abs(np.sum(np.abs(gI * dI), axis=1)) + np.abs(gE * dE) + np.abs(gkP * dkP) + np.abs(gkJ * dkJ)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale), np.max(np.abs(lhs - rhs) / scale)


def test_run_gradient_matches_complex_step_and_fd():
    p, om, u = _problem(n=6, K=24, steps=4)
    st = p.state
    s0 = orc.OState(st.I, st.vol, st.mom, st.etot)
    L, gI, gk = orc.adjoint(om, p.dirs, p.weights, p.phys, p.dt, s0, st.rho, st.kP, st.ks, p.steps, u)
    assert np.count_nonzero(gk) > 0

    def loss_cs(kap=None, I0=None):
        s = orc.OState(st.I if I0 is None else I0, st.vol, st.mom, st.etot)
        kk = st.kP if kap is None else kap
        sS, _ = orc.run(om, p.dirs, p.weights, p.phys, p.dt, s, st.rho, kk, kk, st.ks, p.steps, complex_step=True)
        return orc.flux_loss(om, p.dirs, p.weights, p.phys.c_light, sS.I, u, complex_step=True)

    h = 1e-30
    rng = np.random.default_rng(3)
    cells = np.argsort(-np.abs(gk))[:4].tolist() + rng.choice(p.mesh.n_cells, 2, replace=False).tolist()
    for c in cells:
        kap = st.kP.astype(complex).copy(); kap[c] += 1j * h * st.kP[c]
        d_cs = loss_cs(kap=kap).imag / h
        assert abs(d_cs - gk[c] * st.kP[c]) <= 1e-12 * abs(L) + 1e-11 * abs(d_cs)
    k_star = 3
    for c in cells[:3]:
        I0 = st.I.astype(complex).copy(); I0[c, k_star] += 1j * h
        d_cs = loss_cs(I0=I0).imag / h
        assert abs(d_cs - gI[c, k_star]) <= 1e-12 * np.abs(gI).max()
    # central finite differences at relative step 1e-6 (the config's recipe)
    c = cells[0]
    def loss_real(kap):
        sS, _ = orc.run(om, p.dirs, p.weights, p.phys, p.dt, s0, st.rho, kap, kap, st.ks, p.steps)
        return orc.flux_loss(om, p.dirs, p.weights, p.phys.c_light, sS.I, u)
    e = 1e-6 * st.kP[c]
    kp, km = st.kP.copy(), st.kP.copy(); kp[c] += e; km[c] -= e
    fd = (loss_real(kp) - loss_real(km)) / (2 * e)
    assert abs(fd - gk[c]) <= 1e-6 * abs(gk[c]) + 1e-9 * abs(L)


def test_gradient_zero_outside_domain_of_dependence():
    p, om, u = _problem(n=10, K=8, steps=2)
    st = p.state
    s0 = orc.OState(st.I, st.vol, st.mom, st.etot)
    L, gI, gk = orc.adjoint(om, p.dirs, p.weights, p.phys, p.dt, s0, st.rho, st.kP, st.ks, p.steps, u)
    # first-order upwinding moves information one face per step: cells farther than `steps`
    # face hops from the upwind cells of the loss faces cannot influence the loss
    N = p.mesh.n_cells
    adj = [[] for _ in range(N)]
    for a, b in p.mesh.face_cells:
        adj[a].append(b); adj[b].append(a)
    fi = np.nonzero(u)[0]
    reach = set(p.mesh.face_cells[fi].ravel().tolist())
    for _ in range(p.steps):
        reach |= {q for r in list(reach) for q in adj[r]}
    far = np.array([i for i in range(N) if i not in reach])
    assert far.size > 0
    assert np.all(gk[far] == 0.0) and np.all(gI[far] == 0.0)
    assert np.count_nonzero(gk) > 0
