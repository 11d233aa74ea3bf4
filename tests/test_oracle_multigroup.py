"""Pins of the oracle's multigroup source update (section 2.3, groups coupled
only through the temperature).

* One group of weight 1 reproduces the grey update (itself pinned against the
  paper's printed thermal equilibrium, closed forms and a brute-force solve).
* G identical groups (same opacities and intensities) with weights 1/G: every
  group gets the grey update of that intensity.
* Per cell, E_g + (4 pi c/cbar) sum_j Wg_j sum_k W_k I_jk and the momentum
  analogue are conserved to roundoff, over many decades of opacity.
* At rest, the multigroup equilibrium (gas at T, group j isotropic at
  (kP_j / kJ_j) a T^4/4pi) is a fixed point.
* The elimination agrees with a brute-force solve of the full implicit system
  (every group and angle plus the temperature: G K + 1 unknowns).
"""
import numpy as np
import pytest
from scipy.optimize import root

import oracle as orc
from paper_2002_08377_amd import inputs as inp


def _cells(N, K, G, rng, v_scale=0.1, decades=(-1, 1)):
    d, w = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2.0, N)
    v = rng.normal(0, v_scale, (N, 3))
    mom = rho[:, None] * v
    etot = rho * 1.5 * T + 0.5 * rho * np.sum(v * v, axis=1)
    I = (T ** 4 / (4 * np.pi))[None, :, None] * (1 + 0.3 * rng.normal(0, 1, (G, N, K))) ** 2
    kP = 10.0 ** rng.uniform(*decades, (G, N))
    kJ = kP * rng.uniform(0.5, 2.0, (G, N))
    ks = 10.0 ** rng.uniform(-2, 0, (G, N))
    return d, w, rho, mom, etot, I, kP, kJ, ks


def test_one_group_is_the_grey_update():
    rng = np.random.default_rng(0)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, mom, etot, I, kP, kJ, ks = _cells(50, 24, 1, rng)
    I1, m1, e1, T1 = orc.source_mg(d, w, np.ones(1), phys, 2e-3, I, rho, mom, etot, kP, kJ, ks)
    Ig, mg, eg, Tg = orc.source(d, w, phys, 2e-3, I[0], rho, mom, etot, kP[0], kJ[0], ks[0])
    np.testing.assert_allclose(I1[0], Ig, rtol=1e-13)
    np.testing.assert_allclose(T1, Tg, rtol=1e-14)
    np.testing.assert_allclose(e1, eg, rtol=1e-14)
    np.testing.assert_allclose(m1, mg, rtol=1e-12, atol=1e-14 * np.abs(mom).max())


def test_identical_groups_reduce_to_grey():
    rng = np.random.default_rng(1)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    G = 3
    d, w, rho, mom, etot, I, kP, kJ, ks = _cells(40, 24, 1, rng, decades=(-1, 3))
    Ig, mg, eg, Tg = orc.source(d, w, phys, 2e-3, I[0], rho, mom, etot, kP[0], kJ[0], ks[0])
    rep = lambda a: np.repeat(a, G, axis=0)
    I1, m1, e1, T1 = orc.source_mg(d, w, np.full(G, 1.0 / G), phys, 2e-3, rep(I), rho, mom, etot, rep(kP), rep(kJ),
                                   rep(ks))
    for j in range(G):
        np.testing.assert_allclose(I1[j], Ig, rtol=1e-12)
    np.testing.assert_allclose(T1, Tg, rtol=1e-13)
    np.testing.assert_allclose(e1, eg, rtol=1e-13)


@pytest.mark.parametrize("decades", [(-1, 1), (2, 6), (-3, 8)])
def test_conservation_per_cell(decades):
    rng = np.random.default_rng(2)
    phys = inp.Physics(c_red=20.0, c_light=100.0)
    G, K = 4, 24
    d, w, rho, mom, etot, I, kP, kJ, ks = _cells(300, K, G, rng, 0.2, decades)
    Wg = rng.uniform(0.2, 1.0, G)
    I1, m1, e1, T1 = orc.source_mg(d, w, Wg, phys, 1e-3, I, rho, mom, etot, kP, kJ, ks)
    E = lambda X: 4 * np.pi * np.einsum("j,jnk,k->n", Wg, X, w)
    F = lambda X: 4 * np.pi * phys.c_light * np.einsum("j,jnk,k,kc->nc", Wg, X, w, d)
    r = phys.c_light / phys.c_red
    np.testing.assert_allclose(e1 + r * E(I1), etot + r * E(I), rtol=2e-14)
    p0 = mom + F(I) / (phys.c_light * phys.c_red)
    p1 = m1 + F(I1) / (phys.c_light * phys.c_red)
    scale = np.abs(mom).max(axis=1, keepdims=True) + np.abs(F(I)).max(axis=1, keepdims=True) / (phys.c_light * phys.c_red)
    assert np.all(np.abs(p1 - p0) <= 1e-13 * scale)
    assert np.all(I1 > 0) and np.all(T1 > 0)


def test_equilibrium_at_rest_is_fixed_point():
    rng = np.random.default_rng(3)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    G, K, N = 3, 24, 20
    d, w, rho, mom, etot, I, kP, kJ, ks = _cells(N, K, G, rng, 0.0)
    T = (etot / (rho * phys.cv))
    I = (kP / kJ)[:, :, None] * (phys.a_rad * T ** 4 / (4 * np.pi))[None, :, None] * np.ones((G, N, K))
    I1, m1, e1, T1 = orc.source_mg(d, w, np.full(G, 0.5), phys, 0.05, I, rho, mom, etot, kP, kJ, ks)
    np.testing.assert_allclose(T1, T, rtol=1e-13)
    np.testing.assert_allclose(I1, I, rtol=1e-12)
    np.testing.assert_allclose(e1, etot, rtol=1e-13)  # (c/cbar)(E^n - E^{n+1}) rounds at ~1e-14


def _brute(d, w, Wg, phys, dt, I, rho, mom, etot, kP, kJ, ks):
    """Every group's eq. 27 for every angle with the group-summed gas equation (G K + 1 unknowns)."""
    c, cb, a = phys.c_light, phys.c_red, phys.a_rad
    G, K = I.shape
    v = mom / rho
    gam = 1.0 / np.sqrt(1.0 - v @ v / c ** 2)
    Gm = gam * (1.0 - d @ v / c)
    Ic = Gm[None, :] ** 4 * I
    Wt = w / Gm ** 2
    Wt /= Wt.sum()
    Tn = (etot - 0.5 * mom @ mom / rho) / (rho * phys.cv)
    y = dt * cb * rho
    sI = Ic.max()

    def resid(x):
        In, Tq = x[:-1].reshape(G, K) * sI, x[-1] * Tn
        J = In @ Wt
        chi = (kJ + ks)[:, None]
        rk = In - Ic - y * Gm[None, :] * ((kP * a * Tq ** 4 / (4 * np.pi))[:, None] + (ks * J)[:, None] - chi * In)
        rT = rho * phys.cv * (Tq - Tn) - dt * c * rho * np.sum(Wg * (4 * np.pi * kJ * J - kP * a * Tq ** 4))
        sT = rho * phys.cv * Tn + dt * c * rho * np.sum(Wg * (4 * np.pi * kJ * np.abs(J) + kP * a * Tq ** 4))
        return np.concatenate([(rk / (sI * (1 + y * chi * Gm[None, :]))).ravel(), [rT / sT]])

    sol = root(resid, np.concatenate([(Ic / sI).ravel(), [1.0]]), method="hybr", tol=1e-15)
    assert np.max(np.abs(resid(sol.x))) < 1e-13
    In, Tq = sol.x[:-1].reshape(G, K) * sI, sol.x[-1] * Tn
    return In / Gm[None, :] ** 4, Tq


@pytest.mark.parametrize("kappa", [0.5, 30.0, 3000.0])
def test_elimination_matches_full_system(kappa):
    rng = np.random.default_rng(int(kappa))
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    G, K, N = 3, 8, 4
    d, w, rho, mom, etot, I, kP, kJ, ks = _cells(N, K, G, rng, 0.2)
    kP = kappa * rng.uniform(0.2, 2.0, (G, N))
    kJ = kP * rng.uniform(0.5, 2.0, (G, N))
    Wg = rng.uniform(0.3, 1.0, G)
    I1, m1, e1, T1 = orc.source_mg(d, w, Wg, phys, 2e-3, I, rho, mom, etot, kP, kJ, ks)
    for i in range(N):
        Ib, Tb = _brute(d, w, Wg, phys, 2e-3, I[:, i], rho[i], mom[i], etot[i], kP[:, i], kJ[:, i], ks[:, i])
        assert abs(T1[i] - Tb) <= 1e-11 * Tb
        np.testing.assert_allclose(I1[:, i], Ib, rtol=1e-10)
