"""Pins of the oracle's source update with temperature-dependent opacities
(section 2.3: Newton-Raphson on the temperature equation).

* With constant opacities (exponents 0) the Newton path gives the grey update of
  the quartic, the paper's own check of its two methods.
* Per cell, E_g + (4 pi c/cbar) E_r and the momentum analogue are conserved.
* The result solves the full implicit system (every angle plus T, with the
  opacities evaluated at T^{n+1}) found by brute force, for exponents of either
  sign, including Kramers-like ones.  Where kJ rises steeply with T the
  temperature equation can have several roots; Newton from T^n takes the one it
  reaches, and that result is checked against every equation of the system.
* At rest, the equilibrium of the T-dependent opacities, I = (kP(T)/kJ(T)) a T^4/4pi,
  is a fixed point.
"""
import numpy as np
import pytest
from scipy.optimize import root

import kt_roots as kt
import oracle as orc
from paper_2002_08377_amd import inputs as inp


def _cells(N, K, rng, v_scale=0.1, decades=(-1, 1)):
    d, w = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2.0, N)
    v = rng.normal(0, v_scale, (N, 3))
    mom = rho[:, None] * v
    etot = rho * 1.5 * T + 0.5 * rho * np.sum(v * v, axis=1)
    I = (T ** 4 / (4 * np.pi))[:, None] * (1 + 0.3 * rng.normal(0, 1, (N, K))) ** 2
    kP0 = 10.0 ** rng.uniform(*decades, N)
    kJ0 = kP0 * rng.uniform(0.5, 2.0, N)
    ks = 10.0 ** rng.uniform(-2, 0, N)
    return d, w, rho, mom, etot, I, kP0, kJ0, ks


def test_constant_opacity_newton_equals_quartic():
    rng = np.random.default_rng(0)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, mom, etot, I, kP0, kJ0, ks = _cells(100, 24, rng, decades=(-1, 4))
    a = orc.source_kT(d, w, phys, 2e-3, I, rho, mom, etot, kP0, kJ0, ks, 1.0, 0.0, 0.0)
    b = orc.source(d, w, phys, 2e-3, I, rho, mom, etot, kP0, kJ0, ks)
    np.testing.assert_allclose(a[3], b[3], rtol=1e-13)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-12)
    # the gas energy is compared on the scale of the cell's total energy: in
    # radiation-dominated cells (c/cbar) E_r far exceeds E_g
    scale = etot + (phys.c_light / phys.c_red) * 4 * np.pi * I @ w
    assert np.all(np.abs(a[2] - b[2]) <= 1e-13 * scale)


@pytest.mark.parametrize("bP,bJ", [(1.0, 1.0), (-3.5, -3.5), (2.0, -1.0)])
def test_conservation_per_cell(bP, bJ):
    rng = np.random.default_rng(1)
    phys = inp.Physics(c_red=20.0, c_light=100.0)
    d, w, rho, mom, etot, I, kP0, kJ0, ks = _cells(200, 24, rng, 0.2, (-1, 3))
    I1, m1, e1, T1 = orc.source_kT(d, w, phys, 1e-3, I, rho, mom, etot, kP0, kJ0, ks, 1.0, bP, bJ)
    E = lambda X: 4 * np.pi * X @ w
    F = lambda X: 4 * np.pi * phys.c_light * (X * w) @ d
    r = phys.c_light / phys.c_red
    np.testing.assert_allclose(e1 + r * E(I1), etot + r * E(I), rtol=2e-14)
    p0 = mom + F(I) / (phys.c_light * phys.c_red)
    p1 = m1 + F(I1) / (phys.c_light * phys.c_red)
    scale = np.abs(mom).max(axis=1, keepdims=True) + np.abs(F(I)).max(axis=1, keepdims=True) / (phys.c_light * phys.c_red)
    assert np.all(np.abs(p1 - p0) <= 1e-13 * scale)
    assert np.all(I1 > 0) and np.all(T1 > 0)


def _brute(d, w, phys, dt, I, rho, mom, etot, kP0, kJ0, ks, Tr, bP, bJ):
    c, cb, a = phys.c_light, phys.c_red, phys.a_rad
    v = mom / rho
    gam = 1.0 / np.sqrt(1.0 - v @ v / c ** 2)
    G = gam * (1.0 - d @ v / c)
    Ic = G ** 4 * I
    Wt = w / G ** 2
    Wt /= Wt.sum()
    Tn = (etot - 0.5 * mom @ mom / rho) / (rho * phys.cv)
    y = dt * cb * rho
    sI = Ic.max()

    def resid(x):
        In, Tq = x[:-1] * sI, x[-1] * Tn
        kP, kJ = kP0 * (Tq / Tr) ** bP, kJ0 * (Tq / Tr) ** bJ
        J = Wt @ In
        rk = In - Ic - y * G * (kP * a * Tq ** 4 / (4 * np.pi) + ks * J - (kJ + ks) * In)
        rT = rho * phys.cv * (Tq - Tn) - dt * c * rho * (4 * np.pi * kJ * J - kP * a * Tq ** 4)
        sT = rho * phys.cv * Tn + dt * c * rho * (4 * np.pi * kJ * abs(J) + kP * a * Tq ** 4)
        return np.concatenate([rk / (sI * (1 + y * (kJ + ks) * G)), [rT / sT]])

    sol = root(resid, np.concatenate([Ic / sI, [1.0]]), method="hybr", tol=1e-15)
    assert np.max(np.abs(resid(sol.x))) < 1e-13
    In, Tq = sol.x[:-1] * sI, sol.x[-1] * Tn
    return In / G ** 4, Tq


@pytest.mark.parametrize("bP,bJ,kappa", [(1.0, 1.0, 3.0), (-3.5, -3.5, 30.0), (2.0, -1.0, 300.0), (0.5, 1.0, 1.0)])
def test_matches_full_system(bP, bJ, kappa):
    rng = np.random.default_rng(int(10 * kappa))
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, mom, etot, I, kP0, kJ0, ks = _cells(5, 8, rng, 0.2)
    kP0 = kappa * rng.uniform(0.5, 2, 5)
    kJ0 = kP0 * rng.uniform(0.5, 2, 5)
    I1, m1, e1, T1 = orc.source_kT(d, w, phys, 2e-3, I, rho, mom, etot, kP0, kJ0, ks, 1.3, bP, bJ)
    for i in range(5):
        Ib, Tb = _brute(d, w, phys, 2e-3, I[i], rho[i], mom[i], etot[i], kP0[i], kJ0[i], ks[i], 1.3, bP, bJ)
        assert abs(T1[i] - Tb) <= 1e-11 * Tb
        np.testing.assert_allclose(I1[i], Ib, rtol=1e-10)


def test_steep_opacity_result_solves_the_full_system():
    """With kJ rising steeply with T the temperature equation can have several roots
    (here Newton from T^n and a brute-force solve started elsewhere find different
    ones); the oracle's result must still satisfy every equation of the implicit
    system: each angle's update and the gas energy equation."""
    rng = np.random.default_rng(10)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, mom, etot, I, kP0, kJ0, ks = _cells(5, 8, rng, 0.2)
    kP0 = rng.uniform(0.5, 2, 5)
    kJ0 = kP0 * rng.uniform(0.5, 2, 5)
    Tr, bP, bJ, dt = 1.3, 0.5, 3.0, 2e-3
    I1, m1, e1, T1 = orc.source_kT(d, w, phys, dt, I, rho, mom, etot, kP0, kJ0, ks, Tr, bP, bJ)
    c, cb, a = phys.c_light, phys.c_red, phys.a_rad
    for i in range(5):
        v = mom[i] / rho[i]
        gam = 1.0 / np.sqrt(1.0 - v @ v / c ** 2)
        G = gam * (1.0 - d @ v / c)
        Wt = w / G ** 2
        Wt /= Wt.sum()
        Tn = (etot[i] - 0.5 * mom[i] @ mom[i] / rho[i]) / (rho[i] * phys.cv)
        y = dt * cb * rho[i]
        Tq = T1[i]
        kP, kJ = kP0[i] * (Tq / Tr) ** bP, kJ0[i] * (Tq / Tr) ** bJ
        In = G ** 4 * I1[i]
        J = Wt @ In
        rk = In - G ** 4 * I[i] - y * G * (kP * a * Tq ** 4 / (4 * np.pi) + ks[i] * J - (kJ + ks[i]) * In)
        assert np.max(np.abs(rk)) <= 1e-12 * np.max(np.abs(G ** 4 * I[i]) * (1 + y * (kJ + ks[i]) * G))
        rT = rho[i] * phys.cv * (Tq - Tn) - dt * c * rho[i] * (4 * np.pi * kJ * J - kP * a * Tq ** 4)
        assert abs(rT) <= 1e-12 * (rho[i] * phys.cv * Tn + dt * c * rho[i] * (4 * np.pi * kJ * J + kP * a * Tq ** 4))


def test_equilibrium_at_rest_is_fixed_point():
    rng = np.random.default_rng(3)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, mom, etot, I, kP0, kJ0, ks = _cells(30, 24, rng, 0.0)
    T = etot / (rho * phys.cv)
    Tr, bP, bJ = 1.2, -2.0, 1.0
    ratio = (kP0 * (T / Tr) ** bP) / (kJ0 * (T / Tr) ** bJ)
    I = (ratio * phys.a_rad * T ** 4 / (4 * np.pi))[:, None] * np.ones((30, 24))
    I1, m1, e1, T1 = orc.source_kT(d, w, phys, 0.05, I, rho, mom, etot, kP0, kJ0, ks, Tr, bP, bJ)
    np.testing.assert_allclose(T1, T, rtol=1e-13)
    np.testing.assert_allclose(I1, I, rtol=1e-12)



def test_steep_laws_take_the_first_root_from_Tn():
    """Which root, where there are several.  The temperature equation f(T) = 0 is written
    again with the angles eliminated in closed form (tests/kt_roots.py, which shares no code
    with the oracle); a dense scan finds all its roots within a factor 1024 of T^n.  For
    these steep laws a share of the cells have several roots, and in some of them several
    lie inside the Newton phase's bracket [T^n, hi] (or [lo, T^n]), so the bracket alone
    does not decide.  The oracle must return the first root met from T^n in the direction
    of f's sign, to within the rounding of f's terms over |f'|: a Newton iteration started
    elsewhere (at the far bracket end, or cold), a bracket searched the wrong way, or a
    step that jumps over the first root fails this."""
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    N, K, Tr = 100, 8, 1.3
    crowded = 0
    for law, (bP, bJ, dt, scale) in enumerate(kt.STEEP_LAWS):
        rng = np.random.default_rng(100 + law)
        d, w, rho, mom, etot, I, kP0, kJ0, ks = kt.steep_cells(N, K, rng, scale, inp.angle_set, phys.cv)
        I1, m1, e1, T1 = orc.source_kT(d, w, phys, dt, I, rho, mom, etot, kP0, kJ0, ks, Tr, bP, bJ)
        several = 0
        for i in range(N):
            args = (d, w, phys, dt, I[i], rho[i], mom[i], etot[i], kP0[i], kJ0[i], ks[i], Tr, bP, bJ)
            Tn = kt.cell_terms(d, w, phys, dt, I[i], rho[i], mom[i], etot[i])[3]
            rs = kt.roots(args, Tn)
            r = kt.first_root(args, Tn, rs)
            assert r is not None, (law, i, Tn, rs)
            lo, hi = kt.bracket(args, Tn)
            inside = [q for q in rs if (Tn <= q <= hi if r > Tn else lo <= q <= Tn)]
            several += len(rs) > 1
            crowded += len(inside) > 1
            assert abs(T1[i] - r) <= kt.root_error_bound(args, r), (law, i, T1[i], rs)
        # the laws are steep enough that the choice matters in a share of the cells
        assert several >= N // 10, (law, several)
    assert crowded >= 3
