"""Pins of the oracle's implicit source step (section 2.3) against what the paper fixes.

* Per cell, the four-step algorithm conserves E_g + (c/cbar) E_r and
  rho v + F_r/(c cbar) exactly (eqs. 35-36 and section 2.3.1), at any stiffness.
* The eliminated temperature equation agrees with a brute-force solve of the
  full backward-Euler system (eq. 27 for every angle plus eq. 32), which pins
  the corrected form of eq. 29.
* Limits: no opacity leaves everything unchanged; pure scattering at rest has a
  closed form; radiation isotropic and thermal in the comoving frame is a fixed
  point for any gas velocity; radiation isotropic in the lab decelerates moving
  gas (drag); at rest the gas heat gain equals (c/cbar) times the radiation
  energy lost, which fixes the intensity normalisation.
* The thermal-equilibrium (section 3.1) and momentum (section 3.2) tests.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import root

import oracle as orc
from paper_2002_08377_amd import inputs as inp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            k, *v = line.split()
            vals[k] = [float(x) for x in v]
    return vals


def _cells(N, K, rng, v_scale=0.1, kappa_decades=(-1, 1), c=100.0, cv=1.5):
    d, w = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2.0, N)
    v = rng.normal(0, v_scale, (N, 3)) * c / 100.0
    ka = 10.0 ** rng.uniform(*kappa_decades, N)
    ks = 10.0 ** rng.uniform(-2, 0, N)
    I = (T ** 4 / (4 * np.pi))[:, None] * (1 + 0.3 * rng.normal(0, 1, (N, K))) ** 2
    mom = rho[:, None] * v
    etot = rho * cv * T + 0.5 * rho * np.sum(v * v, axis=1)
    return d, w, rho, T, mom, etot, ka, ks, I


def _moments(d, w, I, c):
    E = 4 * np.pi * I @ w
    F = 4 * np.pi * c * (I * w) @ d
    return E, F


@pytest.mark.parametrize("decades,vs", [((-1, 1), 0.1), ((2, 6), 0.1), ((-3, 8), 0.3)])
def test_conservation_per_cell(decades, vs):
    rng = np.random.default_rng(1)
    phys = inp.Physics(c_red=20.0, c_light=100.0)
    d, w, rho, T, mom, etot, ka, ks, I = _cells(500, 24, rng, vs, decades)
    dt = 1e-3
    I1, m1, e1, T1 = orc.source(d, w, phys, dt, I, rho, mom, etot, ka, ka, ks)
    E0, F0 = _moments(d, w, I, phys.c_light)
    E1, F1 = _moments(d, w, I1, phys.c_light)
    r = phys.c_light / phys.c_red
    tot0 = etot + r * E0
    np.testing.assert_allclose(e1 + r * E1, tot0, rtol=2e-15 * 8)
    p0 = mom + F0 / (phys.c_light * phys.c_red)
    p1 = m1 + F1 / (phys.c_light * phys.c_red)
    scale = np.abs(mom).max(axis=1, keepdims=True) + np.abs(F0).max(axis=1, keepdims=True) / (phys.c_light * phys.c_red)
    assert np.all(np.abs(p1 - p0) <= 1e-14 * scale)
    assert np.all(I1 > 0) and np.all(T1 > 0)


def _brute(d, w, phys, dt, I, rho, mom, etot, kP, kJ, ks):
    """Solve eq. 27 for every angle together with eq. 32 as one (K+1)-unknown system."""
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
        J = Wt @ In
        rk = In - Ic - y * G * (kP * a * Tq ** 4 / (4 * np.pi) + ks * J - (kJ + ks) * In)
        rT = rho * phys.cv * (Tq - Tn) - dt * c * rho * (4 * np.pi * kJ * J - kP * a * Tq ** 4)
        # each equation divided by the size of its largest term
        sT = rho * phys.cv * Tn + dt * c * rho * (4 * np.pi * kJ * abs(J) + kP * a * Tq ** 4)
        return np.concatenate([rk / (sI * (1 + y * (kJ + ks) * G)), [rT / sT]])

    sol = root(resid, np.concatenate([Ic / sI, [1.0]]), method="hybr", tol=1e-15)
    assert np.max(np.abs(resid(sol.x))) < 1e-14
    In, Tq = sol.x[:-1] * sI, sol.x[-1] * Tn
    return In / G ** 4, Tq


@pytest.mark.parametrize("K,kappa", [(8, 0.5), (24, 3.0), (24, 300.0), (48, 5e4)])
def test_elimination_matches_full_system(K, kappa):
    rng = np.random.default_rng(K)
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, T, mom, etot, ka, ks, I = _cells(6, K, rng, 0.2)
    kP = np.full(6, kappa) * rng.uniform(0.5, 2, 6)
    kJ = kP * rng.uniform(0.5, 2, 6)
    dt = 2e-3
    I1, m1, e1, T1 = orc.source(d, w, phys, dt, I, rho, mom, etot, kP, kJ, ks)
    for i in range(6):
        Ib, Tb = _brute(d, w, phys, dt, I[i], rho[i], mom[i], etot[i], kP[i], kJ[i], ks[i])
        assert abs(T1[i] - Tb) <= 1e-11 * Tb
        np.testing.assert_allclose(I1[i], Ib, rtol=1e-10)


def test_printed_jcom_form_differs():
    """The form printed as eq. 29 (no rho in the numerator, (kJ + ks) in the denominator)
    violates the per-angle update it is derived from; the derived form satisfies it."""
    rng = np.random.default_rng(3)
    K = 24
    phys = inp.Physics(c_red=30.0, c_light=100.0)
    d, w, rho, T, mom, etot, ka, ks, I = _cells(1, K, rng, 0.0)
    dt = 2e-3
    I1, m1, e1, T1 = orc.source(d, w, phys, dt, I, rho, mom, etot, ka, ka, ks)
    # v = 0: comoving = lab, W~ = W; with the oracle's T', eq. 28 must give back I' with J~ = sum W I'
    y = dt * phys.c_red * rho[0]
    chi = ka[0] + ks[0]
    B = T1[0] ** 4 / (4 * np.pi)
    J_true = w @ I1[0]
    rhs = (I[0] + y * (ka[0] * B + ks[0] * J_true)) / (1 + y * chi)
    np.testing.assert_allclose(I1[0], rhs, rtol=1e-13)
    s_I = np.sum(w * I[0] / (1 + dt * phys.c_red * chi))
    s_G = np.sum(w / (1 + dt * phys.c_red * chi))
    J_printed = (s_I + s_G * dt * phys.c_red * ka[0] * B) / (1 - dt * phys.c_red * rho[0] * chi * s_G)
    assert abs(J_printed - J_true) > 1e-3 * J_true


def test_no_opacity_changes_nothing():
    rng = np.random.default_rng(2)
    phys = inp.Physics()
    d, w, rho, T, mom, etot, ka, ks, I = _cells(50, 24, rng, 0.3)
    z = np.zeros(50)
    I1, m1, e1, T1 = orc.source(d, w, phys, 1e-2, I, rho, mom, etot, z, z, z)
    np.testing.assert_allclose(I1, I, rtol=1e-15)
    np.testing.assert_allclose(T1, T, rtol=1e-14)
    np.testing.assert_allclose(e1, etot, rtol=1e-15)
    np.testing.assert_allclose(m1, mom, rtol=0, atol=1e-16 * np.abs(mom).max())


def test_pure_scattering_at_rest():
    rng = np.random.default_rng(4)
    phys = inp.Physics(c_red=50.0, c_light=100.0)
    d, w, rho, T, mom, etot, ka, ks, I = _cells(40, 48, rng, 0.0)
    mom[:] = 0.0
    etot = rho * phys.cv * T
    z = np.zeros(40)
    dt = 3e-3
    I1, m1, e1, T1 = orc.source(d, w, phys, dt, I, rho, mom, etot, z, z, ks)
    x = (dt * phys.c_red * rho * ks)[:, None]
    J = (I @ w)[:, None]
    np.testing.assert_allclose(I1, (I + x * J) / (1 + x), rtol=1e-14)
    np.testing.assert_allclose(I1 @ w, I @ w, rtol=1e-14)
    np.testing.assert_allclose(T1, T, rtol=1e-14)


def test_comoving_equilibrium_is_fixed_point():
    rng = np.random.default_rng(5)
    phys = inp.Physics(c_red=10.0, c_light=100.0)
    K, N = 80, 30
    d, w = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2.0, N)
    v = rng.normal(0, 8.0, (N, 3))  # up to ~0.2 c
    gam = 1 / np.sqrt(1 - np.sum(v * v, 1) / phys.c_light ** 2)
    G = gam[:, None] * (1 - v @ d.T / phys.c_light)
    I = (T ** 4 / (4 * np.pi))[:, None] / G ** 4
    mom = rho[:, None] * v
    etot = rho * phys.cv * T + 0.5 * rho * np.sum(v * v, 1)
    ka = 10.0 ** rng.uniform(-2, 4, N)
    ks = rng.uniform(0, 1, N)
    I1, m1, e1, T1 = orc.source(d, w, phys, 1e-2, I, rho, mom, etot, ka, ka, ks)
    np.testing.assert_allclose(I1, I, rtol=1e-13)
    np.testing.assert_allclose(T1, T, rtol=1e-13)
    np.testing.assert_allclose(m1, mom, rtol=1e-12)
    np.testing.assert_allclose(e1, etot, rtol=1e-13)
    # the lab flux of such a field is along v: F = (4/3) E v to first order in v/c
    E, F = _moments(d, w, I, phys.c_light)
    slow = np.linalg.norm(v, axis=1) < 3.0
    np.testing.assert_allclose(F[slow] / E[slow, None], 4.0 / 3.0 * v[slow], atol=0.2 * 3.0 ** 2 / phys.c_light)


def test_radiation_drag_opposes_motion():
    phys = inp.Physics(c_red=100.0, c_light=100.0)
    K = 80
    d, w = inp.angle_set(K)
    rho = np.array([1.0]); T = np.array([1.0])
    v = np.array([[5.0, -2.0, 1.0]])
    I = np.full((1, K), 1.0 / (4 * np.pi))
    mom = rho[:, None] * v
    etot = rho * phys.cv * T + 0.5 * rho * np.sum(v * v, 1)
    k = np.array([2.0])
    I1, m1, e1, T1 = orc.source(d, w, phys, 1e-3, I, rho, mom, etot, k, k, np.array([0.5]))
    dm = m1[0] - mom[0]
    assert dm @ v[0] < 0
    assert np.linalg.norm(np.cross(dm, v[0])) < 1e-6 * np.linalg.norm(dm) * np.linalg.norm(v[0])


def test_heat_gain_equals_radiation_loss_at_rest():
    rng = np.random.default_rng(6)
    phys = inp.Physics(c_red=7.0, c_light=100.0)
    N, K = 60, 24
    d, w = inp.angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2.0, N)
    I = np.tile(rng.uniform(0.01, 1.0, (N, 1)), (1, K))  # isotropic: F stays zero, v stays zero
    mom = np.zeros((N, 3))
    etot = rho * phys.cv * T
    ka = 10.0 ** rng.uniform(-2, 5, N)
    I1, m1, e1, T1 = orc.source(d, w, phys, 1e-2, I, rho, mom, etot, ka, ka, np.full(N, 0.1))
    E0, _ = _moments(d, w, I, phys.c_light)
    E1, _ = _moments(d, w, I1, phys.c_light)
    lhs = rho * phys.cv * (T1 - T)
    rhs = phys.c_light / phys.c_red * (E0 - E1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-13 * np.abs(etot).max())
    np.testing.assert_allclose(e1 - etot, rhs, rtol=1e-13, atol=3e-14 * np.abs(etot).max())


def test_quartic_root_to_an_ulp():
    rng = np.random.default_rng(7)
    for _ in range(3000):
        A = 10.0 ** rng.uniform(-14, 14)
        B = 10.0 ** rng.uniform(-8, 8)
        C = 10.0 ** rng.uniform(-8, 8)
        T = orc.quartic_root(A, B, C)
        f = lambda t: Fraction(A) * Fraction(t) ** 4 + Fraction(B) * Fraction(t) - Fraction(C)
        lo, hi = np.nextafter(T, 0.0), np.nextafter(T, np.inf)
        lo2, hi2 = np.nextafter(lo, 0.0), np.nextafter(hi, np.inf)
        assert f(lo2) <= 0 <= f(hi2), (A, B, C, T)
    # no absorption: T = C/B exactly
    assert orc.quartic_root(0.0, 2.0, 3.0) == 1.5


def test_thermal_relaxation_closed_form():
    """Uniform isotropic radiation and gas at rest: one very long implicit step lands on the root of
    rho cv T + (c/cbar) a T^4 = rho cv T0 + (c/cbar) E_r0 (section 3.1)."""
    phys = inp.Physics(c_red=10.0, c_light=100.0)
    K = 24
    d, w = inp.angle_set(K)
    rho = np.array([0.7]); T0 = 0.4; Tr = 1.6
    I = np.full((1, K), Tr ** 4 / (4 * np.pi))
    etot = rho * phys.cv * T0
    k = np.array([3.0])
    I1, m1, e1, T1 = orc.source(d, w, phys, 1e12, I, rho, np.zeros((1, 3)), etot, k, k, np.array([0.1]))
    r = phys.c_light / phys.c_red
    rhs = rho[0] * phys.cv * T0 + r * Tr ** 4
    roots = np.roots([r, 0, 0, rho[0] * phys.cv, -rhs])
    Teq = max(z.real for z in roots if abs(z.imag) < 1e-9 and z.real > 0)
    assert abs(T1[0] - Teq) < 1e-10 * Teq
    np.testing.assert_allclose(I1[0], Teq ** 4 / (4 * np.pi), rtol=1e-10)


@pytest.mark.parametrize("kappa", [1.0, 100.0])
def test_thermal_equilibrium_cgs_matches_printed(kappa):
    g = _read_golden("thermal_equilibrium.txt")
    a = 7.5657e-15
    c = 2.99792458e10
    kB, mH = 1.380649e-16, 1.6735575e-24
    gamma = 5.0 / 3.0
    phys = inp.Physics(c_red=c, c_light=c, a_rad=a, gamma=gamma)
    cv = kB / ((gamma - 1) * mH)
    rho = np.array(g["rho_cgs"])
    K = 24
    d, w = inp.angle_set(K)
    I = np.full((1, K), a * g["T_rad_K"][0] ** 4 / (4 * np.pi))
    etot = rho * cv * g["T_gas_K"][0]

    class P:  # the gas constant of atomic hydrogen, mu = 1
        pass
    P.c_red, P.c_light, P.a_rad, P.cv = c, c, a, cv
    kap = np.array([kappa])
    t_eq = rho[0] * cv / (4 * kappa * rho[0] * c * a * 100.0 ** 3)
    T1 = None
    for _ in range(60):
        I, mom, etot, T1 = orc.source(d, w, P, 5 * t_eq, I, rho, np.zeros((1, 3)), etot, kap, kap,
                                      np.zeros(1))
    T_eq = T1[0]
    printed = g["T_eq_printed_K"][0]
    assert abs(T_eq - printed) / printed < g["rel_tol"][0]
    # and radiation has the same temperature
    Tr = (4 * np.pi * I[0].mean() / a) ** 0.25
    assert abs(Tr - T_eq) < 1e-6 * T_eq


@pytest.mark.parametrize("kappa", [1.0, 100.0])
def test_momentum_exchange_conserves_total(kappa):
    g = _read_golden("momentum_conservation.txt")
    phys = inp.Physics(c_red=100.0, c_light=100.0)
    K = 80
    d, w = inp.angle_set(K)
    N = 4
    rho = np.ones(N)
    I = np.where(d[:, 0] >= g["mu_min"][0], 1.0, 0.0)[None, :].repeat(N, 0)
    mom = np.zeros((N, 3))
    etot = rho * phys.cv * 0.5
    kap = np.full(N, kappa)
    _, F0 = _moments(d, w, I, phys.c_light)
    p0 = mom + F0 / (phys.c_light * phys.c_red)
    worst = 0.0
    for _ in range(20):
        I, mom, etot, T = orc.source(d, w, phys, 0.01, I, rho, mom, etot, kap, kap, np.zeros(N))
        _, F = _moments(d, w, I, phys.c_light)
        p = mom + F / (phys.c_light * phys.c_red)
        worst = max(worst, np.max(np.abs(p - p0)) / np.abs(p0).max())
    assert worst < 1e-13 < g["max_error_fraction_printed"][0]
    assert np.all(mom[:, 0] > 0)  # the gas was pushed along +x
