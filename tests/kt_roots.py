"""The temperature equation of the source update with power-law opacities (section 2.3,
eqs. 27-32 with kP, kJ evaluated at T^{n+1}), written independently of the oracle for
pinning which root its Newton iteration returns.

For a trial temperature T every angle's implicit update is linear in the angle's new
comoving intensity and in the mean intensity J = sum_k W~_k I_k:
    I_k (1 + y (kJ + ks) G_k) = Ic_k + y G_k (kP a T^4 / 4 pi + ks J),
so J follows from one linear equation, and the gas energy equation leaves the scalar
    f(T) = rho cv (T - T^n) - dt c rho (4 pi kJ J(T) - kP a T^4).
Its roots are the temperatures at which the whole system holds.  Here they are found by
a dense logarithmic scan for sign changes and refined by Brent's method.  Where there are
several, the one the source update is meant to take is the first met from T^n in the
direction of f's sign (f < 0 at T^n: the smallest root above it; f > 0: the largest root
below it), the root that continues T^n.
"""
import numpy as np
from scipy.optimize import brentq


def cell_terms(d, w, phys, dt, I, rho, mom, etot):
    """Boost factors, comoving intensities, normalised comoving weights, T^n and y of one cell."""
    c = phys.c_light
    v = mom / rho
    gam = 1.0 / np.sqrt(1.0 - v @ v / c ** 2)
    G = gam * (1.0 - d @ v / c)
    Wt = w / G ** 2
    Wt = Wt / Wt.sum()
    Tn = (etot - 0.5 * mom @ mom / rho) / (rho * phys.cv)
    return G, G ** 4 * I, Wt, Tn, dt * phys.c_red * rho


def scalar_f(T, d, w, phys, dt, I, rho, mom, etot, kP0, kJ0, ks, Tr, bP, bJ):
    """f at the temperatures T (any shape) and the size of its terms (same shape), for
    rounding bounds: rho cv (T + T^n) + dt c rho (4 pi kJ |J| + kP a T^4)."""
    G, Ic, Wt, Tn, y = cell_terms(d, w, phys, dt, I, rho, mom, etot)
    T = np.asarray(T, dtype=np.float64)
    t = T.reshape(-1, 1)
    kP, kJ = kP0 * (t / Tr) ** bP, kJ0 * (t / Tr) ** bJ
    A = 1.0 / (1.0 + y * (kJ + ks) * G)
    B = phys.a_rad * t ** 4 / (4.0 * np.pi)
    WAG = (Wt * A * G).sum(axis=1, keepdims=True)
    J = ((Wt * A * Ic).sum(axis=1, keepdims=True) + y * kP * B * WAG) / (1.0 - y * ks * WAG)
    c = phys.c_light
    rad = 4.0 * np.pi * kJ * J - kP * phys.a_rad * t ** 4
    f = rho * phys.cv * (t - Tn) - dt * c * rho * rad
    size = rho * phys.cv * (t + Tn) + dt * c * rho * (4.0 * np.pi * kJ * np.abs(J) + kP * phys.a_rad * t ** 4)
    return f.reshape(T.shape), size.reshape(T.shape)


def roots(args, Tn, span=1024.0, points=20001):
    """Every root of f in [T^n / span, T^n span] that the scan resolves (sign changes between
    grid points 0.07% apart at the defaults), each refined to rounding."""
    grid = Tn * np.exp(np.linspace(-np.log(span), np.log(span), points))
    f, _ = scalar_f(grid, *args)
    sc = np.nonzero(np.sign(f[:-1]) * np.sign(f[1:]) < 0)[0]
    one = lambda t: float(scalar_f(t, *args)[0])
    return [brentq(one, grid[j], grid[j + 1], xtol=1e-300, rtol=1e-15) for j in sc]


def first_root(args, Tn, rs):
    """Of the roots rs, the first met from T^n in the direction of f's sign (None if none)."""
    f0 = float(scalar_f(Tn, *args)[0])
    side = [r for r in rs if r > Tn] if f0 < 0 else [r for r in rs if r < Tn]
    return None if not side else (min(side) if f0 < 0 else max(side))


def bracket(args, Tn, limit=200):
    """The far end's search of the safeguard's reading: from T^n, double while f < 0, halve
    while f > 0.  Returns [lo, hi] from that search; the Newton phase then works in
    [T^n, hi] (f < 0 at T^n) or [lo, T^n]."""
    one = lambda t: float(scalar_f(t, *args)[0])
    lo = hi = Tn
    f0 = one(Tn)
    n = 0
    if f0 < 0.0:
        while one(hi) < 0.0 and n < limit:
            lo, hi, n = hi, 2.0 * hi, n + 1
    elif f0 > 0.0:
        while one(lo) > 0.0 and n < limit:
            hi, lo, n = lo, 0.5 * lo, n + 1
    return lo, hi


def root_error_bound(args, r, eps=1e-12):
    """Rounding bound on a computed root near r: eps times the size of f's terms over |f'(r)|."""
    h = 1e-6 * r
    fp = (float(scalar_f(r + h, *args)[0]) - float(scalar_f(r - h, *args)[0])) / (2.0 * h)
    return eps * float(scalar_f(r, *args)[1]) / abs(fp)


# Steep laws (kJ rising with a high power of T) under which a share of the cells have
# several roots within a factor 1024 of T^n: (bP, bJ, dt, opacity scale).
STEEP_LAWS = [(0.5, 6.0, 2e-3, 1.0), (0.0, 8.0, 1e-2, 1.0), (-2.0, 12.0, 1e-2, 0.1), (0.5, 20.0, 1e-2, 0.01)]


def steep_cells(N, K, rng, scale, angle_set, cv):
    """Per-cell gas and intensity states for the steep laws (T ~ 0.5-2, |v| ~ 0.2 c-units,
    intensities within ~30% of the local Planck value), opacities scaled by `scale`."""
    d, w = angle_set(K)
    rho = np.exp(rng.normal(0, 0.5, N))
    T = rng.uniform(0.5, 2.0, N)
    v = rng.normal(0, 0.2, (N, 3))
    mom = rho[:, None] * v
    etot = rho * cv * T + 0.5 * rho * np.sum(v * v, axis=1)
    I = (T ** 4 / (4 * np.pi))[:, None] * (1 + 0.3 * rng.normal(0, 1, (N, K))) ** 2
    ks = 10.0 ** rng.uniform(-2, 0, N)
    kP0 = scale * rng.uniform(0.5, 2, N)
    kJ0 = kP0 * rng.uniform(0.5, 2, N)
    return d, w, rho, mom, etot, I, kP0, kJ0, ks
