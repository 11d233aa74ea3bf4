"""Approximate pin of the oracle in the diffusion limit (section 3.3).

In pure scattering (absorption zero, gas at rest) with a mean free path
lambda = 1/(rho chi) well above the cell size and well below the width of the
profile, the radiation energy density diffuses with D = cbar lambda / 3.  The
1/3 is sum_k W_k n_x^2 of the angle set, which is exactly 1/3 for the
octant-symmetric sets used here.  The paper's closed-form profile is read with
L v_d = D (its v_d is not defined in the text).

First-order upwinding and the first-order time step add a diffusion error
proportional to the cell size h (the scheme is not asymptotic preserving).  The
pin is therefore a convergence statement, not a fixed tolerance.  On unjittered
periodic lattices of 16^3, 32^3 and 64^3 cells (dt = 0.3 h / cbar):

* the excess D_eff - D falls at every refinement;
* each halving of h divides the excess by 1.4 to 2.4 (first order);
* the Richardson extrapolation 2 D_eff(64) - D_eff(32) lies within 8% of D.

D_eff comes from the growth of the x-variance of E_r between two times after a
transient of ten mean free times.
"""
import numpy as np

import oracle as orc
from paper_2002_08377_amd import inputs as inp

LAM = 0.05     # mean free path (box = 1)
SIG0 = 0.08    # initial Gaussian width of E_r
BG = 1e-3      # uniform background (exactly preserved, subtracted when measuring)


def _effective_diffusion(n, K=8):
    mesh = inp.voronoi_mesh(n, jitter=0.0, rng=np.random.default_rng(0))
    N = mesh.n_cells
    dirs, W = inp.angle_set(K)
    phys = inp.Physics()
    dt = 0.3 * (1.0 / n) / phys.c_red
    x = mesh.gen[:, 0]
    E = np.exp(-0.5 * ((x - 0.5) / SIG0) ** 2) + BG
    I = np.repeat((E / (4 * np.pi))[:, None], K, axis=1)
    rho, zero, ks = np.ones(N), np.zeros(N), np.full(N, 1.0 / LAM)
    om = orc.OracleMesh(mesh, np.zeros((N, 3)))
    st = orc.OState(I, mesh.vol.copy(), np.zeros((N, 3)), np.ones(N))

    def variance(s):
        w = s.vol * (4 * np.pi * (s.I @ W) - BG)
        xm = np.sum(w * x) / np.sum(w)
        return np.sum(w * (x - xm) ** 2) / np.sum(w)

    D = phys.c_red * LAM / 3.0
    n0 = int(round(10 * LAM / phys.c_red / dt))
    n1 = int(round(0.25 * SIG0 ** 2 / D / dt))
    s, _ = orc.run(om, dirs, W, phys, dt, st, rho, zero, zero, ks, n0)
    v0 = variance(s)
    s, _ = orc.run(om, dirs, W, phys, dt, s, rho, zero, zero, ks, n1)
    return (variance(s) - v0) / (2 * n1 * dt), D


def test_diffusion_limit_converges_to_cbar_lambda_over_3():
    d16, D = _effective_diffusion(16)
    d32, _ = _effective_diffusion(32)
    d64, _ = _effective_diffusion(64)
    e16, e32, e64 = d16 - D, d32 - D, d64 - D
    assert e16 > e32 > e64 > 0
    assert 1.4 < e16 / e32 < 2.4 and 1.4 < e32 / e64 < 2.4
    assert abs((2 * d64 - d32) - D) < 0.08 * D
