"""Pins of whole oracle steps (transport then source; section 2 and section 2.3.1).

On a periodic mesh, transport conserves every angle's charge sum V I and the
source conserves E_g + (c/cbar) E_r and rho v + F_r/(c cbar) per cell, so a
whole step balances energy and momentum to roundoff once the gas is measured on
the new cell volumes (the gas is not advected over the radiation step):
  sum V' (E_g' - E_g) + (c/cbar) (sum V' E_r' - sum V E_r) = 0.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2002_08377_amd import inputs as inp


@pytest.mark.parametrize("scheme,index", [("upwind1", 0), ("plm_vl2", 1)])
def test_step_balances_energy_and_momentum(scheme, index):
    p = inp.make_problem(index, n=8, K=24, steps=3)
    st = p.state
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    s = orc.OState(st.I, st.vol, st.mom, st.etot)
    for _ in range(3):
        s1, T = orc.step(om, p.dirs, p.weights, p.phys, p.dt, s, st.rho, st.kP, st.kJ, st.ks, scheme)
        d0 = orc.diagnostics(p.dirs, p.weights, p.phys, s.I, s.vol, s.etot, s.mom)
        g0 = orc.diagnostics(p.dirs, p.weights, p.phys, s.I, s1.vol, s.etot, s.mom)
        d1 = orc.diagnostics(p.dirs, p.weights, p.phys, s1.I, s1.vol, s1.etot, s1.mom)
        dE = (d1[0] - g0[0]) + (d1[1] - d0[1])
        assert abs(dE) <= 1e-14 * (d0[0] + d0[1])
        dP = (d1[2:5] - g0[2:5]) + (d1[5:8] - d0[5:8])
        assert np.all(np.abs(dP) <= 1e-14 * (np.abs(g0[2:5]).sum() + np.abs(d0[5:8]).sum()))
        assert d1[8] > 0 and d1[9] == 0
        s = s1


def test_stationary_mesh_conserves_total_energy_over_a_run():
    p = inp.make_problem(0, n=8, K=24, steps=6)
    st = p.state
    om = orc.OracleMesh(p.mesh, np.zeros_like(st.mesh_vel))  # still mesh: volumes fixed
    s0 = orc.OState(st.I, st.vol, st.mom, st.etot)
    sS, _ = orc.run(om, p.dirs, p.weights, p.phys, p.dt, s0, st.rho, st.kP, st.kJ, st.ks, p.steps)
    d0 = orc.diagnostics(p.dirs, p.weights, p.phys, s0.I, s0.vol, s0.etot, s0.mom)
    d1 = orc.diagnostics(p.dirs, p.weights, p.phys, sS.I, sS.vol, sS.etot, sS.mom)
    assert abs((d1[0] + d1[1]) - (d0[0] + d0[1])) <= 1e-14 * (d0[0] + d0[1])
