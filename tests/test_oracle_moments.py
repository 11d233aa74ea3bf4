"""Pins of the oracle's per-cell angle moments (section 2.1: E_r = 4 pi J / c,
F_r = 4 pi H, P_r = 4 pi K / c, with intensities in energy-density units).

* The trace of P_r equals E_r for any field (every direction is a unit vector).
* An isotropic field on an octant-symmetric set carries no flux and the
  pressure of an ideal radiation gas, P_r = (E_r / 3) identity.
* A single beam along n_k (the free-streaming limit) has E_r = 4 pi W_k I,
  F_r = c E_r n_k and P_r = E_r n_k n_k, component by component.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2002_08377_amd import inputs as inp

C = 100.0
IDX = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]  # P_xx, P_yy, P_zz, P_xy, P_xz, P_yz


def test_trace_of_pressure_is_energy():
    dirs, W = inp.angle_set(48)
    I = np.random.default_rng(0).uniform(0.0, 2.0, (50, 48))
    m = orc.moments(dirs, W, C, I)
    assert np.allclose(m[:, 4] + m[:, 5] + m[:, 6], m[:, 0], rtol=1e-14, atol=0)


@pytest.mark.parametrize("K", [8, 24, 80])
def test_isotropic_field_is_an_ideal_radiation_gas(K):
    dirs, W = inp.angle_set(K)
    I = np.outer(np.array([0.5, 1.0, 3.0]), np.ones(K))
    m = orc.moments(dirs, W, C, I)
    E = 4.0 * np.pi * I[:, 0]
    assert np.allclose(m[:, 0], E, rtol=1e-14)
    assert np.max(np.abs(m[:, 1:4])) < 1e-13 * C * E.max()
    for c in range(3):
        assert np.allclose(m[:, 4 + c], E / 3.0, rtol=1e-14)
    assert np.max(np.abs(m[:, 7:10])) < 1e-14 * E.max()


@pytest.mark.parametrize("k", [0, 5, 17, 23])
def test_single_beam_is_free_streaming(k):
    dirs, W = inp.angle_set(24)
    I = np.zeros((1, 24))
    I[0, k] = 2.5
    m = orc.moments(dirs, W, C, I)[0]
    E = 4.0 * np.pi * W[k] * 2.5
    n = dirs[k]
    assert m[0] == pytest.approx(E, rel=1e-15)
    assert np.allclose(m[1:4], C * E * n, rtol=1e-14, atol=1e-14 * C * E)
    assert np.allclose(m[4:10], [E * n[a] * n[b] for a, b in IDX], rtol=1e-14, atol=1e-15 * E)
