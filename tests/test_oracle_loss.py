"""Pins of the oracle's emergent-flux loss, the objective of the adjoint workloads.

The loss sums, over the faces whose generator pair straddles the plane x = 1/2, a signed
weight u_f times the radiative flux through the face, A_f F_r . n_f, with
F_r = 4 pi c sum_k W_k n_k I_k (section 2.1, the flux moment in energy-density units), each
angle taking the intensity of its upwind cell (the cell that angle leaves through the
face).  What fixes its value independently of the code:

* the plane faces tile a surface that separates the periodic box into two slabs, so
  sum_f (orientation) A_f n_f is the cross-section (1, 0, 0);
* a field that is the same in every cell has no upwind choice: the loss is the flux moment
  of the pinned angle-moment routine dotted into each face;
* on an unjittered lattice with the left slab filled isotropically and the right slab
  empty, the emergent flux through the plane is the half-range moment of the angle set,
  4 pi c sum_k W_k max(0, n_k,x), and zero in the other direction;
* a one-cell indicator field contributes only through the angles leaving that cell;
* the loss is linear in I, so it equals the inner product of I with its seed dL/dI.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2002_08377_amd import inputs as inp

FOURPI = 4.0 * np.pi


def _setup(n=8, K=24, jitter=0.2, seed=41):
    m = inp.voronoi_mesh(n, jitter, seed=seed)
    d, w = inp.angle_set(K)
    om = orc.OracleMesh(m, np.zeros((m.n_cells, 3)))
    ids, sign = inp.plane_faces(m)
    unit = np.zeros(m.n_faces)
    unit[ids] = sign
    return m, d, w, om, ids, sign, unit


def test_plane_faces_span_the_cross_section():
    m, d, w, om, ids, sign, unit = _setup()
    S = np.sum((sign * m.face_area[ids])[:, None] * m.face_normal[ids], axis=0)
    np.testing.assert_allclose(S, [m.box ** 2, 0.0, 0.0], atol=1e-14)


@pytest.mark.parametrize("c_light", [100.0, 7.0])
def test_uniform_beam_through_the_plane(c_light):
    """One angle populated identically in every cell: the loss with unit weights is the flux
    of that beam through the unit cross-section, 4 pi c W_k n_k,x."""
    m, d, w, om, ids, sign, unit = _setup()
    N, K = m.n_cells, d.shape[0]
    for k in range(K):
        I = np.zeros((N, K))
        I[:, k] = 1.0
        L = orc.flux_loss(om, d, w, c_light, I, unit)
        assert abs(L - FOURPI * c_light * w[k] * d[k, 0]) <= 1e-13 * FOURPI * c_light * w[k]


def test_uniform_field_random_weights_is_the_flux_moment():
    """A cell-uniform field with random weights: sum_f u_f A_f n_f . F_r, with F_r from the
    angle-moment routine (pinned by its own identities)."""
    m, d, w, om, ids, sign, unit = _setup()
    N, K = m.n_cells, d.shape[0]
    rng = np.random.default_rng(42)
    u = inp.loss_face_weights(m, rng)
    I = np.tile(rng.uniform(0.2, 3.0, size=K), (N, 1))
    Fr = orc.moments(d, w, 100.0, I[:1])[0, 1:4]
    expect = np.sum(u[ids] * m.face_area[ids] * (m.face_normal[ids] @ Fr))
    L = orc.flux_loss(om, d, w, 100.0, I, u)
    assert abs(L - expect) <= 1e-13 * np.sum(np.abs(u[ids]) * m.face_area[ids]) * np.abs(Fr).max()


@pytest.mark.parametrize("K", [8, 24, 80])
def test_half_space_emergent_flux_on_a_lattice(K):
    """Unjittered lattice, left slab (generators at x < 1/2) isotropic with I = 1, right slab
    empty: every plane face has normal +x and area h^2, and only the angles leaving the left
    slab see a filled upwind cell, so L = 4 pi c sum_k W_k max(0, n_k,x).  Reversed fill
    (right slab full) gives the mirror image -4 pi c sum_k W_k max(0, -n_k,x)."""
    m, d, w, om, ids, sign, unit = _setup(n=8, K=K, jitter=0.0)
    N = m.n_cells
    left = m.gen[:, 0] < 0.5
    c = 100.0
    I = np.where(left[:, None], 1.0, 0.0) * np.ones((N, K))
    L = orc.flux_loss(om, d, w, c, I, unit)
    half = np.sum(w * np.maximum(0.0, d[:, 0]))
    assert abs(L - FOURPI * c * half) <= 1e-13 * FOURPI * c
    L2 = orc.flux_loss(om, d, w, c, 1.0 - I, unit)
    assert abs(L2 + FOURPI * c * np.sum(w * np.maximum(0.0, -d[:, 0]))) <= 1e-13 * FOURPI * c
    # the discrete half-range moment approximates the continuum value 1/4 (emergent flux pi I)
    assert abs(half - 0.25) < 0.05


def test_one_cell_indicator_only_outgoing_angles():
    """I = 1 in one cell (every angle), 0 elsewhere: a plane face of that cell contributes
    u_f A_f 4 pi c W_k (n_k . n_f) for exactly the angles whose direction leaves the cell
    through it (n_k . n_out > 0, n_out the face normal pointing away from the cell)."""
    m, d, w, om, ids, sign, unit = _setup()
    N, K = m.n_cells, d.shape[0]
    rng = np.random.default_rng(43)
    u = inp.loss_face_weights(m, rng)
    touching = np.unique(m.face_cells[ids].ravel())
    for c in rng.choice(touching, size=6, replace=False):
        I = np.zeros((N, K))
        I[c] = 1.0
        expect = 0.0
        for f in ids:
            a, b = m.face_cells[f]
            if c not in (a, b):
                continue
            n_out = m.face_normal[f] if c == a else -m.face_normal[f]
            mu = d @ m.face_normal[f]
            leaving = d @ n_out > 0.0
            expect += u[f] * m.face_area[f] * FOURPI * 100.0 * np.sum(w[leaving] * mu[leaving])
        L = orc.flux_loss(om, d, w, 100.0, I, u)
        assert expect != 0.0
        assert abs(L - expect) <= 1e-13 * FOURPI * 100.0 * np.abs(u).max() * m.face_area.max()


def test_loss_is_the_seed_inner_product():
    """The loss is linear in I: L(I) = <dL/dI, I> for any field, and the seed holds one
    entry per plane face and angle (the upwind cell's)."""
    m, d, w, om, ids, sign, unit = _setup()
    N, K = m.n_cells, d.shape[0]
    rng = np.random.default_rng(44)
    u = inp.loss_face_weights(m, rng)
    _, seed = orc.flux_loss(om, d, w, 100.0, np.zeros((N, K)), u, want_seed=True)
    for _ in range(3):
        I = rng.uniform(0.0, 2.0, size=(N, K))
        L = orc.flux_loss(om, d, w, 100.0, I, u)
        assert abs(L - np.sum(seed * I)) <= 1e-13 * np.sum(np.abs(seed * I))
    cells = m.face_cells[ids]
    on_plane = np.zeros(N, dtype=bool)
    on_plane[cells.ravel()] = True
    assert np.all(seed[~on_plane] == 0.0)
    # every (face, angle) pair with n_k . n_f != 0 lands on exactly one of its two cells
    nz = np.count_nonzero(seed)
    assert nz <= ids.size * K
