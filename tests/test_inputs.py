"""Pins of the seeded input generators: angle sets and periodic Voronoi meshes.

The angle sets are checked against the moment identities an angular quadrature
must satisfy (section 2.3: weights are solid-angle elements summing to one;
the moments of section 2.1 need sum W n = 0 and sum W n n = I/3 for an
isotropic field).  The meshes are checked against geometric identities and
against scipy's Voronoi tessellation.
"""
import numpy as np
import pytest

from paper_2002_08377_amd import inputs as inp


@pytest.mark.parametrize("K", [8, 24, 48, 80])
def test_angle_set_moments(K):
    d, w = inp.angle_set(K)
    assert d.shape == (K, 3)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=0, atol=2e-16)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w @ d, 0.0, atol=1e-16)
    np.testing.assert_allclose((d * w[:, None]).T @ d, np.eye(3) / 3.0, atol=2e-16)
    # odd moments vanish
    for p in [(3, 0, 0), (1, 1, 1), (2, 1, 0), (1, 0, 0)]:
        assert abs(np.sum(w * d[:, 0] ** p[0] * d[:, 1] ** p[1] * d[:, 2] ** p[2])) < 1e-16
    # fourth moments of an isotropic distribution (one direction per octant cannot carry them)
    if K > 8:
        assert abs(np.sum(w * d[:, 0] ** 4) - 0.2) < 1e-15
        assert abs(np.sum(w * d[:, 0] ** 2 * d[:, 1] ** 2) - 1.0 / 15.0) < 1e-15
    # octant symmetry: every direction has its antipode
    for k in range(K):
        assert np.min(np.linalg.norm(d + d[k], axis=1)) < 1e-15


def test_angle_set_s4_mu1():
    # with three directions per octant the construction is the textbook S4 set, mu_1 = 0.3500212
    d, _ = inp.angle_set(24)
    assert abs(np.min(np.abs(d)) - 0.3500212) < 1e-7


@pytest.mark.parametrize("K", [8, 24, 48, 80, 120])
def test_adjacent_pair_order(K):
    """The reordering puts each antipode right after its angle and keeps the weights with
    their directions; the problem's intensity columns follow the same permutation."""
    d, w = inp.angle_set(K)
    perm = inp.adjacent_pair_order(K)
    assert sorted(perm.tolist()) == list(range(K))
    da, wa = d[perm], w[perm]
    assert np.array_equal(da[1::2], -da[0::2]) and np.array_equal(wa[1::2], wa[0::2])
    p = inp.make_problem(0, n=6, K=K, steps=1)
    q = inp.with_angle_order(p, perm)
    assert np.array_equal(q.dirs, p.dirs[perm]) and np.array_equal(q.weights, p.weights[perm])
    assert np.array_equal(q.state.I, p.state.I[:, perm]) and q.state.I.flags["C_CONTIGUOUS"]
    assert np.array_equal(q.state.etot, p.state.etot) and q.mesh is p.mesh
    with pytest.raises(ValueError):
        inp.adjacent_pair_order(7)


@pytest.mark.parametrize("n,jitter", [(6, 0.2), (8, 0.2), (12, 0.2), (7, 0.05)])
def test_voronoi_invariants(n, jitter):
    m = inp.voronoi_mesh(n, jitter, seed=11)
    N, F = m.n_cells, m.n_faces
    assert N == n ** 3
    assert abs(m.vol.sum() - 1.0) < 1e-13
    assert np.all(m.face_cells[:, 0] < m.face_cells[:, 1])
    assert np.all(m.face_area > 0)
    # closure: sum_f A n = 0 per cell (outward normals)
    An = m.face_area[:, None] * m.face_normal
    clo = np.zeros((N, 3))
    np.add.at(clo, m.face_cells[:, 0], An)
    np.add.at(clo, m.face_cells[:, 1], -An)
    assert np.abs(clo).max() < 1e-14 * m.h ** 2 * 100
    # V_i = (1/3) sum_f A_f (c_f - r_i) . n_f with outward normal
    i, j = m.face_cells[:, 0], m.face_cells[:, 1]
    hi = np.einsum("fc,fc->f", m.face_centroid - m.gen[i], m.face_normal) * m.face_area
    cj = m.face_centroid - m.face_shift * m.box
    hj = np.einsum("fc,fc->f", cj - m.gen[j], -m.face_normal) * m.face_area
    V = np.zeros(N)
    np.add.at(V, i, hi / 3.0)
    np.add.at(V, j, hj / 3.0)
    np.testing.assert_allclose(V, m.vol, rtol=1e-12)
    # the face lies on the bisector: centroid equidistant from both generators
    rj = m.gen[j] + m.face_shift * m.box
    di = np.linalg.norm(m.face_centroid - m.gen[i], axis=1)
    dj = np.linalg.norm(m.face_centroid - rj, axis=1)
    np.testing.assert_allclose(di, dj, rtol=1e-12)
    # normal along r_j - r_i
    u = (rj - m.gen[i]) / np.linalg.norm(rj - m.gen[i], axis=1)[:, None]
    np.testing.assert_allclose(u, m.face_normal, atol=1e-15)
    # centre of mass inside the cell: closer to its own generator than to its neighbours' bisectors
    assert np.all(np.einsum("fc,fc->f", m.com[i] - 0.5 * (m.gen[i] + rj), m.face_normal) < 0)


def test_voronoi_both_sides_agree():
    n = 7
    m = inp.voronoi_mesh(n, 0.2, seed=5)
    vol, com, fc, fs, fa, fn, fcen = inp.voronoi_from_generators(n, m.gen, m.cell_lat, 0.2, 1.0, mode=1)
    assert fc.shape[0] == 2 * m.n_faces
    table = {(int(a), int(b), tuple(int(x) for x in s)): ar for (a, b), s, ar in zip(fc, fs, fa)}
    for (a, b), s, ar in zip(fc, fs, fa):
        other = table[(int(b), int(a), tuple(-int(x) for x in s))]
        assert abs(other - ar) <= 1e-11 * max(ar, 1e-3 * m.h ** 2)


def test_voronoi_matches_scipy():
    from scipy.spatial import ConvexHull, Voronoi
    n = 6
    m = inp.voronoi_mesh(n, 0.2, seed=3)
    pts = np.concatenate([m.gen + np.array([sx, sy, sz]) for sx in (-1, 0, 1) for sy in (-1, 0, 1)
                          for sz in (-1, 0, 1)])
    vor = Voronoi(pts)
    N = m.n_cells
    base = 13 * N  # the (0,0,0) image block
    vols = np.array([ConvexHull(vor.vertices[vor.regions[vor.point_region[base + i]]]).volume for i in range(N)])
    np.testing.assert_allclose(vols, m.vol, rtol=1e-12)
    # face count: a ridge inside the central block is one face; a ridge to an image block is half of one
    inb = lambda p: base <= p < base + N
    faces = sum(1.0 if (inb(p) and inb(q)) else 0.5 for p, q in vor.ridge_points if inb(p) or inb(q))
    assert faces == m.n_faces


def test_unjittered_lattice_is_cubic():
    m = inp.voronoi_mesh(6, 0.0, seed=0)
    assert m.n_faces == 3 * m.n_cells
    np.testing.assert_allclose(m.face_area, m.h ** 2, rtol=1e-13)
    np.testing.assert_allclose(m.vol, m.h ** 3, rtol=1e-13)
    np.testing.assert_allclose(m.com, m.gen, atol=1e-15)


def test_config_recipe_is_seeded():
    p1 = inp.make_problem(0)
    p2 = inp.make_problem(0)
    assert np.array_equal(p1.state.I, p2.state.I)
    assert np.array_equal(p1.mesh.gen, p2.mesh.gen)
    assert p1.mesh.n_cells == 1728 and p1.dirs.shape == (24, 3) and p1.steps == 10
    st = p1.state
    assert np.all(st.rho > 0) and np.all(st.I > 0)
    assert 0.1 <= st.kP.min() and st.kP.max() <= 10.0
    # total energy holds thermal plus kinetic parts
    e_int = st.etot - 0.5 * np.sum(st.mom ** 2, axis=1) / st.rho
    np.testing.assert_allclose(e_int, st.rho * p1.phys.cv * st.T, rtol=1e-13)
    assert abs(p1.dt - 0.3 * np.min(p1.mesh.vol) ** (1 / 3) / 100.0) < 1e-18
