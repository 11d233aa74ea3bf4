"""A beam-and-shadow set-up after the paper's shadow test (section 3.5), as inputs only.

A layer of emitter cells at y = 0.1 beams along +y into the angles within the
opening cosine of +y (the 4 angles nearest +y of the level-symmetric set); an
optically thick sphere (radius 0.15, centre (0.5, 0.4, 0.5)) stands in the beam;
an absorbing boundary layer at y = 0.9 stops the periodic wrap; the medium is
near-vacuum, the gas at rest.  Radiation energy is then measured in a band of y
above the sphere, straight behind it (shadow) and far to the side (lit).
"""
import numpy as np

from paper_2002_08377_amd import inputs as inp

EMITTER, BOUNDARY = 2, 1  # the library's and the oracle's cell kinds


def shadow_problem(n, K, steps, cos_open=0.95):
    p = inp.make_problem(0, n=n, K=K, steps=steps)
    st = p.state
    st.mesh_vel[:] = 0.0
    st.mom[:] = 0.0
    st.kP[:] = 1e-3
    st.kJ[:] = 1e-3
    st.ks[:] = 0.0
    st.I *= 1e-3
    g, h = p.mesh.gen, p.mesh.h
    x, y, z = g[:, 0], g[:, 1], g[:, 2]
    src = np.nonzero(np.abs(y - 0.1) < 0.6 * h)[0]
    top = np.nonzero(np.abs(y - 0.9) < 0.6 * h)[0]
    clump = np.nonzero((x - 0.5) ** 2 + (y - 0.4) ** 2 + (z - 0.5) ** 2 < 0.15 ** 2)[0]
    st.kP[clump] = st.kJ[clump] = 1e4 / st.rho[clump]
    st.kP[src] = st.kJ[src] = 50.0  # emitters radiate through their opacity
    cells = np.concatenate([src, top])
    kinds = np.array([EMITTER] * src.size + [BOUNDARY] * top.size)
    d = np.tile([0.0, 1.0, 0.0], (cells.size, 1))
    T = np.concatenate([np.full(src.size, 2.0), np.zeros(top.size)])
    co = np.concatenate([np.full(src.size, cos_open), np.full(top.size, 2.0)])
    band = (y > 0.62) & (y < 0.75)
    regions = {
        "shadow": band & (np.abs(x - 0.5) < 0.06) & (np.abs(z - 0.5) < 0.06),
        "lit": band & ((np.abs(x - 0.5) > 0.3) | (np.abs(z - 0.5) > 0.3)),
    }
    return p, (cells, kinds, T, d, co), regions


def radiation_energy(I, weights):
    return 4.0 * np.pi * (I @ weights)
