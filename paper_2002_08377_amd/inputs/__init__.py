"""Seeded synthetic inputs for the radiation step.

This module generates inputs only -- meshes, angle sets and initial states --
and holds none of the radiation method's arithmetic (no face velocity, no
flux, no source term).  Both the HIP library and the CPU oracle are fed the
same arrays from here; neither imports the other.

* ``voronoi_mesh``: periodic Voronoi tessellation of a jittered cubic lattice
  (generators at lattice sites plus a uniform jitter of +-``jitter`` spacings),
  cells numbered in Morton (Z-curve) order of their lattice site so that
  spatial neighbours sit close in memory.
* ``angle_set``: equal-weight octant-symmetric direction sets of size
  8 * m(m+1)/2 (8, 24, 48, 80, ...) from the level-symmetric construction.
* ``initial_state`` / ``make_config``: gas, opacity and intensity draws for
  the five workloads (plain forward 12^3 x 24 angles; PLM 64^3 x 80;
  adjoint 32^3 x 48; throughput 128^3 x 80; adjoint at scale 96^3 x 80).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libvoronoi.so")
_lib = None

MASTER_SEED = 2002083770


def build_voronoi(force: bool = True) -> str:
    """Compile the host Voronoi builder (plain C, OpenMP) in-tree."""
    src = os.path.join(_HERE, "voronoi.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_voronoi(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.vor_count.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_int,
                                  P, P, P, P]
        lib.vor_count.restype = ctypes.c_int
        lib.vor_faces.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_int,
                                  P, P, P, P, P, P]
        lib.vor_faces.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def morton_order(n: int) -> np.ndarray:
    """Lattice sites (a,b,c) of an n^3 grid sorted by their Morton code; returns [N,3] int32."""
    idx = np.arange(n, dtype=np.int64)
    c, b, a = np.meshgrid(idx, idx, idx, indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    code = np.zeros(a.shape, dtype=np.int64)
    for bit in range(21):
        code |= ((a >> bit) & 1) << (3 * bit)
        code |= ((b >> bit) & 1) << (3 * bit + 1)
        code |= ((c >> bit) & 1) << (3 * bit + 2)
    order = np.argsort(code, kind="stable")
    return np.stack([a[order], b[order], c[order]], axis=1).astype(np.int32)


@dataclass
class Mesh:
    """Periodic Voronoi mesh in a cube of side ``box``; faces listed once (cell0 < cell1)."""
    n: int
    box: float
    gen: np.ndarray          # [N,3] generator positions
    com: np.ndarray          # [N,3] centres of mass (same periodic frame as gen)
    vol: np.ndarray          # [N]   cell volumes
    cell_lat: np.ndarray     # [N,3] lattice site of each cell
    face_cells: np.ndarray   # [F,2] int32 (i, j), i < j
    face_shift: np.ndarray   # [F,3] int8: image of j adjacent to i is gen[j] + shift*box
    face_area: np.ndarray    # [F]
    face_normal: np.ndarray  # [F,3] unit, from i towards j
    face_centroid: np.ndarray  # [F,3] in the frame of cell i

    @property
    def n_cells(self) -> int:
        return self.gen.shape[0]

    @property
    def n_faces(self) -> int:
        return self.face_cells.shape[0]

    @property
    def h(self) -> float:
        return self.box / self.n


def voronoi_from_generators(n: int, gen: np.ndarray, cell_lat: np.ndarray, jitter: float, box: float = 1.0,
                            mode: int = 0):
    """Tessellate; ``mode`` 0 lists each face once, 1 lists every face from both sides."""
    lib = _load()
    N = n ** 3
    gen = np.ascontiguousarray(gen, dtype=np.float64)
    cell_lat = np.ascontiguousarray(cell_lat, dtype=np.int32)
    lat_cell = np.empty(N, dtype=np.int32)
    lat_cell[(cell_lat[:, 2].astype(np.int64) * n + cell_lat[:, 1]) * n + cell_lat[:, 0]] = np.arange(N)
    counts = np.zeros(N, dtype=np.int64)
    vol = np.zeros(N)
    com = np.zeros((N, 3))
    bad = ctypes.c_int64(-1)
    rc = lib.vor_count(n, box, jitter, _ptr(gen), _ptr(cell_lat), _ptr(lat_cell), mode, _ptr(counts),
                       _ptr(vol), _ptr(com), ctypes.byref(bad))
    if rc:
        raise RuntimeError(f"voronoi builder failed with code {rc} at cell {bad.value}")
    off = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    F = int(off[-1])
    fc = np.empty((F, 2), dtype=np.int32)
    fs = np.empty((F, 3), dtype=np.int8)
    fa = np.empty(F)
    fn = np.empty((F, 3))
    fcen = np.empty((F, 3))
    rc = lib.vor_faces(n, box, jitter, _ptr(gen), _ptr(cell_lat), _ptr(lat_cell), mode, _ptr(off), _ptr(fc),
                       _ptr(fs), _ptr(fa), _ptr(fn), _ptr(fcen))
    if rc:
        raise RuntimeError(f"voronoi builder failed in face pass with code {rc}")
    return vol, com, fc, fs, fa, fn, fcen


def voronoi_mesh(n: int, jitter: float = 0.2, rng: np.random.Generator | None = None, seed: int = 0,
                 box: float = 1.0) -> Mesh:
    """Jittered-lattice periodic Voronoi mesh with n^3 cells in Morton order."""
    if rng is None:
        rng = np.random.default_rng(seed)
    h = box / n
    # jitter drawn per lattice site in (z, y, x) C order, then read in Morton order
    jit = rng.uniform(-jitter, jitter, size=(n, n, n, 3))
    cell_lat = morton_order(n)
    a, b, c = cell_lat[:, 0], cell_lat[:, 1], cell_lat[:, 2]
    gen = (cell_lat.astype(np.float64) + 0.5 + jit[c, b, a]) * h
    vol, com, fc, fs, fa, fn, fcen = voronoi_from_generators(n, gen, cell_lat, jitter, box)
    return Mesh(n=n, box=box, gen=gen, com=com, vol=vol, cell_lat=cell_lat, face_cells=fc, face_shift=fs,
                face_area=fa, face_normal=fn, face_centroid=fcen)


# ----------------------------------------------------------------------------------------------
# angle sets
# ----------------------------------------------------------------------------------------------

def _octant_points(m: int, mu1: float) -> np.ndarray:
    if m == 1:
        return np.full((1, 3), 1.0 / np.sqrt(3.0))
    delta = (1.0 - 3.0 * mu1 * mu1) / (m - 1)
    mu = np.sqrt(mu1 * mu1 + delta * np.arange(m))
    pts = [(mu[i], mu[j], mu[m - 1 - i - j]) for i in range(m) for j in range(m - i)]
    return np.array(pts)


def angle_set(K: int) -> tuple[np.ndarray, np.ndarray]:
    """Equal-weight, octant-symmetric unit vectors, K = 8*m(m+1)/2.

    First-octant points (mu_i, mu_j, mu_k) with i+j+k = m-1 and
    mu_i^2 = mu_1^2 + i*(1 - 3 mu_1^2)/(m-1); all 8 sign flips, ordered so that
    direction k + K/2 is the antipode of direction k; weights 1/K.
    mu_1 is fixed by bisection so that the quadrature integrates n_x^4 exactly
    (mean 1/5), the classic level-symmetric choice.
    """
    m = 1
    while 8 * m * (m + 1) // 2 < K:
        m += 1
    if 8 * m * (m + 1) // 2 != K:
        raise ValueError(f"K={K} is not of the form 8*m(m+1)/2")
    if m == 1:
        mu1 = 1.0 / np.sqrt(3.0)
    else:
        def fourth(mu1):
            p = _octant_points(m, mu1)
            return np.mean(p[:, 0] ** 4) - 0.2
        lo, hi = 1e-6, 1.0 / np.sqrt(3.0) - 1e-12
        flo = fourth(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            fm = fourth(mid)
            if (fm > 0) == (flo > 0):
                lo, flo = mid, fm
            else:
                hi = mid
        mu1 = 0.5 * (lo + hi)
    oct_pts = _octant_points(m, mu1)
    # octants with z > 0 first; the second half repeats them negated, so that
    # direction k + K/2 is the antipode of direction k
    upper = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (-1, -1, 1)]
    dirs = [oct_pts * np.array(s) for s in upper] + [-oct_pts * np.array(s) for s in upper]
    d = np.concatenate(dirs, axis=0)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    w = np.full(K, 1.0 / K)
    return np.ascontiguousarray(d), w


def adjacent_pair_order(K: int) -> np.ndarray:
    """Permutation taking an angle set whose direction k + K/2 is the antipode of direction k
    (the order of ``angle_set``) to the order in which direction 2p + 1 is the antipode of
    direction 2p: new position 2p holds old angle p, new position 2p + 1 old angle p + K/2.
    Index any per-angle array with it (``dirs[perm]``, ``I[:, perm]``)."""
    if K % 2:
        raise ValueError("an antipodal set has an even number of angles")
    perm = np.empty(K, dtype=np.int64)
    perm[0::2] = np.arange(K // 2)
    perm[1::2] = np.arange(K // 2) + K // 2
    return perm


# ----------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------

@dataclass
class Config:
    name: str
    n: int
    K: int
    steps: int
    scheme: str            # "upwind1" or "plm_vl2"
    kappa_mode: str        # "loguniform" or "optical_depth"
    index: int


CONFIGS = [
    Config("forward_12c_24a", 12, 24, 10, "upwind1", "loguniform", 0),
    Config("plm_64c_80a", 64, 80, 100, "plm_vl2", "optical_depth", 1),
    Config("adjoint_32c_48a", 32, 48, 20, "upwind1", "loguniform", 2),
    Config("throughput_128c_80a", 128, 80, 50, "upwind1", "loguniform", 3),
    Config("adjoint_96c_80a", 96, 80, 40, "upwind1", "loguniform", 4),
]


@dataclass
class Physics:
    c_red: float = 100.0
    c_light: float = 100.0
    a_rad: float = 1.0
    gamma: float = 5.0 / 3.0

    @property
    def cv(self) -> float:
        # code units with k_B / (mu m_p) = 1: rho*cv = rho / (gamma - 1)
        return 1.0 / (self.gamma - 1.0)


@dataclass
class State:
    """Initial per-cell state; all float64, intensities [N,K]."""
    rho: np.ndarray
    mom: np.ndarray
    etot: np.ndarray
    kP: np.ndarray
    kJ: np.ndarray
    ks: np.ndarray
    I: np.ndarray
    vol: np.ndarray
    mesh_vel: np.ndarray
    T: np.ndarray


@dataclass
class Problem:
    mesh: Mesh
    dirs: np.ndarray
    weights: np.ndarray
    state: State
    phys: Physics
    dt: float
    steps: int
    scheme: str
    config: Config | None = None
    seeds: dict = field(default_factory=dict)


def with_angle_order(prob: Problem, perm: np.ndarray) -> Problem:
    """The same problem with its angles (directions, weights, intensity columns) permuted."""
    st = dataclasses.replace(prob.state, I=np.ascontiguousarray(prob.state.I[:, perm]))
    return dataclasses.replace(prob, dirs=np.ascontiguousarray(prob.dirs[perm]),
                               weights=np.ascontiguousarray(prob.weights[perm]), state=st)


SEED_STREAMS = ("jitter", "rho", "T", "v", "kappa", "I_noise", "omega", "fd_cells")


def seed_streams(index: int) -> dict:
    ss = np.random.SeedSequence(MASTER_SEED + index)
    kids = ss.spawn(len(SEED_STREAMS))
    return {k: np.random.default_rng(s) for k, s in zip(SEED_STREAMS, kids)}


def initial_state(mesh: Mesh, K: int, rngs: dict, phys: Physics, kappa_mode: str = "loguniform",
                  v_sigma: float = 0.1) -> State:
    N = mesh.n_cells
    rho = np.exp(rngs["rho"].normal(0.0, 0.5, size=N))
    T = rngs["T"].uniform(0.5, 2.0, size=N)
    v = rngs["v"].normal(0.0, v_sigma, size=(N, 3))
    if kappa_mode == "loguniform":
        ka = 10.0 ** rngs["kappa"].uniform(-1.0, 1.0, size=N)
    elif kappa_mode == "optical_depth":
        tau = 10.0 ** rngs["kappa"].uniform(-3.0, 3.0, size=N)
        ka = tau / (rho * mesh.h)
    else:
        raise ValueError(kappa_mode)
    ks = np.full(N, 0.1)
    noise = rngs["I_noise"].normal(0.0, 1.0, size=(N, K))
    I = (phys.a_rad * T ** 4 / (4.0 * np.pi))[:, None] * (1.0 + 0.1 * noise)
    mom = rho[:, None] * v
    etot = rho * phys.cv * T + 0.5 * rho * np.sum(v * v, axis=1)
    return State(rho=rho, mom=np.ascontiguousarray(mom), etot=etot, kP=ka.copy(), kJ=ka.copy(), ks=ks,
                 I=np.ascontiguousarray(I), vol=mesh.vol.copy(), mesh_vel=np.ascontiguousarray(v.copy()), T=T)


def courant_dt(mesh: Mesh, c_red: float, cfl: float = 0.3) -> float:
    """dt = cfl * min cell size / c_red with cell size V^(1/3)."""
    return cfl * float(np.min(mesh.vol) ** (1.0 / 3.0)) / c_red


def make_problem(index: int, n: int | None = None, K: int | None = None, steps: int | None = None,
                 jitter: float = 0.2) -> Problem:
    """The seeded recipe of workload ``index`` (optionally at a reduced size)."""
    cfg = CONFIGS[index]
    n = cfg.n if n is None else n
    K = cfg.K if K is None else K
    steps = cfg.steps if steps is None else steps
    rngs = seed_streams(index)
    phys = Physics()
    mesh = voronoi_mesh(n, jitter=jitter, rng=rngs["jitter"])
    dirs, w = angle_set(K)
    st = initial_state(mesh, K, rngs, phys, cfg.kappa_mode)
    return Problem(mesh=mesh, dirs=dirs, weights=w, state=st, phys=phys, dt=courant_dt(mesh, phys.c_red),
                   steps=steps, scheme=cfg.scheme, config=cfg, seeds=rngs)


def plane_faces(mesh: Mesh, x0: float = 0.5) -> tuple[np.ndarray, np.ndarray]:
    """Faces whose generator pair straddles the plane x = x0 without wrapping.

    Returns (face ids, orientation) with orientation +1 when the face normal
    (cell0 -> cell1) points towards +x, else -1.
    """
    i = mesh.face_cells[:, 0]
    j = mesh.face_cells[:, 1]
    xi = mesh.gen[i, 0]
    xj = mesh.gen[j, 0] + mesh.face_shift[:, 0] * mesh.box
    no_wrap = mesh.face_shift[:, 0] == 0
    cross = no_wrap & (((xi < x0) & (xj > x0)) | ((xi > x0) & (xj < x0)))
    ids = np.nonzero(cross)[0].astype(np.int32)
    sign = np.where(xj[ids] > xi[ids], 1, -1).astype(np.int8)
    return ids, sign


def loss_face_weights(mesh: Mesh, rng: np.random.Generator, x0: float = 0.5) -> np.ndarray:
    """Signed per-face loss weight u_f = orientation * omega_f, omega ~ U[0,1] on plane faces, 0 elsewhere."""
    ids, sign = plane_faces(mesh, x0)
    omega = rng.uniform(0.0, 1.0, size=ids.shape[0])
    u = np.zeros(mesh.n_faces)
    u[ids] = sign * omega
    return u


def fd_cells(mesh: Mesh, rng: np.random.Generator, count: int = 16, hops: float = 4.0,
             x0: float = 0.5) -> np.ndarray:
    """`count` distinct cells whose generators lie within `hops` lattice spacings of the
    loss plane x = x0 (inside the domain of dependence of a few first-order steps),
    drawn without replacement; used for finite-difference checks of gradients."""
    near = np.nonzero(np.abs(mesh.gen[:, 0] - x0) < hops * mesh.h)[0]
    return np.sort(rng.choice(near, size=min(count, near.size), replace=False))
