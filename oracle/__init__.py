"""TEST INFRASTRUCTURE: the FP64 CPU oracle of the radiation step.

Plain C (``rt_oracle.c``, OpenMP over angles or cells) behind ctypes.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package; the product path (the HIP library and its binding) never
does, and shares no code with it.

Functions take a mesh object with the attributes ``gen, com, vol, face_cells,
face_shift, face_area, face_normal, face_centroid, box`` (numpy arrays) plus
the generator velocities, and plain numpy state arrays.  Everything is FP64;
``*_cs`` variants run the same C source compiled with complex numbers for
complex-step derivatives.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

FOURPI = 4.0 * np.pi


def build(force: bool = True) -> str:
    """Compile the oracle: the C source twice (real, complex) into one shared library."""
    src = os.path.join(_HERE, "rt_oracle.c")
    if force or not os.path.exists(_LIB):
        o1 = _LIB + ".real.o"
        o2 = _LIB + ".cs.o"
        flags = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC"]
        subprocess.check_call(flags + ["-c", src, "-o", o1])
        subprocess.check_call(flags + ["-DOR_COMPLEX", "-c", src, "-o", o2])
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", tmp, o1, o2, "-lm"])
        os.replace(tmp, _LIB)
        for o in (o1, o2):
            os.remove(o)
    return _LIB


class _OMesh(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_faces", ctypes.c_int64), ("gen", ctypes.c_void_p),
                ("com", ctypes.c_void_p), ("vol", ctypes.c_void_p), ("mesh_vel", ctypes.c_void_p),
                ("face_cells", ctypes.c_void_p), ("face_shift", ctypes.c_void_p), ("face_area", ctypes.c_void_p),
                ("face_normal", ctypes.c_void_p), ("face_centroid", ctypes.c_void_p), ("box", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P, D, I64, INT = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int
        MP = ctypes.POINTER(_OMesh)
        sig = {
            "or_face_speed": [MP, P],
            "or_volume_rate": [MP, P, P],
            "or_advance_volume": [I64, P, D, P, P],
            "or_transport_upwind": [MP, P, INT, P, D, D, P, P, P, P],
            "or_transport_upwind_cs": [MP, P, INT, P, D, D, P, P, P, P],
            "or_gradient_limited": [MP, INT, P, P],
            "or_gradient_limited_cs": [MP, INT, P, P],
            "or_transport_plm": [MP, P, INT, P, D, D, P, P, P, P, P, P],
            "or_transport_plm_cs": [MP, P, INT, P, D, D, P, P, P, P, P, P],
            "or_source": [I64, INT, P, P, D, D, D, D, D, P, P, P, P, P, P, P, P],
            "or_source_cs": [I64, INT, P, P, D, D, D, D, D, P, P, P, P, P, P, P, P],
            "or_diagnostics": [I64, INT, P, P, D, D, P, P, P, P, P],
            "or_moments": [I64, INT, P, P, D, P, P],
            "or_transport_upwind_vjp": [MP, P, INT, P, D, D, P, P, P, P],
            "or_source_vjp": [I64, INT, P, P, D, D, D, D, D, P, P, P, P, P, P, P, P, P, P, P, P],
            "or_marked_cells": [I64, P, P, P, P, P, D, INT, P, D, D, D, D, P, P, P, P, P],
            "or_source_mg": [I64, INT, INT, P, P, P, D, D, D, D, D, P, P, P, P, P, P, P, P],
            "or_source_kT": [I64, INT, P, P, D, D, D, D, D, P, P, P, P, P, P, P, D, D, D, P],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = None
        lib.or_num_threads.argtypes = []
        lib.or_num_threads.restype = INT
        lib.or_set_num_threads.argtypes = [INT]
        lib.or_set_num_threads.restype = None
        lib.or_quartic_root.argtypes = [D, D, D]
        lib.or_quartic_root.restype = D
        for name in ("or_flux_loss", "or_flux_loss_cs"):
            getattr(lib, name).argtypes = [MP, INT, P, P, D, P, P, P, P]
            getattr(lib, name).restype = None
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"], "arrays must be C-contiguous numpy"
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


class OracleMesh:
    """Holds the mesh arrays (kept alive) and the ctypes view of them."""

    def __init__(self, mesh, mesh_vel):
        self.n_cells = int(mesh.gen.shape[0])
        self.n_faces = int(mesh.face_cells.shape[0])
        self._keep = dict(
            gen=_f64(mesh.gen), com=_f64(mesh.com), vol=_f64(mesh.vol), mesh_vel=_f64(mesh_vel),
            face_cells=np.ascontiguousarray(mesh.face_cells, dtype=np.int32),
            face_shift=np.ascontiguousarray(mesh.face_shift, dtype=np.int8),
            face_area=_f64(mesh.face_area), face_normal=_f64(mesh.face_normal),
            face_centroid=_f64(mesh.face_centroid))
        k = self._keep
        self.c = _OMesh(self.n_cells, self.n_faces, _p(k["gen"]), _p(k["com"]), _p(k["vol"]), _p(k["mesh_vel"]),
                        _p(k["face_cells"]), _p(k["face_shift"]), _p(k["face_area"]), _p(k["face_normal"]),
                        _p(k["face_centroid"]), float(mesh.box))
        self.vol = k["vol"]
        self.wn = self.face_speed()
        self.D = self.volume_rate(self.wn)

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def face_speed(self):
        wn = np.empty(self.n_faces)
        _load().or_face_speed(self.ref, _p(wn))
        return wn

    def volume_rate(self, wn):
        D = np.empty(self.n_cells)
        _load().or_volume_rate(self.ref, _p(_f64(wn)), _p(D))
        return D

    def advance_volume(self, vol, dt):
        out = np.empty(self.n_cells)
        _load().or_advance_volume(self.n_cells, _p(self.D), float(dt), _p(_f64(vol)), _p(out))
        return out


# ------------------------------------------------------------------------------------------------
# elementary steps
# ------------------------------------------------------------------------------------------------

def transport_upwind(om: OracleMesh, dirs, c_red, dt, I, vol, complex_step=False):
    """First-order upwind transport over dt; returns (I_out, vol_out)."""
    K = dirs.shape[0]
    vol = _f64(vol)
    vol_out = om.advance_volume(vol, dt)
    if complex_step:
        I = _c128(I)
        out = np.empty_like(I)
        _load().or_transport_upwind_cs(om.ref, _p(om.wn), K, _p(_f64(dirs)), c_red, dt, _p(I), _p(vol),
                                       _p(vol_out), _p(out))
    else:
        I = _f64(I)
        out = np.empty_like(I)
        _load().or_transport_upwind(om.ref, _p(om.wn), K, _p(_f64(dirs)), c_red, dt, _p(I), _p(vol),
                                    _p(vol_out), _p(out))
    return out, vol_out


def gradient_limited(om: OracleMesh, I, complex_step=False):
    """Limited S10 gradient of every angle, layout [N, 3, K]."""
    N, K = I.shape
    if complex_step:
        I = _c128(I)
        g = np.empty((N, 3, K), dtype=np.complex128)
        _load().or_gradient_limited_cs(om.ref, K, _p(I), _p(g))
    else:
        I = _f64(I)
        g = np.empty((N, 3, K))
        _load().or_gradient_limited(om.ref, K, _p(I), _p(g))
    return g


def transport_plm(om: OracleMesh, dirs, c_red, dt, I_base, I_half, grad, vol, complex_step=False):
    K = dirs.shape[0]
    vol = _f64(vol)
    vol_out = om.advance_volume(vol, dt)
    cast = _c128 if complex_step else _f64
    I_base, I_half, grad = cast(I_base), cast(I_half), cast(grad)
    out = np.empty_like(I_base)
    fn = _load().or_transport_plm_cs if complex_step else _load().or_transport_plm
    fn(om.ref, _p(om.wn), K, _p(_f64(dirs)), c_red, dt, _p(I_base), _p(I_half), _p(grad), _p(vol), _p(vol_out),
       _p(out))
    return out, vol_out


def source(dirs, W, phys, dt, I, rho, mom, etot, kP, kJ, ks, complex_step=False):
    """Implicit source step on copies; returns (I', mom', etot', T')."""
    N, K = I.shape
    cast = _c128 if complex_step else _f64
    I, mom, etot, kP, kJ = cast(I).copy(), cast(mom).copy(), cast(etot).copy(), cast(kP), cast(kJ)
    T = np.empty(N, dtype=I.dtype)
    fn = _load().or_source_cs if complex_step else _load().or_source
    fn(N, K, _p(_f64(dirs)), _p(_f64(W)), phys.c_red, phys.c_light, phys.a_rad, phys.cv, dt, _p(I),
       _p(_f64(rho)), _p(mom), _p(etot), _p(kP), _p(kJ), _p(_f64(ks)), _p(T))
    return I, mom, etot, T


def flux_loss(om: OracleMesh, dirs, W, c_light, I, face_weight, want_seed=False, complex_step=False):
    N, K = I.shape
    fw = _f64(face_weight)
    if complex_step:
        I = _c128(I)
        out = np.zeros(1, dtype=np.complex128)
        _load().or_flux_loss_cs(om.ref, K, _p(_f64(dirs)), _p(_f64(W)), c_light, _p(I), _p(fw), None, _p(out))
        return complex(out[0])
    I = _f64(I)
    seed = np.zeros_like(I) if want_seed else None
    out = np.zeros(1)
    _load().or_flux_loss(om.ref, K, _p(_f64(dirs)), _p(_f64(W)), c_light, _p(I), _p(fw), _p(seed), _p(out))
    L = float(out[0])
    return (L, seed) if want_seed else L


def num_threads() -> int:
    """Threads used by the oracle's OpenMP loops."""
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops from now on (n >= 1)."""
    _load().or_set_num_threads(int(n))


def quartic_root(A, B, C):
    """Positive root of A T^4 + B T - C = 0 as the source step solves it."""
    return _load().or_quartic_root(float(A), float(B), float(C))


def moments(dirs, W, c_light, I):
    """Per-cell angle moments [N, 10]: E_r, F_r (3), P_r (xx, yy, zz, xy, xz, yz), section 2.1."""
    I = _f64(I)
    N, K = I.shape
    out = np.empty((N, 10))
    _load().or_moments(N, K, _p(_f64(dirs)), _p(_f64(W)), float(c_light), _p(I), _p(out))
    return out


def diagnostics(dirs, W, phys, I, vol, etot, mom):
    N, K = I.shape
    out = np.empty(10)
    _load().or_diagnostics(N, K, _p(_f64(dirs)), _p(_f64(W)), phys.c_red, phys.c_light, _p(_f64(I)),
                           _p(_f64(vol)), _p(_f64(etot)), _p(_f64(mom)), _p(out))
    return out


def transport_upwind_vjp(om: OracleMesh, dirs, c_red, dt, vol, lam_out):
    K = dirs.shape[0]
    vol = _f64(vol)
    vol_out = om.advance_volume(vol, dt)
    lam_out = _f64(lam_out)
    lam_in = np.empty_like(lam_out)
    _load().or_transport_upwind_vjp(om.ref, _p(om.wn), K, _p(_f64(dirs)), c_red, dt, _p(vol), _p(vol_out),
                                    _p(lam_out), _p(lam_in))
    return lam_in


def source_vjp(dirs, W, phys, dt, I, rho, mom, etot, kP, kJ, ks, lamI, lamE, lamM):
    """Reverse of ``source``: returns (lamI_in, lamE_in, lamM_in, dL/dkP, dL/dkJ)."""
    N, K = I.shape
    lamI, lamE, lamM = _f64(lamI).copy(), _f64(lamE).copy(), _f64(lamM).copy()
    dkP = np.zeros(N)
    dkJ = np.zeros(N)
    _load().or_source_vjp(N, K, _p(_f64(dirs)), _p(_f64(W)), phys.c_red, phys.c_light, phys.a_rad, phys.cv, dt,
                          _p(_f64(I)), _p(_f64(rho)), _p(_f64(mom)), _p(_f64(etot)), _p(_f64(kP)), _p(_f64(kJ)),
                          _p(_f64(ks)), _p(lamI), _p(lamE), _p(lamM), _p(dkP), _p(dkJ))
    return lamI, lamE, lamM, dkP, dkJ


# ------------------------------------------------------------------------------------------------
# whole steps and runs (section 2: transport, then the source; van Leer two-stage form for PLM)
# ------------------------------------------------------------------------------------------------

class OState:
    """Evolving state of a run: intensities, volumes, gas momentum and total energy."""

    def __init__(self, I, vol, mom, etot):
        self.I, self.vol, self.mom, self.etot = I, vol, mom, etot

    def copy(self):
        return OState(self.I.copy(), self.vol.copy(), self.mom.copy(), self.etot.copy())


def step(om: OracleMesh, dirs, W, phys, dt, st: OState, rho, kP, kJ, ks, scheme="upwind1",
         complex_step=False, with_source=True):
    """One radiation step.

    upwind1: transport over dt (first order), then the source over dt.
    plm_vl2 (section 2, steps 2b-5, van Leer): stage 1 = first-order transport
    over dt/2 and the source over dt/2 (on a copy of the gas) giving the
    half-step state; stage 2 = fluxes from the limited linear reconstruction of
    the half-step state applied over dt to the start-of-step charges, then the
    source over dt on the start-of-step gas.
    """
    if scheme == "upwind1":
        I1, v1 = transport_upwind(om, dirs, phys.c_red, dt, st.I, st.vol, complex_step)
        if not with_source:
            return OState(I1, v1, st.mom.copy(), st.etot.copy()), None
        I2, m2, e2, T = source(dirs, W, phys, dt, I1, rho, st.mom, st.etot, kP, kJ, ks, complex_step)
        return OState(I2, v1, m2, e2), T
    if scheme == "plm_vl2":
        Ih, vh = transport_upwind(om, dirs, phys.c_red, 0.5 * dt, st.I, st.vol, complex_step)
        if with_source:
            Ih, _, _, _ = source(dirs, W, phys, 0.5 * dt, Ih, rho, st.mom, st.etot, kP, kJ, ks, complex_step)
        g = gradient_limited(om, Ih, complex_step)
        I1, v1 = transport_plm(om, dirs, phys.c_red, dt, st.I, Ih, g, st.vol, complex_step)
        if not with_source:
            return OState(I1, v1, st.mom.copy(), st.etot.copy()), None
        I2, m2, e2, T = source(dirs, W, phys, dt, I1, rho, st.mom, st.etot, kP, kJ, ks, complex_step)
        return OState(I2, v1, m2, e2), T
    raise ValueError(scheme)


def run(om: OracleMesh, dirs, W, phys, dt, st0: OState, rho, kP, kJ, ks, steps, scheme="upwind1",
        complex_step=False, record=False):
    """Run ``steps`` steps; with record=True also return per-step (I*, vol, mom, etot) for the adjoint."""
    st = st0.copy()
    if complex_step:
        st = OState(_c128(st.I), st.vol.copy(), _c128(st.mom), _c128(st.etot))
    tape = []
    T = None
    for _ in range(steps):
        if record:
            assert scheme == "upwind1"
            Istar, v1 = transport_upwind(om, dirs, phys.c_red, dt, st.I, st.vol)
            tape.append((Istar, st.vol.copy(), st.mom.copy(), st.etot.copy()))
            I2, m2, e2, T = source(dirs, W, phys, dt, Istar, rho, st.mom, st.etot, kP, kJ, ks)
            st = OState(I2, v1, m2, e2)
        else:
            st, T = step(om, dirs, W, phys, dt, st, rho, kP, kJ, ks, scheme, complex_step)
    return (st, T, tape) if record else (st, T)


def adjoint(om: OracleMesh, dirs, W, phys, dt, st0: OState, rho, kappa_a, ks, steps, face_weight):
    """Loss on the final intensities and its gradients w.r.t. I^0 and the tied opacity kP = kJ = kappa_a.

    Returns (L, dL/dI0 [N,K], dL/dkappa_a [N]).
    """
    stS, _, tape = run(om, dirs, W, phys, dt, st0, rho, kappa_a, kappa_a, ks, steps, record=True)
    L, lamI = flux_loss(om, dirs, W, phys.c_light, stS.I, face_weight, want_seed=True)
    N = stS.I.shape[0]
    lamE = np.zeros(N)
    lamM = np.zeros((N, 3))
    dk = np.zeros(N)
    for Istar, vol, mom, etot in reversed(tape):
        lamI, lamE, lamM, dkP, dkJ = source_vjp(dirs, W, phys, dt, Istar, rho, mom, etot, kappa_a, kappa_a, ks,
                                                lamI, lamE, lamM)
        dk += dkP + dkJ
        lamI = transport_upwind_vjp(om, dirs, phys.c_red, dt, vol, lamI)
    return L, lamI, dk


RT_CELL_BOUNDARY = 1
RT_CELL_EMITTER = 2


def marked_cells(dirs, phys, dt, st: OState, rho, kP, cells, kinds, T_eff, direction, cos_open, tau):
    """Boundary and emitter cells (sections 2.4-2.5) applied after a step; returns a new OState.

    cells, kinds [n] int; T_eff, cos_open [n]; direction [n][3] unit vectors; tau > 0."""
    out = st.copy()
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    assert np.unique(cells).size == cells.size, "marked cells must be distinct"
    K = out.I.shape[1]
    _load().or_marked_cells(cells.size, _p(cells), _p(kinds), _p(_f64(T_eff)), _p(_f64(direction)),
                            _p(_f64(cos_open)), float(tau), K, _p(_f64(dirs)), phys.c_red, phys.c_light,
                            phys.a_rad, float(dt), _p(out.I), _p(_f64(rho)), _p(out.mom), _p(out.etot),
                            _p(_f64(kP)))
    return out


def source_mg(dirs, W, Wg, phys, dt, I, rho, mom, etot, kP, kJ, ks):
    """Multigroup source update (section 2.3 generalised to groups coupled through T^4 only).

    I [G][N][K], kP/kJ/ks [G][N], Wg [G]; returns (I', mom', etot', T^{n+1})."""
    I = _f64(I).copy()
    G, N, K = I.shape
    mom = _f64(mom).copy()
    etot = _f64(etot).copy()
    T = np.zeros(N)
    _load().or_source_mg(N, K, G, _p(_f64(dirs)), _p(_f64(W)), _p(_f64(Wg)), phys.c_red, phys.c_light, phys.a_rad,
                         phys.cv, float(dt), _p(I), _p(_f64(rho)), _p(mom), _p(etot), _p(_f64(kP)), _p(_f64(kJ)),
                         _p(_f64(ks)), _p(T))
    return I, mom, etot, T


def source_kT(dirs, W, phys, dt, I, rho, mom, etot, kP0, kJ0, ks, T_ref, bP, bJ):
    """Source update with power-law opacities kX(T) = kX0 (T/T_ref)^bX at T^{n+1} (Newton on T).

    Returns (I', mom', etot', T^{n+1})."""
    I = _f64(I).copy()
    N, K = I.shape
    mom = _f64(mom).copy()
    etot = _f64(etot).copy()
    T = np.zeros(N)
    _load().or_source_kT(N, K, _p(_f64(dirs)), _p(_f64(W)), phys.c_red, phys.c_light, phys.a_rad, phys.cv,
                         float(dt), _p(I), _p(_f64(rho)), _p(mom), _p(etot), _p(_f64(kP0)), _p(_f64(kJ0)),
                         _p(_f64(ks)), float(T_ref), float(bP), float(bJ), _p(T))
    return I, mom, etot, T
