"""Python binding of librtmm.so (the C ABI in include/rtmm.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Torch tensors supply device memory and the current stream; they are
checked (device, dtype, contiguity, size) and passed as raw pointers.  If the
library is missing or fails to load, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtmm.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EHIP, RT_ENONFINITE, RT_ESTATE = 0, -1, -2, -3, -4, -5
F64, F32 = 0, 1
SRC_TAPE = 10  # doubles per cell of a source tape (RT_SRC_TAPE)
UPWIND1, PLM_VL2 = 0, 1
MESH_PLM, MESH_ADJOINT = 1, 2
K_MAX = 128
NDIAG = 10

DIAG_NAMES = ("gas_energy", "rad_energy", "gas_mom_x", "gas_mom_y", "gas_mom_z", "rad_mom_x", "rad_mom_y",
              "rad_mom_z", "min_I", "n_nonfinite")


class RTError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("c_red", ctypes.c_double), ("c_light", ctypes.c_double), ("a_rad", ctypes.c_double),
                ("cv", ctypes.c_double), ("dt", ctypes.c_double), ("dtype", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


class _Angles(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("layout", ctypes.c_int32), ("dir", ctypes.c_void_p),
                ("weight", ctypes.c_void_p)]


CELL_BOUNDARY, CELL_EMITTER = 1, 2
ANGLES_GENERAL, ANGLES_ANTIPODAL, ANGLES_ANTIPODAL_ADJACENT = 0, 1, 2


_lib = None

_SIGS = {
    "rt_mesh_upload": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32] +
                      [ctypes.c_void_p] * 9 + [ctypes.c_double, ctypes.c_void_p],
    "rt_mesh_free": [ctypes.c_void_p],
    "rt_mesh_info": [ctypes.c_void_p] * 6,
    "rt_mesh_geometry": [ctypes.c_void_p] * 4,
    "rt_transport_step": [ctypes.c_void_p] * 7,
    "rt_source_implicit": [ctypes.c_void_p] * 12,
    "rt_step": [ctypes.c_void_p] * 14,
    "rt_step_taped": [ctypes.c_void_p] * 16,
    "rt_gradient": [ctypes.c_void_p] * 6,
    "rt_step_adjoint": [ctypes.c_void_p] * 17,
    "rt_step_adjoint_run": [ctypes.c_void_p] * 3 + [ctypes.c_int32] + [ctypes.c_void_p] * 12,
    "rt_flux_loss": [ctypes.c_void_p] * 8,
    "rt_flux_loss_noalloc": [ctypes.c_void_p] * 8,
    "rt_diagnostics": [ctypes.c_void_p] * 9,
    "rt_moments": [ctypes.c_void_p] * 6,
    "rt_angles_layout": [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "rt_angles_check": [ctypes.c_void_p, ctypes.c_void_p],
    "rt_angles_release": [ctypes.c_void_p],
    "rt_marked_upload": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64] + [ctypes.c_void_p] * 5
                        + [ctypes.c_double, ctypes.c_void_p],
    "rt_marked_free": [ctypes.c_void_p],
    "rt_source_implicit_mg": [ctypes.c_void_p] * 3 + [ctypes.c_int32] + [ctypes.c_void_p] * 10,
    "rt_source_implicit_kT": [ctypes.c_void_p] * 10 + [ctypes.c_double] * 3 + [ctypes.c_void_p] * 2,
    "rt_step_kT": [ctypes.c_void_p] * 12 + [ctypes.c_double] * 3 + [ctypes.c_void_p] * 2,
    "rt_step_mg": [ctypes.c_void_p] * 3 + [ctypes.c_int32] + [ctypes.c_void_p] * 12,
    "rt_marked_apply": [ctypes.c_void_p] * 10,
}


def lib():
    """Load librtmm.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2002_08377_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.rt_strerror.argtypes = [ctypes.c_int]
        L.rt_strerror.restype = ctypes.c_char_p
        L.rt_last_error.argtypes = []
        L.rt_last_error.restype = ctypes.c_char_p
        L.rt_version.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(fn, rc):
    if rc != RT_OK:
        L = lib()
        raise RTError(fn, rc, f"{L.rt_strerror(rc).decode()}: {L.rt_last_error().decode()}")


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, shape, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def torch_dtype(dtype: int):
    return torch.float32 if dtype == F32 else torch.float64


def angles_layout(dirs, weights) -> int:
    """The library's classification of a host angle set (one of the ANGLES_* values)."""
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    out = ctypes.c_int32(-1)
    _check("rt_angles_layout", lib().rt_angles_layout(int(d.shape[0]), d.ctypes.data_as(ctypes.c_void_p),
                                                     w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)))
    return out.value


class AngleSet:
    """Directions [K,3] and weights [K] resident on the device (float64), with their layout.

    The layout is detected from the host arrays unless given.  An antipodal layout is then
    verified by the library against the device copies (rt_angles_check), which raises
    RTError for a false claim; the claim is released when the set is freed."""

    def __init__(self, dirs, weights, device="cuda", layout=None, stream=None):
        self.layout = angles_layout(dirs, weights) if layout is None else int(layout)
        self.dirs = torch.as_tensor(np.ascontiguousarray(dirs, dtype=np.float64), device=device)
        self.weights = torch.as_tensor(np.ascontiguousarray(weights, dtype=np.float64), device=device)
        self.K = int(self.dirs.shape[0])
        self.c = _Angles(self.K, self.layout, self.dirs.data_ptr(), self.weights.data_ptr())
        self._checked = False
        _check("rt_angles_check", lib().rt_angles_check(ctypes.byref(self.c), _stream(stream)))
        self._checked = True

    def free(self):
        """Forget the library's record of this set's verified layout."""
        if getattr(self, "_checked", False) and _lib is not None:
            _lib.rt_angles_release(ctypes.byref(self.c))
            self._checked = False

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Mesh:
    """An uploaded mesh (owns the library's rt_mesh)."""

    def __init__(self, gen, com, vol, mesh_vel, face_cells, face_shift, face_area, face_normal, face_centroid,
                 box, k_max, flags=0, stream=None):
        L = lib()
        arrs = dict(gen=_host(gen, np.float64), com=_host(com, np.float64), vol=_host(vol, np.float64),
                    w=_host(mesh_vel, np.float64), fc=_host(face_cells, np.int32), fs=_host(face_shift, np.int8),
                    fa=_host(face_area, np.float64), fn=_host(face_normal, np.float64),
                    fcen=_host(face_centroid, np.float64))
        N, F = arrs["gen"].shape[0], arrs["fc"].shape[0]
        ptr = ctypes.c_void_p()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        rc = L.rt_mesh_upload(ctypes.byref(ptr), N, F, int(k_max), int(flags), p(arrs["gen"]), p(arrs["com"]),
                              p(arrs["vol"]), p(arrs["w"]), p(arrs["fc"]), p(arrs["fs"]), p(arrs["fa"]),
                              p(arrs["fn"]), p(arrs["fcen"]), float(box), _stream(stream))
        _check("rt_mesh_upload", rc)
        self._ptr = ptr
        self.n_cells, self.n_faces, self.k_max, self.flags = N, F, int(k_max), int(flags)

    @classmethod
    def from_inputs(cls, mesh, mesh_vel, k_max, flags=0, stream=None):
        """Upload a mesh object with the attributes of the input generator's Mesh."""
        return cls(mesh.gen, mesh.com, mesh.vol, mesh_vel, mesh.face_cells, mesh.face_shift, mesh.face_area,
                   mesh.face_normal, mesh.face_centroid, mesh.box, k_max, flags, stream)

    @property
    def ptr(self):
        if self._ptr is None:
            raise RuntimeError("mesh was freed")
        return self._ptr

    def free(self):
        if getattr(self, "_ptr", None) is not None and _lib is not None:
            _lib.rt_mesh_free(self._ptr)
        self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        n, f, h = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        k, fl = ctypes.c_int32(), ctypes.c_int32()
        _check("rt_mesh_info", lib().rt_mesh_info(self.ptr, ctypes.byref(n), ctypes.byref(f), ctypes.byref(h),
                                                   ctypes.byref(k), ctypes.byref(fl)))
        return dict(n_cells=n.value, n_faces=f.value, n_half_faces=h.value, k_max=k.value, flags=fl.value)

    def geometry(self, stream=None):
        """(face normal speeds [F], volume rates [N]) as float64 device tensors."""
        wn = torch.empty(self.n_faces, dtype=torch.float64, device="cuda")
        D = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        _check("rt_mesh_geometry", lib().rt_mesh_geometry(self.ptr, ctypes.c_void_p(wn.data_ptr()),
                                                           ctypes.c_void_p(D.data_ptr()), _stream(stream)))
        return wn, D


class MarkedCells:
    """Boundary and emitter cells uploaded to the library (owns the rt_marked)."""

    def __init__(self, n_cells, cells, kinds, T_eff, direction, cos_open, tau, stream=None):
        L = lib()
        arrs = dict(cell=_host(cells, np.int32), kind=_host(kinds, np.int32), T=_host(T_eff, np.float64),
                    d=_host(direction, np.float64), co=_host(cos_open, np.float64))
        n = arrs["cell"].shape[0]
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
        ptr = ctypes.c_void_p()
        rc = L.rt_marked_upload(ctypes.byref(ptr), int(n_cells), n, p(arrs["cell"]), p(arrs["kind"]), p(arrs["T"]),
                                p(arrs["d"]), p(arrs["co"]), float(tau), _stream(stream))
        _check("rt_marked_upload", rc)
        self._ptr = ptr
        self.n, self.n_cells = n, int(n_cells)

    @property
    def ptr(self):
        if self._ptr is None:
            raise RuntimeError("marked cells were freed")
        return self._ptr

    def free(self):
        if getattr(self, "_ptr", None) is not None and _lib is not None:
            _lib.rt_marked_free(self._ptr)
        self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def marked_apply(mesh, params, angles, marked, I, rho, mom, etot, kP, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    f = torch.float64
    rc = lib().rt_marked_apply(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), marked.ptr,
                               _dev(I, td, (N, K), "I"), _dev(rho, f, (N,), "rho"), _dev(mom, f, (N, 3), "mom"),
                               _dev(etot, f, (N,), "etot"), _dev(kP, f, (N,), "kP"), _stream(stream))
    _check("rt_marked_apply", rc)


def source_implicit_kT(mesh, params, angles, I, rho, mom, etot, kP0, kJ0, ks, T_ref, bP, bJ, T_new=None,
                       stream=None):
    """Source with power-law opacities kX(T) = kX0 (T/T_ref)^bX at T^{n+1}."""
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_source_implicit_kT(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I, td, (N, K), "I"),
                                     *_gas(mesh, rho, mom, etot, kP0, kJ0, ks), float(T_ref), float(bP), float(bJ),
                                     _dev(T_new, torch.float64, (N,), "T_new", True), _stream(stream))
    _check("rt_source_implicit_kT", rc)


def step_kT(mesh, params, angles, I_in, I_out, vol, rho, mom, etot, kP0, kJ0, ks, T_ref, bP, bJ, T_new=None,
            stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_step_kT(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I_in, td, (N, K), "I_in"),
                          _dev(I_out, td, (N, K), "I_out"), _dev(vol, torch.float64, (N,), "vol"),
                          *_gas(mesh, rho, mom, etot, kP0, kJ0, ks), float(T_ref), float(bP), float(bJ),
                          _dev(T_new, torch.float64, (N,), "T_new", True), _stream(stream))
    _check("rt_step_kT", rc)


def _gas_mg(mesh, G, group_weight, rho, mom, etot, kP, kJ, ks):
    N = mesh.n_cells
    f = torch.float64
    return (_dev(group_weight, f, (G,), "group_weight"), _dev(rho, f, (N,), "rho"), _dev(mom, f, (N, 3), "mom"),
            _dev(etot, f, (N,), "etot"), _dev(kP, f, (G, N), "kP"), _dev(kJ, f, (G, N), "kJ"),
            _dev(ks, f, (G, N), "ks"))


def source_implicit_mg(mesh, params, angles, group_weight, I, rho, mom, etot, kP, kJ, ks, T_new=None, stream=None):
    """Multigroup source: I [G, N, K] (group-major), kP/kJ/ks [G, N], group_weight [G]."""
    N, K = _shapes(mesh, angles)
    G = int(I.shape[0])
    td = torch_dtype(params.dtype)
    wg, rho_, mom_, etot_, kP_, kJ_, ks_ = _gas_mg(mesh, G, group_weight, rho, mom, etot, kP, kJ, ks)
    rc = lib().rt_source_implicit_mg(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), G, wg,
                                     _dev(I, td, (G, N, K), "I"), rho_, mom_, etot_, kP_, kJ_, ks_,
                                     _dev(T_new, torch.float64, (N,), "T_new", True), _stream(stream))
    _check("rt_source_implicit_mg", rc)


def step_mg(mesh, params, angles, group_weight, I_in, I_out, vol, rho, mom, etot, kP, kJ, ks, T_new=None,
            stream=None):
    N, K = _shapes(mesh, angles)
    G = int(I_in.shape[0])
    td = torch_dtype(params.dtype)
    wg, rho_, mom_, etot_, kP_, kJ_, ks_ = _gas_mg(mesh, G, group_weight, rho, mom, etot, kP, kJ, ks)
    rc = lib().rt_step_mg(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), G, wg,
                          _dev(I_in, td, (G, N, K), "I_in"), _dev(I_out, td, (G, N, K), "I_out"),
                          _dev(vol, torch.float64, (N,), "vol"), rho_, mom_, etot_, kP_, kJ_, ks_,
                          _dev(T_new, torch.float64, (N,), "T_new", True), _stream(stream))
    _check("rt_step_mg", rc)


def make_params(c_red, c_light, a_rad, cv, dt, dtype=F64, scheme=UPWIND1) -> Params:
    return Params(float(c_red), float(c_light), float(a_rad), float(cv), float(dt), int(dtype), int(scheme))


def _shapes(mesh, angles):
    return mesh.n_cells, angles.K


def transport_step(mesh, params, angles, I_in, I_out, vol, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_transport_step(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c),
                                 _dev(I_in, td, (N, K), "I_in"), _dev(I_out, td, (N, K), "I_out"),
                                 _dev(vol, torch.float64, (N,), "vol"), _stream(stream))
    _check("rt_transport_step", rc)


def _gas(mesh, rho, mom, etot, kP, kJ, ks):
    N = mesh.n_cells
    f = torch.float64
    return (_dev(rho, f, (N,), "rho"), _dev(mom, f, (N, 3), "mom"), _dev(etot, f, (N,), "etot"),
            _dev(kP, f, (N,), "kP"), _dev(kJ, f, (N,), "kJ"), _dev(ks, f, (N,), "ks"))


def source_implicit(mesh, params, angles, I, rho, mom, etot, kP, kJ, ks, T_new=None, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_source_implicit(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I, td, (N, K), "I"),
                                  *_gas(mesh, rho, mom, etot, kP, kJ, ks),
                                  _dev(T_new, torch.float64, (N,), "T_new", True), _stream(stream))
    _check("rt_source_implicit", rc)


def step(mesh, params, angles, I_in, I_out, vol, rho, mom, etot, kP, kJ, ks, T_new=None, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_step(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I_in, td, (N, K), "I_in"),
                       _dev(I_out, td, (N, K), "I_out"), _dev(vol, torch.float64, (N,), "vol"),
                       *_gas(mesh, rho, mom, etot, kP, kJ, ks), _dev(T_new, torch.float64, (N,), "T_new", True),
                       _stream(stream))
    _check("rt_step", rc)


def step_taped(mesh, params, angles, I_in, I_out, I_star, vol, rho, mom, etot, kP, kJ, ks, T_new=None,
               src_tape=None, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_step_taped(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I_in, td, (N, K), "I_in"),
                             _dev(I_out, td, (N, K), "I_out"), _dev(I_star, td, (N, K), "I_star", True),
                             _dev(vol, torch.float64, (N,), "vol"), *_gas(mesh, rho, mom, etot, kP, kJ, ks),
                             _dev(T_new, torch.float64, (N,), "T_new", True),
                             _dev(src_tape, torch.float64, (N, SRC_TAPE), "src_tape", True), _stream(stream))
    _check("rt_step_taped", rc)


def gradient(mesh, params, angles, I, grad, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_gradient(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I, td, (N, K), "I"),
                           _dev(grad, td, (N, 3, K), "grad"), _stream(stream))
    _check("rt_gradient", rc)


def step_adjoint(mesh, params, angles, I_star, vol_n, rho, mom_n, etot_n, kP, kJ, ks, lamI, lamE, lamM,
                 dkP=None, dkJ=None, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    f = torch.float64
    rc = lib().rt_step_adjoint(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c),
                               _dev(I_star, td, (N, K), "I_star"), _dev(vol_n, f, (N,), "vol_n"),
                               _dev(rho, f, (N,), "rho"), _dev(mom_n, f, (N, 3), "mom_n"),
                               _dev(etot_n, f, (N,), "etot_n"), _dev(kP, f, (N,), "kP"), _dev(kJ, f, (N,), "kJ"),
                               _dev(ks, f, (N,), "ks"), _dev(lamI, td, (N, K), "lamI"), _dev(lamE, f, (N,), "lamE"),
                               _dev(lamM, f, (N, 3), "lamM"), _dev(dkP, f, (N,), "dkP", True),
                               _dev(dkJ, f, (N,), "dkJ", True), _stream(stream))
    _check("rt_step_adjoint", rc)


def step_adjoint_run(mesh, params, angles, I_next, src_tape, rho, kP, kJ, ks, lamI, lamE, lamM, dkP=None,
                     dkJ=None, stream=None):
    """Reverse of len(I_next) taped steps (lists of per-step tensors, entry i for step i: its
    output intensities and its source tape)."""
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    f = torch.float64
    n = len(I_next)
    if len(src_tape) != n:
        raise ValueError("I_next and src_tape need one entry per step")
    arr = lambda xs: (ctypes.c_void_p * max(n, 1))(*xs)
    ps = arr([_dev(x, td, (N, K), f"I_next[{i}]") for i, x in enumerate(I_next)])
    pt = arr([_dev(x, f, (N, SRC_TAPE), f"src_tape[{i}]") for i, x in enumerate(src_tape)])
    rc = lib().rt_step_adjoint_run(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), n, ps, pt,
                                   _dev(rho, f, (N,), "rho"), _dev(kP, f, (N,), "kP"), _dev(kJ, f, (N,), "kJ"),
                                   _dev(ks, f, (N,), "ks"), _dev(lamI, td, (N, K), "lamI"),
                                   _dev(lamE, f, (N,), "lamE"), _dev(lamM, f, (N, 3), "lamM"),
                                   _dev(dkP, f, (N,), "dkP", True), _dev(dkJ, f, (N,), "dkJ", True), _stream(stream))
    _check("rt_step_adjoint_run", rc)


def flux_loss(mesh, params, angles, I, face_weight, loss, seed=None, stream=None):
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_flux_loss(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I, td, (N, K), "I"),
                            _dev(face_weight, torch.float64, (mesh.n_faces,), "face_weight"),
                            _dev(loss, torch.float64, (1,), "loss"), _dev(seed, td, (N, K), "seed", True),
                            _stream(stream))
    _check("rt_flux_loss", rc)


def flux_loss_noalloc(mesh, params, angles, I, face_weight, loss, seed=None, stream=None):
    """rt_flux_loss_noalloc: flux_loss with the partial sums in the library's static scratch."""
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_flux_loss_noalloc(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c),
                                    _dev(I, td, (N, K), "I"),
                                    _dev(face_weight, torch.float64, (mesh.n_faces,), "face_weight"),
                                    _dev(loss, torch.float64, (1,), "loss"), _dev(seed, td, (N, K), "seed", True),
                                    _stream(stream))
    _check("rt_flux_loss_noalloc", rc)


def moments(mesh, params, angles, I, out, stream=None):
    """Per-cell angle moments into out [N, 10] (FP64): E_r, F_r (3), P_r (xx, yy, zz, xy, xz, yz)."""
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    rc = lib().rt_moments(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I, td, (N, K), "I"),
                          _dev(out, torch.float64, (N, 10), "moments"), _stream(stream))
    _check("rt_moments", rc)


def diagnostics(mesh, params, angles, I, vol, etot, mom, stream=None, allow_nonfinite=False):
    """Returns the RT_NDIAG totals as a numpy array (synchronises the stream)."""
    N, K = _shapes(mesh, angles)
    td = torch_dtype(params.dtype)
    out = np.zeros(NDIAG)
    rc = lib().rt_diagnostics(mesh.ptr, ctypes.byref(params), ctypes.byref(angles.c), _dev(I, td, (N, K), "I"),
                              _dev(vol, torch.float64, (N,), "vol"), _dev(etot, torch.float64, (N,), "etot"),
                              _dev(mom, torch.float64, (N, 3), "mom"), out.ctypes.data_as(ctypes.c_void_p),
                              _stream(stream))
    if rc == RT_ENONFINITE and allow_nonfinite:
        return out
    _check("rt_diagnostics", rc)
    return out
