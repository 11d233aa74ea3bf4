"""The C ABI without a GPU: the library loads, exports every function rtmm.h declares,
and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2002_08377_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rtmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    names = _declared()
    assert len(names) >= 14
    L = rt.lib()
    for n in names:
        assert hasattr(L, n), n


def test_version_and_strerror():
    L = rt.lib()
    assert L.rt_version() == 1
    assert L.rt_strerror(rt.RT_EINVAL) == b"invalid argument"
    assert L.rt_strerror(12345) == b"unknown error"


def test_upload_rejects_bad_meshes_on_the_host():
    L = rt.lib()
    out = ctypes.c_void_p()
    rc = L.rt_mesh_upload(ctypes.byref(out), 0, 0, 8, 0, *([None] * 9), 1.0, None)
    assert rc == rt.RT_EINVAL and out.value is None
    assert b"n_cells" in L.rt_last_error()
    # a two-cell "mesh" whose faces do not close
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    gen = np.zeros((2, 3)); com = np.zeros((2, 3)); vol = np.ones(2); w = np.zeros((2, 3))
    fc = np.array([[0, 1]], dtype=np.int32); fs = np.zeros((1, 3), dtype=np.int8)
    fa = np.ones(1); fn = np.array([[1.0, 0, 0]]); fcen = np.zeros((1, 3))
    rc = L.rt_mesh_upload(ctypes.byref(out), 2, 1, 8, 0, p(gen), p(com), p(vol), p(w), p(fc), p(fs), p(fa), p(fn),
                          p(fcen), 1.0, None)
    assert rc == rt.RT_EINVAL and b"not closed" in L.rt_last_error()
    fc_bad = np.array([[0, 2]], dtype=np.int32)
    rc = L.rt_mesh_upload(ctypes.byref(out), 2, 1, 8, 0, p(gen), p(com), p(vol), p(w), p(fc_bad), p(fs), p(fa),
                          p(fn), p(fcen), 1.0, None)
    assert rc == rt.RT_EINVAL and b"invalid cells" in L.rt_last_error()
    rc = L.rt_mesh_upload(ctypes.byref(out), 2, 1, 500, 0, p(gen), p(com), p(vol), p(w), p(fc), p(fs), p(fa),
                          p(fn), p(fcen), 1.0, None)
    assert rc == rt.RT_EINVAL and b"k_max" in L.rt_last_error()


def test_calls_reject_null_mesh():
    """Every call that takes a mesh refuses a NULL one on the host, before any device work."""
    L = rt.lib()
    prm = rt.make_params(1.0, 1.0, 1.0, 1.5, 0.1)
    rc = L.rt_step(None, ctypes.byref(prm), None, *([None] * 11))
    assert rc == rt.RT_EINVAL
    for name in ("rt_transport_step", "rt_source_implicit", "rt_step_taped", "rt_gradient", "rt_step_adjoint",
                 "rt_step_adjoint_run",
                 "rt_flux_loss", "rt_moments", "rt_diagnostics", "rt_source_implicit_mg", "rt_step_mg",
                 "rt_source_implicit_kT", "rt_step_kT", "rt_marked_apply"):
        fn = getattr(L, name)
        args = []
        for i, t in enumerate(fn.argtypes):
            if i == 1:
                args.append(ctypes.byref(prm))
            elif t is ctypes.c_double:
                args.append(1.0)
            elif t in (ctypes.c_int, ctypes.c_int32, ctypes.c_int64):
                args.append(1)
            else:
                args.append(None)
        assert fn(*args) == rt.RT_EINVAL, name
    assert L.rt_mesh_free(None) == rt.RT_OK


def test_params_layout_matches_header():
    # c_red, c_light, a_rad, cv, dt (5 doubles) then dtype, scheme (2 int32)
    assert ctypes.sizeof(rt.Params) == 48
    assert rt.Params.dtype.offset == 40 and rt.Params.scheme.offset == 44
    assert ctypes.sizeof(rt._Angles) == 24 and rt._Angles.layout.offset == 4 and rt._Angles.dir.offset == 8


def test_angle_layout_detection():
    from paper_2002_08377_amd import inputs as inp
    for K in (8, 24, 48, 80):
        d, w = inp.angle_set(K)
        assert rt.angles_layout(d, w) == rt.ANGLES_ANTIPODAL
        # any perturbation or reordering breaks the exact antipodal layout
        d2 = d.copy(); d2[K - 1] = -d2[0]
        assert rt.angles_layout(d2, w) == rt.ANGLES_GENERAL
        w2 = w.copy(); w2[0] *= 1.0 + 1e-15
        assert rt.angles_layout(d, w2) == rt.ANGLES_GENERAL
        assert rt.angles_layout(d[:-1], w[:-1]) == rt.ANGLES_GENERAL
        # antipodes side by side
        perm = inp.adjacent_pair_order(K)
        da, wa = d[perm], w[perm]
        assert rt.angles_layout(da, wa) == rt.ANGLES_ANTIPODAL_ADJACENT
        da2 = da.copy(); da2[3] = da2[2]
        assert rt.angles_layout(da2, wa) == rt.ANGLES_GENERAL
        wa2 = wa.copy(); wa2[K - 1] *= 1.0 + 1e-15
        assert rt.angles_layout(da, wa2) == rt.ANGLES_GENERAL
        # swapping two pairs keeps every pair adjacent
        sw = np.arange(K); sw[[0, 1, 2, 3]] = [2, 3, 0, 1]
        assert rt.angles_layout(da[sw], wa[sw]) == rt.ANGLES_ANTIPODAL_ADJACENT
    # a two-angle set satisfies both definitions: the K/2 one is reported
    d2 = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    assert rt.angles_layout(d2, np.array([0.5, 0.5])) == rt.ANGLES_ANTIPODAL
    L = rt.lib()
    out = ctypes.c_int32()
    assert L.rt_angles_layout(0, None, None, ctypes.byref(out)) == rt.RT_EINVAL


def test_marked_upload_validates_on_the_host():
    """Every rejection happens before any device call (this test needs no GPU)."""
    L = rt.lib()
    out = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    cell = np.array([0, 3], dtype=np.int32)
    kind = np.array([rt.CELL_BOUNDARY, rt.CELL_EMITTER], dtype=np.int32)
    T = np.array([1.0, 2.0])
    d = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    co = np.array([0.9, 0.5])

    def up(n_cells=10, cell=cell, kind=kind, T=T, d=d, co=co, tau=0.1):
        rc = L.rt_marked_upload(ctypes.byref(out), n_cells, cell.shape[0], p(cell), p(kind), p(T), p(d), p(co),
                                tau, None)
        return rc, L.rt_last_error()

    assert up(n_cells=3)[0] == rt.RT_EINVAL                       # n > n_cells
    rc, msg = up(n_cells=4, cell=np.array([0, 4], dtype=np.int32))
    assert rc == rt.RT_EINVAL and b"out of range" in msg
    rc, msg = up(cell=np.array([3, 3], dtype=np.int32))
    assert rc == rt.RT_EINVAL and b"marked twice" in msg
    rc, msg = up(kind=np.array([1, 7], dtype=np.int32))
    assert rc == rt.RT_EINVAL and b"kind" in msg
    rc, msg = up(T=np.array([1.0, -1.0]))
    assert rc == rt.RT_EINVAL and b"T_eff" in msg
    rc, msg = up(d=np.array([[0.0, 1.0, 0.0], [1.0, 1.0, 0.0]]))
    assert rc == rt.RT_EINVAL and b"unit" in msg
    rc, msg = up(co=np.array([0.9, np.nan]))
    assert rc == rt.RT_EINVAL and b"NaN" in msg
    rc, msg = up(tau=0.0)
    assert rc == rt.RT_EINVAL and b"tau" in msg
    assert out.value is None
    assert L.rt_marked_free(None) == rt.RT_OK


def test_angles_check_rejects_bad_claims_on_the_host():
    """rt_angles_check refuses NULL sets, K out of range and unknown layouts before it
    reads any device memory (the contents of a set, unit directions and normalised weights,
    are checked on its device copy: a GPU test covers that), and releasing a claim that was
    never recorded does nothing."""
    L = rt.lib()
    assert L.rt_angles_check(None, None) == rt.RT_EINVAL
    assert L.rt_angles_release(None) == rt.RT_EINVAL
    bogus = 0x1000  # never dereferenced on these paths
    for K, layout, d, w in ((0, 0, bogus, bogus), (rt.K_MAX + 1, 0, bogus, bogus), (8, 1, None, bogus),
                            (8, 7, bogus, bogus)):
        a = rt._Angles(K, layout, d, w)
        assert L.rt_angles_check(ctypes.byref(a), None) == rt.RT_EINVAL, (K, layout)
    a = rt._Angles(8, rt.ANGLES_GENERAL, bogus, bogus)
    assert L.rt_angles_release(ctypes.byref(a)) == rt.RT_OK


def test_last_error_is_per_thread():
    """rt_last_error() returns the calling thread's own last failure: two threads that fail in
    different ways, many times over and interleaved, each read back their own message."""
    import threading
    L = rt.lib()
    out = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    gen = np.zeros((2, 3)); com = np.zeros((2, 3)); vol = np.ones(2); w = np.zeros((2, 3))
    fc_bad = np.array([[0, 2]], dtype=np.int32); fs = np.zeros((1, 3), dtype=np.int8)
    fa = np.ones(1); fn = np.array([[1.0, 0, 0]]); fcen = np.zeros((1, 3))
    results = {}
    barrier = threading.Barrier(2)

    def empty_mesh():
        msgs = set()
        barrier.wait()
        for _ in range(2000):
            assert L.rt_mesh_upload(ctypes.byref(ctypes.c_void_p()), 0, 0, 8, 0, *([None] * 9), 1.0, None) \
                == rt.RT_EINVAL
            msgs.add(L.rt_last_error())
        results["empty"] = msgs

    def bad_cells():
        msgs = set()
        barrier.wait()
        for _ in range(2000):
            assert L.rt_mesh_upload(ctypes.byref(ctypes.c_void_p()), 2, 1, 8, 0, p(gen), p(com), p(vol), p(w),
                                    p(fc_bad), p(fs), p(fa), p(fn), p(fcen), 1.0, None) == rt.RT_EINVAL
            msgs.add(L.rt_last_error())
        results["cells"] = msgs

    threads = [threading.Thread(target=empty_mesh), threading.Thread(target=bad_cells)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert len(results["empty"]) == 1 and b"n_cells" in next(iter(results["empty"]))
    assert len(results["cells"]) == 1 and b"invalid cells" in next(iter(results["cells"]))
    assert out.value is None


def _lattice(n=3):
    """A valid periodic cubic lattice of n^3 unit-box cells (three faces per cell), host arrays
    in the argument order of rt_mesh_upload."""
    h = 1.0 / n
    N, F = n ** 3, 3 * n ** 3
    gen = np.zeros((N, 3)); vel = np.zeros((N, 3)); vol = np.full(N, h ** 3)
    fc = np.zeros((F, 2), dtype=np.int32); fs = np.zeros((F, 3), dtype=np.int8)
    fa = np.full(F, h * h); fn = np.zeros((F, 3)); fcen = np.zeros((F, 3))
    for z in range(n):
        for y in range(n):
            for x in range(n):
                c = (x, y, z)
                i = x + n * (y + n * z)
                gen[i] = [(v + 0.5) * h for v in c]
                vel[i] = [0.1, 0.05, 0.0]
                for a in range(3):
                    cn = list(c)
                    cn[a] = (c[a] + 1) % n
                    f = 3 * i + a
                    fc[f] = (i, cn[0] + n * (cn[1] + n * cn[2]))
                    fs[f, a] = 1 if c[a] + 1 == n else 0
                    fn[f, a] = 1.0
                    fcen[f] = gen[i]
                    fcen[f, a] += 0.5 * h
    return dict(gen=gen, com=gen.copy(), vol=vol, vel=vel, fc=fc, fs=fs, fa=fa, fn=fn, fcen=fcen)


def _upload(m, k_max=8, flags=0, box=1.0):
    L = rt.lib()
    out = ctypes.c_void_p()
    p = lambda a: None if a is None else np.ascontiguousarray(a).ctypes.data_as(ctypes.c_void_p)
    keep = {k: (None if v is None else np.ascontiguousarray(v)) for k, v in m.items()}
    N, F = keep["gen"].shape[0] if keep["gen"] is not None else 27, keep["fc"].shape[0] if keep["fc"] is not None else 81
    rc = L.rt_mesh_upload(ctypes.byref(out), N, F, k_max, flags, p(keep["gen"]), p(keep["com"]), p(keep["vol"]),
                          p(keep["vel"]), p(keep["fc"]), p(keep["fs"]), p(keep["fa"]), p(keep["fn"]), p(keep["fcen"]),
                          box, None)
    return rc, out.value, L.rt_last_error()


def _mutate(key, index, value):
    def f(m):
        m[key] = m[key].copy()
        m[key][index] = value
        return m
    return f


MESH_DEFECTS = [
    ("NaN position", _mutate("gen", (4, 1), np.nan), b"gen_pos"),
    ("infinite centre of mass", _mutate("com", (7, 0), np.inf), b"com"),
    ("NaN velocity", _mutate("vel", (0, 2), np.nan), b"mesh_vel"),
    ("NaN centroid", _mutate("fcen", (10, 0), np.nan), b"face_centroid"),
    ("zero volume", _mutate("vol", 3, 0.0), b"volume"),
    ("NaN volume", _mutate("vol", 5, np.nan), b"volume"),
    ("negative area", _mutate("fa", 2, -1e-3), b"area"),
    ("NaN area", _mutate("fa", 8, np.nan), b"area"),
    ("normal not unit", _mutate("fn", (6, 0), 0.9), b"not unit"),
    ("NaN normal", _mutate("fn", (6, 1), np.nan), b"not unit"),
    ("cell out of range", _mutate("fc", (9, 1), 27), b"invalid cells"),
    ("negative cell", _mutate("fc", (9, 0), -1), b"invalid cells"),
    ("face of a cell with itself", _mutate("fc", (12, 1), 4), b"invalid cells"),
    ("shift outside {-1,0,1}", _mutate("fs", (5, 0), 2), b"shift"),
    ("faces that do not close", _mutate("fa", 13, 1.5 / 9.0), b"not closed"),
    ("a NULL array", lambda m: dict(m, fcen=None), b"NULL"),
]


@pytest.mark.parametrize("name,mutate,why", MESH_DEFECTS, ids=[d[0] for d in MESH_DEFECTS])
def test_upload_refuses_each_mesh_defect_on_the_host(name, mutate, why):
    """A valid 3^3 periodic lattice with one defect at a time: every defect is refused with
    RT_EINVAL before any device memory is touched (this runs without a GPU), *out stays NULL
    and the message names the defect."""
    m = _lattice()
    assert (m["fc"][12] == [4, 5]).all()  # face 12 joins cells 4 and 5, so (4, 4) is a self-face
    rc, out, msg = _upload(mutate(m))
    assert rc == rt.RT_EINVAL and out is None, (name, rc, msg)
    assert why in msg, (name, msg)


@pytest.mark.parametrize("kw,why", [(dict(k_max=0), b"k_max"), (dict(k_max=129), b"k_max"),
                                    (dict(flags=8), b"flags"), (dict(box=0.0), b"box"),
                                    (dict(box=float("nan")), b"box")])
def test_upload_refuses_bad_scalars_on_the_host(kw, why):
    rc, out, msg = _upload(_lattice(), **kw)
    assert rc == rt.RT_EINVAL and out is None and why in msg, (kw, msg)
