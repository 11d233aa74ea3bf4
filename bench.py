"""Throughput of the radiation step on one MI355X.

Workload (the throughput configuration): a periodic jittered-lattice Voronoi
mesh of 128^3 = 2,097,152 cells, 80 discrete ordinates, first-order upwind
transport plus the implicit source, 50 steps; inputs seeded and synthetic,
resident in HBM before timing starts.  Both precision forms run on the same
GPU from the same initial state: FP32 intensities/transport with the FP64
source solve and bookkeeping (the headline `value`) and all-FP64.

Prints ONE JSON line.  `value` = cell-angle updates per second of the FP32
form (N cells * K angles * steps / wall time of the timed steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU peak available to these kernels: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one FP32 or FP64
# operation per lane per clock (an FMA counts once).  Packed FP32 math is disabled at compile time, so
# FP32 and FP64 share this peak (the FP64 vector rate, 78.6 TFLOP/s counting an FMA as two flops).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic operations per cell-angle of a first-order step: about 6 per face and angle with each
# face's flux computed once (3 for s = (dt cbar A n).n_k - dt A w.n, 2 for the upwind choice, 1 for the
# flux), and about 38 for the implicit source (boost, comoving sums, update, bookkeeping).
SOURCE_OPS_PER_CA = 38.0
FACE_OPS_PER_FA = 6.0
WORKLOAD_INDEX = 3  # 128^3 cells x 80 angles x 50 steps


def algorithmic_bytes(N, F, K, dtype):
    """Bytes one fused first-order step must move at minimum: each intensity read and written
    once (N K s_I), each face's cell pair and (A n, A w.n) once, the half-face index (row pointers
    and one signed id per half-face), and 120 B of FP64 cell state (V, D, rho, mom r/w, E_g r/w,
    kP, kJ, ks, V')."""
    sI = 4 if dtype == "f32" else 8
    sg = 4 if dtype == "f32" else 8
    return N * K * 2 * sI + F * (8 + 4 * sg) + (N + 1) * 4 + 2 * F * 4 + 120 * N


def plm_algorithmic_bytes(N, F, K, dtype):
    """Bytes one PLM-VL2 step must move at minimum: stage 1 is a first-order step; the gradient
    reads the half-step intensities and writes three components per cell-angle, with each face's
    cell pair and two 3-vectors of estimator weights; stage 2 is a first-order step that also
    reads the half-step intensities and the gradient, with each face's two extrapolation offsets."""
    sI = 4 if dtype == "f32" else 8
    sg = 4 if dtype == "f32" else 8
    first = algorithmic_bytes(N, F, K, dtype)
    gradient = N * K * 4 * sI + F * (8 + 6 * sg)
    stage2 = first + N * K * 4 * sI + F * 6 * sg
    return first + gradient + stage2


def algorithmic_ops(N, F, K):
    return N * K * SOURCE_OPS_PER_CA + F * K * FACE_OPS_PER_FA


# The sources the step kernel is compiled from: its file and every header it includes.
STEP_KERNEL_SOURCES = ("paper_2002_08377_amd/csrc/k_step.hip", "paper_2002_08377_amd/csrc/rt_step_common.h",
                       "paper_2002_08377_amd/csrc/rt_device.h", "paper_2002_08377_amd/csrc/rt_internal.h",
                       "include/rtmm.h")


def kernel_source_hash():
    """Hash of the step kernel's sources: the counter summary is used only while they are unchanged."""
    h = hashlib.sha256()
    for rel in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    ent = data.get("kernels", {}).get(kernel_key)
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def run_form(prob, mesh, angles, dtype_code, steps, warmup, log):
    import torch
    from paper_2002_08377_amd import rt
    st = prob.state
    ph = prob.phys
    params = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, prob.dt, dtype_code, rt.UPWIND1)
    td = rt.torch_dtype(dtype_code)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    # the initial state, kept on the device so the restart below is a device copy (a host upload
    # between the warm-up and the timed steps would leave the GPU idle long enough to clock down)
    init = {"I": d(st.I).to(td).contiguous(), "vol": d(st.vol), "mom": d(st.mom), "etot": d(st.etot)}
    I = init["I"].clone()
    I2 = torch.empty_like(I)
    vol, mom, etot = init["vol"].clone(), init["mom"].clone(), init["etot"].clone()
    rho, kP, kJ, ks = d(st.rho), d(st.kP), d(st.kJ), d(st.ks)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        rt.step(mesh, params, angles, I, I2, vol, rho, mom, etot, kP, kJ, ks, stream=stream)
        I, I2 = I2, I
    # restart from the initial state so both forms advance the same trajectory
    I.copy_(init["I"])
    vol.copy_(init["vol"]); mom.copy_(init["mom"]); etot.copy_(init["etot"])
    del init
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        rt.step(mesh, params, angles, I, I2, vol, rho, mom, etot, kP, kJ, ks, stream=stream)
        ev[i][1].record(stream)
        I, I2 = I2, I
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    diag = rt.diagnostics(mesh, params, angles, I, vol, etot, mom)
    log(f"  dtype={'f32' if dtype_code == rt.F32 else 'f64'}: {wall * 1e3 / steps:.3f} ms/step wall, "
        f"kernel mean {np.mean(kern_ms):.3f} ms, min I {diag[8]:.3e}")
    return dict(wall=wall, kernel_ms=float(np.mean(kern_ms)), I=I.double().cpu().numpy(), diag=diag,
                etot=etot.cpu().numpy())


def run_fwd_adj(log, warmup=1, reps=2, ckpt=8):
    """Forward + adjoint throughput on the checkpointed workload (96^3 cells, 80 angles, 40 steps,
    FP32 transport, checkpoints every 8 steps): cell-angle updates per second of the forward steps,
    the time covering the forward pass, the recompute and the adjoint of all steps.  Beside it the
    same pass with every step taped during the forward pass (no checkpoints, no recompute), which
    holds all 40 steps' records at once, and the FP64 form's checkpointed pass, whose loss and
    gradients the FP32 form's are compared with (normwise: max |difference| / max |FP64|)."""
    import torch
    from paper_2002_08377_amd import autograd as ag
    from paper_2002_08377_amd import inputs as inp
    from paper_2002_08377_amd import rt
    t0 = time.perf_counter()
    p0 = inp.make_problem(4)
    N, K = p0.state.I.shape
    # antipodes stored beside their angles, as in the step measurement (the loss and the
    # gradients do not depend on the storage order)
    p = inp.with_angle_order(p0, inp.adjacent_pair_order(K))
    st, ph = p.state, p.phys
    log(f"fwd+adj workload: {N} cells x {K} angles x {p.steps} steps; inputs built in "
        f"{time.perf_counter() - t0:.1f} s")
    mesh = rt.Mesh.from_inputs(p.mesh, st.mesh_vel, k_max=K, flags=rt.MESH_ADJOINT)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    angles = rt.AngleSet(p.dirs, p.weights)
    systems = {code: ag.RTSystem(mesh, rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, code), angles,
                                 d(st.rho), d(st.ks), d(st.vol)) for code in (rt.F32, rt.F64)}
    fw = d(inp.loss_face_weights(p.mesh, p.seeds["omega"]))
    kap, etot, mom = d(st.kP), d(st.etot), d(st.mom)
    I0 = {rt.F32: d(st.I).float(), rt.F64: d(st.I)}

    def once(every, code):
        x = [t.clone().requires_grad_() for t in (I0[code], kap, etot, mom)]
        system = systems[code]
        IS = ag.rt_steps(*x, system, p.steps, every)[0]
        L = ag.flux_loss(IS, fw, system)
        L.backward()
        return float(L.detach()), x[0].grad, x[1].grad

    def timed(every, code):
        for _ in range(warmup):
            once(every, code)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = once(every, code)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, res, torch.cuda.max_memory_allocated()

    dt, (L32, gI32, gk32), mem = timed(ckpt, rt.F32)
    dt_all, (_, _, gk_all), mem_all = timed(p.steps, rt.F32)
    dt64, (L64, gI64, gk64), mem64 = timed(ckpt, rt.F64)
    nrm = lambda a, b: float((a.double() - b).abs().max() / b.abs().max())
    agree = {"loss": abs(L32 - L64) / abs(L64), "dL_dI0": nrm(gI32, gI64), "dL_dkappa": nrm(gk32, gk64)}
    ok = bool(torch.isfinite(gk32).all() and torch.isfinite(gI32).all())
    angles.free()
    mesh.free()
    log(f"  fwd+adj: {dt * 1e3:.1f} ms per pass of {p.steps} steps (checkpoints every {ckpt}); "
        f"{dt_all * 1e3:.1f} ms with every step taped; FP64 {dt64 * 1e3:.1f} ms; FP32 vs FP64: "
        + ", ".join(f"{k} {v:.1e}" for k, v in agree.items()))
    return {"value": N * K * p.steps / dt, "unit": "cell-angle updates/s", "ms_per_pass": dt * 1e3,
            "workload": f"adjoint_{round(N ** (1 / 3))}c_{K}a", "cells": N, "angles": K, "steps": p.steps,
            "checkpoint_every": ckpt, "dtype": "f32", "angle_order": "antipodes adjacent",
            "gradient_finite": ok, "peak_device_GB": round(mem / 1e9, 2),
            "tape_every_step": {"value": N * K * p.steps / dt_all, "ms_per_pass": dt_all * 1e3,
                                "gradient_finite": bool(torch.isfinite(gk_all).all()),
                                "peak_device_GB": round(mem_all / 1e9, 2)},
            "fp64": {"value": N * K * p.steps / dt64, "ms_per_pass": dt64 * 1e3, "dtype": "f64",
                     "peak_device_GB": round(mem64 / 1e9, 2)},
            "f32_vs_f64": agree}


def run_plm(log):
    """The PLM workload (64^3 cells, 80 angles, 100 van Leer steps, optical depths 1e-3..1e3 per
    cell): throughput of both precision forms, and the total-energy drift over the 100 steps of
    the same workload on a still mesh (with moving faces the gas energy density is not advected
    with the cell volumes, hydrodynamics being outside the step, so only a still mesh conserves
    sum V (E_g + (c/cbar) E_r) exactly)."""
    import torch
    from paper_2002_08377_amd import inputs as inp
    from paper_2002_08377_amd import rt
    p0 = inp.make_problem(1)
    N, K = p0.state.I.shape
    F = p0.mesh.n_faces
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    # both forms with each antipode stored beside its angle (their faster order), as in the step
    # measurement
    p_adj = inp.with_angle_order(p0, inp.adjacent_pair_order(K))
    orders = {"f64": p_adj, "f32": p_adj}
    out = {"workload": f"plm_{round(N ** (1 / 3))}c_{K}a", "cells": N, "angles": K, "steps": p0.steps,
           "scheme": "plm_vl2", "angle_order": "antipodes adjacent"}
    for still in (False, True):
        w = np.zeros_like(p0.state.mesh_vel) if still else p0.state.mesh_vel
        mesh = rt.Mesh.from_inputs(p0.mesh, w, k_max=K, flags=rt.MESH_PLM)
        for name, code in (("f64", rt.F64), ("f32", rt.F32)):
            p = orders[name]
            st, ph = p.state, p.phys
            angles = rt.AngleSet(p.dirs, p.weights)
            prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, code, rt.PLM_VL2)
            td = rt.torch_dtype(code)
            I = d(st.I).to(td)
            I2 = torch.empty_like(I)
            vol, mom, etot = d(st.vol), d(st.mom), d(st.etot)
            rho, kP, kJ, ks = d(st.rho), d(st.kP), d(st.kJ), d(st.ks)
            d0 = rt.diagnostics(mesh, prm, angles, I, vol, etot, mom)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(p.steps):
                rt.step(mesh, prm, angles, I, I2, vol, rho, mom, etot, kP, kJ, ks)
                I, I2 = I2, I
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            d1 = rt.diagnostics(mesh, prm, angles, I, vol, etot, mom)
            if still:
                e0, e1 = d0[0] + d0[1], d1[0] + d1[1]
                out.setdefault("energy_drift_still_mesh", {})[name] = abs(e1 - e0) / e0
            else:
                ms = dt * 1e3 / p.steps
                out[name] = {"value": N * K * p.steps / dt, "unit": "cell-angle updates/s", "ms_per_step": ms,
                             "roofline": _roofline(ms, plm_algorithmic_bytes(N, F, K, name))}
                log(f"  plm {name}: {dt * 1e3 / p.steps:.3f} ms/step")
        mesh.free()
    log(f"  plm energy drift over {p.steps} steps (still mesh): {out['energy_drift_still_mesh']}")
    return out


def _ms_per_call(fn, reps, warmup=2):
    """Mean time of `reps` calls of fn on the current stream (HIP events around the whole run)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _roofline(ms, nbytes, ops=None):
    """HBM roofline of `nbytes` algorithmic bytes in `ms`, with the ALU one of `ops` (if given)
    beside it."""
    t = ms * 1e-3
    hbm = {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_per_launch": int(nbytes)}
    if ops is None:
        return hbm
    alu = {"bound": "alu", "achieved": round(ops / t / 1e12, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "Top/s",
           "frac": round(ops / t / 1e12 / ALU_PEAK_TOPS, 4), "algorithmic_per_launch": int(ops)}
    out = dict(hbm)
    out["other"] = alu
    return out


def run_extensions(prob, mesh, angles, log, reps=5):
    """The extension rows on the throughput mesh (128^3 cells, 80 angles), FP32 transport form:
    multigroup (4 groups: a step of 4 transports plus the multigroup source, and that source alone),
    temperature-dependent opacities (Kramers-like power laws, exponent -3.5: the step and its source
    alone), boundary/emitter cells (1% of the cells marked: one application) and the per-cell
    angle moments (one read of I, 10 doubles written per cell).  Each kernel's
    roofline counts its algorithmic bytes (each value read and written once); the multigroup source
    also its ~38 operations per cell, angle and group.  The kappa(T) source is bound by FP64
    arithmetic (each Newton evaluation re-forms the comoving sums over all angles), whose count
    depends on the cell, so only its HBM fraction is given."""
    import torch
    from paper_2002_08377_amd import rt
    st, ph = prob.state, prob.phys
    N, K = st.I.shape
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, prob.dt, rt.F32)
    rho, ks = d(st.rho), d(st.ks)
    out = {"workload": f"throughput_{round(N ** (1 / 3))}c_{K}a", "cells": N, "angles": K, "dtype": "f32"}

    # multigroup
    G = 4
    wg = d([0.1, 0.2, 0.3, 0.4])
    scale = np.array([0.3, 1.0, 3.0, 10.0])[:, None]
    kPg, kJg, ksg = d(scale * st.kP[None, :]), d(scale * st.kJ[None, :]), d(np.tile(st.ks, (G, 1)))
    Ig = torch.as_tensor(st.I, device="cuda").float().unsqueeze(0).repeat(G, 1, 1).contiguous()
    Ig2 = torch.empty_like(Ig)
    vol, mom, etot = d(st.vol), d(st.mom), d(st.etot)
    bufs = [Ig, Ig2]

    def mg_step():
        rt.step_mg(mesh, prm, angles, wg, bufs[0], bufs[1], vol, rho, mom, etot, kPg, kJg, ksg)
        bufs.reverse()

    ms_step = _ms_per_call(mg_step, reps)
    ms_src = _ms_per_call(lambda: rt.source_implicit_mg(mesh, prm, angles, wg, bufs[0], rho, mom, etot, kPg, kJg,
                                                        ksg), reps)
    src_bytes = G * N * K * 4 * 2 + N * (72 + 24 * G)
    out["multigroup"] = {"groups": G, "ms_per_step": round(ms_step, 4),
                         "value": N * K * G / (ms_step * 1e-3), "unit": "cell-angle-group updates/s",
                         "source_kernel": "k_source_mg", "source_ms": round(ms_src, 4),
                         "roofline": _roofline(ms_src, src_bytes, N * K * G * SOURCE_OPS_PER_CA)}
    log(f"  multigroup ({G} groups): {ms_step:.3f} ms/step, source {ms_src:.3f} ms")
    del Ig, Ig2, bufs, kPg, kJg, ksg

    # temperature-dependent opacities
    I = torch.as_tensor(st.I, device="cuda").float().contiguous()
    I2 = torch.empty_like(I)
    vol, mom, etot = d(st.vol), d(st.mom), d(st.etot)
    kP0, kJ0 = d(st.kP), d(st.kJ)
    law = (1.0, -3.5, -3.5)
    bufs = [I, I2]

    def kT_step():
        rt.step_kT(mesh, prm, angles, bufs[0], bufs[1], vol, rho, mom, etot, kP0, kJ0, ks, *law)
        bufs.reverse()

    ms_step = _ms_per_call(kT_step, reps)
    ms_src = _ms_per_call(lambda: rt.source_implicit_kT(mesh, prm, angles, bufs[0], rho, mom, etot, kP0, kJ0, ks,
                                                        *law), reps)
    out["opacity_T"] = {"law": {"T_ref": law[0], "bP": law[1], "bJ": law[2]}, "ms_per_step": round(ms_step, 4),
                        "value": N * K / (ms_step * 1e-3), "unit": "cell-angle updates/s",
                        "source_kernel": "k_source_kT", "source_ms": round(ms_src, 4),
                        "roofline": _roofline(ms_src, N * K * 4 * 2 + N * 96)}
    log(f"  kappa(T): {ms_step:.3f} ms/step, source {ms_src:.3f} ms")

    # boundary and emitter cells
    rng = np.random.default_rng(2002)
    M = N // 100
    cells = rng.choice(N, M, replace=False)
    kinds = np.where(np.arange(M) % 2 == 0, rt.CELL_BOUNDARY, rt.CELL_EMITTER)
    dirs = rng.normal(size=(M, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    mk = rt.MarkedCells(N, cells, kinds, rng.uniform(0.5, 2.0, M), dirs, np.full(M, 0.8), 4.0 * prob.dt)
    kP = d(st.kP)
    ms_mk = _ms_per_call(lambda: rt.marked_apply(mesh, prm, angles, mk, bufs[0], rho, mom, etot, kP), reps)
    mk_bytes = M * (K * 4 * 2 + 8 + 48 + 16 + 8 + 48)
    out["marked_cells"] = {"marked": M, "ms_per_apply": round(ms_mk, 4), "kernel": "k_marked",
                           "roofline": _roofline(ms_mk, mk_bytes)}
    log(f"  marked cells ({M}): {ms_mk:.3f} ms per application")
    mk.free()

    # per-cell angle moments (E_r, F_r, P_r)
    mo = torch.empty((N, 10), dtype=torch.float64, device="cuda")
    ms_mo = _ms_per_call(lambda: rt.moments(mesh, prm, angles, bufs[0], mo), reps)
    out["moments"] = {"ms": round(ms_mo, 4), "kernel": "k_moments",
                      "roofline": _roofline(ms_mo, N * K * 4 + N * 80)}
    log(f"  moments: {ms_mo:.3f} ms")
    return out


def counters_summary(pmc_dir, copy_bytes):
    """HBM bytes per launch of the step kernels from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE,
    KiB per dispatch) over a bench run with --copy-calibration; each counter is scaled by what it reads
    for the calibration kernel (copy_bytes read and copy_bytes written per launch)."""
    import csv
    import glob
    vals = {}
    for name in ("FETCH_SIZE", "WRITE_SIZE"):
        for path in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as f:
                for r in csv.DictReader(f):
                    if r["Counter_Name"] != name:
                        continue
                    kn = r["Kernel_Name"]
                    key = ("copy" if "neg" in kn else
                           "step_upwind1_f32" if "k_step<float" in kn else
                           "step_upwind1_f64" if "k_step<double" in kn else None)
                    if key:
                        vals.setdefault((name, key), []).append(float(r["Counter_Value"]) * 1024.0)
    out = {}
    scale = {}
    for name in ("FETCH_SIZE", "WRITE_SIZE"):
        cp = vals.get((name, "copy"))
        scale[name] = copy_bytes / float(np.median(cp)) if cp else 1.0
    for key in ("step_upwind1_f32", "step_upwind1_f64"):
        fe, wr = vals.get(("FETCH_SIZE", key)), vals.get(("WRITE_SIZE", key))
        if fe and wr:
            f_b = float(np.mean(fe)) * scale["FETCH_SIZE"]
            w_b = float(np.mean(wr)) * scale["WRITE_SIZE"]
            out[key] = {"fetch_bytes_per_launch": f_b, "write_bytes_per_launch": w_b,
                        "hbm_bytes_per_launch": f_b + w_b, "launches": len(fe)}
    return {"source_hash": kernel_source_hash(), "scale": scale, "kernels": out}


def copy_bandwidth(n, log, reps=20):
    """Achievable HBM bandwidth of a plain streaming kernel on this GPU: torch's copy of n FP32
    values (an intensity-sized array, read once and written once), timed with HIP events over
    `reps` calls after two warm-up calls."""
    import torch
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    ms = _ms_per_call(lambda: y.copy_(x), reps)
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    log(f"copy bandwidth: {gbs:.0f} GB/s ({ms:.4f} ms per copy of {n * 4} bytes)")
    del x, y
    return {"kernel": "torch copy_ of an FP32 array of the intensities' size", "bytes_per_launch": 2 * n * 4,
            "ms": round(ms, 4), "achieved": round(gbs, 1), "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def cpu_model():
    """The host CPU as /proc/cpuinfo names it: model name, family / model / stepping, cache size."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if info:
                        break  # the first processor's block is enough
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("vendor_id", "model name", "cpu family", "model", "stepping", "cache size", "cpu MHz"):
                    info.setdefault(k, v)
    except OSError:
        return None
    if not info:
        return None
    return (f"{info.get('model name', '?')} (vendor {info.get('vendor_id', '?')}, family {info.get('cpu family', '?')}"
            f", model {info.get('model', '?')}, stepping {info.get('stepping', '?')}, cache {info.get('cache size', '?')})")


def cpu_config_timings(log):
    """The oracle at the plain forward workload (12^3 cells x 24 angles x 10 first-order steps, all
    of it) and at the PLM workload (64^3 cells x 80 angles, PLM-VL2: 3 of its 100 steps on all
    threads, 1 on one thread), cell-angle updates per second."""
    import oracle as orc
    from paper_2002_08377_amd import inputs as inp
    out = {}
    threads = orc.num_threads()
    for index, scheme, steps, one in ((0, "upwind1", 10, 10), (1, "plm_vl2", 3, 1)):
        p = inp.make_problem(index)
        st = p.state
        N, K = st.I.shape
        om = orc.OracleMesh(p.mesh, st.mesh_vel)
        s0 = orc.OState(st.I, st.vol, st.mom, st.etot)
        t0 = time.perf_counter()
        orc.run(om, p.dirs, p.weights, p.phys, p.dt, s0, st.rho, st.kP, st.kJ, st.ks, steps, scheme)
        dt = time.perf_counter() - t0
        orc.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            orc.run(om, p.dirs, p.weights, p.phys, p.dt, s0, st.rho, st.kP, st.kJ, st.ks, one, scheme)
            d1 = time.perf_counter() - t0
        finally:
            orc.set_num_threads(threads)
        name = p.config.name
        out[name] = {"value": N * K * steps / dt, "unit": "cell-angle updates/s", "cores": threads,
                     "sample": f"{steps} of the {p.config.steps} {scheme} FP64 steps ({dt:.2f} s)",
                     "one_thread": {"value": N * K * one / d1, "unit": "cell-angle updates/s", "cores": 1,
                                    "sample": f"{one} step(s) ({d1:.2f} s)"}}
        log(f"  oracle {name}: {steps} steps in {dt:.2f} s on {threads} threads, {one} in {d1:.2f} s on 1")
    return out


def gpu_steps_from_initial(prob, mesh, angles, dtype_code, steps, inv):
    """`steps` fused steps of both forms' workload from its initial state: the intensities (put back
    in the problem's angle order with `inv`, as float64 on the host) and the new temperatures."""
    import torch
    from paper_2002_08377_amd import rt
    st, ph = prob.state, prob.phys
    params = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, prob.dt, dtype_code, rt.UPWIND1)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    I = d(st.I).to(rt.torch_dtype(dtype_code)).contiguous()
    I2 = torch.empty_like(I)
    vol, mom, etot = d(st.vol), d(st.mom), d(st.etot)
    rho, kP, kJ, ks = d(st.rho), d(st.kP), d(st.kJ), d(st.ks)
    T = torch.zeros_like(vol)
    for _ in range(steps):
        rt.step(mesh, params, angles, I, I2, vol, rho, mom, etot, kP, kJ, ks, T)
        I, I2 = I2, I
    out = I.double().cpu().numpy()
    return (out if inv is None else np.ascontiguousarray(out[:, inv])), T.cpu().numpy()


def parity_vs_oracle(gpu, ref_I, ref_T, steps):
    """Errors of the GPU forms against the oracle after the same `steps` steps: normwise
    max|d| / max|ref| and element-wise max |d| / |ref|, for the intensities and the temperature."""
    out = {"steps": steps, "reference": "FP64 oracle, same workload and initial state"}
    for name, (I, T) in gpu.items():
        dI, dT = np.abs(I - ref_I), np.abs(T - ref_T)
        out[name] = {"I_norm": float(dI.max() / np.abs(ref_I).max()), "I_elem": float((dI / np.abs(ref_I)).max()),
                     "T_norm": float(dT.max() / np.abs(ref_T).max()), "T_elem": float((dT / np.abs(ref_T)).max())}
    return out


def cpu_baseline(prob, steps, log, one_thread_steps=1):
    """The FP64 oracle (plain C, OpenMP) on the host cores: `steps` full steps of the same workload
    on all its threads, then `one_thread_steps` on one thread.  Returns the timing object and the
    oracle's state and temperatures after the `steps` steps."""
    import oracle as orc
    st = prob.state
    om = orc.OracleMesh(prob.mesh, st.mesh_vel)
    s0 = orc.OState(st.I, st.vol, st.mom, st.etot)
    N, K = st.I.shape
    threads = orc.num_threads()
    t0 = time.perf_counter()
    so, To = orc.run(om, prob.dirs, prob.weights, prob.phys, prob.dt, s0, st.rho, st.kP, st.kJ, st.ks, steps)
    dt = time.perf_counter() - t0
    log(f"  oracle: {steps} steps in {dt:.2f} s on {threads} threads")
    out = dict(value=N * K * steps / dt, unit="cell-angle updates/s", cores=threads, kind="oracle",
               sample=f"{steps} full FP64 first-order steps of the {N}-cell x {K}-angle workload "
                      f"({dt:.1f} s)", cpu_model=cpu_model(), nproc=os.cpu_count())
    if one_thread_steps > 0:
        orc.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            orc.run(om, prob.dirs, prob.weights, prob.phys, prob.dt, s0, st.rho, st.kP, st.kJ, st.ks,
                    one_thread_steps)
            d1 = time.perf_counter() - t0
        finally:
            orc.set_num_threads(threads)
        log(f"  oracle: {one_thread_steps} step(s) in {d1:.2f} s on 1 thread")
        out["one_thread"] = dict(value=N * K * one_thread_steps / d1, unit="cell-angle updates/s", cores=1,
                                 sample=f"{one_thread_steps} full step(s) of the same workload ({d1:.1f} s)")
    return out, so.I, To


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=None, help="override cells per side (default 128)")
    ap.add_argument("--cpu-steps", type=int, default=10, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--forms", default="f32,f64", help="precision forms to run (f32, f64)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also negate an FP32 intensity-sized array into another 3 times (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    ap.add_argument("--no-fwd-adj", action="store_true", help="skip the forward+adjoint measurement")
    ap.add_argument("--no-plm", action="store_true", help="skip the PLM throughput / energy-drift measurement")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the multigroup / kappa(T) / marked-cell measurements")
    ap.add_argument("--counters-summary", metavar="PMC_DIR",
                    help="write profiles/traffic.json from rocprofv3 FETCH_SIZE / WRITE_SIZE output and exit")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    if args.counters_summary:
        from paper_2002_08377_amd import inputs as inp
        n = args.n or 128
        K = inp.CONFIGS[WORKLOAD_INDEX].K
        summ = counters_summary(args.counters_summary, n ** 3 * K * 4)
        summ["command"] = ("rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --kernel-include-regex 'k_step|neg' "
                           "--output-format csv -- python3 bench.py --steps 2 --warmup 1 --cpu-steps 0 "
                           "--no-fwd-adj --no-plm --no-extensions --copy-calibration")
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
            json.dump(summ, f, indent=1)
        print(json.dumps(summ))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2002_08377_amd import inputs as inp
    from paper_2002_08377_amd import rt

    rt.lib()
    t0 = time.perf_counter()
    prob = inp.make_problem(WORKLOAD_INDEX, n=args.n)
    N, K, F = prob.mesh.n_cells, prob.dirs.shape[0], prob.mesh.n_faces
    log(f"workload: {N} cells, {F} faces, {K} angles; inputs built in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    mesh = rt.Mesh.from_inputs(prob.mesh, prob.state.mesh_vel, k_max=K)
    angles = rt.AngleSet(prob.dirs, prob.weights)
    log(f"mesh upload (host arrays, includes the half-face table build): {time.perf_counter() - t0:.2f} s")

    if args.copy_calibration:
        x = torch.ones(N * K, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)  # one read and one write of N K 4 bytes, a kernel named for neg
        torch.cuda.synchronize()
        log(f"copy calibration: 3 negated copies of {N * K * 4} bytes")
        del x, y
    copy_bw = copy_bandwidth(N * K, log)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    # Angle order (the same directions; a storage choice of the caller): both forms run fastest
    # with each antipode stored beside its angle (FP32: each lane moves two pairs with one
    # 16-byte access; FP64: one pair per 16-byte access).  Results are put back in the
    # first order for the comparison.
    perm = inp.adjacent_pair_order(K)
    inv = np.argsort(perm)
    p_adj, a_adj = inp.with_angle_order(prob, perm), rt.AngleSet(prob.dirs[perm], prob.weights[perm])
    setup = {"f32": (p_adj, a_adj, inv), "f64": (p_adj, a_adj, inv)}
    res = {}
    for name, code in (("f32", rt.F32), ("f64", rt.F64)):
        if name in forms:
            p_form, a_form, inv = setup[name]
            res[name] = run_form(p_form, mesh, a_form, code, args.steps, args.warmup, log)
            if inv is not None:
                res[name]["I"] = np.ascontiguousarray(res[name]["I"][:, inv])
    if not ("f32" in res and "f64" in res):
        mesh.free()
        print(json.dumps({name: {"ms_per_step": r["wall"] * 1e3 / args.steps, "kernel_ms": r["kernel_ms"]}
                          for name, r in res.items()}), flush=True)
        return

    ca = N * K * args.steps
    err = float(np.max(np.abs(res["f32"]["I"] - res["f64"]["I"])) / np.max(np.abs(res["f64"]["I"])))

    def roof(name):
        """The HBM roofline of the fused step kernel (its algorithmic bytes over its mean launch
        time), with the vector-ALU one of its algorithmic operations beside it, and both times at
        peak."""
        t = res[name]["kernel_ms"] * 1e-3
        b = algorithmic_bytes(N, F, K, name)
        ops = algorithmic_ops(N, F, K)
        hbm = {"bound": "hbm", "achieved": round(b / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_per_launch": int(b)}
        alu = {"bound": "alu", "achieved": round(ops / t / 1e12, 3), "peak": round(ALU_PEAK_TOPS, 2),
               "unit": "Top/s", "frac": round(ops / t / 1e12 / ALU_PEAK_TOPS, 4), "algorithmic_per_launch": int(ops)}
        t_hbm, t_alu = b / (HBM_PEAK_GBS * 1e9), ops / (ALU_PEAK_TOPS * 1e12)
        out = dict(hbm)
        out["traffic"] = measured_traffic(f"step_upwind1_{name}")
        if copy_bw:
            out["frac_of_copy"] = round(hbm["achieved"] / copy_bw["achieved"], 4)
        out["kernel"] = "k_step (fused upwind transport + implicit source)"
        out["kernel_ms"] = round(res[name]["kernel_ms"], 4)
        out["time_at_peak_ms"] = {"hbm": round(t_hbm * 1e3, 4), "alu": round(t_alu * 1e3, 4)}
        out["other"] = alu
        return out

    out = {
        "metric": "cell-angle updates/s per RT step (fwd)",
        "value": ca / res["f32"]["wall"],
        "unit": "cell-angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["f32"]["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"throughput_{round(N ** (1 / 3))}c_{K}a", "cells": N, "faces": F, "angles": K,
                   "steps": args.steps, "scheme": "upwind1",
                   "precision": "FP32 intensities and transport, FP64 source solve and bookkeeping",
                   "angle_order": "level-symmetric S8 set; antipode of angle k at k + 1 for even k",
                   "mesh": "periodic Voronoi of a +-0.2 jittered cubic lattice, Morton-ordered cells"},
        "roofline": roof("f32"),
        "fp64": {"value": ca / res["f64"]["wall"], "ms_per_step": res["f64"]["wall"] * 1e3 / args.steps,
                 "dtype": "f64", "roofline": roof("f64")},
        "copy_bandwidth": copy_bw,
        "f32_over_f64": res["f64"]["wall"] / res["f32"]["wall"],
        "f32_vs_f64_rel_err_I": err,
    }
    if not args.no_extensions:
        out["extensions"] = run_extensions(prob, mesh, angles, log)
    gpu_short = {}
    if args.cpu_steps > 0:
        # both forms over the oracle's steps, for the accuracy comparison after the CPU baseline
        for name, code in (("f32", rt.F32), ("f64", rt.F64)):
            p_form, a_form, inv_form = setup[name]
            gpu_short[name] = gpu_steps_from_initial(p_form, mesh, a_form, code, args.cpu_steps, inv_form)
    mesh.free()
    if not args.no_fwd_adj:
        out["fwd_adj"] = run_fwd_adj(log)
    if not args.no_plm:
        out["plm"] = run_plm(log)
    if args.cpu_steps > 0:
        out["cpu_baseline"], ref_I, ref_T = cpu_baseline(prob, args.cpu_steps, log)
        out["cpu_baseline"]["configs"] = cpu_config_timings(log)
        out["parity_vs_oracle"] = parity_vs_oracle(gpu_short, ref_I, ref_T, args.cpu_steps)
        log(f"  vs oracle after {args.cpu_steps} steps: " + ", ".join(
            f"{k} I {v['I_norm']:.2e} (elem {v['I_elem']:.2e}) T {v['T_norm']:.2e}"
            for k, v in out["parity_vs_oracle"].items() if isinstance(v, dict)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
