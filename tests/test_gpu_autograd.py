"""Differentiable radiation steps with checkpoint / recompute, through the C ABI.

* The recompute of the backward pass uses the taped step, which must give the
  fused step's values bit for bit and store the transported intensities exactly
  as the transport call alone gives them; fused and split calls also agree bit
  for bit, in both precision forms and in the paired and general lane layouts.
* The gradient of the emergent-flux loss through `RTSteps` (FP64) matches the
  oracle's hand-written reverse mode to 1e-10 (normwise) and the loss to 1e-12.
* The checkpoint interval changes memory, never values: gradients are equal bit
  for bit for every interval, including ones that do not divide the step count.
* Gradients with respect to all four inputs (I^0, kappa_a, E_g^0, (rho v)^0)
  agree with central differences of the GPU forward along random directions.
* At the adjoint workload's full size (32^3 cells, 48 angles, 20 steps) the
  gradient at the 16 seeded cells near the loss plane matches central finite
  differences to 1e-6 relative, plus the rounding floor of a difference quotient,
  64 eps S / (2 e), where S is the summed magnitude of the loss's terms (the loss,
  -0.026 here, is a small difference of face fluxes summing to ~115 in magnitude,
  so a relative step of 1e-6 would sit below that floor).  Steps: 1e-4 relative
  for kappa_a, 1e-3 for the intensity (the loss is nearly linear in it).
* At the checkpointed workload's full size (96^3 cells, 80 angles, 40 steps,
  checkpoints every 8) the FP32-transport gradient is compared with the FP64 one.
"""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_helpers import elem_err, regime_problem, rel_err
from paper_2002_08377_amd import inputs as inp
from paper_2002_08377_amd import rt
from paper_2002_08377_amd.autograd import RTSystem, flux_loss, rt_steps

pytestmark = pytest.mark.gpu


def _d(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _system(p, dtype=rt.F64, layout=None):
    st = p.state
    mesh = rt.Mesh.from_inputs(p.mesh, st.mesh_vel, k_max=p.dirs.shape[0], flags=rt.MESH_ADJOINT)
    ph = p.phys
    prm = rt.make_params(ph.c_red, ph.c_light, ph.a_rad, ph.cv, p.dt, dtype)
    system = RTSystem(mesh, prm, rt.AngleSet(p.dirs, p.weights, layout=layout), _d(st.rho), _d(st.ks), _d(st.vol))
    return system, dict(I0=_d(st.I), kap=_d(st.kP), etot=_d(st.etot), mom=_d(st.mom))


def _grads(system, x, fw, steps, ckpt, gas_w=None):
    I0, kap, etot, mom = (x[k].clone().requires_grad_() for k in ("I0", "kap", "etot", "mom"))
    IS, ES, MS = rt_steps(I0, kap, etot, mom, system, steps, ckpt)
    L = flux_loss(IS, fw, system)
    if gas_w is not None:
        L = L + (gas_w[0] * ES).sum() + (gas_w[1] * MS).sum()
    L.backward()
    torch.cuda.synchronize()
    return L.item(), I0.grad, kap.grad, etot.grad, mom.grad


def _loss_fwd(system, x, fw, steps, gas_w=None):
    """The same loss by plain fused steps (no autograd)."""
    with torch.no_grad():
        IS, ES, MS = rt_steps(x["I0"], x["kap"], x["etot"], x["mom"], system, steps, steps or 1)
        L = flux_loss(IS, fw, system)
        if gas_w is not None:
            L = L + (gas_w[0] * ES).sum() + (gas_w[1] * MS).sum()
    return L.item()


@pytest.mark.parametrize("K", [24, 80])
@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
@pytest.mark.parametrize("layout", [None, rt.ANGLES_GENERAL, "adjacent"])
def test_fused_step_equals_split_calls_bitwise(dtype, K, layout):
    p = inp.make_problem(0, n=7, K=K, steps=1)
    if layout == "adjacent":  # antipodes side by side
        p, layout = inp.with_angle_order(p, inp.adjacent_pair_order(K)), None
    st = p.state
    system, x = _system(p, dtype, layout)
    td = rt.torch_dtype(dtype)
    s = [dict(I=x["I0"].to(td), I2=torch.empty_like(x["I0"].to(td)), vol=_d(st.vol), mom=_d(st.mom),
              etot=_d(st.etot), T=torch.zeros_like(x["kap"])) for _ in range(2)]
    a, b = s
    rt.step(system.mesh, system.params, system.angles, a["I"], a["I2"], a["vol"], system.rho, a["mom"], a["etot"],
            x["kap"], x["kap"], system.ks, a["T"])
    rt.transport_step(system.mesh, system.params, system.angles, b["I"], b["I2"], b["vol"])
    rt.source_implicit(system.mesh, system.params, system.angles, b["I2"], system.rho, b["mom"], b["etot"],
                       x["kap"], x["kap"], system.ks, b["T"])
    torch.cuda.synchronize()
    for k in ("I2", "vol", "mom", "etot", "T"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("K", [24, 80])
@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_taped_step_equals_step_and_records_transport(dtype, K):
    p = inp.make_problem(0, n=7, K=K, steps=1)
    st = p.state
    system, x = _system(p, dtype)
    td = rt.torch_dtype(dtype)
    s = [dict(I=x["I0"].to(td), I2=torch.empty_like(x["I0"].to(td)), vol=_d(st.vol), mom=_d(st.mom),
              etot=_d(st.etot), T=torch.zeros_like(x["kap"])) for _ in range(2)]
    a, b = s
    Istar = torch.full_like(a["I"], float("nan"))
    Itr = torch.empty_like(a["I"])
    vtr = _d(st.vol)
    rt.step(system.mesh, system.params, system.angles, a["I"], a["I2"], a["vol"], system.rho, a["mom"], a["etot"],
            x["kap"], x["kap"], system.ks, a["T"])
    rt.step_taped(system.mesh, system.params, system.angles, b["I"], b["I2"], Istar, b["vol"], system.rho, b["mom"],
                  b["etot"], x["kap"], x["kap"], system.ks, b["T"])
    rt.transport_step(system.mesh, system.params, system.angles, x["I0"].to(td), Itr, vtr)
    torch.cuda.synchronize()
    for k in ("I2", "vol", "mom", "etot", "T"):
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(Istar, Itr)


def test_taped_step_rejects_overlap_and_plm():
    p = inp.make_problem(0, n=7, K=24, steps=1)
    system, x = _system(p)
    I = x["I0"].clone()
    I2 = torch.empty_like(I)
    with pytest.raises(rt.RTError):
        rt.step_taped(system.mesh, system.params, system.angles, I, I2, I, _d(p.state.vol), system.rho,
                      x["mom"].clone(), x["etot"].clone(), x["kap"], x["kap"], system.ks)
    plm = rt.make_params(p.phys.c_red, p.phys.c_light, p.phys.a_rad, p.phys.cv, p.dt, rt.F64, rt.PLM_VL2)
    with pytest.raises(rt.RTError):
        rt.step_taped(system.mesh, plm, system.angles, I, I2, torch.empty_like(I), _d(p.state.vol), system.rho,
                      x["mom"].clone(), x["etot"].clone(), x["kap"], x["kap"], system.ks)


@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_zero_steps_is_the_identity(dtype):
    """No steps: the outputs are the inputs and the gradients pass straight through."""
    p = inp.make_problem(0, n=6, K=24, steps=1)
    system, x = _system(p, dtype)
    td = rt.torch_dtype(dtype)
    I0 = x["I0"].to(td).clone().requires_grad_()
    kap, etot, mom = (x[k].clone().requires_grad_() for k in ("kap", "etot", "mom"))
    IS, ES, MS = rt_steps(I0, kap, etot, mom, system, 0, 8)
    assert torch.equal(IS, I0.detach()) and torch.equal(ES, etot.detach()) and torch.equal(MS, mom.detach())
    (2.0 * IS.sum() + 3.0 * ES.sum() + 4.0 * MS.sum()).backward()
    assert torch.all(I0.grad == 2.0) and torch.all(etot.grad == 3.0) and torch.all(mom.grad == 4.0)
    assert torch.all(kap.grad == 0.0)
    system.mesh.free()


def test_gradient_matches_oracle():
    p = inp.make_problem(2, n=8, K=24, steps=5)
    st = p.state
    system, x = _system(p)
    u = inp.loss_face_weights(p.mesh, np.random.default_rng(4))
    L, gI, gk, _, _ = _grads(system, x, _d(u), p.steps, 2)
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    Lo, gIo, gko = orc.adjoint(om, p.dirs, p.weights, p.phys, p.dt, orc.OState(st.I, st.vol, st.mom, st.etot),
                               st.rho, st.kP, st.ks, p.steps, u)
    assert abs(L - Lo) <= 1e-12 * abs(Lo)
    assert rel_err(gI.cpu().numpy(), gIo) < 1e-10
    assert rel_err(gk.cpu().numpy(), gko) < 1e-10


@pytest.mark.parametrize("fast", [False, True])
@pytest.mark.parametrize("dtype", [rt.F64, rt.F32])
def test_checkpoint_interval_leaves_gradients_unchanged(dtype, fast):
    """Bitwise the same gradients for every checkpoint interval, with the backward pass's
    recompute overlapped on a second stream or not (7 steps: 1 to 7 segments, odd and even
    counts, a short last segment).  The segment boundaries take the end-of-step volumes from
    the forward's records, the fused reverse forms them itself: with faces moving at ~0.3 cbar
    (every volume changing by a large fraction of an ulp's worth of dt D per step) the two
    must still agree bit for bit."""
    p = (regime_problem("reduced_fast", index=2, n=8, K=48, steps=7) if fast
         else inp.make_problem(2, n=8, K=48, steps=7))
    system, x = _system(p, dtype)
    fw = _d(inp.loss_face_weights(p.mesh, np.random.default_rng(5)))
    system.overlap = False
    ref = _grads(system, x, fw, p.steps, 1)
    for overlap in (False, True):
        system.overlap = overlap
        for ckpt in (1, 2, 3, 7, 10):
            got = _grads(system, x, fw, p.steps, ckpt)
            assert got[0] == ref[0]
            for a, b in zip(got[1:], ref[1:]):
                assert torch.equal(a, b), (ckpt, overlap)


def test_automatic_checkpoint_interval_gives_the_same_gradients():
    """ckpt_every=None (every step taped when the records fit in half the free memory, as they
    do here) against explicit intervals: bitwise the same loss and gradients."""
    p = inp.make_problem(2, n=8, K=24, steps=5)
    system, x = _system(p, rt.F32)
    fw = _d(inp.loss_face_weights(p.mesh, np.random.default_rng(6)))
    ref = _grads(system, x, fw, p.steps, 5)
    got = _grads(system, x, fw, p.steps, None)
    assert got[0] == ref[0]
    for a, b in zip(got[1:], ref[1:]):
        assert torch.equal(a, b)


def test_all_input_gradients_match_directional_differences():
    p = inp.make_problem(2, n=8, K=24, steps=4)
    system, x = _system(p)
    rng = np.random.default_rng(6)
    N, K = p.state.I.shape
    fw = _d(inp.loss_face_weights(p.mesh, rng))
    gas_w = (_d(rng.normal(size=N)), _d(rng.normal(size=(N, 3))))
    L, gI, gk, gE, gM = _grads(system, x, fw, p.steps, 3, gas_w)
    grads = dict(I0=gI, kap=gk, etot=gE, mom=gM)
    for key in ("I0", "kap", "etot", "mom"):
        base = x[key]
        delta = _d(rng.normal(size=tuple(base.shape))) * base.abs()
        h = 1e-6
        xp = dict(x); xp[key] = base + h * delta
        xm = dict(x); xm[key] = base - h * delta
        fd = (_loss_fwd(system, xp, fw, p.steps, gas_w) - _loss_fwd(system, xm, fw, p.steps, gas_w)) / (2 * h)
        an = float((grads[key] * delta).sum())
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9 * abs(L), (key, fd, an)


def _loss_term_magnitude(p, u, IS):
    """S = sum over loss faces of |u_f| 4 pi c A_f sum_k W_k |n_k . n_f| I_up: the scale of
    the rounding error of one loss evaluation (not an expected value)."""
    m = p.mesh
    f = np.nonzero(u)[0]
    mu = m.face_normal[f] @ p.dirs.T
    Iup = np.where(mu > 0, IS[m.face_cells[f, 0]], IS[m.face_cells[f, 1]])
    return 4 * np.pi * p.phys.c_light * float(
        np.sum(np.abs(u[f]) * m.face_area[f] * np.sum(p.weights * np.abs(mu) * Iup, axis=1)))


@pytest.mark.timeout(600)
def test_adjoint_32c_48a_full_size_matches_finite_differences():
    """Full size of the adjoint workload: 32^3 cells, 48 angles, 20 steps, FP64: the whole
    gradient against the oracle's, and 16 seeded cells against central differences."""
    p = inp.make_problem(2)
    system, x = _system(p)
    u = inp.loss_face_weights(p.mesh, p.seeds["omega"])
    fw = _d(u)
    cells = inp.fd_cells(p.mesh, p.seeds["fd_cells"])
    L, gI, gk, _, _ = _grads(system, x, fw, p.steps, 8)
    with torch.no_grad():
        IS = rt_steps(x["I0"], x["kap"], x["etot"], x["mom"], system, p.steps, p.steps)[0]
    floor = 64 * np.finfo(np.float64).eps * _loss_term_magnitude(p, u, IS.cpu().numpy())
    gk = gk.cpu().numpy()
    gI = gI.cpu().numpy()
    # the whole gradient against the oracle's reverse mode (normwise, and element-wise over
    # the entries above 1e-8 of the largest; the rest are the tails of the domain of dependence)
    st = p.state
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    Lo, gIo, gko = orc.adjoint(om, p.dirs, p.weights, p.phys, p.dt, orc.OState(st.I, st.vol, st.mom, st.etot),
                               st.rho, st.kP, st.ks, p.steps, u)
    err = {"L": abs(L - Lo) / abs(Lo), "gI": rel_err(gI, gIo), "gk": rel_err(gk, gko),
           "gI_elem": elem_err(gI, gIo, 1e-8 * np.abs(gIo).max()), "gk_elem": elem_err(gk, gko, 1e-8 * np.abs(gko).max())}
    print("adjoint 32^3 x 48 x 20 vs oracle:", {k: f"{v:.2e}" for k, v in err.items()})
    assert err["L"] < 1e-12 and err["gI"] < 1e-10 and err["gk"] < 1e-10, err
    assert err["gI_elem"] < 1e-8 and err["gk_elem"] < 1e-8, err
    assert np.array_equal(gk == 0.0, gko == 0.0)
    k_star = p.seeds["fd_cells"].integers(0, p.dirs.shape[0], size=cells.size)
    assert np.count_nonzero(gk[cells]) > 0
    kap0 = x["kap"].cpu().numpy()
    I00 = x["I0"].cpu().numpy()
    for c, k in zip(cells, k_star):
        e = 1e-4 * kap0[c]
        xp, xm = dict(x), dict(x)
        kp, km = kap0.copy(), kap0.copy(); kp[c] += e; km[c] -= e
        xp["kap"], xm["kap"] = _d(kp), _d(km)
        fd = (_loss_fwd(system, xp, fw, p.steps) - _loss_fwd(system, xm, fw, p.steps)) / (2 * e)
        assert abs(fd - gk[c]) <= 1e-6 * abs(gk[c]) + floor / (2 * e), ("kappa", c, fd, gk[c])
        e = 1e-3 * I00[c, k]
        Ip, Im = I00.copy(), I00.copy(); Ip[c, k] += e; Im[c, k] -= e
        xp, xm = dict(x), dict(x)
        xp["I0"], xm["I0"] = _d(Ip), _d(Im)
        fd = (_loss_fwd(system, xp, fw, p.steps) - _loss_fwd(system, xm, fw, p.steps)) / (2 * e)
        assert abs(fd - gI[c, k]) <= 1e-6 * abs(gI[c, k]) + floor / (2 * e), ("I0", c, k, fd, gI[c, k])



@pytest.mark.timeout(900)
def test_fwd_adj_96c_80a_matches_oracle():
    """Full size and length of the checkpointed workload against the oracle's reverse mode:
    96^3 cells, 80 angles (antipodes side by side, as the bench times it), 40 steps,
    checkpoints every 8.  One oracle run (loss and both gradients, FP64); the GPU's FP64 form
    within 1e-12 (loss) and 1e-10 (gradients, normwise; element-wise 1e-8 over the entries
    above 1e-8 of the largest), its FP32-transport form within 1e-5 (loss, dL/dI0) and 1e-4
    (dL/dkappa)."""
    p = inp.with_angle_order(inp.make_problem(4), inp.adjacent_pair_order(80))
    st = p.state
    u = inp.loss_face_weights(p.mesh, p.seeds["omega"])
    print("oracle reverse mode, 96^3 x 80 x 40 ...", flush=True)
    om = orc.OracleMesh(p.mesh, st.mesh_vel)
    Lo, gIo, gko = orc.adjoint(om, p.dirs, p.weights, p.phys, p.dt, orc.OState(st.I, st.vol, st.mom, st.etot),
                               st.rho, st.kP, st.ks, p.steps, u)
    del om
    fw = _d(u)
    for dtype in (rt.F64, rt.F32):
        system, x = _system(p, dtype)
        L, gI, gk, _, _ = _grads(system, x, fw, p.steps, 8)
        gI, gk = gI.double().cpu().numpy(), gk.cpu().numpy()
        system.mesh.free()
        del system, x
        torch.cuda.empty_cache()
        err = {"L": abs(L - Lo) / abs(Lo), "gI": rel_err(gI, gIo), "gk": rel_err(gk, gko),
               "gI_elem": elem_err(gI, gIo, 1e-8 * np.abs(gIo).max()),
               "gk_elem": elem_err(gk, gko, 1e-8 * np.abs(gko).max())}
        print(f"fwd+adj 96^3 x 80 x 40, {'FP64' if dtype == rt.F64 else 'FP32'} vs oracle:",
              {k: f"{v:.2e}" for k, v in err.items()}, flush=True)
        if dtype == rt.F64:
            assert err["L"] < 1e-12 and err["gI"] < 1e-10 and err["gk"] < 1e-10, err
            assert err["gI_elem"] < 1e-8 and err["gk_elem"] < 1e-8, err
        else:
            assert err["L"] < 1e-5 and err["gI"] < 1e-5 and err["gk"] < 1e-4, err

def test_fwd_adj_96c_80a_f32_against_f64():
    """Full size of the checkpointed workload: 96^3 cells, 80 angles, 40 steps, checkpoints every 8."""
    p = inp.make_problem(4)
    fw = None
    res = {}
    for dtype in (rt.F64, rt.F32):
        system, x = _system(p, dtype)
        if fw is None:
            fw = _d(inp.loss_face_weights(p.mesh, p.seeds["omega"]))
        L, gI, gk, _, _ = _grads(system, x, fw, p.steps, 8)
        res[dtype] = (L, gI.cpu().numpy(), gk.cpu().numpy())
        system.mesh.free()
        del system, x
        torch.cuda.empty_cache()
    L64, gI64, gk64 = res[rt.F64]
    L32, gI32, gk32 = res[rt.F32]
    eL, eI, ek = abs(L32 - L64) / abs(L64), rel_err(gI32, gI64), rel_err(gk32, gk64)
    print(f"f32 vs f64 at 96^3 x 80 x 40: loss {eL:.2e} dL/dI0 {eI:.2e} dL/dkappa {ek:.2e}")
    assert eL < 1e-5 and eI < 1e-5 and ek < 1e-4
