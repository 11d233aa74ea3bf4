"""Differentiable radiation steps: a torch.autograd.Function over the C ABI.

The forward pass advances S first-order steps (transport then implicit source,
sections 2.2-2.3) with the fused step call and keeps a checkpoint of the state
(I, E_g, rho v, V) at the start of every segment of `ckpt_every` steps.  The
backward pass walks the segments in reverse: it restores the segment's
checkpoint, re-runs its steps with the taped step call (the same fused kernel,
so the same values bit for bit, each step's output kept in a buffer of its own,
which also stores a per-cell tape: the sums and temperature of the source solve,
the start-of-step volume and momentum), and then reverses the segment's steps with
one run-adjoint call (the transpose of each step fused with the source reverse of
the step before it).  The last segment is taped during the forward pass already
(the backward starts there), so it is not run again.  Peak memory is therefore one
checkpoint per segment plus `ckpt_every` recorded steps, instead of all S steps.

The opacities are tied, kappa_P = kappa_J = kappa_a, so dL/dkappa_a is the sum
of the two partial derivatives; the library increments both into one buffer.
Every step of the computation runs in the library's kernels; this module only
allocates buffers and orders calls on the current stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import rt


@dataclass
class RTSystem:
    """Everything of the problem except the differentiable inputs: the uploaded mesh
    (with RT_MESH_ADJOINT scratch), the step parameters (first-order scheme), the
    angle set, and the per-cell density, scattering opacity and initial volumes.
    With `overlap` the backward pass recomputes the next segment on a second stream
    while it reverses the current one (two sets of step records instead of one).  Off by
    default: at 96^3 x 80 x 40 (checkpoints every 8) the FP32 pass took 70.8 ms with it
    against 67.0 ms without, the FP64 pass 112.1 against 112.7 ms; the fused reverse
    kernel holds 160 of a SIMD's 512 registers per lane in each of its three waves, which
    leaves no room for a step kernel's wave beside them."""

    mesh: rt.Mesh
    params: rt.Params
    angles: rt.AngleSet
    rho: torch.Tensor
    ks: torch.Tensor
    vol0: torch.Tensor
    overlap: bool = False

    def check(self):
        if self.params.scheme != rt.UPWIND1:
            raise ValueError("the adjoint covers the first-order upwind scheme only")
        if not (self.mesh.flags & rt.MESH_ADJOINT):
            raise ValueError("the mesh must be uploaded with MESH_ADJOINT")


def _gas_views(gas):
    """Volume [N], momentum [N, 3] and gas energy [N]: contiguous views of one [5 N] buffer."""
    N = gas.shape[0] // 5
    return gas[:N], gas[N:4 * N].view(N, 3), gas[4 * N:]


def _record(N, dev):
    """One step's source tape: what the reverse needs of the step besides I* (the source
    solve's sums and temperature, the start-of-step volume and momentum)."""
    return torch.empty((N, rt.SRC_TAPE), dtype=torch.float64, device=dev)


class RTSteps(torch.autograd.Function):
    """(I^0, kappa_a, E_g^0, (rho v)^0) -> (I^S, E_g^S, (rho v)^S) after n_steps steps.

    Gradients flow to all four tensor inputs.  ckpt_every >= 1 sets the segment
    length of the recompute (the last segment may be shorter)."""

    @staticmethod
    def forward(ctx, I0, kappa_a, etot0, mom0, system: RTSystem, n_steps: int, ckpt_every: int):
        system.check()
        if n_steps < 0 or ckpt_every < 1:
            raise ValueError("n_steps >= 0 and ckpt_every >= 1 required")
        td = rt.torch_dtype(system.params.dtype)
        I = I0.detach().to(td).contiguous().clone()
        I2 = torch.empty_like(I)
        kap = kappa_a.detach().contiguous()
        # volume, momentum and gas energy live in one buffer, so that a checkpoint or a tape
        # record of them is a single copy
        gas = torch.empty(5 * I.shape[0], dtype=torch.float64, device=I.device)
        vol, mom, etot = _gas_views(gas)
        vol.copy_(system.vol0.detach())
        mom.copy_(mom0.detach())
        etot.copy_(etot0.detach())
        ckpts = []
        last = ((n_steps - 1) // ckpt_every) * ckpt_every if n_steps else 0  # first step of the last segment
        tape = []
        for n in range(n_steps):
            if n % ckpt_every == 0 and n < last:  # the last segment is taped instead
                ckpts.append((I.clone(), gas.clone()))
            if n >= last:
                # the last segment: tape it now (the taped step gives the fused step's values),
                # each step's output in a buffer of its own, kept for the reverse
                rec = (torch.empty_like(I), _record(I.shape[0], I.device))
                rt.step_taped(system.mesh, system.params, system.angles, I, rec[0], None, vol, system.rho, mom,
                              etot, kap, kap, system.ks, src_tape=rec[1])
                tape.append(rec)
                I = rec[0]
            else:
                rt.step(system.mesh, system.params, system.angles, I, I2, vol, system.rho, mom, etot, kap, kap,
                        system.ks)
                I, I2 = I2, I
        ctx.system = system
        ctx.n_steps = n_steps
        ctx.ckpt_every = ckpt_every
        ctx.ckpts = ckpts
        ctx.last_tape = tape
        # the returned intensities are the last step's record: saving them makes autograd refuse
        # a backward pass after they were changed in place
        ctx.save_for_backward(kap, I)
        ctx.in_dtype = I0.dtype
        return I, etot.clone(), mom.clone()

    @staticmethod
    def backward(ctx, gI, gE, gM):
        kap, _ = ctx.saved_tensors
        s = ctx.system
        td = rt.torch_dtype(s.params.dtype)
        N, K = s.mesh.n_cells, s.angles.K
        dev = kap.device
        lamI = (gI.to(td).contiguous().clone() if gI is not None
                else torch.zeros((N, K), dtype=td, device=dev))
        lamE = (gE.to(torch.float64).contiguous().clone() if gE is not None
                else torch.zeros(N, dtype=torch.float64, device=dev))
        lamM = (gM.to(torch.float64).contiguous().clone() if gM is not None
                else torch.zeros((N, 3), dtype=torch.float64, device=dev))
        dk = torch.zeros(N, dtype=torch.float64, device=dev)
        L = ctx.ckpt_every
        n_seg = (ctx.n_steps + L - 1) // L
        main = torch.cuda.current_stream(dev)
        # With overlap, the recompute of segment k - 1 runs on a second stream while this one
        # reverses segment k (they share no buffer), and two sets of step records alternate
        # between the segments; without it one set serves every segment in stream order.
        overlap = s.overlap and n_seg >= 2
        side = torch.cuda.Stream(device=dev) if overlap else main
        nsets = 2 if overlap else 1
        m = min(L, ctx.n_steps)
        last_set = (n_seg - 1) % nsets
        sets = []
        for k in range(nsets):
            # the forward pass's records of the last segment are reused for recomputed segments
            # once that segment's reverse (enqueued first) has read them; not its last output,
            # which the caller holds
            tI = [rec[0] for rec in ctx.last_tape[:-1]] if k == last_set else []
            tR = [rec[1] for rec in ctx.last_tape] if k == last_set else []
            tI += [torch.empty((N, K), dtype=td, device=dev) for _ in range(m - len(tI))]
            tR += [_record(N, dev) for _ in range(m - len(tR))]
            sets.append((tI, tR))

        def recompute(seg):
            """Enqueue the taped recompute of segment `seg` on the current stream: each step
            writes its output into the next record buffer, where the reverse reads it."""
            tI, tR = sets[seg % nsets]
            # each checkpoint is read once, so the recompute starts from its own buffers
            cur, gas = ctx.ckpts[seg]
            vol, mom, etot = _gas_views(gas)
            tape = []
            for n in range(min(L, ctx.n_steps - seg * L)):
                rt.step_taped(s.mesh, s.params, s.angles, cur, tI[n], None, vol, s.rho, mom, etot, kap, kap, s.ks,
                              src_tape=tR[n])
                cur = tI[n]
                tape.append((tI[n], tR[n]))
            return tape

        recomputed, reversed_ev = {}, {}
        if overlap:
            side.wait_stream(main)  # the checkpoints and records come from the forward pass
        for seg in reversed(range(n_seg)):
            if overlap and seg >= 1:
                with torch.cuda.stream(side):
                    if seg + 1 in reversed_ev:
                        side.wait_event(reversed_ev[seg + 1])  # its record set was segment seg + 1's
                    tape_prev = recompute(seg - 1)
                    ev = torch.cuda.Event()
                    ev.record(side)
                    recomputed[seg - 1] = (tape_prev, ev)
            if seg == n_seg - 1:
                tape = ctx.last_tape  # taped by the forward pass (it has no checkpoint)
            elif overlap:
                tape, ev = recomputed.pop(seg)
                main.wait_event(ev)
            else:
                tape = recompute(seg)  # after the reverse of seg + 1 has read the one record set
            rt.step_adjoint_run(s.mesh, s.params, s.angles, [i for i, _ in tape], [r for _, r in tape], s.rho,
                                kap, kap, s.ks, lamI, lamE, lamM, dk, dk, stream=main)
            ev = torch.cuda.Event()
            ev.record(main)
            reversed_ev[seg] = ev
        ctx.ckpts = None
        ctx.last_tape = None
        return lamI.to(ctx.in_dtype), dk, lamE, lamM, None, None, None


class FluxLoss(torch.autograd.Function):
    """The weighted emergent-flux loss of the library (rt_flux_loss) as a scalar
    tensor; its gradient with respect to I comes from the same call's seed output."""

    @staticmethod
    def forward(ctx, I, face_weight, system: RTSystem):
        loss = torch.zeros(1, dtype=torch.float64, device=I.device)
        Ic = I.detach().contiguous()
        # when I needs a gradient the same launch writes the seed dL/dI, kept for backward
        seed = torch.zeros_like(Ic) if ctx.needs_input_grad[0] else None
        rt.flux_loss(system.mesh, system.params, system.angles, Ic, face_weight, loss, seed)
        ctx.seed = seed
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        return ctx.seed * g.to(ctx.seed.dtype), None, None


def record_bytes(system: RTSystem) -> int:
    """Device bytes of one taped step's record: its output intensities and its source tape."""
    elem = 4 if system.params.dtype == rt.F32 else 8
    return system.mesh.n_cells * (system.angles.K * elem + rt.SRC_TAPE * 8)


def auto_checkpoint_interval(system: RTSystem, n_steps: int, budget_bytes: int) -> int:
    """The segment length for `n_steps` steps whose taped records fit in `budget_bytes`: all
    steps (nothing recomputed) when they fit, else the longest segment that fits (at least 1).
    A segment of L steps holds L records while it is reversed; the checkpoints of the other
    segments (an intensity copy and the gas state each) are counted too."""
    if n_steps <= 0:
        return 1
    rec = record_bytes(system)
    ckpt = rec + 5 * 8 * system.mesh.n_cells
    for L in range(n_steps, 0, -1):
        n_ckpt = (n_steps + L - 1) // L - 1
        if L * rec + n_ckpt * ckpt <= budget_bytes:
            return L
    return 1


def rt_steps(I0, kappa_a, etot0, mom0, system: RTSystem, n_steps: int, ckpt_every: int | None = 8):
    """S steps as one differentiable function.  ckpt_every=None picks the interval from the free
    device memory: every step taped in the forward pass (no recompute) when the records fit in
    half of it, else the longest segment that fits."""
    if ckpt_every is None:
        free, _ = torch.cuda.mem_get_info(I0.device)
        ckpt_every = auto_checkpoint_interval(system, n_steps, free // 2)
    return RTSteps.apply(I0, kappa_a, etot0, mom0, system, n_steps, ckpt_every)


def flux_loss(I, face_weight, system: RTSystem):
    return FluxLoss.apply(I, face_weight, system)
