"""Differentiable multi-step rollout of the CT-MHD step for PyTorch.

`rollout(cons, bface, params, dx, nsteps, every=5)` advances the interior
state (cons: (5, n2, n1, n0), bface: (3, n2, n1, n0), float64 CUDA tensors)
by `nsteps` library steps and returns the final state; gradients flow back
through the hand-written adjoint of the step (ctmhd_step_adjoint).

The step is differentiated with its dt values frozen (taken from the forward
rollout, or given) and without flux correction, so the library is called with
fofc = 0 in both directions.  With params in the FP32 form the forward steps
(and their recomputation) run in that form, and each adjoint step is the FP64
adjoint evaluated at the FP32-form states: the gradient of the FP64 step
along the FP32-form trajectory, whose states differ from the FP64 ones at the
FP32 form's error level.  The forward keeps a copy of the state every
`every` steps; the backward pass restores each checkpoint, recomputes the
states of that segment and applies the adjoint step by step, newest first.
In the FP64 form the backward records the steps of each segment again
(ctmhd_step_record, bitwise the forward's steps) and reverses them from
their tapes (ctmhd_step_adjoint_tape), so that no adjoint step recomputes
its first stage.  Memory: nsteps / every states plus the tapes of one
segment (every x 34 arrays); work: one forward, one recorded recomputation
of every step, and nsteps tape adjoints.  In the FP32 form the segment's
states are recomputed in that form and each is reversed by
ctmhd_step_adjoint.

With `tape=True` (FP64 form) every forward step is a recorded step
(ctmhd_step_record): it keeps S^n, the first-stage state and the face arrays
of both stages, and the backward pass reverses each step from its tape
(ctmhd_step_adjoint_tape) with no recomputation at all.  Memory: 34 ghosted
arrays per step instead of 8 per checkpoint.
"""
from __future__ import annotations

import torch

from . import ctmhd


class _Box:
    """Ghosted device state of one box plus the workspaces of both directions.
    The 8 fields of the state and of the two adjoint buffers are slices of one
    contiguous tensor each, so a snapshot or a restore is a single copy."""

    def __init__(self, params: ctmhd.Params, n, dx, device):
        self.params = params
        # the adjoint is built for the FP64 form; the FP32 form's forward is
        # differentiated through it
        self.adj_params = ctmhd.Params.from_buffer_copy(params)
        self.adj_params.precision = ctmhd.PRECISION["fp64"]
        self.ng = ctmhd.required_ghosts(params)

        def packed():
            st = ctmhd.BoxState(n, self.ng, dx, device)
            buf = torch.zeros((8,) + tuple(st.cons[0].shape), dtype=torch.float64, device=device)
            st.cons = [buf[m] for m in range(5)]
            st.bface = [buf[5 + a] for a in range(3)]
            return st, buf

        self.state, self.buf = packed()
        self.g_in, self.gin_buf = packed()
        self.g_out, self.gout_buf = packed()
        self.step_ws = torch.empty(ctmhd.workspace_bytes(params, self.state.box), dtype=torch.uint8,
                                   device=device)
        nb = ctmhd.adjoint_workspace_bytes(self.adj_params, self.state.box)
        if nb == 0:
            raise ctmhd.CtmhdError("this configuration has no adjoint: "
                                   + ctmhd.lib().ctmhd_last_error().decode())
        self.adj_ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.sl = (slice(None),) + self.state.interior()
        self.tape_bytes = ctmhd.tape_bytes(self.adj_params, self.state.box)
        self.rec_ws = None

    def new_tape(self):
        t = torch.empty(self.tape_bytes, dtype=torch.uint8, device=self.buf.device)
        if t.data_ptr() % 256:
            raise ctmhd.CtmhdError("tape allocation is not 256-byte aligned")
        return t

    def record(self, dt_fixed, tape):
        """One FP64 step that records its tape (dt_fixed: device scalar or None
        for the CFL dt)."""
        if self.rec_ws is None:
            self.rec_ws = torch.empty(ctmhd.workspace_bytes(self.adj_params, self.state.box),
                                      dtype=torch.uint8, device=self.buf.device)
        ctmhd.ctmhd_step_record(self.adj_params, self.state.box, self.state.cons,
                                self.state.bface, dt_fixed, tape, self.rec_ws)

    def reverse_tapes(self, tapes, gc, gb):
        """dL/dS^0 of the recorded steps tapes[0..] given dL/dS^N (interior
        tensors).  The output of one step is the input of the next one back
        (the adjoint reads interior values only), so the two cotangent
        buffers alternate without copies."""
        self.gin_buf[(slice(0, 5),) + self.sl[1:]] = gc
        self.gin_buf[(slice(5, 8),) + self.sl[1:]] = gb
        src, dst = (self.g_in, self.gin_buf), (self.g_out, self.gout_buf)
        for tape in reversed(tapes):
            ctmhd.ctmhd_step_adjoint_tape(self.adj_params, self.state.box, tape, src[0].cons,
                                          src[0].bface, dst[0].cons, dst[0].bface, self.adj_ws)
            src, dst = dst, src
        v = src[1][self.sl]
        return v[:5].clone(), v[5:].clone()

    def load(self, cons, bface):
        self.buf[(slice(0, 5),) + self.sl[1:]] = cons
        self.buf[(slice(5, 8),) + self.sl[1:]] = bface

    def snapshot(self):
        return self.buf.clone()

    def restore(self, snap):
        self.buf.copy_(snap)

    def interior(self):
        v = self.buf[self.sl]
        return v[:5], v[5:]

    def step(self, dt_fixed, dt_out):
        ctmhd.ctmhd_step(self.params, self.state.box, self.state.cons, self.state.bface, 1,
                         dt_fixed, dt_out, None, self.step_ws)

    def adjoint(self, dt, gc, gb):
        """dL/dS of the current state given dL/dS' of the next one (interior
        (5|3, n2, n1, n0) tensors); the state is left unchanged."""
        self.gin_buf[(slice(0, 5),) + self.sl[1:]] = gc
        self.gin_buf[(slice(5, 8),) + self.sl[1:]] = gb
        ctmhd.ctmhd_step_adjoint(self.adj_params, self.state.box, self.state.cons, self.state.bface,
                                 dt, self.g_in.cons, self.g_in.bface, self.g_out.cons,
                                 self.g_out.bface, self.adj_ws)
        v = self.gout_buf[self.sl]
        return v[:5].clone(), v[5:].clone()


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cons, bface, params, dx, nsteps, every, dt_fixed, tape):
        n = (cons.shape[3], cons.shape[2], cons.shape[1])
        box = _Box(params, n, dx, cons.device)
        box.load(cons.detach(), bface.detach())
        dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=cons.device)
        if dt_fixed is not None:
            dts.copy_(torch.as_tensor(dt_fixed, dtype=torch.float64, device=cons.device))
        ctx.tapes = None
        if tape:
            tapes = []
            for i in range(nsteps):
                tapes.append(box.new_tape())
                box.record(dts[i:i + 1] if dt_fixed is not None else None, tapes[-1])
            ctx.box, ctx.tapes, ctx.dts, ctx.nsteps = box, tapes, dts, nsteps
            c, b = box.interior()
            return c.clone(), b.clone()
        checkpoints = []
        for i in range(nsteps):
            if i % every == 0:
                checkpoints.append(box.snapshot())
            if dt_fixed is not None:
                box.step(dts[i:i + 1], None)
            else:
                box.step(None, dts[i:i + 1])
        ctx.box, ctx.checkpoints, ctx.dts = box, checkpoints, dts
        ctx.nsteps, ctx.every = nsteps, every
        c, b = box.interior()
        return c.clone(), b.clone()

    @staticmethod
    def backward(ctx, gc, gb):
        box = ctx.box
        gc = gc.contiguous() if gc is not None else torch.zeros_like(box.interior()[0])
        gb = gb.contiguous() if gb is not None else torch.zeros_like(box.interior()[1])
        if ctx.tapes is not None:
            return box.reverse_tapes(ctx.tapes, gc, gb) + (None,) * 6
        dts, every = ctx.dts, ctx.every
        nseg = len(ctx.checkpoints)
        fp64 = box.params.precision == ctmhd.PRECISION["fp64"]
        for s in range(nseg - 1, -1, -1):
            first = s * every
            last = min(first + every, ctx.nsteps)
            box.restore(ctx.checkpoints[s])
            if fp64:
                # the segment recomputed as recorded steps (bitwise the steps
                # of the forward), then reversed from their tapes: no adjoint
                # step recomputes its first stage
                tapes = []
                for i in range(first, last):
                    tapes.append(box.new_tape())
                    box.record(dts[i:i + 1], tapes[-1])
                gc, gb = box.reverse_tapes(tapes, gc, gb)
                continue
            # FP32 form: states first .. last-1 of this segment, recomputed in
            # that form from its checkpoint, each reversed by the FP64 adjoint
            states = [box.snapshot()]
            for i in range(first, last - 1):
                box.step(dts[i:i + 1], None)
                states.append(box.snapshot())
            for i in range(last - 1, first - 1, -1):
                box.restore(states[i - first])
                gc, gb = box.adjoint(dts[i:i + 1], gc, gb)
        return gc, gb, None, None, None, None, None, None


def rollout(cons, bface, params: ctmhd.Params, dx, nsteps, every=5, dt_fixed=None, tape=False):
    """Differentiable `nsteps`-step rollout (see the module docstring).  The
    library parameters must have fofc = 0 (FP64 or FP32 form; tape=True: FP64
    only); dt_fixed: None (CFL dt from the forward rollout, then frozen) or
    nsteps values."""
    if params.fofc:
        raise ValueError("the differentiable rollout takes steps without flux correction (fofc=0)")
    if every < 1:
        raise ValueError("every must be >= 1")
    if tape and params.precision != ctmhd.PRECISION["fp64"]:
        raise ValueError("recorded steps (tape=True) are FP64 steps")
    return _Rollout.apply(cons, bface, params, dx, int(nsteps), int(every), dt_fixed, bool(tape))


def conserved_from_primitives(rho, u, p, bface, gamma=5.0 / 3.0):
    """Torch (differentiable) version of the conserved state of cell
    primitives and face fields (cell-centred b = mean of the two faces,
    periodic)."""
    bc = torch.stack([0.5 * (bface[a] + torch.roll(bface[a], -1, dims=2 - a)) for a in range(3)])
    m = rho.unsqueeze(0) * u
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(0) + 0.5 * (bc * bc).sum(0)
    return torch.cat([rho.unsqueeze(0), m, e.unsqueeze(0)], 0)


def kinetic_energy(cons, dx):
    """Total kinetic energy sum(|m|^2 / (2 rho)) dV of an interior state."""
    vol = float(dx[0] * dx[1] * dx[2])
    return 0.5 * ((cons[1:4] ** 2).sum(0) / cons[0]).sum() * vol

