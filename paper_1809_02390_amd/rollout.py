"""Checkpointed forward and adjoint of a rollout, and its torch.autograd.Function.

The map differentiated is

    rho0 --lbm_init--> f(0) = f^eq(rho0, u0, eta(rho0))  (zero u0 unless given)
         --n x lbm_step--> f(n) --> rho_T = sum_i f_i(n),

with the parameters sigma, W and T_r entering through theta = (G'^2, K', R T)
of the self-tuning EOS (main Eqs. 20-23).

Forward: f(0) is saved once (lbm_save_state); the lattice then steps on
(lbm_step, two steps per launch), its state copied to a checkpoint after
every ``every``-th step; with every = 1 the steps run from checkpoint buffer
to checkpoint buffer instead (lbm_step_saved_chain), so that no state is
copied.  Backward: from the last segment to the first, the segment's states
are recomputed from its checkpoint (lbm_step_saved_chain, bit for bit the
forward's) and the adjoint steps run back through them
(lbm_adjoint_run); lbm_adjoint_init closes with dL/d rho0, and

    dL/d(sigma, W, T_r) = J^T dL/d theta,   J = lbm_param_jacobian,

applied by the library (lbm_adjoint_params).

Backward with more than one segment: the recomputation of the next segment
runs on a second context and stream while the adjoint steps run back
through the current one (two sets of segment states, ordered by events).

Device memory: ceil(n / every) + 1 checkpoints + 2 (every - 1) segment
states and the second context's two state buffers (every - 1 with one
segment) + two adjoint states (11 fields each), all FP32 over nx*ny nodes.  With
every = 1 every state is kept and nothing is recomputed (the forward +
adjoint then moves 54 + 124 instead of 36 + 54 + 124 bytes per node and
step: the two-step kernel reads and writes each node's state once per two
steps, 36 B per step, plus 18 B when it also stores the state between them;
at 2048^2 x 1000 steps that is 151 GB of checkpoints, which HBM3E holds).  Any every > 1 recomputes n - ceil(n / every) forward steps, about
the whole forward pass, so ``every="auto"`` keeps every state when they fit
in free device memory and otherwise takes every = ceil(sqrt(n)), the
interval that keeps the fewest states.  Every step of the path runs in the
HIP library; this module only orders the calls.
"""
from __future__ import annotations

import math

import torch

from .lbm import (Lattice, lbm_adjoint_bytes, lbm_adjoint_params, lbm_adjoint_run, lbm_adjoint_theta,
                  lbm_checkpoint_bytes, lbm_step_saved_chain)


def rollout_bytes(nsteps, every, state_bytes, adjoint_bytes):
    """Device bytes a Rollout holds besides the lattice's own buffers:
    checkpoints, two sets of segment states (with more than one segment:
    one recomputed while the adjoint runs through the other) and the A/B
    buffers of the recomputing context, and the two adjoint states."""
    ckpt = -(-nsteps // every) + 1
    nseg = -(-nsteps // every)
    pool = 2 * (every - 1) + 2 if every > 1 and nseg > 1 else every - 1
    return (ckpt + pool) * state_bytes + 2 * adjoint_bytes


def choose_every(nsteps, state_bytes, adjoint_bytes, free_bytes, margin=0.8):
    """Checkpoint interval: 1 if every state fits in margin * free_bytes,
    else ceil(sqrt(nsteps)); ValueError if not even that fits."""
    if rollout_bytes(nsteps, 1, state_bytes, adjoint_bytes) <= margin * free_bytes:
        return 1
    every = max(2, math.ceil(math.sqrt(max(nsteps, 1))))
    need = rollout_bytes(nsteps, every, state_bytes, adjoint_bytes)
    if need > margin * free_bytes:
        raise ValueError(f"a rollout of {nsteps} steps needs {need / 2**30:.1f} GiB of device memory at "
                         f"every = {every}; {free_bytes / 2**30:.1f} GiB are free")
    return every


def free_device_bytes(device):
    """Free device memory, counting what torch's caching allocator holds unused."""
    dev = torch.device(device)
    free, _ = torch.cuda.mem_get_info(dev)
    return free + torch.cuda.memory_reserved(dev) - torch.cuda.memory_allocated(dev)


class Rollout:
    """Forward rollout with checkpoints, then one adjoint sweep."""

    def __init__(self, nx, ny, nsteps, every="auto", device="cuda", **kw):
        if kw.get("storage", "fp32") not in ("fp32", 0):
            raise ValueError("the adjoint is defined for FP32 storage only")
        if nsteps < 0 or (every != "auto" and int(every) < 1):
            raise ValueError("nsteps >= 0 and every >= 1 (or 'auto') are required")
        self.lat = Lattice(nx, ny, device=device, **kw)
        self.kw = kw
        self.rec = None  # context recomputing segments on a stream of its own (backward)
        if every == "auto":
            every = choose_every(int(nsteps), lbm_checkpoint_bytes(self.lat.params),
                                 lbm_adjoint_bytes(self.lat.params), free_device_bytes(self.lat.f_a.device))
        self.nx, self.ny, self.nsteps, self.every = nx, ny, int(nsteps), int(every)
        self.starts = list(range(0, self.nsteps, self.every))
        self.ckpt = [None] * (len(self.starts) + 1)  # states at the starts, then the final state
        self.pool = []  # segment states beyond the checkpoint (backward)
        self.pools = ([], [])  # the same, two sets (backward with more than one segment)
        self.inputs = None

    def _conv(self, a):
        if a is None:
            return None
        return torch.as_tensor(a).to(device=self.lat.f_a.device, dtype=torch.float32).reshape(
            self.ny, self.nx).contiguous()

    def forward(self, rho0, ux0=None, uy0=None):
        """rho_T (ny, nx) float32 after nsteps steps from f^eq(rho0)."""
        lat = self.lat
        self.inputs = (self._conv(rho0), self._conv(ux0), self._conv(uy0))
        lat.init(*self.inputs)
        self.ckpt[0] = lat.save_state(self.ckpt[0])
        if self.every == 1:
            for s in range(len(self.starts)):
                if self.ckpt[s + 1] is None:
                    self.ckpt[s + 1] = lat.checkpoint_buffer()
            lat.step_saved_chain(self.ckpt)
            lat.load_state(self.ckpt[-1], self.nsteps)
        else:
            for s, t0 in enumerate(self.starts):
                lat.step(min(self.every, self.nsteps - t0))
                self.ckpt[s + 1] = lat.save_state(self.ckpt[s + 1])
        return lat.moments()[0]

    def _segment_states(self, s):
        """States of times t0 .. t0 + m - 1 of segment s, recomputed from its
        checkpoint in one native call."""
        m = min(self.every, self.nsteps - self.starts[s])
        while len(self.pool) < m - 1:
            self.pool.append(self.lat.checkpoint_buffer())
        states = [self.ckpt[s]] + self.pool[:m - 1]
        self.lat.step_saved_chain(states)
        return states

    def backward_state(self, lam_T):
        """Adjoint of f(0) (an adjoint-state buffer) for Lambda(T) = lam_T
        (9, ny, nx); leaves dL/d theta of the steps in the accumulator."""
        lat = self.lat
        lbm_adjoint_theta(lat.ctx, read=False, reset=True)
        a, b = lat.adjoint_seed(lam_T), lat.adjoint_buffer()
        if len(self.starts) > 1 and self.every > 1:
            return self._backward_overlapped(a, b)
        for s in reversed(range(len(self.starts))):
            out = lat.adjoint_run(self._segment_states(s), a, b)
            if out is b:
                a, b = b, a
        return a

    def _backward_overlapped(self, a, b):
        """The adjoint sweep with the recomputation of segment s - 1 on a
        second context and stream while the adjoint steps run back through
        segment s: two sets of segment states alternate, ordered by events
        (a set is recomputed only after the adjoint that read it, the adjoint
        of a segment only after its recomputation).  The same library calls
        in the same order per stream as the sequential sweep, so the same
        bits."""
        lat = self.lat
        dev = lat.f_a.device
        cur, main = torch.cuda.current_stream(dev), lat.stream
        if self.rec is None:
            self.rec = Lattice(self.nx, self.ny, device=dev, stream=torch.cuda.Stream(dev), **self.kw)
        side = self.rec.stream
        for pool in self.pools:
            while len(pool) < self.every - 1:
                pool.append(lat.checkpoint_buffer())
        main.wait_stream(cur)
        side.wait_stream(main)  # checkpoints written, segment buffers allocated
        sb, ab = lbm_checkpoint_bytes(lat.params), lbm_adjoint_bytes(lat.params)
        ready, free = {}, [None, None]

        def recompute(s):
            k = s % 2
            if free[k] is not None:
                side.wait_event(free[k])  # the adjoint that read this set has run
            m = min(self.every, self.nsteps - self.starts[s])
            states = [self.ckpt[s]] + self.pools[k][:m - 1]
            if m > 1:
                lbm_step_saved_chain(self.rec.ctx, states, sb)
            ev = torch.cuda.Event()
            ev.record(side)
            ready[s] = (ev, states)

        recompute(len(self.starts) - 1)
        for s in reversed(range(len(self.starts))):
            if s > 0:
                recompute(s - 1)
            ev, states = ready.pop(s)
            main.wait_event(ev)
            if lbm_adjoint_run(lat.ctx, states, a, b, sb, ab) == 1:
                a, b = b, a
            fe = torch.cuda.Event()
            fe.record(main)
            free[s % 2] = fe
        main.wait_stream(side)
        cur.wait_stream(main)
        return a

    def backward(self, grad_rho_T):
        """(dL/d rho0 (ny, nx) float32, dL/d theta (3,), dL/d(sigma, W, T_r) (3,))
        for dL/d rho_T = grad_rho_T."""
        if self.inputs is None:
            raise RuntimeError("backward before forward")
        g = self._conv(grad_rho_T)
        adj0 = self.backward_state(g.expand(9, self.ny, self.nx).contiguous())
        rho0, ux0, uy0 = self.inputs
        drho0 = self.lat.adjoint_init(rho0, adj0, ux0, uy0)
        dp, dth = lbm_adjoint_params(self.lat.ctx, reset=True)
        return drho0, dth, dp

    def release(self):
        if self.rec is not None:
            torch.cuda.current_stream(self.lat.f_a.device).wait_stream(self.rec.stream)
            self.rec.close()
            self.rec = None
        self.ckpt = [None] * (len(self.starts) + 1)
        self.pool = []
        self.pools = ([], [])
        self.lat.close()


class LBMRollout(torch.autograd.Function):
    """rho_T = LBMRollout.apply(rho0, sigma, width, tr, nsteps, every, options).

    every is the checkpoint interval or "auto" (see choose_every).

    rho0 is an (ny, nx) CUDA tensor; sigma, width and tr are Python floats
    or scalar tensors (gradients are returned for tensors); options is a dict
    of further make_params keywords (s_p, varpi, ...) or None."""

    @staticmethod
    def forward(ctx, rho0, sigma, width, tr, nsteps, every, options):
        ny, nx = rho0.shape
        r = Rollout(nx, ny, int(nsteps), every, device=rho0.device, sigma=float(sigma), width=float(width),
                    tr=float(tr), **dict(options or {}))
        out = r.forward(rho0.detach())
        ctx.rollout = r
        ctx.rho_dtype = rho0.dtype
        ctx.meta = [(p.dtype, p.device) if torch.is_tensor(p) else None for p in (sigma, width, tr)]
        return out

    @staticmethod
    def backward(ctx, grad):
        drho0, _, dp = ctx.rollout.backward(grad)
        ctx.rollout.release()
        params = [None if m is None else torch.tensor(v, dtype=m[0], device=m[1]) for m, v in zip(ctx.meta, dp)]
        return (drho0.to(ctx.rho_dtype), *params, None, None, None)


def lbm_rollout(rho0, sigma, width, tr, nsteps, every="auto", **options):
    """Differentiable rho_T of an nsteps rollout from f^eq(rho0)."""
    return LBMRollout.apply(rho0, sigma, width, tr, nsteps, every, options)
