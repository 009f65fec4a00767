"""Differentiable droplet rollout: torch.autograd.Function over the HIP step.

displacement_loss(zeta, q0, q5, ...) runs `steps` coupled steps of the droplet
on the GPU and returns L = (z_c(T) - z_c(0))^2, the squared displacement along
z of the phi-weighted droplet centre.  Its backward runs the hand-written
adjoint of the step in reverse.  With checkpoint = k the forward pass keeps a
state every k steps and the reverse pass replays each segment with recording
steps (state buffers and u, F, drho records) before reversing it; with checkpoint = 0
the forward pass keeps the lean record of every step (Q, phi of each time and
drho, u, F of its step: all the reverse of a step reads, about 52 B per site
in float32) and the reverse pass replays nothing.  Gradients: dL/dzeta, dL/dq0
(float64 device sums) and dL/dq5 (the initial Q field, 5 stored components);
phi(0) and the initial populations are held fixed.  run_recorded /
backward_recorded keep whole states instead of lean records, and
backward_segments_lean replays segments into lean records.
"""
from __future__ import annotations

import numpy as np
import torch

from .sim import Sim


def run_segments(sim: Sim, steps: int, checkpoint: int):
    """Advance `steps` steps, returning the checkpoint states taken every `checkpoint` steps."""
    ckpts = []
    t = 0
    while t < steps:
        ckpts.append(sim.get_state())
        n = min(checkpoint, steps - t)
        sim.step(n)
        t += n
    return ckpts


def run_recorded(sim: Sim, steps: int):
    """Advance `steps` steps keeping every state and step record (no replay in the
    reverse pass; device memory grows as steps x (state + record) bytes).
    Returns (states[0..steps], records[0..steps-1]); the context ends at states[-1]."""
    states = [sim.get_state()]
    recs = []
    for _ in range(steps):
        states.append(torch.empty_like(states[0]))
        recs.append(sim.record_buffer())
        sim.step_record(states[-2], states[-1], recs[-1])
    sim.set_state(states[-1])
    return states, recs


def backward_recorded(sim: Sim, states, recs, adj):
    """Reverse pass over a run_recorded history; adj as in backward_segments.
    Returns (zeta_bar, q0_bar)."""
    zb = qb = 0.0
    other = torch.empty_like(adj)
    cur, nxt = adj, other
    for j in reversed(range(len(recs))):
        zb, qb = sim.adjoint_step(states[j], cur, nxt, rec=recs[j], zeta_bar=zb, q0_bar=qb, fetch=j == 0)
        cur, nxt = nxt, cur
    if cur is not adj:
        adj.copy_(cur)
    return zb, qb


def backward_segments(sim: Sim, ckpts, steps: int, checkpoint: int, adj):
    """Reverse pass over the checkpointed segments.

    adj holds the adjoint of the final state on entry and the adjoint of the
    initial state on return.  Each segment is replayed from its checkpoint with
    recording steps (state buffers and u, F, drho records), then reversed step by
    step.  Returns (zeta_bar, q0_bar)."""
    zb = qb = 0.0
    states = [None] * (checkpoint + 1)
    recs = [None] * checkpoint
    other = torch.empty_like(adj)
    cur, nxt = adj, other
    for s in reversed(range(len(ckpts))):
        t0 = s * checkpoint
        n = min(checkpoint, steps - t0)
        states[0] = ckpts[s]
        for j in range(n):
            if recs[j] is None:
                recs[j] = sim.record_buffer()
            if j + 1 < n:
                if states[j + 1] is None:
                    states[j + 1] = torch.empty_like(ckpts[s])
                sim.step_record(states[j], states[j + 1], recs[j])
            else:  # the segment's end state is never read: record only
                sim.step_record(states[j], None, recs[j])
        for j in reversed(range(n)):
            last = s == 0 and j == 0  # the parameter sums are fetched once, after the last reverse step
            zb, qb = sim.adjoint_step(states[j], cur, nxt, rec=recs[j], zeta_bar=zb, q0_bar=qb, fetch=last)
            cur, nxt = nxt, cur
    if cur is not adj:
        adj.copy_(cur)
    return zb, qb


def backward_segments_overlapped(sim: Sim, replay: Sim, ckpts, steps: int, checkpoint: int, adj,
                                 replay_stream):
    """backward_segments with the replay of segment s-1 running on a second context
    (`replay`, same parameters, created on `replay_stream`) while segment s is
    reversed on `sim`'s stream.  A recording step touches only the state buffers
    and records it is given, so the two contexts share nothing but those buffers,
    which are double-buffered per segment; events order each reverse after its
    segment's replay and each replay after the reverse that last used its buffers.
    `sim` must run on torch's current stream.  The result equals backward_segments
    bit for bit.  Returns (zeta_bar, q0_bar)."""
    main_stream = torch.cuda.current_stream()
    nseg = len(ckpts)
    bufs = []
    for _ in range(min(2, nseg)):
        bufs.append(([None] + [torch.empty_like(ckpts[0]) for _ in range(checkpoint)],
                     [sim.record_buffer() for _ in range(checkpoint)]))
    replayed = [torch.cuda.Event() for _ in range(nseg)]
    reversed_ = [torch.cuda.Event() for _ in range(nseg)]

    def replay_segment(s):
        states, recs = bufs[s % 2]
        with torch.cuda.stream(replay_stream):
            if s + 2 < nseg:  # this buffer set was last used by the reverse of segment s + 2
                replay_stream.wait_event(reversed_[s + 2])
            n = min(checkpoint, steps - s * checkpoint)
            states[0] = ckpts[s]
            for j in range(n):
                replay.step_record(states[j], states[j + 1] if j + 1 < n else None, recs[j])
            replayed[s].record(replay_stream)

    zb = qb = 0.0
    other = torch.empty_like(adj)
    cur, nxt = adj, other
    replay_segment(nseg - 1)
    for s in reversed(range(nseg)):
        if s > 0:
            replay_segment(s - 1)
        main_stream.wait_event(replayed[s])
        states, recs = bufs[s % 2]
        n = min(checkpoint, steps - s * checkpoint)
        for j in reversed(range(n)):
            last = s == 0 and j == 0
            zb, qb = sim.adjoint_step(states[j], cur, nxt, rec=recs[j], zeta_bar=zb, q0_bar=qb, fetch=last)
            cur, nxt = nxt, cur
        reversed_[s].record(main_stream)
    if cur is not adj:
        adj.copy_(cur)
    return zb, qb


def run_lean(sim: Sim, steps: int):
    """Advance `steps` steps keeping the lean record of every step (no replay in the
    reverse pass; device memory grows as steps x lean-record bytes)."""
    recs = []
    for _ in range(steps):
        recs.append(sim.lean_record_buffer())
        sim.step_record_lean(recs[-1])
    return recs


def backward_lean(sim: Sim, recs, adj):
    """Reverse pass over run_lean's records; adj as in backward_segments.
    Returns (zeta_bar, q0_bar)."""
    zb = qb = 0.0
    other = torch.empty_like(adj)
    cur, nxt = adj, other
    for j in reversed(range(len(recs))):
        zb, qb = sim.adjoint_step_lean(recs[j], cur, nxt, zeta_bar=zb, q0_bar=qb, fetch=j == 0)
        cur, nxt = nxt, cur
    if cur is not adj:
        adj.copy_(cur)
    return zb, qb


def backward_segments_lean(sim: Sim, ckpts, steps: int, checkpoint: int, adj):
    """Reverse pass over checkpointed segments: each segment is replayed from its
    checkpoint into lean records (the context's own state advances through it),
    then reversed.  adj as in backward_segments; returns (zeta_bar, q0_bar)."""
    zb = qb = 0.0
    recs = [None] * checkpoint
    other = torch.empty_like(adj)
    cur, nxt = adj, other
    for s in reversed(range(len(ckpts))):
        n = min(checkpoint, steps - s * checkpoint)
        sim.set_state(ckpts[s])
        for j in range(n):
            if recs[j] is None:
                recs[j] = sim.lean_record_buffer()
            sim.step_record_lean(recs[j])
        for j in reversed(range(n)):
            last = s == 0 and j == 0
            zb, qb = sim.adjoint_step_lean(recs[j], cur, nxt, zeta_bar=zb, q0_bar=qb, fetch=last)
            cur, nxt = nxt, cur
    if cur is not adj:
        adj.copy_(cur)
    return zb, qb


class _DropletRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, zeta, q0, q5, params, phi, steps, checkpoint, precision, lattice, fd_scheme):
        p = dict(params, zeta=float(zeta), q0=float(q0))
        q5_np = q5.detach().to("cpu", torch.float64).numpy()
        sim = Sim(p, np.asarray(phi, dtype=np.float64), q5_np, precision=precision, lattice=lattice,
                  fd_scheme=fd_scheme, stream=torch.cuda.current_stream())
        zc0 = float(sim.centre()[0][2])
        ckpts = run_lean(sim, steps) if checkpoint == 0 else run_segments(sim, steps, checkpoint)
        zcT = float(sim.centre()[0][2])
        ctx.sim, ctx.ckpts, ctx.zc0 = sim, ckpts, zc0
        ctx.steps, ctx.checkpoint = steps, checkpoint
        ctx.q5_meta = (q5.dtype, q5.device)
        return torch.tensor((zcT - zc0) ** 2, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        sim = ctx.sim
        adj = sim.adjoint_buffer()
        sim.seed_centre(ctx.zc0, adj)
        if ctx.checkpoint == 0:
            zb, qb = backward_lean(sim, ctx.ckpts, adj)
        else:
            zb, qb = backward_segments(sim, ctx.ckpts, ctx.steps, ctx.checkpoint, adj)
        _, qbar, _ = sim.adjoint_parts(adj)
        g = float(grad_out)
        dtype, device = ctx.q5_meta
        q5_grad = (qbar * g).to(device=device, dtype=dtype)
        sim.close()
        ctx.sim = ctx.ckpts = None
        return (torch.tensor(g * zb, dtype=torch.float64), torch.tensor(g * qb, dtype=torch.float64), q5_grad,
                None, None, None, None, None, None, None)


def displacement_loss(zeta, q0, q5, *, params: dict, phi, steps: int, checkpoint: int = 20,
                      precision: str = "fp32", lattice: str = "d3q19", fd_scheme: str = "euler2"):
    """Squared z-displacement of the droplet centre after `steps` steps (differentiable).

    zeta, q0: 0-dim tensors; q5: [5, nz, ny, nx] tensor (CPU or CUDA); phi: numpy
    [nz, ny, nx]; params: the model parameter dict (its zeta / q0 are replaced).
    checkpoint: states kept every `checkpoint` steps and segments replayed in the
    reverse pass; 0 keeps the lean record of every step instead (no replay).
    lattice: 'd3q19' or the paper's 'd3q15' scheme; fd_scheme: 'euler2' or the paper's
    predictor-corrector 'pc4'.
    """
    return _DropletRollout.apply(zeta, q0, q5, params, phi, steps, checkpoint, precision, lattice, fd_scheme)
