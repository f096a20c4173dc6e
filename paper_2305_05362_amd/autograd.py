"""Differentiable RAM rollout: torch.autograd.Function over n operator-split
steps, with gradients with respect to the initial state Q0, the residual
velocity dv and the per-row bulk velocity v0.

Forward: n steps of (bulk shift, residual), keeping one state every
``checkpoint`` steps (or, with checkpoint 0, every state and post-shift
state, so the backward pass needs no recomputation).  Backward: for each
segment, newest first, recompute the segment from its checkpoint with
ram_step_record (every state and every post-shift state), then walk it
backwards with ram_step_adjoint_steps (per step the residual transpose,
dv-bar accumulating, then the shift transpose, v0-bar accumulating; one tile
plan for the segment).

With ``recon`` (RAM_RECON_PLM or RAM_RECON_PPM) the bulk shift is the limited
one of Section 3.1: the forward runs ram_step_limited /
ram_step_limited_record, and each backward step is ram_step_limited_adjoint
(the residual's transpose, then the limited shift's transposed Jacobian at
the state the shift read, in one pass).  Every step of both directions runs in the library's HIP
kernels; torch only holds the tensors.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _lib as R


def _steps(ctx, rows, q, v0, dv, dt, order, k, scan, recon):
    if recon:
        ctx.ram_step_limited(rows, q, v0, dv, dt, recon, k)
    else:
        ctx.ram_step(rows, q, v0, dv, dt, order, k, scan)


def _record(ctx, rows, traj, half, v0, dv, dt, order, k, scan, recon):
    if recon:
        ctx.ram_step_limited_record(rows, traj, half, v0, dv, dt, recon, k)
    else:
        ctx.ram_step_record(rows, traj, half, v0, dv, dt, order, k, scan)


def _step_adjoint(ctx, rows, q_fwd, q_half, dv, qbar, out, v0, dt, order, recon, dvbar,
                  v0bar):
    """out = (one step's Jacobian)^T qbar; dvbar, v0bar accumulate."""
    if not recon:
        ctx.ram_step_adjoint(rows, q_fwd, q_half, dv, qbar, out, v0, dt, order, dvbar, v0bar)
        return
    ctx.ram_step_limited_adjoint(rows, q_fwd, q_half, dv, qbar, out, v0, dt, recon, dvbar,
                                 v0bar)


def _walk_back(ctx, rows, traj, half, dv, qbar, tmp, v0, dt, order, recon, k, dvbar,
               v0bar):
    """qbar (in place): the gradient of the segment's last state back to its
    first, through its k recorded steps (one call without a limiter: the
    steps share the shift's tile plan)."""
    if not recon:
        ctx.ram_step_adjoint_steps(rows, traj, half, dv, qbar, tmp, v0, dt, order, k,
                                   dvbar, v0bar)
        return
    cur, oth = qbar, tmp
    for i in range(k - 1, -1, -1):
        _step_adjoint(ctx, rows, traj[i], None if half is None else half[i], dv,
                      cur, oth, v0, dt, order, recon, dvbar, v0bar)
        cur, oth = oth, cur
    if cur is not qbar:
        qbar.copy_(cur)


def _rollout(ctx: R.Context, rows: R.Rows, q0, dv, v0, dt, order, n_steps,
             checkpoint, scan, keep, recon=0):
    q = q0.clone()
    saved = [q0.detach().clone()] if keep else []
    done = 0
    while done < n_steps:
        k = min(checkpoint, n_steps - done)
        _steps(ctx, rows, q, v0, dv, dt, order, k, scan, recon)
        done += k
        if keep and done < n_steps:
            saved.append(q.detach().clone())
    return q, saved


class RamRollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, q0, dv, v0, rows: R.Rows, dt: float, order: int,
                n_steps: int, checkpoint: int, scan: int, recon: int):
        ctx = R.context(q0.device.index)
        dvc = None if dv is None else dv.detach().contiguous()
        v0c = v0.detach().contiguous()
        fctx.rows = rows
        fctx.dt, fctx.order, fctx.n_steps = float(dt), int(order), int(n_steps)
        fctx.checkpoint, fctx.scan, fctx.recon = int(checkpoint), int(scan), int(recon)
        fctx.has_dv = dv is not None
        fctx.stored = checkpoint <= 0 or checkpoint >= n_steps
        if fctx.stored:
            # keep every state and every post-shift state: no recomputation
            # in the backward pass ((2n+1) states of memory)
            qc = q0.detach().contiguous().reshape(-1)
            traj = torch.empty((n_steps + 1, qc.numel()), dtype=qc.dtype, device=qc.device)
            half = torch.empty((n_steps, qc.numel()), dtype=qc.dtype,
                               device=qc.device) if dvc is not None else None
            traj[0].copy_(qc)
            _record(ctx, rows, traj, half, v0c, dvc, dt, order, n_steps, scan, recon)
            q = traj[n_steps].clone().reshape(q0.shape)
            fctx.save_for_backward(v0.detach(), *([dvc] if dvc is not None else []), traj,
                                   *([half] if half is not None else []))
            return q
        q, saved = _rollout(ctx, rows, q0.detach().contiguous(), dvc, v0c, dt, order,
                            n_steps, checkpoint, scan, keep=True, recon=recon)
        fctx.save_for_backward(v0.detach(), *([dvc] if dvc is not None else []), *saved)
        return q

    @staticmethod
    def backward(fctx, gq):
        ctx = R.context(gq.device.index)
        tensors = fctx.saved_tensors
        v0 = tensors[0]
        if fctx.has_dv:
            dv, checkpoints = tensors[1], tensors[2:]
        else:
            dv, checkpoints = None, tensors[1:]
        rows, dt, order, scan, recon = fctx.rows, fctx.dt, fctx.order, fctx.scan, fctx.recon
        qbar = gq.contiguous().clone()
        tmp = torch.empty_like(qbar)
        # only the gradients an input asks for: the v0 term (the
        # reconstruction at every shifted node) and the dv accumulation are
        # skipped in the kernels when v0 or dv needs none
        want_dv = dv is not None and fctx.needs_input_grad[1]
        want_v0 = fctx.needs_input_grad[2]
        dvbar = torch.zeros_like(dv) if want_dv else None
        v0bar = torch.zeros_like(v0, dtype=torch.float64) if want_v0 else None
        if fctx.stored:
            traj = checkpoints[0]
            half = checkpoints[1] if dv is not None else None
            _walk_back(ctx, rows, traj, half, dv, qbar, tmp, v0, dt, order, recon,
                       fctx.n_steps, dvbar, v0bar)
            return (qbar, dvbar, None if v0bar is None else v0bar.to(v0.dtype), None, None,
                    None, None, None, None, None)
        n_seg = len(checkpoints)
        seg = min(fctx.checkpoint, fctx.n_steps)
        traj = torch.empty((seg + 1, qbar.numel()), dtype=qbar.dtype, device=qbar.device)
        half = torch.empty((seg, qbar.numel()), dtype=qbar.dtype,
                           device=qbar.device) if dv is not None else None
        for sgi in range(n_seg - 1, -1, -1):
            start = sgi * fctx.checkpoint
            k = min(fctx.checkpoint, fctx.n_steps - start)
            # recompute the segment keeping every state and, with a residual,
            # the state each residual step read (one fused launch per step)
            traj[0].copy_(checkpoints[sgi].reshape(-1))
            _record(ctx, rows, traj, half, v0, dv, dt, order, k, scan, recon)
            _walk_back(ctx, rows, traj, half, dv, qbar, tmp, v0, dt, order, recon, k,
                       dvbar, v0bar)
        return (qbar, dvbar, None if v0bar is None else v0bar.to(v0.dtype), None, None, None,
                None, None, None, None)


def rollout(q0: torch.Tensor, rows: R.Rows, v0: torch.Tensor,
            dv: Optional[torch.Tensor], dt: float, order: int, n_steps: int,
            checkpoint: int = 20, scan: int = R.RAM_SCAN_F64,
            recon: int = 0) -> torch.Tensor:
    """Differentiable n-step rollout; gradients flow to q0, dv and v0.

    checkpoint: keep one state every `checkpoint` steps and recompute each
    segment in the backward pass; 0 (or >= n_steps) keeps every state and
    post-shift state instead ((2n+1) states of memory, no recomputation).
    recon: 0 for the order-`order` Lagrange shift (with `scan`), or
    RAM_RECON_PLM / RAM_RECON_PPM for the limited shift (order and scan are
    then unused).  The backward pass forms the dv and v0 gradients only when
    those tensors require them."""
    return RamRollout.apply(q0, dv, v0, rows, dt, order, n_steps, checkpoint, scan, recon)
