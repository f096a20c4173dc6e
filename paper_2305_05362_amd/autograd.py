"""Differentiable RAM rollout: torch.autograd.Function over n operator-split
steps, with gradients with respect to the initial state Q0, the residual
velocity dv and the per-row bulk velocity v0.

Forward: n steps of (bulk shift, residual), keeping one state every
``checkpoint`` steps.  Backward: for each segment, newest first, recompute the
segment from its checkpoint with ram_step_record (every state and every
post-shift state), then walk it backwards with ram_step_adjoint (the residual
transpose, dv-bar accumulating, then the shift transpose, v0-bar
accumulating).  Every step of both directions runs in
the library's HIP kernels; torch only holds the tensors.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _lib as R


def _rollout(ctx: R.Context, rows: R.Rows, q0, dv, v0, dt, order, n_steps,
             checkpoint, scan, keep):
    q = q0.clone()
    saved = [q0.detach().clone()] if keep else []
    done = 0
    while done < n_steps:
        k = min(checkpoint, n_steps - done)
        ctx.ram_step(rows, q, v0, dv, dt, order, k, scan)
        done += k
        if keep and done < n_steps:
            saved.append(q.detach().clone())
    return q, saved


class RamRollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, q0, dv, v0, rows: R.Rows, dt: float, order: int,
                n_steps: int, checkpoint: int, scan: int):
        ctx = R.context(q0.device.index)
        dvc = None if dv is None else dv.detach().contiguous()
        q, saved = _rollout(ctx, rows, q0.detach().contiguous(), dvc,
                            v0.detach().contiguous(), dt, order, n_steps,
                            checkpoint, scan, keep=True)
        fctx.rows = rows
        fctx.dt, fctx.order, fctx.n_steps = float(dt), int(order), int(n_steps)
        fctx.checkpoint, fctx.scan = int(checkpoint), int(scan)
        fctx.has_dv = dv is not None
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
        rows, dt, order, scan = fctx.rows, fctx.dt, fctx.order, fctx.scan
        qbar = gq.contiguous().clone()
        tmp = torch.empty_like(qbar)
        dvbar = torch.zeros_like(dv) if dv is not None else None
        v0bar = torch.zeros_like(v0, dtype=torch.float64)
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
            ctx.ram_step_record(rows, traj, half, v0, dv, dt, order, k, scan)
            for i in range(k - 1, -1, -1):
                ctx.ram_step_adjoint(rows, traj[i], None if half is None else half[i], dv,
                                     qbar, tmp, v0, dt, order, dvbar, v0bar)
                qbar, tmp = tmp, qbar
        return qbar, dvbar, v0bar.to(v0.dtype), None, None, None, None, None, None


def rollout(q0: torch.Tensor, rows: R.Rows, v0: torch.Tensor,
            dv: Optional[torch.Tensor], dt: float, order: int, n_steps: int,
            checkpoint: int = 20, scan: int = R.RAM_SCAN_F64) -> torch.Tensor:
    """Differentiable n-step rollout; gradients flow to q0, dv and v0."""
    return RamRollout.apply(q0, dv, v0, rows, dt, order, n_steps, checkpoint, scan)
