"""Differentiable RAM rollout: torch.autograd.Function over n operator-split
steps, with gradients with respect to the initial state Q0, the residual
velocity dv and the per-row bulk velocity v0.

Forward: n steps of (bulk shift, residual), keeping one state every
``checkpoint`` steps.  Backward: for each segment, newest first, recompute the
segment from its checkpoint keeping the pre-shift and pre-residual states,
then walk it backwards through the residual adjoint (dv-bar accumulates) and
the shift adjoint (v0-bar accumulates).  Every step of both directions runs in
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
        for sgi in range(n_seg - 1, -1, -1):
            start = sgi * fctx.checkpoint
            k = min(fctx.checkpoint, fctx.n_steps - start)
            # recompute the segment, keeping the state before each shift and
            # the state the residual step read
            pre_shift, pre_res = [], []
            q = checkpoints[sgi].clone()
            for _ in range(k):
                pre_shift.append(q)
                h = torch.empty_like(q)
                ctx.ram_shift(rows, q, h, v0, dt, order, scan)
                if dv is not None:
                    pre_res.append(h)
                    q = torch.empty_like(h)
                    ctx.ram_residual(rows, h, q, dv, dt)
                else:
                    q = h
            for i in range(k - 1, -1, -1):
                if dv is not None:
                    ctx.ram_residual_adjoint(rows, pre_res[i], dv, qbar, tmp, dt, dvbar)
                    qbar, tmp = tmp, qbar
                ctx.ram_shift_adjoint(rows, pre_shift[i], qbar, tmp, v0, dt, order,
                                      v0bar, scan)
                qbar, tmp = tmp, qbar
        return qbar, dvbar, v0bar.to(v0.dtype), None, None, None, None, None, None


def rollout(q0: torch.Tensor, rows: R.Rows, v0: torch.Tensor,
            dv: Optional[torch.Tensor], dt: float, order: int, n_steps: int,
            checkpoint: int = 20, scan: int = R.RAM_SCAN_F64) -> torch.Tensor:
    """Differentiable n-step rollout; gradients flow to q0, dv and v0."""
    return RamRollout.apply(q0, dv, v0, rows, dt, order, n_steps, checkpoint, scan)
