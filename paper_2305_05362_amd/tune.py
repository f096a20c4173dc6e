"""Autotuner for the launch schedule of the shared-mesh step kernel.

The direct-sum step kernel on a mesh shared by every row comes with 2, 3, 4 or
5 shifted nodes per thread (tiles of 511, 767, 1023 or 1279 destination cells,
four fewer with the residual fused in).  Which one is fastest depends on the
row length (how well tiles divide it), the precision, the order and the GPU:
larger tiles launch fewer workgroups and re-read less of the neighbouring
tiles' windows, smaller ones keep more waves in flight.  ``tune_step`` times
each candidate on the caller's own arrays and leaves the fastest set on the
context; ``tuned_schedule`` does so once per problem shape and remembers the
answer in a JSON file.

    python -m paper_2305_05362_amd.tune [--rows R --cols N] [--f64] [--order P]

tunes a polar disk of the given shape (synthetic, seeded) and prints the
timings.  ``choose_index`` adds the closed-form mesh-density index (for a
mesh built from a known density) as one more candidate.  Every timing runs the
library's own kernels; nothing here computes any part of the step.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import _lib as R

CANDIDATES = (0, 2, 3, 4, 5)
DEFAULT_CACHE = os.environ.get(
    "RAM_TUNE_CACHE",
    os.path.join(os.path.expanduser("~"), ".cache", "ram_mi355x", "schedules.json"))


def _time_steps(ctx, rows, q, v0, dv, dt, order, scan, steps, reps) -> float:
    """Seconds per step, the best of `reps` timed calls of `steps` steps (the
    first, untimed call captures the step loop's graph)."""
    work = q.clone()
    ctx.ram_step(rows, work, v0, dv, dt, order, steps, scan)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        work.copy_(q)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.ram_step(rows, work, v0, dv, dt, order, steps, scan)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del work
    return best / steps


def tune_step(ctx, rows, q, v0, dv, dt: float, order: int,
              scan: int = R.RAM_SUM_DIRECT, steps: int = 40, reps: int = 3,
              candidates: Sequence[int] = CANDIDATES) -> Tuple[int, Dict[int, float]]:
    """Time every candidate schedule on these arrays; set the fastest on the
    context and return it with the microseconds per step of each."""
    if scan != R.RAM_SUM_DIRECT or not rows.shared or rows.n_cols <= 0:
        return ctx.get_schedule(), {}
    us = {}
    for items in candidates:
        ctx.set_schedule(items)
        us[items] = _time_steps(ctx, rows, q, v0, dv, dt, order, scan, steps, reps) * 1e6
    best = min(us, key=us.get)
    ctx.set_schedule(best)
    return best, us


def choose_index(ctx, rows, q, v0, dv, dt: float, order: int, density, best_us: float,
                 scan: int = R.RAM_SUM_DIRECT, steps: int = 40, reps: int = 3):
    """The mesh-density index (Section 3.2.1) as one more candidate: with the
    shared mesh's density `density` = ((a, b, c), xmin, xmax) set, time the
    default schedule and keep the index if it beats `best_us` (the best
    schedule's microseconds per step with the bucket index).  Leaves the
    context configured for the winner; returns (use_density, us_per_step)."""
    saved = ctx.get_schedule()
    bump, xmin, xmax = density
    ctx.set_schedule(0)
    ctx.set_mesh_density(bump, xmin, xmax)
    us = _time_steps(ctx, rows, q, v0, dv, dt, order, scan, steps, reps) * 1e6
    if us < best_us:
        return True, us
    ctx.set_mesh_density(None)
    ctx.set_schedule(saved)
    return False, us


def shape_key(rows, q, dv, order: int, scan: int) -> str:
    """What the choice depends on: device, row count and length, precision,
    order, fused residual or not."""
    name = torch.cuda.get_device_name(q.device).replace(" ", "_")
    dt = "f64" if q.dtype == torch.float64 else "f32"
    return (f"{name}|rows={rows.n_rows}|cols={rows.n_cols}|{dt}|p={order}|scan={scan}"
            f"|residual={int(dv is not None)}")


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_schedule(ctx, rows, q, v0, dv, dt: float, order: int,
                   scan: int = R.RAM_SUM_DIRECT, cache_path: Optional[str] = DEFAULT_CACHE,
                   retune: bool = False, **kw) -> Tuple[int, Dict[int, float], bool]:
    """The schedule for this problem shape: from the cache when present (and
    not `retune`), else measured by tune_step and stored.  The choice is set on
    the context.  Returns (items_per_thread, timings, from_cache)."""
    key = shape_key(rows, q, dv, order, scan)
    cache = load_cache(cache_path) if cache_path else {}
    ent = cache.get(key)
    if ent and not retune and int(ent.get("items", 0)) in CANDIDATES:
        ctx.set_schedule(int(ent["items"]))
        return int(ent["items"]), {int(k): v for k, v in ent.get("us", {}).items()}, True
    best, us = tune_step(ctx, rows, q, v0, dv, dt, order, scan, **kw)
    if cache_path and us:
        cache[key] = {"items": best, "us": {str(k): round(v, 2) for k, v in us.items()},
                      "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
        save_cache(cache, cache_path)
    return best, us, False


def main(argv=None):
    from . import workloads as W
    p = argparse.ArgumentParser()
    p.add_argument("--rows", type=int, default=2048)
    p.add_argument("--cols", type=int, default=16384)
    p.add_argument("--order", type=int, default=5)
    p.add_argument("--f64", action="store_true")
    p.add_argument("--steps", type=int, default=40)
    p.add_argument("--cache", default=None, help="JSON cache to update (default: none)")
    a = p.parse_args(argv)
    dev = torch.device("cuda:0")
    wl = W.polar(a.rows, a.cols, 5, a.order, a.steps, sigma=0.01, noise=0.0)
    dtype = torch.float64 if a.f64 else torch.float32
    rows = R.Rows.from_workload(wl, dev)
    q = torch.as_tensor(wl.q0.reshape(-1), dtype=dtype, device=dev)
    dv = torch.as_tensor(wl.dv.reshape(-1), dtype=dtype, device=dev)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=dev)
    ctx = R.context(0)
    best, us, cached = tuned_schedule(ctx, rows, q, v0, dv, wl.dt, a.order,
                                      cache_path=a.cache, retune=True, steps=a.steps)
    print(json.dumps({"shape": shape_key(rows, q, dv, a.order, R.RAM_SUM_DIRECT),
                      "best_items_per_thread": best,
                      "us_per_step": {str(k): round(v, 2) for k, v in us.items()}}))


if __name__ == "__main__":
    main()
