#!/usr/bin/env python3
"""Throughput of the RAM advection step on one MI355X.

Workload: the production-shaped polar disk, 2048 rows x 16384 azimuthal cells
(periodic-bump azimuthal mesh 10x finer inside |phi| < 0.2, log radii on
[0.4, 2.5]), Keplerian per-row bulk speed, residual velocity from the noisy
sine recipe, order-5 interpolation of the cumulative, van Leer residual step.
All inputs are seeded synthetic data resident in HBM before timing starts.

Prints one JSON line.  ``value`` is the forward step throughput (bulk shift +
residual, one step = every cell updated once) of the FP32-state path whose
cumulative differences are summed directly from the window masses
(RAM_SUM_DIRECT), with the launch schedule the autotuner picks before the
timed region.  Beside it: the FP32 path with two-sum and with FP64 prefix
sums, the FP64 paths (prefix sums, and direct sums with their own schedule),
forward+adjoint, the closed-form mesh-density index, the STD baseline on the
same mesh (time-step ratio, per-step overhead, accuracy), the 2D split step
(RAM along the azimuth, then the radial step) against STD's split step, the
step on a state of centre values with the fourth-order <Q> conversion, the
limited PLM /
PPM reconstructions, the one-step error against the FP64 path (held to the
oracle by the GPU tests), the dominant kernel's HBM roofline, and the CPU
oracle's throughput on a bounded sample (run on this host's cores).

    python bench.py [--steps K] [--warmup W] [--adj-steps A] [--no-cpu] [--items N]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s per RAM step (fwd, fwd+adjoint) vs FP64 plain at stated L1 err"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--adj-steps", type=int, default=100)
    p.add_argument("--checkpoint", type=int, default=20)
    p.add_argument("--fp64-steps", type=int, default=200)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-stretched", action="store_true",
                   help="skip the stretched-mesh disk (its step runs the same kernels at the "
                        "same launch shape as the headline: a kernel trace of the headline "
                        "leaves it out)")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--items", type=int, default=-1,
                   help="launch schedule of the headline step: 0 the streaming kernels "
                        "(256-cell wave tiles), 2..5 the general kernel with that many "
                        "shifted nodes per thread; -1: let the autotuner choose (untimed, "
                        "before the timed region)")
    p.add_argument("--index", choices=("auto", "bucket", "density"), default="auto",
                   help="source-cell index of the headline kernel: the bucket index, the "
                        "closed-form mesh-density index, or the autotuner's choice")
    p.add_argument("--profile-pass", action="store_true",
                   help="short run for hardware-counter passes: the headline kernel "
                        "for --steps steps, the PPM step kernel for --steps steps, "
                        "--steps 2D split steps (headline + radial kernel), --steps "
                        "steps on centre values (conversion kernels), then a plain "
                        "copy of COPY_BYTES")
    return p.parse_args()


COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_sh_f32_direct_polar2048x16384_traffic.md")
# the streaming step's two kernels (the default schedule)
UNI_KERNEL = "k_step_uni<5, 2, true>"
GEN_KERNEL = "k_step_gen<5, 2, true, 3>"
TRAFFIC_FILE_UNI = os.path.join(ROOT, "profiles", "k_step_uni_f32_polar2048x16384_traffic.md")
TRAFFIC_FILE_GEN = os.path.join(ROOT, "profiles", "k_step_gen_f32_polar2048x16384_traffic.md")
# the limited (PPM) FP32 step's two streaming kernels
TRAFFIC_FILE_PPM_UNI = os.path.join(ROOT, "profiles", "k_step_uni_lim_f32_ppm_polar2048x16384_traffic.md")
TRAFFIC_FILE_PPM_GEN = os.path.join(ROOT, "profiles", "k_step_gen_lim_f32_ppm_polar2048x16384_traffic.md")
PPM_UNI_KERNEL = "k_step_uni_lim<2, 2, true>"
PPM_GEN_KERNEL = "k_step_gen_lim<2, 2, true>"
# the per-row streaming shift (cfg3 ragged batch, two-sum prefix)
RAG_KERNEL = "k_step_rag<5, 1>"
TRAFFIC_FILE_RAG = os.path.join(ROOT, "profiles", "k_step_rag_f32_twosum_cfg3_traffic.md")
TRAFFIC_FILE_RADIAL = os.path.join(ROOT, "profiles", "k_radial_f32_polar2048x16384_traffic.md")
TRAFFIC_FILE_AVG4 = os.path.join(ROOT, "profiles", "k_average4_f32_polar2048x16384_traffic.md")
TRAFFIC_FILE_ADJ_UNI = os.path.join(ROOT, "profiles", "k_adjf_uni_f32_polar2048x16384_traffic.md")
TRAFFIC_FILE_ADJ_GEN = os.path.join(ROOT, "profiles", "k_adjf_gen_f32_polar2048x16384_traffic.md")
ADJ_UNI_KERNEL = "k_adjf_uni<5, true, true>"
ADJ_GEN_KERNEL = "k_adjf_gen<5, true, true>"
TRAFFIC_FILE_LADJ = os.path.join(ROOT, "profiles", "k_ladj_shift_f32_ppm_polar2048x16384_traffic.md")
LADJ_KERNEL = "k_ladj<2, false, false>"
TRAFFIC_FILE_LSADJ = os.path.join(ROOT, "profiles", "k_ladj_step_f32_ppm_polar2048x16384_traffic.md")
LSADJ_KERNEL = "k_ladj<2, true, true>"
# the FP64 plain path's kernel (window prefix sums, fused residual)
TRAFFIC_FILE_F64 = os.path.join(ROOT, "profiles", "k_step64_f64_prefix_polar2048x16384_traffic.md")
F64_KERNEL = "k_step64<5, 2, 0, true>"


def _finite(v):
    """The result with every non-finite float replaced by None (strict JSON)."""
    if isinstance(v, dict):
        return {k: _finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def load_traffic(path, kernel):
    """Measured HBM bytes per launch of a kernel, if the committed counter
    summary was taken on the current kernel sources and on this
    instantiation (`kernel`, as rocprofv3 names it)."""
    from paper_2305_05362_amd.build import kernel_digest
    from paper_2305_05362_amd.rocprof_summary import read_traffic
    rec = read_traffic(path)
    if not rec or rec.get("source_digest") != kernel_digest(kernel):
        return None
    if rec.get("kernel_name", "").split("::")[-1] != kernel:
        return None
    return rec


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the RAM rows shard without communication "
              "and this build runs on a single MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_05362_amd import _lib as R
    from paper_2305_05362_amd import workloads as W
    from paper_2305_05362_amd.autograd import rollout

    R.load_library()           # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = W.cfg5()
    n_cells = wl.n_cells
    order = wl.order
    rows = R.Rows.from_workload(wl, dev)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=dev)
    q64 = torch.as_tensor(wl.q0.reshape(-1), dtype=torch.float64, device=dev)
    dv64 = torch.as_tensor(wl.dv.reshape(-1), dtype=torch.float64, device=dev)
    q32 = q64.float()
    dv32 = dv64.float()
    ctx = R.context(0)

    def events():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_steps(q0, dv, scan, steps, warmup, rws=None, vv=None, dtt=None):
        # A multi-step call captures its step loop into a graph on first use
        # and replays it afterwards: one untimed call of the timed length
        # captures it (its result is discarded), then the state restarts from
        # q0, takes `warmup` steps, and `steps` steps are timed (a replay).
        rws = rows if rws is None else rws
        vv = v0 if vv is None else vv
        dtt = wl.dt if dtt is None else dtt
        q = q0.clone()
        ctx.ram_step(rws, q, vv, dv, dtt, order, steps, scan)
        q.copy_(q0)
        ctx.ram_step(rws, q, vv, dv, dtt, order, warmup, scan)
        torch.cuda.synchronize()
        a, b = events()
        a.record()
        ctx.ram_step(rws, q, vv, dv, dtt, order, steps, scan)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3, q

    def time_kernel(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = events()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / reps

    # --- launch schedule of the headline kernel: autotuned, or as given ----
    # candidates: 2..5 shifted nodes per thread with the bucket index, and the
    # closed-form index of the disk's periodic-bump mesh (Section 3.2.1)
    from paper_2305_05362_amd.tune import choose_index, tuned_schedule
    density = (wl.meta["bump"], -math.pi, math.pi)
    given = args.items >= 0
    if given:
        ctx.set_schedule(args.items)
        items, tune_us = args.items, {}
    else:
        items, tune_us, _ = tuned_schedule(ctx, rows, q32, v0, dv32, wl.dt, order,
                                           R.RAM_SUM_DIRECT, cache_path=None)
    dens_us = None
    if args.index == "density" or (args.index == "auto" and not given):
        if args.index == "density":
            ctx.set_schedule(0)
            ctx.set_mesh_density(*density)
            use_density = True
        else:
            use_density, dens_us = choose_index(ctx, rows, q32, v0, dv32, wl.dt, order,
                                                density, tune_us[items])
        if use_density:
            items = 4
    else:
        use_density = False
    idx = 1 if use_density else 0
    schedule = {"items_per_thread": items,
                "kernel": ("streaming: k_step_uni (uniform-run tiles) + k_step_gen (the rest), "
                           "256-cell wave tiles") if items == 0 and not use_density
                else "general k_step_sh",
                "tile_cells": 256 if items == 0 and not use_density
                else 256 * (items or 4) - 5,
                "index": "mesh-density closed form" if use_density else "bucket",
                "tuned_us_per_step": {str(k): round(v, 2) for k, v in tune_us.items()},
                "density_index_us_per_step": None if dens_us is None else round(dens_us, 2),
                "how": "given" if (given or args.index != "auto")
                       else "autotuned before the timed region"}

    if args.profile_pass:
        q = q32.clone()
        ctx.ram_step(rows, q, v0, dv32, wl.dt, order, args.steps, R.RAM_SUM_DIRECT)
        q.copy_(q32)
        ctx.ram_step_limited(rows, q, v0, dv32, wl.dt, R.RAM_RECON_PPM, args.steps)
        # 2D split steps: the radial kernel (and as many more headline steps)
        u_p = torch.as_tensor(W.radial_velocity(wl, 5).reshape(-1), dtype=torch.float32,
                              device=dev)
        re_p = torch.as_tensor(wl.meta["r_edges"], dtype=torch.float64, device=dev)
        q.copy_(q32)
        ctx.ram_step_split2d(rows, q, v0, dv32, re_p, u_p, wl.dt, order, args.steps,
                             R.RAM_SUM_DIRECT)
        # steps on centre values: the conversion kernel, both directions
        q.copy_(q32)
        ctx.ram_step_point4(rows, q, v0, dv32, wl.dt, order, args.steps, R.RAM_SUM_DIRECT)
        # backward steps with every gradient (Q, dv, v0): the adjoint kernel
        half = torch.empty_like(q32)
        ctx.ram_shift(rows, q32, half, v0, wl.dt, order, R.RAM_SUM_DIRECT)
        qb_in, qb_out = torch.ones_like(q32), torch.empty_like(q32)
        dvb, v0b = torch.zeros_like(dv32), torch.zeros_like(v0)
        for _ in range(args.steps):
            ctx.ram_step_adjoint(rows, q32, half, dv32, qb_in, qb_out, v0, wl.dt, order, dvb,
                                 v0b)
        # the limited (PPM) shift's adjoint, alone and with the residual's
        for _ in range(args.steps):
            ctx.ram_shift_limited_adjoint(rows, q32, qb_in, qb_out, v0, wl.dt,
                                          R.RAM_RECON_PPM)
        for _ in range(args.steps):
            ctx.ram_step_limited_adjoint(rows, q32, half, dv32, qb_in, qb_out, v0, wl.dt,
                                         R.RAM_RECON_PPM, dvb, v0b)
        # FP64 steps (the plain path: window prefix sums)
        q6 = q64.clone()
        ctx.ram_step(rows, q6, v0, dv64, wl.dt, order, args.steps, R.RAM_SCAN_F64)
        del q6
        # the per-row streaming shift: the cfg3 ragged batch, two-sum prefix
        wl3 = W.cfg3()
        rows3 = R.Rows.from_workload(wl3, dev)
        q3 = torch.as_tensor(wl3.q0, dtype=torch.float32, device=dev)
        ctx.ram_step(rows3, q3, torch.as_tensor(wl3.v0, dtype=torch.float64, device=dev),
                     None, wl3.dt, order, max(4, args.steps), R.RAM_SCAN_F32_TWOSUM)
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "steps": args.steps, "items": items,
                          "index": idx, "copy_bytes": COPY_BYTES}), flush=True)
        return

    # --- headline: FP32 state, cumulative differences summed directly ------
    # one fused shift+residual kernel per step (plus one mesh-table and one
    # window-plan kernel per call): the region time over the steps is the
    # fused kernel's average launch duration
    HEAD = R.RAM_SUM_DIRECT
    t_ts, q_ts = time_steps(q32, dv32, HEAD, args.steps, args.warmup)
    value = n_cells * args.steps / t_ts / 1e9
    t_fused = t_ts / args.steps
    # --- the mesh-density index: closed-form source cells (Section 3.2.1) ---
    # the azimuthal mesh is the periodic bump; the closed form runs with the
    # default schedule
    ctx.set_schedule(0)
    ctx.set_mesh_density(None)
    t_b, _ = time_steps(q32, dv32, HEAD, max(1, args.steps // 4), args.warmup)
    ctx.set_mesh_density(*density)
    t_d, _ = time_steps(q32, dv32, HEAD, max(1, args.steps // 4), args.warmup)
    ctx.set_mesh_density(*density) if use_density else ctx.set_mesh_density(None)
    ctx.set_schedule(items)
    kd = max(1, args.steps // 4)
    fast_index = {"value": round(n_cells * kd / t_d / 1e9, 3), "steps": kd,
                  "us_per_step": round(t_d / kd * 1e6, 2),
                  "bucket_index_us_per_step": round(t_b / kd * 1e6, 2),
                  "mesh": "periodic bump a=%.1f b=%.1f c=%.0f on [-pi, pi)" % wl.meta["bump"]}
    # --- FP32 state, compensated FP32 prefix sums ---------------------------
    k2s = max(1, args.steps // 4)
    t_two, _ = time_steps(q32, dv32, R.RAM_SCAN_F32_TWOSUM, k2s, args.warmup)
    v_two = n_cells * k2s / t_two / 1e9
    # --- FP32 state, FP64 prefix sums ---------------------------------------
    k2 = max(1, args.steps // 4)
    t_f64s, _ = time_steps(q32, dv32, R.RAM_SCAN_F64, k2, args.warmup)
    v_f64s = n_cells * k2 / t_f64s / 1e9
    # --- FP32 state, plain FP32 prefix sums ----------------------------------
    t_p32, _ = time_steps(q32, dv32, R.RAM_SCAN_F32, k2, args.warmup)
    v_p32 = n_cells * k2 / t_p32 / 1e9

    def mode_rec(v, t, k, nbytes, kernel):
        us = t / k * 1e6
        return {"value": round(v, 3), "steps": k, "us_per_step": round(us, 2),
                "algorithmic_bytes_per_cell": nbytes,
                "hbm_frac": round(nbytes * n_cells / (t / k) / 1e9 / HBM_PEAK_GBS, 4),
                "kernel": kernel}
    fp32_kernel = ("k_step_uni + k_step_gen (the streaming kernels; the mode's prefix in "
                   "the searching tiles)" if items == 0 and not use_density else "k_step_sh")
    def fp64_kernel_of(sched, density):
        return ("k_step64 (the streaming plan, tiles of 256 cells a wave, every node's "
                "weights in FP64)" if sched == 0 and not density else "k_step_sh")
    fp64_kernel = fp64_kernel_of(items, use_density)
    tr_f64 = load_traffic(TRAFFIC_FILE_F64, F64_KERNEL) if items == 0 and not use_density else None
    # --- FP64 plain path ----------------------------------------------------
    t64, q_64 = time_steps(q64, dv64, R.RAM_SCAN_F64, args.fp64_steps, args.warmup)
    v64 = n_cells * args.fp64_steps / t64 / 1e9
    # --- FP64 with direct sums, its own tuned schedule ----------------------
    ctx.set_mesh_density(None)
    items64, tune64, _ = tuned_schedule(ctx, rows, q64, v0, dv64, wl.dt, order,
                                        R.RAM_SUM_DIRECT, cache_path=None)
    t64d, _ = time_steps(q64, dv64, R.RAM_SUM_DIRECT, args.fp64_steps, args.warmup)
    v64d = n_cells * args.fp64_steps / t64d / 1e9
    ctx.set_schedule(items)                  # back to the headline's configuration
    if use_density:
        ctx.set_mesh_density(*density)

    # --- STD baseline on the same mesh (Section 4.2's comparison) ------------
    # STD: the upwind van Leer step with the full velocity v0 + dv, at the time
    # step its Courant rule allows; RAM: the split step at the residual's.
    # Over a physical time T, RAM takes T/dt_ram steps, STD T/dt_std.
    vfull_h = wl.v0[:, None] + wl.dv
    dt_std = W.residual_cfl_dt(wl.edges, vfull_h, 0.5)
    vfull = torch.as_tensor(vfull_h.reshape(-1), dtype=torch.float32, device=dev)
    ks = max(1, args.steps // 4)
    qa_, qb_ = q32.clone(), torch.empty_like(q32)
    ctx.ram_residual(rows, qa_, qb_, vfull, dt_std)
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    for _ in range(ks):
        ctx.ram_residual(rows, qa_, qb_, vfull, dt_std)
        qa_, qb_ = qb_, qa_
    b.record()
    torch.cuda.synchronize()
    t_std = a.elapsed_time(b) / 1e3 / ks
    # accuracy over T = 20 RAM steps with dv = 0 (a pure shift): both against
    # one FP64 shift by v0 T (the remap is exact for any shift size up to its
    # interpolation error) on rows through the density bump
    n_ram = 20
    T = n_ram * wl.dt
    v0_h = wl.v0
    dt_std0 = W.residual_cfl_dt(wl.edges, np.broadcast_to(v0_h[:, None], wl.dv.shape), 0.5)
    n_std = int(math.ceil(T / dt_std0))
    pick_a = np.array([1000, 1024, 1040])
    q_ram = torch.as_tensor(wl.q0.reshape(-1), dtype=torch.float64, device=dev)
    ctx.ram_step(rows, q_ram, v0, None, wl.dt, order, n_ram, R.RAM_SCAN_F64)
    vz = torch.as_tensor(np.broadcast_to(v0_h[:, None], wl.dv.shape).reshape(-1),
                         dtype=torch.float64, device=dev)
    q_s, q_t = torch.as_tensor(wl.q0.reshape(-1), dtype=torch.float64, device=dev), None
    q_t = torch.empty_like(q_s)
    for _ in range(n_std):
        ctx.ram_residual(rows, q_s, q_t, vz, T / n_std)
        q_s, q_t = q_t, q_s
    torch.cuda.synchronize()
    q_one = torch.as_tensor(wl.q0.reshape(-1), dtype=torch.float64, device=dev)
    q_ref1 = torch.empty_like(q_one)
    ctx.ram_shift(rows, q_one, q_ref1, v0, T, order, R.RAM_SCAN_F64)
    torch.cuda.synchronize()
    ref_a = q_ref1.cpu().numpy().reshape(wl.n_rows, -1)[pick_a].reshape(-1)
    del q_one, q_ref1

    def err_a(qd):
        g = qd.cpu().numpy().reshape(wl.n_rows, -1)[pick_a].reshape(-1)
        return float(np.sum(np.abs(g - ref_a)) / np.sum(np.abs(ref_a)))
    std_baseline = {
        "std": "upwind van Leer with the full velocity v0 + dv (the residual kernel)",
        "dt_ram": wl.dt, "dt_std": dt_std, "dt_ratio": round(wl.dt / dt_std, 2),
        "cfl_rule": "dt = 0.5 min_f min(dx_{f-1}, dx_f) / |v_f|, v = dv (RAM) or v0 + dv (STD)",
        "ram_step_us": round(t_ts / args.steps * 1e6, 2),
        "overhead_ram_over_std": round((t_ts / args.steps) / t_std, 3),
        "speedup_same_physical_time": round((wl.dt / dt_std) * t_std / (t_ts / args.steps), 2),
        "std_step_us": round(t_std * 1e6, 2),
        "accuracy_dv0": {"T": T, "ram_steps": n_ram, "std_steps": n_std,
                         "rows": pick_a.tolist(),
                         "ram_rel_l1_vs_one_shift": err_a(q_ram),
                         "std_rel_l1_vs_one_shift": err_a(q_s)}}
    del qa_, qb_, vfull, vz, q_s, q_t, q_ram

    # --- the 2D split step (Section 3's dimensional splitting, Section 4.2) --
    # RAM along the azimuth (the step above), then the radial upwind step with
    # a seeded radial velocity; STD: the residual kernel with the full
    # azimuthal velocity, then the same radial step.  Time steps from the
    # advective terms of Section 4.2's 2D Courant rule.
    u_h = W.radial_velocity(wl, 5)
    re_h = wl.meta["r_edges"]
    dt2_ram = W.cfl_2d_dt(wl.edges, re_h, wl.dv, u_h, 0.5)
    dt2_std = W.cfl_2d_dt(wl.edges, re_h, vfull_h, u_h, 0.5)
    re_d = torch.as_tensor(re_h, dtype=torch.float64, device=dev)
    u32 = torch.as_tensor(u_h.reshape(-1), dtype=torch.float32, device=dev)
    k2d = max(1, args.steps // 4)

    def time_split(recon):
        q = q32.clone()
        ctx.ram_step_split2d(rows, q, v0, dv32, re_d, u32, dt2_ram, order, k2d, HEAD,
                             recon)                                    # captures
        q.copy_(q32)
        torch.cuda.synchronize()
        a, b = events()
        a.record()
        ctx.ram_step_split2d(rows, q, v0, dv32, re_d, u32, dt2_ram, order, k2d, HEAD, recon)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / k2d

    t2_ram = time_split(0)
    t2_plm = time_split(R.RAM_RECON_PLM)
    vfull2 = torch.as_tensor(vfull_h.reshape(-1), dtype=torch.float32, device=dev)
    qa_, qb_ = q32.clone(), torch.empty_like(q32)

    def std2d():
        ctx.ram_residual(rows, qa_, qb_, vfull2, dt2_std)
        ctx.ram_radial_step(rows, qb_, qa_, re_d, u32, dt2_std)
    t2_std = time_kernel(std2d, k2d)
    t_rad = time_kernel(lambda: ctx.ram_radial_step(rows, q32, qb_, re_d, u32, dt2_ram), 50)
    tr_rad = load_traffic(TRAFFIC_FILE_RADIAL, "k_radial<float, 16>")
    del qa_, qb_, vfull2
    split_2d = {
        "radial": "upwind van Leer along r in polar geometry, closed edges; u = 0.01 "
                  "r^-1/2 sin(phi) zeta (zeta ~ N(0,1))",
        "cfl_rule": "dt = 0.5 / max_cells(|v_phi| / dphi + |u| / dr), v_phi = dv (RAM) "
                    "or v0 + dv (STD)",
        "dt_ram": dt2_ram, "dt_std": dt2_std, "dt_ratio": round(dt2_ram / dt2_std, 2),
        "ram_split_step_us": round(t2_ram * 1e6, 2),
        "ram_plm_split_step_us": round(t2_plm * 1e6, 2),
        "std_split_step_us": round(t2_std * 1e6, 2),
        "overhead_ram_over_std": round(t2_ram / t2_std, 3),
        "speedup_same_physical_time": round((dt2_ram / dt2_std) * t2_std / t2_ram, 2),
        "speedup_same_physical_time_plm": round((dt2_ram / dt2_std) * t2_std / t2_plm, 2),
        "value": round(n_cells / t2_ram / 1e9, 3), "unit": "Gcell-updates/s",
        "steps": k2d,
        "radial_kernel_us": round(t_rad * 1e6, 2),
        "radial_algorithmic_bytes_per_cell": 12,
        "radial_hbm_frac": round(12.0 * n_cells / t_rad / 1e9 / HBM_PEAK_GBS, 4),
        "radial_traffic": None if tr_rad is None else round(tr_rad["traffic_bytes_per_launch"])}
    del u32

    # --- a state of centre values (Section 3.1's fourth-order <Q>) ----------
    # each step converts the centre values to cell averages, takes the step
    # and converts back: three kernels a step on the same disk
    kp4 = max(1, args.steps // 4)
    qp = q32.clone()
    ctx.ram_step_point4(rows, qp, v0, dv32, wl.dt, order, kp4, HEAD)       # captures
    qp.copy_(q32)
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    ctx.ram_step_point4(rows, qp, v0, dv32, wl.dt, order, kp4, HEAD)
    b.record()
    torch.cuda.synchronize()
    t_p4 = a.elapsed_time(b) / 1e3 / kp4
    t_avg = time_kernel(lambda: ctx.ram_cell_average(rows, q32, qp, False), 50)
    tr_avg = load_traffic(TRAFFIC_FILE_AVG4, "k_average4<float, 0>")
    del qp
    # accuracy against the exact solution: centre values of a smooth periodic
    # function on a smoothly stretched mesh (x = xi + 0.5 sin xi), shifted by
    # 0.2137 of the period in one step of order 5, FP64, with and without the
    # conversion
    s_p4 = 0.2137 * 2.0 * math.pi
    acc = {}
    for n_p in (256, 512):
        xi = np.linspace(-math.pi, math.pi, n_p + 1)
        xm = xi + 0.5 * np.sin(xi)
        xm[0], xm[-1] = -math.pi, math.pi
        cm = 0.5 * (xm[1:] + xm[:-1])
        fm = lambda t: np.sin(t) + 0.3 * np.cos(3.0 * t)
        rw = R.Rows(torch.as_tensor(xm, dtype=torch.float64, device=dev), 1, n_p, None, True)
        one_v = torch.ones(1, dtype=torch.float64, device=dev)
        qa = torch.as_tensor(fm(cm), dtype=torch.float64, device=dev)
        qb = qa.clone()
        ctx.ram_step_point4(rw, qa, one_v, None, s_p4, order, 1)
        ctx.ram_step(rw, qb, one_v, None, s_p4, order, 1, R.RAM_SCAN_F64)
        torch.cuda.synchronize()
        want = fm(cm - s_p4)
        acc[n_p] = (float(np.max(np.abs(qa.cpu().numpy() - want))),
                    float(np.max(np.abs(qb.cpu().numpy() - want))))
    point4 = {
        "what": "state of centre values: convert to cell averages (<Q> = Q + dx^2 Q''/24), "
                "step, convert back",
        "value": round(n_cells / t_p4 / 1e9, 3), "unit": "Gcell-updates/s", "steps": kp4,
        "step_us": round(t_p4 * 1e6, 2),
        "overhead_over_step": round(t_p4 / t_fused, 3),
        "conversion_kernel_us": round(t_avg * 1e6, 2),
        "conversion_algorithmic_bytes_per_cell": 8,
        "conversion_hbm_frac": round(8.0 * n_cells / t_avg / 1e9 / HBM_PEAK_GBS, 4),
        "conversion_traffic": None if tr_avg is None
        else round(tr_avg["traffic_bytes_per_launch"]),
        "accuracy": {"mesh": "x = xi + 0.5 sin(xi) on [-pi, pi), shift 0.2137 periods, "
                             "order 5, FP64, max error against the exact centre values",
                     "with_conversion": {str(k): v[0] for k, v in acc.items()},
                     "centre_values_as_averages": {str(k): v[1] for k, v in acc.items()},
                     "order_with": round(math.log2(acc[256][0] / acc[512][0]), 2),
                     "order_without": round(math.log2(acc[256][1] / acc[512][1]), 2)}}

    # --- ragged rows with per-row meshes (4096 rows of 64..8192 cells) ------
    wl3 = W.cfg3()
    rows3 = R.Rows.from_workload(wl3, dev)
    v03 = torch.as_tensor(wl3.v0, dtype=torch.float64, device=dev)
    q3 = torch.as_tensor(wl3.q0, dtype=torch.float32, device=dev)
    k3 = max(1, args.steps // 5)
    t3, _ = time_steps(q3, None, R.RAM_SCAN_F32_TWOSUM, k3, args.warmup, rows3, v03, wl3.dt)
    t3p, _ = time_steps(q3, None, R.RAM_SCAN_F32, k3, args.warmup, rows3, v03, wl3.dt)
    t3s, _ = time_steps(q3, None, R.RAM_SUM_DIRECT, k3, args.warmup, rows3, v03, wl3.dt)
    rag_rec = load_traffic(TRAFFIC_FILE_RAG, RAG_KERNEL)
    t3d, _ = time_steps(q3.double(), None, R.RAM_SCAN_F64, k3, args.warmup, rows3, v03,
                        wl3.dt)
    # one step of each FP32 path against the FP64 one from the same
    # FP32-rounded start: the plain FP32 window prefix shows the cancellation
    # the compensated one removes.  (Over many steps the unlimited order-5
    # interpolant is unstable on the rows whose neighbouring cells differ up
    # to 20x in size -- the oracle diverges on them too, order 3 and the
    # limited reconstructions do not -- and would amplify rounding there.)
    ones = {}
    for name, dtp, scan in (("f32_twosum", torch.float32, R.RAM_SCAN_F32_TWOSUM),
                            ("f32_plain_prefix", torch.float32, R.RAM_SCAN_F32),
                            ("f64", torch.float64, R.RAM_SCAN_F64)):
        qq = q3.to(dtp).clone()
        ctx.ram_step(rows3, qq, v03, None, wl3.dt, order, 1, scan)
        ones[name] = qq
    torch.cuda.synchronize()
    e3 = lambda a32: float((a32.double() - ones["f64"]).abs().sum() / ones["f64"].abs().sum())
    ragged = {"workload": "4096 ragged rows, 64..8192 cells (16.9 M), per-row stretched "
                          "meshes, shift only, order 5", "steps": k3,
              "kernel": ("FP32: k_step_rag (255-cell wave tiles; each call plans every "
                         "node's weights and window cell once, k_plan_rag, inside the "
                         "timed call); FP64: k_step"),
              "f32_twosum": round(wl3.n_cells * k3 / t3 / 1e9, 3),
              "f32_plain_prefix": round(wl3.n_cells * k3 / t3p / 1e9, 3),
              "f32_direct": round(wl3.n_cells * k3 / t3s / 1e9, 3),
              "f64": round(wl3.n_cells * k3 / t3d / 1e9, 3),
              "traffic_f32_twosum": None if rag_rec is None else rag_rec["traffic_bytes_per_launch"],
              "traffic_over_algorithmic_f32_twosum": (None if rag_rec is None else
                                                      round(rag_rec["traffic_over_algorithmic"], 3)),
              "unit": "Gcell-updates/s",
              "algorithmic_bytes_per_cell": {"f32": 16, "f64": 24,
                                             "note": "Q in, Q out, the row's FP64 nodes"},
              "hbm_frac": {"f32_twosum": round(16.0 * wl3.n_cells * k3 / t3 / 1e9
                                               / HBM_PEAK_GBS, 4),
                           "f32_plain_prefix": round(16.0 * wl3.n_cells * k3 / t3p / 1e9
                                                     / HBM_PEAK_GBS, 4),
                           "f32_direct": round(16.0 * wl3.n_cells * k3 / t3s / 1e9
                                               / HBM_PEAK_GBS, 4),
                           "f64": round(24.0 * wl3.n_cells * k3 / t3d / 1e9
                                        / HBM_PEAK_GBS, 4)},
              "one_step_rel_l1_vs_f64": {"f32_twosum": e3(ones["f32_twosum"]),
                                         "f32_plain_prefix": e3(ones["f32_plain_prefix"])}}
    del ones

    # --- the disk on a mesh of random cell sizes (every tile searching) -----
    # the headline's rows, shifts and residual on widths 8**u: no uniform run,
    # so the step's time is the searching tiles' (the arbitrary-mesh case)
    def time_stretched():
        wls = W.stretched_disk()
        rows_s = R.Rows.from_workload(wls, dev)
        v0s = torch.as_tensor(wls.v0, dtype=torch.float64, device=dev)
        qs32 = torch.as_tensor(wls.q0.reshape(-1), dtype=torch.float32, device=dev)
        dvs32 = torch.as_tensor(wls.dv.reshape(-1), dtype=torch.float32, device=dev)
        sched_keep = ctx.get_schedule()
        ctx.set_schedule(0)
        spaths = ctx.ram_step_tile_paths(rows_s, v0s, wls.dt, order, True).cpu().numpy()
        ks = max(1, args.steps // 5)
        stretched = {"workload": wls.name + " (the disk's rows, shifts and residual; azimuthal "
                                 "cell widths 8**u, u ~ U[0,1)), FP32, order 5, fused residual, "
                                 "default schedule",
                     "steps": ks, "unit": "Gcell-updates/s", "algorithmic_bytes_per_cell": 12,
                     "tiles": {"uniform_run": int((spaths == R.RAM_TILE_UNIFORM).sum()),
                               "searching": int((spaths == R.RAM_TILE_WINDOW).sum()),
                               "direct": int((spaths == R.RAM_TILE_DIRECT).sum())}}
        for name, scan in (("f32_direct", R.RAM_SUM_DIRECT),
                           ("f32_twosum", R.RAM_SCAN_F32_TWOSUM)):
            ts, _ = time_steps(qs32, dvs32, scan, ks, args.warmup, rows_s, v0s, wls.dt)
            stretched[name] = round(wls.n_cells * ks / ts / 1e9, 3)
            stretched[name + "_us_per_step"] = round(ts / ks * 1e6, 2)
            stretched[name + "_hbm_frac"] = round(12.0 * wls.n_cells * ks / ts / 1e9
                                                  / HBM_PEAK_GBS, 4)
        ctx.set_schedule(sched_keep)
        del rows_s, qs32, dvs32, v0s
        return stretched

    stretched = None
    if not args.no_stretched:
        stretched = time_stretched()

    # --- growth of max |Q| per configuration (reading C14) ------------------

    # the unlimited order-p interpolant can amplify on rough meshes; each
    # config reports max|Q_T| / max|Q_0| over its configured steps (FP64),
    # and for the ragged rows the first 10-step mark where an order's max |Q|
    # has more than doubled, with the limited reconstructions beside them
    def growth(rws, qq, vv, dd, dtt, od, steps, chunk=10, recon=0):
        q = qq.clone()
        m0 = float(q.abs().max())
        first = None
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            if recon:
                for _ in range(k):
                    tmp = torch.empty_like(q)
                    ctx.ram_shift_limited(rws, q, tmp, vv, dtt, recon)
                    q = tmp
            else:
                ctx.ram_step(rws, q, vv, dd, dtt, od, k, R.RAM_SCAN_F64)
            done += k
            m = float(q.abs().max())
            if first is None and not (m <= 2.0 * m0):
                first = done
        return {"steps": steps, "max_growth": float(q.abs().max()) / m0,
                "first_step_doubled": first}
    stability = {"note": "FP64 paths; max|Q_T| / max|Q_0| and the first 10-step mark where "
                         "max|Q| exceeded twice its start (null: never)"}
    q3d = q3.double()
    for od in (1, 3, 5):
        stability[f"cfg3_ragged_order{od}"] = growth(rows3, q3d, v03, None, wl3.dt, od, 200)
    for name, rc in (("plm", R.RAM_RECON_PLM), ("ppm", R.RAM_RECON_PPM)):
        stability[f"cfg3_ragged_{name}"] = growth(rows3, q3d, v03, None, wl3.dt, 0, 200,
                                                  recon=rc)
    del q3d, q3
    stability["cfg5_disk_order5"] = growth(rows, q64, v0, dv64, wl.dt, order, 200)
    for cfg in (1, 2, 4):
        wc = W.CONFIGS[cfg]()
        rc_ = R.Rows.from_workload(wc, dev)
        qc = torch.as_tensor(wc.q0.reshape(-1), dtype=torch.float64, device=dev)
        dc = None if wc.dv is None else torch.as_tensor(wc.dv.reshape(-1), dtype=torch.float64,
                                                        device=dev)
        vc = torch.as_tensor(wc.v0, dtype=torch.float64, device=dev)
        stability[f"cfg{cfg}"] = growth(rc_, qc, vc, dc, wc.dt, wc.order, wc.steps, chunk=50)
        del rc_, qc, dc, vc, wc
    torch.cuda.synchronize()

    # --- the shift-only and residual-only kernels on their own --------------
    h32 = torch.empty_like(q32)
    o32 = torch.empty_like(q32)
    reps = 50
    t_shift = time_kernel(lambda: ctx.ram_shift(rows, q32, h32, v0, wl.dt, order, HEAD),
                          reps)
    t_res = time_kernel(lambda: ctx.ram_residual(rows, h32, o32, dv32, wl.dt), reps)
    fused_bytes = 12.0 * n_cells         # read Q, read dv, write Q'' (FP32)
    kernels = {"step_fused_f32_direct_us": t_fused * 1e6,
               "shift_only_f32_direct_us": t_shift * 1e6,
               "residual_only_f32_us": t_res * 1e6,
               "fused_algorithmic_bytes_per_cell": 12,
               "shift_only_algorithmic_bytes_per_cell": 8,
               "residual_only_algorithmic_bytes_per_cell": 12}
    achieved = fused_bytes / t_fused / 1e9
    # a plain device copy of the same order of bytes on this machine, for scale
    src_c = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst_c = torch.empty_like(src_c)
    t_copy = time_kernel(lambda: dst_c.copy_(src_c), 20)
    copy_gbs = 2.0 * COPY_BYTES / t_copy / 1e9
    del src_c, dst_c
    streaming = items == 0 and not use_density
    if streaming:
        # one step = the uniform-run tiles' kernel, then the other tiles'
        head_kernel = f"{UNI_KERNEL} + {GEN_KERNEL}"
        tru = load_traffic(TRAFFIC_FILE_UNI, UNI_KERNEL)
        trg = load_traffic(TRAFFIC_FILE_GEN, GEN_KERNEL)
        traffic = None if tru is None or trg is None else \
            tru["traffic_bytes_per_launch"] + trg["traffic_bytes_per_launch"]
        paths = ctx.ram_step_tile_paths(rows, v0, wl.dt, order, True).cpu().numpy()
        tiles = {"uniform_run": int((paths == R.RAM_TILE_UNIFORM).sum()),
                 "searching": int((paths == R.RAM_TILE_WINDOW).sum()),
                 "direct": int((paths == R.RAM_TILE_DIRECT).sum()), "cells_per_tile": 256}
    else:
        head_kernel = f"k_step_sh<float, 5, 3, 2, 0, {items or 4}, {idx}>"
        tr = load_traffic(TRAFFIC_FILE, head_kernel)
        traffic = None if tr is None else tr["traffic_bytes_per_launch"]
        tiles = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "traffic_unit": "HBM bytes per step (FETCH_SIZE + WRITE_SIZE, copy-scaled, "
                                "summed over the step's kernels)",
                "traffic_over_algorithmic": None if traffic is None
                else round(traffic / fused_bytes, 3),
                "algorithmic_bytes_per_launch": fused_bytes,
                "algorithmic_unit": "12 B a cell (Q in, dv in, Q out; FP32) x 33554432 cells, "
                                    "per step",
                "copy_achieved": round(copy_gbs, 1),
                "copy_note": "torch device copy of 256 MiB (read + write) on the same GPU",
                "tiles": tiles,
                "kernel": head_kernel + " (FP32, order 5, direct sums, fused residual; "
                          + ("the step's two kernels timed together by HIP events around "
                             "the step loop" if streaming
                             else f"{items or 4} nodes per thread, "
                                  f"{'closed-form' if idx else 'bucket'} index") + ")"}

    # --- limited reconstructions (PLM / PPM bulk shift, then the residual) --
    # two kernels a step: the limited shift and the residual step alone
    def time_limited(q0, dv, recon, steps, warmup):
        q = q0.clone()
        ctx.ram_step_limited(rows, q, v0, dv, wl.dt, recon, steps)     # captures
        q.copy_(q0)
        ctx.ram_step_limited(rows, q, v0, dv, wl.dt, recon, warmup)
        torch.cuda.synchronize()
        a, b = events()
        a.record()
        ctx.ram_step_limited(rows, q, v0, dv, wl.dt, recon, steps)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3

    # one fused kernel a step (limited shift + residual): its average launch
    # is the region time over the steps; algorithmic bytes as the headline
    limited = {"unit": "Gcell-updates/s", "steps": max(1, args.steps // 4),
               "step_algorithmic_bytes_per_cell": {"f32": 12, "f64": 24},
               "kernel": ("FP32: k_step_uni_lim (uniform-run tiles at the tile's theta) + "
                          "k_step_gen_lim (the rest: windows of up to 400 cells tabulated in "
                          "LDS -- slopes, interfaces, each cell's cubic -- wider ones integrated "
                          "from global memory) on the streaming plan; FP64: k_step_sh<double, "
                          "3 (PLM) / 5 "
                          "(PPM), direct sums, fused residual, recon>")}
    kl = limited["steps"]
    tr_pu = load_traffic(TRAFFIC_FILE_PPM_UNI, PPM_UNI_KERNEL)
    tr_pg = load_traffic(TRAFFIC_FILE_PPM_GEN, PPM_GEN_KERNEL)
    tr_ppm = (tr_pu["traffic_bytes_per_launch"] + tr_pg["traffic_bytes_per_launch"]
              if tr_pu and tr_pg else None)
    for name, recon in (("plm", R.RAM_RECON_PLM), ("ppm", R.RAM_RECON_PPM)):
        for tag, qq, dd, nb in (("f32", q32, dv32, 12.0), ("f64", q64, dv64, 24.0)):
            t_l = time_limited(qq, dd, recon, kl, args.warmup)
            hh = torch.empty_like(qq)
            t_sh = time_kernel(lambda: ctx.ram_shift_limited(rows, qq, hh, v0, wl.dt, recon),
                               reps)
            del hh
            ent = {"value": round(n_cells * kl / t_l / 1e9, 3),
                   "step_kernel_us": round(t_l / kl * 1e6, 2),
                   "hbm_frac": round(nb * n_cells / (t_l / kl) / 1e9 / HBM_PEAK_GBS, 4),
                   "shift_only_kernel_us": round(t_sh * 1e6, 2)}
            if name == "ppm" and tag == "f32":
                ent["traffic"] = None if tr_ppm is None else round(tr_ppm)
                ent["traffic_over_algorithmic"] = (None if tr_ppm is None
                                                   else round(tr_ppm / (12.0 * n_cells), 3))
            limited[f"{name}_{tag}"] = ent
    # forward + adjoint of the PPM rollout (checkpointed, FP32 state): each
    # backward step is the residual adjoint, then the limited shift adjoint
    kla = max(1, args.adj_steps // 2)
    qa = q32.clone().requires_grad_(True)
    dva = dv32.clone().requires_grad_(True)
    v0a = v0.clone().requires_grad_(True)
    g = torch.ones_like(q32)
    out = rollout(qa, rows, v0a, dva, wl.dt, order, min(kla, 10), args.checkpoint,
                  recon=R.RAM_RECON_PPM)
    out.backward(g)                      # warm-up
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    out = rollout(qa, rows, v0a, dva, wl.dt, order, kla, args.checkpoint,
                  recon=R.RAM_RECON_PPM)
    out.backward(g)
    b.record()
    torch.cuda.synchronize()
    t_lfa = a.elapsed_time(b) / 1e3
    del out
    # the same with every state kept ((2 kla + 1) states in HBM, no recompute
    # of the forward in the backward pass); one untimed pass first so the
    # allocator holds the trajectory's memory
    out = rollout(qa, rows, v0a, dva, wl.dt, order, kla, 0, recon=R.RAM_RECON_PPM)
    out.backward(g)
    del out
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    out = rollout(qa, rows, v0a, dva, wl.dt, order, kla, 0, recon=R.RAM_RECON_PPM)
    out.backward(g)
    b.record()
    torch.cuda.synchronize()
    t_lfa_all = a.elapsed_time(b) / 1e3
    del out
    hh, oo = torch.ones_like(q32), torch.empty_like(q32)
    t_ladj = time_kernel(lambda: ctx.ram_shift_limited_adjoint(
        rows, q32, hh, oo, v0, wl.dt, R.RAM_RECON_PPM), reps)
    # one limited step backwards with every gradient (the residual's
    # transpose fused)
    dvb_l, v0b_l = torch.zeros_like(dv32), torch.zeros_like(v0)
    g1 = torch.ones_like(q32)
    t_lsadj = time_kernel(lambda: ctx.ram_step_limited_adjoint(
        rows, q32, q32, dv32, g1, oo, v0, wl.dt, R.RAM_RECON_PPM, dvb_l, v0b_l), reps)
    del hh, oo, dvb_l, v0b_l, g1
    tr_ladj = load_traffic(TRAFFIC_FILE_LADJ, LADJ_KERNEL)
    tr_lsadj = load_traffic(TRAFFIC_FILE_LSADJ, LSADJ_KERNEL)
    limited["ppm_f32"]["fwd_adjoint"] = {
        "value": round(n_cells * kla / t_lfa / 1e9, 3),
        "steps": kla, "checkpoint": args.checkpoint,
        "value_all_states_kept": round(n_cells * kla / t_lfa_all / 1e9, 3),
        "state_memory_gb_all_states_kept": round((2 * kla + 1) * n_cells * 4 / 1e9, 1),
        "shift_adjoint_kernel": LADJ_KERNEL,
        "shift_adjoint_call_us": round(t_ladj * 1e6, 2),
        "shift_adjoint_algorithmic_bytes_per_cell": 12,
        "shift_adjoint_hbm_frac_of_call": round(12.0 * n_cells / t_ladj / 1e9 / HBM_PEAK_GBS, 4),
        "shift_adjoint_traffic": None if tr_ladj is None
        else round(tr_ladj["traffic_bytes_per_launch"]),
        "step_adjoint_kernel": LSADJ_KERNEL + " (residual transpose fused, every gradient)",
        "step_adjoint_call_us": round(t_lsadj * 1e6, 2),
        "step_adjoint_algorithmic_bytes_per_cell": 28,
        "step_adjoint_hbm_frac_of_call": round(28.0 * n_cells / t_lsadj / 1e9 / HBM_PEAK_GBS, 4),
        "step_adjoint_traffic": None if tr_lsadj is None
        else round(tr_lsadj["traffic_bytes_per_launch"])}

    # --- forward + adjoint (checkpointed rollout) ---------------------------
    ka = args.adj_steps
    qa = q32.clone().requires_grad_(True)
    dva = dv32.clone().requires_grad_(True)
    v0a = v0.clone().requires_grad_(True)
    g = torch.ones_like(q32)
    out = rollout(qa, rows, v0a, dva, wl.dt, order, min(ka, 20), args.checkpoint, HEAD)
    out.backward(g)                      # warm-up
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    out = rollout(qa, rows, v0a, dva, wl.dt, order, ka, args.checkpoint, HEAD)
    out.backward(g)
    b.record()
    torch.cuda.synchronize()
    t_adj = a.elapsed_time(b) / 1e3
    v_adj = n_cells * ka / t_adj / 1e9
    # the same with every state kept ((2 ka + 1) states in HBM, no recompute);
    # one untimed pass first so the allocator holds the trajectory's memory
    del out
    out = rollout(qa, rows, v0a, dva, wl.dt, order, ka, 0, HEAD)
    out.backward(g)
    del out
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    out = rollout(qa, rows, v0a, dva, wl.dt, order, ka, 0, HEAD)
    out.backward(g)
    b.record()
    torch.cuda.synchronize()
    t_adj_all = a.elapsed_time(b) / 1e3
    v_adj_all = n_cells * ka / t_adj_all / 1e9
    del out
    # the same rollout when only Q0 needs a gradient (v0 a fixed profile, dv
    # given): the kernels skip the dv and v0 terms
    qo_ = q32.clone().requires_grad_(True)
    out = rollout(qo_, rows, v0, dv32, wl.dt, order, min(ka, 20), args.checkpoint, HEAD)
    out.backward(g)
    torch.cuda.synchronize()
    a, b = events()
    a.record()
    out = rollout(qo_, rows, v0, dv32, wl.dt, order, ka, args.checkpoint, HEAD)
    out.backward(g)
    b.record()
    torch.cuda.synchronize()
    v_adj_q0 = n_cells * ka / (a.elapsed_time(b) / 1e3) / 1e9
    del out, qo_
    # one backward step with every gradient, alone: the call (its mesh tables,
    # tile plan and edge sums included) against the step's algorithmic bytes;
    # then the same steps walked back over a recorded trajectory in one call
    # (ram_step_adjoint_steps: one tile plan for all of them), per step
    half = torch.empty_like(q32)
    ctx.ram_shift(rows, q32, half, v0, wl.dt, order, R.RAM_SUM_DIRECT)
    qb_in, qb_out = torch.ones_like(q32), torch.empty_like(q32)
    dvb, v0b = torch.zeros_like(dv32), torch.zeros_like(v0)
    t_adj_call = time_kernel(lambda: ctx.ram_step_adjoint(rows, q32, half, dv32, qb_in, qb_out,
                                                          v0, wl.dt, order, dvb, v0b), 20)
    ks = 20
    traj_s = torch.empty((ks + 1, n_cells), dtype=torch.float32, device=dev)
    half_s = torch.empty((ks, n_cells), dtype=torch.float32, device=dev)
    traj_s[0].copy_(q32)
    ctx.ram_step_record(rows, traj_s, half_s, v0, dv32, wl.dt, order, ks, HEAD)
    qb_s, work_s = torch.ones_like(q32), torch.empty_like(q32)
    t_adj_steps = time_kernel(lambda: ctx.ram_step_adjoint_steps(
        rows, traj_s, half_s, dv32, qb_s, work_s, v0, wl.dt, order, ks, dvb, v0b), 3) / ks
    del traj_s, half_s, qb_s, work_s
    adj_bytes = 28 * n_cells
    tr_au = load_traffic(TRAFFIC_FILE_ADJ_UNI, ADJ_UNI_KERNEL)
    tr_ag = load_traffic(TRAFFIC_FILE_ADJ_GEN, ADJ_GEN_KERNEL)
    adj_traffic = None if tr_au is None or tr_ag is None else \
        tr_au["traffic_bytes_per_launch"] + tr_ag["traffic_bytes_per_launch"]
    apaths = ctx.ram_step_tile_paths(rows, v0, wl.dt, order, False).cpu().numpy()
    adjoint_step = {
        "kernel": f"{ADJ_UNI_KERNEL} + {ADJ_GEN_KERNEL} (FP32, order 5, fused residual "
                  "transpose, every gradient; tiles of 256 cells a wave on the shift's plan)",
        "tiles": {"uniform_run": int((apaths == R.RAM_TILE_UNIFORM).sum()),
                  "searching": int((apaths == R.RAM_TILE_WINDOW).sum()),
                  "direct": int((apaths == R.RAM_TILE_DIRECT).sum())},
        "call_us": round(t_adj_call * 1e6, 2),
        "per_step_us_in_a_multi_step_call": round(t_adj_steps * 1e6, 2),
        "multi_step_call_steps": ks,
        "algorithmic_bytes_per_cell": 28,
        "bytes_note": "Qbar in and out, Q half-step, dv, dvbar read and written, Q for v0bar",
        "hbm_frac_of_call": round(adj_bytes / t_adj_call / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_frac_per_step_multi_step": round(adj_bytes / t_adj_steps / 1e9 / HBM_PEAK_GBS, 4),
        "traffic": None if adj_traffic is None else round(adj_traffic),
        "traffic_unit": "HBM bytes per step, both kernels (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "traffic_over_algorithmic": None if adj_traffic is None
        else round(adj_traffic / adj_bytes, 3)}
    del half, qb_in, qb_out, dvb, v0b

    # --- accuracy: one FP32 step against the FP64 path (itself held to the
    # oracle at 1e-12 by the GPU tests) from the same FP32-rounded input, over
    # the whole disk; rollout drift
    n = wl.n_cols
    q32w = q32.double()
    dv32w = dv32.double()

    def rel_gpu(a32, b64):
        return float((a32.double() - b64).abs().sum() / b64.abs().sum())

    one = q32.clone()
    ctx.ram_step(rows, one, v0, dv32, wl.dt, order, 1, HEAD)
    ref64 = q32w.clone()
    ctx.ram_step(rows, ref64, v0, dv32w, wl.dt, order, 1, R.RAM_SCAN_F64)
    torch.cuda.synchronize()
    err1 = rel_gpu(one, ref64)
    for name, recon in (("plm", R.RAM_RECON_PLM), ("ppm", R.RAM_RECON_PPM)):
        one = q32.clone()
        ctx.ram_step_limited(rows, one, v0, dv32, wl.dt, recon, 1)
        ref64 = q32w.clone()
        ctx.ram_step_limited(rows, ref64, v0, dv32w, wl.dt, recon, 1)
        torch.cuda.synchronize()
        limited[f"{name}_f32"]["one_step_rel_l1_vs_fp64_path"] = rel_gpu(one, ref64)
    del one, ref64, q32w, dv32w
    # drift of the FP32 rollout against the FP64 path after the same steps
    q_ref = q64.clone()
    ctx.ram_step(rows, q_ref, v0, dv64, wl.dt, order, args.steps + args.warmup,
                 R.RAM_SCAN_F64)
    torch.cuda.synchronize()
    drift = float((q_ts.double() - q_ref).abs().sum() / q_ref.abs().sum())

    # --- CPU oracle baseline on a bounded sample ----------------------------
    cpu = None
    oracle_err = None
    if not args.no_cpu:
        import oracle                      # the CPU baseline leg only
        cores = len(os.sched_getaffinity(0))

        def cpu_model_string():
            fields = {}
            try:
                with open("/proc/cpuinfo") as fh:
                    for line in fh:
                        if ":" in line:
                            k_, v_ = line.split(":", 1)
                            fields.setdefault(k_.strip(), v_.strip())
            except OSError:
                return None
            return (f"{fields.get('model name', '?')} (family {fields.get('cpu family', '?')}, "
                    f"model {fields.get('model', '?')}, stepping {fields.get('stepping', '?')}, "
                    f"{fields.get('cpu MHz', '?')} MHz)")

        def run_oracle(orows, q, vv, dd, dtt, od, steps, nthreads):
            t0 = time.perf_counter()
            out_ = oracle.step(orows, q, vv, dd, dtt, od, steps, nthreads=nthreads)
            return time.perf_counter() - t0, out_

        # the headline workload: the first rows of the disk, as many FP64
        # steps as fit the time budget, on every core this process may use
        n_s = 128
        sub = oracle.Rows(np.arange(n_s + 1) * n, wl.edges, True)
        qs = wl.q0[:n_s].astype(np.float64)
        t1, _ = run_oracle(sub, qs, wl.v0[:n_s], wl.dv[:n_s], wl.dt, order, 1, cores)
        steps_s = max(1, int(args.cpu_seconds / max(t1, 1e-3)))
        tc, _ = run_oracle(sub, qs, wl.v0[:n_s], wl.dv[:n_s], wl.dt, order, steps_s, cores)
        # one thread on a smaller sample (the same rows' first 16)
        n_1 = 16
        sub1 = oracle.Rows(np.arange(n_1 + 1) * n, wl.edges, True)
        k_1 = max(1, steps_s // 4)
        t_1, _ = run_oracle(sub1, wl.q0[:n_1].astype(np.float64), wl.v0[:n_1], wl.dv[:n_1],
                            wl.dt, order, k_1, 1)
        # every configuration: configs 1-3 over their full step counts on every
        # core (config 3 on one thread over its first 64 rows), configs 4-5 over
        # a 20-step window; one thread over bounded samples of each
        plan = {}

        def rate(cells, steps, sec):
            return round(cells * steps / sec / 1e9, 5)
        for cfg in (1, 2, 3, 4, 5):
            wc = wl3 if cfg == 3 else (wl if cfg == 5 else W.CONFIGS[cfg]())
            orows_c = oracle.Rows.from_workload(wc)
            q0c = wc.q0.reshape(-1).astype(np.float64)
            dvc = None if wc.dv is None else wc.dv.reshape(-1)
            full = cfg in (1, 2, 3)
            st_all = wc.steps if full else 20
            t_all, _ = run_oracle(orows_c, q0c, wc.v0, dvc, wc.dt, wc.order, st_all, cores)
            ent = {"all_cores": {"threads": cores, "steps": st_all, "cells": wc.n_cells,
                                 "seconds": round(t_all, 3),
                                 "value": rate(wc.n_cells, st_all, t_all)}}
            # one thread: the whole batch for config 1, the first rows otherwise
            nr = wc.n_rows if cfg == 1 else min(wc.n_rows, {2: 64, 3: 64, 4: 16, 5: 4}[cfg])
            if wc.n_cols > 0:
                w1 = W.Workload("s", nr, wc.n_cols, np.arange(nr + 1) * wc.n_cols, wc.edges, True,
                                wc.q0.reshape(wc.n_rows, -1)[:nr],
                                None if wc.dv is None else wc.dv.reshape(wc.n_rows, -1)[:nr],
                                wc.v0[:nr], wc.dt, wc.order, wc.steps)
            else:
                nc1 = int(wc.row_ptr[nr])
                w1 = W.Workload("s", nr, 0, wc.row_ptr[:nr + 1], wc.edges[:nc1 + nr], False,
                                wc.q0[:nc1], None, wc.v0[:nr], wc.dt, wc.order, wc.steps)
            st_1 = wc.steps if cfg in (1, 3) else 20
            t_one, _ = run_oracle(oracle.Rows.from_workload(w1), w1.q0.reshape(-1).astype(
                np.float64), w1.v0, None if w1.dv is None else w1.dv.reshape(-1), w1.dt,
                w1.order, st_1, 1)
            ent["one_thread"] = {"rows": nr, "steps": st_1, "cells": w1.n_cells,
                                 "seconds": round(t_one, 3),
                                 "value": rate(w1.n_cells, st_1, t_one)}
            if not full:
                ent["extrapolation"] = (f"full run of {wc.steps} steps: about "
                                        f"{t_all * wc.steps / st_all:.0f} s on every core")
            plan[f"cfg{cfg}"] = ent
            del orows_c
        # the GPU's results against the oracle after the same 20 steps from the
        # same start, on sampled rows (FP64 state; the headline FP32 path from
        # the FP32-rounded start)
        pick = np.array([0, 1, 700, 1024, 1025, 1700, 2046, 2047])
        sw_ = W.Workload("pick", len(pick), n, np.arange(len(pick) + 1) * n, wl.edges, True,
                         wl.q0[pick], wl.dv[pick], wl.v0[pick], wl.dt, order, 20)
        orp = oracle.Rows.from_workload(sw_)
        area = (np.diff(wl.edges)[None, :] * 0.5 *
                np.diff(np.asarray(wl.meta["r_edges"]) ** 2)[pick][:, None]).reshape(-1)
        ref64 = oracle.step(orp, sw_.q0.reshape(-1), sw_.v0, sw_.dv.reshape(-1), wl.dt, order,
                            20, nthreads=cores)
        q32h = wl.q0.astype(np.float32).astype(np.float64)[pick]
        dv32h = wl.dv.astype(np.float32).astype(np.float64)[pick]
        ref32 = oracle.step(orp, q32h.reshape(-1), sw_.v0, dv32h.reshape(-1), wl.dt, order, 20,
                            nthreads=cores)
        g64 = q64.clone()
        ctx.ram_step(rows, g64, v0, dv64, wl.dt, order, 20, R.RAM_SCAN_F64)
        g32 = q32.clone()
        ctx.ram_step(rows, g32, v0, dv32, wl.dt, order, 20, HEAD)
        torch.cuda.synchronize()

        def rel_w(got, ref):
            return float(np.sum(np.abs(got - ref) * area) / np.sum(np.abs(ref) * area))
        got64 = g64.cpu().numpy().reshape(wl.n_rows, -1)[pick].reshape(-1)
        got32 = g32.double().cpu().numpy().reshape(wl.n_rows, -1)[pick].reshape(-1)
        oracle_err = {"steps": 20, "rows": pick.tolist(),
                      "norm": "rel-L1 weighted by cell area (r dr dphi)",
                      "fp64_plain_rel_l1": rel_w(got64, ref64),
                      "fp32_direct_rel_l1": rel_w(got32, ref32),
                      "fp32_direct_max_cell_rel": float(np.max(np.abs(got32 - ref32))
                                                        / np.max(np.abs(ref32)))}
        del g64, g32
        cpu = {"value": n_s * n * steps_s / tc / 1e9, "unit": "Gcell-updates/s",
               "cores": cores, "kind": "oracle",
               "sample": f"first {n_s} of 2048 rows x 16384 cells, {steps_s} FP64 steps "
                         f"(shift + residual), {tc:.1f} s, {cores} threads "
                         f"(os.sched_getaffinity)",
               "single_thread_value": n_1 * n * k_1 / t_1 / 1e9,
               "single_thread_sample": f"first {n_1} rows, {k_1} steps, {t_1:.1f} s",
               "cpu_model": cpu_model_string(),
               "configs": plan}

    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_ts / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "polar disk 2048 rows x 16384 cells, periodic-bump "
                               "azimuthal mesh (10x refined |phi|<0.2), Keplerian v0, "
                               "order-5 shift + van Leer residual",
                   "rows": wl.n_rows, "cols": n, "order": order,
                   "cumulative_differences": "summed directly from FP32 masses (no prefix)",
                   "dt": wl.dt},
        "fwd_adjoint": {"value": round(v_adj, 3), "unit": "Gcell-updates/s",
                        "steps": ka, "checkpoint": args.checkpoint},
        "fwd_adjoint_q0_grad_only": {"value": round(v_adj_q0, 3), "unit": "Gcell-updates/s",
                                     "steps": ka, "checkpoint": args.checkpoint},
        "adjoint_step": adjoint_step,
        "fwd_adjoint_all_states_kept": {"value": round(v_adj_all, 3),
                                        "unit": "Gcell-updates/s", "steps": ka,
                                        "state_memory_gb": round((2 * ka + 1) * n_cells * 4
                                                                 / 1e9, 1)},
        "fp32_fp64scan": mode_rec(v_f64s, t_f64s, k2, 12, fp32_kernel),
        "fp32_twosum_prefix": mode_rec(v_two, t_two, k2s, 12, fp32_kernel),
        "fp32_plain_prefix": mode_rec(v_p32, t_p32, k2, 12, fp32_kernel),
        "fp64_plain": dict(mode_rec(v64, t64, args.fp64_steps, 24, fp64_kernel),
                           cumulative_differences="FP64 window prefix sums",
                           traffic=tr_f64["traffic_bytes_per_launch"] if tr_f64 else None,
                           traffic_over_algorithmic=(round(tr_f64["traffic_over_algorithmic"], 3)
                                                     if tr_f64 else None)),
        "fp64_direct": dict(mode_rec(v64d, t64d, args.fp64_steps, 24,
                                     fp64_kernel_of(items64, False)),
                            cumulative_differences="summed directly in FP64",
                            items_per_thread=items64,
                            tuned_us_per_step={str(k): round(v, 2) for k, v in tune64.items()}),
        "mixed_speedup_vs_fp64": round(value / v64, 3),
        "mixed_speedup_vs_fp64_direct": round(value / v64d, 3),
        "error": {"one_step_rel_l1_vs_fp64_path": err1,
                  "rollout_rel_l1_vs_fp64_path": drift,
                  "rollout_steps": args.steps + args.warmup,
                  "vs_oracle": oracle_err},
        "stability": stability,
        "schedule": schedule,
        "fast_index": fast_index,
        "std_baseline": std_baseline,
        "split_2d": split_2d,
        "centre_values_4th_order": point4,
        "ragged_cfg": ragged,
        "stretched_disk": stretched,
        "limited_reconstructions": limited,
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(_finite(res), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
