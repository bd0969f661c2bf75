#!/usr/bin/env python3
"""Benchmark of the SMPC plan step on one MI355X.

Workload (the reactive-replanning configuration): K = 4096 rollouts, H = 40
steps, dt = 0.02 s, a 200^3 float32 signed distance grid at 0.01 m built from 20
boxes and 20 spheres drifting at 0.2 m/s, a target moving on a 0.3 m circle, the
7-DoF arm with 28 collision spheres and 240 self-collision pairs, temperature 1.
All inputs are seeded synthetic data and are resident in device memory before
timing starts.

One step = one control period of the closed loop on a fresh grid: one plan step
(smpc_plan_step_then_bounds) that reads the joint state and nominal sequence the
previous period left on the device, executes u*_0 for one period and shifts the
nominal sequence (receding horizon), and whose rollout launch also builds the coarse
lower bounds of the next period's grid over the cells the arm can reach (as
smpc_grid_coarse_min_ball with smpc_robot_reach) into the second of two tables
(--no-fuse-bounds: each period builds its own grid's bounds by a launch of their
own before its plan step).  The grids of consecutive periods (built on the device
from the scene's occupancy) and the disturbances cycle through pools of distinct
device buffers.

Printed: one JSON line with rollout-steps/s (K*H per second) from back-to-back
periods, per-period latency percentiles (each period synchronised on its own: the
bounds of its own grid, then smpc_plan_step), the
rollout-cost kernel's duration against the FP32 VALU peak (and the L2 side when its
counters match the sources), the same plan steps on one static grid, and the FP64
oracle's closed loop on one host thread.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout-steps/s (K·H/s) at K=4096,H=40; p50/p99 plan-step latency"
# Algorithmic work of one rollout step (FP32 FLOP, FMA = 2): integration, FK,
# sphere centres, trilinear distance lookups, self pairs, limits, pose log map.
FLOP_PER_ROLLOUT_STEP = 4300.0
# Logical distance-field gathers per rollout step: 28 spheres x 8 corners x 4 B.
GATHER_BYTES_PER_ROLLOUT_STEP = 896.0
PEAK_FP32_TFLOPS = 157.3

# HBM traffic of one rollout-cost launch on the default workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over dispatches), each
# scaled by what the counter reads for a plain 256 MiB device copy (FETCH_SIZE
# reads half the bytes copied: x2; WRITE_SIZE reads them all: x1).  Valid only for
# the kernel sources it was taken on: bench.py reports null traffic when their
# hash differs.
ROLLOUT_TRAFFIC = {"sources_sha256": "188e26cae7c3a2936ac4d546c21edf32063817c72ba26a689ab890931367897c",
                   "fetch_kib": 2740.7, "fetch_scale": 2.0,
                   "write_kib": 853.8, "write_scale": 1.0}
# The same for one occupancy update (pixel and voxel pass together) at 200^3, 640x480.
OGM_TRAFFIC = {"sources_sha256": "188e26cae7c3a2936ac4d546c21edf32063817c72ba26a689ab890931367897c",
               "fetch_kib": 673.8 + 20301.4, "fetch_scale": 2.0,
               "write_kib": 1200.5 + 39062.5, "write_scale": 1.0}


# L2 requests of one rollout-cost launch on the default workload (rocprofv3 --pmc
# TCC_REQ_sum, per dispatch), taken on the kernel sources named by the hash.  The L2
# side of the roofline counts 128 B per request against the L2 peak of
# PEAK_L2_GBPS: 8 XCDs x 16 channels x 128 B per clock x 2.4 GHz.
ROLLOUT_L2 = {"sources_sha256": "188e26cae7c3a2936ac4d546c21edf32063817c72ba26a689ab890931367897c", "tcc_req": 226746.3}
PEAK_L2_GBPS = 8 * 16 * 128 * 2.4


def rollout_l2(k1_ms):
    if not ROLLOUT_L2["sources_sha256"] or ROLLOUT_L2["sources_sha256"] != kernel_sources_sha256():
        return None
    gbs = ROLLOUT_L2["tcc_req"] * 128.0 / (k1_ms * 1e-3) / 1e9
    return {"achieved": round(gbs, 1), "peak": round(PEAK_L2_GBPS, 1), "unit": "GB/s",
            "frac": round(gbs / PEAK_L2_GBPS, 4), "requests_per_launch": ROLLOUT_L2["tcc_req"],
            "bytes_per_request": 128}


def kernel_sources_sha256(names=("smpc_kernels.hip", "smpc_internal.h")) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2512_22575_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes(t):
    if t is None or t["sources_sha256"] != kernel_sources_sha256(t.get("sources",
                                                                       ("smpc_kernels.hip",
                                                                        "smpc_internal.h"))):
        return None
    return round(1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def rollout_traffic_bytes():
    return traffic_bytes(ROLLOUT_TRAFFIC)


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--latency-steps", type=int, default=300)
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--pool", type=int, default=16, help="distinct noise buffers cycled")
    ap.add_argument("--grids", type=int, default=16,
                    help="distinct consecutive-period grids cycled by the closed loop")
    ap.add_argument("--static-steps", type=int, default=200,
                    help="extra figure: plan steps on one grid with its bounds built once")
    ap.add_argument("--paper-shaped", action="store_true",
                    help="time periods at the paper's M = 512 on its 150x150x25 map at 0.02 m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="default run only: skip the serving, variant, distance-field and "
                         "occupancy summaries appended to the line")
    ap.add_argument("--no-coarse", action="store_true",
                    help="plan without the coarse lower bounds of the grid")
    ap.add_argument("--no-fuse-bounds", action="store_true",
                    help="build each period's bounds by a launch of their own before its plan "
                         "step instead of in the previous period's merge launch")
    ap.add_argument("--K", type=int, default=4096)
    ap.add_argument("--H", type=int, default=40)
    ap.add_argument("--n", type=int, default=200, help="grid side in voxels")
    ap.add_argument("--serving", action="store_true",
                    help="run the multi-controller serving benchmark instead")
    ap.add_argument("--controllers", type=int, default=64)
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=2000.0, help="mean arrivals per second")
    ap.add_argument("--budget-mib", type=int, default=512, help="server HBM budget")
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--variants", action="store_true",
                    help="time the float16-grid and on-device-sampling variants of the plan "
                         "step against the float32 path (mid and reactive workloads)")
    ap.add_argument("--ogm", action="store_true",
                    help="time the occupancy update (640x480 depth image into the 200^3 map, "
                         "robot mask on) and the mapping-to-plan pipeline instead")
    ap.add_argument("--edt", action="store_true",
                    help="time the distance-field construction (200^3 occupancy -> signed "
                         "field) and the construction + plan step pipeline instead")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (to scale "
                         "HBM byte counters) and exit")
    return ap.parse_args()


def calibrate_copy(mib: int) -> None:
    """A plain copy kernel of known size, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": 3}), flush=True)


def serving_bench(args) -> dict:
    """Poisson request stream over many controllers through the batching server."""
    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import serving as SV

    t_gen = time.perf_counter()
    rob, ctl = SV.make_controllers(5, args.controllers)
    trace = SV.make_trace(5, ctl, args.requests, args.rate)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    grids = [torch.from_numpy(c.grid).to(dev) for c in ctl]
    planner = S.Planner(rob, device=0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    total_rs = sum(ctl[r.controller].K * ctl[r.controller].H for r in trace)
    n = len(trace)

    def new_server():
        srv = S.Server(planner, hbm_budget_bytes=args.budget_mib << 20, max_batch=args.max_batch)
        ids = [srv.add_controller(g, c.origin, c.voxel, c.K, c.H, c.dt, c.lam, c.weights,
                                  c.sigma) for g, c in zip(grids, ctl)]
        return srv, ids

    def run(srv, ids, realtime):
        done_t, batches = {}, 0
        i = 0
        t0 = time.perf_counter()
        while len(done_t) < n:
            now = time.perf_counter() - t0
            while i < n and (not realtime or trace[i].t_arrival <= now):
                r = trace[i]
                srv.submit(i, ids[r.controller], r.q0, r.qd0, r.T_goal, r.seed)
                i += 1
            if srv.pump(stream):
                batches += 1
            for c in srv.poll():
                if c.status != S.SMPC_OK:
                    raise RuntimeError(f"request {c.tag}: status {c.status}")
                done_t[c.tag] = time.perf_counter() - t0
        span = max(done_t.values())
        lat = np.array([done_t[k] - (trace[k].t_arrival if realtime else 0.0) for k in range(n)])
        return span, lat * 1e3, batches

    # Warm-up pass (first launches, allocations), then the timed passes.
    srv, ids = new_server()
    run(srv, ids, realtime=False)
    srv.close()
    srv, ids = new_server()
    rt_span, rt_lat, rt_batches = run(srv, ids, realtime=True)
    srv.close()
    srv, ids = new_server()
    sat_span, _, sat_batches = run(srv, ids, realtime=False)
    srv.close()

    # Sequential plain plan steps (one call per request, each waited for).
    U = [torch.zeros((c.H, 7), device=dev) for c in ctl]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in trace:
        c = ctl[r.controller]
        planner.plan_step(q0=r.q0, qd0=r.qd0, T_goal=r.T_goal, grid=grids[r.controller],
                          origin=c.origin, voxel=c.voxel, noise=None, K=c.K, H=c.H,
                          U_in=U[r.controller], U_out=U[r.controller], dt=c.dt, lam=c.lam,
                          weights=c.weights, seed=r.seed, sigma=c.sigma, stream=stream)
        torch.cuda.synchronize()
    seq_span = time.perf_counter() - t0
    out = {
        "metric": "serving: plan-request latency (arrival to completion) and aggregate "
                  "rollout-steps/s",
        "value": round(float(np.percentile(rt_lat, 99)), 4),
        "unit": "ms (p99 latency)",
        "higher_is_better": False,
        "n_gpus": 1,
        "data": "synthetic",
        "dtype": "f32",
        "config": {"workload": f"{args.controllers} controllers (K in 256..4096, H in 16/32/64, "
                               f"grids 64^3..160^3), {n} requests, Poisson {args.rate:g}/s",
                   "budget_mib": args.budget_mib, "max_batch": args.max_batch,
                   "total_rollout_steps": int(total_rs)},
        "realtime": {"p50_ms": round(float(np.percentile(rt_lat, 50)), 4),
                     "p99_ms": round(float(np.percentile(rt_lat, 99)), 4),
                     "max_ms": round(float(rt_lat.max()), 4),
                     "batches": rt_batches, "span_s": round(rt_span, 4),
                     "replanning_budget_ms": 20.0},
        "saturated": {"rollout_steps_per_s": round(total_rs / sat_span, 1),
                      "span_ms": round(sat_span * 1e3, 3), "batches": sat_batches},
        "sequential_plain": {"rollout_steps_per_s": round(total_rs / seq_span, 1),
                             "span_ms": round(seq_span * 1e3, 3)},
        "setup_s": round(t_gen, 1),
    }
    planner.close()
    return out


# Compulsory traffic of the distance-field construction per voxel: the occupancy
# byte read and the float32 field written.
EDT_BYTES_PER_VOXEL = 5.0
# HBM traffic of one construction at 200^3 (reactive scene; the three kernels together),
# counted and scaled as ROLLOUT_TRAFFIC, valid for the sources named.
EDT_TRAFFIC = {"sources": ("smpc_edt.hip", "smpc_internal.h"),
               "sources_sha256": "119e5d909baa710898ce1b79cae4da3b9b58fdbe07621595edc881dfe20977b3",
               "fetch_kib": 4090.6 + 33223.0 + 31089.6, "fetch_scale": 2.0,
               "write_kib": 15625.0 + 33071.8 + 33859.8, "write_scale": 1.0}
PEAK_HBM_GBPS = 8000.0


def edt_bench(args) -> dict:
    """Distance field from occupancy on the device, alone and followed by a plan step.

    The reactive scene is advanced by one control period per pool entry, so
    consecutive constructions see moving obstacles; occupancy grids are resident in
    device memory (their host-to-device copy is timed separately, from pinned memory).
    """
    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import workload as W

    K, H, n = args.K, args.H, args.n
    sc = W.ReactiveScenario(seed=3, K=K, H=H, n=n)
    dev = torch.device("cuda:0")
    pool = max(1, min(args.pool, 8))
    occs_np = []
    for _ in range(pool):
        occs_np.append(sc.occupancy().astype(np.uint8))
        sc.advance()
    occs = [torch.from_numpy(o).to(dev) for o in occs_np]
    nvox = n ** 3
    need = S.smpc_edt_workspace_bytes(n, n, n)
    work = torch.empty((need + 3) // 4, dtype=torch.int32, device=dev)
    phi = torch.empty((n, n, n), device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def edt(i):
        st = S.smpc_edt(occs[i % pool].data_ptr(), n, n, n, sc.VOXEL, phi.data_ptr(), None,
                        work.data_ptr(), need, stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_status_string(st))

    for i in range(args.warmup):
        edt(i)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        edt(i)
    ev1.record()
    torch.cuda.synchronize()
    edt_ms = ev0.elapsed_time(ev1) / args.steps

    # Host-to-device copy of one occupancy grid from pinned memory.
    pinned = torch.from_numpy(occs_np[0]).pin_memory()
    staging = torch.empty_like(occs[0])
    ev0.record()
    for _ in range(20):
        staging.copy_(pinned, non_blocking=True)
    ev1.record()
    torch.cuda.synchronize()
    h2d_ms = ev0.elapsed_time(ev1) / 20

    # Construction followed by a warm-started plan step on the fresh field.
    noise = [torch.from_numpy(sc.noise()).to(dev) for _ in range(4)]
    U = [torch.zeros((H, 7), device=dev), torch.zeros((H, 7), device=dev)]
    planner = S.Planner(sc.robot, device=0)
    coarse = torch.empty(S.smpc_grid_coarse_cells(n, n, n), device=dev)
    plans = [S.plan_args(sc.q0, sc.qd0, sc.target(), phi, sc.origin, sc.VOXEL, noise[i % 4],
                         U[i % 2], U[(i + 1) % 2], K, H, sc.DT, 1.0, sc.weights, coarse=coarse)
             for i in range(args.steps)]

    def pipeline(i):
        edt(i)
        st = S.smpc_grid_coarse_min_ball(phi, S.GRID_F32, sc.origin, sc.VOXEL, *planner.robot_reach(),
                                         coarse.data_ptr(), stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, "smpc_grid_coarse_min_ball")
        st = S.smpc_plan_step(planner._ctx, plans[i], stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_last_error(planner._ctx))

    for i in range(min(args.warmup, args.steps)):
        pipeline(i)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        pipeline(i)
    ev1.record()
    torch.cuda.synchronize()
    pipe_ms = ev0.elapsed_time(ev1) / args.steps
    planner.close()

    achieved = EDT_BYTES_PER_VOXEL * nvox / (edt_ms * 1e-3) / 1e9
    extra = {}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import edt as E
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            E.signed_distance(occs_np[0], float(np.float32(sc.VOXEL)))
            dt = time.perf_counter() - t0
        extra["cpu_baseline"] = {
            "value": round(nvox / dt, 1), "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"one {n}^3 construction of the same scene (separable FH in float64 "
                      f"numpy, both fields and phi), {dt:.2f} s on one host thread"}
    return {
        "metric": "voxels/s of signed distance field construction (occupancy -> field)",
        "value": round(nvox / (edt_ms * 1e-3), 1),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(edt_ms, 6),
        "higher_is_better": True,
        "dtype": "u32 squared distances, f64 -> f32 field",
        "data": "synthetic",
        "config": {"workload": f"reactive scene occupancy {n}^3 at 0.01 m, 20 boxes and 20 "
                               f"spheres drifting at 0.2 m/s, {pool} consecutive periods",
                   "grid": [n] * 3},
        "roofline": {"bound": "hbm", "kernel": "smpc_edt (3 kernels)",
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": traffic_bytes(EDT_TRAFFIC) if n == 200 else None,
                     "bytes_per_voxel": EDT_BYTES_PER_VOXEL},
        "occupancy_h2d_ms": round(h2d_ms, 5),
        "pipeline_ms_per_step": round(pipe_ms, 5),
        "pipeline": f"smpc_edt, smpc_grid_coarse_min_ball, then smpc_plan_step (K={K}, H={H}) "
                    "on the new field",
        **extra,
    }


# Compulsory traffic of one occupancy update: per voxel the float32 log-odds read and
# written and the occupancy byte written; per pixel the depth read and the cleaned
# depth written.
OGM_BYTES_PER_VOXEL = 9.0
OGM_BYTES_PER_PIXEL = 8.0


def ogm_bench(args) -> dict:
    """Occupancy update of the 200^3 map from one depth image, alone and as the first
    stage of the mapping-to-plan pipeline (map update, field, bounds, plan step).

    The reactive scene is advanced by one control period per pool entry and rendered
    from a fixed camera; images are resident in device memory.  The images hold the
    primitives only (the input generator does no kinematics); the robot mask is on,
    so every valid return still takes the sphere test and the voxels inside the arm
    at q0 are reset.
    """
    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import camera as C
    from synth import workload as W

    K, H, n = args.K, args.H, args.n
    sc = W.ReactiveScenario(seed=3, K=K, H=H, n=n)
    dev = torch.device("cuda:0")
    cam = C.default_camera(640, 480)
    pool = max(1, min(args.pool, 8))
    planner = S.Planner(sc.robot, device=0)
    depths_np = []
    for _ in range(pool):
        depths_np.append(C.render_depth(cam, sc.prims))
        sc.advance()
    depths = [torch.from_numpy(d).to(dev) for d in depths_np]
    scam = S.make_camera(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.T_wc,
                         cam.min_depth, cam.max_depth)
    prm = S.make_ogm_params(tol=0.025, l_hit=0.85, l_miss=-0.4, l_min=-2.0, l_max=3.5,
                            l_occ=0.0, robot_pad=0.01)
    L = torch.zeros((n, n, n), device=dev)
    occ = torch.zeros((n, n, n), dtype=torch.uint8, device=dev)
    work = torch.empty(S.smpc_ogm_workspace_bytes(cam.width, cam.height) // 4, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def ogm(i):
        planner.ogm_update(depth=depths[i % pool], cam=scam, log_odds=L, origin=sc.origin,
                           voxel=sc.VOXEL, prm=prm, work=work, q=sc.q0, occ_out=occ,
                           stream=stream)

    for i in range(args.warmup):
        ogm(i)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        ogm(i)
    ev1.record()
    torch.cuda.synchronize()
    ogm_ms = ev0.elapsed_time(ev1) / args.steps

    # Map update, distance field of the new occupancy, bounds, warm-started plan step.
    nvox = n ** 3
    need = S.smpc_edt_workspace_bytes(n, n, n)
    ework = torch.empty((need + 3) // 4, dtype=torch.int32, device=dev)
    phi = torch.empty((n, n, n), device=dev)
    coarse = torch.empty(S.smpc_grid_coarse_cells(n, n, n), device=dev)
    noise = [torch.from_numpy(sc.noise()).to(dev) for _ in range(4)]
    U = [torch.zeros((H, 7), device=dev), torch.zeros((H, 7), device=dev)]
    plans = [S.plan_args(sc.q0, sc.qd0, sc.target(), phi, sc.origin, sc.VOXEL, noise[i % 4],
                         U[i % 2], U[(i + 1) % 2], K, H, sc.DT, 1.0, sc.weights, coarse=coarse)
             for i in range(args.steps)]

    def pipeline(i):
        ogm(i)
        st = S.smpc_edt(occ.data_ptr(), n, n, n, sc.VOXEL, phi.data_ptr(), None,
                        ework.data_ptr(), need, stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, "smpc_edt")
        st = S.smpc_grid_coarse_min_ball(phi, S.GRID_F32, sc.origin, sc.VOXEL, *planner.robot_reach(),
                                         coarse.data_ptr(), stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, "smpc_grid_coarse_min_ball")
        st = S.smpc_plan_step(planner._ctx, plans[i], stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_last_error(planner._ctx))

    for i in range(min(args.warmup, args.steps)):
        pipeline(i)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        pipeline(i)
    ev1.record()
    torch.cuda.synchronize()
    pipe_ms = ev0.elapsed_time(ev1) / args.steps
    planner.close()

    npix = cam.width * cam.height
    bytes_ = OGM_BYTES_PER_VOXEL * nvox + OGM_BYTES_PER_PIXEL * npix
    achieved = bytes_ / (ogm_ms * 1e-3) / 1e9
    extra = {}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import ogm as G
        from oracle import smpc_oracle as O
        robot = sc.robot.rounded_f32()
        q = np.asarray(sc.q0, np.float32).astype(np.float64)
        centres = O.sphere_centres(robot, O.forward_kinematics(robot, q[None]))[0]
        prm_d = dict(tol=0.025, l_hit=0.85, l_miss=-0.4, l_min=-2.0, l_max=3.5, l_occ=0.0,
                     robot_pad=0.01)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            G.ogm_update(np.zeros((n, n, n), np.float32), depths_np[0], cam,
                         np.asarray(sc.origin, np.float64), float(np.float32(sc.VOXEL)), prm_d,
                         centres, robot.sphere_radius)
            dt = time.perf_counter() - t0
        extra["cpu_baseline"] = {
            "value": round(nvox / dt, 1), "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"one update of the {n}^3 map from one 640x480 image with the robot mask "
                      f"(float64 numpy), {dt:.2f} s on one host thread"}
    return {
        "metric": "voxels/s of occupancy update (one depth image into the log-odds map)",
        "value": round(nvox / (ogm_ms * 1e-3), 1),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ogm_ms, 6),
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"reactive scene {n}^3 log-odds map at 0.01 m, 640x480 depth "
                               f"images of 20 boxes and 20 spheres, robot mask on at q0, "
                               f"{pool} consecutive periods",
                   "grid": [n] * 3, "image": [cam.width, cam.height]},
        "roofline": {"bound": "hbm", "kernel": "smpc_ogm_update (2 kernels)",
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": traffic_bytes(OGM_TRAFFIC) if (n, cam.width) == (200, 640) else None,
                     "bytes_per_voxel": OGM_BYTES_PER_VOXEL,
                     "bytes_per_pixel": OGM_BYTES_PER_PIXEL},
        "pipeline_ms_per_step": round(pipe_ms, 5),
        "pipeline": f"smpc_ogm_update, smpc_edt on its occupancy, smpc_grid_coarse_min_ball, then "
                    f"smpc_plan_step (K={K}, H={H}) on the new field",
        **extra,
    }


def variants_bench(args) -> dict:
    """Plan-step time with the grid in float16 (clamped to +-2 m) and/or the disturbances
    sampled on the device (Philox, sigma 0.5), against float32 grid + disturbance
    buffer, on the mid workload (K=1024, H=32, 64^3) and the reactive one (K=4096,
    H=40, 200^3).  Coarse bounds are built for each grid outside the timed region.
    Warm-started back-to-back steps, events on the launch stream."""
    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import workload as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    cases = {"mid K=1024 H=32 64^3 at 0.03 m": W.mid(),
             "reactive K=4096 H=40 200^3 at 0.01 m": W.ReactiveScenario(seed=3).inputs()}
    out = {}
    for name, inp in cases.items():
        K, H = inp.K, inp.H
        g32 = torch.from_numpy(np.ascontiguousarray(inp.grid)).to(dev)
        g16 = torch.empty(g32.shape, dtype=torch.int16, device=dev)
        ncells = S.smpc_grid_coarse_cells(*reversed(tuple(g32.shape)))
        c32 = torch.empty(ncells, device=dev)
        c16 = torch.empty(ncells, device=dev)
        for st in (S.smpc_grid_to_f16(g32.data_ptr(), g16.data_ptr(), g32.numel(), 2.0, stream),
                   S.smpc_grid_coarse_min(g32, S.GRID_F32, c32.data_ptr(), stream),
                   S.smpc_grid_coarse_min(g16, S.GRID_F16, c16.data_ptr(), stream)):
            if st != S.SMPC_OK:
                raise S.SMPCError(st, "grid preparation")
        noise = torch.from_numpy(np.ascontiguousarray(inp.noise)).to(dev)
        U = [torch.zeros((H, 7), device=dev), torch.zeros((H, 7), device=dev)]
        planner = S.Planner(inp.robot, device=0)
        sigma = [0.5] * 7

        def step(i, f16, sample):
            planner.plan_step(q0=inp.q0, qd0=inp.qd0, T_goal=inp.T_goal,
                              grid=g16 if f16 else g32, origin=inp.origin, voxel=inp.voxel,
                              noise=None if sample else noise, U_in=U[i % 2],
                              U_out=U[(i + 1) % 2], dt=inp.dt, lam=inp.lam,
                              weights=inp.weights, stream=stream, seed=1000 + i, sigma=sigma,
                              grid_dtype=S.GRID_F16 if f16 else S.GRID_F32, K=K, H=H,
                              coarse=c16 if f16 else c32)

        row = {}
        for label, f16, sample in (("f32 grid, noise buffer", False, False),
                                   ("f16 grid, noise buffer", True, False),
                                   ("f32 grid, device sampling", False, True),
                                   ("f16 grid, device sampling", True, True)):
            for i in range(args.warmup):
                step(i, f16, sample)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record()
            for i in range(args.steps):
                step(i, f16, sample)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / args.steps
            row[label] = {"ms_per_step": round(ms, 6),
                          "rollout_steps_per_s": round(K * H / (ms * 1e-3), 1)}
        base = row["f32 grid, noise buffer"]["ms_per_step"]
        for v in row.values():
            v["speedup_vs_f32_buffer"] = round(base / v["ms_per_step"], 4)
        out[name] = row
        planner.close()
    return {
        "metric": "plan-step time of the float16-grid and device-sampling variants",
        "unit": "ms per step", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": False, "data": "synthetic", "dtype": "f32 arithmetic, f16 grid",
        "variants": out,
        "errors": "stated by tests/test_variants_gpu.py against the FP64 oracle",
    }


def paper_shaped_bench(args) -> dict:
    """Periods at the paper's own setting: M = 512 samples, 150 x 150 x 25 map at 0.02 m,
    50 Hz (H = 40; the paper does not state it).  One period = coarse bounds of the map
    (cells within the arm's reach) + a receding-horizon plan step, warm-started, back to
    back; then single periods with synchronisation for the latency."""
    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import workload as W

    inp = W.paper_shaped()
    K, H = inp.noise.shape[0], inp.noise.shape[1]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    grid = torch.from_numpy(np.ascontiguousarray(inp.grid)).to(dev)
    nz, ny, nx = inp.grid.shape
    coarse = torch.empty(S.smpc_grid_coarse_cells(nx, ny, nz), device=dev)
    rng = np.random.default_rng(16)
    noise = [torch.from_numpy(W.sample_noise(rng, K, H)).to(dev) for _ in range(8)]
    U = [torch.zeros((H, 7), device=dev), torch.zeros((H, 7), device=dev)]
    X = [torch.from_numpy(np.concatenate([inp.q0, inp.qd0]).astype(np.float32)).to(dev)]
    X.append(torch.zeros_like(X[0]))
    u0 = torch.zeros((7,), device=dev)
    planner = S.Planner(inp.robot, device=0)
    reach_c, reach_r = planner.robot_reach()

    def period(i):
        st = S.smpc_grid_coarse_min_ball(grid, S.GRID_F32, inp.origin, inp.voxel, reach_c,
                                         reach_r, coarse.data_ptr(), stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, "smpc_grid_coarse_min_ball")
        planner.plan_step(q0=inp.q0, qd0=inp.qd0, T_goal=inp.T_goal, grid=grid,
                          origin=inp.origin, voxel=inp.voxel, noise=noise[i % 8],
                          U_in=U[i % 2], U_out=U[(i + 1) % 2], dt=inp.dt, lam=inp.lam,
                          weights=inp.weights, stream=stream, coarse=coarse, receding=True,
                          u0_out=u0, state_in=X[i % 2], state_out=X[(i + 1) % 2])

    for i in range(args.warmup):
        period(i)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for i in range(args.steps):
        period(i)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    lat = []
    for i in range(min(args.steps, 100)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        period(i)
        b.record()
        b.synchronize()
        lat.append(a.elapsed_time(b))
    planner.close()
    return {
        "metric": "period time at the paper's sample count and map (bounds + plan step)",
        "ms_per_step": round(ms, 6), "rollout_steps_per_s": round(K * H / (ms * 1e-3), 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 5),
                       "p99": round(float(np.percentile(lat, 99)), 5)},
        "config": {"workload": f"M=K={K}, H={H}, dt=0.02 s, map {nx}x{ny}x{nz} at 0.02 m "
                               "(3 x 3 x 0.5 m) from 10 boxes and 10 spheres, static map",
                   "K": int(K), "H": int(H), "grid": [int(nx), int(ny), int(nz)]},
        "paper_context": "5.322 ms per replanning iteration at M=512 on an RTX 3090 (the "
                         "paper's figure; its horizon and per-stage split are not stated)",
    }


def cpu_baseline(sc, grids_np, noises_np, K, H, periods):
    """The FP64 oracle's closed loop on the host: ``periods`` control periods of the
    same scene (plan step, execution of u*_0, shift), one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import smpc_oracle as O
    rob = sc.robot.rounded_f32()
    q, qd = sc.q0.astype(np.float64), sc.qd0.astype(np.float64)
    U = np.zeros((H, 7))
    t_sc = sc.t
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for i in range(periods):
            ref = O.plan_step(rob, q, qd, sc.target(), grids_np[i], sc.origin,
                              np.float32(sc.VOXEL), noises_np[i], U, np.float32(sc.DT), 1.0,
                              sc.weights)
            q, qd = O.execute_first_control(q, qd, ref["U_star"], np.float32(sc.DT))
            U = O.shift_nominal(ref["U_star"])
            sc.t += sc.DT
        dt = time.perf_counter() - t0
    sc.t = t_sc
    return {"value": round(periods * K * H / dt, 1), "unit": "rollout-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{periods} closed-loop periods (K={K}, H={H}) of the same scene on its "
                      f"first grids, float64 numpy, {dt:.2f} s on one host thread"}


def build_grid_pool(S, sc, n_grids, dev, stream):
    """Signed distance grids of consecutive control periods of the scene: occupancy on
    the host, the exact field on the device (smpc_edt), resident in HBM."""
    import torch
    n = sc.N
    need = S.smpc_edt_workspace_bytes(n, n, n)
    work = torch.empty((need + 3) // 4, dtype=torch.int32, device=dev)
    occs, grids = [], []
    for _ in range(n_grids):
        occ = torch.from_numpy(sc.occupancy().astype(np.uint8)).to(dev)
        phi = torch.empty((n, n, n), device=dev)
        st = S.smpc_edt(occ.data_ptr(), n, n, n, sc.VOXEL, phi.data_ptr(), None, work.data_ptr(),
                        need, stream)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, "smpc_edt")
        occs.append(occ)
        grids.append(phi)
        sc.advance()
    torch.cuda.synchronize()
    del occs, work
    return grids


def secondary_results(args) -> dict:
    """The serving, variant, distance-field and occupancy-update benchmarks, run after the
    headline's timed work with their own (shorter) step counts and no CPU baselines, and
    summarised, so that the default run's record carries them.  A failure in one of
    them is reported in its entry and does not affect the headline figures."""
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup, sub.no_cpu_baseline = 100, 10, True
    res = {}

    def run(name, fn, pick):
        try:
            res[name] = pick(fn(sub))
        except Exception as e:  # noqa: BLE001 -- reported, never hides the headline
            res[name] = {"error": f"{type(e).__name__}: {e}"}

    run("serving", serving_bench, lambda r: {
        "workload": r["config"]["workload"], "p50_ms": r["realtime"]["p50_ms"],
        "p99_ms": r["realtime"]["p99_ms"],
        "saturated_rollout_steps_per_s": r["saturated"]["rollout_steps_per_s"],
        "sequential_rollout_steps_per_s": r["sequential_plain"]["rollout_steps_per_s"]})
    run("variants", variants_bench, lambda r: {
        w: {k: v["speedup_vs_f32_buffer"] for k, v in row.items()} | {
            "f32_ms_per_step": row["f32 grid, noise buffer"]["ms_per_step"]}
        for w, row in r["variants"].items()})
    run("edt", edt_bench, lambda r: {
        "workload": r["config"]["workload"], "ms_per_step": r["ms_per_step"],
        "voxels_per_s": r["value"], "pipeline_ms_per_step": r["pipeline_ms_per_step"]})
    run("paper_shaped", paper_shaped_bench, lambda r: {
        "workload": r["config"]["workload"], "ms_per_step": r["ms_per_step"],
        "latency_p50_ms": r["latency_ms"]["p50"], "latency_p99_ms": r["latency_ms"]["p99"],
        "paper_ms_per_iteration": 5.322})
    run("ogm", ogm_bench, lambda r: {
        "workload": r["config"]["workload"], "ms_per_step": r["ms_per_step"],
        "voxels_per_s": r["value"], "pipeline_ms_per_step": r["pipeline_ms_per_step"]})
    res["what"] = ("bench.py --serving / --variants / --paper-shaped / --edt / --ogm with 100 "
                   "timed steps "
                   "(serving: its own request stream); their full records come from those "
                   "flags")
    return res


def main():
    args = parse_args()
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the plan step is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    for flag, fn in (("serving", serving_bench), ("edt", edt_bench), ("ogm", ogm_bench),
                     ("variants", variants_bench), ("paper_shaped", paper_shaped_bench)):
        if getattr(args, flag):
            print(json.dumps(fn(args)), flush=True)
            return
    import ctypes

    import torch

    from paper_2512_22575_amd import smpc as S
    from synth import workload as W

    K, H, n = args.K, args.H, args.n
    sc = W.ReactiveScenario(seed=3, K=K, H=H, n=n)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    lib = S.load_library()
    t_setup = time.perf_counter()
    n_grids = max(1, args.grids)
    grids = build_grid_pool(S, sc, n_grids, dev, stream)
    sc.t = 0.0
    n_pool = max(1, args.pool)
    noise_np = [sc.noise() for _ in range(n_pool)]
    noise = [torch.from_numpy(x).to(dev) for x in noise_np]
    t_setup = time.perf_counter() - t_setup
    use_coarse = not args.no_coarse
    # Two bounds tables: period i reads table i mod 2 while its launches build the next
    # period's bounds into the other one.
    tables = [torch.empty(S.smpc_grid_coarse_cells(n, n, n), device=dev) for _ in range(2)]
    coarse = tables[0] if use_coarse else None
    costs = torch.empty((K,), device=dev)
    stats = torch.empty((4,), device=dev)
    planner = S.Planner(sc.robot, device=0)
    ctx = planner._ctx
    # The bounds are built for the cells the arm's spheres can reach (smpc_robot_reach);
    # the other cells get -inf, so plan steps are exact whatever the arm does.
    reach_c, reach_r = planner.robot_reach()
    reach_cp = (ctypes.c_float * 3)(*[float(x) for x in reach_c])
    # Closed loop on the device: two nominal sequences and two joint states alternate.
    U = [torch.zeros((H, 7), device=dev), torch.zeros((H, 7), device=dev)]
    X0 = torch.from_numpy(np.concatenate([sc.q0, sc.qd0]).astype(np.float32)).to(dev)
    X = [X0.clone(), torch.zeros_like(X0)]
    u0 = torch.zeros((7,), device=dev)
    u0_host = torch.zeros((7,), pin_memory=True)

    total = args.warmup + args.steps + 2 * args.latency_steps + 2 * args.profile_steps
    plans, grid_structs = [], []
    for i in range(total):
        g = grids[i % n_grids]
        plans.append(S.plan_args(sc.q0, sc.qd0, sc.target(), g, sc.origin, sc.VOXEL,
                                 noise[i % n_pool], U[i % 2], U[(i + 1) % 2], K, H, sc.DT, 1.0,
                                 sc.weights, costs_out=costs, stats_out=stats,
                                 coarse=tables[i % 2] if use_coarse else None,
                                 receding=True, u0_out=u0, state_in=X[i % 2],
                                 state_out=X[(i + 1) % 2]))
        sc.t += sc.DT
    for g in grids:
        grid_structs.append(S.smpc_grid(ctypes.c_void_p(g.data_ptr()), n, n, n, S.GRID_F32,
                                        (ctypes.c_float * 3)(*[float(x) for x in sc.origin]),
                                        float(sc.VOXEL), None))
    plan_ptrs = [ctypes.byref(a) for a in plans]
    grid_ptrs = [ctypes.byref(g) for g in grid_structs]
    table_ptrs = [ctypes.c_void_p(t.data_ptr()) for t in tables]
    sp = ctypes.c_void_p(stream)

    fuse = use_coarse and not args.no_fuse_bounds

    def bounds(i):
        st = lib.smpc_grid_coarse_min_ball(grid_ptrs[i % n_grids], reach_cp, reach_r,
                                           table_ptrs[i % 2], sp)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, "smpc_grid_coarse_min_ball")

    def serial_period(i):
        """One control period on a fresh grid: bounds of the new grid, then the plan step
        (which executes u*_0 and shifts the nominal sequence on the device)."""
        if use_coarse:
            bounds(i)
        st = lib.smpc_plan_step(ctx, plan_ptrs[i], sp)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_last_error(ctx))

    def period(i):
        """One control period; fused, the plan step's rollout launch also builds the bounds
        of the next period's grid, into the table this step does not read."""
        if not fuse:
            serial_period(i)
            return
        st = lib.smpc_plan_step_then_bounds(ctx, plan_ptrs[i], grid_ptrs[(i + 1) % n_grids],
                                            reach_cp, reach_r, table_ptrs[(i + 1) % 2], sp)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_last_error(ctx))

    if fuse:
        bounds(0)  # the first period's bounds; each period then builds the next one's
    # Warm-up (untimed).
    for i in range(args.warmup):
        period(i)
    torch.cuda.synchronize()

    # Throughput: periods back to back on one stream.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    base = args.warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for i in range(base, base + args.steps):
        period(i)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = K * H / (ms_per_step * 1e-3)
    s = stats.cpu().numpy()
    if s[3] != 0.0:
        raise RuntimeError(f"plan step reported status {s[3]}")
    x_end = X[(base + args.steps) % 2].cpu().numpy()
    if not np.all(np.isfinite(x_end)):
        raise RuntimeError("closed-loop state is not finite")

    # Latency: each period alone, bounds then plan step (the map of a period is not
    # known a period ahead), with u*_0 written by the merge kernel straight into pinned
    # host memory (device time between events; host time from the first call to u*_0 on
    # the host).
    base += args.steps
    lat_dev, lat_host = [], []
    for i in range(base, base + args.latency_steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        plans[i].u0_out = ctypes.c_void_p(u0_host.data_ptr())  # the merge writes it there
        h0 = time.perf_counter()
        a.record()
        serial_period(i)
        b.record()
        b.synchronize()
        lat_host.append((time.perf_counter() - h0) * 1e3)
        lat_dev.append(a.elapsed_time(b))
    lat_dev = np.array(lat_dev)
    lat_host = np.array(lat_host)

    # The plan step alone, the bounds of its grid built beforehand (a map that arrived
    # before the period started): the same measurement around smpc_plan_step only.
    base += args.latency_steps
    ps_dev, ps_host = [], []
    for i in range(base, base + args.latency_steps):
        if use_coarse:
            bounds(i)
            torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        h0 = time.perf_counter()
        plans[i].u0_out = ctypes.c_void_p(u0_host.data_ptr())
        a.record()
        st = lib.smpc_plan_step(ctx, plan_ptrs[i], sp)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_last_error(ctx))
        b.record()
        b.synchronize()
        ps_host.append((time.perf_counter() - h0) * 1e3)
        ps_dev.append(a.elapsed_time(b))
    ps_dev = np.array(ps_dev)
    ps_host = np.array(ps_host)

    # Per-kernel durations from events recorded by the library on the launch stream;
    # the bounds build between events of its own.
    base += args.latency_steps
    planner.profile_enable(args.profile_steps)
    cb = []
    for i in range(base, base + args.profile_steps):
        if use_coarse:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            st = lib.smpc_grid_coarse_min_ball(grid_ptrs[i % n_grids], reach_cp, reach_r,
                                               table_ptrs[i % 2], sp)
            e1.record()
            cb.append((e0, e1))
        st = lib.smpc_plan_step(ctx, plan_ptrs[i], sp)
        if st != S.SMPC_OK:
            raise S.SMPCError(st, S.smpc_last_error(ctx))
    torch.cuda.synchronize()
    k1_ms, k2_ms = planner.profile_read(args.profile_steps)
    k1f_ms = k2f_ms = None
    if fuse:  # the rollout launch that also builds the next period's bounds
        base += args.profile_steps
        bounds(base)
        planner.profile_enable(args.profile_steps)
        for i in range(base, base + args.profile_steps):
            period(i)
        torch.cuda.synchronize()
        k1f_ms, k2f_ms = planner.profile_read(args.profile_steps)
    planner.profile_enable(0)
    coarse_ms = float(np.mean([a.elapsed_time(b) for a, b in cb])) if cb else 0.0
    k1_avg = float(np.mean(k1_ms))
    flop = FLOP_PER_ROLLOUT_STEP * K * H
    achieved = flop / (k1_avg * 1e-3) / 1e12
    gather_gbs = GATHER_BYTES_PER_ROLLOUT_STEP * K * H / (k1_avg * 1e-3) / 1e9

    # The same plan steps on one static grid whose bounds are built once (cache-warm).
    static = None
    if args.static_steps > 0:
        g0 = grids[0]
        c0 = None
        if use_coarse:
            c0 = torch.empty_like(coarse)
            st = lib.smpc_grid_coarse_min_ball(grid_ptrs[0], reach_cp, reach_r,
                                               ctypes.c_void_p(c0.data_ptr()), sp)
            if st != S.SMPC_OK:
                raise S.SMPCError(st, "smpc_grid_coarse_min_ball")
        splans = [S.plan_args(sc.q0, sc.qd0, plans[i].T_goal, g0, sc.origin, sc.VOXEL,
                              noise[i % n_pool], U[i % 2], U[(i + 1) % 2], K, H, sc.DT, 1.0,
                              sc.weights, costs_out=costs, stats_out=stats, coarse=c0,
                              receding=True, u0_out=u0, state_in=X[i % 2],
                              state_out=X[(i + 1) % 2])
                  for i in range(args.warmup + args.static_steps)]
        for i in range(args.warmup):
            lib.smpc_plan_step(ctx, ctypes.byref(splans[i]), sp)
        torch.cuda.synchronize()
        ev0.record()
        for i in range(args.warmup, args.warmup + args.static_steps):
            st = lib.smpc_plan_step(ctx, ctypes.byref(splans[i]), sp)
            if st != S.SMPC_OK:
                raise S.SMPCError(st, S.smpc_last_error(ctx))
        ev1.record()
        torch.cuda.synchronize()
        sms = ev0.elapsed_time(ev1) / args.static_steps
        static = {"ms_per_step": round(sms, 6), "rollout_steps_per_s": round(K * H / (sms * 1e-3), 1),
                  "steps": args.static_steps,
                  "what": "plan steps (receding, state on the device) on one grid whose bounds "
                          "are built once, outside the timed region"}

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"reactive replanning closed loop, fresh grid per period: K={K} "
                        f"rollouts x H={H} steps, dt=0.02 s, {n}^3 f32 ESDF at 0.01 m from 40 "
                        f"primitives drifting 0.2 m/s, target on a 0.3 m circle, 7-DoF arm, "
                        f"28 spheres, {sc.robot.n_pairs} self pairs",
            "K": K, "H": H, "grid": [n] * 3, "voxel_m": 0.01, "lambda": 1.0,
            "period": ("plan step that executes u*_0 and shifts the nominal sequence on "
                       "the device, its rollout launch also building the coarse bounds "
                       "(cells within the arm's reach) of the next period's grid into the "
                       "other of two tables" if fuse else
                       "coarse bounds of the period's grid (cells within the arm's reach) + "
                       "plan step that executes u*_0 and shifts the nominal sequence on the "
                       "device" if use_coarse else
                       "plan step that executes u*_0 and shifts the nominal sequence on the "
                       "device (no coarse bounds)"),
            "grids": f"{n_grids} distinct consecutive-period grids resident in HBM "
                     f"({n_grids * n ** 3 * 4 / 2 ** 20:.0f} MiB), cycled",
            "noise": f"{n_pool} pre-sampled device buffers (float32), cycled",
            "setup_s": round(t_setup, 1),
        },
        "latency_ms": {
            "p50": round(float(np.percentile(lat_dev, 50)), 5),
            "p99": round(float(np.percentile(lat_dev, 99)), 5),
            "mean": round(float(np.mean(lat_dev)), 5),
            "host_p50": round(float(np.percentile(lat_host, 50)), 5),
            "host_p99": round(float(np.percentile(lat_host, 99)), 5),
            "steps": int(args.latency_steps),
            "what": "one period alone, coarse bounds of its grid then the plan step, on "
                    "the device (events), and on the host until u*_0 is in host memory "
                    "(written there by the merge kernel: pinned host memory as u0_out)",
            "plan_step": {
                "p50": round(float(np.percentile(ps_dev, 50)), 5),
                "p99": round(float(np.percentile(ps_dev, 99)), 5),
                "host_p50": round(float(np.percentile(ps_host, 50)), 5),
                "host_p99": round(float(np.percentile(ps_host, 99)), 5),
                "what": "the plan step alone (smpc_plan_step, u*_0 to host memory), the "
                        "bounds of its grid built before the call",
            },
        },
        "host_ms_per_step": round(wall * 1e3 / args.steps, 5),
        "kernels_ms": {"coarse_bounds": round(coarse_ms, 6),
                       "rollout_cost": round(k1_avg, 6),
                       "merge": round(float(np.mean(k2_ms)), 6),
                       "fused_period": (
                           {"rollout_with_next_bounds": round(float(np.mean(k1f_ms)), 6),
                            "merge": round(float(np.mean(k2f_ms)), 6)}
                           if k1f_ms is not None else None)},
        "roofline": {
            "bound": "alu",
            "kernel": "rollout_cost_kernel",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": rollout_traffic_bytes(),
            "flop_per_launch": flop,
            "gather_GBps": round(gather_gbs, 1),
        },
        "static_grid": static,
        "paper_context": "5.322 ms per replanning iteration at M=512 on an RTX 3090 "
                         "(H not stated); not the same workload",
    }
    l2 = rollout_l2(k1_avg)
    if l2 is not None:
        out["roofline"]["l2"] = l2
    if not args.no_cpu_baseline:
        sc2 = W.ReactiveScenario(seed=3, K=K, H=H, n=n)
        periods = 2
        grids_np = [g.cpu().numpy() for g in grids[:periods]]
        out["cpu_baseline"] = cpu_baseline(sc2, grids_np, noise_np, K, H, periods)
    planner.close()
    if not args.no_secondary:
        out["secondary"] = secondary_results(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
