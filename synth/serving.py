"""Seeded serving workload: many independent controllers and a Poisson request stream.

Recipe (the paper runs one controller at 50 Hz; this scales that to a
multi-controller service):

* n_controllers controllers, each with K in {256, 1024, 2048, 4096}, H in {16, 32, 64},
  its own n^3 grid with n in [64, 160], voxel in [0.01, 0.03] m, built from 10..60
  primitives (half boxes, half spheres), dt = 0.02 s, lambda = 1, sigma = 0.5;
* n_requests requests with exponential inter-arrival times (mean 1/rate); each
  picks a controller uniformly, carries that controller's current joint state and
  a target pose, and a per-request sampling seed.

Grids are generated on the host (exact EDT), which dominates the set-up time.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import robot as robot_mod
from . import workload as W


@dataclasses.dataclass
class Controller:
    K: int
    H: int
    n: int
    voxel: float
    grid: np.ndarray      # (n, n, n) float32
    origin: np.ndarray    # (3,) float32
    dt: float
    lam: float
    sigma: np.ndarray     # (7,) float32
    weights: dict
    q0: np.ndarray        # initial joint state
    T_goal: np.ndarray


@dataclasses.dataclass
class Request:
    t_arrival: float      # seconds from the start of the trace
    controller: int
    q0: np.ndarray
    qd0: np.ndarray
    T_goal: np.ndarray
    seed: int


def make_controllers(seed: int, n_controllers: int, n_range=(64, 160), voxel_range=(0.01, 0.03),
                     prim_range=(10, 60), Ks=(256, 1024, 2048, 4096), Hs=(16, 32, 64)):
    rng = np.random.default_rng(seed)
    rob = robot_mod.make_robot(seed)
    out = []
    for _ in range(n_controllers):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        voxel = W.f32s(rng.uniform(*voxel_range))
        n_prims = int(rng.integers(prim_range[0], prim_range[1] + 1))
        grid, origin, _, _ = W.make_scene_grid(rng, n, voxel, n_prims // 2, n_prims - n_prims // 2)
        out.append(Controller(
            K=int(rng.choice(Ks)), H=int(rng.choice(Hs)), n=n, voxel=voxel, grid=grid,
            origin=origin, dt=W.f32s(0.02), lam=1.0, sigma=W.f32(np.full(7, 0.5)),
            weights={k: W.f32s(v) for k, v in W.DEFAULT_WEIGHTS.items()},
            q0=W.f32(robot_mod.random_joint_config(rng, rob, shrink=0.1)),
            T_goal=W.f32(W.random_target_pose(rng))))
    return rob, out


def make_trace(seed: int, controllers: list[Controller], n_requests: int, rate_hz: float):
    rng = np.random.default_rng(seed + 1)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    reqs = []
    for i in range(n_requests):
        c = int(rng.integers(len(controllers)))
        ctl = controllers[c]
        reqs.append(Request(t_arrival=float(t[i]), controller=c, q0=ctl.q0.copy(),
                            qd0=W.f32(np.zeros(7)), T_goal=ctl.T_goal.copy(),
                            seed=int(rng.integers(1 << 62))))
    return reqs
