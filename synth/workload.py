"""Seeded plan-step workloads.

Every input of a plan step is produced here from a seed: robot, start state,
target pose, distance grid, nominal sequence and the sampled disturbances.  All
floating-point inputs are rounded to float32 once, here, so the GPU path and the
FP64 oracle consume identical numbers.

Recipes (the paper's benchmark scenes are not available; these stand in for them):

* ``tiny``      K=64,   H=16, dt=0.05, grid 32^3 at 0.05 m from 5 boxes.
* ``mid``       K=1024, H=32, dt=0.02, grid 64^3 at 0.03 m from 10 boxes + 10 spheres.
* ``reactive``  K=4096, H=40, dt=0.02, grid 200^3 at 0.01 m from 20 boxes + 20
  spheres drifting at 0.2 m/s; the target moves on a 0.3 m circle at 0.5 rad/s.

Common to all: q0 ~ U(position limits), qd0 = 0, nominal sequence 0, noise
eps = sigma * N(0, 1) with sigma = 0.5 rad/s^2 per joint, temperature 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import robot as robot_mod
from . import scene as scene_mod

F32 = np.float32

# Cost weights.  The paper prints none; these defaults follow the workload
# description (translation weight 10, rotation weight 2, 0.03 m activation
# distance) and otherwise pick moderate penalties.
DEFAULT_WEIGHTS = dict(
    w_pose_t=10.0, w_pose_r=2.0,      # Q_k = diag(w_t I3, w_r I3)
    w_term_t=10.0, w_term_r=2.0,      # Q_H
    w_env=100.0, d_act=0.03,          # environment hinge
    w_self=100.0,                     # self-collision hinge
    w_q=10.0, w_qd=10.0, w_qdd=10.0,  # joint-limit penalties
    limit_margin_frac=0.05,           # tightening margin as a fraction of the range
    w_smooth=0.01,                    # acceleration smoothness
    w_ns=0.0,                         # null-space regularisation
)

WEIGHT_FIELDS = tuple(DEFAULT_WEIGHTS.keys())


@dataclasses.dataclass
class PlanInputs:
    """One plan step's inputs, float32 where the GPU consumes float32."""

    robot: robot_mod.Robot
    q0: np.ndarray          # (7,) f32
    qd0: np.ndarray         # (7,) f32
    T_goal: np.ndarray      # (4, 4) f32, row-major SE(3)
    grid: np.ndarray        # (nz, ny, nx) f32 signed distance, metres
    origin: np.ndarray      # (3,) f32, corner of voxel (0,0,0)
    voxel: float            # f32-representable
    noise: np.ndarray       # (K, H, 7) f32
    U_bar: np.ndarray       # (H, 7) f32
    dt: float
    lam: float
    weights: dict

    @property
    def K(self) -> int:
        return int(self.noise.shape[0])

    @property
    def H(self) -> int:
        return int(self.noise.shape[1])


def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=F32)


def f32s(x: float) -> float:
    """Round a Python float to the nearest float32 value."""
    return float(np.float32(x))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation matrix from a random unit quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def pose_matrix(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def random_target_pose(rng: np.random.Generator) -> np.ndarray:
    """Target pose: uniform random orientation, position in the arm's front workspace."""
    t = rng.uniform([0.25, -0.45, 0.15], [0.65, 0.45, 0.85])
    return pose_matrix(random_rotation(rng), t)


def sample_noise(rng: np.random.Generator, K: int, H: int, sigma=0.5) -> np.ndarray:
    """eps ~ N(0, sigma^2) iid per joint, drawn in float64 and rounded to float32."""
    sigma = np.broadcast_to(np.asarray(sigma, np.float64), (robot_mod.N_DOF,))
    return f32(rng.standard_normal((K, H, robot_mod.N_DOF)) * sigma)


def make_scene_grid(rng: np.random.Generator, n: int, voxel: float, n_boxes: int,
                    n_spheres: int, speed: float = 0.0):
    origin = scene_mod.grid_origin(n, voxel)
    side = n * voxel
    lo = origin + 0.05 * side
    hi = origin + 0.95 * side
    prims = scene_mod.random_primitives(rng, lo, hi, n_boxes, n_spheres, speed=speed)
    occ = scene_mod.occupancy(prims, (n, n, n), origin, voxel)
    grid = scene_mod.signed_distance_grid(occ, voxel)
    return grid, f32(origin), prims, (lo, hi)


def make_inputs(seed: int, K: int, H: int, dt: float, n: int, voxel: float, n_boxes: int,
                n_spheres: int, lam: float = 1.0, sigma=0.5, weights: dict | None = None,
                speed: float = 0.0, robot_seed: int | None = None) -> PlanInputs:
    rng = np.random.default_rng(seed)
    rob = robot_mod.make_robot(seed if robot_seed is None else robot_seed)
    grid, origin, _, _ = make_scene_grid(rng, n, voxel, n_boxes, n_spheres, speed)
    q0 = f32(robot_mod.random_joint_config(rng, rob))
    qd0 = f32(np.zeros(robot_mod.N_DOF))
    T_goal = f32(random_target_pose(rng))
    noise = sample_noise(rng, K, H, sigma)
    w = dict(DEFAULT_WEIGHTS if weights is None else weights)
    return PlanInputs(robot=rob, q0=q0, qd0=qd0, T_goal=T_goal, grid=grid, origin=origin,
                      voxel=f32s(voxel), noise=noise, U_bar=f32(np.zeros((H, robot_mod.N_DOF))),
                      dt=f32s(dt), lam=f32s(lam), weights={k: f32s(v) for k, v in w.items()})


def tiny(seed: int = 1) -> PlanInputs:
    """K=64, H=16, dt=0.05, 32^3 grid at 0.05 m from 5 boxes, lambda=1."""
    return make_inputs(seed, K=64, H=16, dt=0.05, n=32, voxel=0.05, n_boxes=5, n_spheres=0)


def mid(seed: int = 2) -> PlanInputs:
    """K=1024, H=32, dt=0.02, 64^3 grid at 0.03 m from 10 boxes and 10 spheres."""
    return make_inputs(seed, K=1024, H=32, dt=0.02, n=64, voxel=0.03, n_boxes=10, n_spheres=10)


def paper_shaped(seed: int = 6, H: int = 40) -> PlanInputs:
    """The paper's own setting as far as it states it: M = 512 samples at 50 Hz (dt =
    0.02 s) on its integrated map of 0.02 m voxels over 3 x 3 x 0.5 m (150 x 150 x 25,
    x and y centred on the base, floor at z = 0), here from 10 boxes and 10 spheres in
    that slab.  The horizon is not stated; H = 40 as in the reactive workload.  Links
    above the slab read its top layer (edge extension)."""
    rng = np.random.default_rng(seed)
    rob = robot_mod.make_robot(seed)
    n, voxel, K = (150, 150, 25), 0.02, 512
    side = np.array(n, np.float64) * voxel
    origin = np.array([-0.5 * side[0], -0.5 * side[1], 0.0])
    prims = scene_mod.random_primitives(rng, origin + 0.05 * side, origin + 0.95 * side, 10, 10)
    grid = scene_mod.signed_distance_grid(scene_mod.occupancy(prims, n, origin, voxel), voxel)
    q0 = f32(robot_mod.random_joint_config(rng, rob))
    T_goal = f32(random_target_pose(rng))
    noise = sample_noise(rng, K, H)
    return PlanInputs(robot=rob, q0=q0, qd0=f32(np.zeros(robot_mod.N_DOF)), T_goal=T_goal,
                      grid=grid, origin=f32(origin), voxel=f32s(voxel), noise=noise,
                      U_bar=f32(np.zeros((H, robot_mod.N_DOF))), dt=f32s(0.02), lam=f32s(1.0),
                      weights={k: f32s(v) for k, v in DEFAULT_WEIGHTS.items()})


class ReactiveScenario:
    """K=4096, H=40, dt=0.02 closed-loop scene: drifting primitives, circling target.

    The grid is 200^3 at 0.01 m (a 2 m cube) from 20 boxes and 20 spheres moving
    at 0.2 m/s and reflecting off the cube walls; it is regenerated on the host
    at every step.  The target position follows c + 0.3 (cos 0.5t, sin 0.5t, 0)
    with a fixed orientation.
    """

    K, H, DT, N, VOXEL = 4096, 40, 0.02, 200, 0.01

    def __init__(self, seed: int = 3, K: int | None = None, H: int | None = None,
                 n: int | None = None, voxel: float | None = None):
        self.K = K or self.K
        self.H = H or self.H
        self.N = n or self.N
        self.VOXEL = voxel or self.VOXEL
        self.rng = np.random.default_rng(seed)
        self.robot = robot_mod.make_robot(seed)
        self.origin = f32(scene_mod.grid_origin(self.N, self.VOXEL))
        side = self.N * self.VOXEL
        self.lo = self.origin + 0.05 * side
        self.hi = self.origin + 0.95 * side
        self.prims = scene_mod.random_primitives(self.rng, self.lo, self.hi, 20, 20, speed=0.2)
        self.q0 = f32(robot_mod.random_joint_config(self.rng, self.robot, shrink=0.1))
        self.qd0 = f32(np.zeros(robot_mod.N_DOF))
        base = random_target_pose(self.rng)
        self.R_goal = base[:3, :3]
        self.centre = base[:3, 3] - np.array([0.3, 0.0, 0.0])
        self.t = 0.0
        self.weights = {k: f32s(v) for k, v in DEFAULT_WEIGHTS.items()}

    def occupancy(self) -> np.ndarray:
        return scene_mod.occupancy(self.prims, (self.N,) * 3, self.origin, self.VOXEL)

    def grid(self) -> np.ndarray:
        return scene_mod.signed_distance_grid(self.occupancy(), self.VOXEL)

    def target(self) -> np.ndarray:
        p = self.centre + 0.3 * np.array([math.cos(0.5 * self.t), math.sin(0.5 * self.t), 0.0])
        return f32(pose_matrix(self.R_goal, p))

    def noise(self) -> np.ndarray:
        return sample_noise(self.rng, self.K, self.H)

    def advance(self) -> None:
        """Advance world time by one control period (primitives drift, target moves)."""
        self.prims = scene_mod.advance_primitives(self.prims, self.DT, self.lo, self.hi)
        self.t += self.DT

    def inputs(self, U_bar: np.ndarray | None = None, grid: np.ndarray | None = None) -> PlanInputs:
        H = self.H
        return PlanInputs(robot=self.robot, q0=self.q0, qd0=self.qd0, T_goal=self.target(),
                          grid=self.grid() if grid is None else grid, origin=self.origin,
                          voxel=f32s(self.VOXEL), noise=self.noise(),
                          U_bar=f32(np.zeros((H, 7))) if U_bar is None else f32(U_bar),
                          dt=f32s(self.DT), lam=1.0, weights=dict(self.weights))


def shift_warm_start(U_star: np.ndarray) -> np.ndarray:
    """Receding-horizon warm start: drop u_0*, append a zero control."""
    U = np.zeros_like(U_star)
    U[:-1] = U_star[1:]
    return U
