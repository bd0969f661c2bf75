"""ctypes binding of libsmpc (include/smpc.h): argument marshalling only.

The functions ``smpc_create``, ``smpc_set_robot``, ``smpc_plan_step``,
``smpc_destroy``, ``smpc_status_string``, ``smpc_last_error`` and
``smpc_version`` mirror the C entry points one to one.  :class:`Planner` is a
convenience wrapper that takes torch tensors (device memory and streams come
from PyTorch); every step of the plan step itself runs in the HIP library.

The library is loaded from this package directory.  If it is missing, loading
raises immediately: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import (POINTER, c_char_p, c_double, c_float, c_int32, c_uint64, c_void_p)

import numpy as np

NDOF = 7
MAX_H = 64
SPHERES_PER_LINK = 4
MAX_SPHERES = 28
MAX_PAIRS = 378
GRID_F32, GRID_F16 = 0, 1

SMPC_OK = 0
SMPC_E_INVALID_ARG = -1
SMPC_E_OOM = -2
SMPC_E_DEVICE = -3
SMPC_E_NUMERIC = -4
SMPC_E_UNSUPPORTED = -5

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsmpc.so")


class smpc_robot_desc(ctypes.Structure):
    _fields_ = [
        ("n_dof", c_int32),
        ("a", c_double * NDOF), ("d", c_double * NDOF), ("alpha", c_double * NDOF),
        ("q_min", c_double * NDOF), ("q_max", c_double * NDOF),
        ("qd_min", c_double * NDOF), ("qd_max", c_double * NDOF),
        ("qdd_min", c_double * NDOF), ("qdd_max", c_double * NDOF),
        ("q_ref", c_double * NDOF),
        ("n_spheres", c_int32),
        ("sphere_link", c_int32 * MAX_SPHERES),
        ("sphere_center", (c_double * 3) * MAX_SPHERES),
        ("sphere_radius", c_double * MAX_SPHERES),
        ("n_pairs", c_int32),
        ("pairs", (c_int32 * 2) * MAX_PAIRS),
    ]


class smpc_cost_weights(ctypes.Structure):
    _fields_ = [(name, c_float) for name in (
        "w_pose_t", "w_pose_r", "w_term_t", "w_term_r", "w_env", "d_act", "w_self",
        "w_q", "w_qd", "w_qdd", "limit_margin_frac", "w_smooth", "w_ns")]


class smpc_grid(ctypes.Structure):
    _fields_ = [
        ("data", c_void_p),
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("dtype", c_int32),
        ("origin", c_float * 3),
        ("voxel", c_float),
        ("coarse", c_void_p),
    ]


class smpc_plan_args(ctypes.Structure):
    _fields_ = [
        ("q0", c_float * NDOF), ("qd0", c_float * NDOF),
        ("T_goal", c_float * 16),
        ("esdf", smpc_grid),
        ("noise", c_void_p),
        ("seed", c_uint64),
        ("sigma", c_float * NDOF),
        ("K", c_int32), ("H", c_int32),
        ("dt", c_float), ("lambda_", c_float),
        ("weights", smpc_cost_weights),
        ("U_in", c_void_p), ("U_out", c_void_p),
        ("costs_out", c_void_p), ("weights_out", c_void_p), ("stats_out", c_void_p),
        ("receding", c_int32),
        ("u0_out", c_void_p), ("state_in", c_void_p), ("state_out", c_void_p),
    ]


class smpc_controller_desc(ctypes.Structure):
    _fields_ = [
        ("esdf", smpc_grid),
        ("K", c_int32), ("H", c_int32),
        ("dt", c_float), ("lambda_", c_float),
        ("weights", smpc_cost_weights),
        ("sigma", c_float * NDOF),
        ("U_star_out", c_void_p),
        ("costs_out", c_void_p),
    ]


class smpc_request(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int64),
        ("controller", c_int32), ("reserved", c_int32),
        ("q0", c_float * NDOF), ("qd0", c_float * NDOF),
        ("T_goal", c_float * 16),
        ("seed", c_uint64),
    ]


class smpc_camera(ctypes.Structure):
    _fields_ = [
        ("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
        ("width", c_int32), ("height", c_int32),
        ("T_wc", c_float * 16),
        ("min_depth", c_float), ("max_depth", c_float),
    ]


class smpc_ogm_params(ctypes.Structure):
    _fields_ = [(name, c_float) for name in (
        "tol", "l_hit", "l_miss", "l_min", "l_max", "l_occ", "robot_pad")]


class smpc_completion(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int64),
        ("controller", c_int32), ("status", c_int32),
        ("u0", c_float * NDOF),
        ("S_min", c_float), ("Z", c_float), ("ess", c_float),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsmpc (once).  Raises OSError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it with `python -m paper_2512_22575_amd.build`")
    # PyTorch wheels bundle their own HIP runtime.  Loading torch first makes this
    # library bind to that same runtime (same soname); the other order leaves two
    # runtimes in the process and device calls fail.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    lib.smpc_create.argtypes = [POINTER(c_void_p), c_int32]
    lib.smpc_create.restype = c_int32
    lib.smpc_destroy.argtypes = [c_void_p]
    lib.smpc_destroy.restype = None
    lib.smpc_set_robot.argtypes = [c_void_p, POINTER(smpc_robot_desc)]
    lib.smpc_set_robot.restype = c_int32
    lib.smpc_plan_step.argtypes = [c_void_p, POINTER(smpc_plan_args), c_void_p]
    lib.smpc_plan_step.restype = c_int32
    lib.smpc_plan_step_noalloc.argtypes = [c_void_p, POINTER(smpc_plan_args), c_void_p]
    lib.smpc_plan_step_noalloc.restype = c_int32
    lib.smpc_plan_step_then_bounds.argtypes = [c_void_p, POINTER(smpc_plan_args),
                                               POINTER(smpc_grid), POINTER(c_float), c_float,
                                               c_void_p, c_void_p]
    lib.smpc_plan_step_then_bounds.restype = c_int32
    lib.smpc_status_string.argtypes = [c_int32]
    lib.smpc_status_string.restype = c_char_p
    lib.smpc_last_error.argtypes = [c_void_p]
    lib.smpc_last_error.restype = c_char_p
    lib.smpc_version.argtypes = []
    lib.smpc_version.restype = c_int32
    lib.smpc_sample_noise.argtypes = [c_uint64, c_int32, c_int32, POINTER(c_float), c_void_p,
                                      c_void_p, c_void_p]
    lib.smpc_sample_noise.restype = c_int32
    lib.smpc_grid_to_f16.argtypes = [c_void_p, c_void_p, ctypes.c_int64, c_float, c_void_p]
    lib.smpc_grid_to_f16.restype = c_int32
    lib.smpc_grid_coarse_cells.argtypes = [c_int32, c_int32, c_int32]
    lib.smpc_grid_coarse_cells.restype = ctypes.c_int64
    lib.smpc_grid_coarse_min.argtypes = [POINTER(smpc_grid), c_void_p, c_void_p]
    lib.smpc_grid_coarse_min_ball.argtypes = [POINTER(smpc_grid), POINTER(c_float), c_float,
                                              c_void_p, c_void_p]
    lib.smpc_grid_coarse_min_ball.restype = c_int32
    lib.smpc_robot_reach.argtypes = [c_void_p, POINTER(c_float), POINTER(c_float)]
    lib.smpc_robot_reach.restype = c_int32
    lib.smpc_grid_coarse_min.restype = c_int32
    lib.smpc_plan_workspace_bytes.argtypes = [c_int32, c_int32]
    lib.smpc_edt_workspace_bytes.argtypes = [c_int32, c_int32, c_int32]
    lib.smpc_edt_workspace_bytes.restype = c_uint64
    lib.smpc_edt.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_float, c_void_p, c_void_p,
                             c_void_p, c_uint64, c_void_p]
    lib.smpc_edt.restype = c_int32
    lib.smpc_plan_workspace_bytes.restype = c_uint64
    lib.smpc_ogm_workspace_bytes.argtypes = [c_int32, c_int32]
    lib.smpc_ogm_workspace_bytes.restype = c_uint64
    lib.smpc_ogm_update.argtypes = [c_void_p, POINTER(c_float), c_void_p, POINTER(smpc_camera),
                                    c_void_p, c_void_p, c_int32, c_int32, c_int32,
                                    POINTER(c_float), c_float, POINTER(smpc_ogm_params),
                                    c_void_p, c_uint64, c_void_p]
    lib.smpc_ogm_update.restype = c_int32
    lib.smpc_server_create.argtypes = [POINTER(c_void_p), c_void_p, c_uint64, c_int32]
    lib.smpc_server_create.restype = c_int32
    lib.smpc_server_destroy.argtypes = [c_void_p]
    lib.smpc_server_destroy.restype = None
    lib.smpc_server_add_controller.argtypes = [c_void_p, POINTER(smpc_controller_desc),
                                               POINTER(c_int32)]
    lib.smpc_server_add_controller.restype = c_int32
    lib.smpc_server_reset_controller.argtypes = [c_void_p, c_int32]
    lib.smpc_server_reset_controller.restype = c_int32
    lib.smpc_server_submit.argtypes = [c_void_p, POINTER(smpc_request)]
    lib.smpc_server_submit.restype = c_int32
    lib.smpc_server_pump.argtypes = [c_void_p, c_void_p, POINTER(c_int32)]
    lib.smpc_server_pump.restype = c_int32
    lib.smpc_server_poll.argtypes = [c_void_p, POINTER(smpc_completion), c_int32, POINTER(c_int32)]
    lib.smpc_server_poll.restype = c_int32
    lib.smpc_server_queued.argtypes = [c_void_p]
    lib.smpc_server_queued.restype = c_int32
    lib.smpc_server_in_flight.argtypes = [c_void_p]
    lib.smpc_server_in_flight.restype = c_int32
    lib.smpc_server_last_error.argtypes = [c_void_p]
    lib.smpc_server_last_error.restype = c_char_p
    lib.smpc_profile_enable.argtypes = [c_void_p, c_int32]
    lib.smpc_profile_enable.restype = c_int32
    lib.smpc_profile_read.argtypes = [c_void_p, POINTER(c_float), POINTER(c_float), c_int32,
                                      POINTER(c_int32)]
    lib.smpc_profile_read.restype = c_int32
    _lib = lib
    return lib


# --- one-to-one wrappers ------------------------------------------------------

def smpc_create(hip_device: int = 0) -> tuple[int, c_void_p]:
    h = c_void_p()
    st = load_library().smpc_create(ctypes.byref(h), int(hip_device))
    return st, h


def smpc_destroy(ctx: c_void_p) -> None:
    load_library().smpc_destroy(ctx)


def smpc_set_robot(ctx: c_void_p, desc: smpc_robot_desc) -> int:
    return load_library().smpc_set_robot(ctx, ctypes.byref(desc))


def smpc_plan_step(ctx: c_void_p, args: smpc_plan_args, stream: int | None) -> int:
    return load_library().smpc_plan_step(ctx, ctypes.byref(args), c_void_p(stream or 0))


def smpc_plan_step_noalloc(ctx: c_void_p, args: smpc_plan_args, stream: int | None) -> int:
    return load_library().smpc_plan_step_noalloc(ctx, ctypes.byref(args), c_void_p(stream or 0))


def smpc_plan_step_then_bounds(ctx: c_void_p, args: smpc_plan_args, next_grid, dtype: int,
                               origin, voxel: float, center, radius: float, coarse_out: int,
                               stream: int | None) -> int:
    """Plan step, and the ball-restricted bounds of next_grid (device tensor [nz][ny][nx]
    at origin / voxel) built by the step's merge launch into coarse_out."""
    nz, ny, nx = (int(x) for x in next_grid.shape)
    g = smpc_grid(c_void_p(_ptr(next_grid)), nx, ny, nz, int(dtype),
                  (c_float * 3)(*[float(x) for x in np.asarray(origin, np.float32)]),
                  float(voxel), None)
    c = (c_float * 3)(*[float(x) for x in np.asarray(center, np.float32)])
    return load_library().smpc_plan_step_then_bounds(ctx, ctypes.byref(args), ctypes.byref(g),
                                                     c, float(radius), c_void_p(coarse_out or 0),
                                                     c_void_p(stream or 0))


def smpc_status_string(status: int) -> str:
    return load_library().smpc_status_string(int(status)).decode()


def smpc_last_error(ctx: c_void_p) -> str:
    return load_library().smpc_last_error(ctx).decode()


def smpc_version() -> int:
    return int(load_library().smpc_version())


def smpc_sample_noise(seed: int, K: int, H: int, sigma, eps_out: int, words_out: int,
                      stream: int | None) -> int:
    """eps_out / words_out are device addresses (0 for none)."""
    sg = (c_float * NDOF)(*[float(x) for x in np.broadcast_to(np.asarray(sigma, np.float32), (NDOF,))])
    return load_library().smpc_sample_noise(int(seed), int(K), int(H), sg, c_void_p(eps_out or 0),
                                            c_void_p(words_out or 0), c_void_p(stream or 0))


def smpc_grid_coarse_cells(nx: int, ny: int, nz: int) -> int:
    return int(load_library().smpc_grid_coarse_cells(int(nx), int(ny), int(nz)))


def smpc_grid_coarse_min(grid, dtype: int, coarse_out: int, stream: int | None) -> int:
    """Coarse lower bounds of a device grid (torch tensor [nz][ny][nx]) into coarse_out."""
    nz, ny, nx = (int(x) for x in grid.shape)
    g = smpc_grid(c_void_p(_ptr(grid)), nx, ny, nz, int(dtype), (c_float * 3)(0.0, 0.0, 0.0),
                  1.0, None)
    return load_library().smpc_grid_coarse_min(ctypes.byref(g), c_void_p(coarse_out or 0),
                                                c_void_p(stream or 0))


def smpc_grid_coarse_min_ball(grid, dtype: int, origin, voxel: float, center, radius: float,
                              coarse_out: int, stream: int | None) -> int:
    """Coarse lower bounds restricted to the cells the lookups of a ball reach (the others
    -inf); grid is a device tensor [nz][ny][nx] at `origin` / `voxel`."""
    nz, ny, nx = (int(x) for x in grid.shape)
    g = smpc_grid(c_void_p(_ptr(grid)), nx, ny, nz, int(dtype),
                  (c_float * 3)(*[float(x) for x in np.asarray(origin, np.float32)]),
                  float(voxel), None)
    c = (c_float * 3)(*[float(x) for x in np.asarray(center, np.float32)])
    return load_library().smpc_grid_coarse_min_ball(ctypes.byref(g), c, float(radius),
                                                    c_void_p(coarse_out or 0),
                                                    c_void_p(stream or 0))


def smpc_robot_reach(ctx: c_void_p):
    """(status, centre (3,), radius) of the ball holding every sphere centre of the robot."""
    c = (c_float * 3)()
    r = c_float()
    st = load_library().smpc_robot_reach(ctx, c, ctypes.byref(r))
    return st, np.array(c[:], np.float32), float(r.value)


def smpc_grid_to_f16(src: int, dst: int, n: int, clamp: float, stream: int | None) -> int:
    return load_library().smpc_grid_to_f16(c_void_p(src or 0), c_void_p(dst or 0), int(n),
                                           float(clamp), c_void_p(stream or 0))


def smpc_profile_enable(ctx: c_void_p, n_steps: int) -> int:
    return load_library().smpc_profile_enable(ctx, int(n_steps))


def smpc_profile_read(ctx: c_void_p, capacity: int):
    """Returns (status, rollout_ms ndarray, merge_ms ndarray)."""
    r = (c_float * capacity)()
    m = (c_float * capacity)()
    n = c_int32(0)
    st = load_library().smpc_profile_read(ctx, r, m, int(capacity), ctypes.byref(n))
    return st, np.array(r[:n.value], np.float64), np.array(m[:n.value], np.float64)


# --- marshalling helpers --------------------------------------------------------

def robot_desc(robot) -> smpc_robot_desc:
    """Fill an smpc_robot_desc from an object with the fields of synth.robot.Robot."""
    d = smpc_robot_desc()
    d.n_dof = NDOF
    for name in ("a", "d", "alpha", "q_min", "q_max", "qd_min", "qd_max", "qdd_min",
                 "qdd_max", "q_ref"):
        getattr(d, name)[:] = [float(x) for x in np.asarray(getattr(robot, name))]
    n_s = int(len(robot.sphere_radius))
    if n_s > MAX_SPHERES:
        raise ValueError(f"{n_s} spheres exceed the ABI limit {MAX_SPHERES}")
    d.n_spheres = n_s
    for s in range(n_s):
        d.sphere_link[s] = int(robot.sphere_link[s])
        d.sphere_center[s][:] = [float(x) for x in robot.sphere_center[s]]
        d.sphere_radius[s] = float(robot.sphere_radius[s])
    pairs = np.asarray(robot.pairs, dtype=np.int64).reshape(-1, 2)
    if pairs.shape[0] > MAX_PAIRS:
        raise ValueError(f"{pairs.shape[0]} pairs exceed the ABI limit {MAX_PAIRS}")
    d.n_pairs = int(pairs.shape[0])
    for i, (a, b) in enumerate(pairs):
        d.pairs[i][0] = int(a)
        d.pairs[i][1] = int(b)
    return d


def cost_weights(w: dict) -> smpc_cost_weights:
    cw = smpc_cost_weights()
    for name, _ in smpc_cost_weights._fields_:
        setattr(cw, name, float(w[name]))
    return cw


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def plan_args(q0, qd0, T_goal, grid, origin, voxel, noise, U_in, U_out, K, H, dt, lam,
              weights: dict, costs_out=None, weights_out=None, stats_out=None, seed: int = 0,
              sigma=None, grid_dtype: int = GRID_F32, coarse=None, receding: bool = False,
              u0_out=None, state_in=None, state_out=None) -> smpc_plan_args:
    """Build smpc_plan_args; tensors are torch tensors on the device (or None)."""
    a = smpc_plan_args()
    a.q0[:] = [float(x) for x in np.asarray(q0, np.float32)]
    a.qd0[:] = [float(x) for x in np.asarray(qd0, np.float32)]
    a.T_goal[:] = [float(x) for x in np.asarray(T_goal, np.float32).reshape(16)]
    nz, ny, nx = (int(s) for s in grid.shape)
    a.esdf = smpc_grid(c_void_p(_ptr(grid)), nx, ny, nz, int(grid_dtype),
                       (c_float * 3)(*[float(x) for x in np.asarray(origin, np.float32)]),
                       float(voxel), c_void_p(_ptr(coarse)))
    a.noise = _ptr(noise)
    a.seed = int(seed)
    a.sigma[:] = [0.5] * NDOF if sigma is None else [float(x) for x in sigma]
    a.K, a.H = int(K), int(H)
    a.dt, a.lambda_ = float(dt), float(lam)
    a.weights = cost_weights(weights)
    a.U_in, a.U_out = _ptr(U_in), _ptr(U_out)
    a.costs_out, a.weights_out, a.stats_out = _ptr(costs_out), _ptr(weights_out), _ptr(stats_out)
    a.receding = 1 if receding else 0
    a.u0_out, a.state_in, a.state_out = _ptr(u0_out), _ptr(state_in), _ptr(state_out)
    return a


class SMPCError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{smpc_status_string(status)} ({status}): {detail}")
        self.status = status


class Planner:
    """Context owning one robot; plan steps take torch tensors on ``cuda:device``."""

    def __init__(self, robot, device: int = 0):
        st, self._ctx = smpc_create(device)
        if st != SMPC_OK:
            raise SMPCError(st, "smpc_create")
        self.device = device
        st = smpc_set_robot(self._ctx, robot_desc(robot))
        if st != SMPC_OK:
            raise SMPCError(st, smpc_last_error(self._ctx))

    def robot_reach(self):
        """(centre, radius) of a ball holding every sphere centre at any joint values."""
        st, c, r = smpc_robot_reach(self._ctx)
        if st != SMPC_OK:
            raise SMPCError(st, "smpc_robot_reach")
        return c, r

    def profile_enable(self, n_steps: int) -> None:
        st = smpc_profile_enable(self._ctx, n_steps)
        if st != SMPC_OK:
            raise SMPCError(st, smpc_last_error(self._ctx))

    def profile_read(self, capacity: int):
        """Per-step kernel durations (ms) of the recorded steps: (rollout_ms, merge_ms)."""
        st, r, m = smpc_profile_read(self._ctx, capacity)
        if st != SMPC_OK:
            raise SMPCError(st, smpc_last_error(self._ctx))
        return r, m

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            smpc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def plan_step(self, *, q0, qd0, T_goal, grid, origin, voxel, noise, U_in, U_out, dt, lam,
                  weights, costs_out=None, weights_out=None, stats_out=None, stream=None,
                  seed: int = 0, sigma=None, grid_dtype: int = GRID_F32, K=None, H=None,
                  coarse=None, receding: bool = False, u0_out=None, state_in=None,
                  state_out=None, noalloc: bool = False, next_bounds=None) -> None:
        """Enqueue one plan step on ``stream`` (default: torch's current stream);
        ``noalloc`` takes the workspace from the library's static device scratch;
        ``next_bounds`` = (grid, dtype, origin, voxel, coarse_out) also builds that grid's
        bounds within the robot's reach into coarse_out (smpc_plan_step_then_bounds)."""
        import torch
        if noise is not None:
            K, H = int(noise.shape[0]), int(noise.shape[1])
        elif K is None or H is None:
            raise ValueError("K and H are required when the plan step samples its own noise")
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        a = plan_args(q0, qd0, T_goal, grid, origin, voxel, noise, U_in, U_out, K, H, dt, lam,
                      weights, costs_out, weights_out, stats_out, seed, sigma, grid_dtype,
                      coarse, receding, u0_out, state_in, state_out)
        if next_bounds is not None:
            if noalloc:
                raise ValueError("next_bounds has no allocation-free form")
            g, dt_g, org, vox, out = next_bounds
            c, r = self.robot_reach()
            st = smpc_plan_step_then_bounds(self._ctx, a, g, dt_g, org, vox, c, r, _ptr(out),
                                            stream)
        else:
            st = (smpc_plan_step_noalloc if noalloc else smpc_plan_step)(self._ctx, a, stream)
        if st != SMPC_OK:
            raise SMPCError(st, smpc_last_error(self._ctx))

    def ogm_update(self, *, depth, cam: smpc_camera, log_odds, origin, voxel,
                   prm: smpc_ogm_params, work, q=None, occ_out=None, stream=None) -> None:
        """Enqueue one occupancy update (tensors on the device; log_odds (nz, ny, nx)
        float32 updated in place); q given: this planner's robot masks the update."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        nz, ny, nx = (int(s) for s in log_odds.shape)
        st = smpc_ogm_update(self._ctx, q, _ptr(depth), cam, _ptr(log_odds), _ptr(occ_out),
                             nx, ny, nz, origin, voxel, prm, _ptr(work),
                             work.numel() * work.element_size(), stream)
        if st != SMPC_OK:
            raise SMPCError(st, smpc_last_error(self._ctx))


class RecedingHorizon:
    """Closed-loop plan steps of one controller with its state on the device.

    Each ``step`` enqueues one plan step from the device-resident joint state and
    nominal sequence; the library executes u*_0 for one period (the rollouts'
    integrator) and shifts the sequence to [u*_1 .. u*_{H-1}, 0] (the receding-horizon
    execution of the paper's Sec. IV-C), so consecutive periods need no host round
    trip.  Two state and two sequence buffers alternate: a step reads one and writes
    the other.  ``state``, ``U`` and ``u0`` are the current device tensors.
    """

    def __init__(self, planner: "Planner", H: int, q0, qd0, U0=None):
        import torch
        dev = torch.device("cuda", planner.device)
        self.planner = planner
        self.H = int(H)
        self._q0 = np.asarray(q0, np.float32)
        self._qd0 = np.asarray(qd0, np.float32)
        self._U = [torch.zeros((self.H, NDOF), device=dev) for _ in range(2)]
        self._X = [torch.zeros((2 * NDOF,), device=dev) for _ in range(2)]
        self.u0 = torch.zeros((NDOF,), device=dev)
        self._cur = 0
        self.set_state(q0, qd0)
        if U0 is not None:
            self.set_nominal(U0)

    @property
    def state(self):
        return self._X[self._cur]

    @property
    def U(self):
        return self._U[self._cur]

    def set_state(self, q, qd) -> None:
        import torch
        x = np.concatenate([np.asarray(q, np.float32), np.asarray(qd, np.float32)])
        self._X[self._cur].copy_(torch.from_numpy(x))

    def set_nominal(self, U) -> None:
        import torch
        self._U[self._cur].copy_(torch.from_numpy(np.asarray(U, np.float32).reshape(self.H, NDOF)))

    def step(self, *, T_goal, grid, origin, voxel, dt, lam, weights, noise=None, seed: int = 0,
             sigma=None, K=None, coarse=None, costs_out=None, weights_out=None, stats_out=None,
             grid_dtype: int = GRID_F32, stream=None, next_bounds=None) -> None:
        """Enqueue one control period on ``stream`` (default: torch's current stream);
        ``next_bounds`` as for Planner.plan_step (the next period's map, when known)."""
        nxt = 1 - self._cur
        self.planner.plan_step(q0=self._q0, qd0=self._qd0, T_goal=T_goal, grid=grid,
                               origin=origin, voxel=voxel, noise=noise, U_in=self._U[self._cur],
                               U_out=self._U[nxt], dt=dt, lam=lam, weights=weights,
                               costs_out=costs_out, weights_out=weights_out, stats_out=stats_out,
                               stream=stream, seed=seed, sigma=sigma, grid_dtype=grid_dtype, K=K,
                               H=self.H, coarse=coarse, receding=True, u0_out=self.u0,
                               state_in=self._X[self._cur], state_out=self._X[nxt],
                               next_bounds=next_bounds)
        self._cur = nxt


def is_finite_float(x) -> bool:
    return math.isfinite(float(x))


# --- serving ---------------------------------------------------------------------

def smpc_plan_workspace_bytes(K: int, H: int) -> int:
    return int(load_library().smpc_plan_workspace_bytes(int(K), int(H)))


def smpc_edt_workspace_bytes(nx: int, ny: int, nz: int) -> int:
    return int(load_library().smpc_edt_workspace_bytes(int(nx), int(ny), int(nz)))


def smpc_edt(occ: int, nx: int, ny: int, nz: int, voxel: float, phi_out: int | None,
             d2_out: int | None, work: int, work_bytes: int, stream: int | None) -> int:
    """Signed distance field of a device occupancy grid (pointers as integers)."""
    return load_library().smpc_edt(c_void_p(occ or 0), int(nx), int(ny), int(nz), float(voxel),
                                   c_void_p(phi_out or 0), c_void_p(d2_out or 0),
                                   c_void_p(work or 0), int(work_bytes), c_void_p(stream or 0))


def make_camera(fx, fy, cx, cy, width, height, T_wc, min_depth, max_depth) -> smpc_camera:
    c = smpc_camera()
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    c.width, c.height = int(width), int(height)
    c.T_wc[:] = [float(x) for x in np.asarray(T_wc, np.float32).reshape(16)]
    c.min_depth, c.max_depth = float(min_depth), float(max_depth)
    return c


def make_ogm_params(tol, l_hit, l_miss, l_min, l_max, l_occ, robot_pad=0.0) -> smpc_ogm_params:
    return smpc_ogm_params(float(tol), float(l_hit), float(l_miss), float(l_min), float(l_max),
                           float(l_occ), float(robot_pad))


def smpc_ogm_workspace_bytes(width: int, height: int) -> int:
    return int(load_library().smpc_ogm_workspace_bytes(int(width), int(height)))


def smpc_ogm_update(ctx, q, depth: int, cam: smpc_camera, log_odds: int, occ_out: int | None,
                    nx: int, ny: int, nz: int, origin, voxel: float, prm: smpc_ogm_params,
                    work: int, work_bytes: int, stream: int | None) -> int:
    """One occupancy update (device pointers as integers; q: 7 joint positions or None)."""
    qa = None
    if q is not None:
        qa = (c_float * NDOF)(*[float(x) for x in np.asarray(q, np.float32).reshape(NDOF)])
    oa = (c_float * 3)(*[float(x) for x in np.asarray(origin, np.float32).reshape(3)])
    return load_library().smpc_ogm_update(
        ctx, qa, c_void_p(depth or 0), ctypes.byref(cam), c_void_p(log_odds or 0),
        c_void_p(occ_out or 0), int(nx), int(ny), int(nz), oa, float(voxel), ctypes.byref(prm),
        c_void_p(work or 0), int(work_bytes), c_void_p(stream or 0))


def smpc_server_create(ctx: c_void_p, hbm_budget_bytes: int, max_batch: int):
    h = c_void_p()
    st = load_library().smpc_server_create(ctypes.byref(h), ctx, int(hbm_budget_bytes),
                                           int(max_batch))
    return st, h


def smpc_server_destroy(server: c_void_p) -> None:
    load_library().smpc_server_destroy(server)


def smpc_server_add_controller(server: c_void_p, desc: smpc_controller_desc):
    cid = c_int32(-1)
    st = load_library().smpc_server_add_controller(server, ctypes.byref(desc), ctypes.byref(cid))
    return st, cid.value


def smpc_server_reset_controller(server: c_void_p, cid: int) -> int:
    return load_library().smpc_server_reset_controller(server, int(cid))


def smpc_server_submit(server: c_void_p, req: smpc_request) -> int:
    return load_library().smpc_server_submit(server, ctypes.byref(req))


def smpc_server_pump(server: c_void_p, stream: int | None):
    n = c_int32(0)
    st = load_library().smpc_server_pump(server, c_void_p(stream or 0), ctypes.byref(n))
    return st, n.value


def smpc_server_poll(server: c_void_p, capacity: int = 256):
    buf = (smpc_completion * capacity)()
    n = c_int32(0)
    st = load_library().smpc_server_poll(server, buf, int(capacity), ctypes.byref(n))
    return st, [buf[i] for i in range(n.value)]


def smpc_server_queued(server: c_void_p) -> int:
    return int(load_library().smpc_server_queued(server))


def smpc_server_in_flight(server: c_void_p) -> int:
    return int(load_library().smpc_server_in_flight(server))


def smpc_server_last_error(server: c_void_p) -> str:
    return load_library().smpc_server_last_error(server).decode()


def controller_desc(grid, origin, voxel, K, H, dt, lam, weights, sigma,
                    grid_dtype: int = GRID_F32, coarse=None, U_star_out=None,
                    costs_out=None) -> smpc_controller_desc:
    d = smpc_controller_desc()
    nz, ny, nx = (int(x) for x in grid.shape)
    d.esdf = smpc_grid(c_void_p(_ptr(grid)), nx, ny, nz, int(grid_dtype),
                       (c_float * 3)(*[float(x) for x in np.asarray(origin, np.float32)]),
                       float(voxel), c_void_p(_ptr(coarse)))
    d.K, d.H = int(K), int(H)
    d.dt, d.lambda_ = float(dt), float(lam)
    d.weights = cost_weights(weights)
    d.sigma[:] = [float(x) for x in np.broadcast_to(np.asarray(sigma, np.float32), (NDOF,))]
    d.U_star_out = c_void_p(_ptr(U_star_out))
    d.costs_out = c_void_p(_ptr(costs_out))
    return d


def request(tag: int, controller: int, q0, qd0, T_goal, seed: int) -> smpc_request:
    r = smpc_request()
    r.tag = int(tag)
    r.controller = int(controller)
    r.reserved = 0
    r.q0[:] = [float(x) for x in np.asarray(q0, np.float32)]
    r.qd0[:] = [float(x) for x in np.asarray(qd0, np.float32)]
    r.T_goal[:] = [float(x) for x in np.asarray(T_goal, np.float32).reshape(16)]
    r.seed = int(seed)
    return r


class Server:
    """Continuous-batching server on a Planner's context (see include/smpc.h)."""

    def __init__(self, planner: "Planner", hbm_budget_bytes: int = 256 << 20, max_batch: int = 64):
        st, self._h = smpc_server_create(planner._ctx, hbm_budget_bytes, max_batch)
        if st != SMPC_OK:
            raise SMPCError(st, smpc_last_error(planner._ctx))
        self._keep = []   # device tensors the controllers reference

    def add_controller(self, grid, origin, voxel, K, H, dt, lam, weights, sigma,
                       grid_dtype: int = GRID_F32, coarse=None, U_star_out=None,
                       costs_out=None) -> int:
        """Register a controller; the optional device tensors U_star_out [H][7] and
        costs_out [K] receive each served request's U* and rollout costs."""
        for t in (grid, coarse, U_star_out, costs_out):
            if t is not None:
                self._keep.append(t)
        st, cid = smpc_server_add_controller(
            self._h, controller_desc(grid, origin, voxel, K, H, dt, lam, weights, sigma, grid_dtype,
                                     coarse, U_star_out, costs_out))
        if st != SMPC_OK:
            raise SMPCError(st, smpc_server_last_error(self._h))
        return cid

    def submit(self, tag, controller, q0, qd0, T_goal, seed) -> None:
        st = smpc_server_submit(self._h, request(tag, controller, q0, qd0, T_goal, seed))
        if st != SMPC_OK:
            raise SMPCError(st, smpc_server_last_error(self._h))

    def pump(self, stream=None) -> int:
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st, n = smpc_server_pump(self._h, stream)
        if st != SMPC_OK:
            raise SMPCError(st, smpc_server_last_error(self._h))
        return n

    def poll(self, capacity: int = 256):
        st, out = smpc_server_poll(self._h, capacity)
        if st != SMPC_OK:
            raise SMPCError(st, "poll")
        return out

    def queued(self) -> int:
        return smpc_server_queued(self._h)

    def in_flight(self) -> int:
        return smpc_server_in_flight(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            smpc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
