"""FP64 CPU oracle for one sampling-based MPC (SMPC) plan step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call this
module; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library.

It computes, plainly and slowly, what one plan step of the paper's planner
(ParaMaP, arXiv:2512.22575, Sec. IV, Algorithm 1) computes, for a fixed set of
sampled disturbances:

1. controls u_k^(m) = ubar_k + eps_k^(m)                       (eq. 27)
2. roll out the dynamics q_{k+1} = f(q_k, u_k)                 (eq. 7)
3. forward kinematics of every link frame                      (eq. 6)
4. running cost at k = 0..H-1 and terminal cost at k = H       (eqs. 9, 16-25, 28)
5. soft weights with the minimum cost subtracted               (eq. 29)
6. updated sequence U* = Ubar + sum_m w^(m) eps^(m)            (eq. 30)

Arithmetic is float64 throughout; inputs are whatever the caller passes (the
tests pass the same float32-rounded values the GPU consumes).  The batch axis m
is vectorised with numpy; the time, joint, sphere and pair loops are explicit.

Readings of points the paper leaves open (each is a documented choice):

* integrator: semi-implicit Euler, qd_{k+1} = qd_k + u_k dt, q_{k+1} = q_k + qd_{k+1} dt
  (the paper only says the control is the joint acceleration);
* kinematics: Craig's modified DH, A_i = RotX(alpha_i) TransX(a_i) RotZ(q_i) TransZ(d_i),
  base frame at the world origin, end effector = frame 7;
* running terms use (q_k, qd_k, u_k) for k = 0..H-1, terminal term uses q_H only;
* distance lookup: trilinear interpolation between voxel centres with the
  query clamped to the grid (edge extension);
* joint-limit margin eps_i = rho (x_max - x_min), applied to q, qd and u;
* Q_k = diag(w_pose_t I3, w_pose_r I3), Q_H = diag(w_term_t I3, w_term_r I3);
* non-finite rollout costs get weight 0; if none is finite, U* = Ubar.
"""
from __future__ import annotations

import numpy as np

N_DOF = 7


# ---------------------------------------------------------------------------
# Dynamics (eq. 7)
# ---------------------------------------------------------------------------

def rollout(q0, qd0, U, dt):
    """Integrate joint accelerations U (M, H, 7) from (q0, qd0) with semi-implicit Euler.

    Returns q, qd of shape (M, H+1, 7) holding states k = 0..H (Algorithm 1, roll-out step).
    """
    U = np.asarray(U, np.float64)
    M, H, n = U.shape
    q = np.empty((M, H + 1, n))
    qd = np.empty((M, H + 1, n))
    q[:, 0] = q0
    qd[:, 0] = qd0
    for k in range(H):
        qd[:, k + 1] = qd[:, k] + U[:, k] * dt
        q[:, k + 1] = q[:, k] + qd[:, k + 1] * dt
    return q, qd


# ---------------------------------------------------------------------------
# Forward kinematics (eq. 6)
# ---------------------------------------------------------------------------

def rot_x(angle):
    """Homogeneous rotation about x; angle is a scalar or an (M,) array."""
    c, s = np.cos(angle), np.sin(angle)
    c, s = np.broadcast_arrays(np.asarray(c, np.float64), np.asarray(s, np.float64))
    T = np.zeros(c.shape + (4, 4))
    T[..., 0, 0] = 1.0
    T[..., 1, 1] = c
    T[..., 1, 2] = -s
    T[..., 2, 1] = s
    T[..., 2, 2] = c
    T[..., 3, 3] = 1.0
    return T


def rot_z(angle):
    c, s = np.cos(angle), np.sin(angle)
    c, s = np.broadcast_arrays(np.asarray(c, np.float64), np.asarray(s, np.float64))
    T = np.zeros(c.shape + (4, 4))
    T[..., 0, 0] = c
    T[..., 0, 1] = -s
    T[..., 1, 0] = s
    T[..., 1, 1] = c
    T[..., 2, 2] = 1.0
    T[..., 3, 3] = 1.0
    return T


def trans(x, y, z):
    T = np.eye(4)
    T[0, 3], T[1, 3], T[2, 3] = x, y, z
    return T


def mdh_joint_transform(alpha, a, theta, d):
    """A = RotX(alpha) TransX(a) RotZ(theta) TransZ(d) for a batch of angles theta."""
    return rot_x(alpha) @ trans(a, 0.0, 0.0) @ rot_z(theta) @ trans(0.0, 0.0, d)


def forward_kinematics(robot, q):
    """Link frames T^0..T^7 for joint configurations q (M, 7) -> (M, 8, 4, 4).

    T^0 = I (base at the world origin), T^i = T^{i-1} A_i(q_i); the end effector
    is T^7 (Sec. IV-A: the last frame of the chain).
    """
    q = np.atleast_2d(np.asarray(q, np.float64))
    M = q.shape[0]
    frames = np.empty((M, N_DOF + 1, 4, 4))
    frames[:, 0] = np.eye(4)
    for i in range(N_DOF):
        A = mdh_joint_transform(robot.alpha[i], robot.a[i], q[:, i], robot.d[i])
        frames[:, i + 1] = frames[:, i] @ A
    return frames


def sphere_centres(robot, frames):
    """World centres p_i of the collision spheres, (M, n_s, 3) (Sec. IV-B-2)."""
    M = frames.shape[0]
    out = np.empty((M, robot.n_spheres, 3))
    for i in range(robot.n_spheres):
        T = frames[:, int(robot.sphere_link[i])]
        c = np.asarray(robot.sphere_center[i], np.float64)
        out[:, i] = T[:, :3, :3] @ c + T[:, :3, 3]
    return out


# ---------------------------------------------------------------------------
# SE(3) logarithm (eqs. 11-15)
# ---------------------------------------------------------------------------

def hat(w):
    """[w]_x for a batch of 3-vectors (M, 3) -> (M, 3, 3)."""
    w = np.asarray(w, np.float64)
    W = np.zeros(w.shape[:-1] + (3, 3))
    W[..., 0, 1] = -w[..., 2]
    W[..., 0, 2] = w[..., 1]
    W[..., 1, 0] = w[..., 2]
    W[..., 1, 2] = -w[..., 0]
    W[..., 2, 0] = -w[..., 1]
    W[..., 2, 1] = w[..., 0]
    return W


def so3_log(R):
    """Rotation vector omega with R = exp([omega]_x), |omega| in [0, pi]; R is (M, 3, 3)."""
    R = np.asarray(R, np.float64)
    vee = np.stack([R[..., 2, 1] - R[..., 1, 2],
                    R[..., 0, 2] - R[..., 2, 0],
                    R[..., 1, 0] - R[..., 0, 1]], axis=-1)          # = 2 sin(theta) n
    sin_t = 0.5 * np.linalg.norm(vee, axis=-1)
    cos_t = 0.5 * (np.trace(R, axis1=-2, axis2=-1) - 1.0)
    theta = np.arctan2(sin_t, cos_t)
    # Generic case: omega = theta / (2 sin theta) * vee (and vee / 2 as theta -> 0).
    safe_sin = np.where(sin_t > 0.0, sin_t, 1.0)
    scale = np.where(theta < 1e-12, 0.5, theta / (2.0 * safe_sin))
    omega = scale[..., None] * vee
    near_pi = (theta >= 1e-12) & (cos_t <= -0.5) & (sin_t <= 1e-3)
    for idx in zip(*np.nonzero(near_pi)):
        # Near pi the skew part vanishes; the axis comes from the symmetric part
        # (R + R^T)/2 - cos(theta) I = (1 - cos(theta)) n n^T.
        B = 0.5 * (R[idx] + R[idx].T) - cos_t[idx] * np.eye(3)
        col = int(np.argmax(np.diag(B)))
        n = B[:, col] / np.linalg.norm(B[:, col])
        if np.dot(n, vee[idx]) < 0:
            n = -n
        omega[idx] = theta[idx] * n
    return omega


def left_jacobian_V(omega):
    """V(theta) of eq. 14 for a batch of rotation vectors (M, 3) -> (M, 3, 3)."""
    omega = np.asarray(omega, np.float64)
    th = np.linalg.norm(omega, axis=-1)
    small = th < 1e-3
    th_safe = np.where(small, 1.0, th)
    th2 = th * th
    # (1 - cos t)/t^2 and (t - sin t)/t^3, by their Taylor series near t = 0.
    c1 = np.where(small, 0.5 - th2 / 24.0 + th2 * th2 / 720.0,
                  (1.0 - np.cos(th_safe)) / th_safe ** 2)
    c2 = np.where(small, 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0,
                  (th_safe - np.sin(th_safe)) / th_safe ** 3)
    W = hat(omega)
    return np.eye(3) + c1[..., None, None] * W + c2[..., None, None] * (W @ W)


def se3_log(T):
    """(v, omega) with log(T) = [[omega]_x, v; 0, 0] (eqs. 12-15); T is (M, 4, 4)."""
    T = np.asarray(T, np.float64)
    omega = so3_log(T[..., :3, :3])
    V = left_jacobian_V(omega)
    v = np.linalg.solve(V, T[..., :3, 3][..., None])[..., 0]        # t = V v (eq. 13)
    return v, omega


def pose_error(T_goal, T_ee):
    """xi = [v; omega] of Delta T = T_g^{-1} T_ee (eqs. 11-15)."""
    Tg = np.asarray(T_goal, np.float64)
    Rg, tg = Tg[:3, :3], Tg[:3, 3]
    D = np.zeros(T_ee.shape)
    D[..., :3, :3] = Rg.T @ T_ee[..., :3, :3]                        # R_Delta = R_g^T R
    D[..., :3, 3] = (T_ee[..., :3, 3] - tg) @ Rg                      # t_Delta = R_g^T (t - t_g)
    D[..., 3, 3] = 1.0
    return se3_log(D)


def pose_cost(T_goal, T_ee, w_t, w_r):
    """1/2 xi^T Q xi with Q = diag(w_t I3, w_r I3) (eqs. 16 and 25)."""
    v, omega = pose_error(T_goal, T_ee)
    return 0.5 * (w_t * np.sum(v * v, axis=-1) + w_r * np.sum(omega * omega, axis=-1))


# ---------------------------------------------------------------------------
# Distance field lookup and collision costs (eqs. 17-20)
# ---------------------------------------------------------------------------

def esdf_lookup(grid, origin, voxel, p):
    """Trilinear phi(p) from a (nz, ny, nx) grid of values at voxel centres.

    Continuous index u = (p - origin)/voxel - 1/2 per axis, clamped to [0, n-1];
    base corner i0 = min(floor(u), n-2), fraction f = u - i0.  A non-finite query
    point has no distance: the result is nan there.
    """
    grid = np.asarray(grid)          # corners are widened to float64 as they are read
    nz, ny, nx = grid.shape
    p = np.asarray(p, np.float64)
    bad = ~np.all(np.isfinite(p), axis=-1)
    p = np.where(bad[..., None], 0.0, p)
    u = (p - np.asarray(origin, np.float64)) / voxel - 0.5
    n = np.array([nx, ny, nz])
    u = np.clip(u, 0.0, n - 1)
    i0 = np.minimum(np.floor(u), n - 2).astype(np.int64)
    f = u - i0
    ix, iy, iz = i0[..., 0], i0[..., 1], i0[..., 2]
    fx, fy, fz = f[..., 0], f[..., 1], f[..., 2]
    phi = np.zeros(p.shape[:-1])
    for bz in (0, 1):
        wz = fz if bz else 1.0 - fz
        for by in (0, 1):
            wy = fy if by else 1.0 - fy
            for bx in (0, 1):
                wx = fx if bx else 1.0 - fx
                phi += wx * wy * wz * grid[iz + bz, iy + by, ix + bx].astype(np.float64)
    return np.where(bad, np.nan, phi)


def env_collision_cost(robot, centres, grid, origin, voxel, w_env, d_act):
    """sum_i w_env max(0, d_act - (phi(p_i) - r_i))^2 (eqs. 17, 19, 20)."""
    total = np.zeros(centres.shape[0])
    for i in range(robot.n_spheres):
        d_env = esdf_lookup(grid, origin, voxel, centres[:, i]) - robot.sphere_radius[i]
        delta = np.maximum(0.0, d_act - d_env)
        total += w_env * delta * delta
    return total


def self_collision_cost(robot, centres, w_self):
    """sum_{(i,j) in S} w_self max(0, -(|p_i - p_j| - (r_i + r_j)))^2 (eqs. 18-20)."""
    total = np.zeros(centres.shape[0])
    for i, j in robot.pairs:
        dist = np.linalg.norm(centres[:, i] - centres[:, j], axis=-1)
        d_self = dist - (robot.sphere_radius[i] + robot.sphere_radius[j])
        delta = np.maximum(0.0, -d_self)
        total += w_self * delta * delta
    return total


# ---------------------------------------------------------------------------
# Joint limits, smoothness, null space (eqs. 21-24)
# ---------------------------------------------------------------------------

def limit_violation(x, lo, hi, margin_frac):
    """delta_i(x) of eq. 21 on the interval tightened by margin_frac of its range."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    eps = margin_frac * (hi - lo)
    lo_e, hi_e = lo + eps, hi - eps
    return np.maximum(0.0, x - hi_e) + np.minimum(0.0, x - lo_e)


def limit_cost(robot, q, qd, qdd, w):
    """sum_i w_q d(q)^2 + w_qd d(qd)^2 + w_qdd d(qdd)^2 (eq. 22) for one time step."""
    rho = w["limit_margin_frac"]
    dq = limit_violation(q, robot.q_min, robot.q_max, rho)
    dqd = limit_violation(qd, robot.qd_min, robot.qd_max, rho)
    dqdd = limit_violation(qdd, robot.qdd_min, robot.qdd_max, rho)
    return (w["w_q"] * np.sum(dq * dq, axis=-1) + w["w_qd"] * np.sum(dqd * dqd, axis=-1)
            + w["w_qdd"] * np.sum(dqdd * dqdd, axis=-1))


def smoothness_cost(qdd, w_s):
    """w_s sum_i qdd_i^2 (eq. 23) for one time step."""
    return w_s * np.sum(qdd * qdd, axis=-1)


def null_space_cost(q, q_ref, w_ns):
    """w_ns sum_i (q_i - q_ref_i)^2 (eq. 24) for one time step."""
    e = q - np.asarray(q_ref, np.float64)
    return w_ns * np.sum(e * e, axis=-1)


# ---------------------------------------------------------------------------
# Rollout cost (eq. 28)
# ---------------------------------------------------------------------------

def running_cost(robot, q, qd, u, T_goal, grid, origin, voxel, w):
    """l(q_k, x_k, u_k): pose + collision + limits + smoothness + null space (Sec. IV-B)."""
    frames = forward_kinematics(robot, q)
    centres = sphere_centres(robot, frames)
    return (pose_cost(T_goal, frames[:, N_DOF], w["w_pose_t"], w["w_pose_r"])
            + env_collision_cost(robot, centres, grid, origin, voxel, w["w_env"], w["d_act"])
            + self_collision_cost(robot, centres, w["w_self"])
            + limit_cost(robot, q, qd, u, w)
            + smoothness_cost(u, w["w_smooth"])
            + null_space_cost(q, robot.q_ref, w["w_ns"]))


def terminal_cost(robot, q_H, T_goal, w):
    """l_f = 1/2 xi(H)^T Q_H xi(H) (eq. 25)."""
    frames = forward_kinematics(robot, q_H)
    return pose_cost(T_goal, frames[:, N_DOF], w["w_term_t"], w["w_term_r"])


def rollout_costs(robot, q0, qd0, T_goal, grid, origin, voxel, U, dt, w):
    """S^(m) = l_f(T_H) + sum_{k<H} l(q_k, x_k, u_k) for every sampled sequence (eq. 28)."""
    U = np.asarray(U, np.float64)
    q, qd = rollout(q0, qd0, U, dt)
    H = U.shape[1]
    S = np.zeros(U.shape[0])
    for k in range(H):
        S += running_cost(robot, q[:, k], qd[:, k], U[:, k], T_goal, grid, origin, voxel, w)
    S += terminal_cost(robot, q[:, H], T_goal, w)
    return S


# ---------------------------------------------------------------------------
# Soft weights and update (eqs. 29-30)
# ---------------------------------------------------------------------------

def soft_weights(S, lam):
    """w^(m) = exp(-(S^(m) - S_min)/lam) / sum_j exp(-(S^(j) - S_min)/lam) (eq. 29).

    Returns (w, S_min, Z) with Z the normaliser; non-finite costs get weight 0 and
    S_min is taken over finite costs.  With no finite cost, w = 0, S_min = nan, Z = 0.
    """
    S = np.asarray(S, np.float64)
    finite = np.isfinite(S)
    if not finite.any():
        return np.zeros_like(S), float("nan"), 0.0
    S_min = float(np.min(S[finite]))
    e = np.where(finite, np.exp(-(np.where(finite, S, S_min) - S_min) / lam), 0.0)
    Z = float(np.sum(e))
    return e / Z, S_min, Z


def update(U_bar, eps, w):
    """U* = Ubar + sum_m w^(m) eps^(m) (eq. 30), over the rollouts with w^(m) > 0.

    Rollouts of weight 0 contribute nothing, also when their disturbance is not
    finite (such rollouts have a non-finite cost and are excluded by eq. 29's reading).
    """
    w = np.asarray(w, np.float64)
    eps = np.asarray(eps, np.float64)
    used = w > 0
    return np.asarray(U_bar, np.float64) + np.tensordot(w[used], eps[used], axes=1)


def plan_step(robot, q0, qd0, T_goal, grid, origin, voxel, noise, U_bar, dt, lam, weights):
    """One pass of Algorithm 1 for given disturbances; returns a dict of float64 results.

    Keys: U_star (H, 7), S (M,), w (M,), S_min, Z, ess (1 / sum w^2), numeric_ok.
    """
    eps = np.asarray(noise, np.float64)
    U = np.asarray(U_bar, np.float64)[None] + eps                      # eq. 27
    S = rollout_costs(robot, q0, qd0, T_goal, grid, origin, voxel, U, dt, weights)
    w, S_min, Z = soft_weights(S, lam)
    ok = bool(np.isfinite(S).any())
    U_star = update(U_bar, eps, w) if ok else np.asarray(U_bar, np.float64).copy()
    ess = float(1.0 / np.sum(w * w)) if ok else 0.0
    return dict(U_star=U_star, S=S, w=w, S_min=S_min, Z=Z, ess=ess, numeric_ok=ok)


# ---------------------------------------------------------------------------
# Receding horizon (Sec. IV-C, last paragraph; Algorithm 1 initialisation)
# ---------------------------------------------------------------------------

def execute_first_control(q0, qd0, U_star, dt):
    """State one control period later when the first control of U* is applied: the
    same semi-implicit Euler step the rollouts use (eq. 7), qd' = qd0 + u*_0 dt, then
    q' = q0 + qd' dt.  Returns (q', qd') in float64."""
    u0 = np.asarray(U_star, np.float64)[0]
    qd1 = np.asarray(qd0, np.float64) + u0 * dt
    q1 = np.asarray(q0, np.float64) + qd1 * dt
    return q1, qd1


def shift_nominal(U_star):
    """Nominal sequence of the next period: u*_0 has been executed, the remaining
    controls move one step forward and the last one is zero (the value Algorithm 1
    starts the sequence from)."""
    U = np.asarray(U_star, np.float64)
    out = np.zeros_like(U)
    out[:-1] = U[1:]
    return out


def merge_shards(results, U_bar, lam):
    """Combine plan_step results of disjoint rollout subsets into the result over their
    union (eqs. 29-30 regrouped): with S_min and Z of each subset, the overall minimum
    is the least S_min, each subset's normaliser is rescaled by exp(-(S_min_g - m)/lam)
    and its weighted disturbance sum (U*_g - Ubar) Z_g likewise.  Returns (U_star, S_min,
    Z); subsets without a finite cost contribute nothing.
    """
    parts = [r for r in results if r["numeric_ok"]]
    U_bar = np.asarray(U_bar, np.float64)
    if not parts:
        return U_bar.copy(), float("nan"), 0.0
    m = min(r["S_min"] for r in parts)
    scale = [np.exp(-(r["S_min"] - m) / lam) for r in parts]
    Z = sum(r["Z"] * c for r, c in zip(parts, scale))
    N = sum((np.asarray(r["U_star"]) - U_bar) * r["Z"] * c for r, c in zip(parts, scale))
    return U_bar + N / Z, float(m), float(Z)


def plan_step_inputs(inp):
    """plan_step on a synth.workload.PlanInputs bundle (robot rounded like the GPU's)."""
    return plan_step(inp.robot.rounded_f32(), inp.q0, inp.qd0, inp.T_goal, inp.grid,
                     inp.origin, inp.voxel, inp.noise, inp.U_bar, inp.dt, inp.lam,
                     inp.weights)
