"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin catches each.

This guards the pins themselves: a pin set that still passes with a dropped
term, a swapped factor, a wrong sign or an off-by-one index is too weak.
"""
import numpy as np
import pytest

from oracle import edt as E
from oracle import ogm as G
from oracle import smpc_oracle as O
from tests import test_oracle_pins as P
from synth import robot as R


def _explicit_euler(q0, qd0, U, dt):
    U = np.asarray(U, np.float64)
    M, H, n = U.shape
    q = np.empty((M, H + 1, n))
    qd = np.empty((M, H + 1, n))
    q[:, 0], qd[:, 0] = q0, qd0
    for k in range(H):
        q[:, k + 1] = q[:, k] + qd[:, k] * dt          # mistake: uses the old velocity
        qd[:, k + 1] = qd[:, k] + U[:, k] * dt
    return q, qd


def _swapped_mdh(alpha, a, theta, d):
    return O.rot_z(theta) @ O.rot_x(alpha) @ O.trans(a, 0.0, 0.0) @ O.trans(0.0, 0.0, d)


def _pose_error_untransposed(T_goal, T_ee):
    Tg = np.asarray(T_goal, np.float64)
    D = np.zeros(T_ee.shape)
    D[..., :3, :3] = Tg[:3, :3] @ T_ee[..., :3, :3]             # mistake: R_g instead of R_g^T
    D[..., :3, 3] = (T_ee[..., :3, 3] - Tg[:3, 3]) @ Tg[:3, :3]
    D[..., 3, 3] = 1.0
    return O.se3_log(D)


def _env_sign_flip(robot, centres, grid, origin, voxel, w_env, d_act):
    total = np.zeros(centres.shape[0])
    for i in range(robot.n_spheres):
        d_env = O.esdf_lookup(grid, origin, voxel, centres[:, i]) - robot.sphere_radius[i]
        total += w_env * np.maximum(0.0, d_env - d_act) ** 2    # mistake: reversed hinge
    return total


def _lookup_no_half_shift(grid, origin, voxel, p):
    return _orig_lookup(grid, origin, voxel, np.asarray(p) - 0.5 * voxel)


def _weights_wrong_sign(S, lam):
    S = np.asarray(S, np.float64)
    e = np.exp((S - S.min()) / lam)
    return e / e.sum(), float(S.min()), float(e.sum())


def _rollout_costs_shifted(robot, q0, qd0, T_goal, grid, origin, voxel, U, dt, w):
    q, qd = O.rollout(q0, qd0, U, dt)
    H = U.shape[1]
    S = np.zeros(U.shape[0])
    for k in range(1, H + 1):                                   # mistake: k = 1..H
        S += O.running_cost(robot, q[:, k], qd[:, k], U[:, k - 1], T_goal, grid, origin, voxel, w)
    S += O.terminal_cost(robot, q[:, H], T_goal, w)
    return S


def _rollout_costs_no_terminal(robot, q0, qd0, T_goal, grid, origin, voxel, U, dt, w):
    q, qd = O.rollout(q0, qd0, U, dt)
    S = np.zeros(U.shape[0])
    for k in range(U.shape[1]):
        S += O.running_cost(robot, q[:, k], qd[:, k], U[:, k], T_goal, grid, origin, voxel, w)
    return S


def _self_no_radius_sum(robot, centres, w_self):
    total = np.zeros(centres.shape[0])
    for i, j in robot.pairs:
        dist = np.linalg.norm(centres[:, i] - centres[:, j], axis=-1)
        total += w_self * np.maximum(0.0, robot.sphere_radius[i] - dist) ** 2   # mistake
    return total


def _fh_1d_no_root_square(f):
    n = f.shape[0]
    out = np.full(n, E.INF, dtype=np.int64)
    roots = [q for q in range(n) if f[q] < E.INF]
    if not roots:
        return out
    v, z = [], []
    for q in roots:
        while True:
            if not v:
                v.append(q), z.append(-np.inf)
                break
            p = v[-1]
            s = (float(f[q]) - float(f[p])) / (2.0 * (q - p))      # mistake: q^2 - p^2 dropped
            if s <= z[-1]:
                v.pop(), z.pop()
                continue
            v.append(q), z.append(s)
            break
    piece = 0
    for p in range(n):
        while piece + 1 < len(v) and z[piece + 1] < p:
            piece += 1
        out[p] = (p - v[piece]) ** 2 + int(f[v[piece]])
    return out


def _signed_distance_no_inside(occ, voxel, transform=None):
    occ = np.asarray(occ, bool)
    d_out = E.edt_separable_fh(occ)
    big = E.no_source_value(occ.shape)
    d_out = np.where(d_out >= E.INF, big, d_out)
    phi = voxel * np.sqrt(d_out.astype(np.float64))                 # mistake: no inside depth
    return phi.astype(np.float32), d_out, np.zeros_like(d_out)


def _pixel_rounded(u):
    return np.round(u)                                  # mistake: nearest pixel corner


def _classify_free_behind(dz, tol, has):
    return has & (np.abs(dz) <= tol), has & (dz > tol)  # mistake: free behind the surface


def _robot_not_reset(L, margin, l_min):
    return L                                            # mistake: robot voxels kept


def _margin_not_applied(x, lo, hi, margin_frac):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return np.maximum(0.0, x - hi) + np.minimum(0.0, x - lo)


def _execute_explicit(q0, qd0, U_star, dt):
    u0 = np.asarray(U_star, np.float64)[0]
    q1 = np.asarray(q0, np.float64) + np.asarray(qd0, np.float64) * dt   # mistake: old velocity
    return q1, np.asarray(qd0, np.float64) + u0 * dt


def _shift_backwards(U_star):
    U = np.asarray(U_star, np.float64)
    out = np.zeros_like(U)
    out[1:] = U[:-1]                                    # mistake: shifted the wrong way
    return out


_orig_lookup = O.esdf_lookup

ROBOT = R.make_robot(0)


def _run_all_pins():
    """Run every pin; return the number that fail."""
    failures = 0
    for name in dir(P):
        if not name.startswith("test_"):
            continue
        fn = getattr(P, name)
        params = []
        code = fn.__code__.co_varnames[:fn.__code__.co_argcount]
        kwargs = {}
        if "robot" in code:
            kwargs["robot"] = ROBOT
        if "theta" in code:
            params = [dict(theta=t) for t in (None, 0.3, 2.0)]
        elif "seed" in code:
            params = [dict(seed=0)]
        else:
            params = [{}]
        for extra in params:
            try:
                fn(**kwargs, **extra)
            except AssertionError:
                failures += 1
            except (ValueError, FloatingPointError, np.linalg.LinAlgError):
                failures += 1
    return failures


MUTANTS = {
    "explicit_euler": ("rollout", _explicit_euler),
    "swapped_mdh_factors": ("mdh_joint_transform", _swapped_mdh),
    "untransposed_goal_rotation": ("pose_error", _pose_error_untransposed),
    "reversed_env_hinge": ("env_collision_cost", _env_sign_flip),
    "lookup_without_half_voxel": ("esdf_lookup", _lookup_no_half_shift),
    "weights_wrong_sign": ("soft_weights", _weights_wrong_sign),
    "running_cost_k_shifted": ("rollout_costs", _rollout_costs_shifted),
    "terminal_cost_dropped": ("rollout_costs", _rollout_costs_no_terminal),
    "self_hinge_missing_radius": ("self_collision_cost", _self_no_radius_sum),
    "limit_margin_dropped": ("limit_violation", _margin_not_applied),
    "fh_intersection_without_squares": ("fh_1d", _fh_1d_no_root_square, E),
    "signed_distance_without_inside": ("signed_distance", _signed_distance_no_inside, E),
    "ogm_pixel_rounded": ("pixel_index", _pixel_rounded, G),
    "ogm_free_behind_surface": ("classify", _classify_free_behind, G),
    "ogm_robot_voxels_not_reset": ("robot_reset", _robot_not_reset, G),
    "executed_control_explicit_euler": ("execute_first_control", _execute_explicit),
    "nominal_shifted_backwards": ("shift_nominal", _shift_backwards),
}


def test_unmutated_oracle_passes_every_pin():
    assert _run_all_pins() == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_is_caught(name, monkeypatch):
    attr, fn, *mod = MUTANTS[name]
    monkeypatch.setattr(mod[0] if mod else O, attr, fn)
    assert _run_all_pins() > 0, f"no pin catches the planted mistake {name!r}"
