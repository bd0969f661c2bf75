"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks one part of the oracle against something other than itself: a
closed form, a hand-derived fixture, a library routine that computes the same
quantity by another route, an invariant, or brute force on a tiny input.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import edt as E
from oracle import ogm as G
from oracle import smpc_oracle as O
from synth import robot as R
from synth import scene as SC
from synth import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_home_pose():
    rows, origins = [], {}
    with open(os.path.join(GOLDEN, "fk_home_pose.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "origin":
                origins[int(parts[1])] = np.array([float(x) for x in parts[2:5]])
            else:
                rows.append([float(x) for x in parts])
    return np.array(rows), origins


@pytest.fixture(scope="module")
def robot():
    return R.make_robot(0)


def zero_weights(**over):
    w = {k: 0.0 for k in W.DEFAULT_WEIGHTS}
    w["limit_margin_frac"] = 0.05
    w.update(over)
    return w


# ---------------------------------------------------------------------------
# Integrator (eq. 7, semi-implicit Euler reading)
# ---------------------------------------------------------------------------

def test_integrator_constant_acceleration_closed_form():
    rng = np.random.default_rng(0)
    q0, qd0, a = rng.normal(size=7), rng.normal(size=7), rng.normal(size=7)
    H, dt = 12, 0.03
    U = np.broadcast_to(a, (3, H, 7)).copy()
    q, qd = O.rollout(q0, qd0, U, dt)
    for k in range(H + 1):
        np.testing.assert_allclose(qd[:, k], np.broadcast_to(qd0 + k * a * dt, (3, 7)), rtol=0,
                                   atol=1e-12)
        expected = q0 + k * dt * qd0 + a * dt * dt * k * (k + 1) / 2
        np.testing.assert_allclose(q[:, k], np.broadcast_to(expected, (3, 7)), rtol=0, atol=1e-12)


def test_integrator_zero_control_is_constant_velocity():
    q0, qd0 = np.arange(7.0), np.linspace(-1, 1, 7)
    q, qd = O.rollout(q0, qd0, np.zeros((2, 9, 7)), 0.05)
    for k in range(10):
        np.testing.assert_allclose(q[:, k], np.broadcast_to(q0 + k * 0.05 * qd0, (2, 7)), atol=1e-13)
        np.testing.assert_allclose(qd[:, k], np.broadcast_to(qd0, (2, 7)), atol=0)


# ---------------------------------------------------------------------------
# Forward kinematics (eq. 6, modified-DH reading)
# ---------------------------------------------------------------------------

def test_fk_home_pose_matches_hand_derivation(robot):
    T7, origins = load_home_pose()
    frames = O.forward_kinematics(robot, np.zeros((1, 7)))
    np.testing.assert_allclose(frames[0, 7], T7, atol=1e-12)
    for i, o in origins.items():
        np.testing.assert_allclose(frames[0, i, :3, 3], o, atol=1e-12)


def test_fk_first_joint_rotates_whole_arm_about_world_z(robot):
    T7, _ = load_home_pose()
    for q1 in (-2.0, 0.3, 1.7):
        q = np.zeros((1, 7))
        q[0, 0] = q1
        expected = np.eye(4)
        expected[:3, :3] = Rotation.from_euler("z", q1).as_matrix()
        np.testing.assert_allclose(O.forward_kinematics(robot, q)[0, 7], expected @ T7,
                                   atol=1e-12)


def test_fk_last_joint_rotates_about_end_effector_z(robot):
    T7, _ = load_home_pose()
    for q7 in (-1.1, 0.8, 2.9):
        q = np.zeros((1, 7))
        q[0, 6] = q7
        rz = np.eye(4)
        rz[:3, :3] = Rotation.from_euler("z", q7).as_matrix()
        np.testing.assert_allclose(O.forward_kinematics(robot, q)[0, 7], T7 @ rz, atol=1e-12)


def test_fk_matches_independent_rotation_library_composition(robot):
    """Compose the same chain with scipy's rotations instead of the oracle's matrices."""
    rng = np.random.default_rng(3)
    q = rng.uniform(-2, 2, size=(5, 7))
    frames = O.forward_kinematics(robot, q)
    for m in range(5):
        Rw, t = np.eye(3), np.zeros(3)
        for i in range(7):
            Rx = Rotation.from_euler("x", robot.alpha[i]).as_matrix()
            t = t + Rw @ (Rx @ np.array([robot.a[i], 0.0, 0.0]))
            Rw = Rw @ Rx @ Rotation.from_euler("z", q[m, i]).as_matrix()
            t = t + Rw @ np.array([0.0, 0.0, robot.d[i]])
        np.testing.assert_allclose(frames[m, 7, :3, :3], Rw, atol=1e-12)
        np.testing.assert_allclose(frames[m, 7, :3, 3], t, atol=1e-12)


def test_fk_link_lengths_do_not_depend_on_configuration(robot):
    rng = np.random.default_rng(4)
    home = O.forward_kinematics(robot, np.zeros((1, 7)))[0, :, :3, 3]
    L0 = np.linalg.norm(np.diff(home, axis=0), axis=1)
    frames = O.forward_kinematics(robot, rng.uniform(-3, 3, size=(20, 7)))
    L = np.linalg.norm(np.diff(frames[:, :, :3, 3], axis=1), axis=2)
    np.testing.assert_allclose(L, np.broadcast_to(L0, L.shape), atol=1e-12)
    # Rotation blocks stay orthonormal.
    Rm = frames[:, 1:, :3, :3]
    np.testing.assert_allclose(Rm @ np.swapaxes(Rm, -1, -2), np.broadcast_to(np.eye(3), Rm.shape),
                               atol=1e-12)


def test_spheres_rigid_on_their_link_and_on_link_segments(robot):
    rng = np.random.default_rng(5)
    q = rng.uniform(-3, 3, size=(10, 7))
    frames = O.forward_kinematics(robot, q)
    p = O.sphere_centres(robot, frames)
    p0 = O.sphere_centres(robot, O.forward_kinematics(robot, np.zeros((1, 7))))[0]
    for link in range(1, 8):
        idx = np.nonzero(robot.sphere_link == link)[0]
        for a_ in idx:
            for b_ in idx:
                d = np.linalg.norm(p[:, a_] - p[:, b_], axis=-1)
                np.testing.assert_allclose(d, np.linalg.norm(p0[a_] - p0[b_]), atol=1e-12)
        if link < 7:
            # The generator places link-i spheres on the segment O_i -> O_{i+1}.
            o_i, o_n = frames[:, link, :3, 3], frames[:, link + 1, :3, 3]
            for j, s in enumerate(idx):
                frac = (j + 0.5) / len(idx)
                np.testing.assert_allclose(p[:, s], o_i + frac * (o_n - o_i), atol=1e-12)


# ---------------------------------------------------------------------------
# Distance lookup (trilinear reading) and the grid generator
# ---------------------------------------------------------------------------

def _linear_grid(n, origin, voxel, g, b):
    centres = SC.voxel_centres(n, origin, voxel)
    return centres @ g + b


def test_trilinear_exact_on_linear_fields():
    rng = np.random.default_rng(6)
    n, voxel = (7, 5, 6), 0.1
    origin = np.array([-0.3, 0.2, 0.05])
    g, b = rng.normal(size=3), 0.7
    grid = _linear_grid(n, origin, voxel, g, b)
    lo = origin + 0.5 * voxel
    hi = origin + (np.array(n) - 0.5) * voxel
    p = rng.uniform(lo, hi, size=(200, 3))
    np.testing.assert_allclose(O.esdf_lookup(grid, origin, voxel, p), p @ g + b, atol=1e-12)


def test_trilinear_reproduces_values_at_voxel_centres():
    rng = np.random.default_rng(7)
    n, voxel, origin = (4, 3, 5), 0.05, np.array([0.1, -0.2, 0.3])
    grid = rng.normal(size=(5, 3, 4))
    centres = SC.voxel_centres(n, origin, voxel)
    vals = O.esdf_lookup(grid, origin, voxel, centres.reshape(-1, 3)).reshape(grid.shape)
    np.testing.assert_allclose(vals, grid, atol=1e-12)


def test_trilinear_clamps_beyond_edges():
    rng = np.random.default_rng(8)
    n, voxel, origin = (4, 4, 4), 0.1, np.zeros(3)
    grid = rng.normal(size=(4, 4, 4))
    inside = np.array([[0.05, 0.2, 0.33]])
    for shift in ([-5.0, 0, 0], [0, 0, 9.0]):
        outside = inside + np.array(shift)
        clamped = np.clip(outside, 0.05, 0.35)
        np.testing.assert_allclose(O.esdf_lookup(grid, origin, voxel, outside),
                                   O.esdf_lookup(grid, origin, voxel, clamped), atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_edt_brute_force_equals_separable_fh_equals_scipy(seed):
    rng = np.random.default_rng(seed)
    occ = rng.uniform(size=(6, 7, 5)) < 0.08
    occ[0, 0, 0] = True
    brute = E.edt_brute_force(occ)
    fh = E.edt_separable_fh(occ)
    np.testing.assert_array_equal(brute, fh)
    np.testing.assert_array_equal(brute, SC.squared_index_edt(occ))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_edt_minplus_equals_brute_force_on_ragged_grids(seed):
    rng = np.random.default_rng(100 + seed)
    for shape in [(5, 9, 4), (1, 1, 7), (6, 1, 1), (3, 8, 1)]:
        occ = rng.uniform(size=shape) < 0.12
        np.testing.assert_array_equal(E.edt_separable_minplus(occ), E.edt_brute_force(occ))


def test_edt_single_source_is_squared_index_distance():
    occ = np.zeros((7, 9, 8), bool)
    c = np.array([2, 5, 3])
    occ[tuple(c)] = True
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in occ.shape], indexing="ij"), -1)
    want = np.sum((idx - c) ** 2, axis=-1)
    for fn in (E.edt_separable_fh, E.edt_separable_minplus):
        np.testing.assert_array_equal(fn(occ), want)


def test_signed_distance_half_space_closed_form():
    """Every voxel with x < 4 occupied: D_out = (x - 3)^2 outside, D_in = (4 - x)^2 inside."""
    occ = np.zeros((3, 5, 10), bool)
    occ[..., :4] = True
    voxel = 0.25
    phi, d_out, d_in = E.signed_distance(occ, voxel)
    x = np.arange(10)
    np.testing.assert_array_equal(d_out[1, 2], np.where(x < 4, 0, (x - 3) ** 2))
    np.testing.assert_array_equal(d_in[1, 2], np.where(x < 4, (4 - x) ** 2, 0))
    np.testing.assert_array_equal(phi[0, 0], np.where(x < 4, -(4 - x), x - 3) * voxel)


def test_signed_distance_empty_and_full_grids():
    shape = (4, 6, 5)
    big = 16 + 36 + 25
    phi, d_out, d_in = E.signed_distance(np.zeros(shape, bool), 0.5)
    assert (d_out == big).all() and (d_in == 0).all()
    assert (phi == np.float32(0.5 * np.sqrt(big))).all()
    phi, d_out, d_in = E.signed_distance(np.ones(shape, bool), 0.5)
    assert (d_out == 0).all() and (d_in == big).all()
    assert (phi == np.float32(-0.5 * np.sqrt(big))).all()


@pytest.mark.parametrize("seed", [0, 1])
def test_signed_distance_equals_library_edt_grid(seed):
    """Both transforms agree bit for bit with the grid built from scipy's exact EDT."""
    rng = np.random.default_rng(seed)
    n = (20, 17, 23)
    voxel = float(np.float32(0.03))
    origin = np.zeros(3)
    prims = [SC.Primitive("box", rng.uniform(0.1, 0.5, 3), rng.uniform(0.05, 0.2, 3), np.zeros(3)),
             SC.Primitive("sphere", rng.uniform(0.1, 0.5, 3), np.array([0.08, 0, 0]), np.zeros(3))]
    occ = SC.occupancy(prims, n, origin, voxel)
    assert 0 < occ.sum() < occ.size
    want = SC.signed_distance_grid(occ, voxel)
    for tr in (E.edt_separable_fh, E.edt_separable_minplus):
        phi, _, _ = E.signed_distance(occ, voxel, transform=tr)
        np.testing.assert_array_equal(phi, want)


def test_fh_1d_against_definition():
    rng = np.random.default_rng(9)
    for _ in range(50):
        f = np.where(rng.uniform(size=17) < 0.3, rng.integers(0, 20, size=17), E.INF)
        out = E.fh_1d(f.astype(np.int64))
        for p in range(17):
            cand = [(p - q) ** 2 + int(f[q]) for q in range(17) if f[q] < E.INF]
            assert out[p] == (min(cand) if cand else E.INF)


def test_signed_grid_values_on_a_box():
    """Free voxels read voxel*sqrt(D) (the paper's EDT, as a distance); occupied read minus depth."""
    n, voxel, origin = (12, 12, 12), 0.1, np.zeros(3)
    box = SC.Primitive("box", np.array([0.6, 0.6, 0.6]), np.array([0.4, 0.4, 0.4]), np.zeros(3))
    occ = SC.occupancy([box], n, origin, voxel)
    phi = SC.signed_distance_grid(occ, voxel)
    # Occupied voxel centres: 0.45..0.75 per axis -> indices 4..7.
    assert occ[4:8, 4:8, 4:8].all() and occ.sum() == 64
    assert phi[5, 5, 9] == pytest.approx(0.2, abs=1e-6)      # two voxels right of the box
    assert phi[5, 5, 8] == pytest.approx(0.1, abs=1e-6)
    assert phi[5, 5, 7] == pytest.approx(-0.1, abs=1e-6)     # surface layer inside
    assert phi[5, 5, 6] == pytest.approx(-0.2, abs=1e-6)
    assert phi[9, 9, 9] == pytest.approx(0.1 * math.sqrt(12), abs=1e-6)


# ---------------------------------------------------------------------------
# Collision terms (eqs. 17-20)
# ---------------------------------------------------------------------------

def test_env_cost_constant_field_closed_form(robot):
    c, w_env, d_act = 0.05, 7.0, 0.03
    grid = np.full((4, 4, 4), c)
    centres = np.random.default_rng(1).uniform(-1, 1, size=(3, robot.n_spheres, 3))
    got = O.env_collision_cost(robot, centres, grid, np.zeros(3), 0.1, w_env, d_act)
    expected = sum(w_env * max(0.0, d_act - c + r) ** 2 for r in robot.sphere_radius)
    np.testing.assert_allclose(got, expected, rtol=1e-13)
    far = np.full((4, 4, 4), 5.0)
    np.testing.assert_array_equal(O.env_collision_cost(robot, centres, far, np.zeros(3), 0.1,
                                                       w_env, d_act), 0.0)


def test_self_cost_two_spheres_closed_form():
    rob = R.make_robot(0, spheres_per_link=1)
    rob.pairs = np.array([[0, 6]], np.int32)
    r0, r6 = rob.sphere_radius[0], rob.sphere_radius[6]
    centres = np.zeros((4, 7, 3))
    seps = np.array([0.0, 0.5 * (r0 + r6), r0 + r6, 2.0])
    centres[:, 6, 0] = seps
    got = O.self_collision_cost(rob, centres, 3.0)
    expected = 3.0 * np.maximum(0.0, r0 + r6 - seps) ** 2
    np.testing.assert_allclose(got, expected, rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# Limits, smoothness, null space (eqs. 21-24)
# ---------------------------------------------------------------------------

def test_limit_violation_hand_values():
    lo, hi = np.array([-1.0]), np.array([3.0])        # range 4, margin 0.1*4 = 0.4
    x = np.array([[-2.0], [-0.6], [0.0], [2.6], [2.9], [4.0]])
    got = O.limit_violation(x, lo, hi, 0.1)[:, 0]
    np.testing.assert_allclose(got, [-1.4, 0.0, 0.0, 0.0, 0.3, 1.4], atol=1e-15)


def test_limit_cost_zero_strictly_inside_and_hand_value(robot):
    w = zero_weights(w_q=2.0, w_qd=3.0, w_qdd=5.0)
    mid = 0.5 * (robot.q_min + robot.q_max)[None]
    zero = np.zeros((1, 7))
    assert O.limit_cost(robot, mid, zero, zero, w)[0] == 0.0
    qd = zero.copy()
    qd[0, 2] = robot.qd_max[2] + 1.0          # 1 + margin beyond the tightened bound
    margin = 0.05 * (robot.qd_max[2] - robot.qd_min[2])
    np.testing.assert_allclose(O.limit_cost(robot, mid, qd, zero, w)[0],
                               3.0 * (1.0 + margin) ** 2, rtol=1e-13)


def test_smoothness_and_null_space_hand_values():
    u = np.array([[1.0, -2.0, 0, 0, 0, 0, 3.0]])
    assert O.smoothness_cost(u, 0.5)[0] == pytest.approx(0.5 * 14.0)
    q = np.array([[1.0, 1, 1, 1, 1, 1, 1]])
    assert O.null_space_cost(q, np.zeros(7), 2.0)[0] == pytest.approx(14.0)


# ---------------------------------------------------------------------------
# SE(3) logarithm and pose error (eqs. 11-16, 25, 33)
# ---------------------------------------------------------------------------

def _random_se3(rng, theta=None):
    if theta is None:
        Rm = Rotation.random(random_state=rng.integers(1 << 31)).as_matrix()
    else:
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        Rm = Rotation.from_rotvec(theta * axis).as_matrix()
    return W.pose_matrix(Rm, rng.uniform(-1, 1, size=3))


def test_log_identity_is_zero():
    v, w = O.se3_log(np.eye(4)[None])
    np.testing.assert_array_equal(v, 0.0)
    np.testing.assert_array_equal(w, 0.0)


@pytest.mark.parametrize("theta", [None, 1e-9, 1e-5, 0.3, 2.0, math.pi - 1e-4, math.pi - 1e-9])
def test_log_against_library_logm_and_expm(theta):
    rng = np.random.default_rng(11)
    for _ in range(5):
        T = _random_se3(rng, theta)
        v, w = O.se3_log(T[None])
        Xi = np.zeros((4, 4))
        Xi[:3, :3] = O.hat(w)[0]
        Xi[:3, 3] = v[0]
        np.testing.assert_allclose(scipy.linalg.expm(Xi), T, atol=1e-10)
        if theta is None or theta < 3.0:
            np.testing.assert_allclose(scipy.linalg.logm(T).real, Xi, atol=1e-8)


def test_log_at_exactly_pi_round_trips():
    for axis in (np.array([1.0, 0, 0]), np.array([0, 0.6, 0.8]), np.array([-1.0, 2.0, 2.0]) / 3):
        T = W.pose_matrix(Rotation.from_rotvec(math.pi * axis).as_matrix(), np.array([0.1, -0.2, 0.3]))
        v, w = O.se3_log(T[None])
        assert np.linalg.norm(w) == pytest.approx(math.pi, abs=1e-9)
        Xi = np.zeros((4, 4))
        Xi[:3, :3] = O.hat(w)[0]
        Xi[:3, 3] = v[0]
        np.testing.assert_allclose(scipy.linalg.expm(Xi), T, atol=1e-9)


def test_rotation_angle_equals_quaternion_orientation_error():
    """|omega| equals e_ori = 2 arccos(|q_g . q|) (eq. 33), computed via quaternions."""
    rng = np.random.default_rng(12)
    for _ in range(50):
        Tg, Te = _random_se3(rng), _random_se3(rng)
        _, w = O.pose_error(Tg, Te[None])
        qg = Rotation.from_matrix(Tg[:3, :3]).as_quat()
        qe = Rotation.from_matrix(Te[:3, :3]).as_quat()
        e_ori = 2 * math.acos(min(1.0, abs(float(np.dot(qg, qe)))))
        assert np.linalg.norm(w) == pytest.approx(e_ori, abs=1e-7)


def test_pure_translation_and_pure_rotation_about_goal_origin():
    rng = np.random.default_rng(13)
    Tg = _random_se3(rng)
    delta = np.array([0.1, -0.3, 0.2])
    Te = Tg.copy()
    Te[:3, 3] = Tg[:3, 3] + delta
    v, w = O.pose_error(Tg, Te[None])
    np.testing.assert_allclose(v[0], Tg[:3, :3].T @ delta, atol=1e-12)
    np.testing.assert_allclose(w[0], 0.0, atol=1e-12)
    Te = Tg.copy()
    Te[:3, :3] = Tg[:3, :3] @ Rotation.from_rotvec([0.2, 0.5, -0.1]).as_matrix()
    v, w = O.pose_error(Tg, Te[None])
    np.testing.assert_allclose(v[0], 0.0, atol=1e-12)
    np.testing.assert_allclose(w[0], [0.2, 0.5, -0.1], atol=1e-12)


def test_pose_cost_weights_translation_and_rotation_blocks():
    rng = np.random.default_rng(14)
    Tg, Te = _random_se3(rng), _random_se3(rng)
    v, w = O.pose_error(Tg, Te[None])
    got = O.pose_cost(Tg, Te[None], 3.0, 0.25)[0]
    assert got == pytest.approx(0.5 * (3.0 * v[0] @ v[0] + 0.25 * w[0] @ w[0]), rel=1e-14)


# ---------------------------------------------------------------------------
# Soft weights and update (eqs. 29-30)
# ---------------------------------------------------------------------------

def test_weights_normalised_shift_invariant_and_argmin_largest():
    rng = np.random.default_rng(15)
    S = rng.uniform(0, 5, size=100)
    w, S_min, Z = O.soft_weights(S, 0.7)
    assert np.all(w >= 0) and w.sum() == pytest.approx(1.0, abs=1e-14)
    assert S_min == S.min() and Z >= 1.0
    assert np.argmax(w) == np.argmin(S)
    w2, _, _ = O.soft_weights(S + 123.0, 0.7)
    np.testing.assert_allclose(w2, w, rtol=1e-12)
    # Closed form on two costs: w = 1/(1 + e^{-d/lam}) for the better one.
    w3, _, _ = O.soft_weights(np.array([1.0, 1.5]), 0.5)
    assert w3[0] == pytest.approx(1.0 / (1.0 + math.exp(-1.0)), rel=1e-14)


def test_weights_temperature_limits():
    S = np.array([3.0, 1.0, 2.0, 1.2])
    w0, _, _ = O.soft_weights(S, 1e-6)
    np.testing.assert_allclose(w0, [0, 1, 0, 0], atol=1e-12)
    winf, _, _ = O.soft_weights(S, 1e9)
    np.testing.assert_allclose(winf, 0.25, atol=1e-9)


def test_weights_ignore_non_finite_costs():
    w, S_min, _ = O.soft_weights(np.array([np.nan, 2.0, np.inf, 1.0]), 1.0)
    assert w[0] == 0 and w[2] == 0 and S_min == 1.0
    assert w[1] + w[3] == pytest.approx(1.0)
    w, S_min, Z = O.soft_weights(np.array([np.nan, np.inf]), 1.0)
    assert np.all(w == 0) and math.isnan(S_min) and Z == 0.0


def test_update_special_cases():
    rng = np.random.default_rng(16)
    Ubar = rng.normal(size=(5, 7))
    eps = rng.normal(size=(9, 5, 7))
    w = rng.uniform(size=9)
    w /= w.sum()
    np.testing.assert_allclose(O.update(Ubar, np.zeros_like(eps), w), Ubar)
    same = np.broadcast_to(eps[0], eps.shape)
    np.testing.assert_allclose(O.update(Ubar, same, w), Ubar + eps[0], atol=1e-14)
    onehot = np.zeros(9)
    onehot[4] = 1
    np.testing.assert_allclose(O.update(Ubar, eps, onehot), Ubar + eps[4])


# ---------------------------------------------------------------------------
# Whole plan step on scenarios with closed-form costs (eq. 28, Algorithm 1)
# ---------------------------------------------------------------------------

def _static_step(robot, T_goal, grid, w, H=6, K=3, q0=None, noise=None, dt=0.05):
    q0 = np.zeros(7) if q0 is None else q0
    noise = np.zeros((K, H, 7)) if noise is None else noise
    return O.plan_step(robot, q0, np.zeros(7), T_goal, grid, np.zeros(3) - 2.0, 0.5, noise,
                       np.zeros((H, 7)), dt, 1.0, w)


def test_composite_env_term_counted_on_k_0_to_H_minus_1(robot):
    T7, _ = load_home_pose()
    c, H = 0.04, 6
    grid = np.full((8, 8, 8), c)
    w = zero_weights(w_env=2.0, d_act=0.03, w_pose_t=1.0, w_pose_r=1.0, w_term_t=1.0,
                     w_term_r=1.0)
    out = _static_step(robot, T7, grid, w, H=H)
    per_step = sum(2.0 * max(0.0, 0.03 - c + r) ** 2 for r in robot.sphere_radius)
    np.testing.assert_allclose(out["S"], H * per_step, rtol=1e-12)


def test_composite_pose_running_and_terminal_weights(robot):
    T7, _ = load_home_pose()
    shift = np.array([0.05, -0.02, 0.03])
    Tg = T7.copy()
    Tg[:3, 3] -= T7[:3, :3] @ shift          # goal displaced so that t_Delta = shift
    grid = np.full((8, 8, 8), 9.0)
    H = 5
    w = zero_weights(w_pose_t=4.0, w_pose_r=1.0, w_term_t=10.0, w_term_r=1.0)
    out = _static_step(robot, Tg, grid, w, H=H)
    n2 = float(shift @ shift)
    np.testing.assert_allclose(out["S"], H * 0.5 * 4.0 * n2 + 0.5 * 10.0 * n2, rtol=1e-12)


def test_composite_self_term_on_home_pose():
    # One sphere at each frame origin: at q = 0, O_5 and O_7 are 0.088 m apart.
    rob = R.make_robot(0, spheres_per_link=1)
    rob.sphere_center = np.zeros((7, 3))
    rob.sphere_radius = np.array([0.01, 0.01, 0.01, 0.01, 0.06, 0.01, 0.05])
    rob.pairs = np.array([[4, 6], [0, 2]], np.int32)    # links 5-7 overlap; 1-3 do not
    T7, _ = load_home_pose()
    H = 4
    out = _static_step(rob, T7, np.full((8, 8, 8), 9.0), zero_weights(w_self=3.0), H=H)
    np.testing.assert_allclose(out["S"], H * 3.0 * (0.11 - 0.088) ** 2, rtol=1e-10)


def test_composite_smoothness_and_acceleration_limit_with_constant_noise(robot):
    T7, _ = load_home_pose()
    H, K = 7, 2
    a = np.array([1.0, -20.0, 0.5, 0, 0, 0, 2.0])
    noise = np.broadcast_to(a, (K, H, 7)).copy()
    w = zero_weights(w_smooth=0.3, w_qdd=2.0)
    out = _static_step(robot, T7, np.full((8, 8, 8), 9.0), w, H=H, K=K, noise=noise)
    dqdd = O.limit_violation(a, robot.qdd_min, robot.qdd_max, 0.05)
    per_step = 0.3 * float(a @ a) + 2.0 * float(dqdd @ dqdd)
    np.testing.assert_allclose(out["S"], H * per_step, rtol=1e-12)
    np.testing.assert_allclose(out["U_star"], a[None].repeat(H, 0), atol=1e-14)


def test_composite_null_space_and_position_limit_static(robot):
    T7, _ = load_home_pose()
    H = 3
    q0 = np.zeros(7)
    q0[3] = 0.5       # joint 4 upper limit is -0.0698: violated
    w = zero_weights(w_ns=0.7, w_q=1.5)
    out = _static_step(robot, T7, np.full((8, 8, 8), 9.0), w, H=H, q0=q0)
    dq = O.limit_violation(q0, robot.q_min, robot.q_max, 0.05)
    per_step = 0.7 * float((q0 - robot.q_ref) @ (q0 - robot.q_ref)) + 1.5 * float(dq @ dq)
    np.testing.assert_allclose(out["S"], H * per_step, rtol=1e-12)


def test_composite_velocity_limit_under_constant_acceleration(robot):
    """qd_k = k a dt under constant a from rest; the qd term sums k = 0..H-1."""
    T7, _ = load_home_pose()
    H, dt = 6, 0.1
    a = np.array([0, 0, 0, 0, 0, 8.0, 0])
    w = zero_weights(w_qd=1.0)
    out = _static_step(robot, T7, np.full((8, 8, 8), 9.0), w, H=H, noise=a[None, None].repeat(H, 1),
                       K=1, dt=dt)
    total = 0.0
    for k in range(H):
        d = O.limit_violation(k * a * dt, robot.qd_min, robot.qd_max, 0.05)
        total += float(d @ d)
    np.testing.assert_allclose(out["S"], total, rtol=1e-12)
    assert total > 0


def test_lambda_to_zero_selects_argmin_rollout():
    inp = W.tiny()
    out = O.plan_step(inp.robot, inp.q0, inp.qd0, inp.T_goal, inp.grid, inp.origin, inp.voxel,
                      inp.noise, inp.U_bar, inp.dt, 1e-7, inp.weights)
    m = int(np.argmin(out["S"]))
    np.testing.assert_allclose(out["U_star"], inp.U_bar + inp.noise[m], atol=1e-12)
    assert out["ess"] == pytest.approx(1.0)


def test_lookup_of_non_finite_point_is_nan():
    grid = np.zeros((3, 3, 3))
    p = np.array([[0.1, 0.1, 0.1], [np.nan, 0.1, 0.1], [0.1, np.inf, 0.1]])
    got = O.esdf_lookup(grid, np.zeros(3), 0.1, p)
    assert got[0] == 0.0 and np.isnan(got[1]) and np.isnan(got[2])


def test_update_excludes_zero_weight_rollouts_even_with_non_finite_noise():
    Ubar = np.zeros((2, 7))
    eps = np.ones((3, 2, 7))
    eps[1] = np.nan
    w = np.array([0.25, 0.0, 0.75])
    np.testing.assert_allclose(O.update(Ubar, eps, w), np.ones((2, 7)))


# ---------------------------------------------------------------------------
# Occupancy mapping by voxel projection (Sec. III-A) and the robot mask (Remark 2)
# ---------------------------------------------------------------------------

OGM_PRM = dict(tol=0.025, l_hit=0.85, l_miss=-0.4, l_min=-2.0, l_max=3.5, l_occ=0.0,
               robot_pad=0.01)


def _axis_camera():
    from synth import camera as C
    T = np.eye(4)
    T[:3, :3] = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])  # optical axis = +x
    T[:3, 3] = [0.0, 0.0, 0.5]
    return C.Camera(fx=100.0, fy=100.0, cx=40.0, cy=30.0, width=80, height=60,
                    T_wc=T.astype(np.float32), min_depth=0.1, max_depth=4.0)


def _wall_scene():
    wall = SC.Primitive("box", np.array([1.1, 0.0, 0.5]), np.array([0.2, 4.0, 4.0]), np.zeros(3))
    return [wall]


def test_ogm_wall_closed_form_along_the_optical_axis():
    """Wall face at x = 1.0 (depth 1.0 exactly): voxel centres at x = 0.02 + 0.04 i on the
    axis are free up to 0.94, occupied at 0.98 and 1.02 (|x - 1| <= 0.025), unchanged behind."""
    from synth import camera as C
    cam = _axis_camera()
    depth = C.render_depth(cam, _wall_scene())
    assert np.all(depth == np.float32(1.0))
    origin = np.array([0.0, -0.02, 0.48])
    L0 = np.zeros((1, 1, 40), np.float32)
    L, occ, _ = G.ogm_update(L0, depth, cam, origin, 0.04, OGM_PRM)
    x = 0.02 + 0.04 * np.arange(40)
    want = np.where(np.abs(x - 1.0) <= 0.025, 0.85, np.where(x < 1.0 - 0.025, -0.4, 0.0))
    want[x < 0.1] = -0.4          # in front of the wall at any depth > 0
    np.testing.assert_array_equal(L[0, 0], want.astype(np.float32))
    np.testing.assert_array_equal(occ[0, 0], want > 0)


def test_ogm_voxels_out_of_view_unchanged():
    from synth import camera as C
    cam = _axis_camera()
    depth = C.render_depth(cam, _wall_scene())
    origin = np.array([-1.0, -3.0, 0.48])
    L0 = np.full((1, 3, 4), 0.3, np.float32)
    L, _, _ = G.ogm_update(L0, depth, cam, origin, 0.5, OGM_PRM)
    # x centres -0.75 (behind the camera), -0.25, 0.25, 0.75; y centres -2.75 .. -1.75:
    # far outside the 40-pixel half width at these depths except none
    np.testing.assert_array_equal(L, L0)


def test_ogm_log_odds_saturate():
    from synth import camera as C
    cam = _axis_camera()
    depth = C.render_depth(cam, _wall_scene())
    origin = np.array([0.0, -0.02, 0.48])
    L = np.zeros((1, 1, 40), np.float32)
    for _ in range(12):
        L, occ, _ = G.ogm_update(L, depth, cam, origin, 0.04, OGM_PRM)
    x = 0.02 + 0.04 * np.arange(40)
    assert np.all(L[0, 0][np.abs(x - 1.0) <= 0.025] == np.float32(3.5))
    assert np.all(L[0, 0][(x < 0.975) & (x > 0.1)] == np.float32(-2.0))


def test_ogm_robot_mask_discards_returns_and_clears_voxels():
    """A robot sphere at (0.6, 0, 0.5), r = 0.1, in front of the wall: its returns are
    discarded (no voxel occupied near it, none cleared behind it along its pixels) and
    the voxels inside it are set to l_min."""
    from synth import camera as C
    cam = _axis_camera()
    c, r = np.array([[0.6, 0.0, 0.5]]), np.array([0.1])
    depth = C.render_depth(cam, _wall_scene(), spheres=c, radii=r)
    cleaned, _ = G.clean_depth(depth, cam, c, r + OGM_PRM["robot_pad"])
    on_robot = (depth > 0) & (depth < 0.9)
    assert on_robot.sum() > 100
    assert np.all(cleaned[on_robot] == 0) and np.all(cleaned[~on_robot] == depth[~on_robot])
    origin = np.array([0.3, -0.3, 0.2])
    vox = 0.03
    L0 = np.full((20, 20, 30), 0.5, np.float32)
    L, occ, _ = G.ogm_update(L0, depth, cam, origin, vox, OGM_PRM, c, r)
    zi, yi, xi = np.meshgrid(*[np.arange(n) for n in L.shape], indexing="ij")
    pw = np.stack([origin[0] + (xi + 0.5) * vox, origin[1] + (yi + 0.5) * vox,
                   origin[2] + (zi + 0.5) * vox], -1)
    inside = np.linalg.norm(pw - c[0], axis=-1) <= r[0] + OGM_PRM["robot_pad"]
    assert inside.sum() > 100 and np.all(L[inside] == np.float32(-2.0))
    # from an unknown map (log-odds 0), nothing near the robot's surface becomes occupied
    near_surface = (np.abs(np.linalg.norm(pw - c[0], axis=-1) - r[0]) < 0.05) & ~inside
    L1, occ1, _ = G.ogm_update(np.zeros_like(L0), depth, cam, origin, vox, OGM_PRM, c, r)
    assert not occ1[near_surface].any()
    # without the mask the sphere's surface is mapped as an obstacle
    _, occ_nomask, _ = G.ogm_update(np.zeros_like(L0), depth, cam, origin, vox, OGM_PRM)
    assert occ_nomask[near_surface].sum() >= 5


def test_ogm_pixel_is_the_square_containing_the_projection():
    """Depth 1.0 left of pixel column 40, 2.0 from it on; a voxel at x = 1.5 projecting to
    u = 39.7 reads the left pixel (behind its surface: unchanged), not the right one."""
    cam = _axis_camera()
    depth = np.where(np.arange(80)[None, :] < 40, 1.0, 2.0) * np.ones((60, 1))
    depth = depth.astype(np.float32)
    y = 0.0045                                   # camera x = -y: u = 100 * 0.0045 / 1.5 ...
    origin = np.array([1.5 - 0.005, y - 0.005, 0.5 - 0.005])
    L, _, _ = G.ogm_update(np.zeros((1, 1, 1), np.float32), depth, cam, origin, 0.01, OGM_PRM)
    assert L[0, 0, 0] == 0.0                     # u = 40 - 0.3 -> pixel 39 (depth 1.0)
    origin2 = origin + np.array([0.0, -0.009, 0.0])   # u = 40 + 0.3 -> pixel 40 (depth 2.0)
    L2, _, _ = G.ogm_update(np.zeros((1, 1, 1), np.float32), depth, cam, origin2, 0.01, OGM_PRM)
    assert L2[0, 0, 0] == np.float32(-0.4)


def _prim_sdf(prims, p):
    d = np.full(p.shape[:-1], np.inf)
    for q in prims:
        if q.kind == "box":
            e = np.abs(p - q.center) - 0.5 * q.size
            out = np.linalg.norm(np.maximum(e, 0.0), axis=-1)
            d = np.minimum(d, out + np.minimum(e.max(axis=-1), 0.0))
        else:
            d = np.minimum(d, np.linalg.norm(p - q.center, axis=-1) - q.size[0])
    return d


def test_ogm_occupied_voxels_lie_on_surfaces():
    """Occupied voxel centres are within tol plus half a voxel and a pixel footprint of a
    primitive surface (analytic signed distances, independent of the projection)."""
    from synth import camera as C
    from synth import workload as W
    sc = W.ReactiveScenario(seed=3)
    cam = C.default_camera(160, 120)
    depth = C.render_depth(cam, sc.prims)
    vox = 0.04
    L, occ, _ = G.ogm_update(np.zeros((40, 50, 50), np.float32), depth, cam, sc.origin, vox,
                            OGM_PRM)
    assert occ.sum() > 50
    zi, yi, xi = np.nonzero(occ)
    pw = np.stack([sc.origin[0] + (xi + 0.5) * vox, sc.origin[1] + (yi + 0.5) * vox,
                   sc.origin[2] + (zi + 0.5) * vox], -1)
    sdf = _prim_sdf(sc.prims, pw)
    footprint = 3.0 / cam.fx * 2.5        # a pixel's width at the farthest depth, generous
    assert np.all(np.abs(sdf) <= OGM_PRM["tol"] + vox * np.sqrt(3) + footprint), float(np.abs(sdf).max())


# ---------------------------------------------------------------------------
# Receding horizon (Sec. IV-C, last paragraph): execute u*_0, shift the rest
# ---------------------------------------------------------------------------

def test_executing_a_constant_control_follows_the_closed_form():
    """n periods that each execute the same control a move the arm as the closed
    form of constant acceleration under the semi-implicit Euler reading:
    qd_n = qd0 + n a dt, q_n = q0 + n dt qd0 + a dt^2 n (n + 1) / 2."""
    rng = np.random.default_rng(5)
    q0, qd0, a = rng.normal(size=7), rng.normal(size=7), rng.normal(size=7)
    dt = 0.02
    q, qd = q0.copy(), qd0.copy()
    for n in range(1, 31):
        q, qd = O.execute_first_control(q, qd, np.vstack([a, rng.normal(size=(3, 7))]), dt)
        np.testing.assert_allclose(qd, qd0 + n * a * dt, rtol=0, atol=1e-12)
        np.testing.assert_allclose(q, q0 + n * dt * qd0 + a * dt * dt * n * (n + 1) / 2,
                                   rtol=0, atol=1e-12)


def test_zero_disturbance_loop_replays_the_nominal_sequence_then_zeros():
    """With every disturbance zero the update returns U* = Ubar (eq. 30), so the
    receding-horizon loop executes the first nominal sequence control by control and
    then zero controls (the shifted-in tail): after n periods the state is state n of
    the open-loop rollout of [Ubar_0, 0, 0, ...]."""
    rng = np.random.default_rng(6)
    H, dt, n_periods = 5, 0.05, 9
    U0 = rng.normal(size=(H, 7))
    q0, qd0 = rng.normal(size=7), rng.normal(size=7)
    ref_q, ref_qd = O.rollout(q0, qd0, np.vstack([U0, np.zeros((n_periods - H, 7))])[None], dt)
    U, q, qd = U0.copy(), q0.copy(), qd0.copy()
    for n in range(1, n_periods + 1):
        U_star = O.update(U, np.zeros((4, H, 7)), np.full(4, 0.25))
        q, qd = O.execute_first_control(q, qd, U_star, dt)
        U = O.shift_nominal(U_star)
        np.testing.assert_allclose(q, ref_q[0, n], rtol=0, atol=1e-12)
        np.testing.assert_allclose(qd, ref_qd[0, n], rtol=0, atol=1e-12)
    assert np.all(U == 0.0)
    assert O.shift_nominal(np.ones((1, 7))).tolist() == [[0.0] * 7]


def test_merging_rollout_shards_equals_the_whole_plan_step():
    """Splitting the K rollouts into disjoint subsets and merging their (S_min, Z, U*)
    gives the plan step over all of them (eqs. 29-30 are sums over rollouts)."""
    from synth import workload as W
    inp = W.make_inputs(21, K=90, H=8, dt=0.05, n=24, voxel=0.05, n_boxes=4, n_spheres=2)
    full = O.plan_step_inputs(inp)
    parts = []
    for lo, hi in ((0, 7), (7, 50), (50, 90)):
        parts.append(O.plan_step(inp.robot.rounded_f32(), inp.q0, inp.qd0, inp.T_goal, inp.grid,
                                 inp.origin, inp.voxel, inp.noise[lo:hi], inp.U_bar, inp.dt,
                                 inp.lam, inp.weights))
    U, m, Z = O.merge_shards(parts, inp.U_bar, inp.lam)
    np.testing.assert_allclose(U, full["U_star"], rtol=0, atol=1e-12)
    assert m == full["S_min"]
    assert Z == pytest.approx(full["Z"], rel=1e-12)
