"""Seeded robot-description generator for the 7-DoF arm used by every workload.

This module only builds *inputs*: a modified-DH table, joint limits, a collision
sphere model and a self-collision pair list.  It holds none of the plan step's
arithmetic and is shared, unchanged, by the oracle tests, the GPU tests and the
benchmark.

Sources
-------
* Kinematic table: the 7-DoF arm of the workloads (modified DH, a/d/alpha), which
  is the Franka Panda geometry.  The paper's robot model is generic (Sec. IV-A,
  eq. (6)); it names no DH table.
* Limits: the paper only names the admissible set (Sec. IV-A, eq. (10)) and the
  tightened interval (Sec. IV-B-3, eq. (21)); the numeric bounds below are the
  public Panda datasheet values.
* Spheres: the paper approximates each link by spheres (Sec. IV-B-2, Fig. 2)
  without numbers.  Here link i carries ``spheres_per_link`` spheres evenly
  spaced along the segment from frame origin O_i to O_{i+1}; link 7 uses the
  segment from O_7 along its own z axis.  Radii are drawn U[r_lo, r_hi].
* Pairs: the paper takes "pairs that may come into contact" (Sec. IV-B-2,
  eq. (18)); here every sphere pair whose links differ by at least
  ``min_link_gap``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_DOF = 7

# Modified-DH (Craig) table: joint i uses entry i of each array (1-based joint
# numbering maps to index i-1).
PANDA_A = (0.0, 0.0, 0.0, 0.0825, -0.0825, 0.0, 0.088)
PANDA_D = (0.333, 0.0, 0.316, 0.0, 0.384, 0.0, 0.0)
PANDA_ALPHA = (0.0, -math.pi / 2, math.pi / 2, math.pi / 2, -math.pi / 2, math.pi / 2,
               math.pi / 2)

PANDA_Q_MIN = (-2.8973, -1.7628, -2.8973, -3.0718, -2.8973, -0.0175, -2.8973)
PANDA_Q_MAX = (2.8973, 1.7628, 2.8973, -0.0698, 2.8973, 3.7525, 2.8973)
PANDA_QD_MAX = (2.175, 2.175, 2.175, 2.175, 2.61, 2.61, 2.61)
PANDA_QDD_MAX = (15.0, 7.5, 10.0, 12.5, 15.0, 20.0, 20.0)


@dataclasses.dataclass
class Robot:
    """A 7-DoF arm with a sphere collision model (all arrays float64)."""

    a: np.ndarray            # (7,) metres
    d: np.ndarray            # (7,) metres
    alpha: np.ndarray        # (7,) radians
    q_min: np.ndarray        # (7,)
    q_max: np.ndarray
    qd_min: np.ndarray
    qd_max: np.ndarray
    qdd_min: np.ndarray
    qdd_max: np.ndarray
    q_ref: np.ndarray        # (7,) null-space reference posture
    sphere_link: np.ndarray  # (n_s,) int, link index 1..7 the sphere is rigidly attached to
    sphere_center: np.ndarray  # (n_s, 3) centre in the frame of its link, metres
    sphere_radius: np.ndarray  # (n_s,) metres
    pairs: np.ndarray        # (n_p, 2) int, sphere index pairs (i < j)

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_radius.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.pairs.shape[0])

    def rounded_f32(self) -> "Robot":
        """Copy with every length/limit rounded to float32 (alpha kept as given).

        The GPU library stores lengths, limits and sphere data in float32 and
        takes cos/sin of alpha in double; giving the oracle this copy makes both
        sides consume the same numbers.
        """
        f = lambda x: np.asarray(x, np.float32).astype(np.float64)  # noqa: E731
        return dataclasses.replace(
            self, a=f(self.a), d=f(self.d), alpha=np.array(self.alpha, np.float64),
            q_min=f(self.q_min), q_max=f(self.q_max), qd_min=f(self.qd_min),
            qd_max=f(self.qd_max), qdd_min=f(self.qdd_min), qdd_max=f(self.qdd_max),
            q_ref=f(self.q_ref), sphere_center=f(self.sphere_center),
            sphere_radius=f(self.sphere_radius))


def _next_origin_in_frame(a_next: float, d_next: float, alpha_next: float) -> np.ndarray:
    """Origin of frame i+1 expressed in frame i for a modified-DH joint.

    With RotX(alpha) TransX(a) RotZ(theta) TransZ(d) the origin of the next frame
    does not depend on theta: it sits at (a, -sin(alpha) d, cos(alpha) d).
    """
    return np.array([a_next, -math.sin(alpha_next) * d_next, math.cos(alpha_next) * d_next])


def make_robot(seed: int = 0, spheres_per_link: int = 4, r_lo: float = 0.04,
               r_hi: float = 0.08, tool_length: float = 0.1, min_link_gap: int = 2,
               a=PANDA_A, d=PANDA_D, alpha=PANDA_ALPHA) -> Robot:
    """Build the arm, its sphere model and its self-collision pairs from a seed."""
    rng = np.random.default_rng(seed)
    a = np.asarray(a, np.float64)
    d = np.asarray(d, np.float64)
    alpha = np.asarray(alpha, np.float64)
    q_min = np.asarray(PANDA_Q_MIN, np.float64)
    q_max = np.asarray(PANDA_Q_MAX, np.float64)
    qd_max = np.asarray(PANDA_QD_MAX, np.float64)
    qdd_max = np.asarray(PANDA_QDD_MAX, np.float64)

    links, centres = [], []
    for link in range(1, N_DOF + 1):
        if link < N_DOF:
            seg_end = _next_origin_in_frame(a[link], d[link], alpha[link])
        else:
            seg_end = np.array([0.0, 0.0, tool_length])
        for j in range(spheres_per_link):
            frac = (j + 0.5) / spheres_per_link
            links.append(link)
            centres.append(frac * seg_end)
    n_s = len(links)
    radius = rng.uniform(r_lo, r_hi, size=n_s)
    sphere_link = np.asarray(links, np.int32)
    pairs = [(i, j) for i in range(n_s) for j in range(i + 1, n_s)
             if abs(int(sphere_link[i]) - int(sphere_link[j])) >= min_link_gap]
    return Robot(a=a, d=d, alpha=alpha, q_min=q_min, q_max=q_max, qd_min=-qd_max,
                 qd_max=qd_max, qdd_min=-qdd_max, qdd_max=qdd_max,
                 q_ref=0.5 * (q_min + q_max), sphere_link=sphere_link,
                 sphere_center=np.asarray(centres, np.float64), sphere_radius=radius,
                 pairs=np.asarray(pairs, np.int32).reshape(-1, 2))


def random_joint_config(rng: np.random.Generator, robot: Robot, shrink: float = 0.0) -> np.ndarray:
    """Uniform joint configuration inside the (optionally shrunk) position limits."""
    lo, hi = robot.q_min, robot.q_max
    span = hi - lo
    return rng.uniform(lo + shrink * span, hi - shrink * span)
