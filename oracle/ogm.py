"""Occupancy update by voxel projection (Sec. III-A) with the robot mask (Remark 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Geometry in float64, the log-odds layer in float32 (the precision it is stored
in).  Readings where the paper leaves the details open:

* a voxel is represented by its centre; its projected depth is the z coordinate of
  the centre in the camera frame, and it reads the pixel whose square contains the
  projection (u = fx x / z + cx, pixel floor(u), likewise v);
* classification against the measured depth d of that pixel with a tolerance tol:
  |z - d| <= tol occupied (log-odds + l_hit), z < d - tol free (+ l_miss), otherwise
  unknown (unchanged); voxels behind the camera, outside the image or on a pixel
  without a return are unknown; the log-odds is clamped to [l_min, l_max] and a
  voxel is occupied when it exceeds l_occ;
* robot mask: the sphere model is padded by robot_pad (returns from the robot lie
  on its sphere surfaces, where "inside" would be decided by rounding); a return
  whose back-projected point (pixel centre, depth d) lies in a padded sphere
  (|p - c| <= r + pad) is discarded before the update, and after it every voxel
  whose centre lies in a padded sphere is set to l_min (free: the robot occupies it).

Decisions that turn floating-point values into integers (pixel index, tolerance
band, sphere membership) are also returned with their margin, so that a test can
tell a decision the float32 kernel may legitimately take the other way.
"""
from __future__ import annotations

import numpy as np


def back_project(depth, fx, fy, cx, cy, T_wc):
    """World points (h, w, 3) of the pixel centres at their depths."""
    h, w = depth.shape
    v, u = np.mgrid[0:h, 0:w]
    d = depth.astype(np.float64)
    pc = np.stack([(u + 0.5 - cx) * d / fx, (v + 0.5 - cy) * d / fy, d], axis=-1)
    T = np.asarray(T_wc, np.float64)
    return pc @ T[:3, :3].T + T[:3, 3]


def sphere_margin(points, centres, radii):
    """min over spheres of |p - c| - r (negative inside some sphere); +inf without spheres."""
    if centres is None or len(centres) == 0:
        return np.full(points.shape[:-1], np.inf)
    c = np.asarray(centres, np.float64)
    r = np.asarray(radii, np.float64)
    m = np.full(points.shape[:-1], np.inf)
    for i in range(len(c)):
        m = np.minimum(m, np.linalg.norm(points - c[i], axis=-1) - r[i])
    return m


def clean_depth(depth, cam, centres=None, radii=None):
    """Valid returns (min_depth <= d <= max_depth) not inside a robot sphere; 0 elsewhere.
    Returns (cleaned depth float32, margin of the sphere test per pixel)."""
    d = depth.astype(np.float64)
    valid = np.isfinite(d) & (d >= cam.min_depth) & (d <= cam.max_depth)
    pts = back_project(np.where(valid, d, 0.0), cam.fx, cam.fy, cam.cx, cam.cy, cam.T_wc)
    m = sphere_margin(pts, centres, radii)
    keep = valid & (m > 0.0)
    return np.where(keep, depth, 0.0).astype(np.float32), np.where(valid, m, np.inf)


def pixel_index(u):
    """Index of the pixel whose square [i, i + 1) contains the coordinate u."""
    return np.floor(u)


def classify(dz, tol, has):
    """(occupied, free) masks from dz = z - d: within the band, or in front of it."""
    return has & (np.abs(dz) <= tol), has & (dz < -tol)


def robot_reset(L, margin, l_min):
    """Voxels whose centre lies in a (padded) robot sphere are set to l_min."""
    return np.where(margin <= 0.0, l_min, L)


def ogm_update(log_odds, depth, cam, origin, voxel, prm, centres=None, radii=None):
    """One update of the float32 log-odds grid (nz, ny, nx) from one depth image.

    prm: dict with tol, l_hit, l_miss, l_min, l_max, l_occ and optionally robot_pad (0).
    Returns (new log-odds float32, occupancy bool, ambiguity margin per voxel): the
    margin is the smallest distance of any decision taken for the voxel to its
    threshold (metres for depth bands and spheres, pixels for pixel borders).
    """
    L = np.asarray(log_odds, np.float32)
    nz, ny, nx = L.shape
    if radii is not None:
        radii = np.asarray(radii, np.float64) + prm.get("robot_pad", 0.0)
    dclean, pix_margin = clean_depth(depth, cam, centres, radii)
    z_i, y_i, x_i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pw = np.stack([origin[0] + (x_i + 0.5) * voxel, origin[1] + (y_i + 0.5) * voxel,
                   origin[2] + (z_i + 0.5) * voxel], axis=-1).astype(np.float64)
    T = np.asarray(cam.T_wc, np.float64)
    pc = (pw - T[:3, 3]) @ T[:3, :3]
    x, y, z = pc[..., 0], pc[..., 1], pc[..., 2]
    in_front = z > 0.0
    zs = np.where(in_front, z, 1.0)
    u = cam.fx * x / zs + cam.cx
    v = cam.fy * y / zs + cam.cy
    iu, iv = pixel_index(u), pixel_index(v)
    inside = in_front & (iu >= 0) & (iu < cam.width) & (iv >= 0) & (iv < cam.height)
    iu_c = np.clip(iu, 0, cam.width - 1).astype(int)
    iv_c = np.clip(iv, 0, cam.height - 1).astype(int)
    d = np.where(inside, dclean[iv_c, iu_c].astype(np.float64), 0.0)
    has = inside & (d > 0.0)
    dz = z - d
    occ_hit, free = classify(dz, prm["tol"], has)
    lo, hi = np.float32(prm["l_min"]), np.float32(prm["l_max"])
    Ln = L.copy()
    Ln = np.where(occ_hit, np.clip(L + np.float32(prm["l_hit"]), lo, hi), Ln)
    Ln = np.where(free, np.clip(L + np.float32(prm["l_miss"]), lo, hi), Ln)
    m_robot = sphere_margin(pw, centres, radii)
    Ln = robot_reset(Ln, m_robot, lo).astype(np.float32)
    occupancy = Ln > np.float32(prm["l_occ"])
    # margins of the decisions
    frac = lambda a: np.abs(a - np.round(a))
    margin = np.abs(m_robot)
    margin = np.minimum(margin, np.where(in_front, np.inf, np.abs(z)))
    margin = np.minimum(margin, np.where(in_front, np.minimum(frac(u), frac(v)), np.inf))
    margin = np.minimum(margin, np.where(has, np.abs(np.abs(dz) - prm["tol"]), np.inf))
    margin = np.minimum(margin, np.where(inside, np.abs(pix_margin[iv_c, iu_c]), np.inf))
    return Ln, occupancy, margin
