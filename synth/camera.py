"""Seeded synthetic depth images: a pinhole camera looking at the scene primitives and
the robot's collision spheres (the paper's depth camera and its datasets are absent).

Depth is the z coordinate in the camera frame of the first hit along each pixel's
ray through the pixel centre (u + 1/2, v + 1/2); pixels without a hit within the
range read 0 (no return).  Rays are cast in float64 and the image is rounded to
float32, the precision the mapping kernels read.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import scene as scene_mod


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    T_wc: np.ndarray          # (4, 4) camera-to-world pose, float32
    min_depth: float = 0.1
    max_depth: float = 4.0


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world pose with the optical axis (+z) from eye towards target, +x to
    the right and +y down in the image."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, y, z, eye
    return T


def default_camera(width: int = 320, height: int = 240, eye=(1.2, -0.9, 0.9),
                   target=(0.0, 0.0, 0.35)) -> Camera:
    f = 0.9 * width
    return Camera(fx=float(np.float32(f)), fy=float(np.float32(f)),
                  cx=float(np.float32(width / 2)), cy=float(np.float32(height / 2)),
                  width=width, height=height,
                  T_wc=look_at(eye, target).astype(np.float32))


def _ray_box(o, d, lo, hi):
    inv = 1.0 / np.where(d == 0.0, 1e-300, d)
    t0 = (lo - o) * inv
    t1 = (hi - o) * inv
    tmin = np.minimum(t0, t1).max(axis=-1)
    tmax = np.maximum(t0, t1).min(axis=-1)
    hit = (tmax >= tmin) & (tmax > 0)
    return np.where(hit, np.where(tmin > 0, tmin, tmax), np.inf)


def _ray_sphere(o, d, c, r):
    """First t > 0 with |o + t d - c| = r (d need not be unit)."""
    oc = o - c
    a = np.sum(d * d, axis=-1)
    b = np.sum(oc * d, axis=-1)
    cc = np.sum(oc * oc, axis=-1) - r * r
    disc = b * b - a * cc
    sq = np.sqrt(np.maximum(disc, 0.0))
    t = (-b - sq) / a
    t = np.where(t > 0, t, (-b + sq) / a)
    return np.where((disc >= 0) & (t > 0), t, np.inf)


def render_depth(cam: Camera, prims: list[scene_mod.Primitive],
                 spheres: np.ndarray | None = None, radii: np.ndarray | None = None) -> np.ndarray:
    """Depth image (height, width) float32 of the primitives and optional extra spheres
    (e.g. the robot's collision spheres in the world frame)."""
    T = np.asarray(cam.T_wc, np.float64)
    v, u = np.mgrid[0:cam.height, 0:cam.width]
    xc = (u + 0.5 - cam.cx) / cam.fx
    yc = (v + 0.5 - cam.cy) / cam.fy
    dirs_c = np.stack([xc, yc, np.ones_like(xc)], axis=-1)        # z = 1: t is the depth
    dirs_w = dirs_c @ T[:3, :3].T
    o = T[:3, 3]
    t = np.full((cam.height, cam.width), np.inf)
    for p in prims:
        if p.kind == "box":
            lo, hi = p.center - 0.5 * p.size, p.center + 0.5 * p.size
            t = np.minimum(t, _ray_box(o, dirs_w, lo, hi))
        else:
            t = np.minimum(t, _ray_sphere(o, dirs_w, p.center, p.size[0]))
    if spheres is not None:
        for c, r in zip(np.asarray(spheres, np.float64), np.asarray(radii, np.float64)):
            t = np.minimum(t, _ray_sphere(o, dirs_w, c, r))
    depth = np.where(np.isfinite(t) & (t >= cam.min_depth) & (t <= cam.max_depth), t, 0.0)
    return depth.astype(np.float32)
