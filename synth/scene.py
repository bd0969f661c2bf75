"""Seeded synthetic scenes: primitives -> occupancy -> signed distance grid.

The plan step takes the distance field as an input (the paper builds it on the
GPU from sensor data, Sec. III; that mapping stage is not part of the plan step).
These generators stand in for the paper's Gazebo scenes, which are not available.

Grid conventions (shared with the C interface):

* array shape ``(nz, ny, nx)``, C order, so the flat index of voxel (ix, iy, iz)
  is ``(iz * ny + iy) * nx + ix`` (x fastest);
* ``origin`` is the corner of voxel (0, 0, 0); voxel centres sit at
  ``origin + (i + 0.5) * voxel``;
* values are signed distances in metres: positive outside obstacles, negative
  inside.  For a free voxel the value is ``voxel * sqrt(D)`` with ``D`` the
  squared index distance to the nearest occupied voxel centre, which is what the
  paper's EDT stores (Sec. III-B, as a squared distance); occupied voxels get the
  negative distance to the nearest free centre.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import ndimage


@dataclasses.dataclass
class Primitive:
    kind: str               # "box" (axis-aligned) or "sphere"
    center: np.ndarray      # (3,)
    size: np.ndarray        # box: full side lengths (3,); sphere: (radius,)
    velocity: np.ndarray    # (3,) m/s, used by drifting scenes

    def contains(self, pts: np.ndarray) -> np.ndarray:
        rel = pts - self.center
        if self.kind == "box":
            return np.all(np.abs(rel) <= 0.5 * self.size, axis=-1)
        return np.sum(rel * rel, axis=-1) <= self.size[0] ** 2


def grid_origin(n: int, voxel: float) -> np.ndarray:
    """Origin (corner) of an n^3 grid centred on the robot base in x/y, floor at z=0."""
    side = n * voxel
    return np.array([-0.5 * side, -0.5 * side, 0.0])


def random_primitives(rng: np.random.Generator, lo: np.ndarray, hi: np.ndarray,
                      n_boxes: int, n_spheres: int, box_side=(0.1, 0.4),
                      sphere_radius=(0.05, 0.2), speed: float = 0.0,
                      keepout_radius: float = 0.15, keepout_height: float = 0.45,
                      max_tries: int = 10000) -> list[Primitive]:
    """Draw boxes and spheres with centres uniform in [lo, hi].

    Primitives that reach into a vertical keep-out cylinder around the robot base
    (radius ``keepout_radius`` up to height ``keepout_height``) are redrawn, so
    the base of the arm does not start buried in an obstacle.
    """
    prims: list[Primitive] = []
    tries = 0
    kinds = ["box"] * n_boxes + ["sphere"] * n_spheres
    for kind in kinds:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("could not place primitives outside the keep-out zone")
            c = rng.uniform(lo, hi)
            if kind == "box":
                size = rng.uniform(box_side[0], box_side[1], size=3)
                reach = 0.5 * np.hypot(size[0], size[1])
                bottom = c[2] - 0.5 * size[2]
            else:
                size = np.array([rng.uniform(sphere_radius[0], sphere_radius[1])])
                reach = size[0]
                bottom = c[2] - size[0]
            vdir = rng.normal(size=3)
            vel = speed * vdir / np.linalg.norm(vdir)
            if np.hypot(c[0], c[1]) - reach < keepout_radius and bottom < keepout_height:
                continue
            prims.append(Primitive(kind, c, size, vel))
            break
    return prims


def voxel_centres(n: tuple[int, int, int], origin: np.ndarray, voxel: float) -> np.ndarray:
    """Voxel centre coordinates, shape (nz, ny, nx, 3) for n = (nx, ny, nz)."""
    nx, ny, nz = n
    xs = origin[0] + (np.arange(nx) + 0.5) * voxel
    ys = origin[1] + (np.arange(ny) + 0.5) * voxel
    zs = origin[2] + (np.arange(nz) + 0.5) * voxel
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def occupancy(prims: list[Primitive], n: tuple[int, int, int], origin: np.ndarray,
              voxel: float) -> np.ndarray:
    """Boolean (nz, ny, nx) grid: a voxel is occupied when its centre lies in a primitive."""
    nx, ny, nz = n
    occ = np.zeros((nz, ny, nx), dtype=bool)
    xs = origin[0] + (np.arange(nx) + 0.5) * voxel
    ys = origin[1] + (np.arange(ny) + 0.5) * voxel
    zs = origin[2] + (np.arange(nz) + 0.5) * voxel
    for p in prims:
        # Only test the primitive's bounding box to keep large grids cheap.
        ext = 0.5 * p.size if p.kind == "box" else np.repeat(p.size[0], 3)
        lo, hi = p.center - ext, p.center + ext
        ix = np.nonzero((xs >= lo[0]) & (xs <= hi[0]))[0]
        iy = np.nonzero((ys >= lo[1]) & (ys <= hi[1]))[0]
        iz = np.nonzero((zs >= lo[2]) & (zs <= hi[2]))[0]
        if ix.size == 0 or iy.size == 0 or iz.size == 0:
            continue
        Z, Y, X = np.meshgrid(zs[iz], ys[iy], xs[ix], indexing="ij")
        inside = p.contains(np.stack([X, Y, Z], axis=-1))
        sub = occ[iz[0]:iz[-1] + 1, iy[0]:iy[-1] + 1, ix[0]:ix[-1] + 1]
        sub |= inside
    return occ


def squared_index_edt(occ: np.ndarray) -> np.ndarray:
    """Exact squared index distance from every voxel centre to the nearest occupied one.

    Occupied voxels get 0.  Grids without any occupied voxel get a large value
    (the sum of squared grid extents), so distances stay finite.  Uses scipy's
    exact Euclidean transform and rounds the squared result to an integer.
    """
    if not occ.any():
        big = sum(s * s for s in occ.shape)
        return np.full(occ.shape, big, dtype=np.int64)
    dist = ndimage.distance_transform_edt(~occ)
    return np.rint(dist * dist).astype(np.int64)


def signed_distance_grid(occ: np.ndarray, voxel: float) -> np.ndarray:
    """phi = voxel * (sqrt(D_out) - sqrt(D_in)) as float32, shape (nz, ny, nx)."""
    d_out = squared_index_edt(occ)
    d_in = squared_index_edt(~occ) if occ.any() else np.zeros(occ.shape, np.int64)
    phi = voxel * (np.sqrt(d_out.astype(np.float64)) - np.sqrt(d_in.astype(np.float64)))
    return phi.astype(np.float32)


def advance_primitives(prims: list[Primitive], dt: float, lo: np.ndarray,
                       hi: np.ndarray) -> list[Primitive]:
    """Move every primitive by velocity*dt, reflecting its centre off [lo, hi]."""
    out = []
    for p in prims:
        c = p.center + p.velocity * dt
        v = p.velocity.copy()
        for ax in range(3):
            if c[ax] < lo[ax]:
                c[ax] = 2 * lo[ax] - c[ax]
                v[ax] = -v[ax]
            elif c[ax] > hi[ax]:
                c[ax] = 2 * hi[ax] - c[ax]
                v[ax] = -v[ax]
        out.append(Primitive(p.kind, c, p.size, v))
    return out
