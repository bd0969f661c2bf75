"""Exact squared Euclidean distance transforms on voxel grids (oracle, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's mapping stage (Sec. III-B) computes the distance field with the
separable exact transform of Felzenszwalb and Huttenlocher: a 1-D squared
distance transform (lower envelope of parabolas) along y, then x, then z, with
occupied voxels as zero-cost sources and every other voxel at a large value.
Two independent routes are given here:

* :func:`edt_separable_fh` follows that description (1-D lower envelopes, axis
  order y, x, z);
* :func:`edt_brute_force` takes the minimum of squared index distances to every
  occupied voxel, for tiny grids.

Both return integer squared index distances on a ``(nz, ny, nx)`` grid.
"""
from __future__ import annotations

import numpy as np

INF = np.iinfo(np.int64).max // 4


def fh_1d(f: np.ndarray) -> np.ndarray:
    """D(p) = min_q ((p - q)^2 + f(q)) for a 1-D sampled function f (int64, INF allowed).

    Lower envelope of the parabolas rooted at the finite samples: scan left to
    right keeping the parabolas that are minimal somewhere, then read the
    envelope off at every sample.
    """
    n = f.shape[0]
    roots = [q for q in range(n) if f[q] < INF]
    out = np.full(n, INF, dtype=np.int64)
    if not roots:
        return out
    v: list[int] = []          # roots of the parabolas in the envelope
    z: list[float] = []        # left boundary of each envelope piece
    for q in roots:
        fq = float(f[q])
        while True:
            if not v:
                v.append(q)
                z.append(-np.inf)
                break
            p = v[-1]
            # Intersection of the parabolas rooted at p and q.
            s = ((fq + q * q) - (float(f[p]) + p * p)) / (2.0 * (q - p))
            if s <= z[-1]:
                v.pop()
                z.pop()
                continue
            v.append(q)
            z.append(s)
            break
    piece = 0
    for p in range(n):
        while piece + 1 < len(v) and z[piece + 1] < p:
            piece += 1
        r = v[piece]
        out[p] = (p - r) * (p - r) + int(f[r])
    return out


def _transform_axis(g: np.ndarray, axis: int) -> np.ndarray:
    moved = np.moveaxis(g, axis, -1)
    out = np.empty_like(moved)
    for idx in np.ndindex(moved.shape[:-1]):
        out[idx] = fh_1d(moved[idx])
    return np.moveaxis(out, -1, axis)


def edt_separable_fh(occ: np.ndarray) -> np.ndarray:
    """Squared index distance to the nearest occupied voxel; passes along y, x, z."""
    g = np.where(occ, 0, INF).astype(np.int64)
    # Array axes are (z, y, x): y is axis 1, x axis 2, z axis 0.
    for axis in (1, 2, 0):
        g = _transform_axis(g, axis)
    return g


def edt_brute_force(occ: np.ndarray) -> np.ndarray:
    """Same quantity by exhaustive search over occupied voxels (tiny grids only)."""
    occ_idx = np.argwhere(occ)
    out = np.full(occ.shape, INF, dtype=np.int64)
    if occ_idx.size == 0:
        return out
    for idx in np.ndindex(occ.shape):
        d = occ_idx - np.asarray(idx)
        out[idx] = int(np.min(np.sum(d * d, axis=1)))
    return out


def edt_separable_minplus(occ: np.ndarray) -> np.ndarray:
    """Same quantity as :func:`edt_separable_fh`, each 1-D pass taken straight from its
    definition D(p) = min_q ((p - q)^2 + f(q)), vectorised over the lines of an axis.

    O(n) work per output sample instead of FH's amortised O(1), but plain numpy, so
    grids of a few million voxels finish in seconds.  Works in int32 with 2^30 as
    "no source" (every finite squared distance here is far below it).
    """
    big = np.int32(1 << 30)
    g = np.where(occ, 0, big).astype(np.int32)
    for axis in (1, 2, 0):
        moved = np.ascontiguousarray(np.moveaxis(g, axis, -1))
        shape = moved.shape
        lines = moved.reshape(-1, shape[-1])
        n = shape[-1]
        q = np.arange(n, dtype=np.int32)
        out = np.empty_like(lines)
        step = max(1, (1 << 20) // n)
        for lo in range(0, lines.shape[0], step):
            blk = lines[lo:lo + step]
            for p in range(n):
                out[lo:lo + step, p] = np.minimum((blk + (p - q) ** 2).min(axis=1), big)
        g = np.moveaxis(out.reshape(shape), -1, axis)
    return np.where(g >= big, INF, g.astype(np.int64))


def no_source_value(shape) -> int:
    """Squared distance given to every voxel when the grid holds no source at all:
    the sum of the squared grid extents, so that distances stay finite."""
    return int(sum(int(s) * int(s) for s in shape))


def signed_distance(occ: np.ndarray, voxel: float, transform=edt_separable_fh):
    """Signed distance grid from occupancy (Sec. III-B, with the sign convention of the
    planner's field: positive outside obstacles, negative inside).

    D_out is the squared index distance of every voxel to the nearest occupied one
    and D_in to the nearest free one (each zero on its own sources); a field without
    any source takes :func:`no_source_value`.  phi = voxel * (sqrt(D_out) - sqrt(D_in)),
    evaluated in float64 and rounded once to float32.

    Returns (phi float32, D_out int64, D_in int64), all shaped like ``occ`` (z, y, x).
    """
    occ = np.asarray(occ, dtype=bool)
    big = no_source_value(occ.shape)
    d_out = transform(occ)
    d_in = transform(~occ)
    d_out = np.where(d_out >= INF, big, d_out)
    d_in = np.where(d_in >= INF, big, d_in)
    phi = float(voxel) * (np.sqrt(d_out.astype(np.float64)) - np.sqrt(d_in.astype(np.float64)))
    return phi.astype(np.float32), d_out, d_in
