"""Candidate cells of points in a jittered Kuhn lattice (meshgen.kuhn_tet_mesh):
mesh structure only, no part of the method.

A lattice vertex moves at most `jitter` spacings per axis, so a cube's six
tetrahedra lie inside the cube widened by `jitter` spacings, and a point
with lattice coordinate u can only be in cubes floor(u) - 1 .. floor(u) + 1
on each axis (for jitter < 1/2).  Cells are numbered cube by cube (x
fastest), six per cube."""
import numpy as np


def kuhn_candidates(points: np.ndarray, n: int) -> np.ndarray:
    """int32 [npoints, 162] ascending candidate cell ids (-1 = none)."""
    m = n - 1
    u = np.floor(points.astype(np.float64) * (n - 1)).astype(np.int64)      # [3, np]
    out = []
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                ci, cj, ck = u[0] + di, u[1] + dj, u[2] + dk
                ok = (ci >= 0) & (ci < m) & (cj >= 0) & (cj < m) & (ck >= 0) & (ck < m)
                cube = ci + m * (cj + m * ck)
                for t in range(6):
                    out.append(np.where(ok, 6 * cube + t, -1))
    cand = np.stack(out, axis=1)
    cand = np.where(cand < 0, np.iinfo(np.int32).max, cand)
    cand.sort(axis=1)
    cand = np.where(cand == np.iinfo(np.int32).max, -1, cand)
    # valid ids first, ascending; the -1 entries are skipped by the locator
    return np.ascontiguousarray(cand, dtype=np.int32)
