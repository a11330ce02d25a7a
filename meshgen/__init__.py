"""Seeded synthetic meshes and vertex fields.

This module only draws inputs: vertex coordinates, cell connectivity and
vertex fields.  It holds none of the compressor's arithmetic, so both the
CPU oracle (under ``oracle/``) and the HIP library can be fed from it
without sharing code.

The shapes follow the paper's workloads (Table I of the paper lists 2-D
airfoil meshes of 0.5M-2M vertices and 3-D meshes of 1.45M-209M vertices):

* 2-D Delaunay triangulations of stratified-jittered points, optionally
  refined 8x in density inside an annulus (an airfoil-like refined band);
* 3-D tetrahedral meshes made of 6 Kuhn tetrahedra per cube of a jittered
  lattice;
* 2-D jittered structured triangulations (two triangles per square).

Every array is C-contiguous and laid out structure-of-arrays:
coordinates ``float32[D, n_v]``, cells ``int32[D+1, n_c]`` (0-based vertex
ids), fields ``float32[n_v]`` or ``float64[n_v]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from itertools import permutations

import numpy as np

__all__ = [
    "Mesh", "delaunay_2d", "stratified_points_2d", "refined_annulus_points",
    "kuhn_tet_mesh", "structured_tri_mesh", "aligned_tri_mesh",
    "field_bumps_2d", "field_front_2d", "field_octaves", "rotated_front_series",
    "config_small_2d", "config_large_2d", "config_tet_3d", "config_learned_series",
    "config_batch", "sliver_mesh",
]


@dataclass
class Mesh:
    """An unstructured simplicial mesh in structure-of-arrays layout."""
    coords: np.ndarray          # float32 [D, n_v]
    cells: np.ndarray           # int32  [D+1, n_c]
    info: dict = dc_field(default_factory=dict)

    @property
    def dim(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.coords.shape[1])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[1])


def _rngs(seed: int, k: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


# ---------------------------------------------------------------------------
# 2-D point sets and triangulations
# ---------------------------------------------------------------------------

def stratified_points_2d(m: int, rng, drop: int = 0) -> np.ndarray:
    """One uniform point per cell of an m x m lattice over [0,1)^2, row-major
    cell order; ``drop`` cells (chosen by ``rng``) receive no point."""
    iy, ix = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    ix = ix.ravel().astype(np.float64)
    iy = iy.ravel().astype(np.float64)
    jit = rng.random((2, m * m))
    pts = np.stack([(ix + jit[0]) / m, (iy + jit[1]) / m])
    if drop:
        keep = np.ones(m * m, dtype=bool)
        keep[rng.choice(m * m, size=drop, replace=False)] = False
        pts = pts[:, keep]
    return pts


def refined_annulus_points(h0: float, rng, center=(0.5, 0.5), radius=0.3,
                           half_width=0.05, refine: float = 8.0) -> np.ndarray:
    """Stratified jittered points with spacing ``h0`` outside the annulus
    ``|r - radius| <= half_width`` and spacing ``h0/sqrt(refine)`` inside it
    (``refine`` times the point density).  Row-major order within each of the
    two lattices, coarse lattice first."""
    out = []
    for spacing, inside in ((h0, False), (h0 / math.sqrt(refine), True)):
        m = int(math.floor(1.0 / spacing))
        iy, ix = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        cx = (ix.ravel() + 0.5) / m
        cy = (iy.ravel() + 0.5) / m
        r = np.hypot(cx - center[0], cy - center[1])
        sel = (np.abs(r - radius) <= half_width) == inside
        jit = rng.random((2, int(sel.sum())))
        out.append(np.stack([(ix.ravel()[sel] + jit[0]) / m,
                             (iy.ravel()[sel] + jit[1]) / m]))
    return np.concatenate(out, axis=1)


def delaunay_2d(points: np.ndarray) -> Mesh:
    """Delaunay triangulation (scipy Qhull) of float64 points [2, n]."""
    from scipy.spatial import Delaunay
    tri = Delaunay(points.T)
    cells = np.ascontiguousarray(tri.simplices.T.astype(np.int32))
    coords = np.ascontiguousarray(points.astype(np.float32))
    return Mesh(coords, cells, {"kind": "delaunay2d"})


def structured_tri_mesh(nx: int, ny: int, rng=None, jitter: float = 0.0,
                        lo=(0.0, 0.0), hi=(1.0, 1.0)) -> Mesh:
    """Jittered structured triangulation: an nx x ny vertex lattice over
    [lo, hi], each vertex displaced by U(-jitter, jitter) lattice spacings,
    two triangles per square.  With jitter <= 0.25 no triangle inverts."""
    hx = (hi[0] - lo[0]) / (nx - 1)
    hy = (hi[1] - lo[1]) / (ny - 1)
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = lo[0] + ix.ravel() * hx
    y = lo[1] + iy.ravel() * hy
    if jitter > 0:
        j = rng.uniform(-jitter, jitter, size=(2, nx * ny))
        x = x + j[0] * hx
        y = y + j[1] * hy
    coords = np.ascontiguousarray(np.stack([x, y]).astype(np.float32))
    qy, qx = np.meshgrid(np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    v00 = (qx + nx * qy).ravel().astype(np.int64)
    v10, v01, v11 = v00 + 1, v00 + nx, v00 + nx + 1
    t = np.empty((3, 2 * v00.size), dtype=np.int64)
    t[:, 0::2] = np.stack([v00, v10, v11])
    t[:, 1::2] = np.stack([v00, v11, v01])
    return Mesh(coords, np.ascontiguousarray(t.astype(np.int32)),
                {"kind": "structured2d", "nx": nx, "ny": ny, "jitter": jitter})


def aligned_tri_mesh(nx: int, ny: int) -> Mesh:
    """Structured triangulation whose vertices sit exactly on the integer
    lattice [0, nx-1] x [0, ny-1]; a grid with origin 0 and spacing 1 then
    puts one grid node exactly on every vertex."""
    return structured_tri_mesh(nx, ny, None, 0.0, (0.0, 0.0),
                               (float(nx - 1), float(ny - 1)))


# ---------------------------------------------------------------------------
# 3-D Kuhn tetrahedral meshes
# ---------------------------------------------------------------------------

_KUHN_PERMS = list(permutations(range(3)))


def _perm_sign(p) -> int:
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def _tet_dets(coords64: np.ndarray, cells: np.ndarray) -> np.ndarray:
    a = coords64[:, cells[0]]
    e1 = coords64[:, cells[1]] - a
    e2 = coords64[:, cells[2]] - a
    e3 = coords64[:, cells[3]] - a
    return (e1[0] * (e2[1] * e3[2] - e2[2] * e3[1])
            + e1[1] * (e2[2] * e3[0] - e2[0] * e3[2])
            + e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]))


def kuhn_tet_mesh(n: int, seed: int, jitter: float = 0.2,
                  chunk: int = 1 << 23) -> Mesh:
    """n^3 vertex lattice over [0,1]^3 (spacing 1/(n-1)), every vertex
    displaced by U(-jitter, jitter)^3 lattice spacings (boundary vertices
    too), six Kuhn tetrahedra per cube.  For the axis permutation (a, b, c)
    the tetrahedron is v0, v0+e_a, v0+e_a+e_b, v0+(1,1,1).  Cells are ordered
    cube by cube (x fastest), then by permutation.  Tetrahedra inverted by
    the jitter get their vertices' offsets re-drawn (seeded) until none is
    inverted; the count is in ``info['redrawn']``."""
    r_pts, r_redraw = _rngs(seed, 2)
    h = 1.0 / (n - 1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()]).astype(np.float64) * h
    del i, j, k
    off = r_pts.uniform(-jitter, jitter, size=(3, n ** 3)) * h

    m = n - 1
    ck, cj, ci = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    v0 = (ci.ravel() + n * cj.ravel() + n * n * ck.ravel()).astype(np.int64)
    del ci, cj, ck
    step = np.array([1, n, n * n], dtype=np.int64)
    cells = np.empty((4, v0.size, 6), dtype=np.int32)
    signs = np.empty(6, dtype=np.int8)
    for t, p in enumerate(_KUHN_PERMS):
        v1 = v0 + step[p[0]]
        v2 = v1 + step[p[1]]
        cells[0, :, t] = v0
        cells[1, :, t] = v1
        cells[2, :, t] = v2
        cells[3, :, t] = v0 + step.sum()
        signs[t] = _perm_sign(p)
    cells = cells.reshape(4, -1)
    cell_sign = np.tile(signs, v0.size)
    del v0

    coords = base + off
    redrawn = 0
    bad = []
    for s in range(0, cells.shape[1], chunk):
        d = _tet_dets(coords, cells[:, s:s + chunk])
        bad.append(s + np.nonzero(d * cell_sign[s:s + chunk] <= 0)[0])
    bad = np.concatenate(bad)
    for _ in range(64):
        if bad.size == 0:
            break
        verts = np.unique(cells[:, bad].ravel())
        redrawn += verts.size
        off[:, verts] = r_redraw.uniform(-jitter, jitter, size=(3, verts.size)) * h
        coords[:, verts] = base[:, verts] + off[:, verts]
        # re-check every tetrahedron of the cubes around the moved vertices
        vi = verts % n
        vj = (verts // n) % n
        vk = verts // (n * n)
        cubes = []
        for dk in (-1, 0):
            for dj in (-1, 0):
                for di in (-1, 0):
                    ok = ((vi + di >= 0) & (vi + di < m) & (vj + dj >= 0)
                          & (vj + dj < m) & (vk + dk >= 0) & (vk + dk < m))
                    cubes.append(((vi + di) + m * (vj + dj) + m * m * (vk + dk))[ok])
        cubes = np.unique(np.concatenate(cubes))
        tets = (cubes[:, None] * 6 + np.arange(6)[None, :]).ravel()
        d = _tet_dets(coords, cells[:, tets])
        bad = tets[d * cell_sign[tets] <= 0]
    if bad.size:
        raise RuntimeError("could not remove inverted tetrahedra")
    return Mesh(np.ascontiguousarray(coords.astype(np.float32)),
                np.ascontiguousarray(cells),
                {"kind": "kuhn3d", "n": n, "jitter": jitter, "redrawn": int(redrawn)})


# ---------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------

def field_bumps_2d(coords: np.ndarray, rng, n_bumps: int = 5,
                   sigma: float = 0.05) -> np.ndarray:
    """sin(4 pi x) cos(3 pi y) plus ``n_bumps`` unit Gaussian bumps of width
    ``sigma`` at uniform random centres (float64)."""
    x = coords[0].astype(np.float64)
    y = coords[1].astype(np.float64)
    f = np.sin(4 * np.pi * x) * np.cos(3 * np.pi * y)
    centres = rng.random((n_bumps, 2))
    for cx, cy in centres:
        f += np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * sigma * sigma))
    return f


def _fourier_noise(x, y, rng, kmax: int = 4):
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          if (kx, ky) != (0, 0)]
    a = rng.standard_normal(len(ks)) / (1.0 + np.array([kx * kx + ky * ky for kx, ky in ks]))
    a /= np.abs(a).sum()
    phi = rng.uniform(0, 2 * np.pi, len(ks))
    out = np.zeros_like(x)
    for (kx, ky), ak, pk in zip(ks, a, phi):
        out += ak * np.cos(2 * np.pi * (kx * x + ky * y) + pk)
    return out


def field_front_2d(coords: np.ndarray, rng, center=(0.5, 0.5), radius=0.3,
                   width=0.01, noise=0.05, noise_rng=None, xy=None) -> np.ndarray:
    """tanh((r - radius)/width) + noise * N(p), N a seeded low-frequency
    Fourier series (wave numbers in [-4, 4]^2, amplitudes ~ N(0,1)/(1+|k|^2),
    normalised to unit L1 norm).  float64."""
    if xy is None:
        x = coords[0].astype(np.float64)
        y = coords[1].astype(np.float64)
    else:
        x, y = xy
    r = np.hypot(x - center[0], y - center[1])
    return np.tanh((r - radius) / width) + noise * _fourier_noise(x, y, rng)


def field_octaves(coords: np.ndarray, rng, octaves: int = 3, modes: int = 4,
                  dtype=np.float32) -> np.ndarray:
    """sum_o 2^-o * (1/modes) * sum_m sin(2 pi 2^o (k_om . p) + phi_om), wave
    vector components drawn from +-{1,2,3}, phases uniform."""
    d = coords.shape[0]
    p = coords.astype(np.float64)
    out = np.zeros(coords.shape[1], dtype=np.float64)
    for o in range(octaves):
        for _ in range(modes):
            k = rng.choice([1, 2, 3], size=d) * rng.choice([-1, 1], size=d)
            phi = rng.uniform(0, 2 * np.pi)
            arg = np.zeros_like(out)
            for a in range(d):
                arg += k[a] * p[a]
            out += (2.0 ** -o) / modes * np.sin(2 * np.pi * (2 ** o) * arg + phi)
    return out.astype(dtype)


def rotated_front_series(coords: np.ndarray, seed: int, steps: int = 9):
    """Time series f_t(p) = f_0(Rot(-t*dtheta)(p - c_r) + c_r), t = 0..steps-1,
    where f_0 is ``field_front_2d``; dtheta ~ U[2, 10] degrees and the centre
    c_r ~ U[0.4, 0.6]^2 so the front moves.  Returns a list of float64."""
    r_field, r_rot = _rngs(seed, 2)
    dtheta = math.radians(r_rot.uniform(2.0, 10.0))
    c = r_rot.uniform(0.4, 0.6, size=2)
    x = coords[0].astype(np.float64) - c[0]
    y = coords[1].astype(np.float64) - c[1]
    state = r_field.bit_generator.state
    out = []
    for t in range(steps):
        th = -t * dtheta
        xr = math.cos(th) * x - math.sin(th) * y + c[0]
        yr = math.sin(th) * x + math.cos(th) * y + c[1]
        r_field.bit_generator.state = state      # same f_0 for every t
        out.append(field_front_2d(None, r_field, xy=(xr, yr)))
    return out


# ---------------------------------------------------------------------------
# Workload configurations (the paper's shapes at synthetic stand-in sizes)
# ---------------------------------------------------------------------------

def config_small_2d(seed: int = 1):
    """20,000 stratified-jittered points on a 142 x 142 lattice (164 cells
    dropped), Delaunay; float64 bumps field; 128 x 128 grid; absolute eb
    1e-3 * range, split 50/50."""
    r_pts, r_field = _rngs(seed, 2)
    mesh = delaunay_2d(stratified_points_2d(142, r_pts, drop=164))
    f = field_bumps_2d(mesh.coords, r_field)
    rng_ = float(f.max() - f.min())
    return mesh, f, dict(dims=(128, 128, 1), eb=1e-3 * rng_, eb_mode="abs", split=0.5)


def config_large_2d(seed: int = 2, h0: float = 7.615e-4, eb: float = 1e-4,
                    dims: int = 2048):
    """~4.0M points refined 8x inside |r - 0.3| <= 0.05, Delaunay; float64
    front + Fourier noise field; dims^2 grid; relative eb.  ``h0`` and
    ``dims`` scale it down for tests."""
    r_pts, r_field = _rngs(seed, 2)
    mesh = delaunay_2d(refined_annulus_points(h0, r_pts))
    f = field_front_2d(mesh.coords, r_field)
    return mesh, f, dict(dims=(dims, dims, 1), eb=eb, eb_mode="rel", split=0.5)


def field_large_2d(coords: np.ndarray, seed: int = 2) -> np.ndarray:
    """The field of config_large_2d(seed) on given vertices (the same mesh
    is also the one config_learned_series builds)."""
    return field_front_2d(coords, _rngs(seed, 2)[1])


def config_tet_3d(seed: int = 3, n: int = 252, dims: int = 256, eb: float = 1e-4,
                  split: float = 0.5):
    """n^3 jittered lattice (+-20% of the spacing), 6 Kuhn tets per cube;
    float32 three-octave sinusoid field; dims^3 grid; relative eb."""
    r_mesh, r_field = np.random.SeedSequence(seed).spawn(2)
    mesh = kuhn_tet_mesh(n, int(r_mesh.generate_state(1)[0]))
    f = field_octaves(mesh.coords, np.random.default_rng(r_field))
    return mesh, f, dict(dims=(dims, dims, dims), eb=eb, eb_mode="rel", split=split)


def config_learned_series(seed: int = 4, h0: float = 7.615e-4, dims: int = 2048,
                          steps: int = 9, mesh=None):
    """The large 2-D mesh with ``steps`` timesteps of its field advected by a
    seeded rigid rotation; relative eb 1e-4; train on t=0, apply to t>=1."""
    if mesh is None:
        r_pts = _rngs(2, 2)[0]
        mesh = delaunay_2d(refined_annulus_points(h0, r_pts))
    series = rotated_front_series(mesh.coords, seed, steps)
    return mesh, series, dict(dims=(dims, dims, 1), eb=1e-4, eb_mode="rel", split=0.5)


def config_batch(seed: int = 5, scale: float = 1.0, n_meshes: int = 12,
                 n_fields: int = 64, log=None):
    """Uneven multi-mesh workload: ``n_meshes`` meshes with vertex counts
    log-uniform in [0.5M, 20M] * scale (the first two forced to the ends),
    even-indexed meshes 2-D jittered structured triangulations, odd-indexed
    3-D Kuhn meshes; field i lives on mesh i mod n_meshes, float32 for even
    i and float64 for odd i, relative eb 1e-3/1e-4/1e-5 by i mod 3, grids
    with about one node per four vertices.  ``log`` (optional) is called
    with a line per generated mesh."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    lo, hi = 0.5e6 * scale, 20e6 * scale
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_meshes))
    sizes[0], sizes[1] = lo, hi
    meshes, grids = [], []
    for m in range(n_meshes):
        ms = int(rng.integers(1 << 31))
        if m % 2 == 0:
            side = max(4, int(round(math.sqrt(sizes[m]))))
            mesh = structured_tri_mesh(side, side, np.random.default_rng(ms), 0.2)
            d = max(2, math.ceil((mesh.n_vertices / 4) ** 0.5))
            grids.append((d, d, 1))
        else:
            side = max(3, int(round(sizes[m] ** (1 / 3))))
            mesh = kuhn_tet_mesh(side, ms)
            d = max(2, math.ceil((mesh.n_vertices / 4) ** (1 / 3)))
            grids.append((d, d, d))
        meshes.append(mesh)
        if log:
            log(f"mesh {m}: {mesh.dim}-D, {mesh.n_vertices} vertices, {mesh.n_cells} cells")
    fields = []
    for i in range(n_fields):
        m = i % n_meshes
        fr = np.random.default_rng(int(rng.integers(1 << 31)))
        dt = np.float32 if i % 2 == 0 else np.float64
        fields.append(dict(mesh=m, data=field_octaves(meshes[m].coords, fr, dtype=dt),
                           eb=(1e-3, 1e-4, 1e-5)[i % 3], eb_mode="rel", split=0.5))
    return meshes, grids, fields


# ---------------------------------------------------------------------------
# Meshes with near-degenerate cells over grid nodes
# ---------------------------------------------------------------------------

def sliver_mesh(dim: int, seed: int = 0):
    """A mesh over [0,1]^dim whose lowest-numbered cells are slivers: thin
    triangles (2-D) or flat tetrahedra (3-D) whose thickness is about 5e-4
    against an extent near 0.8, laid across rows (2-D) or planes (3-D) of
    the grid returned with it, so that grid nodes lie strictly inside them.
    Each sliver's base sits 1e-4 below the nominal row / plane position and
    its apex 4e-4 above, so FP32 rounding of node positions (about 1e-7)
    cannot move a node across.  The rest of the mesh is an unjittered
    structured triangulation (13 x 11) or Kuhn lattice (9^3) covering the
    box, so every node is located.  Returns (mesh, dims, field float32)."""
    rng = np.random.default_rng(seed)
    if dim == 2:
        base = structured_tri_mesh(13, 11)
        dims = (41, 37)
        slivers = []
        for row in (9, 20):                 # horizontal slivers across node rows
            y = row / (dims[1] - 1)
            slivers.append([(0.05, y - 1e-4), (0.95, y - 1e-4), (0.5, y + 4e-4)])
        col = 30                            # a vertical one across a node column
        x = col / (dims[0] - 1)
        slivers.append([(x - 1e-4, 0.05), (x + 4e-4, 0.5), (x - 1e-4, 0.95)])
    else:
        base = kuhn_tet_mesh(9, seed, jitter=0.0)
        dims = (17, 15, 13)
        z = 6 / (dims[2] - 1)
        x = 4 / (dims[0] - 1)
        slivers = [
            [(0.1, 0.1, z - 1e-4), (0.9, 0.15, z - 1e-4), (0.3, 0.9, z - 1e-4), (0.5, 0.45, z + 4e-4)],
            [(x - 1e-4, 0.1, 0.1), (x - 1e-4, 0.9, 0.2), (x - 1e-4, 0.2, 0.9), (x + 4e-4, 0.5, 0.5)],
        ]
    nv = base.n_vertices
    extra = np.array([p for s in slivers for p in s], np.float64).T
    coords = np.ascontiguousarray(np.concatenate([base.coords, extra.astype(np.float32)], axis=1))
    k = dim + 1
    sc = (nv + np.arange(len(slivers) * k, dtype=np.int32)).reshape(len(slivers), k).T
    cells = np.ascontiguousarray(np.concatenate([sc, base.cells], axis=1).astype(np.int32))
    mesh = Mesh(coords, cells, {"kind": f"sliver{dim}d", "n_slivers": len(slivers)})
    return mesh, dims, field_octaves(coords, rng)
