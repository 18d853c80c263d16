"""Seeded synthetic inputs: surface meshes, random vectors and workload sizes.

This module produces the *inputs* of the AIMx operator -- triangle meshes,
random complex vectors, wavenumbers, grid sizes and patch centres -- and
nothing of the method's arithmetic (no quadrature, no stencil, no kernel).
It is the only module shared by the CPU oracle side (tests, bench baseline)
and the GPU library side; it imports neither.

Workload shapes stand in for the paper's test structures: a sphere
(Sec. "Overlapping basis and test functions", a 1 m sphere meshed with flat
triangles) and arrays of conductor boxes (the array examples of Sec.
"Results", which use 3rd-order stencils).  The paper's own geometries are not
available and are not recreated.

Seeds follow ``numpy.random.default_rng(1000 * workload + stream)`` with
stream 0 = geometry jitter, 1 = Gaussian input vector, 2 = right-hand-side
patches, 3 = uneven-batch shapes, 4 = training geometries.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Sphere of ``20 * 4**level`` flat triangles with vertices on the sphere.

    Each subdivision splits every triangle into four through its edge
    midpoints, which are then pushed out to the sphere.  Faces are oriented
    with outward normals.  Returns ``(vertices float64[nv,3], triangles
    int32[nt,3])``.
    """
    v, f = _icosahedron()
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        key = e[:, 0] * (nv + 1) + e[:, 1]
        uniq, inv = np.unique(key, return_inverse=True)
        a = uniq // (nv + 1)
        b = uniq % (nv + 1)
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        v = np.concatenate([v, mid], axis=0)
        nf = f.shape[0]
        m01 = nv + inv[:nf]
        m12 = nv + inv[nf:2 * nf]
        m20 = nv + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], m01, m20], axis=1),
            np.stack([f[:, 1], m12, m01], axis=1),
            np.stack([f[:, 2], m20, m12], axis=1),
            np.stack([m01, m12, m20], axis=1),
        ], axis=0)
    v = v * radius + np.asarray(center, dtype=np.float64)
    return np.ascontiguousarray(v), np.ascontiguousarray(f.astype(np.int32))


def box_surface(lo, size, edge: float):
    """Closed surface of an axis-aligned box cut into squares of side about
    ``edge``, each square split into two triangles (outward normals).

    Returns ``(vertices, triangles)`` with vertices shared between faces.
    """
    lo = np.asarray(lo, dtype=np.float64)
    size = np.asarray(size, dtype=np.float64)
    counts = [max(1, int(round(s / edge))) for s in size]
    verts = []
    tris = []
    base = 0
    # (normal axis, side, the two in-plane axes in right-handed order)
    for ax in range(3):
        u_ax, v_ax = (ax + 1) % 3, (ax + 2) % 3
        for side in (0, 1):
            nu, nv = counts[u_ax], counts[v_ax]
            uu = lo[u_ax] + size[u_ax] * np.arange(nu + 1) / nu
            vv = lo[v_ax] + size[v_ax] * np.arange(nv + 1) / nv
            U, V = np.meshgrid(uu, vv, indexing="ij")
            P = np.empty((nu + 1, nv + 1, 3))
            P[..., ax] = lo[ax] + side * size[ax]
            P[..., u_ax] = U
            P[..., v_ax] = V
            verts.append(P.reshape(-1, 3))
            idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1) + base
            a = idx[:-1, :-1].ravel()
            b = idx[1:, :-1].ravel()
            c = idx[1:, 1:].ravel()
            d = idx[:-1, 1:].ravel()
            # (u, v, ax) is right-handed, so a->b->c is counter-clockwise seen
            # from +ax; flip on the low side to keep normals outward.
            if side == 1:
                t = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
            else:
                t = np.concatenate([np.stack([a, c, b], 1), np.stack([a, d, c], 1)])
            tris.append(t)
            base += (nu + 1) * (nv + 1)
    V = np.concatenate(verts)
    T = np.concatenate(tris)
    # merge duplicated vertices along box edges
    key = np.round(V / (edge * 1e-6)).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    V = V[first]
    T = inv.reshape(-1)[T]
    return np.ascontiguousarray(V), np.ascontiguousarray(T.astype(np.int32))


def merge_meshes(parts):
    vs, ts, off = [], [], 0
    for v, t in parts:
        vs.append(v)
        ts.append(t + off)
        off += v.shape[0]
    return np.concatenate(vs), np.concatenate(ts).astype(np.int32)


def box_array(nx: int = 4, ny: int = 4, size=(1.0, 1.0, 4.0), gap: float = 0.5,
              jitter: float = 0.05, edge: float = 0.1, seed: int = 2000):
    """``nx * ny`` boxes on a square lattice in the x-y plane with seeded
    uniform position jitter in ``[-jitter, jitter]^3`` per box."""
    rng = np.random.default_rng(seed)
    size = np.asarray(size, dtype=np.float64)
    pitch = size[:2] + gap
    parts = []
    for ix in range(nx):
        for iy in range(ny):
            lo = np.array([ix * pitch[0], iy * pitch[1], 0.0])
            lo = lo + rng.uniform(-jitter, jitter, size=3)
            parts.append(box_surface(lo, size, edge))
    return merge_meshes(parts)


# --------------------------------------------------------------------------
# vectors
# --------------------------------------------------------------------------

def complex_gaussian(n: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """``(N(0,1) + j N(0,1)) / sqrt(2)`` samples, shape ``[n]`` or ``[nrhs, n]``."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (nrhs, n)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / math.sqrt(2.0)


def triangle_centroids(V, T):
    """Mean of each triangle's three vertices (used only to place patches)."""
    return (V[T[:, 0]] + V[T[:, 1]] + V[T[:, 2]]) / 3.0


def patch_centres(V, T, count: int, seed: int) -> np.ndarray:
    """Centres of Gaussian excitation patches: centroids of ``count``
    seeded random triangles."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(T.shape[0], size=count, replace=False)
    return triangle_centroids(V, T)[idx]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """One synthetic workload: mesh, grid, stencil order, wavenumbers."""
    name: str
    vertices: np.ndarray
    triangles: np.ndarray
    order: int                  # stencil order n; (n+1)^3 nodes per point
    dims: tuple                 # unpadded grid points (Nx, Ny, Nz)
    h: float                    # grid spacing (<= 0: derived by the library)
    near_factor: float          # near-region threshold in units of h
    k: np.ndarray               # wavenumbers
    seed_base: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.triangles.shape[0])

    @property
    def near_threshold(self) -> float:
        return self.near_factor * self.h


def derived_spacing(V, dims, margin: int = 2) -> float:
    """Isotropic spacing that fits the vertex bounding box into ``dims``
    points with ``margin`` spare nodes per side."""
    ext = V.max(axis=0) - V.min(axis=0)
    return float(max(ext[a] / (dims[a] - 1 - 2 * margin) for a in range(3)))


def sphere_small() -> Workload:
    """Radius-0.5 level-3 icosphere (1,280 triangles), k = 2*pi, 16^3 grid,
    h = 0.1, 2nd-order stencil, near threshold 2h."""
    V, T = icosphere(3, 0.5)
    return Workload("sphere-1280", V, T, 2, (16, 16, 16), 0.1, 2.0,
                    np.array([2 * math.pi]), 1000)


def box_array_large() -> Workload:
    """4x4 array of 1x1x4 boxes (57,600 triangles), 3rd-order stencil,
    128x128x64 grid, near threshold 3h, k = 2*pi."""
    V, T = box_array(seed=2000)
    dims = (128, 128, 64)
    h = derived_spacing(V, dims)
    return Workload("boxarray-57600", V, T, 3, dims, h, 3.0,
                    np.array([2 * math.pi]), 2000)


def sweep_small(nfreq: int = 64, rhs_per_freq: int = 8) -> Workload:
    """The small sphere at ``nfreq`` wavenumbers from pi to 2*pi, with
    ``rhs_per_freq`` Gaussian patches shared by every frequency."""
    w = sphere_small()
    k = 2 * math.pi * (0.5 + 0.5 * np.arange(nfreq) / max(nfreq - 1, 1))
    w = Workload("sphere-1280-sweep", w.vertices, w.triangles, 2, w.dims, w.h,
                 2.0, k, 3000)
    w.extra["patches"] = patch_centres(w.vertices, w.triangles, rhs_per_freq, 3002)
    w.extra["sigma"] = 0.2
    w.extra["rhs_per_freq"] = rhs_per_freq
    return w


def sphere_large(level: int = 7) -> Workload:
    """Radius-6 icosphere (327,680 triangles at level 7), 256^3 grid,
    2nd-order stencil, near threshold 2h, k = 2*pi."""
    V, T = icosphere(level, 6.0)
    dims = (256, 256, 256)
    h = derived_spacing(V, dims)
    return Workload("sphere-327680", V, T, 2, dims, h, 2.0,
                    np.array([2 * math.pi]), 4000)


def efie_sphere(level: int = 6) -> Workload:
    """Radius-6 icosphere (81,920 triangles, 122,880 RWG functions at level
    6), 128^3 grid (h about lambda/10), 2nd-order stencil, near threshold 2h,
    k = 2*pi: the RWG EFIE's measured size."""
    V, T = icosphere(level, 6.0)
    dims = (128, 128, 128)
    h = derived_spacing(V, dims)
    return Workload(f"sphere-{T.shape[0]}-rwg", V, T, 2, dims, h, 2.0,
                    np.array([2 * math.pi]), 4100)


def sphere_tiny(level: int = 1, radius: float = 0.5, dims=(8, 8, 8), h: float = 0.2,
                k: float = 2 * math.pi) -> Workload:
    """Very small sphere for brute-force checks (80 triangles at level 1)."""
    V, T = icosphere(level, radius)
    return Workload(f"sphere-{T.shape[0]}", V, T, 2, tuple(dims), h, 2.0,
                    np.array([k]), 9000)


def small_box_array(seed: int = 7000) -> Workload:
    """2x1 array of 0.4x0.4x0.8 boxes meshed at edge 0.1 -- a small 3rd-order
    stencil case whose grid spans several FFT tiles with ragged sizes."""
    V, T = box_array(nx=2, ny=1, size=(0.4, 0.4, 0.8), gap=0.3, jitter=0.03,
                     edge=0.1, seed=seed)
    dims = (32, 16, 16)
    h = derived_spacing(V, dims)
    return Workload("boxarray-small", V, T, 3, dims, h, 3.0,
                    np.array([2 * math.pi]), seed)


def ellipsoid(level: int, radii, center=(0.0, 0.0, 0.0)):
    """Icosphere of the given level stretched to semi-axes ``radii``."""
    V, T = icosphere(level, 1.0)
    return V * np.asarray(radii, dtype=np.float64) + np.asarray(center, dtype=np.float64), T


def learned_pc_geometries(count: int, seed: int = 5004, level: int = 3,
                          k: float = 5.0) -> list:
    """Ellipsoids for the learned preconditioner: semi-axes drawn uniformly in
    [0.35, 0.6] with ``seed`` (training sets and held-out sets use different
    seeds), all on a 16^3 grid at h = 0.1 with 2nd-order stencils and a 2h
    near threshold, at wavenumber k."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        radii = rng.uniform(0.35, 0.6, size=3)
        V, T = ellipsoid(level, radii)
        out.append(Workload(f"ellipsoid-{seed}-{i}", V, T, 2, (16, 16, 16), 0.1, 2.0,
                            np.array([k]), seed, extra={"radii": radii}))
    return out


def _pow2_at_least(v: float, lo: int = 32, hi: int = 128) -> int:
    p = lo
    while p < v and p < hi:
        p *= 2
    return p


def sphere_resonance_margin(ka: float) -> float:
    """min over n <= ka + 5 of (ka)^2 |j_n(ka)| |h_n(ka)|.  The interior
    Dirichlet problem of a sphere of radius a resonates where j_n(ka) = 0;
    this measure is about |sin(ka - n pi/2)| for n well below ka and tends to
    zero at a resonance, so a draw with a small margin is rejected."""
    from scipy.special import spherical_jn, spherical_yn
    n = np.arange(int(ka + 5) + 1)
    j = spherical_jn(n, ka)
    y = spherical_yn(n, ka)
    return float(np.min(ka * ka * np.abs(j) * np.hypot(j, y)))


def box_resonance_gap(k: float, size) -> float:
    """Distance from k to the nearest interior Dirichlet wavenumber of a box
    with sides ``size`` (pi sqrt((l/a)^2 + (m/b)^2 + (n/c)^2), l, m, n >= 1),
    relative to the mean spacing of those wavenumbers near k (Weyl's law:
    about 2 pi^2 / (volume k^2)).  Small values mean a near-resonant draw."""
    a, b, c = (float(v) for v in size)
    lmax = [int(k * v / math.pi) + 2 for v in (a, b, c)]
    l = np.arange(1, lmax[0] + 1)[:, None, None] / a
    m = np.arange(1, lmax[1] + 1)[None, :, None] / b
    n = np.arange(1, lmax[2] + 1)[None, None, :] / c
    km = math.pi * np.sqrt(l * l + m * m + n * n)
    spacing = 2 * math.pi ** 2 / (a * b * c * k * k)
    return float(np.min(np.abs(km - k)) / spacing)


def uneven_batch(count: int = 32, seed: int = 5003, n_range=(5000, 120000)) -> list:
    """Uneven geometries for one batched solve.  Each instance draws a kind
    (icosphere of level 4-6, a box, or a 2x2 to 4x4 box array), a wavenumber
    k ~ U[2 pi, 6 pi] and an edge length ~ U[lambda/12, lambda/8], and is
    meshed at that edge, keeping 5k-120k triangles (draws outside the range
    are redrawn).  A sphere's radius follows from its level and edge, so ka
    varies continuously; draws near an interior resonance of the closed
    surface, where the single-layer operator is nearly singular, are redrawn:
    spheres need ``sphere_resonance_margin(ka) >= 0.15``, boxes (and each box
    of an array) ``box_resonance_gap >= 0.3`` of the local mode spacing.
    Grids are a power of two per axis (32-128 points, so 64-256 padded) with
    the spacing the library would derive for them, 2nd-order stencils and a
    2h near threshold."""
    rng = np.random.default_rng(seed)
    # mean edge of a unit-radius icosphere per level
    unit_edge = {}
    out = []
    while len(out) < count:
        kind = int(rng.integers(3))
        k = float(rng.uniform(2 * math.pi, 6 * math.pi))
        lam = 2 * math.pi / k
        edge = lam / float(rng.uniform(8.0, 12.0))
        if kind == 0:
            level = int(rng.integers(4, 7))
            if level not in unit_edge:
                V1, T1 = icosphere(level, 1.0)
                e = np.linalg.norm(V1[T1[:, 1]] - V1[T1[:, 0]], axis=1)
                unit_edge[level] = float(e.mean())
            radius = edge / unit_edge[level]
            if sphere_resonance_margin(k * radius) < 0.15:
                continue
            V, T = icosphere(level, radius)
            name = f"sphere-L{level}"
        elif kind == 1:
            size = rng.uniform(2.0, 8.0, size=3) * lam
            if box_resonance_gap(k, size) < 0.3:
                continue
            V, T = box_surface(np.zeros(3), size, edge)
            name = "box"
        else:
            nx, ny = (int(v) for v in rng.integers(2, 5, size=2))
            a, c = rng.uniform(1.0, 2.0) * lam, rng.uniform(2.0, 4.0) * lam
            bseed = int(rng.integers(1 << 30))
            if box_resonance_gap(k, (a, a, c)) < 0.3:
                continue
            V, T = box_array(nx, ny, size=(a, a, c), gap=0.5 * lam, jitter=0.05 * lam,
                             edge=edge, seed=bseed)
            name = f"boxarray-{nx}x{ny}"
        if not (n_range[0] <= T.shape[0] <= n_range[1]):
            continue
        ext = V.max(axis=0) - V.min(axis=0)
        dims = tuple(_pow2_at_least(ext[a] / edge + 6) for a in range(3))
        h = derived_spacing(V, dims)
        i = len(out)
        out.append(Workload(f"{name}-{T.shape[0]}", V, T, 2, dims, h, 2.0, np.array([k]),
                            seed * 100 + i, extra={"kind": name, "edge": edge}))
    return out
