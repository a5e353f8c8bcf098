"""Seeded synthetic inputs: closed PEC surface meshes and plane-wave excitations.

This module is the only code shared by the CPU oracle and the GPU library's
callers.  It produces *inputs* only (vertex/triangle arrays, incidence
directions, polarisation vectors, random vectors) and holds none of the
method's arithmetic: no basis functions, no Green's function, no quadrature.

Workloads stand in for the paper's plane-wave scattering from spheres
(Sec. VII, spheres of 0.2, 2 and 4 wavelengths): icospheres of radius 1 m and
cube-sphere families (sphere, ellipsoid, rounded cube) of a stated size.

All triangles are returned counter-clockwise seen from outside (outward
normal), with int32 vertex indices and float64 coordinates.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosphere", "cube_sphere", "spherical_frame", "planewave_set",
    "grid_planewaves", "random_directions", "uneven_batch", "complex_gaussian",
    "mean_edge_length",
]


def _orient_outward(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Flip triangles whose normal points towards the origin (star-shaped solids)."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, (a + b + c) / 3.0) < 0
    T = T.copy()
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def icosphere(level: int, radius: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Subdivided icosahedron projected onto a sphere.

    Level L has F = 20*4^L triangles and N = 30*4^L edges (RWG unknowns):
    level 2 -> 320 / 480, level 4 -> 5120 / 7680, level 5 -> 20480 / 30720.
    Each subdivision replaces a triangle by its 4 children stored consecutively,
    so triangle index order is hierarchical (spatially local).
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    tris = np.array(F, dtype=np.int64)
    tris = _orient_outward(np.array(verts), tris)
    for _ in range(level):
        mid: dict[tuple[int, int], int] = {}

        def midpoint(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key not in mid:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        new = []
        for a, b, c in tris:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            new += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = np.array(new, dtype=np.int64)
    Vout = np.array(verts, dtype=np.float64) * radius
    return Vout, tris.astype(np.int32)


def cube_sphere(n: int, family: str = "sphere", axes=(1.0, 1.0, 1.0),
                exponent: float = 6.0) -> tuple[np.ndarray, np.ndarray]:
    """Cube surface with an n x n grid per face, each quad split on a fixed diagonal,
    then mapped to a smooth closed surface.

    V = 6n^2 + 2, F = 12n^2, N = 18n^2.  Families:
      "sphere":    p / |p|_2
      "ellipsoid": sphere scaled by semi-axes `axes`
      "rounded_cube": p / |p|_e (superellipsoid, exponent e, default 6)
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    key_to_idx: dict[tuple[int, int, int], int] = {}
    pts: list[tuple[int, int, int]] = []

    def vid(ix: int, iy: int, iz: int) -> int:
        k = (ix, iy, iz)
        if k not in key_to_idx:
            key_to_idx[k] = len(pts)
            pts.append(k)
        return key_to_idx[k]

    tris = []
    # integer lattice coordinates in [-n, n] with step 2 (cube [-1,1]^3 scaled by n)
    faces = []
    for axis in range(3):
        for side in (-1, 1):
            faces.append((axis, side))
    for axis, side in faces:
        u_ax, v_ax = [a for a in range(3) if a != axis]
        grid = np.empty((n + 1, n + 1), dtype=np.int64)
        for i in range(n + 1):
            for j in range(n + 1):
                c = [0, 0, 0]
                c[axis] = side * n
                c[u_ax] = -n + 2 * i
                c[v_ax] = -n + 2 * j
                grid[i, j] = vid(*c)
        for i in range(n):
            for j in range(n):
                a, b, c_, d = grid[i, j], grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]
                tris.append((a, b, c_))
                tris.append((a, c_, d))
    P = np.array(pts, dtype=np.float64) / n
    if family in ("sphere", "ellipsoid"):
        Q = P / np.linalg.norm(P, axis=1, keepdims=True)
        if family == "ellipsoid":
            Q = Q * np.asarray(axes, dtype=np.float64)[None, :]
    elif family == "rounded_cube":
        Q = P / (np.sum(np.abs(P) ** exponent, axis=1, keepdims=True) ** (1.0 / exponent))
    else:
        raise ValueError(f"unknown family {family!r}")
    T = _orient_outward(Q, np.array(tris, dtype=np.int64))
    return Q, T.astype(np.int32)


def mean_edge_length(V: np.ndarray, T: np.ndarray) -> float:
    """Mean length over unique undirected edges."""
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.mean(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1)))


def spherical_frame(u: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """theta-hat and phi-hat unit vectors at unit direction(s) u (R x 3).

    At the poles phi is taken as 0, giving theta-hat = +-x-hat, phi-hat = y-hat.
    """
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    th = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    rho = np.hypot(u[:, 0], u[:, 1])
    ph = np.where(rho > 1e-15, np.arctan2(u[:, 1], u[:, 0]), 0.0)
    theta_hat = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=1)
    phi_hat = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=1)
    return theta_hat, phi_hat


def planewave_set(incidence: np.ndarray, pol: str | np.ndarray = "theta") -> tuple[np.ndarray, np.ndarray]:
    """Plane waves arriving *from* unit directions `incidence` (R x 3).

    Returns (dirs, pols): propagation direction d = -incidence and a real unit
    polarisation vector perpendicular to d.  `pol` is "theta", "phi", or an
    array of angles psi (radians) mixing theta-hat and phi-hat.
    """
    u = np.atleast_2d(np.asarray(incidence, dtype=np.float64))
    u = u / np.linalg.norm(u, axis=1, keepdims=True)
    th, ph = spherical_frame(u)
    if isinstance(pol, str):
        e = th if pol == "theta" else ph
    else:
        psi = np.asarray(pol, dtype=np.float64).reshape(-1, 1)
        e = np.cos(psi) * th + np.sin(psi) * ph
    return -u, e


def grid_planewaves(ntheta: int = 16, nphi: int = 16) -> tuple[np.ndarray, np.ndarray]:
    """theta_i = (i+1/2) pi / ntheta, phi_j = 2 pi j / nphi, times {theta-hat, phi-hat}.

    Returns 2*ntheta*nphi (dirs, pols), ordered (i, j, polarisation)."""
    dirs, pols = [], []
    for i in range(ntheta):
        t = (i + 0.5) * math.pi / ntheta
        for j in range(nphi):
            p = 2.0 * math.pi * j / nphi
            u = np.array([[math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)]])
            for which in ("theta", "phi"):
                d, e = planewave_set(u, which)
                dirs.append(d[0])
                pols.append(e[0])
    return np.array(dirs), np.array(pols)


def random_directions(count: int, seed: int) -> np.ndarray:
    """Uniform on S^2 as normalised standard Gaussian 3-vectors (numpy PCG64, seeded)."""
    g = np.random.default_rng(seed).standard_normal((count, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def complex_gaussian(n: int, seed: int, cols: int | None = None) -> np.ndarray:
    """Seeded standard complex Gaussian vector (n,) or block (cols, n), complex128."""
    rng = np.random.default_rng(seed)
    shape = (n,) if cols is None else (cols, n)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def uneven_batch(count: int = 64, seed: int = 4, nmin: int = 500, nmax: int = 6000,
                 edges_per_wavelength: float = 10.0, max_rhs: int = 32):
    """Uneven batch of closed PEC surfaces (spheres, ellipsoids, rounded cubes).

    Target N is log-uniform on [nmin, nmax]; the cube-sphere resolution is
    n = clamp(round(sqrt(N/18)), 6, 18) so N = 18 n^2.  Ellipsoid semi-axes are
    (1, r1, r2) with r_i ~ U[1, 3].  k = 2 pi / (edges_per_wavelength * mean edge).
    Each problem gets 1..max_rhs plane waves with incidence uniform on S^2 and a
    polarisation angle psi ~ U[0, 2 pi) in the (theta-hat, phi-hat) frame.
    """
    rng = np.random.default_rng(seed)
    fams = ("sphere", "ellipsoid", "rounded_cube")
    out = []
    for _ in range(count):
        target = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        n = int(min(18, max(6, round(math.sqrt(target / 18.0)))))
        fam = fams[int(rng.integers(0, 3))]
        axes = (1.0, float(rng.uniform(1, 3)), float(rng.uniform(1, 3)))
        V, T = cube_sphere(n, fam, axes=axes)
        h = mean_edge_length(V, T)
        k = 2.0 * math.pi / (edges_per_wavelength * h)
        nrhs = int(rng.integers(1, max_rhs + 1))
        g = rng.standard_normal((nrhs, 3))
        inc = g / np.linalg.norm(g, axis=1, keepdims=True)
        psi = rng.uniform(0.0, 2.0 * math.pi, nrhs)
        dirs, pols = planewave_set(inc, psi)
        out.append(dict(family=fam, n=n, axes=axes, V=V, T=T, k=k, dirs=dirs, pols=pols))
    return out
