"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generation only: triangulated spheres and ellipsoids,
incident-wave parameters, random vectors, problem mixes and arrival streams.
It contains none of the method's arithmetic (no kernels, quadrature,
frequencies or transforms), so both the oracle and the GPU path may use it
without sharing method code.

The paper's test geometry is a polyhedral approximation of the unit sphere
built from flat triangles (Section 7.1); the icosphere below is such a
polyhedron, refined by midpoint subdivision with projection to the sphere.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DEFAULT_SEED = 20060518


def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def icosphere(level: int):
    """Unit-sphere polyhedron with 20*4**level flat triangles.

    Returns (vertices float64 (nv,3), triangles int32 (M,3)); triangles are
    ordered counter-clockwise seen from outside (outward normals).
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = (np.asarray(verts[a]) + np.asarray(verts[b])) * 0.5
                p /= np.linalg.norm(p)
                verts.append(tuple(p))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.asarray(nf, dtype=np.int64)
    V = np.asarray(verts, dtype=np.float64)
    # orient outward
    P = V[f]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    flip = np.einsum("ij,ij->i", n, P.mean(axis=1)) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return V, f.astype(np.int32)


def ellipsoid(level: int, axes):
    """Icosphere scaled by the semi-axes (a, b, c)."""
    V, T = icosphere(level)
    return V * np.asarray(axes, dtype=np.float64)[None, :], T


def two_spheres(level: int, distance: float = 6.0):
    """Two unit icospheres with centres `distance` apart on the x axis (two
    scatterers; far apart, their clusters form large admissible blocks)."""
    V, T = icosphere(level)
    V2 = V + np.asarray([distance, 0.0, 0.0])[None, :]
    return np.concatenate([V, V2]), np.concatenate([T, T + len(V)]).astype(np.int32)


def level_for_triangles(M: int) -> int:
    for k in range(0, 8):
        if 20 * 4 ** k == M:
            return k
    raise ValueError(f"no icosphere level has {M} triangles")


@dataclasses.dataclass
class PlaneWave:
    """Gaussian-pulse plane wave u(x,t) = A exp(-((t - x.d - t0)/sigma)^2)."""
    direction: tuple = (1.0, 0.0, 0.0)
    sigma: float = 0.25
    t0: float = 1.5
    amplitude: float = 1.0


@dataclasses.dataclass
class Workload:
    name: str
    level: int
    N: int
    T: float
    wave: PlaneWave
    axes: tuple = (1.0, 1.0, 1.0)

    @property
    def M(self) -> int:
        return 20 * 4 ** self.level

    def mesh(self):
        if self.axes == (1.0, 1.0, 1.0):
            return icosphere(self.level)
        return ellipsoid(self.level, self.axes)


# The five synthetic workloads (sphere sizes, step counts and pulse of the
# benchmark configurations).
C1 = Workload("sphere320_N32_T4", 2, 32, 4.0, PlaneWave())
C2 = Workload("sphere1280_N64_T4", 3, 64, 4.0, PlaneWave())
C3 = Workload("sphere5120_N128_T6", 4, 128, 6.0, PlaneWave())
C5_LARGE = Workload("sphere20480_N256_T6", 5, 256, 6.0, PlaneWave())
C0_TINY = Workload("sphere80_N8_T2", 1, 8, 2.0, PlaneWave())


def random_direction(rng):
    d = rng.standard_normal(3)
    return tuple((d / np.linalg.norm(d)).tolist())


def problem_mix(count: int = 48, seed: int = DEFAULT_SEED, levels=(1, 2, 3, 4),
                steps=(16, 32, 64, 128), T: float = 4.0):
    """Uneven batch of independent problems: spheres or ellipsoids of
    random refinement level, random step count, direction and pulse width."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        level = int(rng.choice(levels))
        N = int(rng.choice(steps))
        if rng.random() < 0.5:
            axes = (1.0, 1.0, 1.0)
        else:
            axes = tuple(float(a) for a in rng.uniform(0.5, 1.5, size=3))
        sigma = float(rng.uniform(0.2, 0.4))
        t0 = max(axes) + 2.0 * sigma
        wave = PlaneWave(random_direction(rng), sigma, t0, 1.0)
        out.append(Workload(f"mix{k}_L{level}_N{N}", level, N, T, wave, axes))
    return out


def poisson_arrivals(rate: float, duration: float, seed: int = DEFAULT_SEED):
    """Arrival times (seconds) of a Poisson stream of the given rate."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.asarray(out)
        out.append(t)


def random_complex(shape, seed: int = DEFAULT_SEED, dtype=np.complex128):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return z.astype(dtype)
