"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and shapes them into point clouds and
right-hand sides. It holds none of the sparsification arithmetic: the
oracle and the HIP library both receive its arrays as plain inputs.

Generator: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  The i-th draw of a stream with seed
``s`` (i = 1, 2, ...) is ``mix(s + i * 0x9E3779B97F4A7C15)``; a uniform
double is ``(x >> 11) * 2**-53`` in [0, 1); normals use Box-Muller.

Workloads follow the paper's experiments: points spread uniformly in the
unit square / cube (Section 5, Examples 5.1-5.2 and the preconditioning
example) and, as a stand-in for the boundary-element surface of the cube
(Section 5.4), points spread uniformly on 2-manifolds (sphere, torus).
"""

from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws ``start+1 .. start+count`` of the splitmix64 stream ``seed``."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits each."""
    x = splitmix64(seed, count, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller on consecutive uniform pairs."""
    half = (count + 1) // 2
    u = uniform(seed, 2 * half)
    u1 = 1.0 - u[0::2]  # (0, 1]
    u2 = u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * half)
    z[0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:count]


def points_square(n: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1]^2, row-major (n, 2)."""
    return uniform(seed, 2 * n).reshape(n, 2)


def points_cube(n: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1]^3, row-major (n, 3)."""
    return uniform(seed, 3 * n).reshape(n, 3)


def points_sphere(n: int, seed: int) -> np.ndarray:
    """n points uniform on the unit sphere surface: g / |g|, g ~ N(0, I3)."""
    g = normal(seed, 3 * n).reshape(n, 3)
    nrm = np.sqrt((g * g).sum(axis=1))
    return g / nrm[:, None]


def points_torus(n: int, seed: int, big_r: float = 1.0, small_r: float = 0.35) -> np.ndarray:
    """n points area-uniform on a torus surface (rejection on the angle theta)."""
    out = np.empty((n, 3))
    got = 0
    start = 0
    while got < n:
        batch = max(64, 2 * (n - got))
        u = uniform(seed, 3 * batch, start=start).reshape(batch, 3)
        start += 3 * batch
        theta = 2.0 * np.pi * u[:, 0]
        phi = 2.0 * np.pi * u[:, 1]
        keep = u[:, 2] * (big_r + small_r) <= big_r + small_r * np.cos(theta)
        theta, phi = theta[keep], phi[keep]
        take = min(n - got, theta.size)
        theta, phi = theta[:take], phi[:take]
        ring = big_r + small_r * np.cos(theta)
        out[got:got + take, 0] = ring * np.cos(phi)
        out[got:got + take, 1] = ring * np.sin(phi)
        out[got:got + take, 2] = small_r * np.sin(theta)
        got += take
    return out


POINT_KINDS = {
    "square": points_square,
    "cube": points_cube,
    "sphere": points_sphere,
    "torus": points_torus,
}


def points(kind: str, n: int, seed: int) -> np.ndarray:
    return POINT_KINDS[kind](n, seed)


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides ~N(0,1), column-major n x nrhs (Fortran-ordered array).

    The stream is ``seed + 1_000_000`` so that it never overlaps the points.
    """
    z = normal(seed + 1_000_000, n * nrhs)
    return np.asfortranarray(z.reshape(nrhs, n).T)


def batch_instances(count: int = 64, seed: int = 4):
    """Instance list of the batched workload: (kind, N, leaf, seed) per instance.

    N is log-uniform in [4096, 65536], the kind cycles cube/sphere/torus and the
    leaf size is uniform in [32, 64].
    """
    u = uniform(seed, 2 * count).reshape(count, 2)
    kinds = ("cube", "sphere", "torus")
    out = []
    for i in range(count):
        n_i = int(round(np.exp(np.log(4096.0) + u[i, 0] * np.log(16.0))))
        leaf_i = 32 + int(np.floor(33.0 * u[i, 1]))
        out.append((kinds[i % 3], n_i, min(leaf_i, 64), 4000 + i))
    return out


# Named workloads.  "kernel_scale" c gives A_ij = c / |x_i - x_j| (i != j),
# A_ii = 1.  Sizes follow the configurations the method is benchmarked on.
WORKLOADS = {
    "square1k": dict(kind="square", n=1024, seed=1, leaf=32, cheb=4, tol=0.0,
                     rank_cap=16, nrhs=1, scale="1/N"),
    "sphere64k": dict(kind="sphere", n=65536, seed=2, leaf=64, cheb=3, tol=1e-8,
                      rank_cap=27, nrhs=16, scale="1/(4piN)"),
    "cube256k": dict(kind="cube", n=262144, seed=3, leaf=64, cheb=4, tol=1e-8,
                     rank_cap=48, nrhs=32, scale="1/(4piN)"),
    "cube1m": dict(kind="cube", n=1048576, seed=5, leaf=128, cheb=4, tol=1e-8,
                   rank_cap=64, nrhs=128, scale="1/(4piN)"),
    # the exp core of Example 5.2: 2 delta_ij + exp(-|r_i - r_j|^2) on the unit cube
    "cube64k_exp": dict(kind="cube", n=65536, seed=6, leaf=64, cheb=4, tol=1e-8,
                        rank_cap=48, nrhs=16, scale="1", kernel="exp", diag=3.0),
}


def kernel_scale(spec: str, n: int) -> float:
    if spec == "1":
        return 1.0
    if spec == "1/N":
        return 1.0 / n
    if spec == "1/(4piN)":
        return 1.0 / (4.0 * np.pi * n)
    raise ValueError(spec)
