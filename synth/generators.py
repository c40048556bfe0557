"""Counter-based seeded generators for the point-cloud workloads.

Every random number is splitmix64 applied to a 64-bit counter built as
``(seed << 40) | (stream << 32) | index``, so any element can be regenerated on its
own and no generator state is carried between calls.  A uniform double on the
53-bit grid is ``(x >> 11) * 2**-53`` in [0, 1).

Workloads (the paper measures on random uniform points, Sec. 2.7 and Sec. 3.7):

* ``uniform_points``  -- i.i.d. uniform in [0, 1)^3, coordinates on the 2^-53 grid.
* ``lattice_points``  -- distinct nodes of a side^3 grid drawn without replacement,
  coordinates (2 i - (side - 1)) / 512 (exact dyadic values, massively cospherical).
* ``cluster_points``  -- anisotropic Gaussian clusters: centres uniform in the ball of
  radius 0.9, per-axis sigma log-uniform in [0.002, 0.05], random rotation.
* ``shell_points``    -- directions uniform on the unit sphere, radius uniform in
  [1 - 1e-4, 1 + 1e-4].
* ``mix_points``      -- lattice + clusters + shell, shuffled.
* ``batch_clouds``    -- many independent clouds, sizes log-uniform, each uniform in
  its own axis-aligned box.
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 2.0 ** -53


def splitmix64(counters: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser of each 64-bit counter (vectorised, wrapping arithmetic)."""
    z = np.asarray(counters, dtype=np.uint64) + _GOLD
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
    return z ^ (z >> np.uint64(31))


def _counters(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    if not (0 <= seed < (1 << 24)) or not (0 <= stream < 256):
        raise ValueError("seed must be < 2^24 and stream < 256")
    if start + count > (1 << 32):
        raise ValueError("a stream holds at most 2^32 draws")
    base = (np.uint64(seed) << np.uint64(40)) | (np.uint64(stream) << np.uint64(32))
    return base + np.arange(start, start + count, dtype=np.uint64)


def _unit(seed: int, stream: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) on the 2^-53 grid."""
    return (splitmix64(_counters(seed, stream, count)) >> np.uint64(11)).astype(np.float64) * _TWO_M53


def _gauss(seed: int, stream: int, count: int) -> np.ndarray:
    """Standard normal draws by the Box-Muller transform of two uniform streams."""
    m = (count + 1) // 2
    u = _unit(seed, stream, 2 * m).reshape(m, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
    t = 2.0 * np.pi * u[:, 1]
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1).reshape(-1)[:count]


def uniform_points(n: int, seed: int) -> np.ndarray:
    """n x 3 fp64 points, i.i.d. uniform in [0, 1)^3."""
    return _unit(seed, 0, 3 * int(n)).reshape(int(n), 3)


def lattice_points(n: int, seed: int, side: int = 160) -> np.ndarray:
    """n distinct nodes of a side^3 lattice, coordinates (2 i - (side - 1)) / 512."""
    total = side ** 3
    if n > total:
        raise ValueError("more lattice points than nodes")
    keys = splitmix64(_counters(seed, 1, total))
    nodes = np.argsort(keys, kind="stable")[: int(n)].astype(np.int64)
    i, rem = np.divmod(nodes, side * side)
    j, k = np.divmod(rem, side)
    ijk = np.stack([i, j, k], axis=1).astype(np.float64)
    return (2.0 * ijk - (side - 1)) / 512.0


def _rotation(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def cluster_points(n: int, seed: int, clusters: int = 50) -> np.ndarray:
    """n points in `clusters` anisotropic, randomly rotated Gaussian clusters."""
    n = int(n)
    g = _gauss(seed, 2, 7 * clusters).reshape(clusters, 7)
    u = _unit(seed, 3, 4 * clusters).reshape(clusters, 4)
    dirs = g[:, 0:3] / np.linalg.norm(g[:, 0:3], axis=1, keepdims=True)
    centres = dirs * (0.9 * np.cbrt(u[:, 0:1]))
    lo, hi = np.log(0.002), np.log(0.05)
    sigmas = np.exp(lo + u[:, 1:4] * (hi - lo))
    sizes = np.full(clusters, n // clusters, dtype=np.int64)
    sizes[: n % clusters] += 1
    z = _gauss(seed, 4, 3 * n).reshape(n, 3)
    out = np.empty((n, 3))
    start = 0
    for c in range(clusters):
        s = int(sizes[c])
        rot = _rotation(g[c, 3:7])
        out[start:start + s] = centres[c] + (z[start:start + s] * sigmas[c]) @ rot.T
        start += s
    return out


def shell_points(n: int, seed: int, thickness: float = 1e-4) -> np.ndarray:
    """n points with uniform directions and radius uniform in [1 - t, 1 + t]."""
    n = int(n)
    g = _gauss(seed, 5, 3 * n).reshape(n, 3)
    r = 1.0 + (2.0 * _unit(seed, 6, n) - 1.0) * thickness
    return g / np.linalg.norm(g, axis=1, keepdims=True) * r[:, None]


def mix_points(seed: int, n_lattice: int = 4_000_000, n_clusters: int = 3_000_000,
               n_shell: int = 3_000_000, side: int = 160) -> np.ndarray:
    """Lattice + clusters + shell, shuffled by a seeded permutation."""
    pts = np.concatenate([
        lattice_points(n_lattice, seed, side),
        cluster_points(n_clusters, seed),
        shell_points(n_shell, seed),
    ])
    perm = np.argsort(splitmix64(_counters(seed, 7, len(pts))), kind="stable")
    return np.ascontiguousarray(pts[perm])


def batch_clouds(num: int, seed_base: int = 3000, nmin: float = 1e3, nmax: float = 2e5):
    """`num` independent clouds; cloud c uses seed seed_base + c.

    Returns (points, offsets): points of cloud c are points[offsets[c]:offsets[c+1]].
    """
    clouds = []
    for c in range(num):
        s = seed_base + c
        u = _unit(s, 8, 7)
        nc = int(round(np.exp(np.log(nmin) + u[0] * (np.log(nmax) - np.log(nmin)))))
        lo = -10.0 + 20.0 * u[1:4]
        ext = np.exp(np.log(0.1) + u[4:7] * (np.log(10.0) - np.log(0.1)))
        clouds.append(lo + uniform_points(nc, s) * ext)
    offsets = np.zeros(num + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum([len(c) for c in clouds])
    return np.concatenate(clouds), offsets
