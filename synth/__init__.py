"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module draws random numbers and builds random 1D vessel trees.  It holds
none of the method's arithmetic (no assembly, no solver, no network): both the
oracle and the HIP library receive its arrays as plain inputs.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), with doubles formed from the
top 53 bits of each output.

The paper draws its graphs from its own (unpublished) dataset: trees with O(1)
to O(10^2) branches inside the unit cube (Section 5.1).  The generator below
produces trees of that shape: root at the cube centre, straight segments of
length U[0.1, 0.25], directions uniform on the sphere, every vertex kept
inside [0.2, 0.8]^3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator; `next_u64` follows the published definition."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform in [lo, hi] inclusive."""
        return lo + min(int(self.uniform() * (hi - lo + 1)), hi - lo)

    def normal_array(self, n: int) -> np.ndarray:
        """n standard normals by the Box-Muller transform (float64)."""
        m = (n + 1) // 2
        u = np.array([self.uniform() for _ in range(2 * m)], dtype=np.float64)
        u1 = 1.0 - u[0::2]  # (0, 1]
        u2 = u[1::2]
        rad = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([rad * np.cos(2 * math.pi * u2), rad * np.sin(2 * math.pi * u2)])
        return z[:n]


def fast_normal(seed: int, n: int) -> np.ndarray:
    """Many standard normals quickly (numpy PCG64 seeded from SplitMix64).

    Used for large random test vectors where drawing through the pure-Python
    generator would be slow; the seed still comes from SplitMix64 so every
    vector is reproducible from one integer.
    """
    s = SplitMix64(seed).next_u64()
    return np.random.Generator(np.random.PCG64(s)).standard_normal(n)


@dataclass
class Instance:
    """One parameter instance mu: a 3D grid size plus a 1D vessel tree.

    vertex_xyz[V,3]    vertex coordinates in the unit cube, vertex 0 = root
    seg[S,2]           (parent vertex, child vertex) per segment
    radius[S], beta[S] vessel radius R and wall permeability per segment
    """
    n_cells: int
    vertex_xyz: np.ndarray
    seg: np.ndarray
    radius: np.ndarray
    beta: np.ndarray
    elems_per_segment: int
    k_omega: float = 1.0
    sigma_omega: float = 0.0
    k_lambda: float = 1.0
    f_lambda: float = 1.0
    n_circle: int = 16
    seed: int = 0
    meta: dict = field(default_factory=dict)
    boundary: str = "dirichlet"    # cube faces: "dirichlet" (u = 0) or "neumann" (natural)
    problem: str = "coupled"       # "coupled" system, or "block3d": the 3D block alone

    @property
    def n_segments(self) -> int:
        return int(self.seg.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.vertex_xyz.shape[0])


BOX_LO, BOX_HI = 0.2, 0.8


def random_tree(rng: SplitMix64, n_segments: int, max_tries: int = 64):
    """Grow a random tree of straight segments.

    For each new segment: pick a parent uniformly among existing vertices;
    draw length L = 0.1 + 0.15 u and a direction uniform on the sphere
    (Archimedes: z = 2u - 1, phi = 2 pi u); accept the end point if it lies in
    [0.2, 0.8]^3, otherwise redraw length and direction (up to `max_tries`),
    then redraw the parent.
    """
    verts = [(0.5, 0.5, 0.5)]
    segs = []
    for _ in range(n_segments):
        while True:
            parent = min(int(rng.uniform() * len(verts)), len(verts) - 1)
            p = verts[parent]
            placed = False
            for _t in range(max_tries):
                length = 0.1 + 0.15 * rng.uniform()
                z = 2.0 * rng.uniform() - 1.0
                phi = 2.0 * math.pi * rng.uniform()
                rxy = math.sqrt(max(0.0, 1.0 - z * z))
                d = (rxy * math.cos(phi), rxy * math.sin(phi), z)
                q = (p[0] + length * d[0], p[1] + length * d[1], p[2] + length * d[2])
                if all(BOX_LO <= c <= BOX_HI for c in q):
                    verts.append(q)
                    segs.append((parent, len(verts) - 1))
                    placed = True
                    break
            if placed:
                break
    return np.array(verts, dtype=np.float64), np.array(segs, dtype=np.int32)


def make_instance(seed: int, n_cells: int, n_segments: int | None = None,
                  seg_range: tuple[int, int] | None = None, elems_per_segment: int = 8,
                  radius: float | tuple[float, float] = 0.005,
                  beta: float | tuple[float, float] = 1.0, **kw) -> Instance:
    """Seeded instance.  A tuple for `radius` draws one R per instance from
    U[lo, hi]; a tuple for `beta` draws one beta per segment from U[lo, hi]."""
    rng = SplitMix64(seed)
    if n_segments is None:
        lo, hi = seg_range
        n_segments = rng.randint(lo, hi)
    v, s = random_tree(rng, n_segments)
    if isinstance(radius, tuple):
        r = radius[0] + (radius[1] - radius[0]) * rng.uniform()
    else:
        r = float(radius)
    rad = np.full(n_segments, r, dtype=np.float64)
    if isinstance(beta, tuple):
        b = np.array([beta[0] + (beta[1] - beta[0]) * rng.uniform() for _ in range(n_segments)])
    else:
        b = np.full(n_segments, float(beta))
    return Instance(n_cells=n_cells, vertex_xyz=v, seg=s, radius=rad, beta=b,
                    elems_per_segment=elems_per_segment, seed=seed, **kw)


# Workload recipes (sizes of the paper's experiments mapped onto the Q1 grids
# used here).  Each returns a list of instances.

def workload_single_fp64():
    """16^3 cells, one tree of 8 segments x 4 elements, R=0.01, beta=1."""
    return [make_instance(1, 16, n_segments=8, elems_per_segment=4, radius=0.01, beta=1.0)]


def workload_single_32():
    """32^3 cells, one tree of 64 segments x 8 elements, R=0.005, beta~U[0.5,2]."""
    return [make_instance(2, 32, n_segments=64, elems_per_segment=8, radius=0.005, beta=(0.5, 2.0))]


def workload_batched_32(count: int = 256):
    """count instances at 32^3, segments ~U{8..128}, R~U[0.003,0.01], 8 elems/segment."""
    return [make_instance(1_000_000 + i, 32, seg_range=(8, 128), elems_per_segment=8,
                          radius=(0.003, 0.01), beta=1.0) for i in range(count)]


def workload_transfer(n_cells: int = 64, count: int | None = None):
    """64^3 (16 instances) or 128^3 (2 instances): 512 segments x 16 elements, R=0.002."""
    if n_cells == 64:
        base, cnt = 2_000_000, 16 if count is None else count
    else:
        base, cnt = 3_000_000, 2 if count is None else count
    return [make_instance(base + i, n_cells, n_segments=512, elems_per_segment=16,
                          radius=0.002, beta=1.0) for i in range(cnt)]


def workload_block3d(n_cells: int = 20, count: int = 16, base: int = 4_000_000):
    """The 3D-block problem of the paper's Section 5 setup: unit cube with
    natural (Neumann) boundary, k_Omega = sigma_Omega = 1e-3, vessel radius
    eps = 1e-3 (beta = 1), trees of 2-96 segments (O(1) to O(10^2) branches),
    P1 elements of about the grid spacing (n_cells / 5 per segment); grids of
    21^3, 41^3, 81^3 nodes for n_cells = 20, 40, 80."""
    E = max(2, n_cells // 5)
    return [make_instance(base + 1000 * n_cells + i, n_cells, seg_range=(2, 96), elems_per_segment=E,
                          radius=1e-3, beta=1.0, k_omega=1e-3, sigma_omega=1e-3, boundary="neumann",
                          problem="block3d") for i in range(count)]


def workload_training_block3d(count: int, n_cells: int = 20, base: int = 30_000):
    """Training graphs of the 3D-block problem (disjoint seeds from the test
    graphs of `workload_block3d`)."""
    E = max(2, n_cells // 5)
    return [make_instance(base + k, n_cells, seg_range=(2, 96), elems_per_segment=E, radius=1e-3, beta=1.0,
                          k_omega=1e-3, sigma_omega=1e-3, boundary="neumann", problem="block3d")
            for k in range(count)]


def workload_training(count: int, n_cells: int = 32, base: int = 10_000):
    """Training graphs: segments ~U{16..128}, R~U[0.002,0.01], beta~U[0.5,2] per segment."""
    return [make_instance(base + k, n_cells, seg_range=(16, 128), elems_per_segment=8,
                          radius=(0.002, 0.01), beta=(0.5, 2.0)) for k in range(count)]


def random_unit_vectors(seed: int, count: int, n: int) -> np.ndarray:
    """count x n random unit vectors, v ~ N(0, I) normalised."""
    out = np.empty((count, n))
    for c in range(count):
        v = fast_normal(seed * 7919 + c, n)
        out[c] = v / np.linalg.norm(v)
    return out
