"""Seeded synthetic point clouds for the Vietoris-Rips filtration front end.

This module only draws inputs: integer point coordinates and a threshold
specification.  It computes no distance, rank, triangle or any other step of
the method, so both the CPU oracle and the HIP path can consume the same bytes
without sharing any of the method's arithmetic.

Threshold specifications are tuples ``(kind, num, den)`` with kind one of
``"full"``, ``"count"``, ``"fraction"`` (num/den of the edges, floored) and
``"sqdist"`` (keep squared distance strictly below num).

The shapes stand in for the paper's benchmarks (Section 4, Section 5): sphere
and torus samples for the WorldMap/Dragon surface data, Gaussian mixtures for
the high-dimensional HIV/Klein data, and uniform planar points at full
threshold for the default "Inf" setting.  None of the paper's datasets is used
or reproduced.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Cloud",
    "quantize_i8",
    "plain64",
    "noisy_circle",
    "mixture",
    "batched",
    "serving_stream",
    "uniform_cloud",
    "lattice_cloud",
    "CONFIGS",
    "config",
]


@dataclass
class Cloud:
    """One build request: row-major points plus a threshold specification."""

    points: np.ndarray  # (n, d) int8 or int32, C-contiguous
    thr: tuple  # (kind, num, den)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def d(self) -> int:
        return int(self.points.shape[1])


def quantize_i8(x: np.ndarray) -> np.ndarray:
    """Round half to even, clip to [-127, 127], cast to int8 (row-major)."""
    return np.ascontiguousarray(np.clip(np.rint(x), -127, 127).astype(np.int8))


def plain64(seed: int = 1, n: int = 64) -> Cloud:
    """64 points in Z^2, coordinates uniform in [0, 1023], full threshold."""
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, 1024, (n, 2), dtype=np.int32)
    return Cloud(np.ascontiguousarray(pts), ("full", 0, 1), name=f"plain{n}_r2_full")


def _circle_xyz(rng, n, radius, sigma, planar=False):
    theta = rng.uniform(0.0, 2.0 * math.pi, n)
    if planar:
        noise = rng.normal(0.0, sigma, (n, 2))
        base = np.stack([radius * np.cos(theta), radius * np.sin(theta)], axis=1)
    else:
        noise = rng.normal(0.0, sigma, (n, 3))
        base = np.stack([radius * np.cos(theta), radius * np.sin(theta), np.zeros(n)], axis=1)
    return base + noise


def noisy_circle(seed: int = 2, n: int = 1000, pct_num: int = 20, pct_den: int = 100) -> Cloud:
    """Radius-100 circle in R^3 plus N(0, 5^2) noise, int8, 20th-percentile edge rank."""
    rng = np.random.default_rng(seed)
    pts = quantize_i8(_circle_xyz(rng, n, 100.0, 5.0))
    return Cloud(pts, ("fraction", pct_num, pct_den), name=f"circle{n}_r3_p{pct_num}")


def _mixture_points(rng, n, d, components=8, sigma=12.0):
    mu = rng.integers(-80, 81, (components, d)).astype(np.float64)
    comp = rng.integers(0, components, n)
    noise = rng.normal(0.0, sigma, (n, d))
    return quantize_i8(mu[comp] + noise)


def mixture(seed: int = 3, n: int = 4000, d: int = 64, pct_num: int = 10, pct_den: int = 100) -> Cloud:
    """8-component Gaussian mixture in R^64 (centres in [-80, 80], sigma 12), int8, 10th percentile."""
    rng = np.random.default_rng(seed)
    pts = _mixture_points(rng, n, d)
    return Cloud(pts, ("fraction", pct_num, pct_den), name=f"mixture{n}_r{d}_p{pct_num}")


def _sphere(rng, n, radius=100.0, sigma=3.0):
    v = rng.normal(0.0, 1.0, (n, 3))
    v /= np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-12)
    return radius * v + rng.normal(0.0, sigma, (n, 3))


def _torus(rng, n, big=80.0, small=30.0, sigma=3.0):
    u = rng.uniform(0.0, 2.0 * math.pi, n)
    v = rng.uniform(0.0, 2.0 * math.pi, n)
    x = (big + small * np.cos(v)) * np.cos(u)
    y = (big + small * np.cos(v)) * np.sin(u)
    z = small * np.sin(v)
    return np.stack([x, y, z], axis=1) + rng.normal(0.0, sigma, (n, 3))


def _shape3(rng, kind, n):
    if kind == 0:
        return _circle_xyz(rng, n, 100.0, 5.0)
    if kind == 1:
        return _sphere(rng, n)
    return _torus(rng, n)


def batched(seed: int = 4, clouds: int = 512, nmin: int = 50, nmax: int = 2000,
            bp_lo: int = 500, bp_hi: int = 2500) -> list[Cloud]:
    """Many R^3 clouds: n log-uniform in [nmin, nmax], threshold u/10^4 of the edges."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(clouds):
        n = int(math.floor(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        u = int(rng.integers(bp_lo, bp_hi + 1))
        pts = quantize_i8(_shape3(rng, c % 3, n))
        out.append(Cloud(pts, ("fraction", u, 10000), name=f"batch{c}", meta={"shape": c % 3}))
    return out


def serving_stream(seed: int = 5, requests: int = 2000, qps: float = 100.0,
                   nmin: int = 100, nmax: int = 5000, bp_lo: int = 500, bp_hi: int = 2000):
    """Poisson request stream: list of (arrival_seconds, Cloud).

    n log-uniform in [nmin, nmax], d uniform in {2, 3, 16, 64}; d=2 planar noisy
    circle, d=3 the circle/sphere/torus mix, d in {16, 64} the Gaussian mixture.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(requests):
        t += float(rng.exponential(1.0 / qps))
        n = int(math.floor(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        d = int((2, 3, 16, 64)[int(rng.integers(0, 4))])
        u = int(rng.integers(bp_lo, bp_hi + 1))
        if d == 2:
            pts = quantize_i8(_circle_xyz(rng, n, 100.0, 5.0, planar=True))
        elif d == 3:
            pts = quantize_i8(_shape3(rng, int(rng.integers(0, 3)), n))
        else:
            pts = _mixture_points(rng, n, d)
        out.append((t, Cloud(pts, ("fraction", u, 10000), name=f"req{r}", meta={"d": d})))
    return out


def sphere_cloud(seed: int, n: int, thr=("fraction", 15, 100)) -> Cloud:
    """n points near a sphere of radius 100 in R^3 (noise 3), int8: a cloud
    whose complex holds a class of dimension 2."""
    rng = np.random.default_rng(seed)
    return Cloud(quantize_i8(_sphere(rng, n)), thr, name=f"sphere{n}_s{seed}")


def uniform_cloud(seed: int, n: int, d: int, lo: int = -127, hi: int = 127,
                  dtype=np.int8, thr=("full", 0, 1)) -> Cloud:
    """Uniform integer points, for tests of arbitrary shapes and dtypes."""
    rng = np.random.default_rng(seed)
    pts = rng.integers(lo, hi + 1, (n, d)).astype(dtype)
    return Cloud(np.ascontiguousarray(pts), thr, name=f"uniform{n}x{d}_s{seed}")


def hamming_matrix(seed: int, n: int, bits: int = 96, flip: float = 0.1, clusters: int = 6):
    """Pairwise Hamming distances (int32 n x n) of n binary sequences of
    `bits` bits drawn around a few random centre sequences (each bit flipped
    with probability `flip`): a stand-in for sequence data such as the
    paper's HIV example, which uses Hamming distances."""
    rng = np.random.default_rng(seed)
    centres = rng.integers(0, 2, (clusters, bits), dtype=np.int8)
    seqs = centres[rng.integers(0, clusters, n)] ^ (rng.random((n, bits)) < flip).astype(np.int8)
    m = (seqs[:, None, :] != seqs[None, :, :]).sum(-1).astype(np.int32)
    return np.ascontiguousarray(m)


def csc_columns(seed: int, ncols: int, mean_len: float, maxvalue: int, empty: float = 0.1,
                long_cols: int = 0, long_len: int = 0, lo: int = 0):
    """A compressed-sparse-column array (colptr int64, v int32): column
    lengths geometric with the given mean, a fraction `empty` of the columns
    empty, `long_cols` columns of `long_len` entries at random places, values
    uniform in lo..lo+maxvalue (ties wherever the range is small)."""
    rng = np.random.default_rng(seed)
    lens = rng.geometric(1.0 / max(mean_len, 1.0), ncols).astype(np.int64) if ncols else np.zeros(0, np.int64)
    lens[rng.random(ncols) < empty] = 0
    if long_cols and ncols:
        lens[rng.choice(ncols, min(long_cols, ncols), replace=False)] = long_len
    colptr = np.zeros(ncols + 1, np.int64)
    np.cumsum(lens, out=colptr[1:])
    v = rng.integers(lo, lo + maxvalue + 1, int(colptr[-1]), dtype=np.int64).astype(np.int32)
    return colptr, v


def full_columns(seed: int, ncols: int, length: int, maxvalue: int):
    """ncols columns of `length` entries each, values uniform in 0..maxvalue:
    the shape of a complete graph's rank matrix stored by column."""
    rng = np.random.default_rng(seed)
    colptr = np.arange(ncols + 1, dtype=np.int64) * length
    v = rng.integers(0, maxvalue + 1, ncols * length, dtype=np.int64).astype(np.int32)
    return colptr, v


def hub_pair(seed: int = 101, m: int = 300, d: int = 64, h: float = 40.0, s: float = 66.8) -> np.ndarray:
    """Two hub points (-h, 0, ...) and (h, 0, ...) and m points at radius s in
    the hyperplane between them (random directions in R^(d-1)), int8.  Under
    a squared-distance threshold between 4h^2 and the typical distance of two
    hyperplane points, every hyperplane point joins both hubs by an edge
    shorter than the hub edge, while few hyperplane points join each other:
    the hub edge has m common older neighbours, with few tetrahedra."""
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((m, d - 1))
    y *= s / np.linalg.norm(y, axis=1, keepdims=True)
    pts = np.zeros((m + 2, d))
    pts[0, 0], pts[1, 0] = -h, h
    pts[2:, 1:] = y
    return quantize_i8(pts)


def hub_cycle(seed: int = 111, m: int = 4200, d: int = 64, h: float = 30.0, s: float = 66.8) -> np.ndarray:
    """Two hubs a = (-h, 0, ...), b = (h, 0, ...), two points x = (-h, 40),
    y = (h - 5, 40) and m points at radius s in the hyperplane between the
    hubs (random directions in R^(d-1)), int8.  The path a-x-y-b is shorter
    than the hub edge and no point is nearer both hubs than they are to each
    other, so the hub edge closes a cycle without a triangle of its own
    value: its column is neither cleared nor apparent, and its cofacets are
    the m hyperplane points (more than one work-group's LDS holds when m
    exceeds 4096)."""
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((m, d - 1))
    y *= s / np.linalg.norm(y, axis=1, keepdims=True)
    pts = np.zeros((m + 4, d))
    pts[0, 0], pts[1, 0] = -h, h
    pts[2, 0], pts[2, 1] = -h, 40.0
    pts[3, 0], pts[3, 1] = h - 5.0, 40.0
    pts[4:, 1:] = y
    return quantize_i8(pts)


def lattice_cloud(seed: int, n: int, side: int = 4, d: int = 2, thr=("full", 0, 1)) -> Cloud:
    """Points drawn from the lattice {0..side-1}^d: many exact distance ties and duplicates."""
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, side, (n, d)).astype(np.int8)
    return Cloud(np.ascontiguousarray(pts), thr, name=f"lattice{n}x{d}_s{seed}")


CONFIGS = {
    "plain64": plain64,
    "circle1000": noisy_circle,
    "mixture4000": mixture,
}


def config(name: str) -> Cloud:
    return CONFIGS[name]()


def f2_csc(seed: int, nrows: int, ncols: int, mean_len: float, empty: float = 0.1, dup: float = 0.0):
    """A random sparse 0/1 pattern in CSC (colptr int64, rows int32): column
    lengths geometric with the given mean, a fraction `empty` of the columns
    empty, rows uniform in 0..nrows-1 and distinct within a column (with
    probability `dup` a column repeats one of its rows, which over F2
    cancels it), rows in random order within a column."""
    rng = np.random.default_rng(seed)
    lens = rng.geometric(1.0 / max(mean_len, 1.0), ncols).astype(np.int64) if ncols else np.zeros(0, np.int64)
    lens = np.minimum(lens, nrows)
    lens[rng.random(ncols) < empty] = 0
    cols = []
    for L in lens:
        r = rng.choice(nrows, int(L), replace=False) if L else np.zeros(0, np.int64)
        if L and rng.random() < dup:
            r = np.concatenate([r, r[:1]])
        cols.append(r)
    colptr = np.zeros(ncols + 1, np.int64)
    np.cumsum([len(c) for c in cols], out=colptr[1:])
    rows = (np.concatenate(cols) if cols else np.zeros(0)).astype(np.int32)
    return colptr, rows
