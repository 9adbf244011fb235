"""Seeded synthetic inputs for the Jacobi3D workload.

This module holds the input recipe only: it draws numbers and lays them
out.  It contains none of the method's arithmetic (no stencil, no
residual, no rounding of iterates) and is the one module that both the
CPU oracle and the GPU path may use.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), in counter
form: the k-th output (k >= 1) of a generator seeded with ``s`` is
``mix64(s + k * GAMMA)`` with the 64-bit golden-gamma increment and the
variant-13 finaliser published with the algorithm.  Because every value
is a function of (seed, stream, global index), a field is identical no
matter how the grid is later decomposed.

Field conventions (Jacobi3D proxy, paper section 4.3):
  * a grid with interior ``nx x ny x nz`` is stored padded as a C array of
    shape ``(nz + 2, ny + 2, nx + 2)``; x is the unit-stride axis;
  * the Dirichlet shell is every cell with a coordinate in {0, n + 1};
  * stream 0 draws the boundary values g ~ U[0, 1) on the shell, the
    interior of the initial iterate is 0;
  * stream 1 draws the source b ~ U[-1, 1) on the interior, 0 on the shell;
  * the draw for a cell uses its flat index in the padded global array.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = float(2.0 ** -53)

STREAM_BOUNDARY = 0
STREAM_SOURCE = 1

DEFAULT_SEED = 12416


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (variant 13) on a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_outputs(seed: int, k: np.ndarray) -> np.ndarray:
    """The k-th outputs (k >= 1, uint64 array) of SplitMix64 seeded with ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GAMMA)


def stream_key(seed: int, stream: int) -> int:
    """Seed of a field's own generator: output ``stream + 1`` of SplitMix64(seed)."""
    return int(splitmix64_outputs(seed, np.array([stream + 1], dtype=np.uint64))[0])


def uniform01(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """U[0, 1) doubles for flat indices ``idx``: top 53 bits of output idx + 1."""
    key = stream_key(seed, stream)
    idx = np.asarray(idx, dtype=np.uint64)
    z = splitmix64_outputs(key, idx + np.uint64(1))
    return (z >> np.uint64(11)).astype(np.float64) * _TWO_M53


def _padded_shape(n):
    nx, ny, nz = (int(v) for v in n)
    return (nz + 2, ny + 2, nx + 2)


def boundary_field(n, seed: int = DEFAULT_SEED) -> np.ndarray:
    """Padded initial iterate: shell = g ~ U[0,1) (stream 0), interior = 0.

    ``n`` is the interior size (nx, ny, nz)."""
    shape = _padded_shape(n)
    u = np.zeros(shape, dtype=np.float64)
    P, R, C = shape
    plane = R * C
    # z = 0 and z = nz + 1 planes
    for z in (0, P - 1):
        idx = np.arange(z * plane, (z + 1) * plane, dtype=np.uint64)
        u[z] = uniform01(seed, STREAM_BOUNDARY, idx).reshape(R, C)
    zs = np.arange(1, P - 1, dtype=np.uint64)[:, None]
    # y = 0 and y = ny + 1 rows of the interior planes
    for y in (0, R - 1):
        idx = zs * np.uint64(plane) + np.uint64(y * C) + np.arange(C, dtype=np.uint64)[None, :]
        u[1:P - 1, y, :] = uniform01(seed, STREAM_BOUNDARY, idx.ravel()).reshape(P - 2, C)
    # x = 0 and x = nx + 1 columns of the interior rows
    ys = np.arange(1, R - 1, dtype=np.uint64)[None, :]
    for x in (0, C - 1):
        idx = zs * np.uint64(plane) + ys * np.uint64(C) + np.uint64(x)
        u[1:P - 1, 1:R - 1, x] = uniform01(seed, STREAM_BOUNDARY, idx.ravel()).reshape(P - 2, R - 2)
    return u


def source_slab(n, z_lo: int, z_hi: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """Planes ``z_lo <= z < z_hi`` of the padded source field (stream 1).

    Interior cells hold 2 * U[0,1) - 1 (exact in binary64), shell cells 0."""
    P, R, C = _padded_shape(n)
    z_lo = max(0, int(z_lo))
    z_hi = min(P, int(z_hi))
    out = np.zeros((max(0, z_hi - z_lo), R, C), dtype=np.float64)
    plane = R * C
    for z in range(max(z_lo, 1), min(z_hi, P - 1)):
        ys = np.arange(1, R - 1, dtype=np.uint64)[:, None]
        xs = np.arange(1, C - 1, dtype=np.uint64)[None, :]
        idx = np.uint64(z * plane) + ys * np.uint64(C) + xs
        out[z - z_lo, 1:R - 1, 1:C - 1] = (
            2.0 * uniform01(seed, STREAM_SOURCE, idx.ravel()).reshape(R - 2, C - 2) - 1.0)
    return out


def source_field(n, seed: int = DEFAULT_SEED) -> np.ndarray:
    """Whole padded source field b ~ U[-1, 1) (stream 1), shell 0."""
    P, _, _ = _padded_shape(n)
    return source_slab(n, 0, P, seed)


def uneven_cuts(total: int, lo: int = 32, hi: int = 160, seed: int = DEFAULT_SEED,
                axis: int = 0) -> list:
    """Rectilinear block edges along one axis, log-uniform in [lo, hi].

    Draws l = round(exp(U(ln lo, ln hi))) from numpy's default generator
    seeded with ``seed + axis`` while more than ``hi`` cells remain; a draw
    that would leave fewer than ``lo`` cells is shortened so the rest stays
    >= lo; the remainder closes the axis.  Every piece lies in [lo, hi]
    (given total >= lo) and the pieces sum to ``total``."""
    if total < lo:
        raise ValueError("axis shorter than the smallest block edge")
    rng = np.random.default_rng(seed + axis)
    cuts = []
    rem = int(total)
    while rem > hi:
        piece = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
        piece = min(max(piece, lo), hi)
        if rem - piece < lo:
            piece = rem - lo
        cuts.append(piece)
        rem -= piece
    cuts.append(rem)
    return cuts


def log_uniform_edges(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """``count`` integer edges round(exp(U(ln lo, ln hi))) from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    e = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    return np.clip(e, lo, hi)


def serving_requests(count: int, rate_per_s: float, seed: int = DEFAULT_SEED,
                     lo: int = 32, hi: int = 384, p_mixed: float = 0.5):
    """Seeded request stream for the solve server.

    Returns a list of dicts with arrival time (Poisson process of the given
    rate), cubic interior edge (log-uniform in [lo, hi]), precision
    ('f64' or 'f32' mixed) and the per-request field seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count) if rate_per_s > 0 else np.zeros(count)
    arrivals = np.cumsum(gaps) - gaps[0] if count else gaps
    edges = log_uniform_edges(count, lo, hi, seed + 7)
    mixed = rng.random(count) < p_mixed
    return [dict(id=i, arrival=float(arrivals[i]), n=int(edges[i]),
                 precision=("f32" if mixed[i] else "f64"), seed=int(seed) + 1000 + i)
            for i in range(count)]


def field_box(n, kind: int, lo, hi, seed: int = DEFAULT_SEED) -> np.ndarray:
    """The box ``lo <= (z, y, x) < hi`` (padded indices) of the padded
    initial iterate (kind 0: shell g, interior 0) or of the source (kind 1:
    interior b, shell 0), drawn by global flat index, so a box of a large
    grid needs no whole-field array."""
    P, R, C = _padded_shape(n)
    if kind not in (0, 1):
        raise ValueError("kind is 0 (boundary) or 1 (source)")
    lo = [int(v) for v in lo]
    hi = [int(v) for v in hi]
    if any(l < 0 or h > m or l >= h for l, h, m in zip(lo, hi, (P, R, C))):
        raise ValueError("box outside the padded grid")
    z = np.arange(lo[0], hi[0], dtype=np.uint64)[:, None, None]
    y = np.arange(lo[1], hi[1], dtype=np.uint64)[None, :, None]
    x = np.arange(lo[2], hi[2], dtype=np.uint64)[None, None, :]
    idx = (z * np.uint64(R) + y) * np.uint64(C) + x
    shell = ((z == 0) | (z == P - 1) | (y == 0) | (y == R - 1) | (x == 0) | (x == C - 1))
    if kind == 0:
        v = uniform01(seed, STREAM_BOUNDARY, idx.ravel()).reshape(idx.shape)
        return np.where(shell, v, 0.0)
    v = 2.0 * uniform01(seed, STREAM_SOURCE, idx.ravel()).reshape(idx.shape) - 1.0
    return np.where(shell, 0.0, v)
