"""Checks that pin the oracle to facts fixed by the mathematics of the method.

Each ``check_*`` takes a sweep function ``sweep_fn(u, b) -> v`` (padded
arrays, shell kept) and returns ``(ok, detail)``.  The real oracle must
pass every check; deliberately broken sweeps (a dropped term, a wrong
sign, a swapped axis, a wrong divisor, in-place updates) must each fail at
least one of them (tests/test_oracle_pins.py).  Nothing here calls the GPU
library.
"""
from __future__ import annotations

import math

import numpy as np


def padded_coords(nx, ny, nz):
    """Integer coordinate arrays (z, y, x) of the padded grid, 0 .. n+1."""
    z, y, x = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def iterate(sweep_fn, u, b, k):
    for _ in range(k):
        u = sweep_fn(u, b)
    return u


# --------------------------------------------------------------- fixed points


def check_constant(sweep_fn):
    """A constant field (interior and shell) is a fixed point; bitwise when
    every partial sum k*c (k <= 6) is exact."""
    for c in (0.0, 1.0, 0.5, 0.375, -2.25):
        u = np.full((6 + 2, 5 + 2, 7 + 2), c)
        v = iterate(sweep_fn, u, None, 4)
        if not np.array_equal(v, u):
            return False, "constant %r moved" % c
    return True, ""


def check_harmonic(sweep_fn):
    """Discrete-harmonic polynomials with matching Dirichlet data are fixed
    points of the b = 0 sweep (the 7-point Laplacian is exact on them)."""
    x, y, z = padded_coords(7, 6, 5)
    for name, u in (("x+y+z", x + y + z), ("xyz", x * y * z), ("x2-y2", x * x - y * y),
                    ("y2-z2", y * y - z * z), ("xy+yz", x * y + y * z), ("2x+3y-5z", 2 * x + 3 * y - 5 * z)):
        v = iterate(sweep_fn, u.copy(), None, 3)
        if not np.array_equal(v, u):
            return False, "harmonic %s moved" % name
    return True, ""


def check_manufactured(sweep_fn):
    """u = x^2 with b = -2 is a fixed point of u' = (s + b)/6 (s = 6x^2 + 2);
    likewise y^2 and z^2.  Pins the sign and scale of the source."""
    x, y, z = padded_coords(6, 7, 5)
    b = np.full(x.shape, -2.0)
    b[0, :, :] = b[-1, :, :] = 0
    b[:, 0, :] = b[:, -1, :] = 0
    b[:, :, 0] = b[:, :, -1] = 0
    for name, u in (("x^2", x * x), ("y^2", y * y), ("z^2", z * z)):
        v = iterate(sweep_fn, u.copy(), b, 3)
        if not np.array_equal(v, u):
            return False, "manufactured %s moved" % name
    return True, ""


# ----------------------------------------------------------------- dynamics


def check_sine_mode(sweep_fn):
    """Eigenmode closed form: u0 = prod sin(p pi i/(n+1)) with zero shell
    decays as lambda^k u0, lambda = mean of the three cosines."""
    nx, ny, nz = 11, 9, 7
    x, y, z = padded_coords(nx, ny, nz)
    for (p, q, r) in ((1, 1, 1), (2, 1, 3)):
        u0 = (np.sin(p * math.pi * x / (nx + 1)) * np.sin(q * math.pi * y / (ny + 1))
              * np.sin(r * math.pi * z / (nz + 1)))
        u0[0, :, :] = u0[-1, :, :] = 0
        u0[:, 0, :] = u0[:, -1, :] = 0
        u0[:, :, 0] = u0[:, :, -1] = 0
        lam = (math.cos(p * math.pi / (nx + 1)) + math.cos(q * math.pi / (ny + 1))
               + math.cos(r * math.pi / (nz + 1))) / 3.0
        k = 20
        uk = iterate(sweep_fn, u0.copy(), None, k)
        err = np.max(np.abs(uk - lam ** k * u0)) / np.max(np.abs(u0))
        if not err < 1e-13:
            return False, "sine mode (%d,%d,%d) error %.3g" % (p, q, r, err)
    return True, ""


def dense_system(nx, ny, nz, g, b):
    """Dense A (6 on the diagonal, -1 per interior face neighbour) and
    b_eff = b + sum of Dirichlet face neighbours, built cell by cell."""
    n = nx * ny * nz

    def lin(i, j, k):
        return ((k - 1) * ny + (j - 1)) * nx + (i - 1)

    A = np.zeros((n, n))
    beff = np.zeros(n)
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                row = lin(i, j, k)
                A[row, row] = 6.0
                beff[row] += 0.0 if b is None else b[k, j, i]
                for (di, dj, dk) in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    a, c, e = i + di, j + dj, k + dk
                    if 1 <= a <= nx and 1 <= c <= ny and 1 <= e <= nz:
                        A[row, lin(a, c, e)] = -1.0
                    else:
                        beff[row] += g[e, c, a]
    return A, beff


def check_dense(sweep_fn):
    """Brute force on tiny grids: one sweep equals D^-1((D - A)u + b_eff)
    built from a dense matrix, and the iterates reach A^-1 b_eff."""
    rng = np.random.default_rng(7)
    for (nx, ny, nz) in ((1, 1, 1), (2, 2, 2), (3, 2, 4), (4, 4, 4)):
        g = rng.random((nz + 2, ny + 2, nx + 2))
        b = np.zeros_like(g)
        b[1:-1, 1:-1, 1:-1] = rng.random((nz, ny, nx)) * 2 - 1
        A, beff = dense_system(nx, ny, nz, g, b)
        u = g.copy()
        u[1:-1, 1:-1, 1:-1] = rng.random((nz, ny, nx))
        flat = u[1:-1, 1:-1, 1:-1].ravel()
        offdiag = -(A - np.diag(np.diag(A)))
        ref = (offdiag @ flat + beff) / 6.0
        got = sweep_fn(u, b)[1:-1, 1:-1, 1:-1].ravel()
        if not np.allclose(got, ref, rtol=4e-16 * 8, atol=1e-15):
            return False, "dense sweep mismatch at %s" % ((nx, ny, nz),)
        exact = np.linalg.solve(A, beff)
        v = iterate(sweep_fn, u, b, 400)[1:-1, 1:-1, 1:-1].ravel()
        if not np.max(np.abs(v - exact)) <= 1e-12 * max(1.0, np.max(np.abs(exact))):
            return False, "dense limit mismatch at %s" % ((nx, ny, nz),)
    return True, ""


def check_monotone(sweep_fn):
    """b = 0, g >= 0, u0 = 0: iterates are pointwise non-decreasing and
    bounded by max g (maximum principle), bitwise in floating point."""
    rng = np.random.default_rng(3)
    g = rng.random((9 + 2, 12 + 2, 10 + 2))
    u = g.copy()
    u[1:-1, 1:-1, 1:-1] = 0.0
    gmax = g.max()
    for _ in range(30):
        v = sweep_fn(u, None)
        if not (np.all(v >= u) and np.all(v <= gmax)):
            return False, "monotonicity/maximum principle violated"
        u = v
    return True, ""


def residual_norm(u, b=None):
    """Residual 2-norm computed independently of the oracle's module."""
    nz, ny, nx = (d - 2 for d in u.shape)
    r = np.zeros((nz, ny, nx))
    for (dz, dy, dx) in ((0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)):
        r += u[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    r -= 6.0 * u[1:-1, 1:-1, 1:-1]
    if b is not None:
        r += b[1:-1, 1:-1, 1:-1]
    return float(np.sqrt(np.sum(r * r)))


def check_residual_decay(sweep_fn):
    """The residual norm decreases strictly (J = I - A/6 is symmetric with
    norm cos(pi/(n+1)) < 1) and the per-sweep ratio tends to cos(pi/(n+1))."""
    n = 16
    rng = np.random.default_rng(11)
    u = rng.random((n + 2, n + 2, n + 2))
    u[1:-1, 1:-1, 1:-1] = 0.0
    prev = residual_norm(u)
    ratio = None
    for _ in range(400):
        u = sweep_fn(u, None)
        cur = residual_norm(u)
        if not cur < prev:
            return False, "residual did not decrease"
        ratio = cur / prev
        prev = cur
    if abs(ratio - math.cos(math.pi / (n + 1))) > 2e-4:
        return False, "asymptotic ratio %.6f" % ratio
    return True, ""


ALL_CHECKS = (check_constant, check_harmonic, check_manufactured, check_sine_mode,
              check_dense, check_monotone, check_residual_decay)


# ------------------------------------------- refinement in low precision --
#
# The refinement's inner sweep runs on the correction d in binary32 or
# bfloat16 storage with binary32 sums and division; its outer step takes a
# binary64 residual and updates u in binary64.  The checks below take
#   lo_sweep_fn(d, rlo, storage) -> d'   (padded binary32 d, interior r_lo)
#   step_fn(u, b, storage, m) -> u'      (one outer step, m inner sweeps)
# and pin them to facts that do not come from the oracle.

def bf16_nearest(x32):
    """binary32 values rounded to the nearest bfloat16 value, ties to the
    one with an even last bit, returned as binary32.  Written as a choice
    between the two bfloat16 neighbours by distance (exact in binary64),
    independently of the oracle's bit arithmetic; finite inputs only."""
    x = np.ascontiguousarray(x32, dtype=np.float32)
    bits = x.view(np.uint32)
    down = (bits & np.uint32(0xFFFF0000)).view(np.float32)
    up_bits = (bits & np.uint32(0xFFFF0000)) + np.uint32(0x10000)
    up = up_bits.view(np.float32)
    xd, dd, ud = x.astype(np.float64), down.astype(np.float64), up.astype(np.float64)
    dist_down, dist_up = np.abs(xd - dd), np.abs(ud - xd)
    down_even = ((bits >> np.uint32(16)) & np.uint32(1)) == 0
    take_up = (dist_up < dist_down) | ((dist_up == dist_down) & ~down_even)
    exact = (bits & np.uint32(0xFFFF)) == 0
    return np.where(exact, x, np.where(take_up, up, down)).astype(np.float32)


def to_storage(x, storage):
    """binary32 (or binary64) values rounded to the storage format, as binary32."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    return bf16_nearest(x32) if storage == "bf16" else x32


def exact_in(x, storage):
    x = np.asarray(x, dtype=np.float64)
    return np.array_equal(to_storage(x, storage).astype(np.float64), x)


def lo_as_sweep(lo_sweep_fn, storage):
    """The inner sweep as a sweep_fn(u, b) of the binary64 checks above, for
    fields whose every value is exact in the storage format (refused
    otherwise, so that a check never tests a rounded copy of its field)."""
    def f(u, b):
        if not exact_in(u, storage) or (b is not None and not exact_in(b, storage)):
            raise ValueError("field not exact in %s" % storage)
        d = np.asarray(u, dtype=np.float32)
        nz, ny, nx = (n - 2 for n in u.shape)
        rlo = np.zeros((nz, ny, nx), np.float32) if b is None else \
            np.ascontiguousarray(b[1:-1, 1:-1, 1:-1], dtype=np.float32)
        return np.asarray(lo_sweep_fn(d, rlo, storage), dtype=np.float64)
    return f


def check_lo_fixed_points(lo_sweep_fn, storage):
    """Constant, discrete-harmonic and manufactured (u = x^2, r_lo = -2)
    fields are fixed points of the inner sweep too: their values and every
    neighbour sum are small integers or short dyadic fractions, exact in
    binary32 and in bfloat16, and s/6 is exact."""
    f = lo_as_sweep(lo_sweep_fn, storage)
    for check in (check_constant, check_harmonic, check_manufactured):
        ok, detail = check(f)
        if not ok:
            return False, "%s (%s)" % (detail, storage)
    return True, ""


def check_lo_monotone(lo_sweep_fn, storage):
    """Zero source, shell g >= 0 in the storage format, d0 = 0: the inner
    iterates are pointwise non-decreasing and bounded by max g, bitwise
    (sums, the division and rounding to nearest are monotone, max g is a
    storage value)."""
    f = lo_as_sweep(lo_sweep_fn, storage)
    rng = np.random.default_rng(13)
    g = to_storage(rng.random((7 + 2, 9 + 2, 8 + 2)), storage).astype(np.float64)
    u = g.copy()
    u[1:-1, 1:-1, 1:-1] = 0.0
    for _ in range(25):
        v = f(u, None)
        if not (np.all(v >= u) and np.all(v <= g.max())):
            return False, "monotonicity/maximum principle violated (%s)" % storage
        u = v
    return True, ""


def check_lo_dense(lo_sweep_fn, storage):
    """Brute force on tiny grids with zero ghosts (the correction equation):
    for small-integer d and r_lo every binary32 sum is exact, so one inner
    sweep is the binary32 quotient of the dense product ((D - A) d + r_lo)
    by 6, rounded to the storage format; and the inner iterates approach
    A^-1 r_lo to within the storage precision."""
    rng = np.random.default_rng(17)
    limit_tol = {"f32": 2e-6, "bf16": 4e-2}[storage]
    for (nx, ny, nz) in ((1, 1, 1), (2, 2, 2), (3, 2, 4), (4, 4, 4)):
        zero = np.zeros((nz + 2, ny + 2, nx + 2))
        A, _ = dense_system(nx, ny, nz, zero, None)
        offdiag = -(A - np.diag(np.diag(A)))
        d = zero.astype(np.float32)
        d[1:-1, 1:-1, 1:-1] = rng.integers(-8, 9, (nz, ny, nx))
        r = rng.integers(-40, 41, (nz, ny, nx)).astype(np.float32)
        num = offdiag @ d[1:-1, 1:-1, 1:-1].ravel().astype(np.float64) + r.ravel()
        ref = to_storage(np.float32(num) / np.float32(6.0), storage)
        got = np.asarray(lo_sweep_fn(d, r, storage))[1:-1, 1:-1, 1:-1].ravel()
        if not np.array_equal(got, ref):
            return False, "dense inner sweep mismatch at %s (%s)" % ((nx, ny, nz), storage)
        exact = np.linalg.solve(A, r.ravel().astype(np.float64))
        e = zero.astype(np.float32)
        for _ in range(300):
            e = lo_sweep_fn(e, r, storage)
        err = np.max(np.abs(np.asarray(e, np.float64)[1:-1, 1:-1, 1:-1].ravel() - exact))
        if not err <= limit_tol * np.max(np.abs(exact)):
            return False, "inner limit off by %.3g at %s (%s)" % (err, (nx, ny, nz), storage)
    return True, ""


def check_ir_limit(step_fn, storage):
    """Refinement with a binary64 outer residual and update converges to the
    exact solution A^-1 b_eff (numpy.linalg.solve of the dense system) to
    binary64 accuracy, whatever the inner storage: each outer step cuts the
    error by the inner solve's accuracy."""
    rng = np.random.default_rng(19)
    for (nx, ny, nz) in ((1, 1, 1), (2, 2, 2), (3, 2, 4), (4, 4, 4)):
        g = rng.random((nz + 2, ny + 2, nx + 2))
        b = np.zeros_like(g)
        b[1:-1, 1:-1, 1:-1] = rng.random((nz, ny, nx)) * 2 - 1
        A, beff = dense_system(nx, ny, nz, g, b)
        exact = np.linalg.solve(A, beff)
        u = g.copy()
        u[1:-1, 1:-1, 1:-1] = 0.0
        for _ in range(30):
            u = step_fn(u, b, storage, 50)
        if not np.array_equal(u[0], g[0]) or not np.array_equal(u[:, 0], g[:, 0]):
            return False, "shell changed (%s)" % storage
        err = np.max(np.abs(u[1:-1, 1:-1, 1:-1].ravel() - exact))
        if not err <= 1e-12 * max(1.0, np.max(np.abs(exact))):
            return False, "refinement limit off by %.3g at %s (%s)" % (err, (nx, ny, nz), storage)
    return True, ""


def load_refinement_cases(path):
    import json
    with open(path) as f:
        return json.load(f)["cases"]


def check_ir_goldens(step_fn, storage, cases):
    """Hand-derived one-outer-step cases (tests/golden/refinement_cases.json):
    the rounding of r through binary32 to the storage format, the correction
    rounded to storage between inner sweeps, binary32 neighbour sums in the
    stencil's order, and the binary64 update; bitwise."""
    for case in cases:
        if case["storage"] != storage:
            continue
        nx, ny, nz = case["n"]
        u0 = np.array(case["u0"], dtype=np.float64).reshape(nz + 2, ny + 2, nx + 2)
        b = np.array(case["b"], dtype=np.float64).reshape(nz + 2, ny + 2, nx + 2)
        got = step_fn(u0, b, storage, case["inner"])[1:-1, 1:-1, 1:-1].ravel()
        exp = np.array([float.fromhex(h) for h in case["expected_hex"]])
        if not np.array_equal(got, exp):
            return False, "golden %s: %s vs %s" % (case["name"], [v.hex() for v in got],
                                                    case["expected_hex"])
    return True, ""
