"""CPU oracle for the Jacobi3D proxy workload -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2102_12416_amd``) and neither imports the other; both take
their inputs from ``synth``.

Two implementations of the same definitions live here:
  * NumPy (this file): the definitions written out with whole-array
    elementwise IEEE operations, for small grids and cross-checks;
  * C (``jacobi_oracle.c``, loaded through ctypes): the same loops, built
    with ``-ffp-contract=off`` and OpenMP over z-planes, for large grids and
    for timing as the CPU baseline.

Method (paper section 4.3, "Proxy Application: Jacobi3D"): Jacobi iteration
for the 3D 7-point stencil on one undecomposed grid, fixed iteration count;
grid, boundary, source and residual conventions as documented in the C file.
The refinement form is split into its steps (``residual_lo``, ``lo_sweep``,
``ir_correct``, ``ir_step``) so that each can be pinned on its own: the
binary32 / bfloat16 inner sweep by fixed points, monotonicity and dense
brute force, the outer step by hand-derived one-step cases for every
rounding point and by convergence to the dense solution.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# ----------------------------------------------------------------- NumPy ---


def interior(a: np.ndarray) -> np.ndarray:
    return a[1:-1, 1:-1, 1:-1]


def neighbour_sum(u: np.ndarray) -> np.ndarray:
    """s = ((((u(x-1) + u(x+1)) + u(y-1)) + u(y+1)) + u(z-1)) + u(z+1) on the interior."""
    s = u[1:-1, 1:-1, :-2] + u[1:-1, 1:-1, 2:]
    s = s + u[1:-1, :-2, 1:-1]
    s = s + u[1:-1, 2:, 1:-1]
    s = s + u[:-2, 1:-1, 1:-1]
    s = s + u[2:, 1:-1, 1:-1]
    return s


def sweep(u: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """One Jacobi sweep: interior <- (s + b) / 6 (s / 6 without a source); shell kept."""
    v = u.copy()
    s = neighbour_sum(u)
    if b is None:
        v[1:-1, 1:-1, 1:-1] = s / 6.0
    else:
        v[1:-1, 1:-1, 1:-1] = (s + interior(b)) / 6.0
    return v


def residual_field(u: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """r = (b + s) - 6u on the interior (residual of A u = b, A = 6I - face sum)."""
    s = neighbour_sum(u)
    if b is None:
        return s - 6.0 * interior(u)
    return (interior(b) + s) - 6.0 * interior(u)


def residual_norm(u: np.ndarray, b: np.ndarray | None = None) -> float:
    """2-norm of the residual, r^2 summed by NumPy's pairwise reduction."""
    r = residual_field(u, b)
    return float(np.sqrt(np.sum((r * r).ravel())))


def jacobi(u0: np.ndarray, iters: int, b: np.ndarray | None = None, every: int = 0):
    """Plain Jacobi for ``iters`` sweeps; returns (final iterate, residual history).

    History holds the residual norm at iterates 0, every, 2*every, ... and at
    the final iterate (when every > 0)."""
    u = u0.copy()
    hist = []
    for k in range(iters):
        if every > 0 and k % every == 0:
            hist.append(residual_norm(u, b))
        u = sweep(u, b)
    if every > 0:
        hist.append(residual_norm(u, b))
    return u, hist


def bf16_round(x: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns (uint16), round to nearest, ties to even."""
    bits = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    upper = (bits >> np.uint32(16)).astype(np.uint32)
    lower = bits & np.uint32(0xFFFF)
    up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    out = (upper + up.astype(np.uint32)).astype(np.uint32)
    nan = (bits & np.uint32(0x7FFFFFFF)) > np.uint32(0x7F800000)
    out = np.where(nan, upper | np.uint32(0x40), out)
    return out.astype(np.uint16)


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def store_lo(x32: np.ndarray, storage: str) -> np.ndarray:
    """Round binary32 values to the storage format ('f32' or 'bf16'), kept as binary32."""
    if storage == "bf16":
        return bf16_to_f32(bf16_round(x32))
    return np.asarray(x32, dtype=np.float32)


def residual_lo(r: np.ndarray, storage: str) -> np.ndarray:
    """Outer-step residual for the inner sweeps: binary64 r rounded to
    binary32, and for 'bf16' from there to bfloat16 (round to nearest even
    both times), kept as binary32 values."""
    return store_lo(np.asarray(r, dtype=np.float64).astype(np.float32), storage)


def lo_sweep(d: np.ndarray, rlo: np.ndarray, storage: str) -> np.ndarray:
    """One inner sweep of the refinement on the padded binary32 correction d
    (zero shell): d' = lo((s(d) + r_lo) / 6) with the neighbour sum s, the
    addition of r_lo (interior-shaped) and the division in binary32, the
    result rounded to the storage format."""
    s = neighbour_sum(d)
    e = d.copy()
    e[1:-1, 1:-1, 1:-1] = store_lo((s + rlo) / np.float32(6.0), storage)
    return e


def ir_correct(u: np.ndarray, r: np.ndarray, storage: str, m: int) -> np.ndarray:
    """The correction part of one outer step: from the binary64 residual r
    (interior-shaped), m inner Jacobi sweeps on A d = r from d = 0 with zero
    ghosts, then u + d in binary64.  storage 'f64' keeps d and r in binary64
    (plain sweeps with r as the source)."""
    shape = u.shape
    v = u.copy()
    if storage == "f64":
        rr = np.zeros(shape)
        rr[1:-1, 1:-1, 1:-1] = r
        d = np.zeros(shape)
        for _ in range(m):
            d = sweep(d, rr)
        v[1:-1, 1:-1, 1:-1] = interior(u) + interior(d)
    else:
        rlo = residual_lo(r, storage)
        d = np.zeros(shape, dtype=np.float32)
        for _ in range(m):
            d = lo_sweep(d, rlo, storage)
        v[1:-1, 1:-1, 1:-1] = interior(u) + interior(d).astype(np.float64)
    return v


def ir_step(u: np.ndarray, b: np.ndarray | None, storage: str, m: int) -> np.ndarray:
    """One outer step: binary64 residual of u, then :func:`ir_correct`."""
    return ir_correct(u, residual_field(u, b), storage, m)


def ir_solve(u0: np.ndarray, b: np.ndarray | None, storage: str = "f32", inner: int = 50,
             rtol: float = 1e-10, max_inner: int = 20000):
    """Mixed-precision iterative refinement with Jacobi inner sweeps.

    storage 'f64' keeps d and r in binary64 (no rounding); 'f32' and 'bf16'
    round r to the storage format (through binary32) and run the inner
    sweeps with binary32 sums and division.  Each outer step computes the
    binary64 residual and its norm, stops when |r|/|r_0| <= rtol or the cap
    (counted in inner sweeps) is reached, else corrects u.  Returns
    (u, rel history per outer check, inner sweeps done, status 0/1)."""
    u = u0.copy()
    r0 = None
    hist = []
    done = 0
    status = 1
    while True:
        r = residual_field(u, b)
        nrm = float(np.sqrt(np.sum((r * r).ravel())))
        if r0 is None:
            r0 = nrm
        rel = nrm / r0 if r0 > 0 else 0.0
        hist.append(rel)
        if rel <= rtol:
            status = 0
            break
        if done >= max_inner:
            break
        m = min(inner, max_inner - done)
        u = ir_correct(u, r, storage, m)
        done += m
    return u, hist, done, status


# --------------------------------------------------------------------- C ---


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle.so (gcc, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    """The C oracle, built on first use."""
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_sweep.argtypes = [dp, dp, dp, i64, i64, i64]
        L.oracle_sweep.restype = None
        L.oracle_residual.argtypes = [dp, dp, i64, i64, i64]
        L.oracle_residual.restype = ctypes.c_double
        L.oracle_residual_sumsq.argtypes = [dp, dp, i64, i64, i64]
        L.oracle_residual_sumsq.restype = ctypes.c_double
        L.oracle_jacobi.argtypes = [dp, dp, i64, i64, i64, i64, i64, dp, i64]
        L.oracle_jacobi.restype = i64
        L.oracle_bf16_round.argtypes = [ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_uint16), i64]
        L.oracle_bf16_round.restype = None
        L.oracle_ir.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int, i64, ctypes.c_double, i64,
                                dp, ctypes.POINTER(i64), dp, i64, ctypes.POINTER(i64)]
        L.oracle_ir.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(u):
    nz, ny, nx = (int(v) - 2 for v in u.shape)
    return nx, ny, nz


def c_sweep(u: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    v = u.copy()
    lib().oracle_sweep(_dptr(u), _dptr(v), _dptr(b), *_dims(u))
    return v


def c_residual_norm(u: np.ndarray, b: np.ndarray | None = None) -> float:
    return float(lib().oracle_residual(_dptr(u), _dptr(b), *_dims(u)))


def c_jacobi(u0: np.ndarray, iters: int, b: np.ndarray | None = None, every: int = 0,
             inplace: bool = False):
    """C version of :func:`jacobi`; returns (final iterate, history list)."""
    u = u0 if inplace else u0.copy()
    cap = (iters // every + 2) if every > 0 else 1
    hist = np.zeros(cap)
    n = lib().oracle_jacobi(_dptr(u), _dptr(b), *_dims(u), int(iters), int(every),
                            _dptr(hist), cap)
    return u, list(hist[:n])


def c_ir_solve(u0: np.ndarray, b: np.ndarray | None, storage: str = "f32", inner: int = 50,
               rtol: float = 1e-10, max_inner: int = 20000):
    """C version of :func:`ir_solve`; same return tuple."""
    code = {"f64": 0, "f32": 1, "bf16": 2}[storage]
    u = u0.copy()
    cap = max_inner // max(inner, 1) + 3
    hist = np.zeros(cap)
    rel = ctypes.c_double()
    done = ctypes.c_int64()
    nh = ctypes.c_int64()
    st = lib().oracle_ir(_dptr(u), _dptr(b), *_dims(u), code, int(inner), float(rtol),
                         int(max_inner), ctypes.byref(rel), ctypes.byref(done),
                         _dptr(hist), cap, ctypes.byref(nh))
    return u, list(hist[:nh.value]), int(done.value), int(st)


def c_bf16_round(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(x.shape, dtype=np.uint16)
    lib().oracle_bf16_round(x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), x.size)
    return out


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))
