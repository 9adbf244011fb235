"""The oracle pinned to facts other than itself (CPU only).

Pins: fixed points (constant, discrete-harmonic, manufactured source),
eigenmode closed form, dense brute force on tiny grids, maximum principle,
residual decay rate, the residual/update identity, iterative refinement
with binary64 inner sweeps equal to plain Jacobi, bfloat16 rounding on
known bit patterns and against torch's conversion, hand-computed golden
cases, and C == NumPy bitwise.  Planted mistakes in copies of the sweep
must each fail at least one pin.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import oracle_pins as pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def np_sweep(u, b):
    return oracle.sweep(u, b)


def c_sweep(u, b):
    return oracle.c_sweep(np.ascontiguousarray(u, dtype=np.float64),
                          None if b is None else np.ascontiguousarray(b, dtype=np.float64))


@pytest.mark.parametrize("impl", [np_sweep, c_sweep], ids=["numpy", "c"])
@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_oracle_passes_pin(impl, check):
    ok, detail = check(impl)
    assert ok, detail


# ----------------------------------------------------- planted mistakes --

def _shifted(u, dz, dy, dx):
    nz, ny, nx = (d - 2 for d in u.shape)
    return u[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


def _mutant(kind):
    def f(u, b):
        v = u.copy()
        terms = [(0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]
        div = 6.0
        bsign = 1.0
        if kind == "dropped_term":
            terms = terms[:-1]
        elif kind == "swapped_axis":          # y-neighbours used twice, z never
            terms = [(0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (0, -1, 0), (0, 1, 0)]
        elif kind == "wrong_index":           # x+1 read from the next row (diagonal cell)
            terms = [(0, 0, -1), (0, 1, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]
        elif kind == "divide_by_7":
            div = 7.0
        elif kind == "source_sign":
            bsign = -1.0
        if kind == "gauss_seidel":            # in-place update: not Jacobi
            nz, ny, nx = (d - 2 for d in u.shape)
            for z in range(1, nz + 1):
                for y in range(1, ny + 1):
                    for x in range(1, nx + 1):
                        s = (v[z, y, x - 1] + v[z, y, x + 1] + v[z, y - 1, x] + v[z, y + 1, x]
                             + v[z - 1, y, x] + v[z + 1, y, x])
                        v[z, y, x] = (s + (0.0 if b is None else b[z, y, x])) / 6.0
            return v
        s = 0.0
        for t in terms:
            s = s + _shifted(u, *t)
        if b is not None:
            s = s + bsign * b[1:-1, 1:-1, 1:-1]
        v[1:-1, 1:-1, 1:-1] = s / div
        return v
    return f


@pytest.mark.parametrize("kind", ["dropped_term", "swapped_axis", "wrong_index", "divide_by_7",
                                  "source_sign", "gauss_seidel"])
def test_planted_mistake_fails_a_pin(kind):
    bad = _mutant(kind)
    failed = [c.__name__ for c in pins.ALL_CHECKS if not c(bad)[0]]
    assert failed, "mutant %s passed every pin" % kind


# --------------------------------------------------------- bitwise C == NumPy

@pytest.mark.parametrize("shape,with_b", [((5, 4, 3), False), ((17, 9, 33), True), ((32, 32, 32), False),
                                          ((1, 7, 2), True)])
def test_c_equals_numpy_bitwise(shape, with_b):
    nx, ny, nz = shape
    u0 = synth.boundary_field(shape, seed=5)
    b = synth.source_field(shape, seed=5) if with_b else None
    a, ha = oracle.jacobi(u0, 25, b, every=5)
    c, hc = oracle.c_jacobi(u0, 25, b, every=5)
    assert np.array_equal(a, c)
    np.testing.assert_allclose(ha, hc, rtol=1e-13)


def test_residual_update_identity():
    """r_k = 6 (u_{k+1} - u_k) in exact arithmetic (D = 6I)."""
    u = synth.boundary_field((12, 10, 14), seed=2)
    b = synth.source_field((12, 10, 14), seed=2)
    for _ in range(5):
        v = oracle.sweep(u, b)
        r = oracle.residual_norm(u, b)
        d = 6.0 * np.sqrt(np.sum((v - u) ** 2))
        assert abs(r - d) <= 1e-12 * r
        assert abs(oracle.c_residual_norm(u, b) - r) <= 1e-13 * r
        assert abs(pins.residual_norm(u, b) - r) <= 1e-13 * r
        u = v


def test_relative_residual_reading_coincide():
    """With u0 = 0 the initial residual equals |b + Dirichlet neighbour sums|,
    the two common readings of 'relative residual'."""
    n = (6, 5, 4)
    u = synth.boundary_field(n, seed=9)
    b = synth.source_field(n, seed=9)
    g = u.copy()
    A, beff = pins.dense_system(*n, g, b)
    assert abs(oracle.residual_norm(u, b) - np.linalg.norm(beff)) <= 1e-13 * np.linalg.norm(beff)


# ------------------------------------------------------------ golden cases

def test_golden_hand_cases():
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    assert cases
    for case in cases:
        nx, ny, nz = case["n"]
        u = np.array(case["u0"], dtype=np.float64).reshape(nz + 2, ny + 2, nx + 2)
        b = None
        if case.get("b") is not None:
            b = np.array(case["b"], dtype=np.float64).reshape(nz + 2, ny + 2, nx + 2)
        for impl in (np_sweep, c_sweep):
            v = u
            for _ in range(case["sweeps"]):
                v = impl(v, b)
            got = v[1:-1, 1:-1, 1:-1].ravel().tolist()
            assert got == case["expected_interior"], case["name"]
        if "residual_u0" in case:
            assert oracle.residual_norm(u, b) == case["residual_u0"], case["name"]


# --------------------------------------------------------------- refinement

def test_ir_f64_inner_equals_plain_jacobi():
    """IR with m binary64 Jacobi inner sweeps from d = 0 is plain Jacobi in
    exact arithmetic: (u + d_{j+1}) = (u + d_j) + D^-1 (b - A (u + d_j))."""
    n = (12, 10, 11)
    u0 = synth.boundary_field(n, seed=3)
    b = synth.source_field(n, seed=3)
    m, outer = 20, 6
    u_ir, hist, done, st = oracle.ir_solve(u0, b, storage="f64", inner=m, rtol=0.0, max_inner=m * outer)
    u_pl, _ = oracle.jacobi(u0, m * outer, b)
    scale = np.max(np.abs(u_pl))
    assert done == m * outer and st == 1
    assert np.max(np.abs(u_ir - u_pl)) <= 1e-13 * scale
    u_c, hist_c, done_c, st_c = oracle.c_ir_solve(u0, b, storage="f64", inner=m, rtol=0.0, max_inner=m * outer)
    assert np.array_equal(u_c, u_ir) and done_c == done


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_ir_low_precision_converges_and_certifies(storage):
    n = (10, 9, 8)
    u0 = synth.boundary_field(n, seed=4)
    b = synth.source_field(n, seed=4)
    u, hist, done, st = oracle.ir_solve(u0, b, storage=storage, inner=50, rtol=1e-10, max_inner=20000)
    assert st == 0 and hist[-1] <= 1e-10
    # certificate, computed by the independent residual of the pins module
    r0 = pins.residual_norm(u0, b)
    assert pins.residual_norm(u, b) / r0 <= 1.0001e-10
    # same sweep count as binary64 refinement within one outer step
    _, h64, d64, _ = oracle.ir_solve(u0, b, storage="f64", inner=50, rtol=1e-10, max_inner=20000)
    assert abs(done - d64) <= 100
    # C and NumPy take identical steps
    uc, hc, dc, sc = oracle.c_ir_solve(u0, b, storage=storage, inner=50, rtol=1e-10, max_inner=20000)
    assert np.array_equal(uc, u) and dc == done and sc == st


# ---------------------------------------- refinement in low precision: pins

REFINE_CASES = pins.load_refinement_cases(os.path.join(GOLDEN, "refinement_cases.json"))


def c_ir_step(u, b, storage, m):
    """One outer step of the C oracle: a solve capped at m inner sweeps with
    rtol = 0, which stops after the first correction (or before it, when the
    residual is exactly zero and the correction would be zero too)."""
    u2, hist, done, _ = oracle.c_ir_solve(np.ascontiguousarray(u), None if b is None else
                                          np.ascontiguousarray(b), storage=storage, inner=m,
                                          rtol=0.0, max_inner=m)
    assert done == m or (done == 0 and hist == [0.0])
    return u2


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("check", [pins.check_lo_fixed_points, pins.check_lo_monotone,
                                   pins.check_lo_dense], ids=lambda c: c.__name__)
def test_oracle_inner_sweep_passes_pin(storage, check):
    ok, detail = check(oracle.lo_sweep, storage)
    assert ok, detail


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("impl", [oracle.ir_step, c_ir_step], ids=["numpy", "c"])
def test_oracle_refinement_step_passes_pins(impl, storage):
    ok, detail = pins.check_ir_goldens(impl, storage, REFINE_CASES)
    assert ok, detail
    ok, detail = pins.check_ir_limit(impl, storage)
    assert ok, detail


def test_refinement_goldens_cover_both_storages():
    kinds = {c["storage"] for c in REFINE_CASES}
    assert kinds == {"f32", "bf16"} and len(REFINE_CASES) >= 7


def _bf16_direct(x64):
    """binary64 values rounded once to 8 significand bits (nearest, ties to
    even): the reading the refinement does NOT take (it goes through binary32)."""
    m, e = np.frexp(np.asarray(x64, dtype=np.float64))
    return np.ldexp(np.rint(m * 256.0), e - 8).astype(np.float32)


def _ir_mutant(kind):
    """One outer step of the refinement with one plausible mistake."""
    def step(u, b, storage, m):
        if kind == "f32_outer":
            u32 = u.astype(np.float32)
            b32 = None if b is None else b.astype(np.float32)
            r = oracle.residual_field(u32, b32).astype(np.float64)
        else:
            r = oracle.residual_field(u, b)
        if kind == "direct_bf16":
            rlo = _bf16_direct(r)
        elif kind == "rlo_unrounded":
            rlo = r.astype(np.float32) if storage == "bf16" else r
        else:
            rlo = oracle.residual_lo(r, storage)
        d = np.zeros(u.shape, dtype=np.float32)
        if kind == "inhomogeneous_ghosts":
            d = u.astype(np.float32)
            d[1:-1, 1:-1, 1:-1] = 0.0
        for _ in range(m):
            e = d.copy()
            if kind == "f64_sums":
                s = oracle.neighbour_sum(d.astype(np.float64))
                v = ((s + rlo.astype(np.float64)) / 6.0).astype(np.float32)
            else:
                s = oracle.neighbour_sum(d)
                v = ((s - rlo) if kind == "rlo_sign" else (s + rlo)) / np.float32(6.0)
            e[1:-1, 1:-1, 1:-1] = v if kind == "d_unrounded" else oracle.store_lo(v, storage)
            d = e
        dd = oracle.store_lo(oracle.interior(d), storage).astype(np.float64)
        v = u.copy()
        if kind == "update_sign":
            v[1:-1, 1:-1, 1:-1] = oracle.interior(u) - dd
        elif kind == "f32_update":
            v[1:-1, 1:-1, 1:-1] = (oracle.interior(u).astype(np.float32)
                                   + dd.astype(np.float32)).astype(np.float64)
        else:
            v[1:-1, 1:-1, 1:-1] = oracle.interior(u) + dd
        return v
    return step


IR_MUTANTS = [(k, s) for k in ("rlo_unrounded", "f64_sums", "rlo_sign", "update_sign", "f32_outer",
                               "f32_update", "inhomogeneous_ghosts") for s in ("f32", "bf16")] + \
    [("direct_bf16", "bf16"), ("d_unrounded", "bf16")]


def test_ir_mutant_harness_without_mistake_passes():
    """The mutant builder with no mistake is the oracle's step, bit for bit."""
    rng = np.random.default_rng(5)
    u = rng.random((6, 5, 7))
    b = rng.random((6, 5, 7)) * 2 - 1
    for storage in ("f32", "bf16"):
        assert np.array_equal(_ir_mutant("none")(u, b, storage, 7), oracle.ir_step(u, b, storage, 7))


@pytest.mark.parametrize("kind,storage", IR_MUTANTS, ids=["%s-%s" % m for m in IR_MUTANTS])
def test_ir_planted_mistake_fails_a_pin(kind, storage):
    bad = _ir_mutant(kind)
    results = [pins.check_ir_goldens(bad, storage, REFINE_CASES), pins.check_ir_limit(bad, storage)]
    assert any(not ok for ok, _ in results), "refinement mutant %s/%s passed every pin" % (kind, storage)


def test_ir_cap_counts_inner_sweeps():
    n = (8, 8, 8)
    u0 = synth.boundary_field(n, seed=1)
    b = synth.source_field(n, seed=1)
    u, hist, done, st = oracle.ir_solve(u0, b, storage="f32", inner=50, rtol=1e-30, max_inner=120)
    assert st == 1 and done == 120 and len(hist) == 4


# ------------------------------------------------------------------ bf16

BF16_CASES = [
    (0x3F800000, 0x3F80),  # 1.0 exact
    (0x3F808000, 0x3F80),  # 1 + 2^-8: tie, upper half even -> stays
    (0x3F818000, 0x3F82),  # 1 + 3*2^-8: tie, upper half odd -> up
    (0x3F808001, 0x3F81),  # just above the tie -> up
    (0x3F807FFF, 0x3F80),  # just below the tie -> down
    (0x80000000, 0x8000),  # -0
    (0x7F800000, 0x7F80),  # +inf
    (0x7F7FFFFF, 0x7F80),  # max finite rounds to +inf
    (0xBF7FFFFF, 0xBF80),  # -(1 - 2^-24) rounds to -1
    (0x00000001, 0x0000),  # smallest subnormal -> +0
]


@pytest.mark.parametrize("impl", [oracle.bf16_round, oracle.c_bf16_round], ids=["numpy", "c"])
def test_bf16_known_patterns(impl):
    x = np.array([c[0] for c in BF16_CASES], dtype=np.uint32).view(np.float32)
    got = impl(x)
    assert [int(v) for v in got] == [c[1] for c in BF16_CASES]
    nan = impl(np.array([np.nan], dtype=np.float32))[0]
    assert (int(nan) & 0x7F80) == 0x7F80 and (int(nan) & 0x7F) != 0


def test_bf16_matches_torch_rne():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * 10.0 ** rng.integers(-30, 30, 100000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.bf16_round(x), ref)
    assert np.array_equal(oracle.c_bf16_round(x), ref)
