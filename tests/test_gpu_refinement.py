"""GPU mixed-precision iterative refinement against the CPU oracle.

The GPU takes the same steps as the oracle's refinement (same sums in the
same order, IEEE division, round-to-nearest-even storage rounding), so the
returned iterate is expected bitwise equal for binary64, binary32 and
bfloat16 storage; the stop is checked against the oracle's own residual
certificate.  With binary64 inner sweeps the refinement is plain Jacobi in
exact arithmetic, so it must agree with the plain GPU path to 1e-13.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import Solver  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,bd", [((20, 18, 16), None), ((33, 26, 21), (17, 13, 11))])
def test_ir_matches_oracle_steps(dtype, n, bd):
    say("IR", dtype, n, bd)
    u0 = synth.boundary_field(n, seed=21)
    b = synth.source_field(n, seed=21)
    ref, hist, done, st = oracle.c_ir_solve(u0, b, storage=dtype, inner=25, rtol=1e-10, max_inner=4000)
    kw = {} if bd is None else dict(block_dims=bd, mode="fused")
    with Solver(n, with_source=True, ir_dtype=dtype, **kw) as s:
        s.load(u0, b)
        info = s.solve_ir(inner=25, rtol=1e-10, max_inner=4000, history=True)
        u = s.store().cpu().numpy()
    assert info["iters"] == done
    assert info["converged"] == (st == 0)
    rel = [h / info["history"][0] for h in info["history"]]
    np.testing.assert_allclose(rel, hist, rtol=1e-9, atol=1e-15)
    assert np.array_equal(u, ref)


def test_ir_f64_inner_equals_plain_jacobi():
    n = (24, 20, 18)
    say("IR f64 inner vs plain", n)
    u0 = synth.boundary_field(n, seed=22)
    b = synth.source_field(n, seed=22)
    with Solver(n, with_source=True, ir_dtype="f64") as s:
        s.load(u0, b)
        s.solve_ir(inner=30, rtol=0.0, max_inner=300)
        u_ir = s.store().cpu().numpy()
    with Solver(n, with_source=True) as p:
        p.load(u0, b)
        p.iterate(300)
        u_pl = p.store().cpu().numpy()
    assert np.max(np.abs(u_ir - u_pl)) <= 1e-13 * np.max(np.abs(u_pl))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ir_certified_to_tolerance(dtype):
    n = (28, 28, 28)
    say("IR certificate", dtype, n)
    u0 = synth.boundary_field(n, seed=23)
    b = synth.source_field(n, seed=23)
    with Solver(n, block_dims=(14, 14, 28), mode="fused", with_source=True, ir_dtype=dtype) as s:
        s.load(u0, b)
        info = s.solve_ir(inner=50, rtol=1e-10, max_inner=20000)
        u = s.store().cpu().numpy()
    assert info["converged"]
    r0 = oracle.c_residual_norm(u0, b)
    assert oracle.c_residual_norm(u, b) / r0 <= 1e-10 * (1 + 1e-9)
    # error against the binary64 refinement's answer at the same tolerance
    u64, _, _, _ = oracle.c_ir_solve(u0, b, storage="f64", inner=50, rtol=1e-10, max_inner=20000)
    err = np.max(np.abs(u - u64)) / np.max(np.abs(u64))
    print("[result] %s max rel error vs binary64 refinement: %.3e" % (dtype, err), flush=True)
    assert err < 1e-6
