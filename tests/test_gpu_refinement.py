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


# ----------------------------------------------------------- full size 1024^3

def _box(n, cell, radius):
    P = (n[2] + 2, n[1] + 2, n[0] + 2)
    lo = [max(0, c - radius) for c in cell]
    hi = [min(P[a], cell[a] + radius + 1) for a in range(3)]
    return lo, hi


def _ir_local_oracle(n, seed, cell, dtype, inner):
    """u after one outer step of `inner` sweeps at one cell: the oracle's
    refinement on the box of radius inner + 2 around it.  The box edge
    holds the exact initial iterate (so the residual is exact) and zero
    corrections, whose error moves one cell per inner sweep and never
    reaches the centre."""
    lo, hi = _box(n, cell, inner + 2)
    u_box = synth.field_box(n, 0, lo, hi, seed=seed)
    b_box = synth.field_box(n, 1, lo, hi, seed=seed)
    ref, _, done, _ = oracle.c_ir_solve(u_box, b_box, storage=dtype, inner=inner, rtol=0.0, max_inner=inner)
    assert done == inner
    return ref[cell[0] - lo[0], cell[1] - lo[1], cell[2] - lo[2]]


def _plain_local_oracle(n, seed, cell, k):
    """Iterate k of the plain sweep with a source at one cell, from the box
    of radius k + 1 around it."""
    lo, hi = _box(n, cell, k + 1)
    box = synth.field_box(n, 0, lo, hi, seed=seed)
    bb = synth.field_box(n, 1, lo, hi, seed=seed)
    for _ in range(k):
        box = oracle.sweep(box, bb)
    return box[cell[0] - lo[0], cell[1] - lo[1], cell[2] - lo[2]]


_CELLS_1024 = [(1, 1, 1), (1024, 1024, 1024), (1, 512, 1024), (1024, 1, 513), (512, 512, 512),
               (513, 1024, 1), (2, 700, 31), (900, 33, 1023)]


def _sample(u, cells):
    import torch
    idx = torch.tensor(cells, device=u.device)
    return u[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()


def _cells_1024():
    rng = np.random.default_rng(1024)
    return _CELLS_1024 + [tuple(int(v) for v in rng.integers(1, 1025, 3)) for _ in range(6)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ir_full_size_1024_sampled(dtype):
    """1024^3 with a source in the launch configuration of the refinement
    benchmark (one block, tile from jc_autotune of the inner sweep, eager
    launches): one outer step of 50 inner sweeps; sampled cells equal the
    oracle's local refinement bit for bit."""
    from paper_2102_12416_amd import synth_field
    n, seed = (1024, 1024, 1024), 12416
    say("IR 1024^3", dtype, "one outer step, sampled")
    cells = _cells_1024()
    with Solver(n, with_source=True, ir_dtype=dtype, use_graphs=False) as s:
        g = synth_field(n, seed, 0)
        b = synth_field(n, seed, 1)
        # the device generator draws the input module's values
        lo, hi = [0, 500, 1000], [3, 530, 1026]
        assert np.array_equal(g[0:3, 500:530, 1000:1026].cpu().numpy(), synth.field_box(n, 0, lo, hi, seed=seed))
        assert np.array_equal(b[0:3, 500:530, 1000:1026].cpu().numpy(), synth.field_box(n, 1, lo, hi, seed=seed))
        s.load(g, b)
        del g, b
        s.autotune(reps=2)
        info = s.solve_ir(inner=50, rtol=0.0, max_inner=50)
        got = _sample(s.store(), cells)
    assert info["iters"] == 50 and not info["converged"]
    for c, v in zip(cells, got):
        assert v == _ir_local_oracle(n, seed, c, dtype, 50), c


def test_plain_source_full_size_1024_sampled():
    """The binary64 sweep with a source at 1024^3 as the refinement
    benchmark times it (tile from jc_autotune, eager launches): sampled cells
    after 6 sweeps equal the oracle's local computation bit for bit."""
    from paper_2102_12416_amd import synth_field
    n, seed = (1024, 1024, 1024), 12416
    say("plain with source 1024^3, sampled")
    cells = _cells_1024()
    with Solver(n, with_source=True, use_graphs=False) as s:
        s.load(synth_field(n, seed, 0), synth_field(n, seed, 1))
        s.autotune(reps=2)
        s.iterate(6)
        got = _sample(s.store(), cells)
    for c, v in zip(cells, got):
        assert v == _plain_local_oracle(n, seed, c, 6), c


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ir_sixteen_cell_tiles_match_oracle(dtype):
    """The refinement passes with 16-cell tiles (8 threads per row) equal
    the oracle's refinement bit for bit."""
    n, bd = (37, 29, 23), (19, 15, 23)
    say("IR 16-cell tiles", dtype)
    u0 = synth.boundary_field(n, seed=31)
    b = synth.source_field(n, seed=31)
    ref, _, done, _ = oracle.c_ir_solve(u0, b, storage=dtype, inner=20, rtol=0.0, max_inner=200)
    with Solver(n, block_dims=bd, mode="fused", with_source=True, ir_dtype=dtype, tile_x=16, tile_y=8,
                z_chunk=16) as s:
        assert s.tile_info()["tile_x"] == 16
        s.load(u0, b)
        info = s.solve_ir(inner=20, rtol=0.0, max_inner=200)
        u = s.store().cpu().numpy()
    assert info["iters"] == done == 200
    assert np.array_equal(u, ref)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ir_autotune_keeps_results(dtype):
    """jc_autotune on a refinement context times the inner sweep; the
    refinement afterwards equals the oracle's bit for bit."""
    n, bd = (40, 34, 30), (20, 34, 15)
    say("IR autotune", dtype)
    u0 = synth.boundary_field(n, seed=41)
    b = synth.source_field(n, seed=41)
    ref, _, done, _ = oracle.c_ir_solve(u0, b, storage=dtype, inner=25, rtol=0.0, max_inner=150)
    with Solver(n, block_dims=bd, mode="fused", with_source=True, ir_dtype=dtype) as s:
        s.load(u0, b)
        tx, ty, zc, us = s.autotune(reps=2)
        assert tx in (16, 32, 64) and (tx // 2) * ty >= 64 and zc >= 1 and us > 0
        info = s.solve_ir(inner=25, rtol=0.0, max_inner=150)
        u = s.store().cpu().numpy()
    assert info["iters"] == done == 150
    assert np.array_equal(u, ref)


def test_ir_autotune_refused_during_a_group_step():
    """A group leaves a refining member mid-step (its r_lo current);
    autotuning it then would destroy that state and is refused."""
    from paper_2102_12416_amd import Group, JcError, _lib as L
    n = (24, 24, 24)
    say("IR autotune state")
    u0 = synth.boundary_field(n, seed=42)
    b = synth.source_field(n, seed=42)
    with Solver(n, with_source=True, ir_dtype="f32") as s:
        s.load(u0, b)
        with Group([s]) as g:
            g.residuals()
        with pytest.raises(JcError) as e:
            s.autotune(reps=1)
        assert e.value.code == L.JC_ERR_STATE
        s.solve_ir(inner=10, rtol=0.0, max_inner=10)     # starts afresh
        s.autotune(reps=1)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ir_one_cell_blocks(dtype):
    """Refinement on blocks one cell wide in x and y."""
    n, bd = (6, 5, 7), (1, 1, 7)
    say("IR one-cell blocks", dtype)
    u0 = synth.boundary_field(n, seed=62)
    b = synth.source_field(n, seed=62)
    ref, _, done, _ = oracle.c_ir_solve(u0, b, storage=dtype, inner=10, rtol=0.0, max_inner=60)
    with Solver(n, block_dims=bd, mode="fused", with_source=True, ir_dtype=dtype) as s:
        s.load(u0, b)
        info = s.solve_ir(inner=10, rtol=0.0, max_inner=60)
        u = s.store().cpu().numpy()
    assert info["iters"] == done == 60
    assert np.array_equal(u, ref)
