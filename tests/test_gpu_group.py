"""Groups: many independent contexts in shared launches.

Each member's iterate after a run of windows is bitwise the same alone
(a one-member group), in a mix with other members of other sizes and
precisions, and through its own context's path; the residual norms a
group reports match each member's own within the reduction-order bar.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import Group, Solver  # noqa: E402

SPECS = [
    dict(n=(40, 36, 33), kw=dict(with_source=True)),
    dict(n=(24, 24, 24), kw=dict(with_source=True, ir_dtype="f32")),
    dict(n=(30, 28, 26), kw=dict(with_source=True, block_dims=(15, 14, 26), mode="fused")),
    dict(n=(17, 19, 23), kw=dict(with_source=False)),
    dict(n=(26, 22, 20), kw=dict(with_source=True, ir_dtype="bf16", block_dims=(13, 22, 10))),
    dict(n=(64, 20, 12), kw=dict(with_source=True, ir_dtype="f64")),
]


def say(*a):
    print("[case]", *a, flush=True)


def make(spec, seed):
    n = spec["n"]
    s = Solver(n, **spec["kw"])
    u0 = synth.boundary_field(n, seed=seed)
    b = synth.source_field(n, seed=seed) if spec["kw"].get("with_source") else None
    s.load(u0, b)
    return s


def run(indices, windows=4, window=50):
    solvers = [make(SPECS[i], seed=100 + i) for i in indices]
    hist = []
    with Group(solvers) as g:
        for _ in range(windows):
            hist.append(g.residuals())
            g.iterate(window)
        hist.append(g.residuals())
    out = [s.store().cpu().numpy() for s in solvers]
    for s in solvers:
        s.close()
    return out, np.array(hist)


def test_alone_equals_mix():
    say("group alone vs mix")
    mix, hmix = run(range(len(SPECS)))
    for i in range(len(SPECS)):
        alone, halone = run([i])
        assert np.array_equal(alone[0], mix[i]), i
        assert np.array_equal(halone[:, 0], hmix[:, i]), i


def test_group_matches_own_path_and_oracle():
    say("group vs own path")
    res, hist = run([0, 3, 1], windows=3, window=50)
    # plain members: 150 sweeps of the oracle
    for k, i in ((0, 0), (1, 3)):
        n = SPECS[i]["n"]
        u0 = synth.boundary_field(n, seed=100 + i)
        b = synth.source_field(n, seed=100 + i) if SPECS[i]["kw"].get("with_source") else None
        ref, rh = oracle.c_jacobi(u0, 150, b, every=50)
        assert np.array_equal(res[k], ref)
        np.testing.assert_allclose(hist[:, k], rh, rtol=1e-12)
    # refining member: three outer steps of 50 inner sweeps, as the oracle's refinement
    n = SPECS[1]["n"]
    u0 = synth.boundary_field(n, seed=101)
    b = synth.source_field(n, seed=101)
    ref, rh, done, _ = oracle.c_ir_solve(u0, b, storage="f32", inner=50, rtol=0.0, max_inner=150)
    assert done == 150
    assert np.array_equal(res[2], ref)
    np.testing.assert_allclose(hist[:, 2] / hist[0, 2], rh, rtol=1e-9)


def test_group_tile_shape_keeps_results():
    say("group tile shapes")
    ref, _ = run([0, 2, 3])
    for tile in ((32, 4, 16), (64, 32, 7), (16, 8, 16)):
        solvers = [make(SPECS[i], seed=100 + i) for i in (0, 2, 3)]
        with Group(solvers, tile=tile) as g:
            for _ in range(4):
                g.residuals()
                g.iterate(50)
            g.residuals()
        got = [s.store().cpu().numpy() for s in solvers]
        for s in solvers:
            s.close()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), tile


def test_mixed_refinement_steps_need_residuals_first():
    """Two refining members that left different groups at different points
    of their step cannot share a launch until jc_group_residuals brings
    both to the same point; the results then still equal the oracle's."""
    import oracle
    import synth
    from paper_2102_12416_amd import Group, JcError, Solver, _lib as L
    n = (20, 18, 16)
    us = [synth.boundary_field(n, seed=71 + i) for i in range(2)]
    bs = [synth.source_field(n, seed=71 + i) for i in range(2)]
    a = Solver(n, with_source=True, ir_dtype="f32").load(us[0], bs[0])
    b = Solver(n, with_source=True, ir_dtype="f32").load(us[1], bs[1])
    with Group([a]) as g:
        g.residuals()
        g.iterate(10)             # a: inner sweeps ran, correction pending
    with Group([b]) as g:
        g.residuals()             # b: r_lo current, no sweeps yet
    with Group([a, b]) as g:
        with pytest.raises(JcError) as e:
            g.iterate(10)
        assert e.value.code == L.JC_ERR_STATE
        g.residuals()
        g.iterate(10)
        g.residuals()
    for s, u0, b0, sweeps in ((a, us[0], bs[0], 20), (b, us[1], bs[1], 10)):
        ref, _, done, _ = oracle.c_ir_solve(u0, b0, storage="f32", inner=10, rtol=0.0, max_inner=sweeps)
        assert done == sweeps
        assert np.array_equal(s.store().cpu().numpy(), ref)
    a.close()
    b.close()
