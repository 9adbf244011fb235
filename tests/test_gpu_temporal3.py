"""Three sweeps per launch (temporal blocking, k_sweep3) against the oracle.

The three-sweep kernel gives every cell's three updates the same sums in
the same order as three one-sweep launches (iterates k + 1 and k + 2 stay in
LDS and registers, rounded to the storage format as stored sweeps would
leave them), so iterates are expected bitwise equal to the oracle's after
any sweep count; a count that is not a multiple of three ends with a
two-sweep launch (remainder 2) or a single sweep (remainder 1)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import Group, Solver, _lib as L  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("mode", ["staged", "fused"])
@pytest.mark.parametrize("rows", [8, 16])
@pytest.mark.parametrize("n,iters,src,zc,t2zc", [
    ((64, 64, 64), 9, False, 0, 0),
    ((70, 19, 37), 7, True, 0, 0),          # ragged tiles, remainder 1
    ((130, 33, 97), 8, False, 32, 0),       # three x tiles, remainder 2
    ((130, 50, 97), 6, True, 0, 13),        # uneven chunks of 12..13 planes
    ((1, 1, 1), 5, False, 0, 0),
    ((2, 3, 1), 4, True, 0, 1),
    ((3, 2, 2), 10, False, 0, 1),           # one-plane chunks, blocks two cells deep
    ((65, 17, 70), 12, True, 16, 0),
    ((127, 40, 33), 11, False, 0, 2),       # odd nx: the last pair holds the x ghost
])
def test_three_sweeps_vs_oracle(mode, rows, n, iters, src, zc, t2zc):
    say("three sweeps", mode, "rows", rows, n, iters, "source" if src else "", "z_chunk", zc, t2zc)
    u0 = synth.boundary_field(n, seed=7)
    b = synth.source_field(n, seed=7) if src else None
    ref, _ = oracle.c_jacobi(u0, iters, b)
    for graphs in (False, True):
        with Solver(n, mode=mode, with_source=src, temporal=3, z_chunk=zc, use_graphs=graphs) as s:
            assert s.temporal_info()["sweeps"] == 3
            if rows != 16 or t2zc:
                s.set_temporal_tiles(rows, t2zc or s.temporal_info()["z_chunk"])
            assert s.temporal_info()["rows"] == rows
            s.load(u0, b)
            s.iterate(iters)
            got = s.store().cpu().numpy()
            assert s.iterations == iters
        assert np.array_equal(got, ref), (graphs, float(np.max(np.abs(got - ref))))


def test_three_sweep_launch_counts():
    """n sweeps take n // 3 three-sweep launches, then one two-sweep launch
    (remainder 2) or one single sweep (remainder 1)."""
    n = (40, 30, 20)
    say("three-sweep launch counts")
    u0 = synth.boundary_field(n, seed=3)
    with Solver(n, temporal=3, use_graphs=False) as s:
        s.load(u0)
        s.set_timing(True)
        s.iterate(7)
        assert s.kernel_time(L.JC_K_SWEEP3)[1] == 2 and s.kernel_time(L.JC_K_SWEEP)[1] == 1
        assert s.kernel_time(L.JC_K_SWEEP2)[1] == 0
        s.iterate(8)
        assert s.kernel_time(L.JC_K_SWEEP3)[1] == 4 and s.kernel_time(L.JC_K_SWEEP2)[1] == 1
        assert s.iterations == 15
        got = s.store().cpu().numpy()
    assert np.array_equal(got, oracle.c_jacobi(u0, 15, None)[0])


def test_three_sweeps_autotune_keeps_results():
    n = (100, 72, 90)
    say("three sweeps autotune")
    u0 = synth.boundary_field(n, seed=9)
    b = synth.source_field(n, seed=9)
    ref, _ = oracle.c_jacobi(u0, 13, b)
    with Solver(n, with_source=True, temporal=3) as s:
        s.load(u0, b)
        s.iterate(5)
        s.autotune(reps=2)
        info = s.temporal_info()
        assert info["sweeps"] == 3 and info["rows"] in (8, 16) and info["z_chunk"] >= 1
        assert s.iterations == 5
        s.iterate(8)
        got = s.store().cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("src", [False, True])
def test_three_sweeps_solve_matches_one_sweep_launches(src):
    """jc_solve with three sweeps per launch: the same checks, residual
    history, stop and iterate as one sweep per launch, and the oracle's."""
    n = (48, 40, 36)
    say("three sweeps solve", "source" if src else "")
    u0 = synth.boundary_field(n, seed=11)
    b = synth.source_field(n, seed=11) if src else None
    out = []
    for temporal in (False, 3):
        with Solver(n, with_source=src, temporal=temporal) as s:
            s.load(u0, b)
            info = s.solve(rtol=1e-6, max_iter=5000, check_every=25, history=True)
            out.append((info, s.store().cpu().numpy()))
    (i0, u_0), (i1, u_1) = out
    assert i0["converged"] and i1["converged"]
    assert i0["iters"] == i1["iters"] and i0["history"] == i1["history"]
    assert np.array_equal(u_0, u_1)
    assert np.array_equal(u_1, oracle.c_jacobi(u0, i1["iters"], b)[0])


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("rows", [8, 16])
@pytest.mark.parametrize("n,inner,t2zc", [((20, 18, 16), 25, 0), ((70, 37, 41), 50, 13), ((2, 3, 1), 4, 1),
                                          ((65, 26, 30), 9, 0), ((33, 20, 17), 6, 5)])
def test_three_sweeps_ir_vs_oracle(dtype, rows, n, inner, t2zc):
    """Refinement with three inner sweeps per launch (iterates k + 1 and
    k + 2 rounded to the storage format) equals the oracle's refinement bit
    for bit; windows of every remainder, and a shorter last window."""
    say("three sweeps IR", dtype, "rows", rows, n, inner, t2zc)
    u0 = synth.boundary_field(n, seed=21)
    b = synth.source_field(n, seed=21)
    total = 2 * inner + 7
    ref, hist, done, _ = oracle.c_ir_solve(u0, b, storage=dtype, inner=inner, rtol=0.0, max_inner=total)
    with Solver(n, with_source=True, ir_dtype=dtype, temporal=3) as s:
        s.set_temporal_tiles(rows, t2zc or s.temporal_info()["z_chunk"])
        s.load(u0, b)
        info = s.solve_ir(inner=inner, rtol=0.0, max_inner=total, history=True)
        got = s.store().cpu().numpy()
    assert info["iters"] == done == total
    rel = [h / info["history"][0] for h in info["history"]]
    np.testing.assert_allclose(rel, hist, rtol=1e-9, atol=1e-15)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("graphs", [False, True])
def test_three_sweep_group_vs_oracle(graphs):
    """A group that sweeps every member three times per launch: members of
    several sizes, with and without a source, starting in either copy; each
    equals the oracle after its own count (windows of every remainder), and
    the residual norms equal a one-sweep group's."""
    specs = [((40, 36, 33), True, 3), ((17, 19, 23), False, 0), ((70, 20, 45), True, 1), ((1, 1, 1), False, 2),
             ((130, 9, 66), False, 5)]
    say("three-sweep group", "graphs" if graphs else "eager")
    norms = []
    for temporal in (3, False):
        solvers, refs = [], []
        for i, (n, src, pre) in enumerate(specs):
            u0 = synth.boundary_field(n, seed=30 + i)
            b = synth.source_field(n, seed=30 + i) if src else None
            s = Solver(n, with_source=src)
            s.load(u0, b)
            s.iterate(pre)
            solvers.append(s)
            refs.append(oracle.c_jacobi(u0, pre + 20, b)[0])
        with Group(solvers, use_graphs=graphs, temporal=temporal) as g:
            g.iterate(7)
            g.iterate(8)
            g.iterate(5)
            norms.append(g.residuals())
        for s, ref, (n, src, pre) in zip(solvers, refs, specs):
            assert s.iterations == pre + 20
            assert np.array_equal(s.store().cpu().numpy(), ref), (temporal, n)
            s.close()
    assert norms[0] == norms[1]


@pytest.mark.parametrize("graphs", [False, True])
def test_three_sweep_group_with_refinement_matches_one_sweep_group(graphs):
    specs = [((40, 36, 33), dict(with_source=True)), ((24, 24, 24), dict(with_source=True, ir_dtype="f32")),
             ((26, 22, 20), dict(with_source=True, ir_dtype="bf16")), ((64, 20, 12), dict(with_source=True,
             ir_dtype="f64")), ((17, 19, 23), {})]
    say("three-sweep group with refinement", "graphs" if graphs else "eager")
    runs = []
    for temporal in (False, 3):
        solvers = []
        for i, (n, kw) in enumerate(specs):
            s = Solver(n, **kw)
            u0 = synth.boundary_field(n, seed=50 + i)
            b = synth.source_field(n, seed=50 + i) if kw.get("with_source") else None
            s.load(u0, b)
            solvers.append(s)
        norms = []
        with Group(solvers, use_graphs=graphs, temporal=temporal) as g:
            for window in (25, 50, 7, 51):
                norms.append(g.residuals())
                g.iterate(window)
            norms.append(g.residuals())
        fields = [s.store().cpu().numpy() for s in solvers]
        iters = [s.iterations for s in solvers]
        for s in solvers:
            s.close()
        runs.append((norms, fields, iters))
    (n0, f0, i0), (n1, f1, i1) = runs
    assert i0 == i1 and n0 == n1
    for a, b in zip(f0, f1):
        assert np.array_equal(a, b)


def test_three_sweep_server_same_results():
    """A server whose lanes sweep three times per launch returns the same
    iterates, sweep counts and residuals as one sweep per launch."""
    from paper_2102_12416_amd.server import Request, Server
    say("three-sweep server")
    reqs = [Request(id=0, arrival=0.0, n=24, precision="f64", seed=701),
            Request(id=1, arrival=0.0, n=40, precision="f64", seed=702),
            Request(id=2, arrival=0.0, n=90, precision="f64", seed=703),
            Request(id=3, arrival=0.0, n=28, precision="f32", seed=704),
            Request(id=4, arrival=0.0, n=16, precision="f64", seed=705)]
    out = []
    for temporal in (False, 3):
        srv = Server(budget_bytes=1 << 34, window=50, rtol=1e-10, max_iter=3000, keep_fields=True,
                     lanes=(32, 64), temporal=temporal)
        out.append(srv.run(reqs, realtime=False))
    for a, b in zip(*out):
        assert (a.id, a.iters, a.converged) == (b.id, b.iters, b.converged)
        assert a.rel_resid == b.rel_resid
        assert np.array_equal(a.field, b.field)


@pytest.mark.parametrize("temporal", [True, 3])
def test_paced_multi_sweep_launches_bitwise(temporal):
    """A pace on the two- or three-sweep launch of a temporal context (set,
    then tuned) only delays work-groups: iterates and refinement results
    stay bitwise the oracle's."""
    n = (130, 50, 97)
    say("paced multi-sweep", temporal)
    u0 = synth.boundary_field(n, seed=17)
    b = synth.source_field(n, seed=17)
    ref, _ = oracle.c_jacobi(u0, 14, b)
    with Solver(n, with_source=True, temporal=temporal, use_graphs=False) as s:
        s.load(u0, b)
        s.set_pace(60)
        assert s.pace == 60
        s.iterate(7)
        p, us_paced, us_free = s.autotune_pace(reps=3)
        assert s.pace == p and us_paced > 0 and us_free > 0
        s.iterate(7)
        assert np.array_equal(s.store().cpu().numpy(), ref)
    ref_ir, _, done, _ = oracle.c_ir_solve(u0, b, storage="bf16", inner=20, rtol=0.0, max_inner=47)
    with Solver(n, with_source=True, ir_dtype="bf16", temporal=temporal) as s:
        s.load(u0, b)
        s.set_pace(80)
        info = s.solve_ir(inner=20, rtol=0.0, max_inner=47)
        assert info["iters"] == done
        assert np.array_equal(s.store().cpu().numpy(), ref_ir)
