"""Temporal blocking (two sweeps per launch) against the CPU oracle.

The two-sweep kernel gives every cell's two updates the same sums in the
same order as two one-sweep launches (iterate k + 1 stays in LDS and
registers), so the iterate is expected bitwise equal to the oracle's after
any number of sweeps; an odd count ends with one single sweep."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import Solver, _lib as L  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("mode", ["staged", "fused"])
@pytest.mark.parametrize("rows", [8, 16, 24])
@pytest.mark.parametrize("n,iters,src,zc,t2zc", [
    ((64, 64, 64), 10, False, 0, 0),
    ((70, 19, 37), 7, True, 0, 0),          # ragged tile in x and y, odd count
    ((130, 33, 97), 8, False, 32, 0),       # three z chunks, three x tiles
    ((130, 50, 97), 6, True, 0, 13),        # eight uneven chunks of 12..13 planes
    ((1, 1, 1), 5, False, 0, 0),
    ((2, 3, 1), 4, True, 0, 1),
    ((65, 17, 70), 9, True, 16, 0),         # z_chunk below the two-sweep minimum
    ((127, 40, 33), 6, False, 0, 2),        # odd nx: the last pair holds the x ghost
])
def test_temporal_vs_oracle(mode, rows, n, iters, src, zc, t2zc):
    say("temporal", mode, "rows", rows, n, iters, "source" if src else "", "z_chunk", zc, t2zc)
    u0 = synth.boundary_field(n, seed=7)
    b = synth.source_field(n, seed=7) if src else None
    ref, _ = oracle.c_jacobi(u0, iters, b)
    for graphs in (False, True):
        with Solver(n, mode=mode, with_source=src, temporal=True, z_chunk=zc, use_graphs=graphs) as s:
            if rows != 16 or t2zc:
                s.set_temporal_tiles(rows, t2zc or s.temporal_info()["z_chunk"])
            assert s.temporal_info()["rows"] == rows
            s.load(u0, b)
            s.iterate(iters)
            got = s.store().cpu().numpy()
            assert s.iterations == iters
        assert np.array_equal(got, ref), (graphs, float(np.max(np.abs(got - ref))))


def test_temporal_autotune_keeps_results():
    """jc_autotune on a temporal context also picks the two-sweep shape;
    the iterate is unchanged by the trials and later sweeps stay exact."""
    n = (100, 72, 90)
    say("temporal autotune")
    u0 = synth.boundary_field(n, seed=9)
    b = synth.source_field(n, seed=9)
    ref, _ = oracle.c_jacobi(u0, 12, b)
    with Solver(n, with_source=True, temporal=True) as s:
        s.load(u0, b)
        s.iterate(5)
        s.autotune(reps=2)
        info = s.temporal_info()
        assert info["rows"] in (8, 16, 24) and info["z_chunk"] >= 1
        assert s.iterations == 5
        s.iterate(7)
        got = s.store().cpu().numpy()
    assert np.array_equal(got, ref)


def test_temporal_launch_counts():
    """n sweeps take n // 2 two-sweep launches and n % 2 single sweeps."""
    n = (40, 30, 20)
    say("temporal launch counts")
    with Solver(n, temporal=True, use_graphs=False) as s:
        s.load(synth.boundary_field(n, seed=3))
        s.set_timing(True)
        s.iterate(7)
        assert s.kernel_time(L.JC_K_SWEEP2)[1] == 3
        assert s.kernel_time(L.JC_K_SWEEP)[1] == 1
        s.iterate(4)
        assert s.kernel_time(L.JC_K_SWEEP2)[1] == 5
        assert s.kernel_time(L.JC_K_SWEEP)[1] == 1
        assert s.iterations == 11


@pytest.mark.parametrize("src", [False, True])
def test_temporal_solve_matches_one_sweep_launches(src):
    """jc_solve with temporal blocking: the same checks, residual history,
    stop and iterate as with one sweep per launch."""
    n = (48, 40, 36)
    say("temporal solve", "source" if src else "")
    u0 = synth.boundary_field(n, seed=11)
    b = synth.source_field(n, seed=11) if src else None
    out = []
    for temporal in (False, True):
        with Solver(n, with_source=src, temporal=temporal) as s:
            s.load(u0, b)
            info = s.solve(rtol=1e-6, max_iter=5000, check_every=25, history=True)
            out.append((info, s.store().cpu().numpy()))
    (i0, u_0), (i1, u_1) = out
    assert i0["converged"] and i1["converged"]
    assert i0["iters"] == i1["iters"]
    assert i0["history"] == i1["history"]
    assert np.array_equal(u_0, u_1)
    ref, _ = oracle.c_jacobi(u0, i1["iters"], b)
    assert np.array_equal(u_1, ref)


def test_temporal_full_size_paper_share():
    """The per-GPU block of the paper's largest Jacobi3D run (512 x 768 x
    1536, one block) in the launch configuration the benchmark times with
    temporal blocking (fused mode, its stored two-sweep shape, graph
    replay): sampled cells after 6
    sweeps equal the oracle's local computation; after 41 sweeps the
    iterate equals the one-sweep launches bit for bit."""
    import torch
    from paper_2102_12416_amd import synth_field
    n, seed = (512, 768, 1536), 12416
    say("temporal 512x768x1536, sampled + bitwise vs one-sweep launches")
    rng = np.random.default_rng(5)
    cells = [tuple(int(rng.integers(1, m + 1)) for m in (n[2], n[1], n[0])) for _ in range(16)]
    cells += [(1, 1, 1), (1536, 768, 512), (1, 768, 1), (1536, 1, 512), (768, 384, 256), (2, 17, 511)]
    from bench import TUNED_TEMPORAL
    rows, zc = TUNED_TEMPORAL["paper_share"]
    with Solver(n, mode="fused", temporal=True) as s:
        s.set_temporal_tiles(rows, zc)
        s.load(synth_field(n, seed, 0))
        s.iterate(6)
        u = s.store()
        idx = torch.tensor(cells, device=u.device)
        got = u[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
        del u
        for c, v in zip(cells, got):
            lo = [max(0, c[a] - 7) for a in range(3)]
            hi = [min((n[2], n[1], n[0])[a] + 2, c[a] + 8) for a in range(3)]
            box = synth.field_box(n, 0, lo, hi, seed=seed)
            for _ in range(6):
                box = oracle.sweep(box)
            assert v == box[c[0] - lo[0], c[1] - lo[1], c[2] - lo[2]], c
        s.iterate(35)
        assert s.iterations == 41
        a = s.store()
        with Solver(n, mode="fused") as one:
            one.load(synth_field(n, seed, 0))
            one.iterate(41)
            assert torch.equal(a, one.store())


def test_temporal_full_size_1024_source_sampled():
    """1024^3 with a source, two sweeps per launch in the configuration the
    refinement benchmark times (shape from jc_autotune, eager launches):
    sampled cells after 6 sweeps equal the oracle's local computation."""
    import torch
    from paper_2102_12416_amd import synth_field
    n, seed = (1024, 1024, 1024), 12416
    say("temporal 1024^3 with source, sampled")
    rng = np.random.default_rng(1024)
    cells = [(1, 1, 1), (1024, 1024, 1024), (1, 512, 1024), (1024, 1, 513), (512, 512, 512), (513, 1024, 1)]
    cells += [tuple(int(v) for v in rng.integers(1, 1025, 3)) for _ in range(8)]
    with Solver(n, with_source=True, use_graphs=False, temporal=True) as s:
        s.load(synth_field(n, seed, 0), synth_field(n, seed, 1))
        s.autotune(reps=2)
        s.iterate(6)
        u = s.store()
        idx = torch.tensor(cells, device=u.device)
        got = u[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    for c, v in zip(cells, got):
        lo = [max(0, c[a] - 7) for a in range(3)]
        hi = [min(1026, c[a] + 8) for a in range(3)]
        box = synth.field_box(n, 0, lo, hi, seed=seed)
        bb = synth.field_box(n, 1, lo, hi, seed=seed)
        for _ in range(6):
            box = oracle.sweep(box, bb)
        assert v == box[c[0] - lo[0], c[1] - lo[1], c[2] - lo[2]], c


# ------------------------------------------------ refinement inner sweeps

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("rows", [8, 16, 24])
@pytest.mark.parametrize("n,inner,t2zc", [((20, 18, 16), 25, 0), ((70, 37, 41), 50, 13), ((2, 3, 1), 4, 1),
                                          ((65, 26, 30), 9, 0)])
def test_temporal_ir_vs_oracle(dtype, rows, n, inner, t2zc):
    """Refinement with two inner sweeps per launch (iterate k + 1 rounded to
    the storage format between them) equals the oracle's refinement bit
    for bit; the last window is shorter than the others (7 sweeps)."""
    say("temporal IR", dtype, "rows", rows, n, inner, t2zc)
    u0 = synth.boundary_field(n, seed=21)
    b = synth.source_field(n, seed=21)
    total = 2 * inner + 7
    ref, hist, done, _ = oracle.c_ir_solve(u0, b, storage=dtype, inner=inner, rtol=0.0, max_inner=total)
    with Solver(n, with_source=True, ir_dtype=dtype, temporal=True) as s:
        s.set_temporal_tiles(rows, t2zc or s.temporal_info()["z_chunk"])
        s.load(u0, b)
        info = s.solve_ir(inner=inner, rtol=0.0, max_inner=total, history=True)
        got = s.store().cpu().numpy()
    assert info["iters"] == done == total
    rel = [h / info["history"][0] for h in info["history"]]
    np.testing.assert_allclose(rel, hist, rtol=1e-9, atol=1e-15)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_temporal_ir_full_size_1024_sampled(dtype):
    """1024^3 with a source, refinement with two inner sweeps per launch in
    the configuration the refinement benchmark times (shape from
    jc_autotune, eager launches): one outer step of 50 inner sweeps;
    sampled cells equal the oracle's local refinement bit for bit."""
    import torch
    from paper_2102_12416_amd import synth_field
    n, seed, inner = (1024, 1024, 1024), 12416, 50
    say("temporal IR 1024^3", dtype)
    rng = np.random.default_rng(77)
    cells = [(1, 1, 1), (1024, 1024, 1024), (1, 512, 1024), (1024, 1, 513), (512, 512, 512)]
    cells += [tuple(int(v) for v in rng.integers(1, 1025, 3)) for _ in range(5)]
    with Solver(n, with_source=True, ir_dtype=dtype, use_graphs=False, temporal=True) as s:
        s.load(synth_field(n, seed, 0), synth_field(n, seed, 1))
        s.autotune(reps=2)
        info = s.solve_ir(inner=inner, rtol=0.0, max_inner=inner)
        u = s.store()
        idx = torch.tensor(cells, device=u.device)
        got = u[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    assert info["iters"] == inner
    for c, v in zip(cells, got):
        lo = [max(0, c[a] - inner - 2) for a in range(3)]
        hi = [min(1026, c[a] + inner + 3) for a in range(3)]
        u_box = synth.field_box(n, 0, lo, hi, seed=seed)
        b_box = synth.field_box(n, 1, lo, hi, seed=seed)
        ref, _, done, _ = oracle.c_ir_solve(u_box, b_box, storage=dtype, inner=inner, rtol=0.0, max_inner=inner)
        assert done == inner
        assert v == ref[c[0] - lo[0], c[1] - lo[1], c[2] - lo[2]], c


def test_temporal_shape_change_replaces_graphs():
    """Windows captured as graphs with one two-sweep shape are dropped when
    the shape changes: later windows use the new shape and stay exact."""
    n = (90, 41, 50)
    say("temporal shape change with graphs")
    u0 = synth.boundary_field(n, seed=13)
    ref, _ = oracle.c_jacobi(u0, 40, None)
    with Solver(n, mode="fused", temporal=True, use_graphs=True) as s:
        s.load(u0)
        s.iterate(10)
        s.iterate(10)                   # replays the captured 10-sweep window
        s.set_temporal_tiles(24, 7)
        assert s.temporal_info()["rows"] == 24
        s.iterate(10)
        s.set_temporal_tiles(8, 50)
        s.iterate(10)
        assert s.iterations == 40
        got = s.store().cpu().numpy()
    assert np.array_equal(got, ref)


# ------------------------------------------------------------------ groups

@pytest.mark.parametrize("tile", [None, (32, 8, 16)])
@pytest.mark.parametrize("graphs", [False, True])
def test_temporal_group_vs_oracle(graphs, tile):
    """A group that sweeps every member twice per launch: members of several
    sizes, with and without a source (two kernel classes), starting from
    different copies; each equals the oracle after its own sweep count, and
    the group's residual norms equal a one-sweep-per-launch group's."""
    from paper_2102_12416_amd import Group
    specs = [((40, 36, 33), True, 3), ((17, 19, 23), False, 0), ((70, 20, 45), True, 1), ((1, 1, 1), False, 2),
             ((130, 9, 66), False, 5)]
    say("temporal group", "graphs" if graphs else "eager", "tile", tile)
    norms = []
    for temporal in (True, False):
        solvers, refs = [], []
        for i, (n, src, pre) in enumerate(specs):
            u0 = synth.boundary_field(n, seed=30 + i)
            b = synth.source_field(n, seed=30 + i) if src else None
            s = Solver(n, with_source=src)
            s.load(u0, b)
            s.iterate(pre)                       # members start in either copy
            solvers.append(s)
            refs.append(oracle.c_jacobi(u0, pre + 17, b)[0])
        with Group(solvers, use_graphs=graphs, temporal=temporal, tile=tile) as g:
            g.iterate(7)
            g.iterate(10)
            norms.append(g.residuals())
        for s, ref, (n, src, pre) in zip(solvers, refs, specs):
            assert s.iterations == pre + 17
            assert np.array_equal(s.store().cpu().numpy(), ref), (temporal, n)
            s.close()
    assert norms[0] == norms[1]


def test_temporal_group_needs_one_block_members():
    from paper_2102_12416_amd import Group, JcError, _lib as L
    say("temporal group validation")
    n = (24, 20, 18)
    with Solver(n, block_dims=(12, 20, 18), mode="fused") as a:
        a.load(synth.boundary_field(n, seed=1))
        with pytest.raises(JcError) as e:
            Group([a], temporal=True)
        assert e.value.code == L.JC_ERR_INVALID


@pytest.mark.parametrize("tile", [None, (32, 8, 16)])
@pytest.mark.parametrize("graphs", [False, True])
def test_temporal_group_with_refinement_matches_one_sweep_group(graphs, tile):
    """Refining members (binary64, binary32, bfloat16 storage) beside plain
    ones in a group that sweeps twice per launch: after outer steps with
    odd and even window lengths, every member's iterate and residual norm
    equal those of the same group sweeping once per launch."""
    from paper_2102_12416_amd import Group
    specs = [((40, 36, 33), dict(with_source=True)), ((24, 24, 24), dict(with_source=True, ir_dtype="f32")),
             ((26, 22, 20), dict(with_source=True, ir_dtype="bf16")), ((64, 20, 12), dict(with_source=True,
             ir_dtype="f64")), ((30, 18, 41), dict(with_source=True, ir_dtype="f32")), ((17, 19, 23), {})]
    say("temporal group with refinement", "graphs" if graphs else "eager")
    runs = []
    for temporal in (False, True):
        solvers = []
        for i, (n, kw) in enumerate(specs):
            s = Solver(n, **kw)
            u0 = synth.boundary_field(n, seed=50 + i)
            b = synth.source_field(n, seed=50 + i) if kw.get("with_source") else None
            s.load(u0, b)
            solvers.append(s)
        norms = []
        with Group(solvers, use_graphs=graphs, temporal=temporal, tile=tile) as g:
            for window in (25, 50, 7, 50):
                norms.append(g.residuals())
                g.iterate(window)
            norms.append(g.residuals())
        fields = [s.store().cpu().numpy() for s in solvers]
        iters = [s.iterations for s in solvers]
        for s in solvers:
            s.close()
        runs.append((norms, fields, iters))
    (n0, f0, i0), (n1, f1, i1) = runs
    assert i0 == i1
    assert n0 == n1
    for a, b in zip(f0, f1):
        assert np.array_equal(a, b)


def test_temporal_server_same_results():
    """A server whose lanes sweep twice per launch (temporal=True keeps its
    size lanes per precision, binary64 and binary32-refined, and every lane
    takes two sweeps per launch) returns the same iterates, sweep counts and
    residuals as one sweep per launch."""
    from paper_2102_12416_amd.server import Request, Server
    say("temporal server")
    reqs = [Request(id=0, arrival=0.0, n=24, precision="f64", seed=701),
            Request(id=1, arrival=0.0, n=40, precision="f64", seed=702),
            Request(id=2, arrival=0.0, n=90, precision="f64", seed=703),
            Request(id=3, arrival=0.0, n=28, precision="f32", seed=704),
            Request(id=4, arrival=0.0, n=16, precision="f64", seed=705)]
    out = []
    for temporal in (False, True):
        srv = Server(budget_bytes=1 << 34, window=50, rtol=1e-10, max_iter=3000, keep_fields=True,
                     lanes=(32, 64), temporal=temporal)
        out.append(srv.run(reqs, realtime=False))
    for a, b in zip(*out):
        assert (a.id, a.iters, a.converged) == (b.id, b.iters, b.converged)
        assert a.rel_resid == b.rel_resid
        assert np.array_equal(a.field, b.field)
