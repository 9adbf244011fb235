"""The continuous-batching solve server on the GPU."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd.server import Request, Server, request_footprint, summarize  # noqa: E402

REQS = [Request(id=0, arrival=0.0, n=24, precision="f64", seed=501),
        Request(id=1, arrival=0.0, n=32, precision="f32", seed=502),
        Request(id=2, arrival=0.0, n=20, precision="f32", seed=503),
        Request(id=3, arrival=0.0, n=40, precision="f64", seed=504),
        Request(id=4, arrival=0.0, n=28, precision="f32", seed=505),
        Request(id=5, arrival=0.0, n=16, precision="f64", seed=506)]


def say(*a):
    print("[case]", *a, flush=True)


def serve(reqs, budget=1 << 34, max_iter=1500, lanes=(64, 160)):
    srv = Server(budget_bytes=budget, window=50, rtol=1e-10, max_iter=max_iter, keep_fields=True, lanes=lanes)
    res = srv.run(reqs, realtime=False)
    return srv, res


def test_each_result_same_alone_and_in_mix():
    say("server alone vs mix")
    _, mix = serve(REQS)
    for r in REQS:
        _, alone = serve([r])
        a, m = alone[0], mix[r.id]
        assert a.iters == m.iters and a.converged == m.converged, r.id
        assert np.array_equal(a.field, m.field), r.id


@pytest.mark.parametrize("lanes", [(), (24,), (20, 28)])
def test_lanes_do_not_change_results(lanes):
    say("server lanes", lanes)
    _, one = serve(REQS, lanes=())
    srv, split = serve(REQS, lanes=lanes)
    assert len(srv.stats["lane_windows"]) == len(lanes) + 1
    for a, m in zip(one, split):
        assert a.iters == m.iters and a.converged == m.converged and a.rel_resid == m.rel_resid, a.id
        assert np.array_equal(a.field, m.field), a.id


def test_results_certified_by_oracle():
    say("server certificates")
    _, res = serve(REQS, max_iter=3000)
    for r, out in zip(REQS, res):
        n = (r.n,) * 3
        u0 = synth.boundary_field(n, seed=r.seed)
        b = synth.source_field(n, seed=r.seed)
        rel = oracle.c_residual_norm(out.field, b) / oracle.c_residual_norm(u0, b)
        if out.converged:
            assert rel <= 1e-10 * (1 + 1e-9), r.id
        else:
            assert out.iters == 3000
        assert abs(rel - out.rel_resid) <= 1e-9 * max(rel, 1e-300) + 1e-14, r.id
        if r.precision == "f64" and out.converged:
            # the plain solve is the oracle's own Jacobi, stopped at the same check
            ref, _ = oracle.c_jacobi(u0, out.iters, b)
            assert np.array_equal(out.field, ref)


def test_admission_respects_budget_and_rejects_oversize():
    say("server budget")
    sizes = [request_footprint(r.n, r.precision) for r in REQS]
    budget = max(sizes) + min(sizes)           # forces queueing
    big = Request(id=99, arrival=0.0, n=200, precision="f64", seed=1)
    assert request_footprint(200, "f64") > budget
    srv, res = serve(REQS + [big], budget=budget, max_iter=500)
    assert srv.stats["peak_bytes"] <= budget
    assert res[-1].rejected and not any(r.rejected for r in res[:-1])
    s = summarize(res, makespan=1.0)
    assert s["served"] == len(REQS) and s["rejected"] == 1


# Requests that join while others are mid-solve: a mix of sizes and
# precisions, admitted one by one as memory frees up (a budget that holds
# only two or three solves) or arriving over time on the wall clock.
JOIN_REQS = [Request(id=i, arrival=0.0, n=n, precision=p, seed=600 + i) for i, (n, p) in enumerate(
    [(40, "f64"), (24, "f32"), (32, "f64"), (20, "f32"), (36, "f32"), (16, "f64"), (28, "f64"), (44, "f32")])]


def joined_mid_solve(res):
    """Ids of requests admitted while another request was on the GPU."""
    return [r.id for r in res if any(o.id != r.id and o.admitted < r.admitted < o.finished for o in res)]


@pytest.mark.parametrize("how", ["budget", "staggered"])
def test_requests_joining_mid_solve_same_as_alone(how):
    """Continuous batching proper: requests admitted while others are
    mid-solve (as memory frees up, or as they arrive) give each the same
    iterate, sweep count, stop and residual as when served alone, and the
    iterate is the oracle's (plain Jacobi, or the refinement) stopped at the
    same check."""
    import dataclasses
    say("server joins mid-solve", how)
    max_iter = 3000
    if how == "budget":
        sizes = sorted(request_footprint(r.n, r.precision) for r in JOIN_REQS)
        budget = sizes[-1] + sizes[-2]
        reqs = JOIN_REQS
        srv = Server(budget_bytes=budget, window=50, rtol=1e-10, max_iter=max_iter, keep_fields=True)
        res = srv.run(reqs, realtime=False)
        assert srv.stats["peak_bytes"] <= budget
    else:
        reqs = [dataclasses.replace(r, arrival=0.02 * i) for i, r in enumerate(JOIN_REQS)]
        srv = Server(budget_bytes=1 << 34, window=50, rtol=1e-10, max_iter=max_iter, keep_fields=True)
        res = srv.run(reqs, realtime=True)
    assert not any(r.rejected for r in res)
    joined = joined_mid_solve(res)
    assert len(joined) >= 3, joined
    for r in reqs:
        _, alone = serve([r], max_iter=max_iter)
        a, m = alone[0], res[r.id]
        assert (a.iters, a.converged, a.rel_resid) == (m.iters, m.converged, m.rel_resid), r.id
        assert np.array_equal(a.field, m.field), r.id
        n = (r.n,) * 3
        u0 = synth.boundary_field(n, seed=r.seed)
        b = synth.source_field(n, seed=r.seed)
        if r.precision == "f64":
            ref, _ = oracle.c_jacobi(u0, m.iters, b)
        else:
            ref, _, done, st = oracle.c_ir_solve(u0, b, storage="f32", inner=50, rtol=1e-10, max_inner=max_iter)
            assert done == m.iters and (st == 0) == m.converged, r.id
        assert np.array_equal(m.field, ref), r.id


def test_group_check_is_the_stopping_rule():
    """jc_group_check: relative residual against the first norm it saw for
    the member's current solve (kept across groups, reset by a load), and
    the stop flag for the tolerance or the sweep cap."""
    from paper_2102_12416_amd import Group, Solver
    say("group check")
    specs = [(20, "f64"), (16, "f32"), (24, "f64")]
    solvers = []
    for i, (n, p) in enumerate(specs):
        s = Solver((n, n, n), mode="fused", with_source=True, ir_dtype="f32" if p == "f32" else None)
        s.load(synth.boundary_field((n, n, n), seed=80 + i), synth.source_field((n, n, n), seed=80 + i))
        solvers.append(s)
    with Group(solvers) as g:
        first = g.check(1e-10, 10 ** 6)
        assert all(rel == 1.0 and not done for rel, done in first)
        g.iterate(50)
        chk = g.check(1e-10, 10 ** 6)
        assert all(0.0 < rel < 1.0 and not done for rel, done in chk)
        # a tolerance above the relative residual stops; the cap stops
        assert all(done for _, done in g.check(2.0, 10 ** 6))
        assert all(done for _, done in g.check(1e-300, 50))
    # r0 is kept across groups: a new group sees the same relative residual
    with Group(solvers[:2]) as g2:
        again = g2.check(1e-10, 10 ** 6)
        for (r1, _), (r2, _) in zip(chk[:2], again):
            assert r1 == r2
    # a load starts a new solve: its first check is 1 again
    n0 = specs[0][0]
    solvers[0].load(synth.boundary_field((n0,) * 3, seed=80), synth.source_field((n0,) * 3, seed=80))
    with Group(solvers[:2]) as g3:
        assert g3.check(1e-10, 10 ** 6)[0] == (1.0, False)
    for s in solvers:
        s.close()


def test_resident_lane_same_results():
    """With resident=True the binary64 requests of edge <= 32 run in a lane
    of their own (each window one launch, one work-group per request): every
    result (sweeps, stop, residual, field) equals the run without it."""
    reqs = REQS + [Request(id=6, arrival=0.0, n=12, precision="f64", seed=507),
                   Request(id=7, arrival=0.0, n=31, precision="f64", seed=508),
                   Request(id=8, arrival=0.0, n=33, precision="f64", seed=509)]
    say("server resident lane")
    kw = dict(budget_bytes=1 << 34, window=50, rtol=1e-10, max_iter=1500, keep_fields=True)
    srv0 = Server(**kw)
    base = srv0.run(reqs, realtime=False)
    srv1 = Server(resident=True, **kw)
    res = srv1.run(reqs, realtime=False)
    assert len(srv1.stats["lane_windows"]) == len(srv0.stats["lane_windows"]) + 1
    assert srv1.stats["lane_windows"][-1] > 0
    for a, m in zip(base, res):
        assert a.iters == m.iters and a.converged == m.converged and a.rel_resid == m.rel_resid, a.id
        assert np.array_equal(a.field, m.field), a.id
