"""Resident sweeps (one work-group keeps a small block on chip for many
sweeps per launch) against the CPU oracle.

Each sweep forms every cell's update with the same sums in the same order
as a one-sweep launch, so the iterate is expected bitwise equal to the
oracle's after any number of sweeps: even and odd block extents (odd nx:
the last thread's second column is the x = nx + 1 ghost; odd nz: a sweep
ends with a one-plane step; nz mod 4: the two step schedules), even and
odd sweep counts, blocks of one to three planes (the source prefetch
wraps into the next sweep at once, or twice), the largest blocks the
kernel takes, and solves whose windows are single launches."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import Solver, _lib as L  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("n,iters,src", [
    ((32, 32, 32), 1, True),
    ((32, 32, 32), 2, False),
    ((32, 32, 32), 37, True),
    ((17, 23, 31), 13, True),      # odd nx, odd nz
    ((17, 23, 31), 8, False),
    ((24, 20, 16), 9, True),       # the 16-plane kernel
    ((9, 5, 15), 6, True),
    ((5, 3, 1), 7, True),          # one plane
    ((6, 4, 2), 5, True),          # two planes
    ((1, 1, 1), 4, True),
    ((2, 1, 3), 3, False),
    ((7, 6, 3), 10, True),
    ((8, 9, 4), 7, True),
    ((10, 3, 5), 8, False),
    ((12, 10, 22), 9, True),       # eleven two-plane steps per sweep
    ((13, 7, 9), 6, False),        # four two-plane steps and one single
    ((64, 8, 32), 11, True),       # 64-cell rows
    ((63, 8, 32), 10, True),
    ((64, 16, 24), 5, True),       # 512 threads, 64-cell rows, near the LDS limit
    ((3, 250, 5), 6, True),        # two pairs per row, 250 rows
])
@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_resident_vs_oracle(n, iters, src, mode):
    say("resident", mode, n, iters, "source" if src else "")
    u0 = synth.boundary_field(n, seed=21)
    b = synth.source_field(n, seed=21) if src else None
    ref, _ = oracle.c_jacobi(u0, iters, b)
    with Solver(n, mode=mode, with_source=src, resident=True) as s:
        s.load(u0, b)
        s.iterate(iters)
        got = s.store().cpu().numpy()
        assert s.iterations == iters
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))


def test_resident_windows_chain():
    """Windows of different lengths in a row (each one launch), then one-sweep
    residual passes in between: the iterate follows the oracle's."""
    n = (20, 18, 27)
    say("resident windows", n)
    u0 = synth.boundary_field(n, seed=22)
    b = synth.source_field(n, seed=22)
    with Solver(n, with_source=True, resident=True) as s:
        s.load(u0, b)
        s.set_timing(True)
        done = 0
        for k in (5, 1, 2, 40, 3):
            s.iterate(k)
            done += k
            ref, _ = oracle.c_jacobi(u0, done, b)
            assert np.array_equal(s.store().cpu().numpy(), ref), done
            np.testing.assert_allclose(s.residual(), oracle.c_residual_norm(ref, b), rtol=1e-12)
        assert s.kernel_time(L.JC_K_RESIDENT)[1] == 5
        assert s.kernel_time(L.JC_K_SWEEP)[1] == 0


@pytest.mark.parametrize("src", [False, True])
def test_resident_solve_matches_one_sweep_launches(src):
    """jc_solve on a resident context: the same checks, residual history, stop
    and iterate as with one sweep per launch, each window one launch."""
    n = (32, 32, 32)
    say("resident solve", "source" if src else "")
    u0 = synth.boundary_field(n, seed=23)
    b = synth.source_field(n, seed=23) if src else None
    out = []
    for resident in (False, True):
        with Solver(n, with_source=src, resident=resident) as s:
            s.load(u0, b)
            s.set_timing(resident)
            info = s.solve(rtol=1e-6, max_iter=5000, check_every=50, history=True)
            if resident:
                launches = s.kernel_time(L.JC_K_RESIDENT)[1]
            out.append((info, s.store().cpu().numpy()))
    (i0, u_0), (i1, u_1) = out
    assert i0["converged"] and i1["converged"]
    assert i0["iters"] == i1["iters"]
    assert i0["history"] == i1["history"]
    assert np.array_equal(u_0, u_1)
    # one launch per window of 49 sweeps between the checks
    assert launches == len(i1["history"]) - 1
    ref, _ = oracle.c_jacobi(u0, i1["iters"], b)
    assert np.array_equal(u_1, ref)


@pytest.mark.parametrize("graphs", [False, True])
def test_resident_group_vs_oracle(graphs):
    """A group of resident members of both kernel classes (with and without a
    source) and both plane-count parities, at different iteration counts
    when the group forms: each member's iterate equals the oracle's."""
    from paper_2102_12416_amd import Group
    specs = [((32, 32, 32), True, 0), ((17, 23, 31), True, 3), ((20, 18, 16), False, 1),
             ((9, 5, 15), False, 0), ((64, 8, 32), True, 2), ((6, 4, 2), True, 5), ((1, 1, 1), True, 1)]
    say("resident group", "graphs" if graphs else "eager")
    solvers, refs = [], []
    for i, (n, src, pre) in enumerate(specs):
        u0 = synth.boundary_field(n, seed=60 + i)
        b = synth.source_field(n, seed=60 + i) if src else None
        s = Solver(n, with_source=src, resident=True).load(u0, b)
        s.iterate(pre)
        solvers.append(s)
        refs.append(oracle.c_jacobi(u0, pre + 45, b)[0])
    with Group(solvers, use_graphs=graphs, resident=True) as g:
        g.iterate(20)
        res = g.residuals()
        g.iterate(24)
        g.iterate(1)
    for s, ref, r in zip(solvers, refs, res):
        assert np.array_equal(s.store().cpu().numpy(), ref)
        s.close()


def test_resident_group_rejects():
    from paper_2102_12416_amd import Group, JcError
    n = (40, 40, 8)        # (nx + 1) / 2 * ny = 800 pairs: too many for one work-group
    s = Solver(n).load(synth.boundary_field(n, seed=70))
    with pytest.raises(JcError) as e:
        Group([s], resident=True)
    assert e.value.code == L.JC_ERR_INVALID
    with pytest.raises(JcError) as e:
        Group([s], resident=True, temporal=True)
    assert e.value.code == L.JC_ERR_INVALID
    s.close()


def test_resident_random_shapes():
    """Seeded random blocks within the kernel's limits, random sweep counts
    and sources, both modes: bitwise the oracle's."""
    rng = np.random.default_rng(2102)
    done = 0
    while done < 24:
        n = (int(rng.integers(1, 65)), int(rng.integers(1, 41)), int(rng.integers(1, 33)))
        pw = 2 * ((n[0] + 1) // 2)
        if (n[0] + 1) // 2 * n[1] > 512 or 8 * (4 * n[1] * pw + 2 * n[2] * n[1] + 2 * n[2] * pw) > 65536:
            continue
        iters = int(rng.integers(1, 12))
        src = bool(rng.integers(0, 2))
        mode = ("staged", "fused")[done % 2]
        say("resident random", n, iters, "source" if src else "", mode)
        u0 = synth.boundary_field(n, seed=100 + done)
        b = synth.source_field(n, seed=100 + done) if src else None
        ref, _ = oracle.c_jacobi(u0, iters, b)
        with Solver(n, mode=mode, with_source=src, resident=True, use_graphs=False) as s:
            s.load(u0, b)
            s.iterate(iters)
            got = s.store().cpu().numpy()
        assert np.array_equal(got, ref), (n, iters, src, mode)
        done += 1
