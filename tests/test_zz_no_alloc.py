"""The allocation-free group binding, jc_group_bind_static, against the
ordinary binding, jc_group_bind with caller scratch.

Both run the same kernels over the same tables, so every member's iterate
and every residual norm must be bitwise the same.  Two static bindings in a
row (the second group smaller than the first) check that a group does not
depend on what the previous one left in the static array.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import JcError, Solver, _lib as L  # noqa: E402
from paper_2102_12416_amd.solver import Group  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


# (interior, block_dims or None, refinement storage or None)
LARGER = [((48, 48, 48), None, None), ((40, 36, 30), (20, 18, 30), None), ((36, 36, 36), None, "f32"),
          ((30, 30, 30), None, "bf16")]
SMALLER = [((24, 24, 24), None, None), ((20, 20, 20), None, "f32")]


def run_group(specs, static, seed, windows=3, sweeps=25):
    stream = torch.cuda.Stream()
    solvers = []
    for i, (n, bd, ir) in enumerate(specs):
        s = Solver(n, block_dims=bd, mode="fused", with_source=True, ir_dtype=ir, use_graphs=False, stream=stream)
        s.load(synth.boundary_field(n, seed=seed + i), synth.source_field(n, seed=seed + i))
        solvers.append(s)
    norms = []
    with Group(solvers, use_graphs=False, stream=stream, static_scratch=static) as g:
        assert (g.scratch is None) == static
        for _ in range(windows):
            norms.append(g.residuals())
            g.iterate(sweeps)
        norms.append(g.residuals())
    fields = [s.store().cpu().numpy() for s in solvers]
    iters = [s.iterations for s in solvers]
    for s in solvers:
        s.close()
    return fields, norms, iters


def test_static_binding_matches_caller_scratch_two_calls():
    for call, (specs, seed) in enumerate([(LARGER, 900), (SMALLER, 950)]):
        say("static group binding, call", call + 1, [s[0] for s in specs])
        f_ref, n_ref, it_ref = run_group(specs, static=False, seed=seed)
        f_st, n_st, it_st = run_group(specs, static=True, seed=seed)
        assert it_st == it_ref
        assert n_st == n_ref
        for a, b in zip(f_st, f_ref):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_static_binding_rejects_oversize_and_a_second_holder():
    say("static group binding: limits")
    stream = torch.cuda.Stream()
    n = (24, 24, 24)
    a = Solver(n, mode="fused", with_source=True, use_graphs=False, stream=stream)
    b = Solver(n, mode="fused", with_source=True, use_graphs=False, stream=stream)
    for s in (a, b):
        s.load(synth.boundary_field(n, seed=1), synth.source_field(n, seed=1))
    with Group([a], use_graphs=False, stream=stream, static_scratch=True):
        with pytest.raises(JcError) as e:
            Group([b], use_graphs=False, stream=stream, static_scratch=True)
        assert e.value.code == L.JC_ERR_STATE
    # released by the first group's destruction
    with Group([b], use_graphs=False, stream=stream, static_scratch=True) as g:
        g.iterate(3)
    # a group whose tables exceed the static array: one 384^3 member in
    # 16 x 8 x 1 tiles (442,368 work items)
    big = Solver((384, 384, 384), mode="fused", with_source=True, use_graphs=False, stream=stream)
    big.load(synth.boundary_field((384, 384, 384), seed=2), synth.source_field((384, 384, 384), seed=2))
    with pytest.raises(JcError) as e:
        Group([big], use_graphs=False, stream=stream, tile=(16, 8, 1), static_scratch=True)
    assert e.value.code == L.JC_ERR_NOMEM
    with Group([big], use_graphs=False, stream=stream, tile=(16, 8, 1)) as g:
        assert g.footprint > L.JC_STATIC_SCRATCH_BYTES
    for s in (a, b, big):
        s.close()
