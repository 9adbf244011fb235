"""Tiles as wide as a block row (96, 128 and 256 cells) against the oracle.

A wide tile sweeps binary64 storage with the same sums in the same order
as any other tile shape, so iterates are bitwise the oracle's; residual
norms (reduction order) are compared at 1e-12 relative.  Block rows of
100 and 300 cells leave ragged tail tiles (4, 44 cells).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

from paper_2102_12416_amd import Group, JcError, Solver, _lib as L  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("tile", [(96, 4, 16), (96, 8, 7), (96, 16, 0), (128, 4, 33), (128, 8, 16),
                                  (128, 16, 0), (256, 4, 16), (256, 8, 0)])
@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_wide_tiles_vs_oracle(tile, mode):
    n, bd = (200, 70, 66), (100, 35, 66)
    say("wide tile", tile, mode, n, bd)
    u0 = synth.boundary_field(n, seed=31)
    b = synth.source_field(n, seed=31)
    ref, hist = oracle.c_jacobi(u0, 9, b, every=3)
    with Solver(n, block_dims=bd, mode=mode, with_source=True, use_graphs=False, tile_x=tile[0],
                tile_y=tile[1], z_chunk=tile[2]) as s:
        ti = s.tile_info()
        assert (ti["tile_x"], ti["tile_y"]) == tile[:2]
        s.load(u0, b)
        info = s.solve(rtol=0.0, max_iter=9, check_every=3, history=True)
        got = s.store().cpu().numpy()
    assert info["iters"] == 9
    assert np.array_equal(got, ref)
    np.testing.assert_allclose(info["history"], hist, rtol=1e-12, atol=0)


@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_wide_tile_single_ragged_block(mode):
    """One block of 300-cell rows in 256-cell tiles (a 44-cell tail tile),
    graph-captured windows."""
    n = (300, 21, 18)
    say("one block", n, "tile 256 x 8", mode)
    u0 = synth.boundary_field(n, seed=32)
    ref, _ = oracle.c_jacobi(u0, 11, None)
    with Solver(n, mode=mode, tile_x=256, tile_y=8, z_chunk=5) as s:
        s.load(u0)
        s.iterate(11)
        got = s.store().cpu().numpy()
    assert np.array_equal(got, ref)


def test_wide_tiles_binary64_refinement_vs_oracle():
    """Refinement with binary64 storage: its outer residual pass and inner
    sweeps run in 128-cell tiles; the iterate and stop equal the oracle's."""
    n, bd = (130, 20, 16), (65, 20, 16)
    say("f64 refinement, tile 128 x 8", n, bd)
    u0 = synth.boundary_field(n, seed=33)
    b = synth.source_field(n, seed=33)
    ref, hist, done, st = oracle.c_ir_solve(u0, b, storage="f64", inner=25, rtol=1e-8, max_inner=3000)
    with Solver(n, block_dims=bd, mode="fused", with_source=True, ir_dtype="f64", tile_x=128, tile_y=8) as s:
        s.load(u0, b)
        info = s.solve_ir(inner=25, rtol=1e-8, max_inner=3000, history=True)
        u = s.store().cpu().numpy()
    assert info["iters"] == done
    assert info["converged"] == (st == 0)
    rel = [h / info["history"][0] for h in info["history"]]
    np.testing.assert_allclose(rel, hist, rtol=1e-9, atol=1e-15)
    assert np.array_equal(u, ref)


def test_wide_group_tile():
    """A group of binary64 members in 96-cell tiles: each member's iterate
    equals the oracle's; a binary32-refining member refuses wide tiles."""
    specs = [((100, 30, 20), dict(with_source=True)),
             ((40, 36, 33), dict(with_source=False, block_dims=(20, 36, 33), mode="fused")),
             ((200, 12, 10), dict(with_source=True, block_dims=(100, 12, 10), mode="fused"))]
    say("group, tile 96 x 8 x 16")
    solvers, refs = [], []
    for i, (n, kw) in enumerate(specs):
        u0 = synth.boundary_field(n, seed=40 + i)
        b = synth.source_field(n, seed=40 + i) if kw.get("with_source") else None
        solvers.append(Solver(n, **kw).load(u0, b))
        refs.append(oracle.c_jacobi(u0, 60, b)[0])
    with Group(solvers, tile=(96, 8, 16)) as g:
        g.residuals()
        g.iterate(30)
        g.residuals()
        g.iterate(30)
    for s, ref in zip(solvers, refs):
        assert np.array_equal(s.store().cpu().numpy(), ref)
        s.close()
    n = (24, 24, 24)
    f32 = Solver(n, with_source=True, ir_dtype="f32").load(synth.boundary_field(n, seed=45),
                                                          synth.source_field(n, seed=45))
    with pytest.raises(JcError) as e:
        Group([f32], tile=(96, 8, 16))
    assert e.value.code == L.JC_ERR_INVALID
    f32.close()


@pytest.mark.parametrize("variant", ["overlap", "host", "metadata", "paced_fused", "paced_staged"])
def test_wide_tiles_other_paths(variant):
    """Wide tiles on the other iteration paths: boundary-first overlapped
    staged iterations (boundary tiles found with the wide tile width), host-
    staged and metadata exchanges, and paced launches (a pace that binds,
    then the tuned one): bitwise the oracle's."""
    n, bd = (200, 70, 66), (100, 35, 66)
    say("wide tile", variant)
    u0 = synth.boundary_field(n, seed=34)
    b = synth.source_field(n, seed=34)
    ref9, _ = oracle.c_jacobi(u0, 9, b)
    ref18, _ = oracle.c_jacobi(u0, 18, b)
    kw = dict(block_dims=bd, with_source=True, tile_x=128, tile_y=8, z_chunk=16)
    if variant == "overlap":
        kw.update(mode="staged", overlap=True)
    elif variant in ("host", "metadata"):
        kw.update(mode="staged", exchange=variant, use_graphs=False, tile_x=96)
    else:
        kw.update(mode=variant.split("_")[1])
    with Solver(n, **kw) as s:
        s.load(u0, b)
        if variant.startswith("paced"):
            s.set_pace(40)
        s.iterate(9)
        assert np.array_equal(s.store().cpu().numpy(), ref9)
        if variant.startswith("paced"):
            s.autotune_pace(reps=3)
            assert np.array_equal(s.store().cpu().numpy(), ref9)
        s.iterate(9)
        assert np.array_equal(s.store().cpu().numpy(), ref18)
