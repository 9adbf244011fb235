"""Property tests of the host logic behind the C-ABI (no GPU): random
rectilinear decompositions and tile shapes.

For any cuts of any grid the blocks tile the grid exactly as the tensor
product of the cuts, every paired face has its reverse with the opposite
face and the face's area as count, global-boundary faces have no
neighbour, and the work list of any valid tile shape (16- to 256-cell
rows) holds exactly the tiles that cover every block once.  Resident
sweeps are accepted for exactly the blocks within the kernel's limits.
"""
import ctypes
import itertools

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as hs

from paper_2102_12416_amd import _lib as L

WIDTHS = (16, 32, 64, 96, 128, 256)
ROWS = (4, 8, 16, 32)


def check(st):
    assert st == 0, L.last_error()


@hs.composite
def cut_lists(draw):
    cuts = []
    for _ in range(3):
        pieces = draw(hs.lists(hs.integers(1, 40), min_size=1, max_size=5))
        cuts.append(pieces)
    return cuts


def create_rect(cuts):
    grid = [sum(c) for c in cuts]
    opt = L.Options()
    opt.ir_dtype = L.JC_NONE
    arrs = [L.i64(c) for c in cuts]
    ptrs = (ctypes.POINTER(ctypes.c_int64) * 3)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_int64)) for a in arrs])
    ctx = ctypes.c_void_p()
    st = L.lib.jc_create_rectilinear(L.i64(grid), ptrs, L.i64([len(c) for c in cuts]), ctypes.byref(opt),
                                     ctypes.byref(ctx))
    return st, ctx, grid


def blocks_of(ctx):
    out = []
    for i in range(L.lib.jc_num_blocks(ctx)):
        v = (ctypes.c_int64 * 17)()
        check(L.lib.jc_block_info(ctx, i, v))
        out.append(list(v))
    return out


def pairs_of(ctx):
    out = []
    for i in range(L.lib.jc_num_pairs(ctx)):
        v = (ctypes.c_int64 * 10)()
        check(L.lib.jc_pair_info(ctx, i, v))
        out.append(list(v))
    return out


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cuts=cut_lists())
def test_rectilinear_blocks_and_pairs(cuts):
    st, ctx, grid = create_rect(cuts)
    assert st == 0, L.last_error()
    try:
        blocks = blocks_of(ctx)
        # the tensor product of the cuts, each piece once
        starts = [list(itertools.accumulate([0] + c[:-1])) for c in cuts]
        want = sorted(((starts[0][i], starts[1][j], starts[2][k]), (cuts[0][i], cuts[1][j], cuts[2][k]))
                      for i in range(len(cuts[0])) for j in range(len(cuts[1])) for k in range(len(cuts[2])))
        got = sorted(((b[3], b[4], b[5]), (b[0], b[1], b[2])) for b in blocks)
        assert got == want
        # pairs: one per direction of every interface between neighbouring blocks
        interfaces = sum((len(cuts[a]) - 1) * len(cuts[(a + 1) % 3]) * len(cuts[(a + 2) % 3]) for a in range(3))
        pairs = pairs_of(ctx)
        assert len(pairs) == 2 * interfaces
        table = {(p[0], p[1]): p for p in pairs}
        assert len(table) == len(pairs)
        for src, f, dst, g, count, slow, fast, off0, off1, ld in pairs:
            a = f // 2
            bs, bt = blocks[src], blocks[dst]
            assert g == f ^ 1 and table[(dst, g)][2] == src and table[(dst, g)][4] == count
            # the shared plane's area: the face of the source block
            other = [x for x in range(3) if x != a]
            assert count == bs[other[0]] * bs[other[1]] == slow * fast
            assert bs[6 + f] == dst and bt[6 + g] == src
            # the blocks touch along the face normal and coincide across it
            if f % 2 == 1:
                assert bs[3 + a] + bs[a] == bt[3 + a]
            else:
                assert bt[3 + a] + bt[a] == bs[3 + a]
            for o in other:
                assert bs[3 + o] == bt[3 + o] and bs[o] == bt[o]
        for b in blocks:
            for f in range(6):
                a = f // 2
                on_boundary = (b[3 + a] == 0) if f % 2 == 0 else (b[3 + a] + b[a] == grid[a])
                assert (b[6 + f] == -1) == on_boundary
    finally:
        L.lib.jc_destroy(ctx)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cuts=cut_lists(), tx=hs.sampled_from(WIDTHS), ty=hs.sampled_from(ROWS), zc=hs.integers(1, 48))
def test_work_list_covers_every_block_once(cuts, tx, ty, zc):
    st, ctx, grid = create_rect(cuts)
    assert st == 0, L.last_error()
    try:
        threads = (tx // 2) * ty
        st = L.lib.jc_set_tiles(ctx, tx, ty, zc)
        if threads < 64 or threads > 1024:
            assert st == L.JC_ERR_INVALID
            return
        want = sum(-(-b[0] // tx) * -(-b[1] // ty) * -(-b[2] // zc) for b in blocks_of(ctx))
        if st == L.JC_ERR_INVALID:
            # only a work list larger than the region sized at creation is refused
            assert "z_chunk" in L.last_error()
            return
        assert st == 0
        out = (ctypes.c_int64 * 4)()
        check(L.lib.jc_tile_info(ctx, out))
        assert tuple(out) == (tx, ty, zc, want)
    finally:
        L.lib.jc_destroy(ctx)


@settings(max_examples=200, deadline=None)
@given(nx=hs.integers(1, 80), ny=hs.integers(1, 600), nz=hs.integers(1, 40), src=hs.booleans())
def test_resident_limits_property(nx, ny, nz, src):
    """A one-block context takes options.resident exactly when the block has
    at most 32 planes, at most 512 cell pairs per plane and an LDS need
    (four plane buffers of (nx + 1) // 2 pairs by ny rows, and the x and y
    ghost rings of every plane) of at most 64 KiB."""
    pw = 2 * ((nx + 1) // 2)
    ok = nz <= 32 and (nx + 1) // 2 * ny <= 512 and 8 * (4 * ny * pw + 2 * nz * ny + 2 * nz * pw) <= 65536
    opt = L.Options()
    opt.ir_dtype = L.JC_NONE
    opt.with_source = int(src)
    opt.resident = 1
    ctx = ctypes.c_void_p()
    g = L.i64((nx, ny, nz))
    st = L.lib.jc_create(g, g, ctypes.byref(opt), ctypes.byref(ctx))
    if ok:
        assert st == 0, L.last_error()
        L.lib.jc_destroy(ctx)
    else:
        assert st == L.JC_ERR_INVALID and "resident" in L.last_error()
