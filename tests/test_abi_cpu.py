"""libjc host logic without a GPU: exports, validation, decomposition,
pairing geometry, footprint and state errors.  No device call is made."""
import ctypes
import os
import re

import pytest

from paper_2102_12416_amd import _lib as L
from paper_2102_12416_amd._lib import check

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(jc_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 20
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for every one of them
    assert names <= set(L.SIGNATURES), sorted(names - set(L.SIGNATURES))


def create(grid, bd, **kw):
    opt = L.Options()
    opt.mode = kw.get("mode", 0)
    opt.with_source = kw.get("with_source", 0)
    opt.ir_dtype = kw.get("ir_dtype", L.JC_NONE)
    opt.ir_enable = kw.get("ir_enable", 0)
    opt.tile_y = kw.get("tile_y", 0)
    opt.z_chunk = kw.get("z_chunk", 0)
    opt.tile_x = kw.get("tile_x", 0)
    opt.temporal = kw.get("temporal", 0)
    opt.overlap = kw.get("overlap", 0)
    opt.resident = kw.get("resident", 0)
    ctx = ctypes.c_void_p()
    st = L.lib.jc_create(L.i64(grid), L.i64(bd), ctypes.byref(opt), ctypes.byref(ctx))
    return st, ctx


def create_rect(grid, cuts):
    opt = L.Options()
    opt.ir_dtype = L.JC_NONE
    arrs = [L.i64(c) for c in cuts]
    ptrs = (ctypes.POINTER(ctypes.c_int64) * 3)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_int64)) for a in arrs])
    ctx = ctypes.c_void_p()
    st = L.lib.jc_create_rectilinear(L.i64(grid), ptrs, L.i64([len(c) for c in cuts]), ctypes.byref(opt),
                                     ctypes.byref(ctx))
    return st, ctx


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


@pytest.mark.parametrize("grid,bd,nb,npairs", [
    ((512, 512, 512), (256, 256, 256), 8, 24),     # 12 interfaces, both directions
    ((768, 768, 768), (96, 96, 96), 512, 2688),    # 3 * 7 * 64 interfaces
    ((64, 64, 64), (64, 64, 64), 1, 0),
    ((37, 29, 23), (16, 8, 10), 3 * 4 * 3, 2 * (2 * 4 * 3 + 3 * 3 * 3 + 3 * 4 * 2)),
])
def test_uniform_decomposition_and_pairing(grid, bd, nb, npairs):
    st, ctx = create(grid, bd)
    assert st == 0, L.last_error()
    try:
        blocks = blocks_of(ctx)
        pairs = pairs_of(ctx)
        assert len(blocks) == nb and len(pairs) == npairs
        # blocks tile the grid exactly
        assert sum(b[0] * b[1] * b[2] for b in blocks) == grid[0] * grid[1] * grid[2]
        for b in blocks:
            for a in range(3):
                assert 0 <= b[3 + a] and b[3 + a] + b[a] <= grid[a]
            # pitch: a multiple of 16 doubles with room for both x ghosts
            assert b[12] % 16 == 0 and b[12] >= b[0] + 2
            assert b[13] == b[12] * (b[1] + 2)
        # every directed pair has its reverse, with opposite faces and equal counts
        table = {(p[0], p[1]): p for p in pairs}
        for p in pairs:
            src, f, dst, g, count, slow, fast, off0, off1, ld = p
            assert ld % 2 == 0 and fast <= ld <= fast + 1
            assert off0 % 256 == 0 and off1 % 256 == 0 and off1 >= off0 + slow * ld * 8
            assert g == f ^ 1
            rev = table[(dst, g)]
            assert rev[2] == src and rev[3] == f and rev[4] == count
            assert slow * fast == count
            # neighbours touch: offsets differ by the source edge along the face normal
            a = f // 2
            bs, bd_ = blocks[src], blocks[dst]
            if f % 2 == 1:
                assert bs[3 + a] + bs[a] == bd_[3 + a]
            else:
                assert bd_[3 + a] + bd_[a] == bs[3 + a]
            assert blocks[src][6 + f] == dst
        # faces on the global boundary have no neighbour
        for i, b in enumerate(blocks):
            for f in range(6):
                a = f // 2
                on_boundary = (b[3 + a] == 0) if f % 2 == 0 else (b[3 + a] + b[a] == grid[a])
                assert (b[6 + f] == -1) == on_boundary
    finally:
        L.lib.jc_destroy(ctx)


def test_remainder_block_is_last():
    st, ctx = create((10, 7, 5), (4, 7, 2))
    assert st == 0
    xs = sorted({(b[3], b[0]) for b in blocks_of(ctx)})
    zs = sorted({(b[5], b[2]) for b in blocks_of(ctx)})
    assert xs == [(0, 4), (4, 4), (8, 2)]
    assert zs == [(0, 2), (2, 2), (4, 1)]
    L.lib.jc_destroy(ctx)


def test_rectilinear_uneven_cuts():
    import synth
    cuts = [synth.uneven_cuts(768, 32, 160, seed=12416, axis=a) for a in range(3)]
    st, ctx = create_rect((768, 768, 768), cuts)
    assert st == 0, L.last_error()
    nb = len(cuts[0]) * len(cuts[1]) * len(cuts[2])
    assert L.lib.jc_num_blocks(ctx) == nb
    blocks = blocks_of(ctx)
    assert sum(b[0] * b[1] * b[2] for b in blocks) == 768 ** 3
    L.lib.jc_destroy(ctx)


@pytest.mark.parametrize("grid,bd", [((0, 4, 4), (1, 1, 1)), ((8, 8, 8), (9, 8, 8)), ((8, 8, 8), (0, 8, 8)),
                                     ((8, -1, 8), (8, 8, 8))])
def test_invalid_geometry(grid, bd):
    st, ctx = create(grid, bd)
    assert st == L.JC_ERR_INVALID
    assert not ctx.value
    assert L.last_error()
    fp = ctypes.c_size_t()
    assert L.lib.jc_footprint(L.i64(grid), L.i64(bd), None, ctypes.byref(fp)) == L.JC_ERR_INVALID


def test_invalid_rectilinear_sum():
    st, ctx = create_rect((10, 10, 10), [[5, 4], [10], [10]])
    assert st == L.JC_ERR_INVALID and "sum" in L.last_error()


def test_invalid_options():
    st, _ = create((8, 8, 8), (8, 8, 8), tile_y=3)
    assert st == L.JC_ERR_INVALID
    st, _ = create((8, 8, 8), (8, 8, 8), mode=7)
    assert st == L.JC_ERR_INVALID


def test_footprint_covers_arrays_and_buffers():
    grid, bd = (512, 512, 512), (256, 256, 256)
    fp = ctypes.c_size_t()
    check(L.lib.jc_footprint(L.i64(grid), L.i64(bd), None, ctypes.byref(fp)))
    pitch = 272                                  # 256 + 2 rounded up to 16 doubles
    arrays = 8 * 2 * pitch * 258 * 258 * 8       # 8 blocks, ping-pong
    bufs = 24 * 2 * 256 * 256 * 8                # 24 pairs, send + receive
    assert arrays + bufs <= fp.value <= (arrays + bufs) * 1.05
    fps = ctypes.c_size_t()
    opt = L.Options()
    opt.with_source = 1
    opt.ir_dtype = L.JC_NONE
    check(L.lib.jc_footprint(L.i64(grid), L.i64(bd), ctypes.byref(opt), ctypes.byref(fps)))
    assert fps.value - fp.value >= 8 * pitch * 258 * 258 * 8


def test_min_surface_parts():
    out = (ctypes.c_int64 * 3)()
    check(L.lib.jc_min_surface_parts(L.i64((512, 512, 512)), 8, out))
    assert tuple(out) == (2, 2, 2)
    check(L.lib.jc_min_surface_parts(L.i64((768, 768, 768)), 512, out))
    assert tuple(out) == (8, 8, 8)
    # a long x axis is cut along x first
    check(L.lib.jc_min_surface_parts(L.i64((4096, 256, 256)), 4, out))
    assert tuple(out) == (4, 1, 1)
    # 1536^3 over 6 devices: any permutation of (1, 2, 3) has minimal area; ties prefer z cuts
    check(L.lib.jc_min_surface_parts(L.i64((1536, 1536, 1536)), 6, out))
    assert tuple(out) == (1, 2, 3)
    assert L.lib.jc_min_surface_parts(L.i64((2, 2, 2)), 27, out) == L.JC_ERR_INVALID


def test_unbound_context_state_errors():
    st, ctx = create((16, 16, 16), (8, 8, 8))
    assert st == 0
    for fn in (L.lib.jc_pack_faces, L.lib.jc_exchange, L.lib.jc_unpack_faces, L.lib.jc_sweep):
        assert fn(ctx) == L.JC_ERR_STATE
    assert L.lib.jc_iterate(ctx, 1) == L.JC_ERR_STATE
    r = ctypes.c_double()
    assert L.lib.jc_residual(ctx, ctypes.byref(r)) == L.JC_ERR_STATE
    assert "bound" in L.last_error()
    # arena checks happen before any device call
    assert L.lib.jc_bind(ctx, None, 0, None) == L.JC_ERR_INVALID
    assert L.lib.jc_bind(ctx, ctypes.c_void_p(4096), 1024, None) == L.JC_ERR_NOMEM
    assert L.lib.jc_bind(ctx, ctypes.c_void_p(4097), 1 << 40, None) == L.JC_ERR_INVALID
    L.lib.jc_destroy(ctx)


def test_destroy_null_is_noop():
    L.lib.jc_destroy(None)


def test_tile_info_and_items():
    st, ctx = create((512, 512, 512), (256, 256, 256), tile_y=4, z_chunk=64)
    assert st == 0
    out = (ctypes.c_int64 * 4)()
    check(L.lib.jc_tile_info(ctx, out))
    assert tuple(out) == (64, 4, 64, 8 * 4 * 64 * 4)
    assert L.lib.jc_num_items(ctx) == out[3]
    L.lib.jc_destroy(ctx)


def test_ir_options_validation_and_footprint():
    opt = L.Options()
    opt.ir_enable = 1
    opt.ir_dtype = 7
    ctx = ctypes.c_void_p()
    assert L.lib.jc_create(L.i64((8, 8, 8)), L.i64((8, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    sizes = {}
    for name, dt in (("none", None), ("f64", L.JC_F64), ("f32", L.JC_F32), ("bf16", L.JC_BF16)):
        o = L.Options()
        o.ir_dtype = L.JC_NONE
        if dt is not None:
            o.ir_enable = 1
            o.ir_dtype = dt
        fp = ctypes.c_size_t()
        check(L.lib.jc_footprint(L.i64((128, 128, 128)), L.i64((64, 64, 64)), ctypes.byref(o), ctypes.byref(fp)))
        sizes[name] = fp.value
    # three refinement arrays per block (d twice, r_lo) in the storage
    # format; rows are padded to whole 128-byte lines (64 bf16 values)
    cells = 8 * 66 * 66 * 66
    for name, es in (("f64", 8), ("f32", 4), ("bf16", 2)):
        extra = sizes[name] - sizes["none"]
        assert 3 * cells * es <= extra <= 3 * cells * es * 2.2, name
    assert sizes["f64"] > sizes["f32"] > sizes["bf16"] > sizes["none"]


def test_solve_ir_needs_refinement_buffers():
    st, ctx = create((16, 16, 16), (16, 16, 16))
    info = L.SolveInfo()
    assert L.lib.jc_solve_ir(ctx, 50, 1e-10, 100, ctypes.byref(info)) == L.JC_ERR_STATE
    L.lib.jc_destroy(ctx)


def test_set_tiles_validation_and_items():
    st, ctx = create((200, 100, 96), (100, 100, 96))
    assert st == 0
    assert L.lib.jc_set_tiles(ctx, 64, 5, 32) == L.JC_ERR_INVALID
    assert L.lib.jc_set_tiles(ctx, 64, 8, 0) == L.JC_ERR_INVALID
    assert L.lib.jc_set_tiles(ctx, 48, 8, 16) == L.JC_ERR_INVALID
    check(L.lib.jc_set_tiles(ctx, 64, 16, 48))
    out = (ctypes.c_int64 * 4)()
    check(L.lib.jc_tile_info(ctx, out))
    # 2 blocks x ceil(100/64) x ceil(100/16) x ceil(96/48)
    assert tuple(out) == (64, 16, 48, 2 * 2 * 7 * 2)
    check(L.lib.jc_set_tiles(ctx, 32, 4, 96))
    check(L.lib.jc_tile_info(ctx, out))
    assert tuple(out) == (32, 4, 96, 2 * 4 * 25 * 1)
    # 16-cell rows: whole waves need at least 8 rows
    assert L.lib.jc_set_tiles(ctx, 16, 4, 16) == L.JC_ERR_INVALID
    check(L.lib.jc_set_tiles(ctx, 16, 8, 16))
    check(L.lib.jc_tile_info(ctx, out))
    # the finest shapes the tuner may pick fit the work-list region
    assert tuple(out) == (16, 8, 16, 2 * 7 * 13 * 6)
    L.lib.jc_destroy(ctx)


def test_wide_tile_shapes():
    # 96-, 128- and 256-cell rows: at most 1024 threads per work-group
    st, ctx = create((200, 100, 96), (100, 100, 96))
    assert st == 0
    out = (ctypes.c_int64 * 4)()
    check(L.lib.jc_set_tiles(ctx, 96, 16, 48))
    check(L.lib.jc_tile_info(ctx, out))
    # 2 blocks x ceil(100/96) x ceil(100/16) x ceil(96/48): a 4-cell tail tile per row
    assert tuple(out) == (96, 16, 48, 2 * 2 * 7 * 2)
    check(L.lib.jc_set_tiles(ctx, 256, 8, 96))
    check(L.lib.jc_tile_info(ctx, out))
    assert tuple(out) == (256, 8, 96, 2 * 1 * 13 * 1)
    check(L.lib.jc_set_tiles(ctx, 128, 16, 32))
    check(L.lib.jc_set_tiles(ctx, 256, 4, 32))
    for shape in ((256, 16, 32), (96, 32, 16), (128, 32, 16), (192, 8, 16), (48, 8, 16)):
        assert L.lib.jc_set_tiles(ctx, *shape) == L.JC_ERR_INVALID, shape
    L.lib.jc_destroy(ctx)
    # as options: the pair is checked when both are given
    st, ctx = create((64, 64, 64), (64, 64, 64), tile_x=256, tile_y=16)
    assert st == L.JC_ERR_INVALID and "1024" in L.last_error()
    for tx in (96, 128, 256):
        st, ctx = create((64, 64, 64), (64, 64, 64), tile_x=tx)
        assert st == 0, tx
        check(L.lib.jc_tile_info(ctx, out))
        assert out[0] == tx and (tx // 2) * out[1] <= 1024
        L.lib.jc_destroy(ctx)


def test_wide_tiles_need_binary64_storage():
    # the refinement's binary32 / bfloat16 correction is swept in tiles of at most 64 cells
    for dt in (L.JC_F32, L.JC_BF16):
        st, _ = create((64, 64, 64), (64, 64, 64), tile_x=96, ir_enable=1, ir_dtype=dt)
        assert st == L.JC_ERR_INVALID and "binary64" in L.last_error()
        st, ctx = create((64, 64, 64), (64, 64, 64), ir_enable=1, ir_dtype=dt)
        assert st == 0
        assert L.lib.jc_set_tiles(ctx, 128, 8, 32) == L.JC_ERR_INVALID
        check(L.lib.jc_set_tiles(ctx, 64, 8, 32))
        L.lib.jc_destroy(ctx)
    st, ctx = create((64, 64, 64), (64, 64, 64), tile_x=128, ir_enable=1, ir_dtype=L.JC_F64)
    assert st == 0
    check(L.lib.jc_set_tiles(ctx, 256, 8, 32))
    L.lib.jc_destroy(ctx)


def resident_lds(nx, ny, nz):
    # four plane buffers of (nx + 1) // 2 pairs by ny rows, and the x and y ghost rings of every plane
    pw = 2 * ((nx + 1) // 2)
    return 8 * (4 * ny * pw + 2 * nz * ny + 2 * nz * pw)


@pytest.mark.parametrize("grid,ok", [((32, 32, 32), True), ((31, 32, 32), True), ((1, 1, 1), True),
                                     ((64, 8, 32), True), ((64, 16, 32), False), ((64, 16, 24), True),
                                     ((33, 32, 32), False), ((32, 32, 33), False), ((2, 512, 8), False),
                                     ((2, 512, 1), True), ((3, 250, 5), True), ((4, 300, 2), False)])
def test_resident_shape_limits(grid, ok):
    """One block of at most 32 planes, (nx + 1) / 2 * ny <= 512 cell pairs
    and an LDS need of at most 64 KiB."""
    nx, ny, nz = grid
    assert ok == (nz <= 32 and (nx + 1) // 2 * ny <= 512 and resident_lds(nx, ny, nz) <= 65536)
    st, ctx = create(grid, grid, resident=1, with_source=1)
    if ok:
        assert st == 0, L.last_error()
        L.lib.jc_destroy(ctx)
    else:
        assert st == L.JC_ERR_INVALID and "resident" in L.last_error()


def test_resident_option_conflicts():
    g = (16, 16, 16)
    st, _ = create(g, (8, 16, 16), resident=1)
    assert st == L.JC_ERR_INVALID and "one block" in L.last_error()
    for kw in (dict(ir_enable=1, ir_dtype=L.JC_F64), dict(temporal=1), dict(overlap=1)):
        st, _ = create(g, g, resident=1, **kw)
        assert st == L.JC_ERR_INVALID and "resident" in L.last_error()
    st, _ = create(g, g, resident=2)
    assert st == L.JC_ERR_INVALID
    st, ctx = create(g, g, resident=1, mode=L.JC_MODE_FUSED)
    assert st == 0
    L.lib.jc_destroy(ctx)


def test_pace_validation_and_reset_by_tiles():
    st, ctx = create((64, 64, 64), (32, 64, 64))
    assert st == 0
    assert L.lib.jc_get_pace(ctx) == 0
    assert L.lib.jc_set_pace(ctx, -1) == L.JC_ERR_INVALID
    assert L.lib.jc_set_pace(ctx, 10001) == L.JC_ERR_INVALID
    check(L.lib.jc_set_pace(ctx, 10000))
    check(L.lib.jc_set_pace(ctx, 148))
    assert L.lib.jc_get_pace(ctx) == 148
    # a pace belongs to a tile shape
    check(L.lib.jc_set_tiles(ctx, 64, 16, 32))
    assert L.lib.jc_get_pace(ctx) == 0
    out = (ctypes.c_int64 * 3)()
    assert L.lib.jc_autotune_pace(ctx, 3, out) == L.JC_ERR_STATE      # not bound
    assert L.lib.jc_autotune_pace(ctx, 0, out) < 0
    L.lib.jc_destroy(ctx)


def test_overlap_option_validation():
    opt = L.Options()
    opt.ir_dtype = L.JC_NONE
    opt.overlap = 1
    ctx = ctypes.c_void_p()
    opt.mode = L.JC_MODE_FUSED
    assert L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    opt.mode = L.JC_MODE_STAGED
    opt.exchange = L.JC_EXCHANGE_HOST
    assert L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    opt.exchange = L.JC_EXCHANGE_DEVICE
    opt.overlap = 2
    assert L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    opt.overlap = 1
    check(L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)))
    L.lib.jc_destroy(ctx)


def test_three_sweeps_per_launch_options():
    opt = L.Options()
    opt.ir_dtype = L.JC_NONE
    ctx = ctypes.c_void_p()
    opt.sweeps_per_launch = 3
    assert L.lib.jc_create(L.i64((40, 30, 20)), L.i64((40, 30, 20)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID                       # needs temporal
    opt.temporal = 1
    opt.sweeps_per_launch = 4
    assert L.lib.jc_create(L.i64((40, 30, 20)), L.i64((40, 30, 20)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    opt.sweeps_per_launch = 3
    check(L.lib.jc_create(L.i64((40, 30, 20)), L.i64((40, 30, 20)), ctypes.byref(opt), ctypes.byref(ctx)))
    out = (ctypes.c_int64 * 3)()
    check(L.lib.jc_temporal_info(ctx, out))
    assert out[0] == 3 and out[1] == 16
    assert L.lib.jc_set_temporal_tiles(ctx, 24, 8) == L.JC_ERR_INVALID   # 8 or 16 rows for three
    check(L.lib.jc_set_temporal_tiles(ctx, 8, 5))
    check(L.lib.jc_temporal_info(ctx, out))
    assert tuple(out) == (3, 8, 5)
    L.lib.jc_destroy(ctx)
    opt.sweeps_per_launch = 0
    check(L.lib.jc_create(L.i64((40, 30, 20)), L.i64((40, 30, 20)), ctypes.byref(opt), ctypes.byref(ctx)))
    check(L.lib.jc_temporal_info(ctx, out))
    assert out[0] == 2
    check(L.lib.jc_set_temporal_tiles(ctx, 24, 8))
    L.lib.jc_destroy(ctx)


def test_sixteen_cell_tile_options():
    st, ctx = create((40, 24, 24), (40, 24, 24), tile_x=16, tile_y=4)
    assert st == L.JC_ERR_INVALID
    st, ctx = create((40, 24, 24), (40, 24, 24), tile_x=16)
    assert st == 0
    out = (ctypes.c_int64 * 4)()
    check(L.lib.jc_tile_info(ctx, out))
    assert out[0] == 16 and out[1] >= 8
    L.lib.jc_destroy(ctx)


def test_temporal_option_needs_one_block():
    st, ctx = create((40, 24, 24), (40, 24, 24), temporal=1)
    assert st == 0
    L.lib.jc_destroy(ctx)
    st, _ = create((40, 24, 24), (20, 24, 24), temporal=1)
    assert st == L.JC_ERR_INVALID and "one block" in L.last_error()
    st, _ = create((8, 8, 8), (8, 8, 8), temporal=2)
    assert st == L.JC_ERR_INVALID and "temporal" in L.last_error()


def test_temporal_tile_shape():
    out = (ctypes.c_int64 * 3)()
    st, ctx = create((40, 24, 100), (40, 24, 100), temporal=1, z_chunk=16)
    assert st == 0
    check(L.lib.jc_temporal_info(ctx, out))
    assert tuple(out) == (2, 16, 8)               # 2 tiles per plane: chunks halved to 8 planes
    st2, big = create((1024, 1024, 1024), (1024, 1024, 1024), temporal=1, z_chunk=512)
    assert st2 == 0
    check(L.lib.jc_temporal_info(big, out))
    assert tuple(out) == (2, 16, 512)             # 1024 tiles per plane x 2 chunks: kept
    L.lib.jc_destroy(big)
    check(L.lib.jc_set_temporal_tiles(ctx, 24, 7))
    check(L.lib.jc_temporal_info(ctx, out))
    assert tuple(out) == (2, 24, 7)
    assert L.lib.jc_set_temporal_tiles(ctx, 12, 7) == L.JC_ERR_INVALID
    check(L.lib.jc_set_temporal_tiles(ctx, 8, 7))
    assert L.lib.jc_set_temporal_tiles(ctx, 16, 0) == L.JC_ERR_INVALID
    L.lib.jc_destroy(ctx)
    st, ctx = create((40, 24, 100), (40, 24, 100))
    assert L.lib.jc_set_temporal_tiles(ctx, 16, 32) == L.JC_ERR_STATE
    check(L.lib.jc_temporal_info(ctx, out))
    assert out[0] == 0
    L.lib.jc_destroy(ctx)


def test_default_tile_width_prefers_fewer_idle_lanes():
    out = (ctypes.c_int64 * 4)()
    for grid, bd, want in (((768, 768, 768), (96, 96, 96), 32), ((512, 512, 512), (256, 256, 256), 64),
                           ((100, 64, 64), (100, 64, 64), 64)):
        st, ctx = create(grid, bd)
        assert st == 0
        check(L.lib.jc_tile_info(ctx, out))
        assert out[0] == want, (grid, bd, out[0])
        L.lib.jc_destroy(ctx)


def test_exchange_mode_validation():
    opt = L.Options()
    opt.ir_dtype = L.JC_NONE
    opt.exchange = 9
    ctx = ctypes.c_void_p()
    assert L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    opt.exchange = L.JC_EXCHANGE_HOST
    opt.mode = L.JC_MODE_FUSED
    assert L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)) == \
        L.JC_ERR_INVALID
    opt.mode = L.JC_MODE_STAGED
    check(L.lib.jc_create(L.i64((8, 8, 8)), L.i64((4, 8, 8)), ctypes.byref(opt), ctypes.byref(ctx)))
    L.lib.jc_destroy(ctx)


def test_server_lane_bounds_validated():
    from paper_2102_12416_amd.server import Server
    with pytest.raises(ValueError):
        Server(budget_bytes=1 << 30, lanes=(160, 64), device="cpu")
    with pytest.raises(ValueError):
        Server(budget_bytes=1 << 30, lanes=(0,), device="cpu")
    with pytest.raises(ValueError):
        Server(budget_bytes=1 << 30, window=30, max_iter=100, device="cpu")
