// Host runtime of libjc: decomposition, face pairing, work lists, arena
// layout, the state machine of the staged exchange, graph-captured
// iteration windows and the solve loops.  Implements include/jc.h.
//
// Paper section 4.3 (Jacobi3D): the domain is split into equal cuboid
// blocks with minimal surface area; each iteration exchanges block halos
// with up to six neighbours and then applies the stencil; a fixed number
// of iterations is run.  The pairing table built here is created once per
// context, like the channels of section 3.2.2: afterwards every transfer
// knows its source and destination buffers without any host message.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "jc_ctx.h"

using namespace jc_rt;

namespace jc_rt {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

}  // namespace jc_rt

namespace {

// ------------------------------------------------------------------ geometry

int64_t items_for(const jc_ctx* c, int tx, int ty, int zc)
{
    int64_t total = 0;
    for (const HostBlock& b : c->blocks) {
        const int64_t nxt = (b.n[0] + tx - 1) / tx;
        const int64_t tyn = (b.n[1] + ty - 1) / ty;
        const int64_t tz = (b.n[2] + zc - 1) / zc;
        total += nxt * tyn * tz;
    }
    return total;
}

// Lanes a tile width leaves idle: x tiles past the end of each block row.
int64_t idle_cells(const jc_ctx* c, int tx)
{
    int64_t idle = 0;
    for (const HostBlock& b : c->blocks)
        idle += ((b.n[0] + tx - 1) / tx * tx - b.n[0]) * b.n[1] * b.n[2];
    return idle;
}

// Default tile: 64 cells wide unless 32 leaves fewer idle lanes by more
// than 1/16 of the cells; 8 rows; z chunks halved from the full depth
// until the launch has at least 4096 tiles (16 per compute unit) or
// chunks reach 16.
void default_tiles(const jc_ctx* c, int* tx, int* ty, int* zc)
{
    int64_t maxz = 1, cells = 0;
    for (const HostBlock& b : c->blocks) {
        maxz = std::max(maxz, b.n[2]);
        cells += b.n[0] * b.n[1] * b.n[2];
    }
    int x = c->opt.tile_x > 0 ? c->opt.tile_x : 64;
    if (c->opt.tile_x <= 0 && (idle_cells(c, 64) - idle_cells(c, 32)) * 16 > cells)
        x = 32;
    int t = c->opt.tile_y > 0 ? c->opt.tile_y : 8;
    int z = c->opt.z_chunk > 0 ? c->opt.z_chunk : (int)std::min<int64_t>(maxz, 1 << 20);
    if (c->opt.z_chunk <= 0) {
        while (z > kMinZChunk && items_for(c, x, t, z) < 4096)
            z = (z + 1) / 2;
    }
    *tx = x;
    *ty = t;
    *zc = z;
}

void build_items(jc_ctx* c)
{
    c->items.clear();
    for (int bi = 0; bi < c->nb(); ++bi) {
        const HostBlock& b = c->blocks[bi];
        const int64_t nch = (b.n[2] + c->z_chunk - 1) / c->z_chunk;
        for (int64_t k = 0; k < nch; ++k)
            for (int64_t y0 = 0; y0 < b.n[1]; y0 += c->tile_y)
                for (int64_t x0 = 0; x0 < b.n[0]; x0 += c->tile_x) {
                    int64_t z0 = 0, zlen = 0;
                    z_chunk_range(b.n[2], c->z_chunk, k, &z0, &zlen);
                    Item it{};
                    it.block = bi;
                    it.x0 = (int32_t)x0;
                    it.y0 = (int32_t)y0;
                    it.z0 = (int32_t)z0;
                    it.zlen = (int32_t)zlen;
                    it.flip = 0;
                    it.owner = 0;
                    c->items.push_back(it);
                }
    }
    // boundary-first iterations: the tiles holding a cell of a paired face
    // plane go first (their sweep writes every face value of the new
    // iterate), the interior tiles after them
    c->n_bnd = 0;
    if (c->opt.overlap && c->np()) {
        auto boundary = [c](const Item& it) {
            const HostBlock& b = c->blocks[it.block];
            return (b.nbr[jc::XM] >= 0 && it.x0 == 0) || (b.nbr[jc::XP] >= 0 && it.x0 + c->tile_x >= b.n[0]) ||
                   (b.nbr[jc::YM] >= 0 && it.y0 == 0) || (b.nbr[jc::YP] >= 0 && it.y0 + c->tile_y >= b.n[1]) ||
                   (b.nbr[jc::ZM] >= 0 && it.z0 == 0) || (b.nbr[jc::ZP] >= 0 && it.z0 + it.zlen >= b.n[2]);
        };
        const auto mid = std::stable_partition(c->items.begin(), c->items.end(), boundary);
        c->n_bnd = mid - c->items.begin();
    }
}

int validate_options(const jc_options* opt)
{
    if (!opt)
        return JC_OK;
    if (opt->mode != JC_MODE_STAGED && opt->mode != JC_MODE_FUSED)
        return fail(JC_ERR_INVALID, "options.mode must be JC_MODE_STAGED or JC_MODE_FUSED");
    if (opt->exchange != JC_EXCHANGE_DEVICE && opt->exchange != JC_EXCHANGE_HOST &&
        opt->exchange != JC_EXCHANGE_METADATA)
        return fail(JC_ERR_INVALID, "options.exchange must be JC_EXCHANGE_DEVICE, _HOST or _METADATA");
    if (opt->exchange != JC_EXCHANGE_DEVICE && opt->mode == JC_MODE_FUSED)
        return fail(JC_ERR_INVALID, "host-staged or metadata exchange needs the staged mode");
    if (opt->debug_epochs != 0)
        return fail(JC_ERR_INVALID, "options.debug_epochs is reserved and must be 0");
    if (opt->tile_x != 0 && !tile_shape_ok(opt->tile_x, 8))
        return fail(JC_ERR_INVALID, "options.tile_x must be 0, 16, 32, 64, 96, 128 or 256");
    if (opt->tile_y != 0 && !tile_shape_ok(64, opt->tile_y))
        return fail(JC_ERR_INVALID, "options.tile_y must be 0, 4, 8, 16 or 32");
    if (opt->tile_x != 0 && opt->tile_y != 0 && !tile_shape_ok(opt->tile_x, opt->tile_y))
        return fail(JC_ERR_INVALID, "options.tile_x / 2 x options.tile_y must be 64 to 1024 threads (a 16-cell "
                                    "tile needs 8 rows or more, a 256-cell tile 8 or fewer)");
    if (opt->tile_x > kNarrowTileMax && opt->ir_enable && opt->ir_dtype != JC_F64)
        return fail(JC_ERR_INVALID, "tiles wider than 64 cells need binary64 storage (options.ir_dtype JC_F64)");
    if (opt->z_chunk < 0)
        return fail(JC_ERR_INVALID, "options.z_chunk must be >= 0");
    if (opt->temporal != 0 && opt->temporal != 1)
        return fail(JC_ERR_INVALID, "options.temporal must be 0 or 1");
    if (opt->overlap != 0 && opt->overlap != 1)
        return fail(JC_ERR_INVALID, "options.overlap must be 0 or 1");
    if (opt->sweeps_per_launch != 0 && opt->sweeps_per_launch != 2 && opt->sweeps_per_launch != 3)
        return fail(JC_ERR_INVALID, "options.sweeps_per_launch must be 0, 2 or 3");
    if (opt->sweeps_per_launch == 3 && !opt->temporal)
        return fail(JC_ERR_INVALID, "options.sweeps_per_launch = 3 needs options.temporal = 1");
    if (opt->overlap && (opt->mode != JC_MODE_STAGED || opt->exchange != JC_EXCHANGE_DEVICE))
        return fail(JC_ERR_INVALID, "options.overlap needs the staged mode with the device exchange");
    if (opt->ir_enable && opt->ir_dtype != JC_F64 && opt->ir_dtype != JC_F32 && opt->ir_dtype != JC_BF16)
        return fail(JC_ERR_INVALID, "options.ir_dtype must be JC_F64, JC_F32 or JC_BF16 when ir_enable is set");
    if (opt->resident != 0 && opt->resident != 1)
        return fail(JC_ERR_INVALID, "options.resident must be 0 or 1");
    if (opt->resident && (opt->ir_enable || opt->temporal || opt->overlap))
        return fail(JC_ERR_INVALID, "options.resident excludes refinement, temporal blocking and overlap");
    return JC_OK;
}

int build_geometry(jc_ctx* c, const int64_t grid[3], const std::vector<int64_t> cuts[3],
                   const jc_options* opt)
{
    int st = validate_options(opt);
    if (st != JC_OK)
        return st;
    if (opt)
        c->opt = *opt;
    for (int a = 0; a < 3; ++a) {
        if (grid[a] < 1 || grid[a] > kMaxEdge)
            return fail(JC_ERR_INVALID, "grid sizes must be in [1, 2^30]");
        int64_t sum = 0;
        for (int64_t v : cuts[a]) {
            if (v < 1)
                return fail(JC_ERR_INVALID, "block edges must be >= 1");
            sum += v;
        }
        if (cuts[a].empty() || sum != grid[a])
            return fail(JC_ERR_INVALID, "block edges along an axis must sum to the grid size");
        c->grid[a] = grid[a];
        c->cuts[a] = cuts[a];
    }
    const int64_t px = (int64_t)cuts[0].size(), py = (int64_t)cuts[1].size(), pz = (int64_t)cuts[2].size();
    if (px * py * pz > (1 << 24))
        return fail(JC_ERR_INVALID, "too many blocks");
    std::vector<int64_t> start[3];
    for (int a = 0; a < 3; ++a) {
        int64_t s = 0;
        for (int64_t v : cuts[a]) {
            start[a].push_back(s);
            s += v;
        }
    }
    auto bidx = [&](int64_t i, int64_t j, int64_t k) { return (int)((k * py + j) * px + i); };
    c->blocks.clear();
    c->pairs.clear();
    for (int64_t k = 0; k < pz; ++k)
        for (int64_t j = 0; j < py; ++j)
            for (int64_t i = 0; i < px; ++i) {
                HostBlock b{};
                b.n[0] = cuts[0][i]; b.n[1] = cuts[1][j]; b.n[2] = cuts[2][k];
                b.off[0] = start[0][i]; b.off[1] = start[1][j]; b.off[2] = start[2][k];
                b.nbr[jc::XM] = i > 0 ? bidx(i - 1, j, k) : -1;
                b.nbr[jc::XP] = i + 1 < px ? bidx(i + 1, j, k) : -1;
                b.nbr[jc::YM] = j > 0 ? bidx(i, j - 1, k) : -1;
                b.nbr[jc::YP] = j + 1 < py ? bidx(i, j + 1, k) : -1;
                b.nbr[jc::ZM] = k > 0 ? bidx(i, j, k - 1) : -1;
                b.nbr[jc::ZP] = k + 1 < pz ? bidx(i, j, k + 1) : -1;
                for (int f = 0; f < 6; ++f)
                    b.pair_out[f] = b.pair_in[f] = -1;
                b.pitch = round_up(b.n[0] + 2, jc::line_elems<double>());
                b.plane = b.pitch * (b.n[1] + 2);
                c->blocks.push_back(b);
            }
    // pairing table: one directed pair per touching face, in block order
    for (int bi = 0; bi < c->nb(); ++bi) {
        HostBlock& b = c->blocks[bi];
        for (int f = 0; f < 6; ++f) {
            if (b.nbr[f] < 0)
                continue;
            HostPair p{};
            p.src_block = bi;
            p.src_face = f;
            p.dst_block = b.nbr[f];
            p.dst_face = jc::opposite(f);
            if (f == jc::XM || f == jc::XP) { p.slow = b.n[2]; p.fast = b.n[1]; }
            else if (f == jc::YM || f == jc::YP) { p.slow = b.n[2]; p.fast = b.n[0]; }
            else { p.slow = b.n[1]; p.fast = b.n[0]; }
            p.count = p.slow * p.fast;
            p.span = p.slow * jc::face_ld(p.fast);
            b.pair_out[f] = (int)c->pairs.size();
            c->pairs.push_back(p);
        }
    }
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& p = c->pairs[q];
        c->blocks[p.dst_block].pair_in[p.dst_face] = q;
        c->max_slow = std::max(c->max_slow, p.slow);
        c->max_fast = std::max(c->max_fast, p.fast);
        c->max_count = std::max(c->max_count, p.span);
    }
    if (c->max_slow > 65535)
        return fail(JC_ERR_INVALID, "a shared block face is longer than 65535 along its slow axis");
    if (c->np() > 65535)
        return fail(JC_ERR_INVALID, "too many face pairs for one launch");
    if (c->nb() > 65535)
        return fail(JC_ERR_INVALID, "too many blocks for one launch");
    if (c->opt.temporal && c->nb() != 1)
        return fail(JC_ERR_INVALID, "options.temporal needs a context of one block (no face pairs)");
    if (c->opt.resident && (c->nb() != 1 || !jc::resident_fits(c->blocks[0].n[0], c->blocks[0].n[1], c->blocks[0].n[2])))
        return fail(JC_ERR_INVALID, "options.resident needs a context of one block of at most 32 planes with "
                                    "(nx + 1) / 2 * ny <= 512 cell pairs and an LDS need within 64 KiB");
    default_tiles(c, &c->tile_x, &c->tile_y, &c->z_chunk);
    build_items(c);
    // the work-list region is sized for the finest tiling the tuner may pick
    c->max_items = std::max<int64_t>({(int64_t)c->items.size(), items_for(c, 32, 4, kMinZChunk),
                                      items_for(c, 16, 8, kMinZChunk)});
    if (c->max_items > (int64_t)1 << 30)
        return fail(JC_ERR_INVALID, "work list too long");
    // arena layout
    size_t off = 0;
    c->off_blocks = off; off = align_up(off + sizeof(BlockDesc) * c->blocks.size(), kAlign);
    c->off_pairs = off; off = align_up(off + sizeof(PairDesc) * std::max<size_t>(1, c->pairs.size()), kAlign);
    c->off_items = off; off = align_up(off + sizeof(Item) * (size_t)c->max_items, kAlign);
    c->off_partials = off; off = align_up(off + sizeof(double) * (size_t)c->max_items, kAlign);
    c->off_ranges = off; off = align_up(off + sizeof(int32_t) * 2, kAlign);
    c->off_result = off; off = align_up(off + sizeof(double) * 4, kAlign);
    for (HostBlock& b : c->blocks) {
        // element (0,0,0) sits 15 elements into a 128-byte line so that
        // cell x = 1 of every row starts a line; 16 elements of slack
        const size_t bytes = align_up(sizeof(double) * (size_t)(b.plane * (b.n[2] + 2) + 16), kAlign);
        b.u_off[0] = off; off += bytes;
        b.u_off[1] = off; off += bytes;
        if (c->opt.with_source) { b.b_off = off; off += bytes; }
    }
    for (HostPair& p : c->pairs) {
        const size_t bytes = align_up(sizeof(double) * (size_t)p.span, kAlign);
        p.buf_off[0] = off; off += bytes;
        p.buf_off[1] = off; off += bytes;
    }
    // compact Dirichlet ghost columns of the unpaired x faces
    int64_t max_xcol = 0;
    for (HostBlock& b : c->blocks) {
        const int64_t col = b.n[2] * jc::face_ld(b.n[1]);
        for (int f = jc::XM; f <= jc::XP; ++f) {
            b.xg_off[f] = 0;
            if (b.pair_in[f] < 0) {
                b.xg_off[f] = off;
                off = align_up(off + sizeof(double) * (size_t)col, kAlign);
                max_xcol = std::max(max_xcol, col);
            }
        }
    }
    c->lo_begin = c->lo_end = off;
    if (c->opt.ir_enable) {
        const size_t es = lo_size(c->opt.ir_dtype);
        const int64_t le = 128 / (int64_t)es;
        for (HostBlock& b : c->blocks) {
            b.lpitch = round_up(b.n[0] + 2, le);
            b.lplane = b.lpitch * (b.n[1] + 2);
            const size_t bytes = align_up(es * (size_t)(b.lplane * (b.n[2] + 2) + le), kAlign);
            b.d_off[0] = off; off += bytes;
            b.d_off[1] = off; off += bytes;
            b.rlo_off = off; off += bytes;
        }
        for (HostPair& p : c->pairs) {
            const size_t bytes = align_up(es * (size_t)p.span, kAlign);
            p.lbuf_off[0] = off; off += bytes;
            p.lbuf_off[1] = off; off += bytes;
        }
        // one zero column serves every unpaired x face of the correction
        c->lxg_off = off;
        off = align_up(off + es * (size_t)std::max<int64_t>(max_xcol, 1), kAlign);
        c->lo_end = off;
    }
    c->footprint = off;
    return JC_OK;
}

std::vector<int64_t> uniform_cuts(int64_t n, int64_t bd)
{
    std::vector<int64_t> v;
    for (int64_t s = 0; s < n; s += bd)
        v.push_back(std::min(bd, n - s));
    return v;
}

int uniform_geometry(jc_ctx* c, const int64_t grid[3], const int64_t block_dims[3], const jc_options* opt)
{
    if (!grid || !block_dims)
        return fail(JC_ERR_INVALID, "grid and block_dims must not be NULL");
    std::vector<int64_t> cuts[3];
    for (int a = 0; a < 3; ++a) {
        if (grid[a] < 1 || grid[a] > kMaxEdge)
            return fail(JC_ERR_INVALID, "grid sizes must be in [1, 2^30]");
        if (block_dims[a] < 1 || block_dims[a] > grid[a])
            return fail(JC_ERR_INVALID, "block_dims must satisfy 1 <= block_dims[i] <= grid[i]");
        if ((grid[a] + block_dims[a] - 1) / block_dims[a] > 65535)
            return fail(JC_ERR_INVALID, "too many blocks along an axis");
        cuts[a] = uniform_cuts(grid[a], block_dims[a]);
    }
    return build_geometry(c, grid, cuts, opt);
}

int rect_geometry(jc_ctx* c, const int64_t grid[3], const int64_t* const cuts[3], const int64_t ncuts[3],
                  const jc_options* opt)
{
    if (!grid || !cuts || !ncuts)
        return fail(JC_ERR_INVALID, "grid, cuts and ncuts must not be NULL");
    std::vector<int64_t> v[3];
    for (int a = 0; a < 3; ++a) {
        if (ncuts[a] < 1 || ncuts[a] > 65535 || !cuts[a])
            return fail(JC_ERR_INVALID, "each axis needs 1..65535 block edges");
        v[a].assign(cuts[a], cuts[a] + ncuts[a]);
    }
    return build_geometry(c, grid, v, opt);
}

}  // namespace

namespace jc_rt {

// ------------------------------------------------------------------ timing

hipEvent_t take_event(jc_ctx* c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

int drain_timing(jc_ctx* c)
{
    if (c->pending.empty())
        return JC_OK;
    JC_HIP(hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float ms = 0.f;
        JC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        c->kernel_ms[p.kind] += ms;
        c->kernel_launches[p.kind] += 1;
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
    return JC_OK;
}

// ------------------------------------------------------------------ steps

int check_ready(jc_ctx* c)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (!c->bound)
        return fail(JC_ERR_STATE, "context is not bound to an arena (jc_bind)");
    if (!c->loaded_u)
        return fail(JC_ERR_STATE, "the iterate has not been loaded (jc_load_field U)");
    if (c->opt.with_source && !c->loaded_b)
        return fail(JC_ERR_STATE, "the source has not been loaded (jc_load_field B)");
    return JC_OK;
}

int do_pack(jc_ctx* c, int slot)
{
    return timed(c, JC_K_PACK, [&] {
        return jc::launch_pack(c->d_blocks(), c->d_pairs(), c->np(), (int)c->max_slow, (int)c->max_fast,
                               c->parity, slot, c->stream);
    });
}

}  // namespace jc_rt

namespace {

// Host staging (the paper's non-GPU-aware path, its "-H" runs): every
// send buffer is copied to pinned host memory, the stream is waited for,
// the host moves the message into the receiver's host buffer, and the
// receive buffer is filled from there.
hipError_t exchange_via_host(jc_ctx* c)
{
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& p = c->pairs[q];
        const hipError_t e = hipMemcpyAsync(c->h_stage + c->h_stage_off[q], c->arena + p.buf_off[0],
                                            sizeof(double) * p.span, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess)
            return e;
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess)
        return e;
    const size_t half = c->h_stage_bytes / 2;
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& p = c->pairs[q];
        std::memcpy(c->h_stage + half + c->h_stage_off[q], c->h_stage + c->h_stage_off[q], sizeof(double) * p.span);
    }
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& p = c->pairs[q];
        e = hipMemcpyAsync(c->arena + p.buf_off[1], c->h_stage + half + c->h_stage_off[q], sizeof(double) * p.span,
                           hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Device transfer announced by host metadata (the GPU Messaging API of
// section 3.2.1): the receiver learns buffer, size and tag from a host
// message sent after the pack, so the host waits for the pack, builds the
// message of every pair, checks it, and only then enqueues the transfer.
hipError_t exchange_with_metadata(jc_ctx* c)
{
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess)
        return e;
    c->meta.resize(c->np());
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& p = c->pairs[q];
        jc_ctx::MetaMsg& m = c->meta[q];
        m.src = p.src_block;
        m.dst = p.dst_block;
        m.bytes = sizeof(double) * p.span;
        m.tag = ((uint64_t)q << 32) | (uint64_t)(c->iters & 0xffffffffu);
    }
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& p = c->pairs[q];
        const jc_ctx::MetaMsg& m = c->meta[q];
        if (m.dst != p.dst_block || m.bytes != sizeof(double) * p.span || (m.tag >> 32) != (uint64_t)q)
            return hipErrorInvalidValue;
    }
    return jc::launch_exchange(c->d_pairs(), c->np(), c->max_count, c->stream);
}

int do_exchange(jc_ctx* c)
{
    return timed(c, JC_K_EXCHANGE, [&] {
        if (c->opt.exchange == JC_EXCHANGE_HOST)
            return exchange_via_host(c);
        if (c->opt.exchange == JC_EXCHANGE_METADATA)
            return exchange_with_metadata(c);
        return jc::launch_exchange(c->d_pairs(), c->np(), c->max_count, c->stream);
    });
}

int do_unpack(jc_ctx* c)
{
    return timed(c, JC_K_UNPACK, [&] {
        return jc::launch_unpack(c->d_blocks(), c->d_pairs(), c->np(), (int)c->max_slow, (int)c->max_fast,
                                 c->parity, c->stream);
    });
}

int do_sweep(jc_ctx* c, bool fused, bool resid)
{
    int st = timed(c, fused ? JC_K_FUSED : JC_K_SWEEP, [&] {
        return jc::launch_sweep(c->d_blocks(), c->d_items(), (int)c->items.size(), c->parity, c->tile_x, c->tile_y,
                                fused, resid, true, c->opt.with_source != 0, c->d_partials(), c->stream,
                                c->opt.ir_enable || c->opt.temporal ? 0u : c->pace);
    });
    if (st != JC_OK)
        return st;
    c->parity ^= 1;
    c->iters += 1;
    if (fused) {
        c->fused_primed = true;
        c->ghost = c->np() ? GHOST_STALE : GHOST_CURRENT;
    } else {
        c->ghost = c->np() ? GHOST_STALE : GHOST_CURRENT;
        c->fused_primed = false;
    }
    return JC_OK;
}

// Planes per two-sweep work-group: the shape set or tuned, else the
// one-sweep z_chunk (at least kTwoStepMinZ), halved down to
// kTwoStepFloorZ while the launch would have fewer than
// kTwoStepMinGroups work-groups (a small grid alone).
int two_step_chunk(const jc_ctx* c)
{
    if (c->t2_zc > 0)
        return c->t2_zc;
    const HostBlock& b = c->blocks[0];
    const int64_t per = ((b.n[0] + 63) / 64) * ((b.n[1] + c->t2_rows - 1) / c->t2_rows);
    int64_t zc = std::max(c->z_chunk, jc_rt::kTwoStepMinZ);
    while (zc > jc_rt::kTwoStepFloorZ && per * ((b.n[2] + zc - 1) / zc) < jc_rt::kTwoStepMinGroups)
        zc = std::max<int64_t>((zc + 1) / 2, jc_rt::kTwoStepFloorZ);
    return (int)zc;
}

// The pace of a temporal context belongs to its deepest launch (the one its
// solve loop runs); the other launches run unpaced.
uint32_t multi_pace(const jc_ctx* c, int depth) { return c->depth() == depth ? c->pace : 0u; }

hipError_t launch_two_step(jc_ctx* c, int rows, int zc, uint32_t pace)
{
    const HostBlock& b = c->blocks[0];
    return jc::launch_sweep2(c->d_blocks(), (int)b.n[0], (int)b.n[1], (int)b.n[2], c->parity, rows, zc,
                             c->opt.with_source != 0, c->stream, pace);
}
hipError_t launch_two_step(jc_ctx* c, int rows, int zc) { return launch_two_step(c, rows, zc, multi_pace(c, 2)); }

// Two inner sweeps of the refinement correction in one launch (copy
// qparity -> qparity ^ 1).
hipError_t launch_ir_two_step(jc_ctx* c, int qparity, int rows, int zc, uint32_t pace)
{
    const HostBlock& b = c->blocks[0];
    return jc::launch_ir_inner2(c->d_blocks(), (int)b.n[0], (int)b.n[1], (int)b.n[2], qparity, rows, zc,
                                c->opt.ir_dtype, c->stream, pace);
}
hipError_t launch_ir_two_step(jc_ctx* c, int qparity, int rows, int zc)
{
    return launch_ir_two_step(c, qparity, rows, zc, multi_pace(c, 2));
}

// Three sweeps in one launch (temporal blocking, three per launch).
hipError_t launch_three_step(jc_ctx* c, int rows, int zc, uint32_t pace)
{
    const HostBlock& b = c->blocks[0];
    return jc::launch_sweep3(c->d_blocks(), nullptr, 0, (int)b.n[0], (int)b.n[1], (int)b.n[2], c->parity, rows, zc,
                             c->opt.with_source != 0, c->stream, pace);
}
hipError_t launch_three_step(jc_ctx* c, int rows, int zc) { return launch_three_step(c, rows, zc, multi_pace(c, 3)); }

hipError_t launch_ir_three_step(jc_ctx* c, int qparity, int rows, int zc, uint32_t pace)
{
    const HostBlock& b = c->blocks[0];
    return jc::launch_ir_inner3(c->d_blocks(), nullptr, 0, (int)b.n[0], (int)b.n[1], (int)b.n[2], qparity, rows, zc,
                                c->opt.ir_dtype, c->stream, pace);
}
hipError_t launch_ir_three_step(jc_ctx* c, int qparity, int rows, int zc)
{
    return launch_ir_three_step(c, qparity, rows, zc, multi_pace(c, 3));
}

// Launches that run n sweeps at depth d (sweeps per launch): n / d full
// launches, then one launch for a remainder (a two-sweep launch for 2, a
// single sweep for 1).
int64_t launches_for(int64_t n, int d)
{
    return d <= 1 ? n : n / d + (n % d != 0);
}

// Copy of d that holds the correction after m inner sweeps: the first
// sweep writes copy 1 and every later launch flips it (a multi-sweep
// launch once).
int ir_final_copy(const jc_ctx* c, int64_t m)
{
    return (int)((1 + launches_for(m - 1, c->depth())) & 1);
}

// Three sweeps in one launch (temporal blocking; one block, no pairs).
int do_sweep3(jc_ctx* c)
{
    int st = timed(c, JC_K_SWEEP3, [&] { return launch_three_step(c, c->t2_rows, two_step_chunk(c)); });
    if (st != JC_OK)
        return st;
    c->parity ^= 1;
    c->iters += 3;
    c->ghost = GHOST_CURRENT;
    c->fused_primed = c->opt.mode == JC_MODE_FUSED;
    return JC_OK;
}

// Two sweeps in one launch (temporal blocking; one block, no pairs).
int do_sweep2(jc_ctx* c)
{
    int st = timed(c, JC_K_SWEEP2, [&] { return launch_two_step(c, c->t2_rows, two_step_chunk(c)); });
    if (st != JC_OK)
        return st;
    c->parity ^= 1;
    c->iters += 2;
    c->ghost = GHOST_CURRENT;
    c->fused_primed = c->opt.mode == JC_MODE_FUSED;
    return JC_OK;
}

// n sweeps in one launch (a resident context: one block that fits on chip).
int do_resident(jc_ctx* c, int64_t n)
{
    const auto& b = c->blocks[0];
    const int nx = (int)b.n[0], ny = (int)b.n[1], nz = (int)b.n[2];
    int st = timed(c, JC_K_RESIDENT, [&] {
        return jc::launch_resident(c->d_blocks(), nullptr, 1, (nx + 1) / 2 * ny, nz,
                                   (size_t)jc::resident_lds_bytes(nx, ny, nz), jc::resident_variant(nz), c->parity, (int)n,
                                   c->opt.with_source != 0, c->stream);
    });
    if (st != JC_OK)
        return st;
    c->parity ^= (int)(n & 1);
    c->iters += n;
    c->ghost = GHOST_CURRENT;
    c->fused_primed = false;
    return JC_OK;
}

int do_halo(jc_ctx* c)
{
    if (c->np() == 0) {
        c->ghost = GHOST_CURRENT;
        return JC_OK;
    }
    int st = do_pack(c, 0);
    if (st == JC_OK) st = do_exchange(c);
    if (st == JC_OK) st = do_unpack(c);
    if (st == JC_OK) {
        c->ghost = GHOST_CURRENT;
        c->fused_primed = false;
    }
    return st;
}

// One staged iteration, boundary first: the tiles that hold a paired face
// plane sweep on the bound stream while the interior tiles sweep on the
// side stream at the same time; as soon as the boundary tiles are done,
// the faces of the new iterate are packed, exchanged and unpacked on the
// bound stream, overlapping the rest of the interior sweep, and the bound
// stream then waits for the interior.  Every cell is computed by the same
// kernel from the same inputs as in one launch, so the iterate is bitwise
// the same.  Hazards: both sweeps read the old copy and write disjoint
// cells of the new one; the halo steps read the new iterate's face planes
// (written by boundary tiles only) and write its ghost planes (which the
// interior tiles neither read nor write: a pair store that reaches the
// x = nx + 1 ghost of a paired face belongs to a boundary tile).
int overlapped_iteration(jc_ctx* c, bool resid)
{
    if (c->ghost != GHOST_CURRENT) {
        int st = do_halo(c);
        if (st != JC_OK)
            return st;
    }
    const bool src = c->opt.with_source != 0;
    const int nb = (int)c->n_bnd, ni = (int)c->items.size() - nb;
    JC_HIP(hipEventRecord(c->ev_fork, c->stream));
    JC_HIP(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    int st = timed(c, JC_K_SWEEP, [&] {
        return jc::launch_sweep(c->d_blocks(), c->d_items(), nb, c->parity, c->tile_x, c->tile_y, false, resid, true,
                                src, c->d_partials(), c->stream);
    });
    if (st != JC_OK)
        return st;
    // the interior tiles, on the side stream
    std::swap(c->stream, c->side);
    st = timed(c, JC_K_SWEEP, [&] {
        return jc::launch_sweep(c->d_blocks(), c->d_items() + nb, ni, c->parity, c->tile_x, c->tile_y, false, resid,
                                true, src, c->d_partials() + nb, c->stream);
    });
    std::swap(c->stream, c->side);
    if (st != JC_OK)
        return st;
    JC_HIP(hipEventRecord(c->ev_join, c->side));
    // the halo of the new iterate (copy parity ^ 1)
    c->parity ^= 1;
    st = do_pack(c, 0);
    if (st == JC_OK)
        st = do_exchange(c);
    if (st == JC_OK)
        st = do_unpack(c);
    c->parity ^= 1;
    if (st != JC_OK)
        return st;
    JC_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    c->parity ^= 1;
    c->iters += 1;
    c->ghost = GHOST_CURRENT;
    c->fused_primed = false;
    return JC_OK;
}

// One full iteration of the context's mode; resid: the sweep also sums
// r^2 of its input iterate into the partials.
int one_iteration(jc_ctx* c, bool resid)
{
    if (c->side && c->opt.mode == JC_MODE_STAGED)
        return overlapped_iteration(c, resid);
    if (c->opt.mode == JC_MODE_FUSED) {
        if (!c->fused_primed && c->np()) {
            int st = do_pack(c, c->parity);
            if (st != JC_OK)
                return st;
            c->fused_primed = true;
        }
        return do_sweep(c, c->np() > 0, resid);
    }
    int st = do_halo(c);
    if (st != JC_OK)
        return st;
    return do_sweep(c, false, resid);
}

int reduce_to_host(jc_ctx* c, double* sumsq)
{
    JC_HIP(jc::launch_reduce(c->d_partials(), c->d_ranges(), 1, c->d_result(), c->stream));
    JC_HIP(hipMemcpyAsync(c->h_result, c->d_result(), sizeof(double), hipMemcpyDeviceToHost, c->stream));
    JC_HIP(hipStreamSynchronize(c->stream));
    int st = drain_timing(c);
    if (st != JC_OK)
        return st;
    *sumsq = c->h_result[0];
    return JC_OK;
}

// Residual of the current iterate by a standalone pass.
int residual_now(jc_ctx* c, double* l2)
{
    bool fused = false;
    if (c->opt.mode == JC_MODE_FUSED && c->np()) {
        if (!c->fused_primed) {
            int st = do_pack(c, c->parity);
            if (st != JC_OK)
                return st;
            c->fused_primed = true;
        }
        fused = true;
    } else if (c->ghost != GHOST_CURRENT) {
        int st = do_halo(c);
        if (st != JC_OK)
            return st;
    }
    int st = timed(c, JC_K_RESIDUAL, [&] {
        return jc::launch_sweep(c->d_blocks(), c->d_items(), (int)c->items.size(), c->parity, c->tile_x, c->tile_y, fused,
                                true, false, c->opt.with_source != 0, c->d_partials(), c->stream);
    });
    if (st != JC_OK)
        return st;
    double s = 0;
    st = reduce_to_host(c, &s);
    if (st != JC_OK)
        return st;
    *l2 = std::sqrt(s);
    if (!std::isfinite(*l2))
        return fail(JC_ERR_NONFINITE, "residual is not finite");
    return JC_OK;
}

// n plain iterations launched eagerly: with temporal blocking, pairs of
// sweeps in one launch each and a last single sweep when n is odd.
int iterate_eager(jc_ctx* c, int64_t n)
{
    if (c->opt.resident) {
        // one launch per 2^30 sweeps
        for (int64_t i = 0; i < n;) {
            const int64_t m = std::min<int64_t>(n - i, (int64_t)1 << 30);
            int st = do_resident(c, m);
            if (st != JC_OK)
                return st;
            i += m;
        }
        return JC_OK;
    }
    int64_t i = 0;
    if (c->depth() == 3) {
        for (; i + 3 <= n; i += 3) {
            int st = do_sweep3(c);
            if (st != JC_OK)
                return st;
        }
    }
    if (c->opt.temporal) {
        for (; i + 2 <= n; i += 2) {
            int st = do_sweep2(c);
            if (st != JC_OK)
                return st;
        }
    }
    for (; i < n; ++i) {
        int st = one_iteration(c, false);
        if (st != JC_OK)
            return st;
    }
    return JC_OK;
}

// n plain iterations, as one graph replay when graphs are enabled.
int iterate_window(jc_ctx* c, int64_t n)
{
    if (n <= 0)
        return JC_OK;
    // a resident window is one launch already: nothing to capture
    const bool graphs = c->opt.use_graphs && c->stream != nullptr && !c->timing &&
                        c->opt.exchange == JC_EXCHANGE_DEVICE && !c->opt.resident;
    if (!graphs)
        return iterate_eager(c, n);
    // the priming pack of fused mode stays outside the graph
    if (c->opt.mode == JC_MODE_FUSED && !c->fused_primed && c->np()) {
        int st = do_pack(c, c->parity);
        if (st != JC_OK)
            return st;
        c->fused_primed = true;
    }
    const auto key = std::make_pair(n, c->parity);
    auto found = c->graphs.find(key);
    if (found == c->graphs.end()) {
        const int parity0 = c->parity;
        const int64_t iters0 = c->iters;
        const int ghost0 = c->ghost;
        const bool primed0 = c->fused_primed;
        JC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int st = iterate_eager(c, n);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &graph);
        // capture only recorded the launches: restore the state and replay
        c->parity = parity0;
        c->iters = iters0;
        c->ghost = ghost0;
        c->fused_primed = primed0;
        if (st != JC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess)
            return fail(JC_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess)
            return fail(JC_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        found = c->graphs.emplace(key, exec).first;
    }
    JC_HIP(hipGraphLaunch(found->second, c->stream));
    // the state after n iterations, as the eager path would leave it
    // (a two-sweep launch flips the copy once)
    const int64_t launches = launches_for(n, c->depth());
    c->parity ^= (int)(launches & 1);
    c->iters += n;
    if (c->np()) {
        c->ghost = GHOST_STALE;
        c->fused_primed = c->opt.mode == JC_MODE_FUSED;
    }
    return JC_OK;
}

void free_graphs(jc_ctx* c)
{
    for (auto& kv : c->graphs)
        (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// Times the two-sweep launch (of the correction on a refinement context)
// over tile rows {8, 16, 24} x z-chunk counts and keeps the fastest (temporal
// contexts; run by jc_autotune after its one-sweep search, on a warm
// device).  Which shape wins depends on how
// the work-groups fill the compute units and on how close in time
// neighbouring tiles read their shared halo rows (an L2 hit), so it is
// measured rather than modelled.  Trial launches read copy `parity` and
// write the other copy: the iterate is unchanged.
int tune_two_step(jc_ctx* c, int reps)
{
    const int64_t nz = c->blocks[0].n[2];
    struct Cand {
        int rows, zc;
        double ms;
    };
    std::vector<Cand> cand;
    const bool three = c->depth() == 3;
    std::vector<int> row_cands;
    if (three)
        row_cands.assign(std::begin(jc_rt::kThreeStepRowCandidates), std::end(jc_rt::kThreeStepRowCandidates));
    else
        row_cands.assign(std::begin(jc_rt::kTwoStepRowCandidates), std::end(jc_rt::kTwoStepRowCandidates));
    for (int rows : row_cands)
        for (int nch : {1, 2, 3, 4, 6, 8, 12, 16}) {
            const int zc = (int)((nz + nch - 1) / nch);
            bool dup = false;
            for (const Cand& k : cand)
                dup = dup || (k.rows == rows && k.zc == zc);
            if (!dup)
                cand.push_back({rows, zc, 0.0});
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    JC_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(JC_ERR_DEVICE, "autotune: hipEventCreate failed");
    }
    // a refinement context is tuned for its inner sweeps (on the zeroed
    // correction arrays, as the one-sweep search left them)
    const bool ir = c->opt.ir_enable != 0;
    auto launch = [&](const Cand& k) {
        if (three)
            return ir ? launch_ir_three_step(c, 1, k.rows, k.zc, 0) : launch_three_step(c, k.rows, k.zc, 0);
        return ir ? launch_ir_two_step(c, 1, k.rows, k.zc, 0) : launch_two_step(c, k.rows, k.zc, 0);
    };
    // milliseconds of n launches after one untimed launch
    auto time_one = [&](const Cand& k, int n, double& ms) -> int {
        hipError_t e = launch(k);
        if (e == hipSuccess)
            e = hipEventRecord(e0, c->stream);
        for (int i = 0; i < n && e == hipSuccess; ++i)
            e = launch(k);
        if (e == hipSuccess)
            e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, e0, e1);
        ms = t;
        return e == hipSuccess ? JC_OK
                               : fail(JC_ERR_DEVICE, std::string("autotune (two-sweep launch): ") + hipGetErrorString(e));
    };
    int st = JC_OK;
    for (size_t i = 0; i < cand.size() && st == JC_OK; ++i)
        st = time_one(cand[i], reps, cand[i].ms);
    if (st == JC_OK) {
        std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
        cand.resize(std::min<size_t>(cand.size(), 3));
        for (Cand& k : cand)
            k.ms = 0;
        for (int round = 0; round < 3 && st == JC_OK; ++round)
            for (size_t i = 0; i < cand.size() && st == JC_OK; ++i) {
                double ms = 0;
                st = time_one(cand[i], reps, ms);
                cand[i].ms += ms;
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != JC_OK)
        return st;
    const Cand best = *std::min_element(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
    c->t2_rows = best.rows;
    c->t2_zc = best.zc;
    c->pace = 0;
    free_graphs(c);
    return JC_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

const char* jc_last_error(void) { return jc_rt::g_err.c_str(); }

int jc_min_surface_parts(const int64_t grid[3], int64_t nblocks, int64_t parts[3])
{
    if (!grid || !parts || nblocks < 1)
        return fail(JC_ERR_INVALID, "grid and parts must not be NULL and nblocks >= 1");
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 1)
            return fail(JC_ERR_INVALID, "grid sizes must be >= 1");
    double best = -1;
    int64_t bp[3] = {0, 0, 0};
    for (int64_t px = 1; px <= nblocks; ++px) {
        if (nblocks % px || px > grid[0])
            continue;
        for (int64_t py = 1; py <= nblocks / px; ++py) {
            if ((nblocks / px) % py || py > grid[1])
                continue;
            const int64_t pz = nblocks / px / py;
            if (pz > grid[2])
                continue;
            // both sides of every cut plane, plus the outer surface
            const double gx = (double)grid[0], gy = (double)grid[1], gz = (double)grid[2];
            const double area = 2.0 * (gy * gz * (double)px + gx * gz * (double)py + gx * gy * (double)pz);
            const bool better = best < 0 || area < best ||
                                (area == best && (pz > bp[2] || (pz == bp[2] && py > bp[1])));
            if (better) {
                best = area;
                bp[0] = px; bp[1] = py; bp[2] = pz;
            }
        }
    }
    if (best < 0)
        return fail(JC_ERR_INVALID, "no decomposition of the grid into that many blocks");
    parts[0] = bp[0]; parts[1] = bp[1]; parts[2] = bp[2];
    return JC_OK;
}

int jc_footprint(const int64_t grid[3], const int64_t block_dims[3], const jc_options* opt, size_t* bytes)
{
    if (!bytes)
        return fail(JC_ERR_INVALID, "bytes must not be NULL");
    jc_ctx tmp;
    int st = uniform_geometry(&tmp, grid, block_dims, opt);
    if (st != JC_OK)
        return st;
    *bytes = tmp.footprint;
    return JC_OK;
}

int jc_footprint_rectilinear(const int64_t grid[3], const int64_t* const cuts[3], const int64_t ncuts[3],
                             const jc_options* opt, size_t* bytes)
{
    if (!bytes)
        return fail(JC_ERR_INVALID, "bytes must not be NULL");
    jc_ctx tmp;
    int st = rect_geometry(&tmp, grid, cuts, ncuts, opt);
    if (st != JC_OK)
        return st;
    *bytes = tmp.footprint;
    return JC_OK;
}

int jc_create(const int64_t grid[3], const int64_t block_dims[3], const jc_options* opt, jc_ctx** out)
{
    if (!out)
        return fail(JC_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    jc_ctx* c = new (std::nothrow) jc_ctx();
    if (!c)
        return fail(JC_ERR_NOMEM, "host allocation failed");
    int st = uniform_geometry(c, grid, block_dims, opt);
    if (st != JC_OK) {
        delete c;
        return st;
    }
    *out = c;
    return JC_OK;
}

int jc_create_rectilinear(const int64_t grid[3], const int64_t* const cuts[3], const int64_t ncuts[3],
                          const jc_options* opt, jc_ctx** out)
{
    if (!out)
        return fail(JC_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    jc_ctx* c = new (std::nothrow) jc_ctx();
    if (!c)
        return fail(JC_ERR_NOMEM, "host allocation failed");
    int st = rect_geometry(c, grid, cuts, ncuts, opt);
    if (st != JC_OK) {
        delete c;
        return st;
    }
    *out = c;
    return JC_OK;
}

void jc_destroy(jc_ctx* c)
{
    if (!c)
        return;
    if (c->bound) {
        (void)hipStreamSynchronize(c->stream);
        free_graphs(c);
        for (auto& p : c->pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipEvent_t e : c->event_pool)
            (void)hipEventDestroy(e);
        if (c->h_result)
            (void)hipHostFree(c->h_result);
        if (c->h_stage)
            (void)hipHostFree(c->h_stage);
    }
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork)
        (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join)
        (void)hipEventDestroy(c->ev_join);
    delete c;
}

int jc_bind(jc_ctx* c, void* dev_arena, size_t bytes, void* hip_stream)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (c->bound)
        return fail(JC_ERR_STATE, "context is already bound");
    if (!dev_arena)
        return fail(JC_ERR_INVALID, "arena must not be NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign)
        return fail(JC_ERR_INVALID, "arena must be 256-byte aligned");
    if (bytes < c->footprint)
        return fail(JC_ERR_NOMEM, "arena smaller than jc_footprint (" + std::to_string(bytes) + " < " +
                                       std::to_string(c->footprint) + ")");
    c->arena = static_cast<char*>(dev_arena);
    c->arena_bytes = bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    JC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_result), sizeof(double) * 4, hipHostMallocDefault));
    if (c->opt.overlap && c->np()) {
        // the halo stream of boundary-first iterations (default priority)
        JC_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        JC_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        JC_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    if (c->opt.exchange == JC_EXCHANGE_HOST && c->np()) {
        size_t off = 0;
        c->h_stage_off.assign(c->np(), 0);
        for (int q = 0; q < c->np(); ++q) {
            c->h_stage_off[q] = off;
            off += align_up(sizeof(double) * (size_t)c->pairs[q].span, kAlign);
        }
        c->h_stage_bytes = 2 * off;
        JC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_stage), c->h_stage_bytes, hipHostMallocDefault));
    }
    c->hdesc.assign(c->blocks.size(), BlockDesc{});
    for (int bi = 0; bi < c->nb(); ++bi) {
        const HostBlock& hb = c->blocks[bi];
        BlockDesc& d = c->hdesc[bi];
        const int64_t lead = jc::line_elems<double>() - 1;
        d.u[0] = reinterpret_cast<double*>(c->arena + hb.u_off[0]) + lead;
        d.u[1] = reinterpret_cast<double*>(c->arena + hb.u_off[1]) + lead;
        d.b = c->opt.with_source ? reinterpret_cast<double*>(c->arena + hb.b_off) + lead : nullptr;
        for (int f = 0; f < 6; ++f)
            for (int s = 0; s < 2; ++s) {
                d.gin[f][s] = hb.pair_in[f] >= 0
                                  ? reinterpret_cast<double*>(c->arena + c->pairs[hb.pair_in[f]].buf_off[s])
                                  : nullptr;
                d.gout[f][s] = hb.pair_out[f] >= 0
                                   ? reinterpret_cast<double*>(c->arena + c->pairs[hb.pair_out[f]].buf_off[s])
                                   : nullptr;
            }
        for (int f = jc::XM; f <= jc::XP; ++f)
            d.xg[f] = hb.pair_in[f] < 0 ? reinterpret_cast<const double*>(c->arena + hb.xg_off[f]) : nullptr;
        for (int a = 0; a < 3; ++a) {
            d.n[a] = (int32_t)hb.n[a];
            d.off[a] = (int32_t)hb.off[a];
        }
        d.pitch = (int32_t)hb.pitch;
        d.plane = hb.plane;
        if (c->opt.ir_enable) {
            const size_t es = lo_size(c->opt.ir_dtype);
            const size_t llead = (128 / es - 1) * es;
            d.d[0] = c->arena + hb.d_off[0] + llead;
            d.d[1] = c->arena + hb.d_off[1] + llead;
            d.rlo = c->arena + hb.rlo_off + llead;
            d.lpitch = (int32_t)hb.lpitch;
            d.lplane = hb.lplane;
            for (int f = 0; f < 6; ++f)
                for (int s = 0; s < 2; ++s) {
                    d.lgin[f][s] = hb.pair_in[f] >= 0 ? c->arena + c->pairs[hb.pair_in[f]].lbuf_off[s] : nullptr;
                    d.lgout[f][s] = hb.pair_out[f] >= 0 ? c->arena + c->pairs[hb.pair_out[f]].lbuf_off[s] : nullptr;
                }
            for (int f = jc::XM; f <= jc::XP; ++f)
                d.lxg[f] = hb.pair_in[f] < 0 ? c->arena + c->lxg_off : nullptr;
        }
    }
    c->hpairs.assign(c->pairs.size(), PairDesc{});
    for (int q = 0; q < c->np(); ++q) {
        const HostPair& hp = c->pairs[q];
        PairDesc& d = c->hpairs[q];
        d.src_block = hp.src_block; d.src_face = hp.src_face;
        d.dst_block = hp.dst_block; d.dst_face = hp.dst_face;
        d.slow = (int32_t)hp.slow; d.fast = (int32_t)hp.fast; d.count = hp.count; d.span = hp.span;
        d.buf[0] = reinterpret_cast<double*>(c->arena + hp.buf_off[0]);
        d.buf[1] = reinterpret_cast<double*>(c->arena + hp.buf_off[1]);
        if (c->opt.ir_enable) {
            d.lbuf[0] = c->arena + hp.lbuf_off[0];
            d.lbuf[1] = c->arena + hp.lbuf_off[1];
        }
    }
    c->hranges[0] = 0;
    c->hranges[1] = (int32_t)c->items.size();
    JC_HIP(hipMemcpyAsync(c->d_blocks(), c->hdesc.data(), sizeof(BlockDesc) * c->hdesc.size(),
                          hipMemcpyHostToDevice, c->stream));
    if (c->np())
        JC_HIP(hipMemcpyAsync(c->d_pairs(), c->hpairs.data(), sizeof(PairDesc) * c->hpairs.size(),
                              hipMemcpyHostToDevice, c->stream));
    JC_HIP(hipMemcpyAsync(c->d_items(), c->items.data(), sizeof(Item) * c->items.size(), hipMemcpyHostToDevice,
                          c->stream));
    JC_HIP(hipMemcpyAsync(c->d_ranges(), c->hranges, sizeof(c->hranges), hipMemcpyHostToDevice, c->stream));
    JC_HIP(hipStreamSynchronize(c->stream));   // host tables may change after this call
    c->bound = true;
    return JC_OK;
}

int jc_load_field(jc_ctx* c, int which, const void* src)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (!c->bound)
        return fail(JC_ERR_STATE, "context is not bound (jc_bind)");
    if (!src)
        return fail(JC_ERR_INVALID, "source array must not be NULL");
    if (which == JC_FIELD_B && !c->opt.with_source)
        return fail(JC_ERR_INVALID, "context was created without a source field");
    if (which != JC_FIELD_U && which != JC_FIELD_B)
        return fail(JC_ERR_INVALID, "which must be JC_FIELD_U or JC_FIELD_B");
    JC_HIP(jc::launch_scatter(c->d_blocks(), c->nb(), c->max_rows(), static_cast<const double*>(src), c->grid[0],
                              c->grid[1],
                              which, c->stream));
    if (which == JC_FIELD_U) {
        c->loaded_u = true;
        c->check_r0 = -1.0;
        c->parity = 0;
        c->iters = 0;
        c->ghost = GHOST_CURRENT;     // the scatter filled every ghost with iterate 0
        c->fused_primed = false;
        c->ir_phase = 0;              // a group's unfinished refinement step belonged to the old iterate
    } else {
        c->loaded_b = true;
    }
    return JC_OK;
}

int jc_store_field(jc_ctx* c, int which, void* dst)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (!c->bound)
        return fail(JC_ERR_STATE, "context is not bound (jc_bind)");
    if (!dst)
        return fail(JC_ERR_INVALID, "destination array must not be NULL");
    if (which == JC_FIELD_B && !c->opt.with_source)
        return fail(JC_ERR_INVALID, "context was created without a source field");
    if (which != JC_FIELD_U && which != JC_FIELD_B)
        return fail(JC_ERR_INVALID, "which must be JC_FIELD_U or JC_FIELD_B");
    if ((which == JC_FIELD_U && !c->loaded_u) || (which == JC_FIELD_B && !c->loaded_b))
        return fail(JC_ERR_STATE, "field was never loaded");
    JC_HIP(jc::launch_gather(c->d_blocks(), c->nb(), c->max_rows(), static_cast<double*>(dst), c->grid[0], c->grid[1],
                             c->grid[2], which, c->parity, c->stream));
    return JC_OK;
}

int jc_pack_faces(jc_ctx* c)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    st = do_pack(c, 0);
    if (st == JC_OK) {
        c->ghost = GHOST_PACKED;
        c->fused_primed = false;
    }
    return st;
}

int jc_exchange(jc_ctx* c)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (c->ghost != GHOST_PACKED)
        return fail(JC_ERR_STATE, "jc_exchange needs jc_pack_faces first");
    st = do_exchange(c);
    if (st == JC_OK)
        c->ghost = GHOST_EXCHANGED;
    return st;
}

int jc_unpack_faces(jc_ctx* c)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (c->ghost != GHOST_EXCHANGED)
        return fail(JC_ERR_STATE, "jc_unpack_faces needs jc_exchange first");
    st = do_unpack(c);
    if (st == JC_OK)
        c->ghost = GHOST_CURRENT;
    return st;
}

int jc_sweep(jc_ctx* c)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (c->np() && c->ghost != GHOST_CURRENT)
        return fail(JC_ERR_STATE, "halo is stale: jc_pack_faces, jc_exchange, jc_unpack_faces first");
    return do_sweep(c, false, false);
}

int jc_iterate(jc_ctx* c, int64_t n)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (n < 0)
        return fail(JC_ERR_INVALID, "n must be >= 0");
    return iterate_window(c, n);
}

int jc_residual(jc_ctx* c, double* host_l2)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (!host_l2)
        return fail(JC_ERR_INVALID, "host_l2 must not be NULL");
    return residual_now(c, host_l2);
}

int jc_solve(jc_ctx* c, double rtol, int64_t max_iter, int64_t check_every, jc_solve_info* info)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (!info)
        return fail(JC_ERR_INVALID, "info must not be NULL");
    if (max_iter < 0 || check_every < 1)
        return fail(JC_ERR_INVALID, "max_iter must be >= 0 and check_every >= 1");
    if (!std::isfinite(rtol))
        return fail(JC_ERR_INVALID, "rtol must be finite");
    info->history_len = 0;
    info->outer = 0;
    const bool checks = rtol > 0 || (info->history && info->history_cap > 0);
    auto record = [&](double r) {
        if (info->history && info->history_len < info->history_cap)
            info->history[info->history_len++] = r;
        info->outer += 1;
    };
    const int64_t start = c->iters;
    double r0 = -1.0, r = 0.0;
    int64_t k = 0;
    int status = JC_MAXITER;
    while (true) {
        if (k == max_iter) {
            st = residual_now(c, &r);
            if (st != JC_OK)
                return st;
            if (r0 < 0)
                r0 = r;
            record(r);
            const double rel = r0 > 0 ? r / r0 : 0.0;
            status = (rtol > 0 && rel <= rtol) ? JC_OK : JC_MAXITER;
            break;
        }
        if (checks && k % check_every == 0) {
            // the sweep out of iterate k also sums r_k^2
            st = one_iteration(c, true);
            if (st != JC_OK)
                return st;
            double s = 0;
            st = reduce_to_host(c, &s);
            if (st != JC_OK)
                return st;
            r = std::sqrt(s);
            if (!std::isfinite(r))
                return fail(JC_ERR_NONFINITE, "residual is not finite at iteration " + std::to_string(start + k));
            if (r0 < 0)
                r0 = r;
            record(r);
            const double rel = r0 > 0 ? r / r0 : 0.0;
            if (rtol > 0 && rel <= rtol) {
                // return iterate k: it is still intact in the other copy
                c->parity ^= 1;
                c->iters -= 1;
                if (c->opt.mode == JC_MODE_FUSED) {
                    // slot `parity` of every face buffer still holds iterate k's faces
                    c->fused_primed = true;
                    c->ghost = c->np() ? GHOST_STALE : GHOST_CURRENT;
                } else {
                    // the halo of iterate k was unpacked into its copy before the sweep
                    c->ghost = GHOST_CURRENT;
                    c->fused_primed = false;
                }
                status = JC_OK;
                break;
            }
            k += 1;
            const int64_t n = std::min(check_every - 1, max_iter - k);
            st = iterate_window(c, n);
            if (st != JC_OK)
                return st;
            k += n;
        } else {
            const int64_t n = checks ? std::min(check_every - (k % check_every), max_iter - k) : max_iter - k;
            st = iterate_window(c, n);
            if (st != JC_OK)
                return st;
            k += n;
        }
    }
    info->iters = c->iters - start;
    info->abs_resid = r;
    info->r0 = r0;
    info->rel_resid = r0 > 0 ? r / r0 : 0.0;
    info->status = status;
    return status;
}

int jc_solve_ir(jc_ctx* c, int inner_sweeps, double rtol, int64_t max_inner, jc_solve_info* info)
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (!info)
        return fail(JC_ERR_INVALID, "info must not be NULL");
    if (!c->opt.ir_enable)
        return fail(JC_ERR_STATE, "context was created without refinement buffers (options.ir_enable)");
    if (inner_sweeps < 1 || max_inner < 0 || !std::isfinite(rtol))
        return fail(JC_ERR_INVALID, "inner_sweeps must be >= 1, max_inner >= 0 and rtol finite");
    const int lo = c->opt.ir_dtype;
    const bool src = c->opt.with_source != 0;
    info->history_len = 0;
    info->outer = 0;
    // d = 0 with zero ghosts, once: sweeps never write a ghost.  A solve
    // starts its refinement afresh from the current iterate, so a group's
    // unfinished step on this context (if any) is dropped.
    st = timed(c, JC_K_IR_OUTER, [&] {
        return jc::launch_zero(c->arena + c->lo_begin, c->lo_end - c->lo_begin, c->stream);
    });
    if (st != JC_OK)
        return st;
    c->ir_phase = 0;
    // faces of the current iterate into slot `parity` of the u buffers
    if (c->np()) {
        st = do_pack(c, c->parity);
        if (st != JC_OK)
            return st;
    }
    const int64_t start = c->iters;
    double r0 = -1.0, r = 0.0;
    int64_t done = 0;
    int status = JC_MAXITER;
    while (true) {
        st = timed(c, JC_K_IR_OUTER, [&] {
            return jc::launch_ir_residual(c->d_blocks(), c->d_items(), (int)c->items.size(), c->parity,
                                          c->tile_x, c->tile_y, src, lo, c->d_partials(), c->stream);
        });
        if (st != JC_OK)
            return st;
        double ss = 0;
        st = reduce_to_host(c, &ss);
        if (st != JC_OK)
            return st;
        r = std::sqrt(ss);
        if (!std::isfinite(r))
            return fail(JC_ERR_NONFINITE, "residual is not finite after " + std::to_string(done) + " inner sweeps");
        if (r0 < 0)
            r0 = r;
        if (info->history && info->history_len < info->history_cap)
            info->history[info->history_len++] = r;
        info->outer += 1;
        const double rel = r0 > 0 ? r / r0 : 0.0;
        if (rel <= rtol) {
            status = JC_OK;
            break;
        }
        if (done >= max_inner)
            break;
        const int64_t m = std::min<int64_t>(inner_sweeps, max_inner - done);
        // the m inner sweeps of a step: first sweep (d_0 = 0) into copy 1,
        // then alternating copies (two sweeps per launch with temporal
        // blocking, and a last single sweep if one is left)
        const int q = ir_final_copy(c, m);
        auto inner_window = [&]() -> int {
            int s2 = timed(c, JC_K_IR_INNER, [&] {
                return jc::launch_ir_first(c->d_blocks(), c->nb(), c->max_rows(), lo, c->stream);
            });
            int qq = 1;
            int64_t j = 1;
            if (c->depth() == 3) {
                for (; j + 3 <= m && s2 == JC_OK; j += 3) {
                    s2 = timed(c, JC_K_IR_INNER,
                               [&] { return launch_ir_three_step(c, qq, c->t2_rows, two_step_chunk(c)); });
                    qq ^= 1;
                }
            }
            if (c->opt.temporal) {
                for (; j + 2 <= m && s2 == JC_OK; j += 2) {
                    s2 = timed(c, JC_K_IR_INNER,
                               [&] { return launch_ir_two_step(c, qq, c->t2_rows, two_step_chunk(c)); });
                    qq ^= 1;
                }
            }
            for (; j < m && s2 == JC_OK; ++j) {
                s2 = timed(c, JC_K_IR_INNER, [&] {
                    return jc::launch_ir_inner(c->d_blocks(), c->d_items(), (int)c->items.size(), qq, c->tile_x,
                                               c->tile_y, lo, c->stream, c->opt.temporal ? 0u : c->pace);
                });
                qq ^= 1;
            }
            return s2;
        };
        if (c->opt.use_graphs && c->stream != nullptr && !c->timing) {
            // one graph per window length (key space apart from jc_iterate's)
            const auto key = std::make_pair(m, 2);
            auto found = c->graphs.find(key);
            if (found == c->graphs.end()) {
                JC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                st = inner_window();
                hipGraph_t graph = nullptr;
                const hipError_t e = hipStreamEndCapture(c->stream, &graph);
                if (st != JC_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return st;
                }
                if (e != hipSuccess)
                    return fail(JC_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
                hipGraphExec_t exec = nullptr;
                const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e2 != hipSuccess)
                    return fail(JC_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
                found = c->graphs.emplace(key, exec).first;
            }
            JC_HIP(hipGraphLaunch(found->second, c->stream));
        } else {
            st = inner_window();
            if (st != JC_OK)
                return st;
        }
        st = timed(c, JC_K_IR_OUTER, [&] {
            return jc::launch_ir_update(c->d_blocks(), c->nb(), c->max_rows(), c->parity, q, lo, c->stream);
        });
        if (st != JC_OK)
            return st;
        done += m;
        c->iters += m;
    }
    // u stayed in its copy; its faces of slot `parity` are current
    c->ghost = c->np() ? GHOST_STALE : GHOST_CURRENT;
    c->fused_primed = c->np() > 0;
    info->iters = c->iters - start;
    info->abs_resid = r;
    info->r0 = r0;
    info->rel_resid = r0 > 0 ? r / r0 : 0.0;
    info->status = status;
    return status;
}

int jc_set_tiles(jc_ctx* c, int tile_x, int tile_y, int z_chunk)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (!tile_shape_ok(tile_x, tile_y, narrow_storage(c)) || z_chunk < 1)
        return fail(JC_ERR_INVALID, "tile_x must be 16, 32, 64, 96, 128 or 256 (above 64 for binary64 storage "
                                    "only), tile_y 4, 8, 16 or 32, tile_x / 2 x tile_y 64 to 1024 threads, and "
                                    "z_chunk >= 1");
    if (items_for(c, tile_x, tile_y, z_chunk) > c->max_items)
        return fail(JC_ERR_INVALID, "z_chunk too small for the work-list region");
    c->tile_x = tile_x;
    c->tile_y = tile_y;
    c->z_chunk = z_chunk;
    c->pace = 0;                           // a pace belongs to a shape
    build_items(c);
    c->hranges[1] = (int32_t)c->items.size();
    free_graphs(c);                        // graphs hold the old launch shapes
    if (c->bound) {
        JC_HIP(hipMemcpyAsync(c->d_items(), c->items.data(), sizeof(Item) * c->items.size(), hipMemcpyHostToDevice,
                              c->stream));
        JC_HIP(hipMemcpyAsync(c->d_ranges(), c->hranges, sizeof(c->hranges), hipMemcpyHostToDevice, c->stream));
        JC_HIP(hipStreamSynchronize(c->stream));
    }
    return JC_OK;
}

int jc_set_temporal_tiles(jc_ctx* c, int rows, int z_chunk)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (!c->opt.temporal)
        return fail(JC_ERR_STATE, "the context was created without temporal blocking");
    if (c->depth() == 3 ? !jc_rt::three_step_rows_ok(rows) : !jc_rt::two_step_rows_ok(rows))
        return fail(JC_ERR_INVALID, c->depth() == 3 ? "rows must be 8 or 16 (three sweeps per launch)"
                                                    : "rows must be 8, 16 or 24");
    if (z_chunk < 1)
        return fail(JC_ERR_INVALID, "z_chunk must be >= 1");
    c->t2_rows = rows;
    c->t2_zc = z_chunk;
    c->pace = 0;                           // a pace belongs to a shape
    free_graphs(c);                        // graphs hold the old launch shapes
    return JC_OK;
}

int jc_temporal_info(const jc_ctx* c, int64_t out[3])
{
    if (!c || !out)
        return fail(JC_ERR_INVALID, "NULL argument");
    out[0] = c->opt.temporal ? c->depth() : 0;
    out[1] = c->t2_rows;
    out[2] = two_step_chunk(c);
    return JC_OK;
}

int jc_set_pace(jc_ctx* c, int64_t ticks)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (ticks < 0 || ticks > kMaxPace)
        return fail(JC_ERR_INVALID, "pace must be in 0 .. " + std::to_string(kMaxPace) + " ticks");
    if ((uint32_t)ticks != c->pace) {
        c->pace = (uint32_t)ticks;
        free_graphs(c);                    // graphs hold the launch arguments
    }
    return JC_OK;
}

int64_t jc_get_pace(const jc_ctx* c) { return c ? (int64_t)c->pace : 0; }

namespace {

// Tune the pace of the context's solve-loop sweep for its current tile
// shape (see pace_wait in jc_kernels.hip).  A pace only helps a launch
// whose work-groups all run at once, or in two rounds: it holds the fast
// ones to a common rate so that none is left running alone at the end.
// The candidates are fractions of the plane-step time of the unpaced
// launch (its time over the planes one work-group marches); each is timed
// over `reps` sweeps in three interleaved rounds after `warm_ms` of
// warm-up, and the fastest is kept, pace 0 included.
// out = {pace, microseconds per sweep with it, without it}.
int tune_pace(jc_ctx* c, int reps, double warm_ms, int64_t out[3])
{
    const bool fused = c->opt.mode == JC_MODE_FUSED && c->np() > 0;
    const bool ir = c->opt.ir_enable != 0;
    int dev = 0, ncu = 0;
    JC_HIP(hipGetDevice(&dev));
    JC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t zmax = 0;
    for (const Item& it : c->items)
        zmax = std::max<int64_t>(zmax, it.zlen);
    int64_t nit = (int64_t)c->items.size();
    const int depth = c->depth();
    if (depth > 1) {
        // the multi-sweep launch of a one-block temporal context
        const HostBlock& b = c->blocks[0];
        const int zc = two_step_chunk(c);
        zmax = zc;
        nit = ((b.n[0] + 63) / 64) * ((b.n[1] + c->t2_rows - 1) / c->t2_rows) * ((b.n[2] + zc - 1) / zc);
    }
    const int64_t rounds = ncu > 0 ? (nit + ncu - 1) / ncu : 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    JC_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(JC_ERR_DEVICE, "pace tuning: hipEventCreate failed");
    }
    const bool was_timing = c->timing;
    c->timing = false;
    // trial sweeps read copy `parity` (copy 1 of the zeroed correction)
    // and write the other copy and face slot: the iterate is unchanged
    auto time_at = [&](uint32_t pace, int n, double& ms) -> int {
        auto one = [&]() -> hipError_t {
            const int zc = two_step_chunk(c);
            if (depth == 3)
                return ir ? launch_ir_three_step(c, 1, c->t2_rows, zc, pace) : launch_three_step(c, c->t2_rows, zc, pace);
            if (depth == 2)
                return ir ? launch_ir_two_step(c, 1, c->t2_rows, zc, pace) : launch_two_step(c, c->t2_rows, zc, pace);
            return ir ? jc::launch_ir_inner(c->d_blocks(), c->d_items(), (int)nit, 1, c->tile_x, c->tile_y,
                                            c->opt.ir_dtype, c->stream, pace)
                      : jc::launch_sweep(c->d_blocks(), c->d_items(), (int)nit, c->parity, c->tile_x, c->tile_y,
                                         fused, false, true, c->opt.with_source != 0, nullptr, c->stream, pace);
        };
        if (one() != hipSuccess || hipEventRecord(e0, c->stream) != hipSuccess)
            return fail(JC_ERR_DEVICE, "pace tuning launch failed");
        for (int i = 0; i < n; ++i)
            if (one() != hipSuccess)
                return fail(JC_ERR_DEVICE, "pace tuning launch failed");
        float tm = 0;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&tm, e0, e1) != hipSuccess)
            return fail(JC_ERR_DEVICE, "pace tuning: timing failed");
        ms = tm;
        return JC_OK;
    };
    int st = JC_OK;
    double warm = 0;
    for (int b = 0; b < 1000 && warm < warm_ms && st == JC_OK; ++b) {
        double ms = 0;
        st = time_at(0, 8, ms);
        warm += ms;
    }
    double base = 0;
    if (st == JC_OK)
        st = time_at(0, reps, base);
    std::vector<uint32_t> cand{0};
    if (st == JC_OK && rounds <= 2 && zmax >= 16) {
        const double step_ticks = base / reps * 1e5 / (double)(rounds * zmax);   // 100 ticks per microsecond
        for (double f : {0.90, 0.91, 0.92, 0.93, 0.94, 0.95, 0.96, 0.97, 0.98}) {
            const double p = step_ticks * f;
            if (p >= 1.0 && p <= (double)kMaxPace && (uint32_t)p != cand.back())
                cand.push_back((uint32_t)p);
        }
    }
    std::vector<double> tot(cand.size(), 0.0);
    for (int r = 0; r < 3 && st == JC_OK && cand.size() > 1; ++r)
        for (size_t i = 0; i < cand.size() && st == JC_OK; ++i) {
            double ms = 0;
            st = time_at(cand[i], reps, ms);
            tot[i] += ms;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = was_timing;
    if (st != JC_OK)
        return st;
    size_t best = 0;
    if (cand.size() > 1) {
        for (size_t i = 1; i < cand.size(); ++i)
            if (tot[i] < tot[best])
                best = i;
        base = tot[0] / 3.0;
    }
    st = jc_set_pace(c, cand[best]);
    if (st != JC_OK)
        return st;
    out[0] = cand[best];
    out[1] = (int64_t)((cand.size() > 1 ? tot[best] / 3.0 : base) * 1000.0 / reps);
    out[2] = (int64_t)(base * 1000.0 / reps);
    return JC_OK;
}

// Common preconditions of the tuners: a loaded context whose trial sweeps
// leave the iterate as it is.
int prepare_tuning(jc_ctx* c)
{
    const bool fused = c->opt.mode == JC_MODE_FUSED && c->np() > 0;
    const bool ir = c->opt.ir_enable != 0;
    if (ir && c->ir_phase != 0)
        return fail(JC_ERR_STATE, "autotune: a group's refinement step is in progress on this context "
                                  "(its r_lo or correction is still to be used)");
    if (ir) {
        // every refinement step rebuilds d from r_lo and no sweep writes a
        // ghost, so trial sweeps on zeroed arrays leave no trace in a solve
        return jc::launch_zero(c->arena + c->lo_begin, c->lo_end - c->lo_begin, c->stream) == hipSuccess
                   ? JC_OK
                   : fail(JC_ERR_DEVICE, "autotune: zeroing the refinement arrays failed");
    }
    if (fused && !c->fused_primed) {
        const int st = do_pack(c, c->parity);
        if (st != JC_OK)
            return st;
        c->fused_primed = true;
    }
    return JC_OK;
}

}  // namespace

int jc_autotune_pace(jc_ctx* c, int reps, int64_t out[3])
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (reps < 1 || !out)
        return fail(JC_ERR_INVALID, "reps must be >= 1 and out not NULL");
    st = prepare_tuning(c);
    if (st != JC_OK)
        return st;
    return tune_pace(c, reps, 150.0, out);
}

int jc_autotune(jc_ctx* c, int reps, int64_t out[4])
{
    int st = check_ready(c);
    if (st != JC_OK)
        return st;
    if (reps < 1 || !out)
        return fail(JC_ERR_INVALID, "reps must be >= 1 and out not NULL");
    const bool fused = c->opt.mode == JC_MODE_FUSED && c->np() > 0;
    // a context with refinement buffers is tuned for the sweep its solve
    // loop runs: the inner sweep of the correction
    const bool ir = c->opt.ir_enable != 0;
    if (ir && c->ir_phase != 0)
        return fail(JC_ERR_STATE, "autotune: a group's refinement step is in progress on this context "
                                  "(its r_lo or correction is still to be used)");
    if (ir) {
        // every refinement step rebuilds d from r_lo and no sweep writes a
        // ghost, so trial sweeps on zeroed arrays leave no trace in a solve
        st = jc::launch_zero(c->arena + c->lo_begin, c->lo_end - c->lo_begin, c->stream) == hipSuccess
                 ? JC_OK
                 : fail(JC_ERR_DEVICE, "autotune: zeroing the refinement arrays failed");
        if (st != JC_OK)
            return st;
    } else if (fused && !c->fused_primed) {
        st = do_pack(c, c->parity);
        if (st != JC_OK)
            return st;
        c->fused_primed = true;
    }
    int64_t maxz = 1;
    for (const HostBlock& b : c->blocks)
        maxz = std::max(maxz, b.n[2]);
    std::vector<int> zcs;
    for (int z = kMinZChunk; z < maxz; z *= 2)
        zcs.push_back(z);
    zcs.push_back((int)maxz);
    struct Shape {
        int x, y, z;
        double ms;
    };
    std::vector<Shape> cand;
    int64_t cells = 0;
    for (const HostBlock& b : c->blocks)
        cells += b.n[0] * b.n[1] * b.n[2];
    for (int xw : kTileXCandidates) {
        // a tile wider than 64 cells is a candidate where it leaves at most
        // 1/8 of its lanes idle (rows that fill it)
        if (xw > kNarrowTileMax && idle_cells(c, xw) * 8 > cells)
            continue;
        for (int t : kTileYCandidates)
            for (int z : zcs)
                if (tile_shape_ok(xw, t, narrow_storage(c)) && items_for(c, xw, t, z) <= c->max_items)
                    cand.push_back({xw, t, z, 0.0});
    }
    if (cand.empty())
        return fail(JC_ERR_INVALID, "no tile shape fits the work-list region");

    hipEvent_t e0 = nullptr, e1 = nullptr;
    JC_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(JC_ERR_DEVICE, "autotune: hipEventCreate failed");
    }
    const bool was_timing = c->timing;
    c->timing = false;
    // trial sweeps read copy `parity` and write the other copy (and face
    // slot parity ^ 1) without swapping: the iterate is unchanged
    auto sweeps = [&](int n) -> int {
        for (int i = 0; i < n; ++i) {
            const hipError_t e =
                ir ? jc::launch_ir_inner(c->d_blocks(), c->d_items(), (int)c->items.size(), 1, c->tile_x,
                                         c->tile_y, c->opt.ir_dtype, c->stream)
                   : jc::launch_sweep(c->d_blocks(), c->d_items(), (int)c->items.size(), c->parity, c->tile_x,
                                      c->tile_y, fused, false, true, c->opt.with_source != 0, nullptr, c->stream);
            if (e != hipSuccess)
                return fail(JC_ERR_DEVICE, std::string("autotune launch: ") + hipGetErrorString(e));
        }
        return JC_OK;
    };
    // milliseconds of `n` sweeps of shape s after one untimed sweep
    auto time_shape = [&](Shape& s, int n, double& ms) -> int {
        int r = jc_set_tiles(c, s.x, s.y, s.z);
        if (r == JC_OK)
            r = sweeps(1);
        if (r == JC_OK && hipEventRecord(e0, c->stream) != hipSuccess)
            r = fail(JC_ERR_DEVICE, "autotune event record failed");
        if (r == JC_OK)
            r = sweeps(n);
        float t = 0;
        if (r == JC_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            r = fail(JC_ERR_DEVICE, "autotune timing failed");
        ms = t;
        return r;
    };
    // The device needs on the order of 100 ms of sustained sweeps before
    // their time settles (a cold start reads up to 8 % slow), so sweeps run
    // for at least 150 ms first.  Every shape is then screened with `reps`
    // sweeps, and the four fastest are timed again in turn over three
    // rounds, so that drift during the search does not pick the winner.
    double warm_total = 0;
    for (int batch = 0; batch < 1000 && warm_total < 150.0 && st == JC_OK; ++batch) {
        double ms = 0;
        st = time_shape(cand[0], 8, ms);
        warm_total += ms;
    }
    for (size_t i = 0; i < cand.size() && st == JC_OK; ++i)
        st = time_shape(cand[i], reps, cand[i].ms);
    if (st == JC_OK) {
        std::stable_sort(cand.begin(), cand.end(), [](const Shape& a, const Shape& b) { return a.ms < b.ms; });
        cand.resize(std::min<size_t>(cand.size(), 4));
        for (Shape& s : cand)
            s.ms = 0;
        for (int round = 0; round < 3 && st == JC_OK; ++round)
            for (size_t i = 0; i < cand.size() && st == JC_OK; ++i) {
                double ms = 0;
                st = time_shape(cand[i], reps, ms);
                cand[i].ms += ms;
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = was_timing;
    if (st != JC_OK)
        return st;
    const Shape best = *std::min_element(cand.begin(), cand.end(),
                                         [](const Shape& a, const Shape& b) { return a.ms < b.ms; });
    st = jc_set_tiles(c, best.x, best.y, best.z);
    int64_t pace_out[3] = {0, 0, 0};
    if (st == JC_OK && !c->opt.temporal)
        st = tune_pace(c, reps, 0.0, pace_out);
    if (st == JC_OK && c->opt.temporal) {
        c->timing = false;
        st = tune_two_step(c, std::max(reps, 2));
        c->timing = was_timing;
        // then the pace of the multi-sweep launch, for the shape just kept
        if (st == JC_OK)
            st = tune_pace(c, std::max(reps, 2), 0.0, pace_out);
        pace_out[0] = 0;                   // out[3] reports the one-sweep launch
    }
    if (st != JC_OK)
        return st;
    out[0] = best.x;
    out[1] = best.y;
    out[2] = best.z;
    out[3] = pace_out[0] ? pace_out[1] : (int64_t)(best.ms * 1000.0 / (3.0 * reps));   // microseconds per sweep
    return JC_OK;
}

int64_t jc_num_blocks(const jc_ctx* c) { return c ? (int64_t)c->blocks.size() : 0; }
int64_t jc_num_pairs(const jc_ctx* c) { return c ? (int64_t)c->pairs.size() : 0; }
int64_t jc_num_items(const jc_ctx* c) { return c ? (int64_t)c->items.size() : 0; }
int64_t jc_iterations(const jc_ctx* c) { return c ? c->iters : 0; }

int jc_block_info(const jc_ctx* c, int64_t i, int64_t out[17])
{
    if (!c || !out || i < 0 || i >= (int64_t)c->blocks.size())
        return fail(JC_ERR_INVALID, "bad context or block index");
    const HostBlock& b = c->blocks[i];
    for (int a = 0; a < 3; ++a) {
        out[a] = b.n[a];
        out[3 + a] = b.off[a];
    }
    for (int f = 0; f < 6; ++f)
        out[6 + f] = b.nbr[f];
    out[12] = b.pitch;
    out[13] = b.plane;
    const int64_t lead = (jc::line_elems<double>() - 1) * (int64_t)sizeof(double);
    out[14] = (int64_t)b.u_off[0] + lead;
    out[15] = (int64_t)b.u_off[1] + lead;
    out[16] = c->parity;
    return JC_OK;
}

int jc_pair_info(const jc_ctx* c, int64_t i, int64_t out[10])
{
    if (!c || !out || i < 0 || i >= (int64_t)c->pairs.size())
        return fail(JC_ERR_INVALID, "bad context or pair index");
    const HostPair& p = c->pairs[i];
    out[0] = p.src_block; out[1] = p.src_face; out[2] = p.dst_block; out[3] = p.dst_face;
    out[4] = p.count; out[5] = p.slow; out[6] = p.fast; out[7] = (int64_t)p.buf_off[0];
    out[8] = (int64_t)p.buf_off[1]; out[9] = jc::face_ld(p.fast);
    return JC_OK;
}

int jc_tile_info(const jc_ctx* c, int64_t out[4])
{
    if (!c || !out)
        return fail(JC_ERR_INVALID, "bad context or output");
    out[0] = c->tile_x;
    out[1] = c->tile_y;
    out[2] = c->z_chunk;
    out[3] = (int64_t)c->items.size();
    return JC_OK;
}

int jc_set_timing(jc_ctx* c, int enable)
{
    if (!c)
        return fail(JC_ERR_INVALID, "NULL context");
    if (!c->bound)
        return fail(JC_ERR_STATE, "context is not bound (jc_bind)");
    int st = drain_timing(c);
    if (st != JC_OK)
        return st;
    c->timing = enable != 0;
    for (int k = 0; k < JC_K_COUNT; ++k) {
        c->kernel_ms[k] = 0;
        c->kernel_launches[k] = 0;
    }
    return JC_OK;
}

int jc_kernel_time(jc_ctx* c, int kind, double* ms_total, int64_t* launches)
{
    if (!c || kind < 0 || kind >= JC_K_COUNT || !ms_total || !launches)
        return fail(JC_ERR_INVALID, "bad arguments");
    int st = drain_timing(c);
    if (st != JC_OK)
        return st;
    *ms_total = c->kernel_ms[kind];
    *launches = c->kernel_launches[kind];
    return JC_OK;
}

}  // extern "C"
