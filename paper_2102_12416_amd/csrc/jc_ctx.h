// Internal state of a libjc context, shared by the host runtime files
// (jc_host.cpp: one context; jc_group.cpp: several contexts per launch).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "jc.h"
#include "jc_kernels.h"
#include "jc_types.h"

using jc::BlockDesc;
using jc::Item;
using jc::PairDesc;

namespace jc_rt {

// Record msg as this thread's last error and return code.
int fail(int code, const std::string& msg);

#define JC_HIP(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(JC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kMaxEdge = (int64_t)1 << 30;    // per-axis limit (int32 cell indices)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

enum GhostState { GHOST_CURRENT = 0, GHOST_PACKED = 1, GHOST_EXCHANGED = 2, GHOST_STALE = 3 };

struct HostBlock {
    int64_t n[3];
    int64_t off[3];
    int nbr[6];
    int pair_out[6];        // pair index whose source is this face, or -1
    int pair_in[6];         // pair index whose destination is this face, or -1
    int64_t pitch, plane;   // binary64 arrays
    size_t u_off[2], b_off; // byte offsets of element (0,0,0)'s line base
    int64_t lpitch, lplane; // refinement arrays (d, r_lo)
    size_t d_off[2], rlo_off;
    size_t xg_off[2];       // compact Dirichlet ghost column of face XM / XP (unpaired faces)
};

struct HostPair {
    int src_block, src_face, dst_block, dst_face;
    int64_t slow, fast, count, span;
    size_t buf_off[2];
    size_t lbuf_off[2];     // refinement face buffers
};

// A block of depth nz is cut into ceil(nz / zc) z chunks of nearly equal
// length (no short tail chunk): chunk k covers planes [z0, z0 + len).
inline void z_chunk_range(int64_t nz, int64_t zc, int64_t k, int64_t* z0, int64_t* len)
{
    const int64_t nch = (nz + zc - 1) / zc;
    *z0 = k * nz / nch;
    *len = (k + 1) * nz / nch - *z0;
}

// Bytes of one element of the refinement storage format.
inline size_t lo_size(int dtype) { return dtype == JC_F64 ? 8 : dtype == JC_F32 ? 4 : 2; }

constexpr int kTileXCandidates[] = {64, 32, 16, 96, 128, 256};
constexpr int kTileYCandidates[] = {4, 8, 16, 32};
constexpr int kNarrowTileMax = 64;

// A tile is 16, 32, 64, 96, 128 or 256 cells wide (two per thread) and
// 4..32 rows; a work-group is whole 64-lane waves and at most 1024 threads
// (a 16-cell tile needs 8 rows, a 256-cell tile at most 8).  Tiles wider
// than 64 cells sweep binary64 storage only: `narrow` is set when the
// swept storage is binary32 or bfloat16 (the refinement's correction).
inline bool tile_shape_ok(int tile_x, int tile_y, bool narrow = false)
{
    bool ok_x = false, ok_y = false;
    for (int x : kTileXCandidates)
        ok_x = ok_x || x == tile_x;
    for (int y : kTileYCandidates)
        ok_y = ok_y || y == tile_y;
    const int threads = (tile_x / 2) * tile_y;
    return ok_x && ok_y && threads >= 64 && threads <= 1024 && (!narrow || tile_x <= kNarrowTileMax);
}
constexpr int kMinZChunk = 16;
// largest pace (ticks of the 100 MHz clock per plane step): each wait of a
// work-group is bounded by 4096 sleeps of 64 cycles, about 100 us
constexpr int64_t kMaxPace = 10000;
// Temporal blocking: default rows of the two-sweep tile (64 cells wide;
// 8, 16 or 24) and the fewest planes per work-group when the chunk follows
// the one-sweep z_chunk (each work-group reads two planes beyond each end).
constexpr int kTwoStepRows = 16;
constexpr int kTwoStepMinZ = 32;
constexpr int kTwoStepFloorZ = 8;
constexpr int64_t kTwoStepMinGroups = 1024;
constexpr int kTwoStepRowCandidates[] = {8, 16, 24};
constexpr int kThreeStepRowCandidates[] = {8, 16};
inline bool two_step_rows_ok(int rows)
{
    bool ok = false;
    for (int r : kTwoStepRowCandidates)
        ok = ok || r == rows;
    return ok;
}
inline bool three_step_rows_ok(int rows) { return rows == 8 || rows == 16; }

}  // namespace jc_rt

using jc_rt::GHOST_CURRENT;
using jc_rt::GHOST_EXCHANGED;
using jc_rt::GHOST_PACKED;
using jc_rt::GHOST_STALE;
using jc_rt::HostBlock;
using jc_rt::HostPair;

struct jc_ctx {
    int64_t grid[3] = {0, 0, 0};
    std::vector<int64_t> cuts[3];
    jc_options opt{};
    std::vector<HostBlock> blocks;
    std::vector<HostPair> pairs;
    int64_t max_slow = 0, max_fast = 0, max_count = 0;
    int tile_x = 64;
    int tile_y = 8;
    int z_chunk = 0;
    // temporal blocking: rows and planes of the two-sweep work-group
    // (t2_zc 0: the one-sweep z_chunk, at least kTwoStepMinZ)
    int t2_rows = jc_rt::kTwoStepRows;
    int t2_zc = 0;
    // pace of the one-sweep launches of the solve loop (jc_set_pace): ticks
    // of the 100 MHz constant clock per plane step; 0 = none
    uint32_t pace = 0;
    // |r_0| of the current solve as first seen by jc_group_check (-1: none
    // yet); reset by jc_load_field(U)
    double check_r0 = -1.0;
    // sweeps per launch of the solve loop: 1, or 2 / 3 with temporal blocking
    int depth() const { return !opt.temporal ? 1 : opt.sweeps_per_launch == 3 ? 3 : 2; }
    // boundary-first iterations (options.overlap): the work list holds the
    // n_bnd tiles with a paired face plane first; the halo of the new
    // iterate moves on `side` between ev_fork and ev_join
    int64_t n_bnd = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<Item> items;
    int64_t max_items = 0;
    // arena layout
    size_t off_blocks = 0, off_pairs = 0, off_items = 0, off_partials = 0, off_ranges = 0,
           off_result = 0, footprint = 0;
    size_t lo_begin = 0, lo_end = 0;   // refinement arrays and buffers
    size_t lxg_off = 0;                 // zero ghost column of the correction (in the refinement region)
    // binding
    char* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    std::vector<BlockDesc> hdesc;
    std::vector<PairDesc> hpairs;
    int32_t hranges[2] = {0, 0};
    double* h_result = nullptr;     // pinned
    // host-staged exchange: pinned send and receive halves, per-pair offsets
    char* h_stage = nullptr;
    size_t h_stage_bytes = 0;
    std::vector<size_t> h_stage_off;
    // metadata messages of the announced exchange
    struct MetaMsg { int src, dst; size_t bytes; uint64_t tag; };
    std::vector<MetaMsg> meta;
    // state
    bool loaded_u = false, loaded_b = false;
    int parity = 0;
    int64_t iters = 0;
    int ghost = GHOST_CURRENT;
    bool fused_primed = false;
    // refinement state used by groups: d arrays zeroed, phase
    // (0: residual due, 1: r_lo current, 2: inner sweeps ran since the
    // last residual), copy q holding the latest correction
    bool ir_zeroed = false;
    int ir_phase = 0;
    int ir_q = 0;
    // graphs keyed by (iterations, start parity, residual-last)
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
    // timing
    bool timing = false;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    double kernel_ms[JC_K_COUNT] = {0};
    int64_t kernel_launches[JC_K_COUNT] = {0};

    BlockDesc* d_blocks() const { return reinterpret_cast<BlockDesc*>(arena + off_blocks); }
    PairDesc* d_pairs() const { return reinterpret_cast<PairDesc*>(arena + off_pairs); }
    Item* d_items() const { return reinterpret_cast<Item*>(arena + off_items); }
    double* d_partials() const { return reinterpret_cast<double*>(arena + off_partials); }
    int32_t* d_ranges() const { return reinterpret_cast<int32_t*>(arena + off_ranges); }
    double* d_result() const { return reinterpret_cast<double*>(arena + off_result); }
    int nb() const { return (int)blocks.size(); }
    int64_t max_rows() const
    {
        int64_t m = 1;
        for (const HostBlock& b : blocks)
            m = b.n[1] * b.n[2] > m ? b.n[1] * b.n[2] : m;
        return m;
    }
    int np() const { return (int)pairs.size(); }
};


namespace jc_rt {

// The context sweeps binary32 or bfloat16 storage (the refinement's
// correction): its tiles are at most 64 cells wide.
inline bool narrow_storage(const jc_ctx* c) { return c->opt.ir_enable && c->opt.ir_dtype != JC_F64; }

hipEvent_t take_event(jc_ctx* c);
int drain_timing(jc_ctx* c);
int check_ready(jc_ctx* c);
int do_pack(jc_ctx* c, int slot);

// Runs `launch` on the context's stream, bracketed by timing events of
// kind `kind` when timing is on.
template <typename F>
int timed(jc_ctx* c, int kind, F&& launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        a = take_event(c);
        b = take_event(c);
        if (!a || !b)
            return fail(JC_ERR_DEVICE, "hipEventCreate failed");
        JC_HIP(hipEventRecord(a, c->stream));
    }
    hipError_t e = launch();
    if (e != hipSuccess)
        return fail(JC_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    if (c->timing) {
        JC_HIP(hipEventRecord(b, c->stream));
        c->pending.push_back({kind, a, b});
    }
    return JC_OK;
}

}  // namespace jc_rt
