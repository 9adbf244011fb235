// Groups: the blocks of several independent contexts swept by shared
// launches (batching many grids, continuous batching of a solve server).
//
// A group owns a joint block table and joint work lists, one list per
// kernel class (plain binary64 with or without a source; refinement by
// storage format and source).  Every launch covers all members of a
// class; each work item carries its member's ping-pong flip, so members
// admitted at different times stay independent.  The tile shape is fixed
// for a group (it never depends on who else is in it), so a member's
// results and residual norms are bitwise the same alone and in any mix.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "jc_ctx.h"

using namespace jc_rt;

namespace {

// Default tile shape of a group; a group's shape is fixed at creation.
constexpr int kGroupTile[3] = {64, 8, 32};

struct Class {
    bool ir = false;     // refinement members
    bool src = false;    // members with a source
    int lo = JC_F64;     // refinement storage
    int bstart = 0, bend = 0;        // joint block range
    int64_t max_rows = 1;            // largest ny * nz of the class's blocks
    size_t item0 = 0;                // first joint item
    std::vector<Item> items;
    size_t item2_0 = 0;              // first joint two-sweep item
    std::vector<Item> items2;        // two-sweep tiles (groups that sweep twice per launch)
    std::vector<int> members;
    // resident sweeps: one item per member, split by launch variant (the
    // kernel's step schedule depends on the parity of (nz + 1) / 2)
    std::vector<Item> itemsr[jc::kResidentVariants];
    size_t itemr0[jc::kResidentVariants] = {};       // first joint resident item of each split
    int max_pairs[jc::kResidentVariants] = {}, max_nz[jc::kResidentVariants] = {};
    int64_t lds[jc::kResidentVariants] = {};
};

// Two-sweep tiles of a group: 64 cells by kGroupTwoStepRows rows, and at
// least kTwoStepMinZ planes (the group's own z chunk if larger).
constexpr int kGroupTwoStepRows = 16;

}  // namespace

struct jc_group {
    std::vector<jc_ctx*> members;
    hipStream_t stream = nullptr;
    bool use_graphs = false;
    int tile[3] = {kGroupTile[0], kGroupTile[1], kGroupTile[2]};
    std::vector<Class> classes;
    std::vector<BlockDesc> desc;        // joint block table, class-major
    std::vector<Item> items;            // joint work list, class-major
    std::vector<Item> items2;           // joint two-sweep work list, class-major
    bool two_step = false;              // every launch sweeps every member twice (or three times)
    bool three_step = false;            // three sweeps of every member per launch
    bool resident = false;              // every window one launch, one work-group per member
    std::vector<Item> itemsr;           // joint resident items, class-major
    std::vector<int32_t> lohi;          // per member: joint item range
    std::vector<int> member_bstart;     // per member: first joint block
    size_t off_desc = 0, off_items = 0, off_items2 = 0, off_itemsr = 0, off_partials = 0, off_lohi = 0, off_out = 0,
           footprint = 0;
    char* scratch = nullptr;
    bool bound = false;
    double* h_out = nullptr;            // pinned, one per member (or h_out_plain)
    std::vector<double> h_out_plain;    // pageable, one per member: the static-scratch binding
    int static_dev = -1;                // device whose static scratch the group holds (-1: none)
    int parity = 0;                     // launch parity; items hold member flips
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
    std::vector<hipEvent_t> events;

    BlockDesc* d_desc() const { return reinterpret_cast<BlockDesc*>(scratch + off_desc); }
    Item* d_items() const { return reinterpret_cast<Item*>(scratch + off_items); }
    Item* d_items2() const { return reinterpret_cast<Item*>(scratch + off_items2); }
    Item* d_itemsr() const { return reinterpret_cast<Item*>(scratch + off_itemsr); }
    double* d_partials() const { return reinterpret_cast<double*>(scratch + off_partials); }
    int32_t* d_lohi() const { return reinterpret_cast<int32_t*>(scratch + off_lohi); }
    double* d_out() const { return reinterpret_cast<double*>(scratch + off_out); }
};

namespace {

int ghip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        return fail(JC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return JC_OK;
}

// Items of one member's blocks with the group's tile shape.
void member_items(const jc_ctx* c, const int tile[3], int bbase, int member, std::vector<Item>& out)
{
    for (int bi = 0; bi < (int)c->blocks.size(); ++bi) {
        const HostBlock& b = c->blocks[bi];
        const int64_t nch = (b.n[2] + tile[2] - 1) / tile[2];
        for (int64_t k = 0; k < nch; ++k)
            for (int64_t y0 = 0; y0 < b.n[1]; y0 += tile[1])
                for (int64_t x0 = 0; x0 < b.n[0]; x0 += tile[0]) {
                    int64_t z0 = 0, zlen = 0;
                    z_chunk_range(b.n[2], tile[2], k, &z0, &zlen);
                    Item it{};
                    it.block = bbase + bi;
                    it.x0 = (int32_t)x0;
                    it.y0 = (int32_t)y0;
                    it.z0 = (int32_t)z0;
                    it.zlen = (int32_t)zlen;
                    it.flip = c->parity;
                    it.owner = member;
                    out.push_back(it);
                }
    }
}

// The faces of every member's current iterate into its slot `parity`.
int prime_faces(jc_group* g)
{
    for (jc_ctx* c : g->members) {
        if (c->np() && !c->fused_primed) {
            const hipError_t e = jc::launch_pack(c->d_blocks(), c->d_pairs(), c->np(), (int)c->max_slow,
                                                 (int)c->max_fast, c->parity, c->parity, g->stream);
            if (e != hipSuccess)
                return ghip(e, "pack");
            c->fused_primed = true;
        }
    }
    return JC_OK;
}

// One sweep of every member.
int group_sweep(jc_group* g)
{
    for (const Class& k : g->classes) {
        const int n = (int)k.items.size();
        if (!k.ir) {
            const hipError_t e = jc::launch_sweep(g->d_desc(), g->d_items() + k.item0, n, g->parity, g->tile[0], g->tile[1],
                                                  true, false, true, k.src, nullptr, g->stream);
            if (e != hipSuccess)
                return ghip(e, "group sweep");
        } else {
            // refinement members: the first inner sweep after a residual
            // starts from d = 0; later ones sweep d
            const jc_ctx* c0 = g->members[k.members[0]];
            hipError_t e;
            if (c0->ir_phase == 1)
                e = jc::launch_ir_first(g->d_desc() + k.bstart, k.bend - k.bstart, k.max_rows, k.lo, g->stream);
            else
                e = jc::launch_ir_inner(g->d_desc(), g->d_items() + k.item0, n, c0->ir_q, g->tile[0], g->tile[1], k.lo,
                                        g->stream);
            if (e != hipSuccess)
                return ghip(e, "group inner sweep");
        }
    }
    return JC_OK;
}

// Two sweeps of every member in one launch per class (every member one
// block; refining members past the first inner sweep of their step).
int group_sweep2(jc_group* g)
{
    for (const Class& k : g->classes) {
        hipError_t e;
        if (!k.ir)
            e = jc::launch_sweep2_items(g->d_desc(), g->d_items2() + k.item2_0, (int)k.items2.size(), g->parity,
                                        kGroupTwoStepRows, k.src, g->stream);
        else
            e = jc::launch_ir_inner2_items(g->d_desc(), g->d_items2() + k.item2_0, (int)k.items2.size(),
                                           g->members[k.members[0]]->ir_q, kGroupTwoStepRows, k.lo, g->stream);
        if (e != hipSuccess)
            return ghip(e, "group two-sweep launch");
    }
    return JC_OK;
}

// Three sweeps of every member in one launch per class (the two-sweep
// tiles serve the three-sweep kernel too: 64 cells by 16 rows).
int group_sweep3(jc_group* g)
{
    for (const Class& k : g->classes) {
        hipError_t e;
        if (!k.ir)
            e = jc::launch_sweep3(g->d_desc(), g->d_items2() + k.item2_0, (int)k.items2.size(), 0, 0, 0, g->parity,
                                  kGroupTwoStepRows, 0, k.src, g->stream);
        else
            e = jc::launch_ir_inner3(g->d_desc(), g->d_items2() + k.item2_0, (int)k.items2.size(), 0, 0, 0,
                                     g->members[k.members[0]]->ir_q, kGroupTwoStepRows, 0, k.lo, g->stream);
        if (e != hipSuccess)
            return ghip(e, "group three-sweep launch");
    }
    return JC_OK;
}

// n sweeps of every member in one launch per class and launch variant
// (resident groups).
int group_resident(jc_group* g, int64_t n)
{
    for (const Class& k : g->classes)
        for (int q = 0; q < jc::kResidentVariants; ++q) {
            if (k.itemsr[q].empty())
                continue;
            const hipError_t e = jc::launch_resident(g->d_desc(), g->d_itemsr() + k.itemr0[q], (int)k.itemsr[q].size(),
                                                     k.max_pairs[q], k.max_nz[q], (size_t)k.lds[q], q, g->parity,
                                                     (int)n, k.src, g->stream);
            if (e != hipSuccess)
                return ghip(e, "group resident launch");
        }
    return JC_OK;
}

// Bookkeeping after one multi-sweep launch of `sweeps` sweeps: every
// member advanced that many sweeps and its iterate (a refining member: its
// correction) moved to the other copy once, as the launch parity did.
void advance2(jc_group* g, int sweeps = 2)
{
    g->parity ^= 1;
    for (const Class& k : g->classes)
        for (int m : k.members) {
            jc_ctx* c = g->members[m];
            c->iters += sweeps;
            if (!k.ir) {
                c->parity ^= 1;
                c->ghost = GHOST_CURRENT;
                c->fused_primed = false;
            } else {
                c->ir_q ^= 1;
                c->ir_phase = 2;
            }
        }
}

// Bookkeeping after n sweeps of every member.
void advance(jc_group* g, int64_t n)
{
    if (n <= 0)
        return;
    g->parity ^= (int)(n & 1);
    for (const Class& k : g->classes) {
        for (int m : k.members) {
            jc_ctx* c = g->members[m];
            c->iters += n;
            if (!k.ir) {
                c->parity ^= (int)(n & 1);
                c->ghost = c->np() ? GHOST_STALE : GHOST_CURRENT;
                c->fused_primed = c->np() > 0;
            } else {
                // first sweep writes copy 1; each later one flips it
                const int q = c->ir_phase == 1 ? 1 : c->ir_q;
                const int64_t later = c->ir_phase == 1 ? n - 1 : n;
                c->ir_q = q ^ (int)(later & 1);
                c->ir_phase = 2;
            }
        }
    }
}

// n sweeps of every member as launches: two-sweep launches first when
// the group sweeps twice per launch, then single sweeps.
int group_run(jc_group* g, int64_t n)
{
    int64_t i = 0;
    int st = JC_OK;
    if (g->resident) {
        for (; i < n && st == JC_OK;) {
            const int64_t m = std::min<int64_t>(n - i, (int64_t)1 << 30);
            st = group_resident(g, m);
            if (st == JC_OK)
                advance(g, m);
            i += m;
        }
        return st;
    }
    if (g->three_step)
        for (; i + 3 <= n && st == JC_OK; i += 3) {
            st = group_sweep3(g);
            advance2(g, 3);
        }
    if (g->two_step)
        for (; i + 2 <= n && st == JC_OK; i += 2) {
            st = group_sweep2(g);
            advance2(g);
        }
    for (; i < n && st == JC_OK; ++i) {
        st = group_sweep(g);
        advance(g, 1);
    }
    return st;
}

}  // namespace

extern "C" {

int jc_group_create(jc_ctx* const* ctxs, int n, void* hip_stream, int flags, const int tile[3], jc_group** out)
{
    if (!out)
        return fail(JC_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    if (!ctxs || n < 1)
        return fail(JC_ERR_INVALID, "a group needs at least one context");
    if (flags & ~15)
        return fail(JC_ERR_INVALID, "unknown group flags");
    if ((flags & 8) && (flags & 6))
        return fail(JC_ERR_INVALID, "resident sweeps (flag 8) exclude flags 2 and 4");
    std::set<const jc_ctx*> seen;
    for (int i = 0; i < n; ++i) {
        jc_ctx* c = ctxs[i];
        int st = check_ready(c);
        if (st != JC_OK)
            return st;
        if (!seen.insert(c).second)
            return fail(JC_ERR_INVALID, "a context appears twice in the group");
        if (c->opt.ir_enable && c->parity != 0)
            return fail(JC_ERR_STATE, "a refining member must hold its iterate in copy 0");
        if ((flags & 6) && c->nb() != 1)
            return fail(JC_ERR_INVALID, "two or three sweeps per launch (flag 2 or 4) needs members of one block");
        if ((flags & 8) && (c->opt.ir_enable || c->nb() != 1 ||
                            !jc::resident_fits(c->blocks[0].n[0], c->blocks[0].n[1], c->blocks[0].n[2])))
            return fail(JC_ERR_INVALID, "resident sweeps (flag 8) need members of one block of at most 32 planes "
                                        "with (nx + 1) / 2 * ny <= 512 cell pairs and an LDS need within 64 KiB, "
                                        "without refinement");
    }
    if (tile) {
        bool narrow = false;
        for (int i = 0; i < n; ++i)
            narrow = narrow || jc_rt::narrow_storage(ctxs[i]);
        const bool ok = jc_rt::tile_shape_ok(tile[0], tile[1], narrow) && tile[2] >= 1;
        if (!ok)
            return fail(JC_ERR_INVALID, "group tile must be {16|32|64|96|128|256 (above 64 only without binary32 "
                                        "or bfloat16 members), 4|8|16|32, >= 1} with 64 to 1024 threads");
    }
    jc_group* g = new (std::nothrow) jc_group();
    if (!g)
        return fail(JC_ERR_NOMEM, "host allocation failed");
    if (tile)
        for (int a = 0; a < 3; ++a)
            g->tile[a] = tile[a];
    g->members.assign(ctxs, ctxs + n);
    g->stream = static_cast<hipStream_t>(hip_stream);
    g->use_graphs = (flags & 1) && g->stream != nullptr;
    g->two_step = (flags & 6) != 0;
    g->three_step = (flags & 4) != 0;
    g->resident = (flags & 8) != 0;
    // classes, in a fixed order
    std::map<std::tuple<int, int, int>, int> cls;
    for (int i = 0; i < n; ++i) {
        const jc_ctx* c = ctxs[i];
        const auto key = std::make_tuple(c->opt.ir_enable ? 1 : 0, c->opt.with_source ? 1 : 0,
                                         c->opt.ir_enable ? c->opt.ir_dtype : JC_F64);
        auto it = cls.find(key);
        if (it == cls.end()) {
            Class k;
            k.ir = std::get<0>(key) != 0;
            k.src = std::get<1>(key) != 0;
            k.lo = std::get<2>(key);
            it = cls.emplace(key, 0).first;
            g->classes.push_back(k);
            it->second = (int)g->classes.size() - 1;
        }
        g->classes[it->second].members.push_back(i);
    }
    g->member_bstart.assign(n, 0);
    g->lohi.assign(2 * n, 0);
    for (Class& k : g->classes) {
        k.bstart = (int)g->desc.size();
        k.item0 = g->items.size();
        for (int m : k.members) {
            const jc_ctx* c = ctxs[m];
            g->member_bstart[m] = (int)g->desc.size();
            k.max_rows = std::max(k.max_rows, c->max_rows());
            const size_t i0 = g->items.size();
            const size_t first = k.items.size();
            member_items(c, g->tile, (int)g->desc.size(), m, k.items);
            if (g->two_step) {
                const int t2[3] = {64, kGroupTwoStepRows, std::max(g->tile[2], jc_rt::kTwoStepMinZ)};
                member_items(c, t2, (int)g->desc.size(), m, k.items2);
            }
            if (g->resident) {
                const int64_t* bn = c->blocks[0].n;
                const int q = jc::resident_variant(bn[2]);
                Item it{};
                it.block = (int32_t)g->desc.size();
                it.zlen = (int32_t)bn[2];
                it.flip = c->parity;
                it.owner = m;
                k.itemsr[q].push_back(it);
                k.max_pairs[q] = std::max<int>(k.max_pairs[q], (int)((bn[0] + 1) / 2 * bn[1]));
                k.max_nz[q] = std::max<int>(k.max_nz[q], (int)bn[2]);
                k.lds[q] = std::max(k.lds[q], jc::resident_lds_bytes(bn[0], bn[1], bn[2]));
            }
            g->desc.insert(g->desc.end(), c->hdesc.begin(), c->hdesc.end());
            g->items.insert(g->items.end(), k.items.begin() + first, k.items.end());
            g->lohi[2 * m] = (int32_t)i0;
            g->lohi[2 * m + 1] = (int32_t)g->items.size();
        }
        k.bend = (int)g->desc.size();
        k.item2_0 = g->items2.size();
        g->items2.insert(g->items2.end(), k.items2.begin(), k.items2.end());
        for (int q = 0; q < jc::kResidentVariants; ++q) {
            k.itemr0[q] = g->itemsr.size();
            g->itemsr.insert(g->itemsr.end(), k.itemsr[q].begin(), k.itemsr[q].end());
        }
    }
    if (g->desc.size() > 65535 || g->items.size() > ((size_t)1 << 30) || g->items2.size() > ((size_t)1 << 30)) {
        delete g;
        return fail(JC_ERR_INVALID, "group too large for one launch");
    }
    size_t off = 0;
    g->off_desc = off; off = align_up(off + sizeof(BlockDesc) * g->desc.size(), kAlign);
    g->off_items = off; off = align_up(off + sizeof(Item) * g->items.size(), kAlign);
    g->off_items2 = off; off = align_up(off + sizeof(Item) * std::max<size_t>(1, g->items2.size()), kAlign);
    g->off_itemsr = off; off = align_up(off + sizeof(Item) * std::max<size_t>(1, g->itemsr.size()), kAlign);
    g->off_partials = off; off = align_up(off + sizeof(double) * g->items.size(), kAlign);
    g->off_lohi = off; off = align_up(off + sizeof(int32_t) * g->lohi.size(), kAlign);
    g->off_out = off; off = align_up(off + sizeof(double) * n, kAlign);
    g->footprint = off;
    g->h_out_plain.assign(n, 0.0);
    *out = g;
    return JC_OK;
}

int jc_group_footprint(const jc_group* g, size_t* bytes)
{
    if (!g || !bytes)
        return fail(JC_ERR_INVALID, "bad group or output");
    *bytes = g->footprint;
    return JC_OK;
}

namespace {

// Attach scratch and upload the tables.  plain: the allocation-free
// binding -- residuals come back through the group's pageable host buffer
// and the group stream is ordered after the members' streams by waiting
// for those streams on the host, so no pinned memory or event is created.
int bind_common(jc_group* g, char* scratch, bool plain)
{
    g->scratch = scratch;
    int st = JC_OK;
    if (plain) {
        g->h_out = g->h_out_plain.data();
        for (jc_ctx* c : g->members)
            if (c->stream != g->stream && st == JC_OK)
                st = ghip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        // the static scratch keeps the last group's contents: clear the
        // range this group uses before its tables go in
        if (st == JC_OK)
            st = ghip(jc::launch_zero(scratch, g->footprint, g->stream), "clear scratch");
    } else {
        st = ghip(hipHostMalloc(reinterpret_cast<void**>(&g->h_out), sizeof(double) * g->members.size(),
                                hipHostMallocDefault), "hipHostMalloc");
        // order the group stream after every member's queued work
        for (jc_ctx* c : g->members) {
            if (c->stream == g->stream || st != JC_OK)
                continue;
            hipEvent_t e = nullptr;
            st = ghip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
            if (st != JC_OK)
                break;
            g->events.push_back(e);
            st = ghip(hipEventRecord(e, c->stream), "hipEventRecord");
            if (st == JC_OK)
                st = ghip(hipStreamWaitEvent(g->stream, e, 0), "hipStreamWaitEvent");
        }
    }
    if (st != JC_OK)
        return st;
    st = ghip(hipMemcpyAsync(g->d_desc(), g->desc.data(), sizeof(BlockDesc) * g->desc.size(),
                             hipMemcpyHostToDevice, g->stream), "upload blocks");
    if (st == JC_OK)
        st = ghip(hipMemcpyAsync(g->d_items(), g->items.data(), sizeof(Item) * g->items.size(),
                                 hipMemcpyHostToDevice, g->stream), "upload items");
    if (st == JC_OK && !g->items2.empty())
        st = ghip(hipMemcpyAsync(g->d_items2(), g->items2.data(), sizeof(Item) * g->items2.size(),
                                 hipMemcpyHostToDevice, g->stream), "upload two-sweep items");
    if (st == JC_OK && !g->itemsr.empty())
        st = ghip(hipMemcpyAsync(g->d_itemsr(), g->itemsr.data(), sizeof(Item) * g->itemsr.size(),
                                 hipMemcpyHostToDevice, g->stream), "upload resident items");
    if (st == JC_OK)
        st = ghip(hipMemcpyAsync(g->d_lohi(), g->lohi.data(), sizeof(int32_t) * g->lohi.size(),
                                 hipMemcpyHostToDevice, g->stream), "upload ranges");
    if (st == JC_OK)
        st = ghip(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    if (st != JC_OK)
        return st;
    g->bound = true;
    return JC_OK;
}

// ---- the library's static group scratch (jc_group_bind_static) ----------
//
// One array per device, in this file: in host code its name stands for a
// host-side symbol, so every use goes through the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept in static_base.  A bound group holds its device's array
// until jc_group_destroy (static_owner).
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[JC_STATIC_SCRATCH_BYTES];
std::mutex static_mu;
char* static_base[kMaxDevices] = {};
const jc_group* static_owner[kMaxDevices] = {};

}  // namespace

int jc_group_bind(jc_group* g, void* dev_scratch, size_t bytes)
{
    if (!g)
        return fail(JC_ERR_INVALID, "NULL group");
    if (g->bound)
        return fail(JC_ERR_STATE, "group is already bound");
    if (!dev_scratch || reinterpret_cast<uintptr_t>(dev_scratch) % kAlign)
        return fail(JC_ERR_INVALID, "scratch must be a 256-byte aligned device pointer");
    if (bytes < g->footprint)
        return fail(JC_ERR_NOMEM, "scratch smaller than jc_group_footprint");
    return bind_common(g, static_cast<char*>(dev_scratch), false);
}

int jc_group_bind_static(jc_group* g)
{
    if (!g)
        return fail(JC_ERR_INVALID, "NULL group");
    if (g->bound)
        return fail(JC_ERR_STATE, "group is already bound");
    if (g->footprint > (size_t)JC_STATIC_SCRATCH_BYTES)
        return fail(JC_ERR_NOMEM, "group needs " + std::to_string(g->footprint) +
                                      " bytes of scratch, more than the static scratch (" +
                                      std::to_string((size_t)JC_STATIC_SCRATCH_BYTES) + " bytes)");
    int dev = -1;
    int st = ghip(hipGetDevice(&dev), "hipGetDevice");
    if (st != JC_OK)
        return st;
    if (dev < 0 || dev >= kMaxDevices)
        return fail(JC_ERR_DEVICE, "device index out of range for the static scratch");
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(static_mu);
        if (static_owner[dev])
            return fail(JC_ERR_STATE, "the static scratch of device " + std::to_string(dev) +
                                          " is held by another bound group (jc_group_destroy it first)");
        if (!static_base[dev]) {
            void* p = nullptr;
            st = ghip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
            if (st != JC_OK)
                return st;
            static_base[dev] = static_cast<char*>(p);
        }
        base = static_base[dev];
        static_owner[dev] = g;
    }
    g->static_dev = dev;
    st = bind_common(g, base, true);
    if (st != JC_OK) {
        std::lock_guard<std::mutex> lock(static_mu);
        static_owner[dev] = nullptr;
        g->static_dev = -1;
        g->bound = false;
    }
    return st;
}

int jc_group_iterate(jc_group* g, int64_t n)
{
    if (!g || !g->bound)
        return fail(!g ? JC_ERR_INVALID : JC_ERR_STATE, "group is not bound (jc_group_bind)");
    if (n < 0)
        return fail(JC_ERR_INVALID, "n must be >= 0");
    for (const Class& k : g->classes)
        if (k.ir) {
            // one launch serves the whole class: its members must be at the
            // same point of their refinement step (jc_group_residuals
            // brings every member there)
            const jc_ctx* c0 = g->members[k.members[0]];
            for (int m : k.members) {
                const jc_ctx* c = g->members[m];
                if (c->ir_phase == 0)
                    return fail(JC_ERR_STATE, "a refining member needs jc_group_residuals before sweeping");
                if (c->ir_phase != c0->ir_phase || c->ir_q != c0->ir_q)
                    return fail(JC_ERR_STATE, "refining members are at different points of their step; "
                                              "call jc_group_residuals first");
            }
        }
    if (n == 0)
        return JC_OK;
    int st = prime_faces(g);
    if (st != JC_OK)
        return st;
    // the first window sweep of refinement members differs from the rest
    int64_t done = 0;
    bool ir_first = false;
    for (const Class& k : g->classes)
        if (k.ir && g->members[k.members[0]]->ir_phase == 1)
            ir_first = true;
    if (ir_first) {
        st = group_sweep(g);
        if (st != JC_OK)
            return st;
        advance(g, 1);
        done = 1;
    }
    const int64_t rest = n - done;
    if (rest <= 0)
        return JC_OK;
    if (!g->use_graphs)
        return group_run(g, rest);
    // graph of `rest` sweeps from the current launch parity; the d copy
    // of refinement members alternates with the launch parity
    int irq = 0;
    for (const Class& k : g->classes)
        if (k.ir)
            irq = g->members[k.members[0]]->ir_q;
    const auto key = std::make_pair(rest, g->parity | (irq << 1));
    auto found = g->graphs.find(key);
    if (found == g->graphs.end()) {
        // record the sweeps on a scratch copy of the member states
        std::vector<int> saved_q, saved_par, saved_phase;
        std::vector<int64_t> saved_it;
        std::vector<int> saved_ghost;
        std::vector<bool> saved_primed;
        for (jc_ctx* c : g->members) {
            saved_q.push_back(c->ir_q);
            saved_par.push_back(c->parity);
            saved_phase.push_back(c->ir_phase);
            saved_it.push_back(c->iters);
            saved_ghost.push_back(c->ghost);
            saved_primed.push_back(c->fused_primed);
        }
        const int gpar = g->parity;
        st = ghip(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (st != JC_OK)
            return st;
        st = group_run(g, rest);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(g->stream, &graph);
        g->parity = gpar;
        for (size_t i = 0; i < g->members.size(); ++i) {
            jc_ctx* c = g->members[i];
            c->ir_q = saved_q[i];
            c->parity = saved_par[i];
            c->ir_phase = saved_phase[i];
            c->iters = saved_it[i];
            c->ghost = saved_ghost[i];
            c->fused_primed = saved_primed[i];
        }
        if (st != JC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        st = ghip(e, "hipStreamEndCapture");
        if (st != JC_OK)
            return st;
        hipGraphExec_t exec = nullptr;
        st = ghip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        (void)hipGraphDestroy(graph);
        if (st != JC_OK)
            return st;
        found = g->graphs.emplace(key, exec).first;
    }
    st = ghip(hipGraphLaunch(found->second, g->stream), "hipGraphLaunch");
    if (st != JC_OK)
        return st;
    // the state after the replay, as the eager launches would leave it
    int64_t i = 0;
    if (g->three_step)
        for (; i + 3 <= rest; i += 3)
            advance2(g, 3);
    if (g->two_step)
        for (; i + 2 <= rest; i += 2)
            advance2(g);
    advance(g, rest - i);
    return JC_OK;
}

int jc_group_residuals(jc_group* g, double* host_l2)
{
    if (!g || !host_l2)
        return fail(JC_ERR_INVALID, "bad group or output");
    if (!g->bound)
        return fail(JC_ERR_STATE, "group is not bound (jc_group_bind)");
    int st = prime_faces(g);
    if (st != JC_OK)
        return st;
    for (const Class& k : g->classes) {
        const int n = (int)k.items.size();
        if (!k.ir) {
            const hipError_t e = jc::launch_sweep(g->d_desc(), g->d_items() + k.item0, n, g->parity, g->tile[0], g->tile[1],
                                                  true, true, false, k.src, g->d_partials() + k.item0, g->stream);
            if (e != hipSuccess)
                return ghip(e, "group residual");
            continue;
        }
        for (int m : k.members) {
            jc_ctx* c = g->members[m];
            const int nb = (int)c->blocks.size();
            BlockDesc* bd = g->d_desc() + g->member_bstart[m];
            if (!c->ir_zeroed) {
                st = ghip(jc::launch_zero(c->arena + c->lo_begin, c->lo_end - c->lo_begin, g->stream), "zero");
                if (st != JC_OK)
                    return st;
                c->ir_zeroed = true;
            }
            if (c->ir_phase == 2) {
                // outer update with the correction of the sweeps just run
                st = ghip(jc::launch_ir_update(bd, nb, c->max_rows(), c->parity, c->ir_q, k.lo, g->stream), "update");
                if (st != JC_OK)
                    return st;
            }
        }
        // refining members keep their iterate in copy 0 (their items' flip is 0)
        const hipError_t e = jc::launch_ir_residual(g->d_desc(), g->d_items() + k.item0, n, 0, g->tile[0], g->tile[1],
                                                    k.src, k.lo, g->d_partials() + k.item0, g->stream);
        if (e != hipSuccess)
            return ghip(e, "group refinement residual");
        for (int m : k.members)
            g->members[m]->ir_phase = 1;
    }
    const int nm = (int)g->members.size();
    st = ghip(jc::launch_reduce(g->d_partials(), g->d_lohi(), nm, g->d_out(), g->stream), "reduce");
    if (st == JC_OK)
        st = ghip(hipMemcpyAsync(g->h_out, g->d_out(), sizeof(double) * nm, hipMemcpyDeviceToHost, g->stream),
                  "copy residuals");
    if (st == JC_OK)
        st = ghip(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    if (st != JC_OK)
        return st;
    int bad = -1;
    for (int m = 0; m < nm; ++m) {
        host_l2[m] = std::sqrt(g->h_out[m]);
        if (!std::isfinite(host_l2[m]) && bad < 0)
            bad = m;
    }
    if (bad >= 0)
        return fail(JC_ERR_NONFINITE, "residual of group member " + std::to_string(bad) + " is not finite");
    return JC_OK;
}

int jc_group_check(jc_group* g, double rtol, int64_t max_iter, double* host_rel, int* host_done)
{
    if (!g || !host_rel || !host_done)
        return fail(JC_ERR_INVALID, "bad group or output");
    if (!std::isfinite(rtol) || max_iter < 0)
        return fail(JC_ERR_INVALID, "rtol must be finite and max_iter >= 0");
    const int nm = (int)g->members.size();
    std::vector<double> l2(nm, 0.0);
    const int st = jc_group_residuals(g, l2.data());
    if (st != JC_OK && st != JC_ERR_NONFINITE)
        return st;
    for (int m = 0; m < nm; ++m) {
        jc_ctx* c = g->members[m];
        if (c->check_r0 < 0)
            c->check_r0 = l2[m];
        host_rel[m] = c->check_r0 > 0 ? l2[m] / c->check_r0 : 0.0;
        host_done[m] = (host_rel[m] <= rtol || c->iters >= max_iter) ? 1 : 0;
    }
    return st;
}

void jc_group_destroy(jc_group* g)
{
    if (!g)
        return;
    if (g->bound)
        (void)hipStreamSynchronize(g->stream);
    for (auto& kv : g->graphs)
        (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : g->events)
        (void)hipEventDestroy(e);
    if (g->h_out && g->h_out != g->h_out_plain.data())
        (void)hipHostFree(g->h_out);
    if (g->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(static_mu);
        if (static_owner[g->static_dev] == g)
            static_owner[g->static_dev] = nullptr;
    }
    delete g;
}

}  // extern "C"
