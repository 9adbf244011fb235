// HIP kernels of libjc for gfx950 (CDNA4, wave64).
//
// Jacobi3D, paper section 4.3: each block of the decomposition is swept
// with the 7-point stencil after its halo has been exchanged with up to
// six neighbours.  The sweep marches along z through a tile of 64 x cells
// by tile_y rows, staging each plane in LDS and keeping the z-1, z and z+1
// values of its own cells in registers, so that every interior value is
// fetched from HBM once per sweep.  The stencil is not a contraction, so
// no matrix cores are used: the kernel is bound by HBM bandwidth (16 bytes
// per cell update in FP64).
//
// Bit-exactness: the neighbour sum is formed in one fixed order and
// divided by 6, correctly rounded (jc_div6.h); the library is built with
// -ffp-contract=off, so no multiply-add is fused and every block of every
// decomposition computes the same bits for the same cell.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "jc_div6.h"
#include "jc_kernels.h"

namespace jc {

namespace {

// Work-groups are dispatched round-robin over the 8 XCDs of the chip
// (work-group i to XCD i mod 8).  Give each XCD a contiguous range of
// logical tiles so that tiles sharing halo rows run under the same L2.
__device__ __forceinline__ int logical_block(int bid, int nblocks)
{
    const int per = nblocks >> 3;           // nblocks is a multiple of 8
    return (bid & 7) * per + (bid >> 3);
}

// Global-memory views of the generic pointers held in the tables: loads
// and stores through them are global (not flat) instructions, which count
// only against the vector-memory counter, so waiting for an LDS write does
// not also wait for every load still in flight.
#define JC_GLOBAL __attribute__((address_space(1)))

// ---- sweep kernel: begin (its source is fingerprinted with recorded counters) ----
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// bfloat16: the upper half of a binary32, rounded to nearest even
__device__ __forceinline__ float bf16_to_f32(uint32_t h)
{
    return __uint_as_float(h << 16);
}

// Round to nearest even without a branch: adding 0x7fff plus the kept
// half's lowest bit carries into the upper half exactly when the dropped
// half is above one half, or equal to it with an odd kept half (equal, bit
// for bit, to the comparison form for every binary32 pattern).  A NaN
// stays a (quiet) NaN.
__device__ __forceinline__ uint32_t f32_to_bf16(float f)
{
    const uint32_t x = __float_as_uint(f);
    const uint32_t rounded = (x + 0x7fffu + ((x >> 16) & 1u)) >> 16;
    const uint32_t quiet_nan = (x >> 16) | 0x40u;
    return __builtin_isnan(f) ? quiet_nan : rounded;   // an unordered self-compare
}

// Storage formats of a swept field: arithmetic type C, and loads / stores
// of the 2-element aligned pair (x, x + 1) that one thread owns.
template <typename T> struct Tr;

template <> struct Tr<double> {
    using C = double;
    __device__ static void ld(const double* p, double& a, double& b)
    {
        const v2d v = *(const v2d JC_GLOBAL*)(p);
        a = v.x;
        b = v.y;
    }
    __device__ static void st(double* p, double a, double b)
    {
        v2d v;
        v.x = a;
        v.y = b;
        *(v2d JC_GLOBAL*)(p) = v;
    }
    __device__ static void st1(double* p, double a) { *(double JC_GLOBAL*)(p) = a; }
    // streaming store: the new iterate is not read again before the next
    // sweep, so it should not displace lines the current sweep re-reads
    __device__ static void stn(double* p, double a, double b)
    {
        v2d v;
        v.x = a;
        v.y = b;
        __builtin_nontemporal_store(v, (v2d JC_GLOBAL*)(p));
    }
    // a pair converted to storage once, stored whole or by element
    using P = v2d;
    __device__ static P pack(double a, double b)
    {
        v2d v;
        v.x = a;
        v.y = b;
        return v;
    }
    __device__ static void stp(double* p, P v) { *(v2d JC_GLOBAL*)(p) = v; }
    __device__ static void stpn(double* p, P v) { __builtin_nontemporal_store(v, (v2d JC_GLOBAL*)(p)); }
    __device__ static void st1a(double* p, P v) { *(double JC_GLOBAL*)(p) = v.x; }
    __device__ static void st1b(double* p, P v) { *(double JC_GLOBAL*)(p) = v.y; }
};

template <> struct Tr<float> {
    using C = float;
    __device__ static void ld(const float* p, float& a, float& b)
    {
        const v2f v = *(const v2f JC_GLOBAL*)(p);
        a = v.x;
        b = v.y;
    }
    __device__ static void st(float* p, float a, float b)
    {
        v2f v;
        v.x = a;
        v.y = b;
        *(v2f JC_GLOBAL*)(p) = v;
    }
    __device__ static void st1(float* p, float a) { *(float JC_GLOBAL*)(p) = a; }
    __device__ static void stn(float* p, float a, float b)
    {
        v2f v;
        v.x = a;
        v.y = b;
        __builtin_nontemporal_store(v, (v2f JC_GLOBAL*)(p));
    }
    using P = v2f;
    __device__ static P pack(float a, float b)
    {
        v2f v;
        v.x = a;
        v.y = b;
        return v;
    }
    __device__ static void stp(float* p, P v) { *(v2f JC_GLOBAL*)(p) = v; }
    __device__ static void stpn(float* p, P v) { __builtin_nontemporal_store(v, (v2f JC_GLOBAL*)(p)); }
    __device__ static void st1a(float* p, P v) { *(float JC_GLOBAL*)(p) = v.x; }
    __device__ static void st1b(float* p, P v) { *(float JC_GLOBAL*)(p) = v.y; }
};

template <> struct Tr<bf16> {
    using C = float;
    __device__ static void ld(const bf16* p, float& a, float& b)
    {
        const uint32_t w = *(const uint32_t JC_GLOBAL*)(p);    // x at the lower address
        a = bf16_to_f32(w & 0xffffu);
        b = bf16_to_f32(w >> 16);
    }
    __device__ static void st(bf16* p, float a, float b)
    {
        *(uint32_t JC_GLOBAL*)(p) = f32_to_bf16(a) | (f32_to_bf16(b) << 16);
    }
    __device__ static void st1(bf16* p, float a) { *(uint16_t JC_GLOBAL*)(p) = (uint16_t)f32_to_bf16(a); }
    __device__ static void stn(bf16* p, float a, float b)
    {
        __builtin_nontemporal_store(f32_to_bf16(a) | (f32_to_bf16(b) << 16), (uint32_t JC_GLOBAL*)(p));
    }
    using P = uint32_t;                           // x in the low half
    __device__ static P pack(float a, float b) { return f32_to_bf16(a) | (f32_to_bf16(b) << 16); }
    __device__ static void stp(bf16* p, P v) { *(uint32_t JC_GLOBAL*)(p) = v; }
    __device__ static void stpn(bf16* p, P v) { __builtin_nontemporal_store(v, (uint32_t JC_GLOBAL*)(p)); }
    __device__ static void st1a(bf16* p, P v) { *(uint16_t JC_GLOBAL*)(p) = (uint16_t)(v & 0xffffu); }
    __device__ static void st1b(bf16* p, P v) { *(uint16_t JC_GLOBAL*)(p) = (uint16_t)(v >> 16); }
};

// Which arrays of a block a sweep works on: the iterate u (with source b)
// or the refinement correction d (with source r_lo).
enum { FIELD_U = 0, FIELD_D = 1 };

template <typename T, int FIELD> struct Fld;

template <typename T> struct Fld<T, FIELD_U> {
    __device__ static const T* src(const BlockDesc* B, int p) { return B->u[p]; }
    __device__ static T* dst(const BlockDesc* B, int p) { return B->u[p ^ 1]; }
    __device__ static const T* source(const BlockDesc* B) { return B->b; }
    __device__ static const T* gin(const BlockDesc* B, int f, int s) { return B->gin[f][s]; }
    __device__ static T* gout(const BlockDesc* B, int f, int s) { return B->gout[f][s]; }
    __device__ static const T* xg(const BlockDesc* B, int f) { return B->xg[f]; }
    __device__ static int64_t pitch(const BlockDesc* B) { return B->pitch; }
    __device__ static int64_t plane(const BlockDesc* B) { return B->plane; }
};

template <typename T> struct Fld<T, FIELD_D> {
    __device__ static const T* src(const BlockDesc* B, int p) { return static_cast<const T*>(B->d[p]); }
    __device__ static T* dst(const BlockDesc* B, int p) { return static_cast<T*>(B->d[p ^ 1]); }
    __device__ static const T* source(const BlockDesc* B) { return static_cast<const T*>(B->rlo); }
    __device__ static const T* gin(const BlockDesc* B, int f, int s)
    {
        return static_cast<const T*>(B->lgin[f][s]);
    }
    __device__ static T* gout(const BlockDesc* B, int f, int s) { return static_cast<T*>(B->lgout[f][s]); }
    __device__ static const T* xg(const BlockDesc* B, int f) { return static_cast<const T*>(B->lxg[f]); }
    __device__ static int64_t pitch(const BlockDesc* B) { return B->lpitch; }
    __device__ static int64_t plane(const BlockDesc* B) { return B->lplane; }
};

struct NoRlo {};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = v + __shfl_xor(v, o, 64);
    return v;
}

// Pacing.  The work-groups of a launch advance at different rates (a tile
// on a Dirichlet face reads its ghosts from a compact column, other tiles
// read their x halo from the neighbour tile's lines, work-groups sit at
// different distances from the memory they stream), and the launch ends
// with the slowest: measured on the 512^3 launch of 256 tiles, they took
// 359-396 us, so the compute units of the fast ones idled through the
// tail.  With a pace, a work-group waits before plane step k until k *
// pace ticks of the chip's constant 100 MHz clock have passed since it
// started: the fast ones are held to the pace and the memory traffic of
// the slow ones runs without their competition, so all finish together.
// The pace is tuned by timing (jc_autotune); 0 = none.  Each wait is
// bounded (4096 short sleeps), and results do not depend on it.
__device__ __forceinline__ void pace_wait(uint64_t due)
{
    for (int i = 0; i < 4096 && __builtin_amdgcn_s_memrealtime() < due; ++i)
        __builtin_amdgcn_s_sleep(1);
}

// Planes of loads a sweep keeps in flight ahead of the plane it computes:
// three.  For binary64 fields at one 16-wave work-group per CU two planes
// of 16-byte loads are too few bytes in flight to cover the memory
// latency; a bfloat16 thread loads only 4 bytes per plane and field, and
// its inner sweep at 1024^3 ran 7 % faster with three planes than with two
// (binary32 the same; four planes gained nothing for either).
template <typename T> constexpr int prefetch_planes() { return 3; }

// One work-group sweeps a tile of 2 TXP x cells (16, 32 or 64; or 96, 128 or
// 256 for binary64 storage) by TY rows of one block, marching along z.  Each thread owns two adjacent x cells of one row
// (one aligned-pair load per plane: cell x = 1 of every row starts a
// 128-byte line).  Per plane the work-group writes the plane -- its cells
// plus a one-cell halo ring -- into an LDS tile, synchronises once (the
// tile is double-buffered by plane parity) and reads its x and y
// neighbours from LDS; the z-1 / z / z+1 values of its own cells stay in
// registers.
//
// Every thread issues the same global loads in every iteration, with
// clamped addresses where it has nothing to fetch, so that the loads of
// the next planes (prefetch_planes<T>()) stay in flight while the current
// one is computed (no divergent branch around a load).  The halo ring is fetched by
// threads with a halo role: the first TXP threads the row above the tile,
// the next TXP the row below, the next TY the column left of it and the
// next TY the column right of it; the rest re-load their own cells.
//
// T / FIELD: the swept field and its storage (binary64 iterate u, or the
// correction d of the refinement stored as binary64, binary32 or
// bfloat16 with binary32 arithmetic).  FUSED: ghost cells of faces that
// have a neighbour block are read from the neighbour's face buffer of the
// input slot (the pairing's pre-posted receive side), ghost cells of
// unpaired x faces from the block's compact Dirichlet ghost columns, and
// every face cell written is also written to this block's face buffer of
// the output slot -- pack, exchange and unpack folded into the sweep.  RES: accumulate r^2
// of the input iterate, r = (b + s) - 6u, into one partial per
// work-group.  STORE: write the new iterate.  SRC: add the source (b for
// u, r_lo for d).  R: also store r rounded to R into the block's r_lo
// array (the outer pass of the refinement).
template <typename T, int FIELD, int TXP, int TY, bool FUSED, bool RES, bool STORE, bool SRC, typename R>
__global__ void __launch_bounds__(TXP * TY)
k_sweep(const BlockDesc* __restrict__ blocks, const Item* __restrict__ items, int nitems,
        int parity, double* __restrict__ partials, uint32_t pace)
{
    static_assert(TY >= 4 && TXP * TY >= 2 * TXP + 2 * TY && (TXP * TY) % 64 == 0,
                  "halo roles need 2 TXP + 2 TY threads; whole waves");
    using C = typename Tr<T>::C;
    using F = Fld<T, FIELD>;
    constexpr bool RLO = !std::is_same<R, NoRlo>::value;
    constexpr int NT = TXP * TY;
    constexpr int W = 2 * TXP;                    // tile width in cells
    constexpr int LW = W + 4;  // LDS row: col 1 = x0, cols 2..W+1 = x0+1..x0+W, up to col W+2
    __shared__ C S[2][TY + 2][LW];
    __shared__ double wsum[NT / 64];

    const int id = logical_block(blockIdx.x, gridDim.x);
    if (id >= nitems)
        return;                                   // uniform over the work-group
    const uint64_t pace_t0 = pace ? __builtin_amdgcn_s_memrealtime() : 0;
    const Item it = items[id];
    const BlockDesc* B = blocks + it.block;
    const int p = parity ^ it.flip;
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    const int t = threadIdx.x;
    const int lx = t % TXP;
    const int ly = t / TXP;
    const int x0 = it.x0, y0 = it.y0;
    const int x_end = min(x0 + W, nx);            // last x cell of the tile
    const int y_end = min(y0 + TY, ny);           // last row of the tile
    const int ly_last = y_end - y0 - 1;
    const int xa = x0 + 2 * lx + 1;               // this thread's cells: xa, xa + 1
    const int y = y0 + ly + 1;
    const bool row_ok = y <= ny;
    const bool a_ok = row_ok && xa <= nx;
    const bool b_ok = row_ok && xa + 1 <= nx;
    const int xlast = (nx - 1) | 1;               // start of the last aligned pair of a row
    const int xa_c = min(xa, xlast);
    const int y_c = min(y, ny);
    const int64_t pitch = F::pitch(B);
    const int64_t plane = F::plane(B);
    const int64_t ldx = face_ld(ny);              // x-face buffers: (z, y) rows
    const int64_t ldy = face_ld(nx);              // y- and z-face buffers: (z, x) / (y, x) rows
    const T* __restrict__ src = F::src(B, p);
    T* __restrict__ dst = F::dst(B, p);
    const C six = C(6);

    // own pair (xa_c, y_c) at plane zz
    const T* own = src + (int64_t)y_c * pitch + xa_c;
    const T* own_lo = own;                                        // plane 0
    const T* own_hi = own + (int64_t)(nz + 1) * plane;            // plane nz + 1
    if (FUSED) {
        const int64_t zi = (int64_t)(y_c - 1) * ldy + (xa_c - 1);
        if (F::gin(B, ZM, p)) own_lo = F::gin(B, ZM, p) + zi;
        if (F::gin(B, ZP, p)) own_hi = F::gin(B, ZP, p) + zi;
    }
    auto own_at = [&](int zz, C& a, C& b) {
        const T* q = own + (int64_t)zz * plane;
        if (FUSED) {
            q = (zz == 0) ? own_lo : q;
            q = (zz == nz + 1) ? own_hi : q;
        }
        Tr<T>::ld(q, a, b);
    };
    const T* sown = SRC ? F::source(B) + (int64_t)y_c * pitch + xa_c : nullptr;

    // halo role: the pair at hbase + zz * hstride
    const int role = t < TXP ? 0 : t < 2 * TXP ? 1 : t < 2 * TXP + TY ? 2 : t < 2 * TXP + 2 * TY ? 3 : 4;
    const T* hbase = own;
    int64_t hstride = plane;
    int hrow = 0, hcol = 0, hcomp = 0;
    bool hv0 = false, hv1 = false;
    if (role <= 1) {
        const int hl = t % TXP;
        const int hx = x0 + 2 * hl + 1;
        const int hx_c = min(hx, xlast);
        const int hy = role == 0 ? y0 : y_end + 1;
        hv0 = hx <= x_end;
        hv1 = hx + 1 <= x_end;
        hbase = src + (int64_t)hy * pitch + hx_c;
        if (FUSED) {
            const T* const gym = F::gin(B, YM, p);    // read uniformly, selected per thread
            const T* const gyp = F::gin(B, YP, p);
            const T* g = (hy == 0) ? gym : (hy == ny + 1) ? gyp : nullptr;
            if (g) {
                hbase = g - ldy + (hx_c - 1);     // value (z - 1, x - 1)
                hstride = ldy;
            }
        }
        hrow = role == 0 ? 0 : ly_last + 2;
        hcol = 2 * hl + 2;
    } else if (role <= 3) {
        const int r = t - 2 * TXP - (role == 3 ? TY : 0);
        const int hy = y0 + r + 1;
        hv0 = hy <= y_end;
        const int hy_c = min(hy, ny);
        const int hx = role == 2 ? x0 : x_end + 1;
        const int ps = (hx & 1) ? hx : hx - 1;    // aligned pair holding hx
        hcomp = (hx & 1) ? 0 : 1;
        hbase = src + (int64_t)hy_c * pitch + ps;
        // Fused: a paired face's ghosts come from the neighbour's face
        // buffer and a Dirichlet face's from its compact ghost column.
        // Staged: from the block's own column, whose 128-byte lines each
        // hold one row's x = 0 ghost and the previous row's x = nx + 1
        // ghost, both read there.  Both faces' pointers are read uniformly
        // and selected per thread (a per-thread pointer load would stall
        // the prologue).
        const T* const gxm = !FUSED ? nullptr : F::gin(B, XM, p) ? F::gin(B, XM, p) : F::xg(B, XM);
        const T* const gxp = !FUSED ? nullptr : F::gin(B, XP, p) ? F::gin(B, XP, p) : F::xg(B, XP);
        const T* g = (hx == 0) ? gxm : (hx == nx + 1) ? gxp : nullptr;
        if (g) {
            const int fi = hy_c - 1;              // value (z - 1, y - 1)
            hbase = g - ldx + (fi & ~1);
            hcomp = fi & 1;
            hstride = ldx;
        }
        hrow = r + 1;
        hcol = role == 2 ? 1 : x_end - x0 + 2;
    }

    // Face stores of the fused epilogue.  Which of this thread's cells lie
    // on an x or y face does not change along z; a tile that touches no
    // paired x or y face (most tiles) skips them with one uniform branch.
    T* const oxm = FUSED ? F::gout(B, XM, p ^ 1) : nullptr;
    T* const oxp = FUSED ? F::gout(B, XP, p ^ 1) : nullptr;
    T* const oym = FUSED ? F::gout(B, YM, p ^ 1) : nullptr;
    T* const oyp = FUSED ? F::gout(B, YP, p ^ 1) : nullptr;
    T* const ozm = FUSED ? F::gout(B, ZM, p ^ 1) : nullptr;
    T* const ozp = FUSED ? F::gout(B, ZP, p ^ 1) : nullptr;
    const bool xy_tile = FUSED && ((x0 == 0 && oxm) || (x_end == nx && oxp) || (y0 == 0 && oym) ||
                                   (y_end == ny && oyp));
    const bool f_xm = a_ok && xa == 1 && oxm;
    const bool f_xpa = a_ok && xa == nx && oxp;
    const bool f_xpb = b_ok && xa + 1 == nx && oxp;
    const bool f_ym = a_ok && y == 1 && oym;
    const bool f_yp = a_ok && y == ny && oyp;

    // LDS slots of this thread's four writes per plane (own x cells, halo
    // values).  A write with nothing to store goes to column 0, which no
    // thread reads, so the writes need no branch.
    const int lds_a = a_ok ? (ly + 1) * LW + 2 * lx + 2 : 0;
    const int lds_b = b_ok ? (ly + 1) * LW + 2 * lx + 3 : 0;
    const int lds_h0 = (role <= 3 && hv0) ? hrow * LW + hcol : 0;
    const int lds_h1 = (role <= 1 && hv1) ? hrow * LW + hcol + 1 : 0;

    const int zf = it.z0 + 1;                     // first plane of the tile
    const int zl = it.z0 + it.zlen;               // last plane of the tile
    // Register rings of RS slots: own cells, halo and source of plane p in
    // slot (p - zf) mod RS.  At step z the loads of plane z + PD are issued
    // (own cells of z - 1 .. z + PD are live), so every value has PD plane
    // steps to arrive.  Every load lands in the slot it is consumed from:
    // no register is copied while its load is in flight (such a copy waits
    // for every outstanding load).  RS is even so that the LDS buffer of a
    // step (its slot's parity) alternates across the unrolled loop.
    constexpr int PD = prefetch_planes<T>();
    static_assert(PD >= 2 && PD <= 4, "prefetch distance 2..4 planes");
    constexpr int RS = (PD + 3) & ~1;
    C ra[RS], rb[RS], ha[RS], hb[RS], sa_[RS], sb_[RS];
    own_at(zf - 1, ra[RS - 1], rb[RS - 1]);
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        own_at(min(zf + k, zl + 1), ra[k], rb[k]);
        Tr<T>::ld(hbase + (int64_t)min(zf + k, zl) * hstride, ha[k], hb[k]);
    }
#pragma unroll
    for (int k = 0; k < RS; ++k)
        sa_[k] = sb_[k] = C(0);
    if (SRC) {
#pragma unroll
        for (int k = 0; k < PD; ++k)
            Tr<T>::ld(sown + (int64_t)min(zf + k, zl) * plane, sa_[k], sb_[k]);
    }

    double acc = 0.0;
    // one plane; K = (z - zf) mod RS, a compile-time slot number
    auto step = [&](int z, auto kc) {
        constexpr int K = decltype(kc)::value;
        constexpr int SM = (K + RS - 1) % RS, SC = K, SP = (K + 1) % RS, SQ = (K + PD) % RS;
        static_assert(K >= 0 && K < RS, "ring slot");
        constexpr int HC = K & 1;                 // LDS buffer of this plane
        if (pace)
            pace_wait(pace_t0 + (uint64_t)(z - zf) * pace);
        // plane z + PD goes in flight first; the last steps re-read planes
        // they already hold (cache hits) instead of branching
        const int zh = min(z + PD, zl);
        own_at(min(z + PD, zl + 1), ra[SQ], rb[SQ]);
        Tr<T>::ld(hbase + (int64_t)zh * hstride, ha[SQ], hb[SQ]);
        if (SRC)
            Tr<T>::ld(sown + (int64_t)zh * plane, sa_[SQ], sb_[SQ]);
        const C c_a = ra[SC], c_b = rb[SC];
        C (*L)[LW] = S[HC];
        C* const Lf = &S[HC][0][0];
        Lf[lds_a] = c_a;
        Lf[lds_b] = c_b;
        Lf[lds_h0] = hcomp ? hb[SC] : ha[SC];
        Lf[lds_h1] = hb[SC];
        __syncthreads();
        const C xm_a = L[ly + 1][2 * lx + 1];
        const C xp_a = b_ok ? c_b : L[ly + 1][2 * lx + 3];
        C sa = xm_a + xp_a;
        sa = sa + L[ly][2 * lx + 2];
        sa = sa + L[ly + 2][2 * lx + 2];
        sa = sa + ra[SM];
        sa = sa + ra[SP];
        C sb = c_a + L[ly + 1][2 * lx + 4];
        sb = sb + L[ly][2 * lx + 3];
        sb = sb + L[ly + 2][2 * lx + 3];
        sb = sb + rb[SM];
        sb = sb + rb[SP];
        const C s_a = sa_[SC], s_b = sb_[SC];
        if (RES) {
            const C r_a = SRC ? (s_a + sa) - six * c_a : sa - six * c_a;
            const C r_b = SRC ? (s_b + sb) - six * c_b : sb - six * c_b;
            acc = acc + (a_ok ? (double)(r_a * r_a) : 0.0);
            acc = acc + (b_ok ? (double)(r_b * r_b) : 0.0);
            if constexpr (RLO) {
                // r rounded to the refinement's storage, through binary32
                R* o = static_cast<R*>(B->rlo) + (int64_t)z * B->lplane + (int64_t)y * B->lpitch + xa;
                if constexpr (std::is_same<R, double>::value) {
                    if (a_ok) Tr<double>::st(o, r_a, r_b);
                } else {
                    if (a_ok) Tr<R>::st(o, (float)r_a, (float)r_b);
                }
            }
        }
        if (STORE) {
            C va, vb;
            if (SRC)
                div6_pair(sa + s_a, sb + s_b, va, vb);
            else
                div6_pair(sa, sb, va, vb);
            // past the last cell of a row the pair's second slot is the
            // x = nx + 1 ghost: write back the value it already holds
            vb = b_ok ? vb : c_b;
            const auto pk = Tr<T>::pack(va, vb);
            if (a_ok)
                Tr<T>::stpn(dst + (int64_t)z * plane + (int64_t)y * pitch + xa, pk);
            if (FUSED) {
                // a face row's padding slot takes the second value of a
                // pair that ends past the face (ld is even)
                const int64_t zfi = (int64_t)(y - 1) * ldy + (xa - 1);
                if (z == 1 && ozm && a_ok) Tr<T>::stp(ozm + zfi, pk);
                if (z == nz && ozp && a_ok) Tr<T>::stp(ozp + zfi, pk);
                if (xy_tile) {
                    const int64_t xfi = (int64_t)(z - 1) * ldx + (y - 1);
                    const int64_t yfi = (int64_t)(z - 1) * ldy + (xa - 1);
                    if (f_xm) Tr<T>::st1a(oxm + xfi, pk);
                    if (f_xpa) Tr<T>::st1a(oxp + xfi, pk);
                    if (f_xpb) Tr<T>::st1b(oxp + xfi, pk);
                    if (f_ym) Tr<T>::stp(oym + yfi, pk);
                    if (f_yp) Tr<T>::stp(oyp + yfi, pk);
                }
            }
        }
    };
#define JC_STEP(k) step(z + (k), std::integral_constant<int, (k)>{})
    int z = zf;
    if constexpr (RS == 4) {
        for (; z + 3 <= zl; z += 4) {
            JC_STEP(0);
            JC_STEP(1);
            JC_STEP(2);
            JC_STEP(3);
        }
        if (z <= zl) JC_STEP(0);
        if (z + 1 <= zl) JC_STEP(1);
        if (z + 2 <= zl) JC_STEP(2);
    } else {
        static_assert(RS == 6, "ring of 4 or 6 slots");
        for (; z + 5 <= zl; z += 6) {
            JC_STEP(0);
            JC_STEP(1);
            JC_STEP(2);
            JC_STEP(3);
            JC_STEP(4);
            JC_STEP(5);
        }
        if (z <= zl) JC_STEP(0);
        if (z + 1 <= zl) JC_STEP(1);
        if (z + 2 <= zl) JC_STEP(2);
        if (z + 3 <= zl) JC_STEP(3);
        if (z + 4 <= zl) JC_STEP(4);
    }
#undef JC_STEP
    if (RES) {
        const double w = wave_sum(acc);
        if ((t & 63) == 0)
            wsum[t >> 6] = w;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int i = 0; i < NT / 64; ++i)
                sum = sum + wsum[i];
            partials[id] = sum;
        }
    }
}

template <typename T, int FIELD, int TXP, int TY, bool SRC, typename R>
hipError_t sweep_flags(const BlockDesc* blocks, const Item* items, int nitems, int parity, bool fused,
                       bool resid, bool store, double* partials, hipStream_t s, uint32_t pace)
{
    const int grid = ((nitems + 7) / 8) * 8;
    const dim3 bs(TXP * TY);
#define JC_SWEEP_CASE(FU, RE, ST)                                                                         \
    if (fused == FU && resid == RE && store == ST) {                                                     \
        hipLaunchKernelGGL((k_sweep<T, FIELD, TXP, TY, FU, RE, ST, SRC, R>), dim3(grid), bs, 0, s, blocks, \
                           items, nitems, parity, partials, pace);                                       \
        return hipGetLastError();                                                                        \
    }
    if constexpr (std::is_same<R, NoRlo>::value) {
        if constexpr (FIELD == FIELD_U) {
            JC_SWEEP_CASE(false, false, true)
            JC_SWEEP_CASE(false, true, true)
            JC_SWEEP_CASE(false, true, false)
            JC_SWEEP_CASE(true, true, true)
            JC_SWEEP_CASE(true, true, false)
        }
        JC_SWEEP_CASE(true, false, true)
    } else {
        JC_SWEEP_CASE(true, true, false)
    }
#undef JC_SWEEP_CASE
    return hipErrorInvalidValue;
}

template <typename T, int FIELD, int TXP, bool SRC, typename R>
hipError_t sweep_rows(const BlockDesc* blocks, const Item* items, int nitems, int parity, int tile_y,
                      bool fused, bool resid, bool store, double* partials, hipStream_t s, uint32_t pace)
{
    // at most 1024 threads per work-group
    switch (tile_y) {
    case 4:
        // a 16-cell tile needs 8 rows for whole waves
        if constexpr (TXP * 4 >= 64)
            return sweep_flags<T, FIELD, TXP, 4, SRC, R>(blocks, items, nitems, parity, fused, resid, store, partials, s, pace);
        else
            return hipErrorInvalidValue;
    case 8:
        if constexpr (TXP * 8 <= 1024)
            return sweep_flags<T, FIELD, TXP, 8, SRC, R>(blocks, items, nitems, parity, fused, resid, store, partials, s, pace);
        else
            return hipErrorInvalidValue;
    case 16:
        if constexpr (TXP * 16 <= 1024)
            return sweep_flags<T, FIELD, TXP, 16, SRC, R>(blocks, items, nitems, parity, fused, resid, store, partials, s, pace);
        else
            return hipErrorInvalidValue;
    case 32:
        if constexpr (TXP * 32 <= 1024)
            return sweep_flags<T, FIELD, TXP, 32, SRC, R>(blocks, items, nitems, parity, fused, resid, store, partials, s, pace);
        else
            return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int FIELD, bool SRC, typename R>
hipError_t sweep_tiles(const BlockDesc* blocks, const Item* items, int nitems, int parity, int tile_x, int tile_y,
                       bool fused, bool resid, bool store, double* partials, hipStream_t s, uint32_t pace)
{
    switch (tile_x) {
    case 16: return sweep_rows<T, FIELD, 8, SRC, R>(blocks, items, nitems, parity, tile_y, fused, resid, store, partials, s, pace);
    case 32: return sweep_rows<T, FIELD, 16, SRC, R>(blocks, items, nitems, parity, tile_y, fused, resid, store, partials, s, pace);
    case 64: return sweep_rows<T, FIELD, 32, SRC, R>(blocks, items, nitems, parity, tile_y, fused, resid, store, partials, s, pace);
    default: break;
    }
    // Tiles as wide as a whole block row of 96, 128 or 256 cells (binary64
    // storage): the x halo is then the block's ghost column, never a
    // neighbour tile's lines.
    if constexpr (sizeof(T) == 8) {
        switch (tile_x) {
        case 96: return sweep_rows<T, FIELD, 48, SRC, R>(blocks, items, nitems, parity, tile_y, fused, resid, store, partials, s, pace);
        case 128: return sweep_rows<T, FIELD, 64, SRC, R>(blocks, items, nitems, parity, tile_y, fused, resid, store, partials, s, pace);
        case 256: return sweep_rows<T, FIELD, 128, SRC, R>(blocks, items, nitems, parity, tile_y, fused, resid, store, partials, s, pace);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

// ---- sweep kernel: end ----

// ---- two-step sweep (temporal blocking): begin (fingerprinted with recorded counters) ----
// Two Jacobi sweeps of the single block of a context without face pairs
// per launch: iterate k is read from copy p and iterate k + 2 written to
// copy p ^ 1; iterate k + 1 lives only in LDS and registers.  T / FIELD as
// for k_sweep: the binary64 iterate u (source b), or the refinement
// correction d in its storage format (source r_lo, zero ghosts), whose
// iterate k + 1 is rounded to that format as a stored sweep would leave
// it.  Each cell's two updates take the same sums in the same order as
// two one-step sweeps, so the result is bitwise the same; HBM moves one
// read and one write per cell for two sweeps instead of two of each.
//
// A work-group owns a tile of 2 TXP x cells by TY rows and a z range, and
// marches along z as the one-step sweep does.  Iterate k + 1 is needed on
// the tile and on a one-cell ring around it, so iterate k is loaded on a
// two-cell ring: one aligned pair per thread over (TXP + 2) pairs by (TY +
// 4) rows.  The first TXP * TY threads (whole waves) own the tile's pairs,
// the next 4 (TXP + 2) the two rows above and the two rows below it, the
// next 2 TY the pair left and the pair right of each tile row.  At plane
// step s every thread writes iterate k of its pair at plane s into LDS,
// the work-group synchronises once, every thread computes iterate k + 1 of
// its pair at plane s (a ghost cell keeps its value: the context has no
// face pairs, so every ghost is a fixed boundary value) into a second LDS
// plane, and the tile threads compute iterate k + 2 at plane s - 1 from
// the previous step's second plane.  Both LDS planes are double-buffered
// by step parity.  Values at cells two steps out of the block (the
// outermost ring of a tile on the block edge) are clamped loads that only
// feed discarded results.
// A value of the arithmetic type rounded to the storage format and back:
// iterate k + 1 is stored between the two sweeps of a one-sweep-per-launch
// run, so the second sweep must read it at storage precision.
template <typename T> __device__ __forceinline__ typename Tr<T>::C storage_round(typename Tr<T>::C v) { return v; }
template <> __device__ __forceinline__ float storage_round<bf16>(float v) { return bf16_to_f32(f32_to_bf16(v)); }

//
// Work: with items null, the tiles of blocks[0] (tiles_x by tiles_y per z
// chunk, nch chunks, ntiles in all) numbered from the work-group index;
// otherwise the work list items[0 .. ntiles), whose tiles must be 2 TXP
// cells by TY rows, each with its block and ping-pong flip (groups).
// A pair of arithmetic values as one LDS access (16 bytes in binary64).
template <typename C> struct Pair2;
template <> struct Pair2<double> { using V = v2d; };
template <> struct Pair2<float> { using V = v2f; };

template <typename T, int FIELD, int TXP, int TY, bool SRC>
__global__ void __launch_bounds__(((TXP + 2) * (TY + 4) + 63) / 64 * 64)
k_sweep2(const BlockDesc* __restrict__ blocks, const Item* __restrict__ items, int parity, int tiles_x,
         int tiles_y, int nch, int ntiles, uint32_t pace)
{
    using C = typename Tr<T>::C;
    using F = Fld<T, FIELD>;
    constexpr int EP = TXP + 2;                   // pairs of an extended row
    constexpr int ER = TY + 4;                    // extended rows
    constexpr int NTILE = TXP * TY;               // tile threads
    static_assert(NTILE % 64 == 0, "tile threads are whole waves");
    using V = typename Pair2<C>::V;
    // LDS row: two pad cells, 2 EP cells, two pad cells, so that every
    // thread's pair is one aligned vector: a pair is written with one
    // access and its neighbours' pairs are read with one access each
    constexpr int LW = 2 * EP + 4;
    constexpr int LN = (ER + 2) * LW;             // LDS plane: pad row, ER rows, pad row
    __shared__ V A[2][LN / 2 + 1];                // iterate k; pair LN / 2: sink of idle lanes
    __shared__ V Bn[2][LN / 2 + 1];               // iterate k + 1

    const int id = logical_block(blockIdx.x, gridDim.x);
    if (id >= ntiles)
        return;                                   // uniform over the work-group
    const uint64_t pace_t0 = pace ? __builtin_amdgcn_s_memrealtime() : 0;
    const BlockDesc* B = blocks;
    int p = parity, x0, y0, zf, zl;
    if (items) {
        const Item it = items[id];
        B = blocks + it.block;
        p = parity ^ it.flip;
        x0 = it.x0;
        y0 = it.y0;
        zf = it.z0 + 1;
        zl = it.z0 + it.zlen;
    } else {
        const int per = tiles_x * tiles_y;
        const int chunk = id / per;
        const int nzb = B->n[2];
        x0 = (id % tiles_x) * (2 * TXP);
        y0 = ((id % per) / tiles_x) * TY;
        zf = (int)((int64_t)chunk * nzb / nch) + 1;
        zl = (int)((int64_t)(chunk + 1) * nzb / nch);
    }
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];

    // this thread's pair (j, r) of the extended region
    const int t = threadIdx.x;
    int j = 0, r = 0;
    bool live = true;
    if (t < NTILE) {
        j = 1 + t % TXP;
        r = 2 + t / TXP;
    } else {
        int q = t - NTILE;
        if (q < 2 * EP) {
            j = q % EP;
            r = q / EP;
        } else if ((q -= 2 * EP) < 2 * EP) {
            j = q % EP;
            r = TY + 2 + q / EP;
        } else if ((q -= 2 * EP) < 2 * TY) {
            j = (q & 1) ? EP - 1 : 0;
            r = 2 + (q >> 1);
        } else {
            live = false;
        }
    }
    const bool tile = t < NTILE;                  // uniform over each wave
    const int xs = x0 - 1 + 2 * j;                // cells xs, xs + 1 (xs odd, >= -1)
    const int ye = y0 - 1 + r;
    const int xs_c = min(xs, nx | 1);             // last pair holding a cell <= nx + 1
    const int ye_c = min(max(ye, 0), ny + 1);
    const bool y_in = ye >= 1 && ye <= ny;
    const bool in_a = live && y_in && xs >= 1 && xs <= nx;
    const bool in_b = live && y_in && xs + 1 >= 1 && xs + 1 <= nx;
    const bool a_ok = tile && ye <= ny && xs <= nx;   // tile cells in the block: stored
    const bool b_ok = tile && ye <= ny && xs + 1 <= nx;
    const int64_t pitch = F::pitch(B);
    const int64_t plane = F::plane(B);
    const int64_t rowoff = (int64_t)ye_c * pitch + xs_c;
    const T* __restrict__ col = F::src(B, p) + rowoff;
    const T* __restrict__ scol = SRC ? F::source(B) + rowoff : nullptr;
    T* __restrict__ dst = F::dst(B, p) + rowoff;

    const int pn = (r + 1) * (LW / 2) + j + 1;    // LDS pair of cells xs, xs + 1
    const int pw = live ? pn : LN / 2;            // the pair this thread writes

    // register rings: iterate k and the source of plane s in slot
    // (s - zf + 1) mod RS, loads issued PD planes ahead; iterate k + 1 of
    // plane s in slot (s - zf + 1) mod 3
    constexpr int PD = 3;
    constexpr int RS = 6;
    const int zhi = min(zl + 2, nz + 1);          // last plane read
    C ua[RS], ub[RS], ba[RS], bb[RS], va[3], vb[3];
#pragma unroll
    for (int k = 0; k < RS; ++k)
        ba[k] = bb[k] = C(0);
    va[0] = vb[0] = va[1] = vb[1] = va[2] = vb[2] = C(0);
    Tr<T>::ld(col + (int64_t)max(zf - 2, 0) * plane, ua[RS - 1], ub[RS - 1]);
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        const int64_t zk = (int64_t)min(zf - 1 + k, zhi) * plane;
        Tr<T>::ld(col + zk, ua[k], ub[k]);
        if (SRC)
            Tr<T>::ld(scol + zk, ba[k], bb[k]);
    }

    const int s_first = zf - 1;
    auto step = [&](int s, auto kc, auto two) {
        constexpr int K = decltype(kc)::value;
        constexpr bool TWO = decltype(two)::value;
        constexpr int SM = (K + RS - 1) % RS, SC = K, SP = (K + 1) % RS, SQ = (K + PD) % RS;
        constexpr int VC = K % 3, VM = (K + 2) % 3, VMM = (K + 1) % 3;
        constexpr int HC = K & 1;
        if (pace)
            pace_wait(pace_t0 + (uint64_t)(s - s_first) * pace);
        const int64_t zq = (int64_t)min(s + PD, zhi) * plane;
        Tr<T>::ld(col + zq, ua[SQ], ub[SQ]);
        if (SRC)
            Tr<T>::ld(scol + zq, ba[SQ], bb[SQ]);
        V* const Ak = A[HC];
        Ak[pw] = V{ua[SC], ub[SC]};
        __syncthreads();
        // iterate k + 1 at plane s
        const V ym = Ak[pn - LW / 2], yp = Ak[pn + LW / 2], xm = Ak[pn - 1], xp = Ak[pn + 1];
        C sa = xm.y + ub[SC];
        sa = sa + ym.x;
        sa = sa + yp.x;
        sa = sa + ua[SM];
        sa = sa + ua[SP];
        C sb = ua[SC] + xp.x;
        sb = sb + ym.y;
        sb = sb + yp.y;
        sb = sb + ub[SM];
        sb = sb + ub[SP];
        C na, nb;
        if (SRC)
            div6_pair(sa + ba[SC], sb + bb[SC], na, nb);
        else
            div6_pair(sa, sb, na, nb);
        const bool z_in = s >= 1 && s <= nz;
        va[VC] = (in_a && z_in) ? storage_round<T>(na) : ua[SC];
        vb[VC] = (in_b && z_in) ? storage_round<T>(nb) : ub[SC];
        Bn[HC][pw] = V{va[VC], vb[VC]};
        // iterate k + 2 at plane s - 1
        if (TWO && tile) {
            const V* const Bk = Bn[HC ^ 1];
            const V ym2 = Bk[pn - LW / 2], yp2 = Bk[pn + LW / 2], xm2 = Bk[pn - 1], xp2 = Bk[pn + 1];
            C qa = xm2.y + vb[VM];
            qa = qa + ym2.x;
            qa = qa + yp2.x;
            qa = qa + va[VMM];
            qa = qa + va[VC];
            C qb = va[VM] + xp2.x;
            qb = qb + ym2.y;
            qb = qb + yp2.y;
            qb = qb + vb[VMM];
            qb = qb + vb[VC];
            C wa2, wb2;
            if (SRC)
                div6_pair(qa + ba[SM], qb + bb[SM], wa2, wb2);
            else
                div6_pair(qa, qb, wa2, wb2);
            // past the last cell of a row the pair's second slot is the
            // x = nx + 1 ghost: write back the value it holds
            wb2 = b_ok ? wb2 : ub[SM];
            if (a_ok)
                Tr<T>::stn(dst + (int64_t)(s - 1) * plane, wa2, wb2);
        }
    };
    using F_ = std::false_type;
    using T_ = std::true_type;
#define JC_STEP2(k) step(s + (k), std::integral_constant<int, ((k) + 2) % RS>{}, T_{})
    int s = zf - 1;
    step(s, std::integral_constant<int, 0>{}, F_{});
    step(s + 1, std::integral_constant<int, 1>{}, F_{});
    s += 2;
    const int s_end = zl + 1;
    for (; s + 5 <= s_end; s += 6) {
        JC_STEP2(0);
        JC_STEP2(1);
        JC_STEP2(2);
        JC_STEP2(3);
        JC_STEP2(4);
        JC_STEP2(5);
    }
    if (s <= s_end) JC_STEP2(0);
    if (s + 1 <= s_end) JC_STEP2(1);
    if (s + 2 <= s_end) JC_STEP2(2);
    if (s + 3 <= s_end) JC_STEP2(3);
    if (s + 4 <= s_end) JC_STEP2(4);
#undef JC_STEP2
}
// ---- two-step sweep: end ----

// ---- three-step sweep (temporal blocking): begin ----
// Three Jacobi sweeps per launch: iterate k from copy p, iterate k + 3 to
// copy p ^ 1; iterates k + 1 and k + 2 live only in LDS and registers.
// The construction of k_sweep2 one level deeper.  Iterate k is loaded on
// a three-cell ring around the tile: TXP + 4 pairs (cells x0 - 3 ..
// x0 + 2 TXP + 4) by TY + 6 rows, one aligned pair per thread.  At plane
// step s every thread writes iterate k of its pair at plane s into LDS,
// the work-group synchronises once, and then
//  - every thread computes iterate k + 1 of its pair at plane s (valid on
//    the tile and a two-cell ring; the outermost values, which would need
//    cells further out, are never read) into LDS plane B;
//  - the threads of the tile and of its one-pair / one-row ring ("mid"
//    threads) compute iterate k + 2 at plane s - 1 from B of the previous
//    step into LDS plane C;
//  - the tile threads compute iterate k + 3 at plane s - 2 from C of the
//    previous step and store it.
// A ghost cell keeps its value at every level (the context has no face
// pairs: every ghost is a fixed boundary value), and iterates k + 1 and
// k + 2 are rounded to the storage format as stored sweeps would leave
// them, so each cell takes the same sums in the same order as in three
// one-step sweeps: the result is bitwise the same.  The three LDS planes
// are double-buffered by step parity, so one barrier per step suffices.
// Thread order: tile threads (whole waves), then the mid ring (rows y0 and
// y0 + TY + 1 over pairs 1 .. TXP + 2, then pairs 1 and TXP + 2 of the tile
// rows), then the rest of the two-cell ring (rows y0 - 1 and y0 + TY + 2
// over pairs 1 .. TXP + 2), then the third ring (the outermost rows, then
// pairs 0 and TXP + 3 of the other rows), whose iterate k + 1 is not
// needed.  Work as for k_sweep2 (items null: the
// tiles of blocks[0]; else a work list of 2 TXP x TY tiles).
template <typename T, int FIELD, int TXP, int TY, bool SRC>
__global__ void __launch_bounds__(((TXP + 4) * (TY + 6) + 63) / 64 * 64)
k_sweep3(const BlockDesc* __restrict__ blocks, const Item* __restrict__ items, int parity, int tiles_x,
         int tiles_y, int nch, int ntiles, uint32_t pace)
{
    using C = typename Tr<T>::C;
    using F = Fld<T, FIELD>;
    constexpr int EP = TXP + 4;                   // pairs of an extended row
    constexpr int ER = TY + 6;                    // extended rows
    constexpr int NTILE = TXP * TY;               // tile threads
    constexpr int NMID = NTILE + 2 * (TXP + 2) + 2 * TY;
    constexpr int NL1 = NMID + 2 * (TXP + 2);
    static_assert(NTILE % 64 == 0, "tile threads are whole waves");
    using V = typename Pair2<C>::V;
    // LDS row: two pad cells, 2 EP cells, two pad cells, so that every
    // thread's pair is one aligned vector: a pair is written with one
    // access and its neighbours' pairs are read with one access each
    constexpr int LW = 2 * EP + 4;
    constexpr int LN = (ER + 2) * LW;             // LDS plane: pad row, ER rows, pad row
    __shared__ V A[2][LN / 2 + 1];                // iterate k; pair LN / 2: sink of idle lanes
    __shared__ V Bn[2][LN / 2 + 1];               // iterate k + 1
    __shared__ V Cn[2][LN / 2 + 1];               // iterate k + 2

    const int id = logical_block(blockIdx.x, gridDim.x);
    if (id >= ntiles)
        return;                                   // uniform over the work-group
    const uint64_t pace_t0 = pace ? __builtin_amdgcn_s_memrealtime() : 0;
    const BlockDesc* B = blocks;
    int p = parity, x0, y0, zf, zl;
    if (items) {
        const Item it = items[id];
        B = blocks + it.block;
        p = parity ^ it.flip;
        x0 = it.x0;
        y0 = it.y0;
        zf = it.z0 + 1;
        zl = it.z0 + it.zlen;
    } else {
        const int per = tiles_x * tiles_y;
        const int chunk = id / per;
        const int nzb = B->n[2];
        x0 = (id % tiles_x) * (2 * TXP);
        y0 = ((id % per) / tiles_x) * TY;
        zf = (int)((int64_t)chunk * nzb / nch) + 1;
        zl = (int)((int64_t)(chunk + 1) * nzb / nch);
    }
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];

    // this thread's pair (j, r) of the extended region
    const int t = threadIdx.x;
    int j = 0, r = 0;
    bool live = true;
    if (t < NTILE) {
        j = 2 + t % TXP;
        r = 3 + t / TXP;
    } else {
        int q = t - NTILE;
        if (q < 2 * (TXP + 2)) {                  // mid rows
            j = 1 + q % (TXP + 2);
            r = q < TXP + 2 ? 2 : TY + 3;
        } else if ((q -= 2 * (TXP + 2)) < 2 * TY) {   // mid pairs of the tile rows
            j = (q & 1) ? TXP + 2 : 1;
            r = 3 + (q >> 1);
        } else if ((q -= 2 * TY) < 2 * (TXP + 2)) {   // second ring: rows 1 and ER - 2
            j = 1 + q % (TXP + 2);
            r = q < TXP + 2 ? 1 : ER - 2;
        } else if ((q -= 2 * (TXP + 2)) < 2 * EP) {   // third ring: rows 0 and ER - 1
            j = q % EP;
            r = q < EP ? 0 : ER - 1;
        } else if ((q -= 2 * EP) < 2 * (ER - 2)) {    // third ring: pairs 0 and EP - 1
            j = (q & 1) ? EP - 1 : 0;
            r = 1 + (q >> 1);
        } else {
            live = false;
        }
    }
    const bool tile = t < NTILE;                  // uniform over each wave
    const bool mid = t < NMID;
    // Iterate k + 1 is needed on the tile and its two-cell ring only (the
    // first NL1 threads); the third ring's threads come last and only load
    // iterate k, so the waves holding none of the first NL1 threads skip the
    // first stage (a wave-uniform branch)
    const bool l1 = (t & ~63) < NL1;
    const int xs = x0 - 3 + 2 * j;                // cells xs, xs + 1 (xs odd, >= -3)
    const int ye = y0 - 2 + r;
    const int xs_c = min(xs, nx | 1);             // last pair holding a cell <= nx + 1
    const int ye_c = min(max(ye, 0), ny + 1);
    const bool y_in = ye >= 1 && ye <= ny;
    const bool in_a = live && y_in && xs >= 1 && xs <= nx;
    const bool in_b = live && y_in && xs + 1 >= 1 && xs + 1 <= nx;
    const bool a_ok = tile && ye <= ny && xs <= nx;   // tile cells in the block: stored
    const bool b_ok = tile && ye <= ny && xs + 1 <= nx;
    const int64_t pitch = F::pitch(B);
    const int64_t plane = F::plane(B);
    const int64_t rowoff = (int64_t)ye_c * pitch + xs_c;
    const T* __restrict__ col = F::src(B, p) + rowoff;
    const T* __restrict__ scol = SRC ? F::source(B) + rowoff : nullptr;
    T* __restrict__ dst = F::dst(B, p) + rowoff;

    const int pn = (r + 1) * (LW / 2) + j + 1;    // LDS pair of cells xs, xs + 1
    const int pw = live ? pn : LN / 2;            // the pair this thread writes

    // register rings: iterate k and the source of plane s in slot
    // (s - zf + 2) mod RS, loads issued PD planes ahead; iterates k + 1 of
    // plane s and k + 2 of plane s - 1 in slot (s - zf + 2) mod 3
    constexpr int PD = 3;
    constexpr int RS = 6;
    const int zlo = max(zf - 3, 0);               // first plane read
    const int zhi = min(zl + 3, nz + 1);          // last plane read
    C ua[RS], ub[RS], ba[RS], bb[RS], va[3], vb[3], wa3[3], wb3[3];
#pragma unroll
    for (int k = 0; k < RS; ++k)
        ba[k] = bb[k] = C(0);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        va[k] = vb[k] = wa3[k] = wb3[k] = C(0);
    Tr<T>::ld(col + (int64_t)zlo * plane, ua[RS - 1], ub[RS - 1]);
    if (SRC)
        Tr<T>::ld(scol + (int64_t)zlo * plane, ba[RS - 1], bb[RS - 1]);
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        const int64_t zk = (int64_t)min(max(zf - 2 + k, 0), zhi) * plane;
        Tr<T>::ld(col + zk, ua[k], ub[k]);
        if (SRC)
            Tr<T>::ld(scol + zk, ba[k], bb[k]);
    }

    // STAGES: 1 = iterate k + 1 only, 2 = also k + 2, 3 = also k + 3
    const int s_first = zf - 2;
    auto step = [&](int s, auto kc, auto stages) {
        constexpr int K = decltype(kc)::value;
        constexpr int ST = decltype(stages)::value;
        constexpr int SM = (K + RS - 1) % RS, SC = K, SP = (K + 1) % RS, SQ = (K + PD) % RS;
        constexpr int S2 = (K + RS - 2) % RS;     // plane s - 2
        constexpr int VC = K % 3, VM = (K + 2) % 3, VMM = (K + 1) % 3;
        constexpr int HC = K & 1;
        if (pace)
            pace_wait(pace_t0 + (uint64_t)(s - s_first) * pace);
        const int64_t zq = (int64_t)min(s + PD, zhi) * plane;
        Tr<T>::ld(col + zq, ua[SQ], ub[SQ]);
        if (SRC)
            Tr<T>::ld(scol + zq, ba[SQ], bb[SQ]);
        V* const Ak = A[HC];
        Ak[pw] = V{ua[SC], ub[SC]};
        __syncthreads();
        // iterate k + 1 at plane s
        if (l1) {
            const V ym = Ak[pn - LW / 2], yp = Ak[pn + LW / 2], xm = Ak[pn - 1], xp = Ak[pn + 1];
            C sa = xm.y + ub[SC];
            sa = sa + ym.x;
            sa = sa + yp.x;
            sa = sa + ua[SM];
            sa = sa + ua[SP];
            C sb = ua[SC] + xp.x;
            sb = sb + ym.y;
            sb = sb + yp.y;
            sb = sb + ub[SM];
            sb = sb + ub[SP];
            C na, nb;
            if (SRC)
                div6_pair(sa + ba[SC], sb + bb[SC], na, nb);
            else
                div6_pair(sa, sb, na, nb);
            const bool z_in = s >= 1 && s <= nz;
            va[VC] = (in_a && z_in) ? storage_round<T>(na) : ua[SC];
            vb[VC] = (in_b && z_in) ? storage_round<T>(nb) : ub[SC];
            Bn[HC][pw] = V{va[VC], vb[VC]};
        }
        // iterate k + 2 at plane s - 1
        if (ST >= 2 && mid) {
            const V* const Bk = Bn[HC ^ 1];
            const V ym = Bk[pn - LW / 2], yp = Bk[pn + LW / 2], xm = Bk[pn - 1], xp = Bk[pn + 1];
            C qa = xm.y + vb[VM];
            qa = qa + ym.x;
            qa = qa + yp.x;
            qa = qa + va[VMM];
            qa = qa + va[VC];
            C qb = va[VM] + xp.x;
            qb = qb + ym.y;
            qb = qb + yp.y;
            qb = qb + vb[VMM];
            qb = qb + vb[VC];
            C na, nb;
            if (SRC)
                div6_pair(qa + ba[SM], qb + bb[SM], na, nb);
            else
                div6_pair(qa, qb, na, nb);
            const bool z_in = s - 1 >= 1 && s - 1 <= nz;
            wa3[VC] = (in_a && z_in) ? storage_round<T>(na) : va[VM];
            wb3[VC] = (in_b && z_in) ? storage_round<T>(nb) : vb[VM];
            Cn[HC][pw] = V{wa3[VC], wb3[VC]};
        }
        // iterate k + 3 at plane s - 2
        if (ST >= 3 && tile) {
            const V* const Ck = Cn[HC ^ 1];
            const V ym = Ck[pn - LW / 2], yp = Ck[pn + LW / 2], xm = Ck[pn - 1], xp = Ck[pn + 1];
            C qa = xm.y + wb3[VM];
            qa = qa + ym.x;
            qa = qa + yp.x;
            qa = qa + wa3[VMM];
            qa = qa + wa3[VC];
            C qb = wa3[VM] + xp.x;
            qb = qb + ym.y;
            qb = qb + yp.y;
            qb = qb + wb3[VMM];
            qb = qb + wb3[VC];
            C oa, ob;
            if (SRC)
                div6_pair(qa + ba[S2], qb + bb[S2], oa, ob);
            else
                div6_pair(qa, qb, oa, ob);
            // past the last cell of a row the pair's second slot is the
            // x = nx + 1 ghost: write back the value it holds
            ob = b_ok ? ob : ub[S2];
            if (a_ok)
                Tr<T>::stn(dst + (int64_t)(s - 2) * plane, oa, ob);
        }
    };
    using One = std::integral_constant<int, 1>;
    using Two = std::integral_constant<int, 2>;
    using Three = std::integral_constant<int, 3>;
    int s = zf - 2;
    step(s, std::integral_constant<int, 0>{}, One{});
    step(s + 1, std::integral_constant<int, 1>{}, One{});
    step(s + 2, std::integral_constant<int, 2>{}, Two{});
    step(s + 3, std::integral_constant<int, 3>{}, Two{});
    s += 4;
#define JC_STEP3(k) step(s + (k), std::integral_constant<int, ((k) + 4) % RS>{}, Three{})
    const int s_end = zl + 2;
    for (; s + 5 <= s_end; s += 6) {
        JC_STEP3(0);
        JC_STEP3(1);
        JC_STEP3(2);
        JC_STEP3(3);
        JC_STEP3(4);
        JC_STEP3(5);
    }
    if (s <= s_end) JC_STEP3(0);
    if (s + 1 <= s_end) JC_STEP3(1);
    if (s + 2 <= s_end) JC_STEP3(2);
    if (s + 3 <= s_end) JC_STEP3(3);
    if (s + 4 <= s_end) JC_STEP3(4);
#undef JC_STEP3
}
// ---- three-step sweep: end ----

// ---- resident sweeps: many sweeps of a small block in one launch ----
//
// The on-chip small-grid solver for the Jacobi sweep of paper section 4.3
// (not a design of the paper: its blocks are swept once per launch and
// exchange halos between sweeps): one work-group holds a whole block of
// at most 32 planes and (nx + 1) / 2 * ny <= 512 cell pairs and runs any
// number of Jacobi sweeps on it without leaving the compute unit, so a
// small solve costs one launch per window instead of one per sweep (or
// per two or three), and the block's cells cross HBM once per launch.
//
// Each thread owns the z columns of two adjacent x cells of one row, in
// registers (element z of the column arrays is plane z; 0 the bottom
// ghost plane; the top ghost plane is kept apart because its index is
// not a compile-time constant).  A sweep marches up the columns two
// planes at a time: every thread writes its iterate-k pairs of planes z
// and z + 1 into two LDS plane buffers, synchronises once, reads its x
// and y neighbours in both planes and forms both updates with the same
// sums in the same order as every other sweep kernel, so results are
// bitwise those of one-sweep launches.  Within a sweep the planes depend
// on iterate k only, so the two planes' dependent chains of additions
// and the division run interleaved; the step is bound by that latency
// and by the LDS round trip, not by bandwidth.  The buffers come in two
// sets that alternate every step, so one barrier per step suffices.  The
// update of plane z + 1 cannot overwrite the column yet (plane z + 2
// still needs its old value), so it waits one step in a register.
//
// The ghost cells around each plane never change: they are copied into
// LDS once (the x = 0 and x = nx + 1 columns and the y = 0 and y = ny + 1
// rows of every plane), and a thread on the block's edge reads its
// neighbour from there instead of from a plane buffer.  The source b is
// re-read from global memory (L2) every sweep, two steps ahead.
//
// Steps are unrolled two sweeps at a time so that the buffer set and the
// source register slot of every step are compile-time constants (step s
// of the launch uses set s & 1; NBODD is the parity of the number of
// steps per sweep, (nz + 1) / 2).

template <int I, int N, typename F>
__device__ __forceinline__ void resident_steps(F& f)
{
    if constexpr (I < N) {
        if (f(std::integral_constant<int, I>{}))
            resident_steps<I + 1, N>(f);
    }
}

template <bool SRC, int NBODD>
__global__ void __launch_bounds__(512)
k_resident(const BlockDesc* __restrict__ blocks, const Item* __restrict__ items, int parity, int nsweeps)
{
    constexpr int NZM = kResidentMaxPlanes;
    extern __shared__ v2d lds_pairs[];
    double* const lds = reinterpret_cast<double*>(lds_pairs);
    const int blk = items ? items[blockIdx.x].block : 0;
    const int p0 = parity ^ (items ? items[blockIdx.x].flip : 0);
    const BlockDesc* B = blocks + blk;
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    const int nb = (nz + 1) >> 1;             // steps per sweep
    const int ep = (nx + 1) >> 1;             // cell pairs per row
    const int pw = 2 * ep;                    // LDS row length
    const int ps = ny * pw;                   // LDS plane buffer length
    const int64_t pitch = B->pitch, plane = B->plane;
    const double* __restrict__ u = B->u[p0];
    double* const P = lds;                    // [2 sets][2 planes][ny][pw]
    double* const RXM = P + 4 * ps;           // [nz][ny]     x = 0
    double* const RXP = RXM + nz * ny;        // [nz][ny]     x = nx + 1
    double* const RYM = RXP + nz * ny;        // [nz][pw]     y = 0
    double* const RYP = RYM + nz * pw;        // [nz][pw]     y = ny + 1
    const int t = threadIdx.x;
    for (int i = t; i < nz * ny; i += blockDim.x) {
        const int64_t o = (int64_t)(i / ny + 1) * plane + (int64_t)(i % ny + 1) * pitch;
        RXM[i] = u[o];
        RXP[i] = u[o + nx + 1];
    }
    for (int i = t; i < nz * pw; i += blockDim.x) {
        const int64_t o = (int64_t)(i / pw + 1) * plane + (i % pw + 1);
        RYM[i] = u[o];
        RYP[i] = u[o + (int64_t)(ny + 1) * pitch];
    }
    const bool live = t < ep * ny;
    const int j = live ? t % ep : 0, y0 = live ? t / ep : 0;
    const bool b_ok = 2 * j + 2 <= nx;        // else the pair's second cell is the x = nx + 1 ghost
    const int64_t own = (int64_t)(y0 + 1) * pitch + 2 * j + 1;

    // LDS offsets of the neighbours in plane 1: in plane buffer 0, or on
    // the block's edge in the ghost ring of plane 1.  Buffer k is k * sb
    // further (sb = 0 on a ring), plane z of a ring (z - 1) * sx further
    // (sx = 0 in the buffers).
    const bool xm_ring = j == 0, xp_ring = j == ep - 1, ym_ring = y0 == 0, yp_ring = y0 == ny - 1;
    const int row = y0 * pw + 2 * j;
    const int o_xm = xm_ring ? 4 * ps + y0 : row - 1;
    const int o_xp = xp_ring ? 4 * ps + nz * ny + y0 : row + 2;
    const int o_ym = ym_ring ? 4 * ps + 2 * nz * ny + 2 * j : row - pw;
    const int o_yp = yp_ring ? 4 * ps + 2 * nz * ny + nz * pw + 2 * j : row + pw;
    const int sx_xm = xm_ring ? ny : 0, sb_xm = xm_ring ? 0 : ps;
    const int sx_xp = xp_ring ? ny : 0, sb_xp = xp_ring ? 0 : ps;
    const int sx_ym = ym_ring ? pw : 0, sb_ym = ym_ring ? 0 : ps;
    const int sx_yp = yp_ring ? pw : 0, sb_yp = yp_ring ? 0 : ps;
    v2d* const w0 = reinterpret_cast<v2d*>(P + row);

    double ca[NZM + 2], cb[NZM + 2];
    {
        const v2d g = *(const v2d JC_GLOBAL*)(u + own);
        ca[0] = g.x;
        cb[0] = g.y;
    }
#pragma unroll
    for (int z = 1; z <= NZM; ++z) {
        if (z <= nz) {
            const v2d v = *(const v2d JC_GLOBAL*)(u + (int64_t)z * plane + own);
            ca[z] = v.x;
            cb[z] = v.y;
        } else {
            ca[z] = cb[z] = 0.0;
        }
    }
    ca[NZM + 1] = cb[NZM + 1] = 0.0;
    double ta, tb;                            // the z = nz + 1 ghosts
    {
        const v2d g = *(const v2d JC_GLOBAL*)(u + (int64_t)(nz + 1) * plane + own);
        ta = g.x;
        tb = g.y;
    }
    // source of the two planes of step s in slot s & 1, loaded two steps
    // ahead (the second plane of a one-plane step repeats the first)
    const int own32 = (int)own;
    double qa[2][2] = {}, qb[2][2] = {};
    auto load_src = [&](int step, double* da, double* db) __attribute__((always_inline)) {
        while (step >= nb)
            step -= nb;
        const int z1 = 2 * step + 1, z2 = z1 + 1 <= nz ? z1 + 1 : z1;
        const v2d q1 = *(const v2d JC_GLOBAL*)(B->b + (int64_t)z1 * plane + own32);
        const v2d q2 = *(const v2d JC_GLOBAL*)(B->b + (int64_t)z2 * plane + own32);
        da[0] = q1.x;
        db[0] = q1.y;
        da[1] = q2.x;
        db[1] = q2.y;
    };
    if (SRC) {
        load_src(0, qa[0], qb[0]);
        load_src(1, qa[1], qb[1]);
    }
    __syncthreads();                          // ghost rings written

    double pa = 0.0, pb = 0.0;                // the update of the plane below, not yet stored
    auto sweep = [&](auto hc) __attribute__((always_inline)) {
        constexpr int H = decltype(hc)::value;
        // running ring offsets of the step's first plane, opaque to the
        // compiler: otherwise it hoists the address of every step out of
        // the sweep loop and holds them all in registers
        int r_xm = o_xm, r_xp = o_xp, r_ym = o_ym, r_yp = o_yp;
        asm volatile("" : "+v"(r_xm), "+v"(r_xp), "+v"(r_ym), "+v"(r_yp));
        auto step = [&](auto ic) __attribute__((always_inline)) -> bool {
            constexpr int I = decltype(ic)::value;
            constexpr int Z = 2 * I + 1;      // the step's first plane
            if (Z > nz)
                return false;
            constexpr int SET = (I + H * NBODD) & 1;
            double s1a = 0.0, s1b = 0.0, s2a = 0.0, s2b = 0.0;
            if (SRC) {
                s1a = qa[SET][0];
                s1b = qb[SET][0];
                s2a = qa[SET][1];
                s2b = qb[SET][1];
                load_src(I + 2, qa[SET], qb[SET]);
            }
            // TWO: planes Z and Z + 1 (else Z alone, the top plane);
            // TOP: the step's last plane is the top plane nz
            auto body = [&](auto twoc, auto topc) __attribute__((always_inline)) {
                constexpr bool TWO = decltype(twoc)::value, TOP = decltype(topc)::value;
                if (live) {
                    v2d w;
                    w.x = ca[Z];
                    w.y = cb[Z];
                    w0[(2 * SET) * (ps / 2)] = w;
                    if (TWO) {
                        w.x = ca[Z + 1];
                        w.y = cb[Z + 1];
                        w0[(2 * SET + 1) * (ps / 2)] = w;
                    }
                }
                __syncthreads();
                const double xm1 = lds[r_xm + (2 * SET) * sb_xm];
                const double xp1 = lds[r_xp + (2 * SET) * sb_xp];
                const v2d ym1 = *reinterpret_cast<const v2d*>(lds + r_ym + (2 * SET) * sb_ym);
                const v2d yp1 = *reinterpret_cast<const v2d*>(lds + r_yp + (2 * SET) * sb_yp);
                double xm2 = 0.0, xp2 = 0.0;
                v2d ym2 = {0.0, 0.0}, yp2 = {0.0, 0.0};
                if (TWO) {
                    xm2 = lds[r_xm + sx_xm + (2 * SET + 1) * sb_xm];
                    xp2 = lds[r_xp + sx_xp + (2 * SET + 1) * sb_xp];
                    ym2 = *reinterpret_cast<const v2d*>(lds + r_ym + sx_ym + (2 * SET + 1) * sb_ym);
                    yp2 = *reinterpret_cast<const v2d*>(lds + r_yp + sx_yp + (2 * SET + 1) * sb_yp);
                }
                // plane Z
                const double a1 = ca[Z], b1 = cb[Z];
                double sa1 = xm1 + b1;
                sa1 = sa1 + ym1.x;
                sa1 = sa1 + yp1.x;
                sa1 = sa1 + ca[Z - 1];
                sa1 = sa1 + (TWO ? ca[Z + 1] : ta);
                double sb1 = a1 + xp1;
                sb1 = sb1 + ym1.y;
                sb1 = sb1 + yp1.y;
                sb1 = sb1 + cb[Z - 1];
                sb1 = sb1 + (TWO ? cb[Z + 1] : tb);
                double va1, vb1;
                if (SRC)
                    div6_pair(sa1 + s1a, sb1 + s1b, va1, vb1);
                else
                    div6_pair(sa1, sb1, va1, vb1);
                vb1 = b_ok ? vb1 : b1;
                if (TWO) {
                    // plane Z + 1
                    const double a2 = ca[Z + 1], b2 = cb[Z + 1];
                    double sa2 = xm2 + b2;
                    sa2 = sa2 + ym2.x;
                    sa2 = sa2 + yp2.x;
                    sa2 = sa2 + a1;
                    sa2 = sa2 + (TOP ? ta : ca[Z + 2]);
                    double sb2 = a2 + xp2;
                    sb2 = sb2 + ym2.y;
                    sb2 = sb2 + yp2.y;
                    sb2 = sb2 + b1;
                    sb2 = sb2 + (TOP ? tb : cb[Z + 2]);
                    double va2, vb2;
                    if (SRC)
                        div6_pair(sa2 + s2a, sb2 + s2b, va2, vb2);
                    else
                        div6_pair(sa2, sb2, va2, vb2);
                    vb2 = b_ok ? vb2 : b2;
                    if (Z > 1) {
                        ca[Z - 1] = pa;
                        cb[Z - 1] = pb;
                    }
                    ca[Z] = va1;
                    cb[Z] = vb1;
                    pa = va2;
                    pb = vb2;
                    if (TOP) {
                        ca[Z + 1] = va2;
                        cb[Z + 1] = vb2;
                    }
                } else {
                    if (Z > 1) {
                        ca[Z - 1] = pa;
                        cb[Z - 1] = pb;
                    }
                    ca[Z] = va1;
                    cb[Z] = vb1;
                }
            };
            if constexpr (Z + 1 <= NZM) {
                if (Z + 1 < nz)
                    body(std::true_type{}, std::false_type{});
                else if (Z + 1 == nz)
                    body(std::true_type{}, std::true_type{});
                else
                    body(std::false_type{}, std::true_type{});
            } else {
                body(std::false_type{}, std::true_type{});
            }
            r_xm += 2 * sx_xm;
            r_xp += 2 * sx_xp;
            r_ym += 2 * sx_ym;
            r_yp += 2 * sx_yp;
            return true;
        };
        resident_steps<0, (NZM + 1) / 2>(step);
    };
    for (int k = 0; k < nsweeps; k += 2) {
        sweep(std::integral_constant<int, 0>{});
        if (k + 1 < nsweeps)
            sweep(std::integral_constant<int, 1>{});
    }

    double* const dst = B->u[p0 ^ (nsweeps & 1)];
    if (live) {
#pragma unroll
        for (int z = 1; z <= NZM; ++z) {
            if (z <= nz) {
                v2d v;
                v.x = ca[z];
                v.y = cb[z];
                *(v2d JC_GLOBAL*)(dst + (int64_t)z * plane + own) = v;
            }
        }
    }
}
// ---- resident sweeps: end ----

// First inner sweep of a refinement step: d_1 = lo((0 + r_lo) / 6)
// (d_0 = 0, so no neighbour is read); writes copy 1 of d and its faces.
template <typename T>
__global__ void __launch_bounds__(256)
k_ir_first(const BlockDesc* __restrict__ blocks)
{
    using C = typename Tr<T>::C;
    const BlockDesc* B = blocks + blockIdx.y;
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    const int64_t lp = B->lpitch, ll = B->lplane;
    const int64_t ldx = face_ld(ny), ldy = face_ld(nx);
    const T* rl = static_cast<const T*>(B->rlo);
    T* d = static_cast<T*>(B->d[1]);
    const int npair = (nx + 1) / 2;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % ny) + 1;
        const int z = (int)(r / ny) + 1;
        for (int k = threadIdx.x; k < npair; k += 256) {
            const int xa = 2 * k + 1;
            const bool b_ok = xa + 1 <= nx;
            const int64_t at = (int64_t)z * ll + (int64_t)y * lp + xa;
            C sa, sb;
            Tr<T>::ld(rl + at, sa, sb);
            const C zero = C(0);
            const C va = div6(zero + sa);
            const C vb = div6(zero + sb);
            C ga, gb;
            Tr<T>::ld(static_cast<const T*>(B->d[1]) + at, ga, gb);   // keeps the x = nx + 1 ghost
            Tr<T>::st(d + at, va, b_ok ? vb : gb);
            T* oxm = static_cast<T*>(B->lgout[XM][1]);
            T* oxp = static_cast<T*>(B->lgout[XP][1]);
            T* oym = static_cast<T*>(B->lgout[YM][1]);
            T* oyp = static_cast<T*>(B->lgout[YP][1]);
            T* ozm = static_cast<T*>(B->lgout[ZM][1]);
            T* ozp = static_cast<T*>(B->lgout[ZP][1]);
            const int64_t xfi = (int64_t)(z - 1) * ldx + (y - 1);
            const int64_t yfi = (int64_t)(z - 1) * ldy + (xa - 1);
            const int64_t zfi = (int64_t)(y - 1) * ldy + (xa - 1);
            if (xa == 1 && oxm) Tr<T>::st1(oxm + xfi, va);
            if (xa == nx && oxp) Tr<T>::st1(oxp + xfi, va);
            if (b_ok && xa + 1 == nx && oxp) Tr<T>::st1(oxp + xfi, vb);
            if (y == 1 && oym) Tr<T>::st(oym + yfi, va, vb);
            if (y == ny && oyp) Tr<T>::st(oyp + yfi, va, vb);
            if (z == 1 && ozm) Tr<T>::st(ozm + zfi, va, vb);
            if (z == nz && ozp) Tr<T>::st(ozp + zfi, va, vb);
        }
    }
}

// Outer update of the refinement: u(copy p) += (double) d(copy q) on the
// interior; the updated face cells go to the u face buffers of slot p.
template <typename T>
__global__ void __launch_bounds__(256)
k_ir_update(const BlockDesc* __restrict__ blocks, int p, int q)
{
    using C = typename Tr<T>::C;
    const BlockDesc* B = blocks + blockIdx.y;
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    const int64_t ldx = face_ld(ny), ldy = face_ld(nx);
    double* u = B->u[p];
    const T* d = static_cast<const T*>(B->d[q]);
    const int npair = (nx + 1) / 2;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % ny) + 1;
        const int z = (int)(r / ny) + 1;
        for (int k = threadIdx.x; k < npair; k += 256) {
            const int xa = 2 * k + 1;
            const bool b_ok = xa + 1 <= nx;
            double* up = u + (int64_t)z * B->plane + (int64_t)y * B->pitch + xa;
            double ua, ub;
            Tr<double>::ld(up, ua, ub);
            C da, db;
            Tr<T>::ld(d + (int64_t)z * B->lplane + (int64_t)y * B->lpitch + xa, da, db);
            const double va = ua + (double)da;
            const double vb = b_ok ? ub + (double)db : ub;
            Tr<double>::st(up, va, vb);
            double* oxm = B->gout[XM][p];
            double* oxp = B->gout[XP][p];
            double* oym = B->gout[YM][p];
            double* oyp = B->gout[YP][p];
            double* ozm = B->gout[ZM][p];
            double* ozp = B->gout[ZP][p];
            const int64_t xfi = (int64_t)(z - 1) * ldx + (y - 1);
            const int64_t yfi = (int64_t)(z - 1) * ldy + (xa - 1);
            const int64_t zfi = (int64_t)(y - 1) * ldy + (xa - 1);
            if (xa == 1 && oxm) Tr<double>::st1(oxm + xfi, va);
            if (xa == nx && oxp) Tr<double>::st1(oxp + xfi, va);
            if (b_ok && xa + 1 == nx && oxp) Tr<double>::st1(oxp + xfi, vb);
            if (y == 1 && oym) Tr<double>::st(oym + yfi, va, vb);
            if (y == ny && oyp) Tr<double>::st(oyp + yfi, va, vb);
            if (z == 1 && ozm) Tr<double>::st(ozm + zfi, va, vb);
            if (z == nz && ozp) Tr<double>::st(ozp + zfi, va, vb);
        }
    }
}

// Zero `words` 8-byte words at p (grid-stride).
__global__ void __launch_bounds__(256)
k_zero(uint64_t* __restrict__ p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
        *(uint64_t JC_GLOBAL*)(p + i) = 0;
}

// Fixed-order sum of one member's partials [ranges[2m], ranges[2m+1]):
// each thread adds a strided subsequence in order, then a fixed tree over
// the work-group.
__global__ void __launch_bounds__(256)
k_reduce(const double* __restrict__ partials, const int32_t* __restrict__ ranges,
         double* __restrict__ out)
{
    const int m = blockIdx.x;
    const int lo = ranges[2 * m], hi = ranges[2 * m + 1];
    double t = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256)
        t = t + partials[i];
    __shared__ double w[4];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0)
        w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0)
        out[m] = ((w[0] + w[1]) + w[2]) + w[3];
}

// Address of the cell (slow, fast) of the plane of face f, at depth
// `ghost` (0: the outermost interior plane, 1: the ghost plane beyond it).
__device__ __forceinline__ int64_t face_cell(const BlockDesc& B, int f, int slow, int fast, int ghost)
{
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    int x, y, z;
    switch (f) {
    case XM: x = ghost ? 0 : 1;            y = fast + 1; z = slow + 1; break;
    case XP: x = ghost ? nx + 1 : nx;      y = fast + 1; z = slow + 1; break;
    case YM: y = ghost ? 0 : 1;            x = fast + 1; z = slow + 1; break;
    case YP: y = ghost ? ny + 1 : ny;      x = fast + 1; z = slow + 1; break;
    case ZM: z = ghost ? 0 : 1;            x = fast + 1; y = slow + 1; break;
    default: z = ghost ? nz + 1 : nz;      x = fast + 1; y = slow + 1; break;
    }
    return (int64_t)z * B.plane + (int64_t)y * B.pitch + x;
}

__global__ void __launch_bounds__(256)
k_pack(const BlockDesc* __restrict__ blocks, const PairDesc* __restrict__ pairs, int parity, int slot)
{
    const PairDesc& P = pairs[blockIdx.z];
    const int slow = blockIdx.y;
    const int fast = blockIdx.x * 256 + threadIdx.x;
    if (slow >= P.slow || fast >= P.fast)
        return;
    const BlockDesc& B = blocks[P.src_block];
    P.buf[slot][(int64_t)slow * face_ld(P.fast) + fast] = B.u[parity][face_cell(B, P.src_face, slow, fast, 0)];
}

__global__ void __launch_bounds__(256)
k_unpack(const BlockDesc* __restrict__ blocks, const PairDesc* __restrict__ pairs, int parity)
{
    const PairDesc& P = pairs[blockIdx.z];
    const int slow = blockIdx.y;
    const int fast = blockIdx.x * 256 + threadIdx.x;
    if (slow >= P.slow || fast >= P.fast)
        return;
    const BlockDesc& B = blocks[P.dst_block];
    B.u[parity][face_cell(B, P.dst_face, slow, fast, 1)] = P.buf[1][(int64_t)slow * face_ld(P.fast) + fast];
}

// The pairing's transfer: every send buffer into the receive buffer
// pre-posted for it.  Buffers are 256-byte aligned with an even number of
// elements: 16-byte vectors.
__global__ void __launch_bounds__(256)
k_exchange(const PairDesc* __restrict__ pairs)
{
    const PairDesc& P = pairs[blockIdx.y];
    const int64_t n2 = P.span >> 1;
    const double2* __restrict__ a = reinterpret_cast<const double2*>(P.buf[0]);
    double2* __restrict__ b = reinterpret_cast<double2*>(P.buf[1]);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (int64_t)gridDim.x * 256)
        b[i] = a[i];
}

// Rows of every block's padded array: blockIdx.y = block; the work-group
// walks rows (z, y) with a stride, lanes cover x in [0, nx+1].
__global__ void __launch_bounds__(256)
k_scatter(const BlockDesc* __restrict__ blocks, const double* __restrict__ g, int64_t gnx,
          int64_t gny, int which)
{
    const BlockDesc& B = blocks[blockIdx.y];
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    const int64_t gpitch = gnx + 2, gplane = (gnx + 2) * (gny + 2);
    const int64_t rows = (int64_t)(ny + 2) * (nz + 2);
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % (ny + 2));
        const int z = (int)(r / (ny + 2));
        const int64_t grow = (int64_t)(B.off[2] + z) * gplane + (int64_t)(B.off[1] + y) * gpitch + B.off[0];
        const int64_t brow = (int64_t)z * B.plane + (int64_t)y * B.pitch;
        const bool col_row = y >= 1 && y <= ny && z >= 1 && z <= nz;
        const int64_t col_at = (int64_t)(z - 1) * face_ld(ny) + (y - 1);
        for (int x = threadIdx.x; x < nx + 2; x += 256) {
            const double v = g[grow + x];
            if (which == 0) {
                B.u[0][brow + x] = v;
                B.u[1][brow + x] = v;
                // the compact Dirichlet ghost columns of unpaired x faces
                if (col_row && x == 0 && B.xg[XM])
                    const_cast<double*>(B.xg[XM])[col_at] = v;
                if (col_row && x == nx + 1 && B.xg[XP])
                    const_cast<double*>(B.xg[XP])[col_at] = v;
            } else {
                const_cast<double*>(B.b)[brow + x] = v;
            }
        }
    }
}

// Interior cells, plus the cells on the global Dirichlet shell.
__global__ void __launch_bounds__(256)
k_gather(const BlockDesc* __restrict__ blocks, double* __restrict__ g, int64_t gnx, int64_t gny,
         int64_t gnz, int which, int parity)
{
    const BlockDesc& B = blocks[blockIdx.y];
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    const int64_t gpitch = gnx + 2, gplane = (gnx + 2) * (gny + 2);
    const int64_t rows = (int64_t)(ny + 2) * (nz + 2);
    const double* src = which == 0 ? B.u[parity] : B.b;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % (ny + 2));
        const int z = (int)(r / (ny + 2));
        const int64_t gy = B.off[1] + y, gz = B.off[2] + z;
        const bool rowin = (y >= 1 && y <= ny && z >= 1 && z <= nz);
        const bool rowshell = (gy == 0 || gy == gny + 1 || gz == 0 || gz == gnz + 1);
        const int64_t grow = gz * gplane + gy * gpitch + B.off[0];
        const int64_t brow = (int64_t)z * B.plane + (int64_t)y * B.pitch;
        for (int x = threadIdx.x; x < nx + 2; x += 256) {
            const int64_t gx = B.off[0] + x;
            const bool in = rowin && x >= 1 && x <= nx;
            const bool shell = rowshell || gx == 0 || gx == gnx + 1;
            if (in || shell)
                g[grow + x] = src[brow + x];
        }
    }
}

// Row kernels: one work-group per row of the largest block, up to 16384.
dim3 row_grid(int nblocks, int64_t max_rows)
{
    int64_t per = max_rows;
    if (per > 16384) per = 16384;
    if (per < 1) per = 1;
    return dim3((unsigned)per, (unsigned)nblocks);
}

}  // namespace

hipError_t launch_sweep(const BlockDesc* blocks, const Item* items, int nitems, int parity,
                        int tile_x, int tile_y, bool fused, bool resid, bool store, bool src, double* partials,
                        hipStream_t s, uint32_t pace)
{
    if (nitems <= 0)
        return hipSuccess;
    return src ? sweep_tiles<double, FIELD_U, true, NoRlo>(blocks, items, nitems, parity, tile_x, tile_y, fused,
                                                             resid, store, partials, s, pace)
               : sweep_tiles<double, FIELD_U, false, NoRlo>(blocks, items, nitems, parity, tile_x, tile_y, fused,
                                                              resid, store, partials, s, pace);
}

hipError_t launch_sweep2(const BlockDesc* blocks, int nx, int ny, int nz, int parity, int tile_y, int z_chunk,
                         bool src, hipStream_t s, uint32_t pace)
{
    if (nx < 1 || ny < 1 || nz < 1 || z_chunk < 1)
        return hipErrorInvalidValue;
    const int64_t tx = (nx + 63) / 64, ty = (ny + tile_y - 1) / tile_y, nch = (nz + z_chunk - 1) / z_chunk;
    const int64_t n = tx * ty * nch;
    if (n > ((int64_t)1 << 30))
        return hipErrorInvalidValue;
    const int grid = (int)((n + 7) / 8 * 8);
#define JC_SWEEP2_CASE(TY, SRC)                                                                               \
    if (tile_y == TY && src == SRC) {                                                                        \
        hipLaunchKernelGGL((k_sweep2<double, FIELD_U, 32, TY, SRC>), dim3(grid), dim3((34 * (TY + 4) + 63) / 64 * 64), \
                           0, s, blocks, nullptr, parity, (int)tx, (int)ty, (int)nch, (int)n, pace);         \
        return hipGetLastError();                                                                            \
    }
    JC_SWEEP2_CASE(8, false)
    JC_SWEEP2_CASE(8, true)
    JC_SWEEP2_CASE(16, false)
    JC_SWEEP2_CASE(16, true)
    JC_SWEEP2_CASE(24, false)
    JC_SWEEP2_CASE(24, true)
#undef JC_SWEEP2_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sweep2_items(const BlockDesc* blocks, const Item* items, int nitems, int parity, int tile_y,
                               bool src, hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
    const int grid = ((nitems + 7) / 8) * 8;
#define JC_SWEEP2_ITEMS_CASE(TY, SRC)                                                                          \
    if (tile_y == TY && src == SRC) {                                                                         \
        hipLaunchKernelGGL((k_sweep2<double, FIELD_U, 32, TY, SRC>), dim3(grid), dim3((34 * (TY + 4) + 63) / 64 * 64), \
                           0, s, blocks, items, parity, 0, 0, 0, nitems, 0u);                                 \
        return hipGetLastError();                                                                             \
    }
    JC_SWEEP2_ITEMS_CASE(8, false)
    JC_SWEEP2_ITEMS_CASE(8, true)
    JC_SWEEP2_ITEMS_CASE(16, false)
    JC_SWEEP2_ITEMS_CASE(16, true)
    JC_SWEEP2_ITEMS_CASE(24, false)
    JC_SWEEP2_ITEMS_CASE(24, true)
#undef JC_SWEEP2_ITEMS_CASE
    return hipErrorInvalidValue;
}

// Three sweeps per launch (k_sweep3): the binary64 iterate, or the
// refinement correction (lo_dtype 0/1/2); tiles of 64 cells by tile_y (8 or
// 16) rows; items null: the tiles of blocks[0] in z chunks of z_chunk planes.
template <typename T, int FIELD, int TY, bool SRC>
hipError_t sweep3_launch(const BlockDesc* blocks, const Item* items, int parity, int tx, int ty, int nch, int n,
                         hipStream_t s, uint32_t pace)
{
    const int grid = ((n + 7) / 8) * 8;
    hipLaunchKernelGGL((k_sweep3<T, FIELD, 32, TY, SRC>), dim3(grid), dim3((36 * (TY + 6) + 63) / 64 * 64), 0, s,
                       blocks, items, parity, tx, ty, nch, n, pace);
    return hipGetLastError();
}

template <typename T, int FIELD, bool SRC>
hipError_t sweep3_rows(const BlockDesc* blocks, const Item* items, int parity, int tile_y, int tx, int ty, int nch,
                       int n, hipStream_t s, uint32_t pace)
{
    if (tile_y == 8)
        return sweep3_launch<T, FIELD, 8, SRC>(blocks, items, parity, tx, ty, nch, n, s, pace);
    if (tile_y == 16)
        return sweep3_launch<T, FIELD, 16, SRC>(blocks, items, parity, tx, ty, nch, n, s, pace);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep3(const BlockDesc* blocks, const Item* items, int nitems, int nx, int ny, int nz, int parity,
                         int tile_y, int z_chunk, bool src, hipStream_t s, uint32_t pace)
{
    int64_t tx = 0, ty = 0, nch = 0, n = nitems;
    if (!items) {
        if (nx < 1 || ny < 1 || nz < 1 || z_chunk < 1 || tile_y < 1)
            return hipErrorInvalidValue;
        tx = (nx + 63) / 64;
        ty = (ny + tile_y - 1) / tile_y;
        nch = (nz + z_chunk - 1) / z_chunk;
        n = tx * ty * nch;
    }
    if (n <= 0)
        return hipSuccess;
    if (n > ((int64_t)1 << 30))
        return hipErrorInvalidValue;
    return src ? sweep3_rows<double, FIELD_U, true>(blocks, items, parity, tile_y, (int)tx, (int)ty, (int)nch, (int)n, s,
                                                    pace)
               : sweep3_rows<double, FIELD_U, false>(blocks, items, parity, tile_y, (int)tx, (int)ty, (int)nch, (int)n,
                                                     s, pace);
}

hipError_t launch_ir_inner3(const BlockDesc* blocks, const Item* items, int nitems, int nx, int ny, int nz,
                            int qparity, int tile_y, int z_chunk, int lo_dtype, hipStream_t s, uint32_t pace)
{
    int64_t tx = 0, ty = 0, nch = 0, n = nitems;
    if (!items) {
        if (nx < 1 || ny < 1 || nz < 1 || z_chunk < 1 || tile_y < 1)
            return hipErrorInvalidValue;
        tx = (nx + 63) / 64;
        ty = (ny + tile_y - 1) / tile_y;
        nch = (nz + z_chunk - 1) / z_chunk;
        n = tx * ty * nch;
    }
    if (n <= 0)
        return hipSuccess;
    if (n > ((int64_t)1 << 30))
        return hipErrorInvalidValue;
    switch (lo_dtype) {
    case 0: return sweep3_rows<double, FIELD_D, true>(blocks, items, qparity, tile_y, (int)tx, (int)ty, (int)nch, (int)n, s, pace);
    case 1: return sweep3_rows<float, FIELD_D, true>(blocks, items, qparity, tile_y, (int)tx, (int)ty, (int)nch, (int)n, s, pace);
    case 2: return sweep3_rows<bf16, FIELD_D, true>(blocks, items, qparity, tile_y, (int)tx, (int)ty, (int)nch, (int)n, s, pace);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_resident(const BlockDesc* blocks, const Item* items, int nitems, int max_pairs, int max_nz,
                           size_t lds_bytes, int variant, int parity, int nsweeps, bool src, hipStream_t s)
{
    const int n = items ? nitems : 1;
    if (n <= 0 || nsweeps <= 0)
        return hipSuccess;
    if (max_pairs < 1 || max_pairs > kResidentMaxPairs || max_nz < 1 || max_nz > kResidentMaxPlanes ||
        lds_bytes > (size_t)kResidentMaxLds || n > 65535 || variant < 0 || variant >= kResidentVariants)
        return hipErrorInvalidValue;
    const dim3 grid(n), block((max_pairs + 63) / 64 * 64);
    // variants (resident_variant): an even or odd number of steps per sweep
#define JC_RESIDENT_CASE(V, KT, KF)                                                                            \
    if (variant == V) {                                                                                        \
        if (src)                                                                                               \
            hipLaunchKernelGGL(KT, grid, block, lds_bytes, s, blocks, items, parity, nsweeps);                   \
        else                                                                                                   \
            hipLaunchKernelGGL(KF, grid, block, lds_bytes, s, blocks, items, parity, nsweeps);                   \
        return hipGetLastError();                                                                              \
    }
    JC_RESIDENT_CASE(0, (k_resident<true, 0>), (k_resident<false, 0>))
    JC_RESIDENT_CASE(1, (k_resident<true, 1>), (k_resident<false, 1>))
#undef JC_RESIDENT_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_ir_inner2_items(const BlockDesc* blocks, const Item* items, int nitems, int qparity, int tile_y,
                                  int lo_dtype, hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
    const int grid = ((nitems + 7) / 8) * 8;
#define JC_IR2_ITEMS_CASE(TY, DT, T)                                                                            \
    if (tile_y == TY && lo_dtype == DT) {                                                                      \
        hipLaunchKernelGGL((k_sweep2<T, FIELD_D, 32, TY, true>), dim3(grid), dim3((34 * (TY + 4) + 63) / 64 * 64), 0, \
                           s, blocks, items, qparity, 0, 0, 0, nitems, 0u);                                    \
        return hipGetLastError();                                                                              \
    }
    JC_IR2_ITEMS_CASE(16, 0, double)
    JC_IR2_ITEMS_CASE(16, 1, float)
    JC_IR2_ITEMS_CASE(16, 2, bf16)
#undef JC_IR2_ITEMS_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_ir_inner2(const BlockDesc* blocks, int nx, int ny, int nz, int qparity, int tile_y, int z_chunk,
                            int lo_dtype, hipStream_t s, uint32_t pace)
{
    if (nx < 1 || ny < 1 || nz < 1 || z_chunk < 1)
        return hipErrorInvalidValue;
    const int64_t tx = (nx + 63) / 64, ty = (ny + tile_y - 1) / tile_y, nch = (nz + z_chunk - 1) / z_chunk;
    const int64_t n = tx * ty * nch;
    if (n > ((int64_t)1 << 30))
        return hipErrorInvalidValue;
    const int grid = (int)((n + 7) / 8 * 8);
#define JC_IR2_CASE(TY, DT, T)                                                                                  \
    if (tile_y == TY && lo_dtype == DT) {                                                                      \
        hipLaunchKernelGGL((k_sweep2<T, FIELD_D, 32, TY, true>), dim3(grid), dim3((34 * (TY + 4) + 63) / 64 * 64), 0, \
                           s, blocks, nullptr, qparity, (int)tx, (int)ty, (int)nch, (int)n, pace);             \
        return hipGetLastError();                                                                              \
    }
    JC_IR2_CASE(8, 0, double)
    JC_IR2_CASE(8, 1, float)
    JC_IR2_CASE(8, 2, bf16)
    JC_IR2_CASE(16, 0, double)
    JC_IR2_CASE(16, 1, float)
    JC_IR2_CASE(16, 2, bf16)
    JC_IR2_CASE(24, 0, double)
    JC_IR2_CASE(24, 1, float)
    JC_IR2_CASE(24, 2, bf16)
#undef JC_IR2_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_ir_residual(const BlockDesc* blocks, const Item* items, int nitems, int parity, int tile_x,
                              int tile_y, bool src, int lo_dtype, double* partials, hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
#define JC_IR_RES(RT)                                                                                  \
    return src ? sweep_tiles<double, FIELD_U, true, RT>(blocks, items, nitems, parity, tile_x, tile_y, true,   \
                                                        true, false, partials, s, 0)                        \
               : sweep_tiles<double, FIELD_U, false, RT>(blocks, items, nitems, parity, tile_x, tile_y, true,  \
                                                         true, false, partials, s, 0);
    switch (lo_dtype) {
    case 0: JC_IR_RES(double)
    case 1: JC_IR_RES(float)
    case 2: JC_IR_RES(bf16)
    default: return hipErrorInvalidValue;
    }
#undef JC_IR_RES
}

hipError_t launch_ir_inner(const BlockDesc* blocks, const Item* items, int nitems, int qparity, int tile_x,
                           int tile_y, int lo_dtype, hipStream_t s, uint32_t pace)
{
    if (nitems <= 0)
        return hipSuccess;
    switch (lo_dtype) {
    case 0: return sweep_tiles<double, FIELD_D, true, NoRlo>(blocks, items, nitems, qparity, tile_x, tile_y, true,
                                                             false, true, nullptr, s, pace);
    case 1: return sweep_tiles<float, FIELD_D, true, NoRlo>(blocks, items, nitems, qparity, tile_x, tile_y, true,
                                                            false, true, nullptr, s, pace);
    case 2: return sweep_tiles<bf16, FIELD_D, true, NoRlo>(blocks, items, nitems, qparity, tile_x, tile_y, true,
                                                           false, true, nullptr, s, pace);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ir_first(const BlockDesc* blocks, int nblocks, int64_t max_rows, int lo_dtype, hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    const dim3 grid = row_grid(nblocks, max_rows);
    switch (lo_dtype) {
    case 0: hipLaunchKernelGGL(k_ir_first<double>, grid, dim3(256), 0, s, blocks); break;
    case 1: hipLaunchKernelGGL(k_ir_first<float>, grid, dim3(256), 0, s, blocks); break;
    case 2: hipLaunchKernelGGL(k_ir_first<bf16>, grid, dim3(256), 0, s, blocks); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ir_update(const BlockDesc* blocks, int nblocks, int64_t max_rows, int p, int q, int lo_dtype,
                            hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    const dim3 grid = row_grid(nblocks, max_rows);
    switch (lo_dtype) {
    case 0: hipLaunchKernelGGL(k_ir_update<double>, grid, dim3(256), 0, s, blocks, p, q); break;
    case 1: hipLaunchKernelGGL(k_ir_update<float>, grid, dim3(256), 0, s, blocks, p, q); break;
    case 2: hipLaunchKernelGGL(k_ir_update<bf16>, grid, dim3(256), 0, s, blocks, p, q); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const int64_t words = (int64_t)(bytes / 8);
    if (words <= 0)
        return hipSuccess;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint64_t*>(p), words);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, const int32_t* ranges, int nmembers, double* out,
                         hipStream_t s)
{
    if (nmembers <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(nmembers), dim3(256), 0, s, partials, ranges, out);
    return hipGetLastError();
}

hipError_t launch_pack(const BlockDesc* blocks, const PairDesc* pairs, int npairs, int max_slow,
                       int max_fast, int parity, int slot, hipStream_t s)
{
    if (npairs <= 0)
        return hipSuccess;
    const dim3 grid((max_fast + 255) / 256, max_slow, npairs);
    hipLaunchKernelGGL(k_pack, grid, dim3(256), 0, s, blocks, pairs, parity, slot);
    return hipGetLastError();
}

hipError_t launch_exchange(const PairDesc* pairs, int npairs, int64_t max_count, hipStream_t s)
{
    if (npairs <= 0)
        return hipSuccess;
    int64_t chunks = (max_count / 2 + 255) / 256;
    if (chunks < 1) chunks = 1;
    if (chunks > 1024) chunks = 1024;
    hipLaunchKernelGGL(k_exchange, dim3((unsigned)chunks, npairs), dim3(256), 0, s, pairs);
    return hipGetLastError();
}

hipError_t launch_unpack(const BlockDesc* blocks, const PairDesc* pairs, int npairs, int max_slow,
                         int max_fast, int parity, hipStream_t s)
{
    if (npairs <= 0)
        return hipSuccess;
    const dim3 grid((max_fast + 255) / 256, max_slow, npairs);
    hipLaunchKernelGGL(k_unpack, grid, dim3(256), 0, s, blocks, pairs, parity);
    return hipGetLastError();
}

hipError_t launch_scatter(const BlockDesc* blocks, int nblocks, int64_t max_rows, const double* global,
                          int64_t gnx, int64_t gny, int which, hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_scatter, row_grid(nblocks, max_rows), dim3(256), 0, s, blocks, global, gnx, gny, which);
    return hipGetLastError();
}

hipError_t launch_gather(const BlockDesc* blocks, int nblocks, int64_t max_rows, double* global, int64_t gnx,
                         int64_t gny, int64_t gnz, int which, int parity, hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_gather, row_grid(nblocks, max_rows), dim3(256), 0, s, blocks, global, gnx, gny, gnz,
                       which, parity);
    return hipGetLastError();
}

}  // namespace jc
