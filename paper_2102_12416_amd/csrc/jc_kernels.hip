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
// divided by 6 with an IEEE division; the library is built with
// -ffp-contract=off, so no multiply-add is fused and every block of every
// decomposition computes the same bits for the same cell.

#include <hip/hip_runtime.h>

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

typedef double v2d __attribute__((ext_vector_type(2)));

// 16-byte load of the aligned pair at p
__device__ __forceinline__ double2 ld2(const double* p)
{
    const v2d v = *(const v2d JC_GLOBAL*)(p);
    return make_double2(v.x, v.y);
}

// 16-byte store of (a, b) to the aligned pair at p
__device__ __forceinline__ void st2(double* p, double a, double b)
{
    v2d v;
    v.x = a;
    v.y = b;
    *(v2d JC_GLOBAL*)(p) = v;
}

__device__ __forceinline__ void st1(double* p, double a)
{
    *(double JC_GLOBAL*)(p) = a;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = v + __shfl_xor(v, o, 64);
    return v;
}

// One work-group sweeps a tile of 64 x cells by TY rows of one block,
// marching along z.  Each thread owns two adjacent x cells of one row
// (one 16-byte load per plane: cell x = 1 of every row starts a 128-byte
// line).  Per plane the work-group writes the plane -- its cells plus a
// one-cell halo ring -- into an LDS tile, synchronises once (the tile is
// double-buffered by plane parity) and reads its x and y neighbours from
// LDS; the z-1 / z / z+1 values of its own cells stay in registers.
//
// Every thread issues the same global loads in every iteration, with
// clamped addresses where it has nothing to fetch, so that the loads of
// the next two planes stay in flight while the current one is computed
// (no divergent branch around a load).  The halo ring is fetched by
// threads with a halo role: threads 0-31 the row above the tile, 32-63
// the row below, the next TY threads the column left of it and the next
// TY the column right of it; the rest re-load their own cells.
//
// FUSED: ghost cells of faces that have a neighbour block are read from
// the neighbour's face buffer of the input slot (the pairing's pre-posted
// receive side), and every face cell written is also written to this
// block's face buffer of the output slot -- pack, exchange and unpack
// folded into the sweep.  RES: accumulate r^2 of the input iterate,
// r = (b + s) - 6u, into one partial per work-group.  STORE: write the
// new iterate (off: residual only).  SRC: the block has a source b.
template <int TY, bool FUSED, bool RES, bool STORE, bool SRC>
__global__ void __launch_bounds__(32 * TY)
k_sweep(const BlockDesc* __restrict__ blocks, const Item* __restrict__ items, int nitems,
        int parity, double* __restrict__ partials)
{
    static_assert(TY >= 4 && 32 * TY >= 64 + 2 * TY, "halo roles need 64 + 2 TY threads");
    constexpr int NT = 32 * TY;
    constexpr int LW = 68;   // LDS row: col 1 = x0, cols 2..65 = x0+1..x0+64, up to col 66
    __shared__ double S[2][TY + 2][LW];
    __shared__ double wsum[NT / 64];

    const int id = logical_block(blockIdx.x, gridDim.x);
    if (id >= nitems)
        return;                                   // uniform over the work-group
    const Item it = items[id];
    const BlockDesc* B = blocks + it.block;
    const int p = parity ^ it.flip;
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    const int t = threadIdx.x;
    const int lx = t & 31;
    const int ly = t >> 5;
    const int x0 = it.x0, y0 = it.y0;
    const int x_end = min(x0 + 64, nx);           // last x cell of the tile
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
    const int64_t pitch = B->pitch;
    const int64_t plane = B->plane;
    const int64_t ldx = face_ld(ny);              // x-face buffers: (z, y) rows
    const int64_t ldy = face_ld(nx);              // y- and z-face buffers: (z, x) / (y, x) rows
    const double* __restrict__ src = B->u[p];
    double* __restrict__ dst = B->u[p ^ 1];

    // own pair (xa_c, y_c) at plane zz
    const double* own = src + (int64_t)y_c * pitch + xa_c;
    const double* own_lo = own;                                   // plane 0
    const double* own_hi = own + (int64_t)(nz + 1) * plane;       // plane nz + 1
    if (FUSED) {
        const int64_t zi = (int64_t)(y_c - 1) * ldy + (xa_c - 1);
        if (B->gin[ZM][p]) own_lo = B->gin[ZM][p] + zi;
        if (B->gin[ZP][p]) own_hi = B->gin[ZP][p] + zi;
    }
    auto own_at = [&](int zz) -> double2 {
        const double* a = own + (int64_t)zz * plane;
        if (FUSED) {
            a = (zz == 0) ? own_lo : a;
            a = (zz == nz + 1) ? own_hi : a;
        }
        return ld2(a);
    };
    const double* bown = SRC ? B->b + (int64_t)y_c * pitch + xa_c : nullptr;

    // halo role: the pair at hbase + zz * hstride (16-byte aligned)
    const int role = t < 32 ? 0 : t < 64 ? 1 : t < 64 + TY ? 2 : t < 64 + 2 * TY ? 3 : 4;
    const double* hbase = own;
    int64_t hstride = plane;
    int hrow = 0, hcol = 0, hcomp = 0;
    bool hv0 = false, hv1 = false;
    if (role <= 1) {
        const int hl = t & 31;
        const int hx = x0 + 2 * hl + 1;
        const int hx_c = min(hx, xlast);
        const int hy = role == 0 ? y0 : y_end + 1;
        hv0 = hx <= x_end;
        hv1 = hx + 1 <= x_end;
        hbase = src + (int64_t)hy * pitch + hx_c;
        if (FUSED) {
            const double* g = (hy == 0) ? B->gin[YM][p] : (hy == ny + 1) ? B->gin[YP][p] : nullptr;
            if (g) {
                hbase = g - ldy + (hx_c - 1);     // value (z - 1, x - 1)
                hstride = ldy;
            }
        }
        hrow = role == 0 ? 0 : ly_last + 2;
        hcol = 2 * hl + 2;
    } else if (role <= 3) {
        const int r = t - 64 - (role == 3 ? TY : 0);
        const int hy = y0 + r + 1;
        hv0 = hy <= y_end;
        const int hy_c = min(hy, ny);
        const int hx = role == 2 ? x0 : x_end + 1;
        const int ps = (hx & 1) ? hx : hx - 1;    // aligned pair holding hx
        hcomp = (hx & 1) ? 0 : 1;
        hbase = src + (int64_t)hy_c * pitch + ps;
        if (FUSED) {
            const double* g = (hx == 0) ? B->gin[XM][p] : (hx == nx + 1) ? B->gin[XP][p] : nullptr;
            if (g) {
                const int fi = hy_c - 1;          // value (z - 1, y - 1)
                hbase = g - ldx + (fi & ~1);
                hcomp = fi & 1;
                hstride = ldx;
            }
        }
        hrow = r + 1;
        hcol = role == 2 ? 1 : x_end - x0 + 2;
    }
    auto halo_at = [&](int zz) -> double2 {
        return ld2(hbase + (int64_t)zz * hstride);
    };

    const int zf = it.z0 + 1;                     // first plane of the tile
    const int zl = it.z0 + it.zlen;               // last plane of the tile
    double2 zm = own_at(zf - 1);
    double2 c = own_at(zf);
    double2 zp = own_at(zf + 1);
    double2 h = halo_at(zf);
    double2 bc = make_double2(0.0, 0.0);
    if (SRC)
        bc = ld2(bown + (int64_t)zf * plane);

    double acc = 0.0;
    for (int z = zf; z <= zl; ++z) {
        // the next planes go in flight first; the last iteration re-reads
        // planes it already holds (cache hits) instead of branching
        const int zn = min(z + 1, zl);
        const double2 zq = own_at(min(z + 2, zl + 1));
        const double2 hn = halo_at(zn);
        double2 bn = make_double2(0.0, 0.0);
        if (SRC)
            bn = ld2(bown + (int64_t)zn * plane);

        double (*T)[LW] = S[z & 1];
        if (a_ok) {
            T[ly + 1][2 * lx + 2] = c.x;
            if (b_ok)
                T[ly + 1][2 * lx + 3] = c.y;
        }
        if (role <= 1) {
            if (hv0) T[hrow][hcol] = h.x;
            if (hv1) T[hrow][hcol + 1] = h.y;
        } else if (role <= 3 && hv0) {
            T[hrow][hcol] = hcomp ? h.y : h.x;
        }
        __syncthreads();
        const double xm_a = T[ly + 1][2 * lx + 1];
        const double xp_a = b_ok ? c.y : T[ly + 1][2 * lx + 3];
        double sa = xm_a + xp_a;
        sa = sa + T[ly][2 * lx + 2];
        sa = sa + T[ly + 2][2 * lx + 2];
        sa = sa + zm.x;
        sa = sa + zp.x;
        double sb = c.x + T[ly + 1][2 * lx + 4];
        sb = sb + T[ly][2 * lx + 3];
        sb = sb + T[ly + 2][2 * lx + 3];
        sb = sb + zm.y;
        sb = sb + zp.y;
        if (RES) {
            const double ra = SRC ? (bc.x + sa) - 6.0 * c.x : sa - 6.0 * c.x;
            const double rb = SRC ? (bc.y + sb) - 6.0 * c.y : sb - 6.0 * c.y;
            acc = acc + (a_ok ? ra * ra : 0.0);
            acc = acc + (b_ok ? rb * rb : 0.0);
        }
        if (STORE) {
            const double va = SRC ? (sa + bc.x) / 6.0 : sa / 6.0;
            // past the last cell of a row the pair's second slot is the
            // x = nx + 1 ghost: write back the value it already holds
            const double vb = b_ok ? (SRC ? (sb + bc.y) / 6.0 : sb / 6.0) : c.y;
            if (a_ok)
                st2(dst + (int64_t)z * plane + (int64_t)y * pitch + xa, va, vb);
            if (FUSED) {
                const int64_t xfi = (int64_t)(z - 1) * ldx + (y - 1);
                const int64_t yfi = (int64_t)(z - 1) * ldy + (xa - 1);
                const int64_t zfi = (int64_t)(y - 1) * ldy + (xa - 1);
                double* oxm = B->gout[XM][p ^ 1];
                double* oxp = B->gout[XP][p ^ 1];
                double* oym = B->gout[YM][p ^ 1];
                double* oyp = B->gout[YP][p ^ 1];
                double* ozm = B->gout[ZM][p ^ 1];
                double* ozp = B->gout[ZP][p ^ 1];
                // a face row's padding slot takes the second value of a
                // pair that ends past the face (ld is even)
                if (a_ok && xa == 1 && oxm) st1(oxm + xfi, va);
                if (a_ok && xa == nx && oxp) st1(oxp + xfi, va);
                if (b_ok && xa + 1 == nx && oxp) st1(oxp + xfi, vb);
                if (a_ok && y == 1 && oym) st2(oym + yfi, va, vb);
                if (a_ok && y == ny && oyp) st2(oyp + yfi, va, vb);
                if (a_ok && z == 1 && ozm) st2(ozm + zfi, va, vb);
                if (a_ok && z == nz && ozp) st2(ozp + zfi, va, vb);
            }
        }
        zm = c;
        c = zp;
        zp = zq;
        h = hn;
        bc = bn;
    }
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

template <int TY, bool SRC>
hipError_t sweep_ty(const BlockDesc* blocks, const Item* items, int nitems, int parity, bool fused,
                    bool resid, bool store, double* partials, hipStream_t s)
{
    const int grid = ((nitems + 7) / 8) * 8;
    const dim3 bs(32 * TY);
#define JC_SWEEP_CASE(F, R, S)                                                                \
    if (fused == F && resid == R && store == S) {                                            \
        hipLaunchKernelGGL((k_sweep<TY, F, R, S, SRC>), dim3(grid), bs, 0, s, blocks, items,  \
                           nitems, parity, partials);                                        \
        return hipGetLastError();                                                            \
    }
    JC_SWEEP_CASE(false, false, true)
    JC_SWEEP_CASE(false, true, true)
    JC_SWEEP_CASE(false, true, false)
    JC_SWEEP_CASE(true, false, true)
    JC_SWEEP_CASE(true, true, true)
    JC_SWEEP_CASE(true, true, false)
#undef JC_SWEEP_CASE
    return hipErrorInvalidValue;
}

template <int TY>
hipError_t sweep_src(const BlockDesc* blocks, const Item* items, int nitems, int parity, bool fused,
                     bool resid, bool store, bool src, double* partials, hipStream_t s)
{
    return src ? sweep_ty<TY, true>(blocks, items, nitems, parity, fused, resid, store, partials, s)
               : sweep_ty<TY, false>(blocks, items, nitems, parity, fused, resid, store, partials, s);
}

// Fixed-order sum of one member's partials: each thread adds a strided
// subsequence in order, then a fixed tree over the work-group.
__global__ void __launch_bounds__(256)
k_reduce(const double* __restrict__ partials, const int32_t* __restrict__ ranges,
         double* __restrict__ out)
{
    const int m = blockIdx.x;
    const int lo = ranges[m], hi = ranges[m + 1];
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
        for (int x = threadIdx.x; x < nx + 2; x += 256) {
            const double v = g[grow + x];
            if (which == 0) {
                B.u[0][brow + x] = v;
                B.u[1][brow + x] = v;
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

}  // namespace

hipError_t launch_sweep(const BlockDesc* blocks, const Item* items, int nitems, int parity,
                        int tile_y, bool fused, bool resid, bool store, bool src, double* partials,
                        hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
    switch (tile_y) {
    case 4: return sweep_src<4>(blocks, items, nitems, parity, fused, resid, store, src, partials, s);
    case 8: return sweep_src<8>(blocks, items, nitems, parity, fused, resid, store, src, partials, s);
    case 16: return sweep_src<16>(blocks, items, nitems, parity, fused, resid, store, src, partials, s);
    case 32: return sweep_src<32>(blocks, items, nitems, parity, fused, resid, store, src, partials, s);
    default: return hipErrorInvalidValue;
    }
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

hipError_t launch_scatter(const BlockDesc* blocks, int nblocks, const double* global, int64_t gnx,
                          int64_t gny, int which, hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(256, nblocks), dim3(256), 0, s, blocks, global, gnx, gny, which);
    return hipGetLastError();
}

hipError_t launch_gather(const BlockDesc* blocks, int nblocks, double* global, int64_t gnx,
                         int64_t gny, int64_t gnz, int which, int parity, hipStream_t s)
{
    if (nblocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(256, nblocks), dim3(256), 0, s, blocks, global, gnx, gny, gnz,
                       which, parity);
    return hipGetLastError();
}

}  // namespace jc
