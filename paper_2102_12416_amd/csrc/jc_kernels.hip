// HIP kernels of libjc for gfx950 (CDNA4, wave64).
//
// Jacobi3D, paper section 4.3: each block of the decomposition is swept
// with the 7-point stencil after its halo has been exchanged with up to
// six neighbours.  The sweep marches along z through a tile of 64 x cells
// (one wavefront per row) and tile_y rows, keeping the z-1, z and z+1
// values of its own column in registers, so that every interior value is
// fetched from HBM once per sweep; the x and y neighbours of a plane are
// re-read from the L1/L2 lines the neighbouring lanes and rows just
// brought in.  The stencil is not a contraction, so no matrix cores are
// used: the kernel is bound by HBM bandwidth (16 bytes per cell update).
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

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = v + __shfl_xor(v, o, 64);
    return v;
}

template <int TY, bool FUSED, bool RES, bool STORE>
__global__ void __launch_bounds__(64 * TY)
k_sweep(const BlockDesc* __restrict__ blocks, const Item* __restrict__ items, int nitems,
        int parity, double* __restrict__ partials)
{
    const int id = logical_block(blockIdx.x, gridDim.x);
    if (id >= nitems)
        return;                              // uniform over the work-group
    const Item it = items[id];
    const BlockDesc* B = blocks + it.block;
    const int p = parity ^ it.flip;
    const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
    const int lx = threadIdx.x & 63;
    const int ly = threadIdx.x >> 6;
    const int x = it.x0 + lx + 1;
    const int y = it.y0 + ly + 1;
    const int64_t pitch = B->pitch;
    const int64_t plane = B->plane;
    const double* __restrict__ src = B->u[p];
    double* __restrict__ dst = B->u[p ^ 1];
    const double* __restrict__ bsrc = B->b;

    double acc = 0.0;
    if (x <= nx && y <= ny) {
        const double* gxm = nullptr; const double* gxp = nullptr;
        const double* gym = nullptr; const double* gyp = nullptr;
        const double* gzm = nullptr; const double* gzp = nullptr;
        double* oxm = nullptr; double* oxp = nullptr;
        double* oym = nullptr; double* oyp = nullptr;
        double* ozm = nullptr; double* ozp = nullptr;
        if (FUSED) {
            gxm = B->gin[XM][p]; gxp = B->gin[XP][p];
            gym = B->gin[YM][p]; gyp = B->gin[YP][p];
            gzm = B->gin[ZM][p]; gzp = B->gin[ZP][p];
            oxm = B->gout[XM][p ^ 1]; oxp = B->gout[XP][p ^ 1];
            oym = B->gout[YM][p ^ 1]; oyp = B->gout[YP][p ^ 1];
            ozm = B->gout[ZM][p ^ 1]; ozp = B->gout[ZP][p ^ 1];
        }
        int z = it.z0 + 1;
        const int64_t col = (int64_t)y * pitch + x;
        const int64_t zf = (int64_t)(y - 1) * nx + (x - 1);     // index in a z-face buffer
        const double* pc = src + (int64_t)z * plane + col;
        const double* azm = (FUSED && z == 1 && gzm) ? gzm + zf : pc - plane;
        double zm = *azm;
        double c = pc[0];
        const int zend = z + it.zlen;
        for (; z < zend; ++z, pc += plane) {
            const int64_t xf = (int64_t)(z - 1) * ny + (y - 1);  // x-face buffer index
            const int64_t yf = (int64_t)(z - 1) * nx + (x - 1);  // y-face buffer index
            const double* azp = (FUSED && z == nz && gzp) ? gzp + zf : pc + plane;
            const double* axm = (FUSED && x == 1 && gxm) ? gxm + xf : pc - 1;
            const double* axp = (FUSED && x == nx && gxp) ? gxp + xf : pc + 1;
            const double* aym = (FUSED && y == 1 && gym) ? gym + yf : pc - pitch;
            const double* ayp = (FUSED && y == ny && gyp) ? gyp + yf : pc + pitch;
            const double zp = *azp;
            const double xm = *axm;
            const double xp = *axp;
            const double ym = *aym;
            const double yp = *ayp;
            double s = xm + xp;
            s = s + ym;
            s = s + yp;
            s = s + zm;
            s = s + zp;
            const int64_t at = (int64_t)z * plane + col;
            double bb = 0.0;
            if (bsrc)
                bb = bsrc[at];
            if (RES) {
                const double r = bsrc ? (bb + s) - 6.0 * c : s - 6.0 * c;
                acc = acc + r * r;
            }
            if (STORE) {
                const double v = bsrc ? (s + bb) / 6.0 : s / 6.0;
                dst[at] = v;
                if (FUSED) {
                    if (x == 1 && oxm) oxm[xf] = v;
                    if (x == nx && oxp) oxp[xf] = v;
                    if (y == 1 && oym) oym[yf] = v;
                    if (y == ny && oyp) oyp[yf] = v;
                    if (z == 1 && ozm) ozm[zf] = v;
                    if (z == nz && ozp) ozp[zf] = v;
                }
            }
            zm = c;
            c = zp;
        }
    }
    if (RES) {
        __shared__ double wsum[TY];
        const double w = wave_sum(acc);
        if ((threadIdx.x & 63) == 0)
            wsum[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < TY; ++i)
                t = t + wsum[i];
            partials[id] = t;
        }
    }
}

template <int TY>
hipError_t sweep_ty(const BlockDesc* blocks, const Item* items, int nitems, int parity, bool fused,
                    bool resid, bool store, double* partials, hipStream_t s)
{
    const int grid = ((nitems + 7) / 8) * 8;
    const dim3 bs(64 * TY);
#define JC_SWEEP_CASE(F, R, S)                                                         \
    if (fused == F && resid == R && store == S) {                                     \
        hipLaunchKernelGGL((k_sweep<TY, F, R, S>), dim3(grid), bs, 0, s, blocks, items, \
                           nitems, parity, partials);                                 \
        return hipGetLastError();                                                     \
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
    P.buf[slot][(int64_t)slow * P.fast + fast] = B.u[parity][face_cell(B, P.src_face, slow, fast, 0)];
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
    B.u[parity][face_cell(B, P.dst_face, slow, fast, 1)] = P.buf[1][(int64_t)slow * P.fast + fast];
}

// The pairing's transfer: every send buffer into the receive buffer
// pre-posted for it.  Buffers are 256-byte aligned; 16-byte vectors.
__global__ void __launch_bounds__(256)
k_exchange(const PairDesc* __restrict__ pairs)
{
    const PairDesc& P = pairs[blockIdx.y];
    const int64_t n2 = P.count >> 1;
    const double2* __restrict__ a = reinterpret_cast<const double2*>(P.buf[0]);
    double2* __restrict__ b = reinterpret_cast<double2*>(P.buf[1]);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (int64_t)gridDim.x * 256)
        b[i] = a[i];
    if ((P.count & 1) && blockIdx.x == 0 && threadIdx.x == 0)
        P.buf[1][P.count - 1] = P.buf[0][P.count - 1];
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
                        int tile_y, bool fused, bool resid, bool store, double* partials,
                        hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
    switch (tile_y) {
    case 1: return sweep_ty<1>(blocks, items, nitems, parity, fused, resid, store, partials, s);
    case 2: return sweep_ty<2>(blocks, items, nitems, parity, fused, resid, store, partials, s);
    case 4: return sweep_ty<4>(blocks, items, nitems, parity, fused, resid, store, partials, s);
    case 8: return sweep_ty<8>(blocks, items, nitems, parity, fused, resid, store, partials, s);
    case 16: return sweep_ty<16>(blocks, items, nitems, parity, fused, resid, store, partials, s);
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
