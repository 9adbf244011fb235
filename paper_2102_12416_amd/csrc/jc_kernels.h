// Launchers of the libjc HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "jc_types.h"
#include "jc_resident.h"

namespace jc {

// Tiles are 64 or 32 x cells wide (two cells per thread); groups use 64.
constexpr int kTileX = 64;

// Sweep / residual over a work list.  parity selects the input copy of
// each item's block (xor the item's flip).  fused: read paired ghosts from
// the face buffers of the input slot and write face values to the output
// slot.  resid: write one partial sum of r^2 per item into partials.
// store: write the new iterate (false = residual only).
// pace: ticks of the constant 100 MHz clock per plane step below which a
// work-group waits (0 = none; see pace_wait in jc_kernels.hip).
hipError_t launch_sweep(const BlockDesc* blocks, const Item* items, int nitems, int parity,
                        int tile_x, int tile_y, bool fused, bool resid, bool store, bool src, double* partials,
                        hipStream_t s, uint32_t pace = 0);

// Two sweeps of the single block of a context without face pairs in one
// launch (binary64): iterate k from copy parity, iterate k + 2 into copy
// parity ^ 1.  Tiles of 64 cells by tile_y (8, 16 or 24) rows by z_chunk planes.
hipError_t launch_sweep2(const BlockDesc* blocks, int nx, int ny, int nz, int parity, int tile_y, int z_chunk,
                         bool src, hipStream_t s, uint32_t pace = 0);
// The same over a work list of 64-cell by tile_y-row tiles of several
// one-block contexts (groups): each item's block, its copy parity ^ flip.
hipError_t launch_sweep2_items(const BlockDesc* blocks, const Item* items, int nitems, int parity, int tile_y,
                               bool src, hipStream_t s);
// The same for two inner sweeps of the refinement correction (copy
// qparity -> qparity ^ 1, source r_lo; tile_y 8, 16 or 24): iterate k + 1 is
// rounded to the storage format between the two sweeps.
hipError_t launch_ir_inner2(const BlockDesc* blocks, int nx, int ny, int nz, int qparity, int tile_y, int z_chunk,
                            int lo_dtype, hipStream_t s, uint32_t pace = 0);
// The same over a work list of 64-cell by 16-row tiles (groups; each
// item's flip must be 0: a refining member holds its iterate in copy 0).
hipError_t launch_ir_inner2_items(const BlockDesc* blocks, const Item* items, int nitems, int qparity, int tile_y,
                                  int lo_dtype, hipStream_t s);

// Three sweeps in one launch (k_sweep3), tiles of 64 cells by tile_y (8 or
// 16) rows.  items null: the single block of blocks[0] (nx, ny, nz) in z
// chunks of z_chunk planes; otherwise the work list items[0 .. nitems) of
// such tiles (groups), each with its block and flip.
hipError_t launch_sweep3(const BlockDesc* blocks, const Item* items, int nitems, int nx, int ny, int nz, int parity,
                         int tile_y, int z_chunk, bool src, hipStream_t s, uint32_t pace = 0);
// The same for the refinement correction (copy qparity -> qparity ^ 1).
hipError_t launch_ir_inner3(const BlockDesc* blocks, const Item* items, int nitems, int nx, int ny, int nz,
                            int qparity, int tile_y, int z_chunk, int lo_dtype, hipStream_t s, uint32_t pace = 0);

// Many sweeps in one launch (k_resident, k_resident_pipe): nsweeps Jacobi
// sweeps of blocks that fit on chip (resident_fits), one work-group per
// block, iterate k from copy parity (xor the item's flip), iterate k +
// nsweeps into copy parity ^ (nsweeps & 1).  items null: blocks[0] alone;
// otherwise one work-group per item (block and flip; every block's
// resident_variant(nz) equal to variant).  max_pairs / max_nz /
// lds_bytes: the largest (nx + 1) / 2 * ny, nz and resident_lds_bytes
// over the blocks swept.
hipError_t launch_resident(const BlockDesc* blocks, const Item* items, int nitems, int max_pairs, int max_nz,
                           size_t lds_bytes, int variant, int parity, int nsweeps, bool src, hipStream_t s);

// Refinement passes (lo_dtype: 0 binary64, 1 binary32, 2 bfloat16 storage
// of d and r_lo).  Residual: r of u[parity] with fused ghosts (face
// buffers of slot parity), partial sums of r^2, r rounded into r_lo.
// Inner: one sweep of d (copy qparity -> qparity ^ 1) with source r_lo.
// First: d_1 = lo(r_lo / 6) into copy 1.  Update: u[p] += d[q] and the
// updated faces into slot p.
hipError_t launch_ir_residual(const BlockDesc* blocks, const Item* items, int nitems, int parity, int tile_x,
                              int tile_y, bool src, int lo_dtype, double* partials, hipStream_t s);
hipError_t launch_ir_inner(const BlockDesc* blocks, const Item* items, int nitems, int qparity, int tile_x,
                           int tile_y, int lo_dtype, hipStream_t s, uint32_t pace = 0);
// max_rows: the largest ny * nz over the blocks (sizes the grid).
hipError_t launch_ir_first(const BlockDesc* blocks, int nblocks, int64_t max_rows, int lo_dtype, hipStream_t s);
hipError_t launch_ir_update(const BlockDesc* blocks, int nblocks, int64_t max_rows, int p, int q, int lo_dtype,
                            hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Sum partials[ranges[2m] .. ranges[2m+1]) in a fixed order into out[m], m < nmembers.
hipError_t launch_reduce(const double* partials, const int32_t* ranges, int nmembers, double* out,
                         hipStream_t s);

// Face pack (interior face plane of u[parity] -> pair buffer slot),
// exchange (slot 0 -> slot 1), unpack (slot 1 -> ghost plane of u[parity]).
hipError_t launch_pack(const BlockDesc* blocks, const PairDesc* pairs, int npairs, int max_slow,
                       int max_fast, int parity, int slot, hipStream_t s);
hipError_t launch_exchange(const PairDesc* pairs, int npairs, int64_t max_count, hipStream_t s);
hipError_t launch_unpack(const BlockDesc* blocks, const PairDesc* pairs, int npairs, int max_slow,
                         int max_fast, int parity, hipStream_t s);

// Global padded array <-> blocks.  which: 0 = iterate (both copies on
// scatter; copy `parity` on gather), 1 = source.
hipError_t launch_scatter(const BlockDesc* blocks, int nblocks, int64_t max_rows, const double* global,
                          int64_t gnx, int64_t gny, int which, hipStream_t s);
hipError_t launch_gather(const BlockDesc* blocks, int nblocks, int64_t max_rows, double* global, int64_t gnx,
                         int64_t gny, int64_t gnz, int which, int parity, hipStream_t s);

}  // namespace jc
