/*
 * jc.h -- C-ABI of libjc, the one-GPU Jacobi3D hot path for MI355X (gfx950).
 *
 * The workload is the Jacobi3D proxy application of "Accelerating
 * Communication for Parallel Programming Models on GPU Systems" (section
 * 4.3): the Jacobi iterative method for the 3D 7-point stencil on a grid
 * decomposed into equal-size cuboid blocks (chosen to minimise surface
 * area), each block exchanging its halo with up to six neighbours, run for
 * a fixed number of iterations.  Here every block lives on one GPU; the
 * halo of each block face travels through a persistent pairing of device
 * buffers fixed when the context is created -- the one-device counterpart of
 * the Channel API of section 3.2.2, where a channel between a pair of
 * objects is created once and afterwards both sides already know the buffer
 * and the tag, so no host metadata message is needed per transfer.
 *
 * Conventions shared by every call
 *  - Grid: interior nx*ny*nz cells, indexed 1..n per axis, surrounded by a
 *    1-cell Dirichlet shell (indices 0 and n+1).  A "global padded array"
 *    is a C array of (nz+2)*(ny+2)*(nx+2) binary64 values, x unit-stride.
 *  - Update: u'(c) = (((((u(x-1)+u(x+1))+u(y-1))+u(y+1))+u(z-1))+u(z+1) [+ b(c)]) / 6,
 *    summed in that order, one IEEE division; strict Jacobi (ping-pong).
 *  - Residual: r = (b + s) - 6u with s the neighbour sum above; its 2-norm.
 *  - Status codes: 0 ok, >0 informational, <0 error.  No C++ exception or
 *    longjmp crosses this interface.  After a negative status,
 *    jc_last_error() returns a message for the calling thread.
 *  - Memory: the caller owns one device arena per context (jc_bind) and
 *    keeps it alive until jc_destroy; the library carves it into blocks,
 *    face buffers and tables and never allocates device memory for a
 *    context.  Host pointers passed in are borrowed for the call only.
 *  - Streams: every call is enqueued asynchronously on the stream given to
 *    jc_bind, except jc_residual, jc_solve and jc_solve_ir, which wait for
 *    the stream before returning.  A context is not thread-safe; distinct
 *    contexts are independent.
 *  - Errors of argument validation are reported before any device work is
 *    enqueued; jc_footprint, jc_create*, the jc_*_info queries and
 *    jc_destroy never touch the device.
 */
#ifndef JC_H
#define JC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    JC_OK = 0,
    JC_MAXITER = 1,          /* solve stopped at its iteration cap (not an error) */
    JC_ERR_INVALID = -1,     /* bad argument */
    JC_ERR_NOMEM = -2,       /* arena smaller than jc_footprint */
    JC_ERR_DEVICE = -3,      /* a HIP call failed */
    JC_ERR_STATE = -4,       /* call out of order (e.g. unpack before exchange) */
    JC_ERR_NONFINITE = -5    /* residual became NaN or infinite */
};

/* ---- storage formats, fields, modes ----------------------------------- */
enum { JC_F64 = 0, JC_F32 = 1, JC_BF16 = 2, JC_NONE = -1 };
enum { JC_FIELD_U = 0, JC_FIELD_B = 1 };
enum {
    JC_MODE_STAGED = 0,      /* per iteration: pack, exchange, unpack, sweep kernels */
    JC_MODE_FUSED = 1        /* per iteration: one launch; ghosts read from the
                                neighbours' face buffers, faces written in the epilogue */
};
/* How jc_exchange moves the faces (staged mode).  DEVICE: the pre-posted
 * pairing, one device copy of every pair, no host work (the Channel
 * analogue).  HOST: host staging, the paper's non-GPU-aware baseline:
 * every send buffer to pinned host memory, a wait for the stream, a host
 * copy into the receiver's host buffer, then back to the device.
 * METADATA: the device copy, but only after a host round trip per
 * iteration -- the host waits for the pack and builds and checks one
 * metadata message (source, destination, size, tag) per pair, as the GPU
 * Messaging API's receiver needs a host message before it can post its
 * receive.  HOST and METADATA disable graph capture. */
enum { JC_EXCHANGE_DEVICE = 0, JC_EXCHANGE_HOST = 1, JC_EXCHANGE_METADATA = 2 };
/* kinds for jc_kernel_time (JC_K_SWEEP2 / JC_K_SWEEP3: the two- and
 * three-sweep launches of temporal blocking; JC_K_RESIDENT: the many-sweep
 * launches of a resident context) */
enum { JC_K_SWEEP = 0, JC_K_PACK = 1, JC_K_EXCHANGE = 2, JC_K_UNPACK = 3,
       JC_K_RESIDUAL = 4, JC_K_FUSED = 5, JC_K_IR_INNER = 6, JC_K_IR_OUTER = 7,
       JC_K_SWEEP2 = 8, JC_K_SWEEP3 = 9, JC_K_RESIDENT = 10, JC_K_COUNT = 11 };

typedef struct jc_ctx jc_ctx;
typedef struct jc_group jc_group;

/* Creation options.  Zero-initialise and set what you need. */
typedef struct jc_options {
    int mode;            /* JC_MODE_STAGED or JC_MODE_FUSED */
    int with_source;     /* 1: the context holds a source field b */
    int ir_dtype;        /* storage of the refinement correction d and residual r_lo:
                            JC_F64, JC_F32 or JC_BF16 (read only when ir_enable = 1) */
    int ir_enable;       /* 1: allocate refinement buffers (d x 2, r_lo, face buffers) */
    int tile_y;          /* rows per tile; 0 = auto */
    int z_chunk;         /* planes per tile; 0 = auto */
    int use_graphs;      /* 1: capture jc_iterate windows as HIP graphs */
    int debug_epochs;    /* reserved, must be 0 */
    int tile_x;          /* cells per tile row: 16, 32, 64, or 96, 128, 256 (binary64
                            storage only: not with an ir_dtype of JC_F32 / JC_BF16);
                            tile_x / 2 x tile_y is 64 to 1024 threads (16 needs
                            tile_y >= 8, 256 tile_y <= 8 or auto); 0 = auto (64, or
                            32 where it idles fewer lanes) */
    int exchange;        /* JC_EXCHANGE_DEVICE (default), _HOST or _METADATA */
    int temporal;        /* 1: temporal blocking -- jc_iterate, the windows of jc_solve
                            and the inner sweeps of jc_solve_ir advance two sweeps per
                            launch (iterate k + 1 stays on chip, so each cell is read and
                            written once per two sweeps; results bitwise equal to
                            one-sweep launches).  Needs a context of one block (no face
                            pairs); the residual sweeps of jc_solve and jc_sweep run one
                            sweep per launch, and groups follow their own flag
                            (jc_group_create).  0: one sweep per launch. */
    int overlap;         /* staged mode with the device exchange: 1 = boundary-first
                            iterations -- the tiles that hold a paired face plane sweep
                            first; then, on a second stream of the library (default
                            priority), the faces of the new iterate are packed, exchanged
                            and unpacked while the interior tiles sweep on the bound
                            stream, which waits for the halo before the next iteration
                            (the computation-communication overlap that
                            overdecomposition allows, sections 2.3 and 6).  Results are
                            bitwise the same as without.  0: pack, exchange, unpack,
                            then the whole sweep. */
    int sweeps_per_launch; /* with temporal = 1: 2 (also 0) or 3.  Three: iterates k + 1
                            and k + 2 stay on chip, so each cell is read and written once
                            per three sweeps (tiles of 8 or 16 rows); a count that is
                            not a multiple of three ends with a two-sweep launch or a
                            single sweep.  Results bitwise the same. */
    int resident;        /* 1: on-chip sweeps for a small grid (the Jacobi sweep of section
                            4.3, many per launch) -- jc_iterate and the windows
                            of jc_solve run as one launch each, whatever their length: one
                            work-group holds the block on chip (its iterate in registers,
                            two planes at a time and the ghost rings in LDS) and sweeps it
                            that many times, so a solve costs one launch per residual check.
                            Needs a context of one block of at most 32 planes with
                            (nx + 1) / 2 * ny <= 512 cell pairs (one thread each) and an LDS
                            need of 8 (4 ny nx' + 2 nz ny + 2 nz nx') bytes within 64 KiB
                            (nx' = nx rounded up to even; for instance 32^3 or 64 x 8 x 32,
                            not 64 x 16 x 32), no refinement, temporal = 0 and overlap = 0;
                            else JC_ERR_INVALID at creation.  Results bitwise equal to
                            one-sweep launches.  After a window only the copy holding the
                            iterate is defined (the other copy holds an older iterate).
                            0: off. */
} jc_options;

/* Result of a solve. */
typedef struct jc_solve_info {
    int64_t iters;       /* sweeps performed (inner sweeps for jc_solve_ir) */
    int64_t outer;       /* outer refinement steps (jc_solve_ir), else checks made */
    double rel_resid;    /* |r_k| / |r_0| at the returned iterate */
    double abs_resid;    /* |r_k| */
    double r0;           /* |r_0| */
    int status;          /* JC_OK (converged), JC_MAXITER, or an error */
    double* history;     /* optional, caller-owned: residual norm at each check */
    int64_t history_cap; /* capacity of history */
    int64_t history_len; /* entries written */
} jc_solve_info;

/* ---- sizing and decomposition (host only) ------------------------------ */

/* Device bytes a context with this geometry and these options needs.
 * grid: interior sizes (nx, ny, nz), each >= 1.  block_dims: block
 * interior sizes, 1 <= block_dims[i] <= grid[i]; when grid is not a
 * multiple, the last block of an axis takes the remainder.
 * Returns JC_ERR_INVALID on bad sizes.  Pure host arithmetic. */
int jc_footprint(const int64_t grid[3], const int64_t block_dims[3],
                 const jc_options* opt, size_t* bytes);
int jc_footprint_rectilinear(const int64_t grid[3], const int64_t* const cuts[3],
                             const int64_t ncuts[3], const jc_options* opt, size_t* bytes);

/* Block counts (px, py, pz) with px*py*pz = nblocks that minimise the total
 * block surface, the decomposition strategy of section 4.3; ties prefer
 * more cuts along z, then y (long unit-stride rows).  parts[i] <= grid[i]. */
int jc_min_surface_parts(const int64_t grid[3], int64_t nblocks, int64_t parts[3]);

/* ---- lifetime -------------------------------------------------------- */

/* Create a context for a uniform decomposition (see jc_footprint).  Builds
 * the blocks, the face pairing table (one entry per directed pair of
 * touching block faces: source block/face, destination block/face = the
 * opposite face, value count, buffer offsets) and the tile work list.
 * Host only; the context is unusable until jc_bind. */
int jc_create(const int64_t grid[3], const int64_t block_dims[3],
              const jc_options* opt, jc_ctx** out);

/* Same for a rectilinear (tensor-product) decomposition: cuts[a] holds
 * ncuts[a] block edges along axis a (x, y, z), each >= 1, summing to grid[a]. */
int jc_create_rectilinear(const int64_t grid[3], const int64_t* const cuts[3],
                          const int64_t ncuts[3], const jc_options* opt, jc_ctx** out);

/* Attach the caller's device arena (>= jc_footprint bytes, 256-byte aligned)
 * and HIP stream (hipStream_t, may be NULL for the null stream; graphs
 * need a non-null stream).  Uploads the tables; enqueued on the stream. */
int jc_bind(jc_ctx* ctx, void* dev_arena, size_t bytes, void* hip_stream);

/* Frees the context's host data (and its graphs and events).  NULL-safe.
 * The arena stays the caller's. */
void jc_destroy(jc_ctx* ctx);

/* Message for the last negative status on this thread ("" if none). */
const char* jc_last_error(void);

/* ---- fields -------------------------------------------------------- */

/* Scatter a device global padded binary64 array into the blocks.
 * JC_FIELD_U: shell = Dirichlet values, interior = initial iterate; both
 * ping-pong copies of every block get their ghosts from it, so the halo of
 * iterate 0 is current afterwards.  JC_FIELD_B: the source (needs
 * with_source).  Resets the iteration count. */
int jc_load_field(jc_ctx* ctx, int which, const void* dev_global_padded);

/* Gather the current iterate (JC_FIELD_U, interior and Dirichlet shell) or
 * the source into a device global padded binary64 array. */
int jc_store_field(jc_ctx* ctx, int which, void* dev_global_padded);

/* ---- the hot path (section 4.3: halo exchange, then stencil) ---------- */

/* Copy the outermost interior plane of every paired block face of the
 * current iterate into that pair's contiguous send buffer, ordered
 * (slow, fast) over the shared plane: -x/+x faces (z, y), -y/+y (z, x),
 * -z/+z (y, x).  The x faces are strided gathers. */
int jc_pack_faces(jc_ctx* ctx);

/* Move every send buffer into the receive buffer pre-posted for it at
 * creation (the pairing); one batched device copy, no host work.
 * JC_ERR_STATE unless jc_pack_faces ran since the last sweep. */
int jc_exchange(jc_ctx* ctx);

/* Copy every receive buffer into the ghost plane of the destination block
 * face.  JC_ERR_STATE unless jc_exchange ran since the last pack. */
int jc_unpack_faces(jc_ctx* ctx);

/* One Jacobi sweep of every block from the current iterate into the other
 * ping-pong buffer, then swap.  JC_ERR_STATE if inter-block ghosts are
 * stale (staged mode: pack, exchange, unpack first). */
int jc_sweep(jc_ctx* ctx);

/* n full iterations.  Staged mode: n x (pack, exchange, unpack, sweep);
 * fused mode: n single launches.  Graph-captured when use_graphs is set
 * and the stream is not the null stream. */
int jc_iterate(jc_ctx* ctx, int64_t n);

/* |r|_2 of the current iterate into *host_l2 (exchanges first if the
 * halo is stale).  Waits for the stream.  JC_ERR_NONFINITE on NaN/Inf. */
int jc_residual(jc_ctx* ctx, double* host_l2);

/* Iterate until |r_k|/|r_0| <= rtol at a check (every check_every sweeps)
 * or max_iter sweeps; rtol <= 0 runs exactly max_iter sweeps and checks at
 * the end (and at every check when history is given).  The residual of a
 * check is computed inside the sweep that follows it, so a converged solve
 * returns iterate k with no extra pass.  Returns JC_OK or JC_MAXITER (also
 * in info->status), or an error. */
int jc_solve(jc_ctx* ctx, double rtol, int64_t max_iter, int64_t check_every,
             jc_solve_info* info);

/* Mixed-precision iterative refinement with Jacobi inner sweeps.
 * Outer step, in binary64: r = (b + s(u)) - 6u over every block, its
 * norm (a fixed-order reduction), the stop test |r|/|r_0| <= rtol, and
 * r_lo = r rounded to the context's ir_dtype (through binary32 for
 * bfloat16, round to nearest even).  Inner: d_0 = 0 with zero ghosts, then
 * inner_sweeps sweeps d' = lo((((((d(x-1)+d(x+1))+d(y-1))+d(y+1))+d(z-1))+d(z+1) + r_lo) / 6)
 * in binary32 arithmetic (binary64 for JC_F64), with the halo of d moved
 * through the face pairing.  Update, binary64: u += d.  Repeats until the
 * test passes or max_inner inner sweeps were run (info->iters counts inner
 * sweeps, info->outer residual checks, history gets |r| of every check).
 * Needs ir_enable at creation.  Waits for the stream.  Returns JC_OK or
 * JC_MAXITER, or an error (JC_ERR_NONFINITE on a NaN/Inf residual). */
int jc_solve_ir(jc_ctx* ctx, int inner_sweeps, double rtol, int64_t max_inner,
                jc_solve_info* info);

/* ---- groups: many contexts in shared launches (batching, serving) ----- */

/* A group sweeps the blocks of several bound, loaded contexts together:
 * one launch per iteration and kernel class (binary64 with / without a
 * source; refinement per storage format), over a joint work list with a
 * tile shape fixed for all groups, so that each member's iterates and
 * residual norms are bitwise the same alone and in any mix.  Members stay
 * independent (own fields, pairing, iteration counts); paired faces move
 * through the face buffers (fused).  Refining members (ir_enable) advance
 * by inner sweeps: jc_group_residuals performs their outer step (update
 * u += d if sweeps ran, binary64 residual, r_lo), jc_group_iterate their
 * inner sweeps; a refining member must hold its iterate in copy 0.
 * ctxs is read during the call; the contexts must outlive the group and
 * must not be used on their own streams while the group exists.
 * flags: bit 0 = capture jc_group_iterate windows as HIP graphs (needs a
 * non-null stream); bit 1 = two sweeps of every member per launch
 * (temporal blocking; every member one block, else JC_ERR_INVALID; tiles
 * of 64 cells x 16 rows x max(planes, 32); the first inner sweep of a
 * refinement step and the last of an odd count are single-sweep launches;
 * results bitwise the same as one sweep per launch); bit 2 = three sweeps
 * per launch (the same conditions and tiles; a count that is not a
 * multiple of three ends with a two-sweep launch or a single sweep);
 * bit 3 = resident sweeps: every jc_group_iterate window is one launch per
 * class and parity of the members' (nz + 1) / 2 with one work-group per
 * member, which keeps its member's block on chip for the whole window
 * (members as for options.resident: one block of at most 32 planes,
 * (nx + 1) / 2 * ny <= 512, the LDS limit there, no refinement; else
 * JC_ERR_INVALID; not with bits 1 and 2; results bitwise the same).
 * tile: {cells per row 16|32|64 (or 96|128|256 when no member refines in
 * binary32 or bfloat16), rows 4|8|16|32 (64 to 1024 threads), planes >= 1} for every
 * launch of the group, or NULL for {64, 8, 32}; members' results do not
 * depend on it, their residual norms do in the last bits, so compare
 * mixes within one tile shape.  Host only until jc_group_bind. */
int jc_group_create(jc_ctx* const* ctxs, int n, void* hip_stream, int flags, const int tile[3],
                    jc_group** out);
/* Device scratch the group needs (joint tables, partial sums). */
int jc_group_footprint(const jc_group* g, size_t* bytes);
/* Attach caller-owned scratch (>= footprint, 256-byte aligned); orders the
 * group stream after every member's queued work; uploads the tables. */
int jc_group_bind(jc_group* g, void* dev_scratch, size_t bytes);
/* For callers that cannot allocate memory -- code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation: jc_group_bind with
 * the library's own device scratch instead of caller memory.  Each device
 * holds one static array of JC_STATIC_SCRATCH_BYTES (16 MiB, kept until
 * the process ends); the group's scratch (jc_group_footprint) must fit in
 * it, else JC_ERR_NOMEM.  The array of the current device (hipGetDevice;
 * the members' arenas must be on it) is held by this group until
 * jc_group_destroy: binding a second group on the same device meanwhile
 * returns JC_ERR_STATE.  The used range is cleared before the tables are
 * uploaded (the array keeps the previous group's contents otherwise).
 * Allocates nothing: no device or pinned memory and no events -- the
 * group stream is ordered after the members' streams by waiting for them
 * on the host, and residuals come back through a pageable host buffer
 * made at jc_group_create.  Everything else is as after jc_group_bind.
 * Graph capture (flags bit 0) instantiates graphs in jc_group_iterate,
 * which allocates: create the group without it for an allocation-free
 * loop.  Overlapping use of one device's array by two groups would race;
 * the ownership rule above rejects it.  Waits for the group stream. */
#define JC_STATIC_SCRATCH_BYTES 16777216
int jc_group_bind_static(jc_group* g);
/* n sweeps of every member (inner sweeps for refining members).
 * JC_ERR_STATE if a refining member's residual is due, or if refining
 * members of one storage format are at different points of their step
 * (after leaving different groups): jc_group_residuals first. */
int jc_group_iterate(jc_group* g, int64_t n);
/* |r|_2 of every member's current iterate into host_l2[members], after the
 * outer step of refining members; waits for the stream.  JC_ERR_NONFINITE
 * if any norm is NaN/Inf (all norms are still written). */
int jc_group_residuals(jc_group* g, double* host_l2);
/* The stopping rule of independent solves in a group (serving): the
 * residual norms of jc_group_residuals, then for every member
 * host_rel[m] = |r| / |r_0| with |r_0| the norm this call saw first for the
 * member's current solve (kept in the context across groups; reset by
 * jc_load_field(U); 0 when |r_0| = 0), and host_done[m] = 1 when
 * host_rel[m] <= rtol or the member has run max_iter sweeps (iterations
 * since its load), else 0.  A member whose norm is NaN or infinite is not
 * done by the test and makes the call return JC_ERR_NONFINITE (all outputs
 * still written).  Waits for the stream. */
int jc_group_check(jc_group* g, double rtol, int64_t max_iter, double* host_rel, int* host_done);
/* Frees the group's host data, graphs and events (waits for its stream).
 * NULL-safe.  The scratch stays the caller's. */
void jc_group_destroy(jc_group* g);

/* ---- introspection (host only) -------------------------------------- */

int64_t jc_num_blocks(const jc_ctx* ctx);
int64_t jc_num_pairs(const jc_ctx* ctx);
int64_t jc_num_items(const jc_ctx* ctx);
/* out[0..2] interior n, out[3..5] global offset (block cell x is global
 * cell offset + x), out[6..11] neighbour block per face (-x,+x,-y,+y,-z,+z;
 * -1 = global boundary), out[12] row pitch in elements, out[13] plane
 * stride in elements, out[14..15] byte offset in the arena of element
 * (0,0,0) of ping-pong copy 0 and 1 (cell (x,y,z) is element
 * z*plane + y*pitch + x), out[16] current copy (0/1, valid once bound). */
int jc_block_info(const jc_ctx* ctx, int64_t i, int64_t out[17]);
/* out = {src_block, src_face, dst_block, dst_face, count, slow, fast,
 *        byte offset in the arena of the send buffer, of the receive
 *        buffer, row length ld}.  A buffer holds value (s, f) of the
 *        shared plane at element s * ld + f (ld = fast rounded up to even). */
int jc_pair_info(const jc_ctx* ctx, int64_t i, int64_t out[10]);
/* Iterations performed since the last jc_load_field(U). */
int64_t jc_iterations(const jc_ctx* ctx);
/* Current tile shape and work-list length: {tile_x, tile_y, z_chunk, items}. */
int jc_tile_info(const jc_ctx* ctx, int64_t out[4]);

/* ---- synthetic inputs ------------------------------------------------- */

/* Fill a device global padded binary64 array (grid = interior nx, ny, nz)
 * with the seeded synthetic field of the Jacobi3D workloads: kind 0 =
 * Dirichlet shell U[0,1), interior 0; kind 1 = source, interior
 * 2 U[0,1) - 1, shell 0.  SplitMix64 in counter form: the field's
 * generator is seeded with output kind + 1 of SplitMix64(seed) and the
 * cell at flat padded index i takes output i + 1; U = top 53 bits * 2^-53.
 * Enqueued on hip_stream.  JC_ERR_INVALID on bad arguments. */
int jc_synth_field(void* dev_global_padded, const int64_t grid[3], uint64_t seed, int kind,
                   void* hip_stream);

/* ---- tile shape ------------------------------------------------------ */

/* Set the sweep's tile shape: tile_x cells per row (16, 32 or 64; or 96,
 * 128 or 256 -- a whole block row -- where the swept storage is binary64,
 * i.e. not on a context refining in binary32 or bfloat16), tile_y rows (4,
 * 8, 16 or 32), with tile_x / 2 x tile_y between 64 and 1024 threads, so
 * that a work-group is whole 64-lane waves (16-cell rows need 8 rows or
 * more, 256-cell rows 8 or fewer), and z_chunk planes per work item (>= 1, within
 * the work-list region sized at creation: >= 16 always fits).  Results
 * are bitwise independent of the shape; residual norms change in the last
 * bits (reduction order).  Uploads the new work list (waits for the stream
 * when bound). */
int jc_set_tiles(jc_ctx* ctx, int tile_x, int tile_y, int z_chunk);

/* Shape of the multi-sweep launch of temporal blocking: rows of its tile
 * (8, 16 or 24 for two sweeps per launch, 8 or 16 for three; the tile is 64
 * cells wide) and planes per work-group (>= 1).
 * Results are bitwise independent of it.  JC_ERR_STATE unless the context
 * was created with temporal = 1. */
int jc_set_temporal_tiles(jc_ctx* ctx, int rows, int z_chunk);
/* out = {sweeps per launch (2 or 3; 0 without temporal blocking), rows,
 * planes per work-group} of the multi-sweep launch.  Until set (jc_set_temporal_tiles or jc_autotune), the planes
 * follow the one-sweep z_chunk, at least 32, halved (down to 8) while a
 * launch would have fewer than 1024 work-groups. */
int jc_temporal_info(const jc_ctx* ctx, int64_t out[3]);

/* Time `reps` sweeps of every valid candidate shape (tile_x in {64, 32,
 * 16}, and 96, 128 or 256 where the storage is binary64 and they leave at
 * most 1/8 of the lanes idle, x tile_y in {4, 8, 16, 32} x z_chunk in {16,
 * 32, 64, ..., depth}) on
 * the bound stream after at least 150 ms of warm-up sweeps, time the four
 * fastest again in turn over three rounds and keep the fastest of those;
 * out = {tile_x, tile_y, z_chunk, microseconds per sweep}.  The sweep timed
 * is the one the context's solve loop runs: the plain sweep, or, on a
 * context with refinement buffers (ir_enable), the inner sweep of the
 * correction (the refinement arrays are zeroed first; every refinement
 * step rebuilds them; JC_ERR_STATE while a group's refinement step is in
 * progress on the context).  With temporal = 1 the two-sweep launch (of
 * the correction, on a context with refinement buffers) is then timed over
 * rows {8, 16, 24} x z chunks of 1/1 .. 1/16 of the depth (max(reps, 2)
 * launches each, the three fastest again over three rounds) and the
 * fastest kept (jc_temporal_info); the one shape serves both two-sweep
 * launches of the context.  The pace of the one-sweep launch is tuned for
 * the chosen shape (jc_autotune_pace); out[3] is then the time with it.  The trial sweeps write only
 * the other ping-pong copy and face slot, so the current iterate and
 * iteration count are unchanged.  Waits for the stream.  Needs a loaded
 * context. */
int jc_autotune(jc_ctx* ctx, int reps, int64_t out[4]);

/* Pace of the launch the context's solve loop runs: the one-sweep launch
 * (the plain sweep, or the inner sweep on a context with refinement
 * buffers), or on a temporal context its two- or three-sweep launch (whose
 * other launches then run unpaced).  The work-groups of a launch advance at different rates and
 * the launch lasts as long as the slowest, so the compute units of the
 * fast ones idle at its end.  With a pace of p ticks of the GPU's constant
 * 100 MHz clock, a work-group that reaches plane step k of its tile before
 * k * p ticks have passed since it started waits (a bounded sleep) until
 * then: the fast work-groups are held to a common rate and all finish
 * together.  Results are bitwise independent of the pace; 0 = none
 * (default).  0 <= ticks <= 10000, else JC_ERR_INVALID.  jc_set_tiles and
 * jc_set_temporal_tiles reset the pace to 0 (a pace belongs to a shape). */
int jc_set_pace(jc_ctx* ctx, int64_t ticks);
int64_t jc_get_pace(const jc_ctx* ctx);
/* Time the context's solve-loop launch, in its current shape, with no
 * pace and with paces of 90, 91, .. 98 % of its measured time per plane step
 * (only where the launch runs its work-groups in one or two rounds on the
 * device's compute units; otherwise the pace stays 0), `reps` sweeps each
 * in three interleaved rounds after 150 ms of warm-up, and keep the
 * fastest.  out = {pace, microseconds per sweep with it, microseconds per
 * sweep without a pace}.  Trial sweeps leave the iterate as it is.  Waits
 * for the stream.  jc_autotune runs the same tuning after it has picked
 * the tile shape. */
int jc_autotune_pace(jc_ctx* ctx, int reps, int64_t out[3]);

/* ---- measurement ----------------------------------------------------- */

/* enable != 0: bracket every kernel launch of this context with HIP events
 * on its stream; jc_kernel_time returns the summed milliseconds and launch
 * count per kind (JC_K_*) since enabling, after waiting for the stream. */
int jc_set_timing(jc_ctx* ctx, int enable);
int jc_kernel_time(jc_ctx* ctx, int kind, double* ms_total, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* JC_H */
