// Device-visible tables shared by the host runtime and the HIP kernels of
// libjc.  Plain structs of pointers and integers, uploaded into the
// caller's arena at bind time and read by the kernels with scalar loads.
#pragma once

#include <stdint.h>

namespace jc {

// bfloat16 storage: the upper 16 bits of a binary32.
struct bf16 {
    uint16_t bits;
};

// Block faces in the order -x, +x, -y, +y, -z, +z.
enum Face { XM = 0, XP = 1, YM = 2, YP = 3, ZM = 4, ZP = 5 };

inline constexpr int opposite(int f) { return f ^ 1; }

// Elements of a 128-byte line: arrays are laid out so that interior
// cell x = 1 of every row starts a line; the x = 0 ghost is the last
// element of the line before.
template <typename T> inline constexpr int64_t line_elems() { return 128 / (int64_t)sizeof(T); }

// One block of the decomposition (a "chare" of the paper): its own
// ghost-padded arrays, indexed (x, y, z) in [0, n+1]^3 as
// base[z * plane + y * pitch + x].
struct BlockDesc {
    double* u[2];            // iterate, ping-pong, element (0,0,0)
    const double* b;         // source, same layout, or null
    void* d[2];              // refinement correction (low precision), ping-pong
    void* rlo;               // refinement residual (low precision)
    // Face buffers of the pairing, per face and per slot.  gin: where the
    // ghost values of face f are read from in fused mode (null: the
    // block's own ghost plane).  gout: where the face values of face f
    // are written in fused mode (null: face on the global boundary).
    double* gin[6][2];
    double* gout[6][2];
    void* lgin[6][2];        // same for the low-precision correction
    void* lgout[6][2];
    // Dirichlet ghost columns of the x faces that have no pair (null for
    // a paired face), laid out like an x face buffer: value (z - 1, y - 1)
    // at (z - 1) * face_ld(ny) + (y - 1).  Fused sweeps read them: there a
    // ghost column of the block arrays would cost a 128-byte line per row
    // for one value; here it is contiguous.  xg: of the iterate (written
    // when u is loaded; both copies hold the same ghosts); lxg: of the
    // refinement correction (zeros).
    const double* xg[2];
    const void* lxg[2];
    int32_t n[3];            // interior nx, ny, nz
    int32_t pitch;           // row pitch (elements) of u and b
    int64_t plane;           // plane stride (elements) of u and b
    int32_t lpitch;          // row pitch of d and rlo
    int32_t pad0;
    int64_t lplane;          // plane stride of d and rlo
    int32_t off[3];          // global interior offset: block cell x is global cell off[0] + x
    int32_t pad1;
};

// One directed face pair: the send side (src block, src face) and the
// receive side pre-posted for it (dst block, opposite face).  buf[0] is
// the send buffer, buf[1] the receive buffer; in fused mode the two are
// the two parity slots the producer and consumer alternate between.
// Buffers hold the shared plane slow-major with rows padded to an even
// length ld = fast rounded up to 2 (so every pair of cells starting at an
// even index is a 16-byte aligned vector): value (s, f) at s * ld + f.
struct PairDesc {
    int32_t src_block, src_face, dst_block, dst_face;
    int32_t slow, fast;      // extents of the shared plane, slow-major
    int64_t count;           // slow * fast values
    int64_t span;            // slow * ld elements per buffer
    double* buf[2];
    void* lbuf[2];           // low-precision buffers for the correction
};

// Row length of a face buffer whose fast extent is `fast`.
inline constexpr int64_t face_ld(int64_t fast) { return (fast + 1) & ~(int64_t)1; }

// A tile of the work list: block, origin (0-based interior offsets), the
// z range, and the ping-pong flip of its owner relative to the launch.
struct Item {
    int32_t block;
    int32_t x0, y0, z0;
    int32_t zlen;
    int32_t flip;
    int32_t owner;           // member index (groups) -- selects the partial slot
    int32_t pad;
};

static_assert(sizeof(Item) == 32, "Item layout");

}  // namespace jc
