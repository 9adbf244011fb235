// Shape limits of the resident sweep kernel (libjc, internal): shared by
// the host runtime, which validates contexts and groups against them, and
// the kernel's launcher.
#pragma once

#include <stdint.h>

namespace jc {

// Blocks that one work-group can sweep many times on chip (the resident
// sweep kernel): at most 32 planes, (nx + 1) / 2 * ny <= 512 cell pairs
// (one thread each), and LDS for four plane buffers plus the ghost ring
// of every plane within 64 KiB.
constexpr int kResidentMaxPlanes = 32;
constexpr int kResidentMaxPairs = 512;
constexpr int64_t kResidentMaxLds = 65536;

inline constexpr int64_t resident_lds_bytes(int64_t nx, int64_t ny, int64_t nz)
{
    const int64_t pw = 2 * ((nx + 1) / 2);
    return 8 * (4 * ny * pw + 2 * nz * ny + 2 * nz * pw);
}

inline constexpr bool resident_fits(int64_t nx, int64_t ny, int64_t nz)
{
    return nx >= 1 && ny >= 1 && nz >= 1 && nz <= kResidentMaxPlanes && (nx + 1) / 2 * ny <= kResidentMaxPairs &&
           resident_lds_bytes(nx, ny, nz) <= kResidentMaxLds;
}

// Launch variant of a block of nz planes (the kernel's step schedule): the
// parity of its number of two-plane steps per sweep, (nz + 1) / 2.
constexpr int kResidentVariants = 2;
inline constexpr int resident_variant(int64_t nz) { return (int)(((nz + 1) / 2) & 1); }

}  // namespace jc
