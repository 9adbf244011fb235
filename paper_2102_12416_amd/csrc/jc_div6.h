// Correctly rounded division by 6 for the Jacobi update (libjc, internal).
//
// The update of the 7-point Jacobi sweep (paper section 4.3) is the
// neighbour sum over 6, with one IEEE division, so that every block of
// every decomposition computes the same bits as a plain s / 6.  The
// general division sequence is long; this is Markstein's correction step
// (Markstein, IBM J. Res. Dev. 34(1), 1990): with y = RN(1/6), q = RN(s y)
// is a faithful quotient, r = s - 6q is exact through an FMA, and
// RN(q + r y) is the correctly rounded quotient while the quotient is a
// normal number.  It fails in two places, and those inputs take the IEEE
// division instead:
//  - tiny s (quotient near or below the normal range; also +-0, whose
//    sign the correction step loses): the fast result is tiny too;
//  - s = +-inf or NaN: q = +-inf, so r = inf - inf is NaN, where s / 6 is
//    +-inf.  The fast result is NaN.
// Both are caught by one test on the fast result: |v| >= T fails for a
// NaN and for every tiny v.  T is chosen so that |v| >= T implies |s| at
// least 1.5 times the threshold of the range where the fast step was
// verified (|s| >= 2^-1000 for binary64, 2^-100 for binary32), while every
// s below that threshold gives |v| < T: the result equals s / 6 for every
// input, binary32 checked over all 2^32 patterns, binary64 over edge sets
// and random patterns.
//
// These functions are __host__ __device__ so that the same code can be
// checked against the host's division.
#pragma once

#include <hip/hip_runtime.h>

namespace jc {

__host__ __device__ __forceinline__ double div6_fast(double s)
{
    const double y = 0x1.5555555555555p-3;
    const double q = s * y;
    return __builtin_fma(__builtin_fma(-6.0, q, s), y, q);
}

__host__ __device__ __forceinline__ float div6_fast(float s)
{
    const float y = 0x1.555556p-3f;
    const float q = s * y;
    return __builtin_fmaf(__builtin_fmaf(-6.0f, q, s), y, q);
}

// true where the fast result v must be replaced by the IEEE quotient
// (v tiny, zero or NaN); written so that a NaN compares as "replace"
__host__ __device__ __forceinline__ bool div6_redo(double v) { return !(__builtin_fabs(v) >= 0x1p-1002); }
__host__ __device__ __forceinline__ bool div6_redo(float v) { return !(__builtin_fabsf(v) >= 0x1p-102f); }

template <typename C>
__host__ __device__ __forceinline__ C div6(C s)
{
    C v = div6_fast(s);
    if (__builtin_expect(div6_redo(v), 0))
        v = s / C(6);
    return v;
}

// A pair with one (rarely taken) branch to the IEEE division.
template <typename C>
__host__ __device__ __forceinline__ void div6_pair(C sa, C sb, C& va, C& vb)
{
    va = div6_fast(sa);
    vb = div6_fast(sb);
    const bool ra = div6_redo(va), rb = div6_redo(vb);
    if (__builtin_expect(ra || rb, 0)) {
        va = ra ? sa / C(6) : va;
        vb = rb ? sb / C(6) : vb;
    }
}

}  // namespace jc
