// Host check of the sweep's division helpers (paper_2102_12416_amd/csrc/
// jc_div6.h) against the host's IEEE division s / 6.
//
// Built host-only (hipcc --offload-host-only) by tests/test_div6_cpu.py.
// binary32: every one of the 2^32 bit patterns (NaN, +-inf and
// subnormals included) through div6 and through div6_pair.  binary64:
// edge sets -- every exponent with significands near 0, 1/2, 1 and the
// top, the neighbourhoods of the switch thresholds, +-0, subnormals, the
// largest finite values, +-inf, NaNs -- and random patterns of every
// exponent.  Results must be bitwise equal, except that any NaN matches
// any NaN (IEEE 754 fixes no payload for an operation's NaN result).
// Prints one line "checked <n32> <n64> mismatches <m>" and exits 0 only
// when m == 0; the first mismatches are listed on stderr.
#include <cinttypes>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "jc_div6.h"

using jc::div6;
using jc::div6_pair;

static uint64_t bits64(double x)
{
    uint64_t u;
    std::memcpy(&u, &x, 8);
    return u;
}
static double from64(uint64_t u)
{
    double x;
    std::memcpy(&x, &u, 8);
    return x;
}
static uint32_t bits32(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return u;
}
static float from32(uint32_t u)
{
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

static bool same64(double a, double b) { return (std::isnan(a) && std::isnan(b)) || bits64(a) == bits64(b); }
static bool same32(float a, float b) { return (std::isnan(a) && std::isnan(b)) || bits32(a) == bits32(b); }

static uint64_t g_bad = 0;
static void bad64(double s, double got, double want)
{
#pragma omp critical
    {
        if (g_bad < 20)
            std::fprintf(stderr, "binary64 s=%a (0x%016" PRIx64 "): got %a want %a\n", s, bits64(s), got, want);
        ++g_bad;
    }
}
static void bad32(float s, float got, float want)
{
#pragma omp critical
    {
        if (g_bad < 20)
            std::fprintf(stderr, "binary32 s=%a (0x%08x): got %a want %a\n", (double)s, bits32(s), (double)got,
                         (double)want);
        ++g_bad;
    }
}

// the host quotient, kept out of any constant folding or contraction
__attribute__((noinline)) static double ieee64(double s) { return s / 6.0; }
__attribute__((noinline)) static float ieee32(float s) { return s / 6.0f; }

static void check64(double s, double partner)
{
    const double want = ieee64(s);
    if (!same64(div6(s), want)) bad64(s, div6(s), want);
    double va, vb;
    div6_pair(s, partner, va, vb);
    if (!same64(va, want)) bad64(s, va, want);
    if (!same64(vb, ieee64(partner))) bad64(partner, vb, ieee64(partner));
}

static uint64_t splitmix(uint64_t& st)
{
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int main()
{
    // ---- binary32: all patterns, each also as the second of a pair ----
    uint64_t n32 = 0;
#pragma omp parallel for schedule(static) reduction(+ : n32)
    for (int64_t hi = 0; hi < (int64_t)1 << 16; ++hi) {
        for (uint32_t lo = 0; lo < (1u << 16); ++lo) {
            const uint32_t u = ((uint32_t)hi << 16) | lo;
            const float s = from32(u);
            const float want = ieee32(s);
            const float got = div6(s);
            if (!same32(got, want)) bad32(s, got, want);
            // pair with a partner that is ordinary, so the branch is taken
            // by one side only, and with the pattern's own negation
            float va, vb;
            div6_pair(s, 1.5f, va, vb);
            if (!same32(va, want) || bits32(vb) != bits32(0.25f)) bad32(s, va, want);
            div6_pair(-s, s, va, vb);
            if (!same32(va, ieee32(-s)) || !same32(vb, want)) bad32(s, vb, want);
            ++n32;
        }
    }

    // ---- binary64: edge sets over every exponent, then random patterns ----
    uint64_t n64 = 0;
    const uint64_t mant_edges[] = {0, 1, 2, 3, 0x5555555555555ull, 0x8000000000000ull, 0xaaaaaaaaaaaaaull,
                                   0xffffffffffffdull, 0xffffffffffffeull, 0xfffffffffffffull};
#pragma omp parallel for schedule(dynamic) reduction(+ : n64)
    for (int e = 0; e < 2048; ++e) {
        uint64_t st = 0x12416ull + (uint64_t)e;
        for (int sign = 0; sign < 2; ++sign) {
            for (uint64_t m : mant_edges) {
                const uint64_t u = ((uint64_t)sign << 63) | ((uint64_t)e << 52) | m;
                check64(from64(u), 1.5);
                ++n64;
            }
            for (int k = 0; k < 20000; ++k) {
                const uint64_t m = splitmix(st) & 0xfffffffffffffull;
                const uint64_t u = ((uint64_t)sign << 63) | ((uint64_t)e << 52) | m;
                const uint64_t v = splitmix(st);
                check64(from64(u), from64(v));
                ++n64;
            }
        }
    }
    // neighbourhoods of the thresholds (s near 2^-1000 and 1.5 * 2^-1000,
    // v near 2^-1002), of the normal range and of the largest values
    const double centres[] = {0x1p-1000, 0x1.8p-1000, 0x1p-1002 * 6.0, 0x1p-1022, 0x1p-1022 * 6.0,
                              0x1p-1074, 0x1.fffffffffffffp+1023, 0x1p+1023, 6.0, 1.0};
    for (double c : centres) {
        const uint64_t u = bits64(c);
        for (int64_t d = -100000; d <= 100000; ++d) {
            const uint64_t w = u + (uint64_t)d;
            if ((w & 0x7ff0000000000000ull) == 0x7ff0000000000000ull) continue;   // ran past the top
            check64(from64(w), 1.0);
            check64(-from64(w), 1.0);
            n64 += 2;
        }
    }
    const double specials[] = {0.0, -0.0, INFINITY, -INFINITY, NAN, -NAN, 0x1p-1074, -0x1p-1074, 3.5e-320,
                               -1.7e308, 1.7e308, 1.0e308, 2.5e307, 6.0, -6.0, 1.0 / 3.0};
    for (double a : specials)
        for (double b : specials) {
            check64(a, b);
            ++n64;
        }
    // signalling and quiet NaN payloads, both signs
    const uint64_t nans[] = {0x7ff0000000000001ull, 0x7ff8000000000001ull, 0xfff0000000000123ull,
                             0xfff8000000000000ull, 0x7fffffffffffffffull};
    for (uint64_t u : nans) {
        check64(from64(u), 2.0);
        ++n64;
    }

    std::printf("checked %" PRIu64 " %" PRIu64 " mismatches %" PRIu64 "\n", n32, n64, g_bad);
    return g_bad == 0 ? 0 : 1;
}
