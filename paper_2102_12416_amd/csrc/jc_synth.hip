// Seeded synthetic inputs generated on the device.
//
// The same recipe as the host-side input module: SplitMix64 (Steele, Lea
// and Flood, OOPSLA 2014) in counter form -- the k-th output (k >= 1) of a
// generator seeded with s is mix64(s + k * gamma) -- with the field's own
// generator seeded by output stream + 1 of SplitMix64(seed), and the
// value of a cell drawn as output (flat padded index + 1).  The top 53
// bits give U[0, 1); the source is 2 U - 1.  Used to build request fields
// in place on the GPU instead of moving them from the host.

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "jc.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// kind 0: shell = U[0,1) (stream 0), interior = 0; kind 1: interior =
// 2 U[0,1) - 1 (stream 1), shell = 0.
__global__ void __launch_bounds__(256)
k_synth(double* __restrict__ out, int64_t nx, int64_t ny, int64_t nz, uint64_t key, int kind)
{
    const int64_t px = nx + 2, py = ny + 2;
    const int64_t total = px * py * (nz + 2);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t x = i % px;
        const int64_t y = (i / px) % py;
        const int64_t z = i / (px * py);
        const bool shell = x == 0 || x == nx + 1 || y == 0 || y == ny + 1 || z == 0 || z == nz + 1;
        double v = 0.0;
        if (shell == (kind == 0)) {
            const uint64_t r = mix64(key + (uint64_t)(i + 1) * kGamma);
            const double u = (double)(r >> 11) * 0x1.0p-53;
            v = kind == 0 ? u : 2.0 * u - 1.0;
        }
        out[i] = v;
    }
}

}  // namespace

extern "C" int jc_synth_field(void* dev_global_padded, const int64_t grid[3], uint64_t seed, int kind,
                              void* hip_stream)
{
    if (!dev_global_padded || !grid || (kind != 0 && kind != 1))
        return JC_ERR_INVALID;
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 1 || grid[a] > ((int64_t)1 << 30))
            return JC_ERR_INVALID;
    const uint64_t key = mix64(seed + (uint64_t)(kind + 1) * kGamma);
    const int64_t total = (grid[0] + 2) * (grid[1] + 2) * (grid[2] + 2);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_synth, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<double*>(dev_global_padded), grid[0], grid[1], grid[2], key, kind);
    return hipGetLastError() == hipSuccess ? JC_OK : JC_ERR_DEVICE;
}
