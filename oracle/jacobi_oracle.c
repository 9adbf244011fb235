/*
 * CPU oracle for the Jacobi3D proxy workload -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  It shares no source, header or helper with the GPU
 * library and must never be used as a fallback for it.
 *
 * What it computes (paper section 4.3, "Proxy Application: Jacobi3D"): the
 * Jacobi iterative method on a 3D grid, here one undecomposed grid, written
 * out as plainly as possible.  Readings of what the paper leaves open:
 *   - 7-point stencil, each interior cell becomes the average of its six
 *     face neighbours (plus b/6 when a source term b is present):
 *     u'(i) = (((((u(x-1) + u(x+1)) + u(y-1)) + u(y+1)) + u(z-1)) + u(z+1) + b) / 6
 *     summed in exactly that order, one IEEE division by 6;
 *   - strict Jacobi: every read is of the previous iterate (two buffers);
 *   - 1-cell Dirichlet shell, never updated;
 *   - residual r = (b + s) - 6 u with s the neighbour sum above, i.e. the
 *     residual of A u = b with A = 6I - (sum of face neighbours);
 *     its 2-norm is the square root of a pairwise (tree) sum of r^2;
 *   - iterative refinement with Jacobi inner sweeps on the correction
 *     equation A d = r, d stored in binary32 or bfloat16 (round to nearest
 *     even), sums and the division in binary32, outer residual and update
 *     in binary64.
 * Arrays are padded (nz+2) x (ny+2) x (nx+2), x unit-stride.
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* One Jacobi sweep: v(interior) from u.  The shell of v is not touched. */
void oracle_sweep(const double* u, double* v, const double* b,
                  int64_t nx, int64_t ny, int64_t nz)
{
    const int64_t sy = nx + 2;
    const int64_t sz = (nx + 2) * (ny + 2);
    int64_t z;
#pragma omp parallel for schedule(static)
    for (z = 1; z <= nz; ++z) {
        for (int64_t y = 1; y <= ny; ++y) {
            for (int64_t x = 1; x <= nx; ++x) {
                const int64_t i = z * sz + y * sy + x;
                double s = u[i - 1] + u[i + 1];
                s = s + u[i - sy];
                s = s + u[i + sy];
                s = s + u[i - sz];
                s = s + u[i + sz];
                if (b)
                    v[i] = (s + b[i]) / 6.0;
                else
                    v[i] = s / 6.0;
            }
        }
    }
}

/* Pairwise (tree) summation: split in halves down to 8 terms. */
static double pairwise_sum(const double* a, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i)
            s = s + a[i];
        return s;
    }
    int64_t h = n / 2;
    return pairwise_sum(a, h) + pairwise_sum(a + h, n - h);
}

/* Sum of r^2 over the interior; r = (b + s) - 6u.  Each z-plane is summed
 * pairwise, then the plane sums are summed pairwise. */
double oracle_residual_sumsq(const double* u, const double* b,
                             int64_t nx, int64_t ny, int64_t nz)
{
    const int64_t sy = nx + 2;
    const int64_t sz = (nx + 2) * (ny + 2);
    double* planes = (double*)malloc(sizeof(double) * (size_t)(nz > 0 ? nz : 1));
    int64_t z;
#pragma omp parallel
    {
        double* row = (double*)malloc(sizeof(double) * (size_t)(nx * ny > 0 ? nx * ny : 1));
#pragma omp for schedule(static)
        for (z = 1; z <= nz; ++z) {
            int64_t k = 0;
            for (int64_t y = 1; y <= ny; ++y) {
                for (int64_t x = 1; x <= nx; ++x) {
                    const int64_t i = z * sz + y * sy + x;
                    double s = u[i - 1] + u[i + 1];
                    s = s + u[i - sy];
                    s = s + u[i + sy];
                    s = s + u[i - sz];
                    s = s + u[i + sz];
                    double r = b ? (b[i] + s) - 6.0 * u[i] : s - 6.0 * u[i];
                    row[k++] = r * r;
                }
            }
            planes[z - 1] = pairwise_sum(row, k);
        }
        free(row);
    }
    double total = pairwise_sum(planes, nz);
    free(planes);
    return total;
}

double oracle_residual(const double* u, const double* b,
                       int64_t nx, int64_t ny, int64_t nz)
{
    return sqrt(oracle_residual_sumsq(u, b, nx, ny, nz));
}

/*
 * Plain Jacobi for `iters` sweeps on the padded grid `u` (shell = Dirichlet
 * values, interior = initial iterate); the final iterate is left in `u`.
 * If `every` > 0, the residual norm of iterates 0, every, 2*every, ... (and
 * of the last iterate) is written to hist (capacity hist_cap); returns the
 * number of history entries written.
 */
int64_t oracle_jacobi(double* u, const double* b, int64_t nx, int64_t ny, int64_t nz,
                      int64_t iters, int64_t every, double* hist, int64_t hist_cap)
{
    const size_t total = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2);
    double* v = (double*)malloc(sizeof(double) * total);
    memcpy(v, u, sizeof(double) * total);
    double* cur = u;
    double* nxt = v;
    int64_t nh = 0;
    for (int64_t k = 0; k < iters; ++k) {
        if (every > 0 && k % every == 0 && nh < hist_cap)
            hist[nh++] = oracle_residual(cur, b, nx, ny, nz);
        oracle_sweep(cur, nxt, b, nx, ny, nz);
        double* t = cur; cur = nxt; nxt = t;
    }
    if (every > 0 && nh < hist_cap)
        hist[nh++] = oracle_residual(cur, b, nx, ny, nz);
    if (cur != u)
        memcpy(u, cur, sizeof(double) * total);
    free(v);
    return nh;
}

/* ------------------------------------------------------------------ */
/* bfloat16: the upper 16 bits of a binary32, rounded to nearest even. */
static uint16_t bf16_from_f32(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    if ((x & 0x7fffffffu) > 0x7f800000u)          /* NaN stays NaN (quiet) */
        return (uint16_t)((x >> 16) | 0x0040u);
    uint32_t lower = x & 0xffffu;
    uint32_t upper = x >> 16;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u)))
        upper += 1u;                               /* carries into the exponent if needed */
    return (uint16_t)upper;
}

static float f32_from_bf16(uint16_t h)
{
    uint32_t x = (uint32_t)h << 16;
    float f;
    memcpy(&f, &x, 4);
    return f;
}

void oracle_bf16_round(const float* in, uint16_t* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = bf16_from_f32(in[i]);
}

/* Low-precision storage: 1 = binary32, 2 = bfloat16 (value kept as float). */
static float store_lo(float x, int storage)
{
    return storage == 2 ? f32_from_bf16(bf16_from_f32(x)) : x;
}

/*
 * Mixed-precision iterative refinement (inner Jacobi on A d = r):
 *   outer: r = (b + s(u)) - 6u in binary64, rel = |r| / |r_0|, stop when
 *          rel <= rtol; r_lo = r rounded to the storage format;
 *   inner: d = 0 (homogeneous shell), `inner` sweeps of
 *          d' = lo((((((d(x-1) + d(x+1)) + d(y-1)) + d(y+1)) + d(z-1)) + d(z+1) + r_lo) / 6)
 *          with binary32 sums and division;
 *   update: u = u + (double) d.
 * storage 0 runs the same refinement with binary64 d and r (no rounding).
 * The cap max_inner counts inner sweeps.  hist receives rel of every outer
 * check.  Returns 0 when converged, 1 when the cap stopped it.
 */
int oracle_ir(double* u, const double* b, int64_t nx, int64_t ny, int64_t nz,
              int storage, int64_t inner, double rtol, int64_t max_inner,
              double* out_rel, int64_t* out_inner, double* hist, int64_t hist_cap,
              int64_t* out_nhist)
{
    const int64_t sy = nx + 2;
    const int64_t sz = (nx + 2) * (ny + 2);
    const size_t total = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2);
    double* r = (double*)calloc(total, sizeof(double));
    double* d64 = (double*)calloc(total, sizeof(double));
    double* e64 = (double*)calloc(total, sizeof(double));
    float* rlo = (float*)calloc(total, sizeof(float));
    float* d32 = (float*)calloc(total, sizeof(float));
    float* e32 = (float*)calloc(total, sizeof(float));
    int64_t done = 0, nh = 0;
    double r0 = -1.0, rel = 1.0;
    int status = 1;
    for (;;) {
        /* outer residual, binary64 */
        int64_t z;
#pragma omp parallel for schedule(static)
        for (z = 1; z <= nz; ++z)
            for (int64_t y = 1; y <= ny; ++y)
                for (int64_t x = 1; x <= nx; ++x) {
                    const int64_t i = z * sz + y * sy + x;
                    double s = u[i - 1] + u[i + 1];
                    s = s + u[i - sy];
                    s = s + u[i + sy];
                    s = s + u[i - sz];
                    s = s + u[i + sz];
                    r[i] = b ? (b[i] + s) - 6.0 * u[i] : s - 6.0 * u[i];
                }
        double nrm = oracle_residual(u, b, nx, ny, nz);
        if (r0 < 0.0)
            r0 = nrm;
        rel = r0 > 0.0 ? nrm / r0 : 0.0;
        if (nh < hist_cap)
            hist[nh++] = rel;
        if (rel <= rtol) { status = 0; break; }
        if (done >= max_inner) { status = 1; break; }
        int64_t m = inner;
        if (m > max_inner - done)
            m = max_inner - done;
        if (storage == 0) {
            memset(d64, 0, sizeof(double) * total);
            memset(e64, 0, sizeof(double) * total);
            for (int64_t j = 0; j < m; ++j) {
#pragma omp parallel for schedule(static)
                for (z = 1; z <= nz; ++z)
                    for (int64_t y = 1; y <= ny; ++y)
                        for (int64_t x = 1; x <= nx; ++x) {
                            const int64_t i = z * sz + y * sy + x;
                            double s = d64[i - 1] + d64[i + 1];
                            s = s + d64[i - sy];
                            s = s + d64[i + sy];
                            s = s + d64[i - sz];
                            s = s + d64[i + sz];
                            e64[i] = (s + r[i]) / 6.0;
                        }
                double* t = d64; d64 = e64; e64 = t;
            }
#pragma omp parallel for schedule(static)
            for (z = 1; z <= nz; ++z)
                for (int64_t y = 1; y <= ny; ++y)
                    for (int64_t x = 1; x <= nx; ++x) {
                        const int64_t i = z * sz + y * sy + x;
                        u[i] = u[i] + d64[i];
                    }
        } else {
#pragma omp parallel for schedule(static)
            for (z = 1; z <= nz; ++z)
                for (int64_t y = 1; y <= ny; ++y)
                    for (int64_t x = 1; x <= nx; ++x) {
                        const int64_t i = z * sz + y * sy + x;
                        rlo[i] = store_lo((float)r[i], storage);
                    }
            memset(d32, 0, sizeof(float) * total);
            memset(e32, 0, sizeof(float) * total);
            for (int64_t j = 0; j < m; ++j) {
#pragma omp parallel for schedule(static)
                for (z = 1; z <= nz; ++z)
                    for (int64_t y = 1; y <= ny; ++y)
                        for (int64_t x = 1; x <= nx; ++x) {
                            const int64_t i = z * sz + y * sy + x;
                            float s = d32[i - 1] + d32[i + 1];
                            s = s + d32[i - sy];
                            s = s + d32[i + sy];
                            s = s + d32[i - sz];
                            s = s + d32[i + sz];
                            e32[i] = store_lo((s + rlo[i]) / 6.0f, storage);
                        }
                float* t = d32; d32 = e32; e32 = t;
            }
#pragma omp parallel for schedule(static)
            for (z = 1; z <= nz; ++z)
                for (int64_t y = 1; y <= ny; ++y)
                    for (int64_t x = 1; x <= nx; ++x) {
                        const int64_t i = z * sz + y * sy + x;
                        u[i] = u[i] + (double)d32[i];
                    }
        }
        done += m;
    }
    *out_rel = rel;
    *out_inner = done;
    *out_nhist = nh;
    free(r); free(d64); free(e64); free(rlo); free(d32); free(e32);
    return status;
}

/* Threads OpenMP will use (1 when built without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
