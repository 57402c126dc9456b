// Pieces of the partial (top-k) factorisation: the random start block of the
// range finder from SplitMix64 (a counter-based generator: Steele, Lea &
// Flood, OOPSLA 2014), FP64 sums of squares (the weight outside the
// subspace), and the diagonal shift of the first Cholesky QR pass (shifted
// Cholesky QR: Fukaya, Kannan, Nakatsukasa, Yamamoto & Yanagisawa, SIAM J.
// Sci. Comput. 42, 2020).
#include <algorithm>

#include "ea_dev.h"
#include "ea_kernels.h"

namespace {

// output(x) = mix(seed + (x + 1) gamma), arithmetic mod 2^64
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed,
                                                         unsigned long long x) {
    unsigned long long z = seed + (x + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 2 u - 1 with u = (top 53 bits) 2^-53: every step is exact in FP64
__device__ __forceinline__ double uniform_pm1(unsigned long long seed, unsigned long long x) {
    const double u = (double)(splitmix64(seed, x) >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

constexpr int SQ_THREADS = 256, SQ_PARTS = 512;

}  // namespace

// out[e] = (2u(base + 2e) - 1) + i (2u(base + 2e + 1) - 1), e = c rows + r
__global__ __launch_bounds__(256) void k_omega(unsigned long long seed, unsigned long long base,
                                               size_t n, double2 *__restrict__ out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        out[e] = make_double2(uniform_pm1(seed, base + 2ull * e),
                              uniform_pm1(seed, base + 2ull * e + 1ull));
}
void launch_omega(unsigned long long seed, unsigned long long base, size_t n, double *out,
                  hipStream_t s) {
    if (n == 0) return;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    k_omega<<<(unsigned)blocks, 256, 0, s>>>(seed, base, n, (double2 *)out);
}

// Sum of |x|^2 over n complex FP64 values: a fixed grid of SQ_PARTS blocks
// (grid-stride), then one block adds the partial sums in a fixed order, so
// the result is the same on every run.
__global__ __launch_bounds__(SQ_THREADS) void k_sumsq_part(const double2 *__restrict__ x, size_t n,
                                                          double *__restrict__ part) {
    __shared__ double red[SQ_THREADS];
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * SQ_THREADS;
    for (size_t e = (size_t)blockIdx.x * SQ_THREADS + threadIdx.x; e < n; e += stride) {
        const double2 v = x[e];
        acc += v.x * v.x + v.y * v.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = SQ_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(SQ_THREADS) void k_sumsq_final(const double *__restrict__ part,
                                                           double *__restrict__ out) {
    __shared__ double red[SQ_THREADS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < SQ_PARTS; i += SQ_THREADS) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = SQ_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}
size_t sumsq_part_doubles() { return SQ_PARTS; }
void launch_sumsq(const double *x, size_t n, double *part, double *out, hipStream_t s) {
    k_sumsq_part<<<SQ_PARTS, SQ_THREADS, 0, s>>>((const double2 *)x, n, part);
    k_sumsq_final<<<1, SQ_THREADS, 0, s>>>(part, out);
}

// out = max(0, a - b)
__global__ void k_resid(const double *__restrict__ a, const double *__restrict__ b,
                        double *__restrict__ out) {
    if (threadIdx.x == 0) out[0] = fmax(0.0, a[0] - b[0]);
}
void launch_resid(const double *a, const double *b, double *out, hipStream_t s) {
    k_resid<<<1, 64, 0, s>>>(a, b, out);
}

// G (n x n, complex FP64): G_ii += rel * trace(G) (real part).
__global__ __launch_bounds__(256) void k_shift_diag(double2 *__restrict__ G, int n, double rel) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += G[(size_t)i * n + i].x;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double shift = rel * red[0];
    for (int i = threadIdx.x; i < n; i += 256) G[(size_t)i * n + i].x += shift;
}
void launch_shift_diag(void *G, int n, double rel, hipStream_t s) {
    if (n > 0) k_shift_diag<<<1, 256, 0, s>>>((double2 *)G, n, rel);
}
