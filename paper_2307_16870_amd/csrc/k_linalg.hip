// Contraction, small dense kernels, column norms, truncation search and
// write-back of the two-site update (paper Sec. V-VI).
#include "ea_dev.h"
#include "ea_kernels.h"

#include <math.h>

// ---------------------------------------------------------------------------
// Two-site contraction with the gate fused in the epilogue.
// A: (chiL*D) x chiM row-major; B: chiM x (D*chiR) row-major; G: D^2 x D^2.
// One thread owns one (l, r) pair and all D*D (t1, t2) accumulators, so the
// gate is applied in registers before the single write of Theta.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(256) void k_theta(const cx<T> *__restrict__ A,
                                               const cx<T> *__restrict__ B,
                                               const cx<T> *__restrict__ G,
                                               cx<T> *__restrict__ W, int chiL, int chiM,
                                               int chiR, int orient) {
    constexpr int TL = 16, TR = 16, KT = 16;
    __shared__ cx<T> As[TL * D][KT + 1];
    __shared__ cx<T> Bs[KT][D][TR + 1];
    __shared__ cx<T> Gs[D * D][D * D];
    const int tid = threadIdx.x;
    const int l0 = blockIdx.y * TL, r0 = blockIdx.x * TR;
    const int tx = tid % 16, ty = tid / 16;
    const int ll = orient == 0 ? tx : ty;  // fastest thread index along the
    const int rl = orient == 0 ? ty : tx;  // contiguous output dimension
    for (int e = tid; e < D * D * D * D; e += 256) Gs[e / (D * D)][e % (D * D)] = G[e];
    cx<T> acc[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) acc[a][b] = zero_cx<T>();
    const int nrowsA = chiL * D;
    for (int k0 = 0; k0 < chiM; k0 += KT) {
        for (int e = tid; e < TL * D * KT; e += 256) {
            int rr = e / KT, kk = e % KT;
            int grow = l0 * D + rr, gk = k0 + kk;
            As[rr][kk] = (grow < nrowsA && gk < chiM) ? A[(size_t)grow * chiM + gk] : zero_cx<T>();
        }
        for (int e = tid; e < KT * D * TR; e += 256) {
            int kk = e / (D * TR), rem = e % (D * TR);
            int t2 = rem / TR, rr = rem % TR;
            int gk = k0 + kk, gr = r0 + rr;
            Bs[kk][t2][rr] = (gk < chiM && gr < chiR)
                                 ? B[(size_t)gk * (D * chiR) + (size_t)t2 * chiR + gr]
                                 : zero_cx<T>();
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < KT; ++kk) {
            cx<T> a[D], b[D];
#pragma unroll
            for (int t = 0; t < D; ++t) {
                a[t] = As[ll * D + t][kk];
                b[t] = Bs[kk][t][rl];
            }
#pragma unroll
            for (int t1 = 0; t1 < D; ++t1)
#pragma unroll
                for (int t2 = 0; t2 < D; ++t2) cmac(acc[t1][t2], a[t1], b[t2]);
        }
        __syncthreads();
    }
    const int l = l0 + ll, r = r0 + rl;
    if (l >= chiL || r >= chiR) return;
#pragma unroll
    for (int s1 = 0; s1 < D; ++s1) {
#pragma unroll
        for (int s2 = 0; s2 < D; ++s2) {
            cx<T> th = zero_cx<T>();
#pragma unroll
            for (int t1 = 0; t1 < D; ++t1)
#pragma unroll
                for (int t2 = 0; t2 < D; ++t2) cmac(th, Gs[s1 * D + s2][t1 * D + t2], acc[t1][t2]);
            const size_t row = (size_t)l * D + s1, col = (size_t)s2 * chiR + r;
            if (orient == 0)
                W[col * (size_t)(D * chiL) + row] = th;
            else
                W[row * (size_t)(D * chiR) + col] = conj(th);
        }
    }
}

template <typename T>
void launch_theta(const void *A, const void *B, const void *G, void *W, int chiL, int chiM,
                  int chiR, int d, int orient, hipStream_t s) {
    dim3 grid((chiR + 15) / 16, (chiL + 15) / 16);
    if (d == 2)
        k_theta<T, 2><<<grid, 256, 0, s>>>((const cx<T> *)A, (const cx<T> *)B,
                                           (const cx<T> *)G, (cx<T> *)W, chiL, chiM, chiR,
                                           orient);
    else
        k_theta<T, 4><<<grid, 256, 0, s>>>((const cx<T> *)A, (const cx<T> *)B,
                                           (const cx<T> *)G, (cx<T> *)W, chiL, chiM, chiR,
                                           orient);
}

// Plain complex GEMM, C = A B, row-major: the matrix-core kernel.
template <typename T>
void launch_gemm(const void *A, const void *B, void *C, int M, int N, int K, int lda, int ldb,
                 int ldc, hipStream_t s) {
    launch_zgemm<T>(0, 0, M, N, K, 1.0, 0.0, A, lda, B, ldb, 0.0, 0.0, C, ldc, s);
}

// ---------------------------------------------------------------------------
// One-site operator: out[l,s,r] = sum_t g[s,t] in[l,t,r].
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(256) void k_apply1(const cx<T> *in, cx<T> *out,
                                                const cx<T> *__restrict__ g, int chiL,
                                                int chiR) {
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)chiL * chiR) return;
    size_t l = idx / chiR, r = idx % chiR;
    cx<T> v[D];
#pragma unroll
    for (int t = 0; t < D; ++t) v[t] = in[(l * D + t) * chiR + r];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        cx<T> acc = zero_cx<T>();
#pragma unroll
        for (int t = 0; t < D; ++t) cmac(acc, g[s * D + t], v[t]);
        out[(l * D + s) * chiR + r] = acc;
    }
}

template <typename T>
void launch_apply1(const void *in, void *out, const void *g, int chiL, int d, int chiR,
                   hipStream_t s) {
    size_t n = (size_t)chiL * chiR;
    int blocks = (int)((n + 255) / 256);
    if (d == 2)
        k_apply1<T, 2><<<blocks, 256, 0, s>>>((const cx<T> *)in, (cx<T> *)out,
                                              (const cx<T> *)g, chiL, chiR);
    else
        k_apply1<T, 4><<<blocks, 256, 0, s>>>((const cx<T> *)in, (cx<T> *)out,
                                              (const cx<T> *)g, chiL, chiR);
}

template <typename T>
__global__ void k_eye(cx<T> *V, int n) {
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    size_t c = idx / n, r = idx % n;
    V[idx] = mk<T>(r == c ? T(1) : T(0), T(0));
}

template <typename T>
void launch_eye(void *V, int n, hipStream_t s) {
    size_t tot = (size_t)n * n;
    k_eye<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((cx<T> *)V, n);
}

// Row-major -> column-major by 32x32 LDS tiles, or an elementwise conjugate.
template <typename T>
__global__ __launch_bounds__(256) void k_to_colmajor(const cx<T> *__restrict__ in,
                                                     cx<T> *__restrict__ out, int M, int N) {
    __shared__ cx<T> tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int j = ty; j < 32; j += 8) {
        int r = r0 + j, c = c0 + tx;
        if (r < M && c < N) tile[j][tx] = in[(size_t)r * N + c];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        int c = c0 + j, r = r0 + tx;
        if (r < M && c < N) out[(size_t)c * M + r] = tile[tx][j];
    }
}

template <typename T>
__global__ void k_conj_copy(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, size_t n) {
    size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) out[idx] = conj(in[idx]);
}

template <typename T>
void launch_to_colmajor(const void *in, void *out, int M, int N, int conj_copy, hipStream_t s) {
    if (conj_copy) {
        size_t n = (size_t)M * N;
        k_conj_copy<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const cx<T> *)in,
                                                                   (cx<T> *)out, n);
    } else {
        dim3 grid((N + 31) / 32, (M + 31) / 32);
        k_to_colmajor<T><<<grid, 256, 0, s>>>((const cx<T> *)in, (cx<T> *)out, M, N);
    }
}

// ---------------------------------------------------------------------------
// Column norms in FP64: one workgroup per column.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_colnorms(const cx<T> *__restrict__ W, int m,
                                                  double *__restrict__ s_out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    const cx<T> *col = W + (size_t)j * m;
    double acc = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        cx<T> v = col[i];
        acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) s_out[j] = sqrt(red[0]);
}

template <typename T>
void launch_colnorms(const void *W, int m, int n, double *s_out, hipStream_t s) {
    k_colnorms<T><<<n, 256, 0, s>>>((const cx<T> *)W, m, s_out);
}

// Unit right vectors: one workgroup per column j divides column j of V
// (n x n) and of W = A V (m x n), both column-major, by the FP64 norm of
// V's column j.  W = A V still holds, V's columns have unit norm to the
// storage precision and W's column norms become the singular values; a
// low-precision rotation sequence otherwise leaves a norm drift in V that
// grows with the number of rotations applied.
template <typename T>
__global__ __launch_bounds__(256) void k_unit_right(cx<T> *__restrict__ W, int m,
                                                    cx<T> *__restrict__ V, int n) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    cx<T> *v = V + (size_t)j * n, *w = W + (size_t)j * m;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const cx<T> a = v[i];
        acc += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (!(red[0] > 0.0)) return;
    const double inv = 1.0 / sqrt(red[0]);
    for (int i = threadIdx.x; i < n; i += 256) {
        const cx<T> a = v[i];
        v[i] = mk<T>((T)(inv * (double)a.x), (T)(inv * (double)a.y));
    }
    for (int i = threadIdx.x; i < m; i += 256) {
        const cx<T> a = w[i];
        w[i] = mk<T>((T)(inv * (double)a.x), (T)(inv * (double)a.y));
    }
}

template <typename T>
void launch_unit_right(void *W, int m, void *V, int n, hipStream_t s) {
    k_unit_right<T><<<n, 256, 0, s>>>((cx<T> *)W, m, (cx<T> *)V, n);
}

// ---------------------------------------------------------------------------
// Sort (descending, ties by index), suffix sums of s^2 and the kept-rank
// search of Sec. VI in one workgroup.
// D(k) = sum_{j>=k} s_j^2; k_f = min{k >= 1: D(k) <= (1-f_t) T}.
// Each thread owns a contiguous chunk of sorted values and sums it from its
// tail (smallest first); chunk totals are combined by a reverse scan.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_sort_trunc(const double *__restrict__ s_raw, int r,
                                                     double f_t, int chi_max, double tau,
                                                     int mode, int forced_k,
                                                     const int *__restrict__ sweeps_dev,
                                                     int *__restrict__ perm,
                                                     double *__restrict__ s_sorted,
                                                     ea_dev_rec *__restrict__ rec,
                                                     const double *__restrict__ resid) {
    __shared__ double key[EA_SORT_MAX];
    __shared__ int idx[EA_SORT_MAX];
    __shared__ double Dsuf[EA_SORT_MAX + 1];
    __shared__ double scan[1024];
    __shared__ int kf_sh, knz_sh;
    const int tid = threadIdx.x, nth = blockDim.x;
    int n_pad = 1;
    while (n_pad < r) n_pad <<= 1;
    for (int i = tid; i < n_pad; i += nth) {
        key[i] = i < r ? s_raw[i] : -1.0;
        idx[i] = i;
    }
    if (tid == 0) {
        kf_sh = resid ? r + 1 : r;
        knz_sh = 0;
    }
    __syncthreads();
    // bitonic sort, descending by key, ascending index on ties
    for (int size = 2; size <= n_pad; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < n_pad; i += nth) {
                int j = i ^ stride;
                if (j > i) {
                    bool desc = (i & size) == 0;
                    double ki = key[i], kj = key[j];
                    int ii = idx[i], ij = idx[j];
                    // "i before j" in descending order
                    bool i_first = (ki > kj) || (ki == kj && ii < ij);
                    if (desc != i_first) {
                        key[i] = kj;
                        key[j] = ki;
                        idx[i] = ij;
                        idx[j] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < r; i += nth) {
        perm[i] = idx[i];
        s_sorted[i] = key[i];
    }
    // suffix sums
    const int chunk = (r + nth - 1) / nth;
    const int b0 = tid * chunk, b1 = min(b0 + chunk, r);
    double loc = 0.0;
    for (int i = b1 - 1; i >= b0; --i) loc += key[i] * key[i];
    scan[tid] = loc;
    __syncthreads();
    // inclusive reverse scan: scan[t] = sum_{u >= t} loc_u  (Hillis-Steele)
    for (int o = 1; o < nth; o <<= 1) {
        double v = (tid + o < nth) ? scan[tid + o] : 0.0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    double acc = (tid + 1 < nth) ? scan[tid + 1] : 0.0;  // sum over later chunks
    for (int i = b1 - 1; i >= b0; --i) {
        acc += key[i] * key[i];
        Dsuf[i] = acc;
    }
    if (tid == 0) Dsuf[r] = 0.0;
    __syncthreads();
    if (resid) {  // the weight outside a partial factorisation's subspace
        const double R = *resid;
        for (int i = tid; i <= r; i += nth) Dsuf[i] += R;
        __syncthreads();
    }
    const double T = Dsuf[0];
    const double s0 = r > 0 ? key[0] : 0.0;
    const double thr = (1.0 - f_t) * T;
    int kmin = resid ? r + 1 : r;
    int cnt = 0;
    for (int k = tid + 1; k <= r; k += nth)
        if (Dsuf[k] <= thr && k < kmin) kmin = k;
    for (int i = tid; i < r; i += nth)
        if (key[i] > tau * s0) ++cnt;
    atomicMin(&kf_sh, kmin);
    atomicAdd(&knz_sh, cnt);
    __syncthreads();
    if (tid == 0) {
        int k_f = kf_sh;
        int k_nz = knz_sh > 1 ? knz_sh : 1;
        if (k_nz > r) k_nz = r;
        int k, capped = 0;
        if (mode == 1) {
            k = k_nz;
        } else {
            k = k_f < k_nz ? k_f : k_nz;
            if (chi_max > 0 && chi_max < k) {
                k = chi_max;
                capped = 1;
            }
            if (forced_k > 0) {
                k = forced_k < r ? forced_k : r;
                capped = 0;
            }
        }
        double disc = Dsuf[k];
        double kept2 = T - disc;
        rec->k = k;
        rec->k_f = k_f;
        rec->k_nz = k_nz;
        rec->capped = capped;
        rec->sweeps = sweeps_dev ? sweeps_dev[0] : 0;
        rec->converged = sweeps_dev ? sweeps_dev[1] : 1;
        rec->r = r;
        rec->total = T;
        rec->disc = disc;
        rec->f = T > 0 ? 1.0 - disc / T : 1.0;
        rec->lnf = T > 0 ? log1p(-disc / T) : 0.0;
        rec->kept2 = kept2;
        rec->scale = (mode == 1 || kept2 <= 0.0) ? 1.0 : 1.0 / sqrt(kept2);
        rec->s0 = s0;
    }
}

void launch_sort_trunc(const double *s_raw, int r, double f_t, int chi_max, double tau,
                       int mode, int forced_k, const int *sweeps_dev, int *perm,
                       double *s_sorted, ea_dev_rec *rec, hipStream_t s, const double *resid) {
    k_sort_trunc<<<1, 1024, 0, s>>>(s_raw, r, f_t, chi_max, tau, mode, forced_k, sweeps_dev,
                                    perm, s_sorted, rec, resid);
}

// ---------------------------------------------------------------------------
// Write-back gather (see launcher comment in ea_kernels.h).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T gather_alpha(const double *s_sorted, const ea_dev_rec *rec, int j,
                                          int es, int ec) {
    double a = 1.0;
    if (es == 1) a *= s_sorted[j];
    if (es == -1) a /= s_sorted[j];
    if (ec) a *= rec->scale;
    return (T)a;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(const cx<T> *__restrict__ src, int ld,
                                                     const int *__restrict__ perm,
                                                     const double *__restrict__ s_sorted,
                                                     const ea_dev_rec *__restrict__ rec,
                                                     int X, int conj_src, int es, int ec,
                                                     cx<T> *__restrict__ out) {
    const int j = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= X) return;
    const T a = gather_alpha<T>(s_sorted, rec, j, es, ec);
    cx<T> v = src[(size_t)perm[j] * ld + x];
    if (conj_src) v = conj(v);
    out[(size_t)j * X + x] = a * v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_t(const cx<T> *__restrict__ src, int ld,
                                                  const int *__restrict__ perm,
                                                  const double *__restrict__ s_sorted,
                                                  const ea_dev_rec *__restrict__ rec, int k,
                                                  int X, int conj_src, int es, int ec,
                                                  cx<T> *__restrict__ out) {
    __shared__ cx<T> tile[32][33];
    const int x0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int jj = ty; jj < 32; jj += 8) {
        int j = j0 + jj, x = x0 + tx;
        if (j < k && x < X) {
            const T a = gather_alpha<T>(s_sorted, rec, j, es, ec);
            cx<T> v = src[(size_t)perm[j] * ld + x];
            if (conj_src) v = conj(v);
            tile[jj][tx] = a * v;
        }
    }
    __syncthreads();
    for (int xx = ty; xx < 32; xx += 8) {
        int x = x0 + xx, j = j0 + tx;
        if (j < k && x < X) out[(size_t)x * k + j] = tile[tx][xx];
    }
}

template <typename T>
void launch_gather(const void *src, int ld, const int *perm, const double *s_sorted,
                   const ea_dev_rec *rec, int k, int X, int conj_src, int es, int ec,
                   int transposed, void *out, hipStream_t s) {
    if (k <= 0 || X <= 0) return;
    if (transposed) {
        dim3 grid((X + 31) / 32, (k + 31) / 32);
        k_gather_t<T><<<grid, 256, 0, s>>>((const cx<T> *)src, ld, perm, s_sorted, rec, k, X,
                                           conj_src, es, ec, (cx<T> *)out);
    } else {
        dim3 grid((X + 255) / 256, k);
        k_gather_rows<T><<<grid, 256, 0, s>>>((const cx<T> *)src, ld, perm, s_sorted, rec, X,
                                              conj_src, es, ec, (cx<T> *)out);
    }
}

template <typename T>
__global__ void k_to_c128(const cx<T> *__restrict__ in, double *__restrict__ out, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        out[2 * i] = (double)in[i].x;
        out[2 * i + 1] = (double)in[i].y;
    }
}
template <typename T>
void launch_to_c128(const void *in, double *out, size_t n, hipStream_t s) {
    k_to_c128<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const cx<T> *)in, out, n);
}
template <typename T>
__global__ void k_from_c128(const double *__restrict__ in, cx<T> *__restrict__ out, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = mk<T>((T)in[2 * i], (T)in[2 * i + 1]);
}
template <typename T>
void launch_from_c128(const double *in, void *out, size_t n, hipStream_t s) {
    k_from_c128<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, (cx<T> *)out, n);
}

__global__ void k_fill_int(int *p, int n, int v) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}
void launch_fill_int(int *p, int n, int v, hipStream_t s) {
    k_fill_int<<<(n + 255) / 256, 256, 0, s>>>(p, n, v);
}

#define INST(T)                                                                              \
    template void launch_theta<T>(const void *, const void *, const void *, void *, int, int, \
                                  int, int, int, hipStream_t);                                \
    template void launch_gemm<T>(const void *, const void *, void *, int, int, int, int, int, \
                                 int, hipStream_t);                                           \
    template void launch_apply1<T>(const void *, void *, const void *, int, int, int,         \
                                   hipStream_t);                                              \
    template void launch_eye<T>(void *, int, hipStream_t);                                    \
    template void launch_to_colmajor<T>(const void *, void *, int, int, int, hipStream_t);    \
    template void launch_colnorms<T>(const void *, int, int, double *, hipStream_t);          \
    template void launch_unit_right<T>(void *, int, void *, int, hipStream_t);                \
    template void launch_gather<T>(const void *, int, const int *, const double *,            \
                                   const ea_dev_rec *, int, int, int, int, int, int, void *,  \
                                   hipStream_t);                                              \
    template void launch_to_c128<T>(const void *, double *, size_t, hipStream_t);             \
    template void launch_from_c128<T>(const double *, void *, size_t, hipStream_t);
INST(float)
INST(double)

template <typename T>
__global__ void k_scale(cx<T> *x, size_t n, T re, T im) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = mk<T>(re, im) * x[i];
}
template <typename T>
void launch_scale(void *x, size_t n, double re, double im, hipStream_t s) {
    k_scale<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((cx<T> *)x, n, (T)re, (T)im);
}
template void launch_scale<float>(void *, size_t, double, double, hipStream_t);
template void launch_scale<double>(void *, size_t, double, double, hipStream_t);
