// Kernels of the reverse pass (vector-Jacobian products) through the
// two-site update: the small elementwise / reduction pieces of the
// truncated-SVD adjoint (see the derivation in the adjoint host source); its
// products use the matrix-core complex GEMM.
#include "ea_dev.h"
#include "ea_kernels.h"

#include <math.h>

// C (M x N) = alpha op(A) op(B) + beta C, row-major (ops 0 and 1 of the
// matrix-core kernel).
template <typename T>
void launch_gemm_ex(int opA, int opB, int M, int N, int K, double ar, double ai, const void *A,
                    int lda, const void *B, int ldb, double br, double bi, void *C, int ldc,
                    hipStream_t s) {
    launch_zgemm<T>(opA, opB, M, N, K, ar, ai, A, lda, B, ldb, br, bi, C, ldc, s);
}

// Y = a X + b Y (n elements)
template <typename T>
__global__ void k_axpby(size_t n, cx<T> a, const cx<T> *__restrict__ X, cx<T> b,
                        cx<T> *__restrict__ Y) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) Y[i] = a * X[i] + b * Y[i];
}
template <typename T>
void launch_axpby(size_t n, double ar, double ai, const void *X, double br, double bi, void *Y,
                  hipStream_t s) {
    if (!n) return;
    k_axpby<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, mk<T>((T)ar, (T)ai),
                                                           (const cx<T> *)X, mk<T>((T)br, (T)bi),
                                                           (cx<T> *)Y);
}

// Y (cols x rows) with Y[j][i] = conj(X[i][j]) * f_i, f_i = scale[i]^power
// (power 0: 1), for i < rows_used; rows beyond rows_used give zero columns.
// X is rows x cols (ldx); Y is cols x ldy.
template <typename T>
__global__ void k_conjT_scaled(int rows, int rows_used, int cols, const cx<T> *__restrict__ X,
                               int ldx, const double *__restrict__ scale, int power,
                               double cst, cx<T> *__restrict__ Y, int ldy) {
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)rows * cols) return;
    const int j = (int)(idx / rows), i = (int)(idx % rows);
    cx<T> v = zero_cx<T>();
    if (i < rows_used) {
        double f = cst;
        if (power == 1) f *= scale[i];
        if (power == -1) f /= scale[i];
        v = (T)f * conj(X[(size_t)i * ldx + j]);
    }
    Y[(size_t)j * ldy + i] = v;
}
template <typename T>
void launch_conjT_scaled(int rows, int rows_used, int cols, const void *X, int ldx,
                         const double *scale, int power, double cst, void *Y, int ldy,
                         hipStream_t s) {
    const size_t n = (size_t)rows * cols;
    if (!n) return;
    k_conjT_scaled<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        rows, rows_used, cols, (const cx<T> *)X, ldx, scale, power, cst, (cx<T> *)Y, ldy);
}

// X[i][j] *= scale[j]^power for a row-major rows x cols matrix (ld).
template <typename T>
__global__ void k_scale_cols(int rows, int cols, cx<T> *__restrict__ X, int ld,
                             const double *__restrict__ scale, int power) {
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)rows * cols) return;
    const int i = (int)(idx / cols), j = (int)(idx % cols);
    const double f = power == 1 ? scale[j] : 1.0 / scale[j];
    cx<T> *p = X + (size_t)i * ld + j;
    *p = (T)f * (*p);
}
template <typename T>
void launch_scale_cols(int rows, int cols, void *X, int ld, const double *scale, int power,
                       hipStream_t s) {
    const size_t n = (size_t)rows * cols;
    if (!n) return;
    k_scale_cols<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, cols, (cx<T> *)X, ld, scale,
                                                               power);
}

// out[j] = Re sum_c X[j][c] Y[c][j]  (j < k; X is k x n (ldx), Y is n x ldy)
template <typename T>
__global__ __launch_bounds__(256) void k_rowdot_re(int n, const cx<T> *__restrict__ X, int ldx,
                                                   const cx<T> *__restrict__ Y, int ldy,
                                                   double *__restrict__ out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) {
        const cx<T> a = X[(size_t)j * ldx + c], b = Y[(size_t)c * ldy + j];
        acc += (double)a.x * (double)b.x - (double)a.y * (double)b.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}
template <typename T>
void launch_rowdot_re(int k, int n, const void *X, int ldx, const void *Y, int ldy, double *out,
                      hipStream_t s) {
    if (k <= 0) return;
    k_rowdot_re<T><<<k, 256, 0, s>>>(n, (const cx<T> *)X, ldx, (const cx<T> *)Y, ldy, out);
}

// out[j] = Re sum_i conj(A[i][j]) B[i][j]  (row-major rows x cols, ld)
template <typename T>
__global__ __launch_bounds__(256) void k_coldot_re(int rows, const cx<T> *__restrict__ A,
                                                   const cx<T> *__restrict__ B, int ld,
                                                   double *__restrict__ out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < rows; i += 256) {
        const cx<T> a = A[(size_t)i * ld + j], b = B[(size_t)i * ld + j];
        acc += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}
template <typename T>
void launch_coldot_re(int rows, int cols, const void *A, const void *B, int ld, double *out,
                      hipStream_t s) {
    if (cols <= 0) return;
    k_coldot_re<T><<<cols, 256, 0, s>>>(rows, (const cx<T> *)A, (const cx<T> *)B, ld, out);
}

// sbar_i = stbar_i / sig - s_i (sum_{j<k} stbar_j s_j) / sig^3 for i < k,
// 0 for k <= i < r  (adjoint of the renormalisation s~ = s_k / ||s_k||).
__global__ __launch_bounds__(256) void k_sbar_renorm(int k, int r, const double *__restrict__ stbar,
                                                     const double *__restrict__ s, double sig,
                                                     double *__restrict__ sbar) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int j = threadIdx.x; j < k; j += 256) acc += stbar[j] * s[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double dot = red[0];
    for (int i = threadIdx.x; i < r; i += 256)
        sbar[i] = i < k ? stbar[i] / sig - s[i] * dot / (sig * sig * sig) : 0.0;
}
void launch_sbar_renorm(int k, int r, const double *stbar, const double *s, double sig,
                        double *sbar, hipStream_t st) {
    k_sbar_renorm<<<1, 256, 0, st>>>(k, r, stbar, s, sig, sbar);
}

// P (r x r) of the SVD adjoint:
//   P_ij = F_ij (s_j (J - J^H)_ij + s_i (K - K^H)_ij),
//   F_ij = D / (D^2 + eta), D = s_j^2 - s_i^2 (exact 1/D when eta = 0),
//   P_ii = sbar_i + i (Im J_ii - Im K_ii) / (2 s_i).
template <typename T>
__global__ void k_svdvjp_P(int r, const cx<T> *__restrict__ J, const cx<T> *__restrict__ K,
                           const double *__restrict__ s, const double *__restrict__ sbar,
                           double eta, cx<T> *__restrict__ P) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= r * r) return;
    const int i = idx / r, j = idx % r;
    if (i == j) {
        const double v = ((double)J[idx].y - (double)K[idx].y) / (2.0 * s[i]);
        P[idx] = mk<T>((T)sbar[i], (T)v);
        return;
    }
    const double D = s[j] * s[j] - s[i] * s[i];
    const double F = eta > 0.0 ? D / (D * D + eta) : (D != 0.0 ? 1.0 / D : 0.0);
    const cx<T> jij = J[idx], jji = J[j * r + i], kij = K[idx], kji = K[j * r + i];
    const double jx = (double)jij.x - (double)jji.x, jy = (double)jij.y + (double)jji.y;
    const double kx = (double)kij.x - (double)kji.x, ky = (double)kij.y + (double)kji.y;
    P[idx] = mk<T>((T)(F * (s[j] * jx + s[i] * kx)), (T)(F * (s[j] * jy + s[i] * ky)));
}
template <typename T>
void launch_svdvjp_P(int r, const void *J, const void *K, const double *s, const double *sbar,
                     double eta, void *P, hipStream_t st) {
    const int n = r * r;
    k_svdvjp_P<T><<<(n + 255) / 256, 256, 0, st>>>(r, (const cx<T> *)J, (const cx<T> *)K, s, sbar,
                                                   eta, (cx<T> *)P);
}

// partial[blk][4] = sum over (l, r) of Abar[l,s,r] conj(A[l,t,r]) for the 2x2 (s,t)
template <typename T>
__global__ __launch_bounds__(256) void k_gbar(const cx<T> *__restrict__ Ab,
                                              const cx<T> *__restrict__ A, int chiL, int chiR,
                                              double *__restrict__ partial) {
    __shared__ double red[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const size_t tot = (size_t)chiL * chiR;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (size_t)gridDim.x * 256) {
        const size_t l = e / chiR, r = e % chiR;
        cx<T> ab[2], a[2];
        for (int t = 0; t < 2; ++t) {
            ab[t] = Ab[(l * 2 + t) * chiR + r];
            a[t] = A[(l * 2 + t) * chiR + r];
        }
        for (int s = 0; s < 2; ++s)
            for (int t = 0; t < 2; ++t) {
                // ab[s] * conj(a[t])
                acc[2 * (2 * s + t)] += (double)ab[s].x * a[t].x + (double)ab[s].y * a[t].y;
                acc[2 * (2 * s + t) + 1] += (double)ab[s].y * a[t].x - (double)ab[s].x * a[t].y;
            }
    }
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 8) partial[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// grad[param] += Re sum_{st} conj(gbar[s,t]) dg[s,t]  (gbar summed over blocks)
__global__ void k_gbar_final(const double *__restrict__ partial, int nblk,
                             const double *__restrict__ dg, double *__restrict__ grad, int param) {
    if (threadIdx.x != 0) return;
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nblk; ++b)
        for (int q = 0; q < 8; ++q) g[q] += partial[b * 8 + q];
    double acc = 0.0;
    for (int e = 0; e < 4; ++e) acc += g[2 * e] * dg[2 * e] + g[2 * e + 1] * dg[2 * e + 1];
    grad[param] += acc;
}

template <typename T>
void launch_gbar_grad(const void *Ab, const void *A, int chiL, int chiR, double *partial,
                      const double *dg, double *grad, int param, hipStream_t s) {
    const size_t tot = (size_t)chiL * chiR;
    int nblk = (int)((tot + 255) / 256);
    if (nblk > 256) nblk = 256;
    if (nblk < 1) nblk = 1;
    k_gbar<T><<<nblk, 256, 0, s>>>((const cx<T> *)Ab, (const cx<T> *)A, chiL, chiR, partial);
    k_gbar_final<<<1, 64, 0, s>>>(partial, nblk, dg, grad, param);
}

// From the Gram matrix G = X^H X = I + E of a nearly orthonormal factor (FP64):
// Y = I - E/2 (the Loewdin correction X <- X Y) and R = I + E/2 (absorbed by
// the neighbour, so that X Y R = X + O(E^2)), both stored in T.
// One workgroup per row i of G = I + E: writes row i of Y = I - E/2 and
// R = I + E/2 and raises *rowsq_max to sum_j |E_ij|^2 if larger (the bit
// pattern of a non-negative double orders like the unsigned integer).
template <typename T>
__global__ __launch_bounds__(256) void k_reorth_factors(int k, const cx<double> *__restrict__ G,
                                                        cx<T> *__restrict__ Y,
                                                        cx<T> *__restrict__ R,
                                                        unsigned long long *rowsq_max) {
    __shared__ double part[4];
    const int i = blockIdx.x;
    const size_t row = (size_t)i * k;
    double sq = 0.0;
    for (int j = threadIdx.x; j < k; j += 256) {
        const double ex = G[row + j].x - (i == j ? 1.0 : 0.0), ey = G[row + j].y;
        sq += ex * ex + ey * ey;
        Y[row + j] = mk<T>((T)((i == j ? 1.0 : 0.0) - 0.5 * ex), (T)(-0.5 * ey));
        R[row + j] = mk<T>((T)((i == j ? 1.0 : 0.0) + 0.5 * ex), (T)(0.5 * ey));
    }
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = part[0] + part[1] + part[2] + part[3];
        atomicMax(rowsq_max, (unsigned long long)__double_as_longlong(t));
    }
}
template <typename T>
void launch_reorth_factors(int k, const void *G, void *Y, void *R, void *rowsq_max,
                           hipStream_t s) {
    k_reorth_factors<T><<<k, 256, 0, s>>>(k, (const cx<double> *)G, (cx<T> *)Y, (cx<T> *)R,
                                          (unsigned long long *)rowsq_max);
}
// Absorb correction C = I + E^2/4 = (G^2 - 2 G + 5 I) / 4 from G = I + E and
// G2 = G G (both FP64): after R = I + E/2 and Y = I - E/2, applying C as
// well gives Y R C = I - E^4/16 in place of Y R = I - E^2/4.
template <typename T>
__global__ void k_reorth_corr(int k, const cx<double> *__restrict__ G2,
                              const cx<double> *__restrict__ G, cx<T> *__restrict__ C) {
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)k * k) return;
    const bool diag = idx / k == idx % k;
    C[idx] = mk<T>((T)(0.25 * (G2[idx].x - 2.0 * G[idx].x + (diag ? 5.0 : 0.0))),
                   (T)(0.25 * (G2[idx].y - 2.0 * G[idx].y)));
}
template <typename T>
void launch_reorth_corr(int k, const void *G2, const void *G, void *C, hipStream_t s) {
    const size_t n = (size_t)k * k;
    k_reorth_corr<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        k, (const cx<double> *)G2, (const cx<double> *)G, (cx<T> *)C);
}
template void launch_reorth_corr<float>(int, const void *, const void *, void *, hipStream_t);
template void launch_reorth_corr<double>(int, const void *, const void *, void *, hipStream_t);
template void launch_reorth_factors<float>(int, const void *, void *, void *, void *,
                                           hipStream_t);
template void launch_reorth_factors<double>(int, const void *, void *, void *, void *,
                                            hipStream_t);

#define INST(T)                                                                                  \
    template void launch_gemm_ex<T>(int, int, int, int, int, double, double, const void *, int,  \
                                    const void *, int, double, double, void *, int, hipStream_t); \
    template void launch_axpby<T>(size_t, double, double, const void *, double, double, void *,  \
                                  hipStream_t);                                                  \
    template void launch_conjT_scaled<T>(int, int, int, const void *, int, const double *, int,  \
                                         double, void *, int, hipStream_t);                      \
    template void launch_scale_cols<T>(int, int, void *, int, const double *, int, hipStream_t); \
    template void launch_rowdot_re<T>(int, int, const void *, int, const void *, int, double *,  \
                                      hipStream_t);                                              \
    template void launch_coldot_re<T>(int, int, const void *, const void *, int, double *,       \
                                      hipStream_t);                                              \
    template void launch_svdvjp_P<T>(int, const void *, const void *, const double *,            \
                                     const double *, double, void *, hipStream_t);               \
    template void launch_gbar_grad<T>(const void *, const void *, int, int, double *,            \
                                      const double *, double *, int, hipStream_t);
INST(float)
INST(double)
