// Blocked Cholesky factorisation G = R^H R of a Hermitian positive definite
// complex FP64 matrix, and the inverse of its factor, for the Cholesky QR
// centre moves (Sec. III: A_c = Q R with Q the new, orthonormal site and R
// absorbed into the neighbour).  With X = Q R and G = X^H X, R is the
// Cholesky factor of G and Q = X R^{-1}; done twice (Cholesky QR2) the
// columns of Q are orthonormal to FP64 rounding while the condition number
// of X stays below about 1e7.  All matrices are row-major n x n with leading
// dimension n.
//
// The host walks the column blocks of width CHOL_NB: this file's kernel
// factors one diagonal block (R_jj and R_jj^{-1}); the panel
// R[j, j+] = R_jj^{-H} G[j, j+] and the trailing update
// G[j+, j+] -= R[j, j+]^H R[j, j+] are matrix-core GEMMs, as are the
// off-diagonal blocks of R^{-1}: Rinv[<j, j] = -Rinv[<j, <j] R[<j, j] Rinv_jj.
#include "ea_dev.h"
#include "ea_kernels.h"

namespace {

constexpr int NB = CHOL_NB;

// Largest diagonal entry of G (n entries, one workgroup) into *dmax.
__global__ __launch_bounds__(256) void k_chol_dmax(const cx<double> *__restrict__ G, int n,
                                                   double *__restrict__ dmax) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, G[(size_t)i * n + i].x);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *dmax = red[0];
}

// Factor the diagonal block at (j0, j0), size nb <= NB, of the (updated) G:
// R[j0.., j0..] <- R_jj (upper triangle; zeros below), Rinv[j0.., j0..] <-
// R_jj^{-1}.  A pivot at or below rel_min * max diag(G) (or not finite)
// marks a breakdown in *flag and is replaced by that bound, so that the
// factorisation still completes with finite values (the host then discards
// it).  One wave; the block lives in LDS and lane l works on column
// t = l % NB, the two lanes of a column splitting every sum by parity.  Row p
// of R is formed left-looking, R[p][t] = (G[p][t] - sum_{k<p} conj(R[k][p])
// R[k][t]) / R[p][p], so the inner loops only read LDS and their loads
// overlap.  The loops stay rolled so that the code fits the instruction
// cache (a fully unrolled, register-resident form ran six times slower).
__global__ __launch_bounds__(64) void k_chol_diag(const cx<double> *__restrict__ G,
                                                  cx<double> *__restrict__ R,
                                                  cx<double> *__restrict__ Rinv, int n, int j0,
                                                  int nb, const double *__restrict__ dmax,
                                                  double rel_min, int *__restrict__ flag) {
    static_assert(NB == 32, "two lanes per column of a 32-wide block");
    __shared__ cx<double> S[NB][NB + 1];   // rows < p: R; rows >= p: G
    __shared__ cx<double> Xi[NB][NB + 1];  // R_jj^{-1}, column c in Xi[.][c]
    __shared__ double piv;
    const int l = threadIdx.x, t = l & (NB - 1), h = l >> 5;
    for (int i = h; i < NB; i += 2)
        S[i][t] = (i < nb && t < nb) ? G[(size_t)(j0 + i) * n + j0 + t] : zero_cx<double>();
    __syncthreads();
    const double dmin = rel_min * *dmax;
    for (int p = 0; p < nb; ++p) {
        cx<double> dot = zero_cx<double>();
        if (t >= p && t < nb) {
#pragma unroll 4
            for (int k = h; k < p; k += 2) cmacc(dot, S[k][p], S[k][t]);
        }
        dot.x += __shfl_xor(dot.x, 32);
        dot.y += __shfl_xor(dot.y, 32);
        if (l == p) {
            double dp = S[p][p].x - dot.x;
            if (!(dp > dmin)) {  // also catches NaN
                *flag = 1;
                dp = dmin > 0.0 ? dmin : 1.0;
            }
            piv = sqrt(dp);
        }
        __syncthreads();
        const double rp = piv;
        if (h == 0 && t >= p && t < nb)
            S[p][t] = t == p ? mk<double>(rp, 0.0) : (1.0 / rp) * (S[p][t] - dot);
        __syncthreads();
    }
    // R_jj^{-1}, column c = t: back substitution of R x = e_c, from the last
    // row up; the sum over j > i is split by parity between the two lanes
    for (int i = nb - 1; i >= 0; --i) {
        cx<double> acc = zero_cx<double>();
        if (t < nb && i < t) {
#pragma unroll 4
            for (int j = i + 1 + h; j <= t; j += 2) cmac(acc, S[i][j], Xi[j][t]);
        }
        acc.x += __shfl_xor(acc.x, 32);
        acc.y += __shfl_xor(acc.y, 32);
        if (h == 0 && t < nb) {
            const cx<double> rhs = mk<double>((i == t ? 1.0 : 0.0) - acc.x, -acc.y);
            Xi[i][t] = i <= t ? (1.0 / S[i][i].x) * rhs : zero_cx<double>();
        }
        __syncthreads();
    }
    for (int i = h; i < nb; i += 2) {
        if (t < nb) {
            const size_t o = (size_t)(j0 + i) * n + j0 + t;
            R[o] = i <= t ? S[i][t] : zero_cx<double>();
            Rinv[o] = Xi[i][t];
        }
    }
}

// Zero the strictly lower triangle of an n x n matrix.
__global__ void k_lower_zero(cx<double> *__restrict__ A, int n) {
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int r = (int)(idx / n), c = (int)(idx % n);
    if (r > c) A[idx] = zero_cx<double>();
}

// Partial sums of |G - I|^2 over rows: block b takes rows 4b .. 4b+3.
__global__ __launch_bounds__(256) void k_offident_part(const cx<double> *__restrict__ G, int n,
                                                       double *__restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int r = 4 * blockIdx.x; r < min(n, 4 * (int)blockIdx.x + 4); ++r)
        for (int c = threadIdx.x; c < n; c += 256) {
            cx<double> v = G[(size_t)r * n + c];
            if (r == c) v.x -= 1.0;
            acc += v.x * v.x + v.y * v.y;
        }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int np,
                                                   double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

// ||G - I||_F^2 of an n x n matrix into *out; part is scratch of (n + 3) / 4
// doubles.
void launch_offident_fro2(const void *G, int n, double *part, double *out, hipStream_t s) {
    const int nb = (n + 3) / 4;
    k_offident_part<<<nb, 256, 0, s>>>((const cx<double> *)G, n, part);
    k_sum_parts<<<1, 256, 0, s>>>(part, nb, out);
}

// Cholesky G = R^H R (G overwritten by its trailing updates) and Rinv = R^{-1}.
// T1 is scratch of n x n.  *flag is set (not cleared) on a breakdown.
// Rinv: the diagonal blocks come from the block factorisations; the rest by
// doubling, inv([[A, B], [0, C]]) = [[A^-1, -A^-1 B C^-1], [0, C^-1]], all
// block pairs of one size in one batched GEMM launch (two per size).
void launch_cholesky_inv(void *G, void *R, void *Rinv, void *T1, int n,
                         double *dmax, double rel_min, int *flag, hipStream_t s) {
    cx<double> *g = (cx<double> *)G, *r = (cx<double> *)R, *ri = (cx<double> *)Rinv,
               *t1 = (cx<double> *)T1;
    const size_t nn = (size_t)n * n;
    k_lower_zero<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(r, n);
    k_lower_zero<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(ri, n);
    k_chol_dmax<<<1, 256, 0, s>>>(g, n, dmax);
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int nb = n - j0 < NB ? n - j0 : NB, j1 = j0 + nb, rest = n - j1;
        k_chol_diag<<<1, 64, 0, s>>>(g, r, ri, n, j0, nb, dmax, rel_min, flag);
        if (rest > 0) {
            // panel R[j, j+] = Rinv_jj^H G[j, j+]
            launch_zgemm<double>(1, 0, nb, rest, nb, 1.0, 0.0, ri + (size_t)j0 * n + j0, n,
                                 g + (size_t)j0 * n + j1, n, 0.0, 0.0, r + (size_t)j0 * n + j1,
                                 n, s);
            // trailing G[j+, j+] -= R[j, j+]^H R[j, j+]
            launch_zgemm<double>(1, 0, rest, rest, nb, -1.0, 0.0, r + (size_t)j0 * n + j1, n,
                                 r + (size_t)j0 * n + j1, n, 1.0, 0.0, g + (size_t)j1 * n + j1,
                                 n, s);
        }
    }
    for (int b = NB; b < n; b *= 2) {
        const int np = n / (2 * b);
        const size_t step = 2 * (size_t)b * (n + 1);  // from one pair's corner to the next
        if (np > 0) {
            // T_q = R[r0 : r0+b, r0+b : r0+2b] Rinv[r0+b : r0+2b, r0+b : r0+2b]
            launch_zgemm_batched<double>(0, 0, b, b, b, 1.0, 0.0, r + b, n, step,
                                         ri + (size_t)b * (n + 1), n, step, 0.0, 0.0, t1, b,
                                         (size_t)b * b, np, s);
            // Rinv[r0 : r0+b, r0+b : r0+2b] = -Rinv[r0 : r0+b, r0 : r0+b] T_q
            launch_zgemm_batched<double>(0, 0, b, b, b, -1.0, 0.0, ri, n, step, t1, b,
                                         (size_t)b * b, 0.0, 0.0, ri + b, n, step, np, s);
        }
        const int r0 = 2 * b * np, b2 = n - r0 - b;
        if (b2 > 0) {  // a last pair whose second block is shorter
            const size_t c0 = (size_t)r0 * (n + 1);
            launch_zgemm<double>(0, 0, b, b2, b2, 1.0, 0.0, r + c0 + b, n,
                                 ri + c0 + (size_t)b * (n + 1), n, 0.0, 0.0, t1, b2, s);
            launch_zgemm<double>(0, 0, b, b2, b, -1.0, 0.0, ri + c0, n, t1, b2, 0.0, 0.0,
                                 ri + c0 + b, n, s);
        }
    }
}
