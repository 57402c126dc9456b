// Householder QR of the matrix handed to the SVD, used to precondition the
// one-sided Jacobi: with Theta = Q R, the Jacobi runs on X = R^H (n x n),
// whose columns are far closer to orthogonal, and the SVD of Theta follows
// as Theta = (Q V_x) S U_x^H.
//
//   k_qr_panel : one workgroup factors a panel of NBK columns (rows j0..m-1)
//                held in registers, column by column: Householder vector,
//                its application to the panel's later columns, and the
//                upper-triangular T of the compact WY form
//                H_1 ... H_nc = I - V T V^H (forward, columnwise)
//   k_qr_rh    : X = R^H from the factored matrix (lower triangular, n x n)
//   k_qr_finish: right vectors W_x / s and the scaled left factor V_x s
//   k_qr_fill  : C = [Y; 0] (m x n) before Q is applied
//
// The trailing updates A <- (I - V T^H V^H) A and the products with Q are
// plain GEMMs (the matrix-core GEMM) issued by the host.  All matrices are
// column-major.
#include "ea_dev.h"
#include "ea_kernels.h"

namespace {

constexpr int QR_NTH = 1024;
constexpr int QR_WAVES = QR_NTH / 64;

template <typename T>
__device__ __forceinline__ cx<T> shfl_xor_cx(cx<T> v, int mask) {
    return mk<T>(__shfl_xor(v.x, mask), __shfl_xor(v.y, mask));
}

// Sum over the 64 lanes of a wave of each of NV per-lane values (NV a power
// of two <= 64) by recursive halving: after the call lane l holds the total
// of value l / (64 / NV) in v[0].
template <typename T, int NV>
__device__ __forceinline__ void wave_reduce_scatter(cx<T> (&v)[NV], int lane) {
    constexpr int L = NV >= 64 ? 6 : NV >= 32 ? 5 : NV >= 16 ? 4 : NV >= 8 ? 3 : NV >= 4 ? 2 : NV >= 2 ? 1 : 0;
    static_assert((1 << L) == NV, "NV must be a power of two <= 64");
#pragma unroll
    for (int st = 0; st < L; ++st) {
        const int half = NV >> (st + 1), mask = 32 >> st;
        const bool upper = (lane & mask) != 0;
#pragma unroll
        for (int k = 0; k < NV / 2; ++k) {
            if (k >= half) continue;
            const cx<T> lo = v[k], hi = v[k + half];  // values, then a select of values
            const cx<T> keep = mk<T>(upper ? hi.x : lo.x, upper ? hi.y : lo.y);
            const cx<T> send = mk<T>(upper ? lo.x : hi.x, upper ? lo.y : hi.y);
            v[k] = keep + shfl_xor_cx(send, mask);
        }
    }
#pragma unroll
    for (int st = L; st < 6; ++st) v[0] = v[0] + shfl_xor_cx(v[0], 32 >> st);
}

template <typename T>
__device__ __forceinline__ cx<T> hh_entry(cx<T> x, int r, int rd, int m) {
    return r == rd ? mk<T>(T(1), T(0)) : (r > rd && r < m ? x : zero_cx<T>());
}

}  // namespace

template <typename T, int RPT, int NBK>
__global__ __launch_bounds__(QR_NTH) void k_qr_panel(cx<T> *__restrict__ A, int m, int n, int j0,
                                                     cx<T> *__restrict__ Vall,
                                                     cx<T> *__restrict__ Tout,
                                                     cx<T> *__restrict__ tau_out) {
    __shared__ double red_d[QR_WAVES];
    __shared__ cx<T> red[QR_WAVES][NBK];
    __shared__ cx<T> wsh[NBK];
    __shared__ cx<T> Tl[NBK][NBK + 1];
    __shared__ cx<T> alpha_sh, scale_sh, tau_sh;
    __shared__ T beta_sh;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int nc = min(NBK, n - j0);
    cx<T> a[RPT][NBK];
    int row[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        row[i] = j0 + tid + QR_NTH * i;
#pragma unroll
        for (int c = 0; c < NBK; ++c)
            a[i][c] = (row[i] < m && c < nc) ? A[(size_t)(j0 + c) * m + row[i]] : zero_cx<T>();
    }
    for (int e = tid; e < NBK * (NBK + 1); e += QR_NTH) Tl[e / (NBK + 1)][e % (NBK + 1)] = zero_cx<T>();
    // entry of the Householder vector of panel column c in slot i (1 on the
    // diagonal); a value, not a reference, so the panel stays in registers
#define EA_VVAL(i, c) hh_entry<T>(a[i][c], row[i], j0 + (c), m)
#pragma clang loop unroll(full)
    for (int j = 0; j < NBK; ++j) {
        if (j >= nc) continue;  // uniform; keeps every register index constant
        const int rd = j0 + j;
        // ---- Householder vector of column j (LAPACK larfg convention) ----
        double ps = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
            if (row[i] > rd && row[i] < m) ps += (double)a[i][j].x * a[i][j].x + (double)a[i][j].y * a[i][j].y;
#pragma unroll
        for (int mask = 32; mask >= 1; mask /= 2) ps += __shfl_xor(ps, mask);
        if (lane == 0) red_d[wave] = ps;
        if (tid == j) alpha_sh = a[0][j];  // the diagonal row j0 + j is thread j's first
        __syncthreads();
        if (tid == 0) {
            double xn2 = 0.0;
            for (int w = 0; w < QR_WAVES; ++w) xn2 += red_d[w];
            const double ar = alpha_sh.x, ai = alpha_sh.y;
            if (xn2 == 0.0 && ai == 0.0) {  // already reduced: H = I
                tau_sh = zero_cx<T>();
                beta_sh = (T)ar;
                scale_sh = zero_cx<T>();
            } else {
                const double beta = -copysign(sqrt(ar * ar + ai * ai + xn2), ar);
                tau_sh = mk<T>((T)((beta - ar) / beta), (T)(-ai / beta));
                beta_sh = (T)beta;
                const double dr = ar - beta, di = ai, dd = dr * dr + di * di;  // 1 / (alpha - beta)
                scale_sh = mk<T>((T)(dr / dd), (T)(-di / dd));
            }
        }
        __syncthreads();
        const cx<T> tau = tau_sh, scale = scale_sh;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
            if (row[i] > rd && row[i] < m) a[i][j] = a[i][j] * scale;
        if (tid == j) a[0][j] = mk<T>(beta_sh, T(0));
        // ---- dot products: c > j: v_j^H a_c (update); c < j: v_c^H v_j (T) ----
        cx<T> p[NBK];
#pragma unroll
        for (int c = 0; c < NBK; ++c) p[c] = zero_cx<T>();
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const cx<T> vj = EA_VVAL(i, j);
#pragma unroll
            for (int c = 0; c < NBK; ++c) {
                if (c > j) cmacc(p[c], vj, a[i][c]);  // p += conj(v_j) a_c
                else if (c < j) cmacc(p[c], EA_VVAL(i, c), vj);
            }
        }
        wave_reduce_scatter<T, NBK>(p, lane);
        if (lane % (64 / NBK) == 0) red[wave][lane / (64 / NBK)] = p[0];
        __syncthreads();
        if (tid < NBK) {
            cx<T> s = zero_cx<T>();
            for (int w = 0; w < QR_WAVES; ++w) s = s + red[w][tid];
            wsh[tid] = s;
        }
        __syncthreads();
        // ---- column j of T: T(c, j) = -tau T(c, c..j-1) u(c..j-1), T(j, j) = tau ----
        if (tid < j) {
            cx<T> s = zero_cx<T>();
            for (int k = tid; k < j; ++k) cmac(s, Tl[tid][k], wsh[k]);
            Tl[tid][j] = zero_cx<T>() - tau * s;
        }
        if (tid == j) Tl[j][j] = tau;
        // ---- apply H_j^H = I - conj(tau) v_j v_j^H to the later columns ----
        const cx<T> ct = conj(tau);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const cx<T> vj = EA_VVAL(i, j);
#pragma unroll
            for (int c = 0; c < NBK; ++c)
                if (c > j) a[i][c] = a[i][c] - ct * vj * wsh[c];
        }
        if (tid == 0) tau_out[rd] = tau;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (row[i] >= m) continue;
#pragma unroll
        for (int c = 0; c < NBK; ++c) {
            if (c >= nc) continue;
            A[(size_t)(j0 + c) * m + row[i]] = a[i][c];
            Vall[(size_t)(j0 + c) * m + row[i]] = EA_VVAL(i, c);
        }
    }
    for (int e = tid; e < NBK * NBK; e += QR_NTH) {
        const int r = e % NBK, c = e / NBK;  // column-major NBK x NBK
        Tout[e] = (r < nc && c < nc) ? Tl[r][c] : zero_cx<T>();
    }
#undef EA_VVAL
}

// X (n x n) = R^H, R the upper triangle of the factored A (m x n).
template <typename T>
__global__ void k_qr_rh(const cx<T> *__restrict__ A, int m, int n, cx<T> *__restrict__ X) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int c = (int)(e / n), r = (int)(e % n);  // X[r][c] = conj(R[c][r])
    X[e] = c <= r ? conj(A[(size_t)r * m + c]) : zero_cx<T>();
}

// Vr[:, j] = Wx[:, j] / s_j (0 if s_j = 0), Vx[:, j] *= s_j.
template <typename T>
__global__ void k_qr_finish(const cx<T> *__restrict__ Wx, cx<T> *__restrict__ Vx,
                            const double *__restrict__ s, int n, cx<T> *__restrict__ Vr) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)n * n) return;
    const int c = (int)(e / n);
    const double sc = s[c];
    const T inv = sc > 0.0 ? (T)(1.0 / sc) : T(0);
    const cx<T> w = Wx[e], v = Vx[e];
    Vr[e] = mk<T>(w.x * inv, w.y * inv);
    Vx[e] = mk<T>(v.x * (T)sc, v.y * (T)sc);
}

// C (m x n) = [Y; 0], Y n x n.
template <typename T>
__global__ void k_qr_fill(const cx<T> *__restrict__ Y, int m, int n, cx<T> *__restrict__ C) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)m * n) return;
    const int c = (int)(e / m), r = (int)(e % m);
    C[e] = r < n ? Y[(size_t)c * n + r] : zero_cx<T>();
}

// Panel width for a panel of mp rows: the panel (rows/1024 x NBK complex
// values per thread) and the NBK partial dot products stay within the 128
// VGPRs a thread of a 1024-thread workgroup has.
int qr_panel_width(int elem_bytes, int mp) {
    const bool f64 = elem_bytes == 16;
    if (mp <= 1024) return f64 ? 8 : 16;
    if (mp <= 2048) return f64 ? 4 : 8;
    return f64 ? 2 : 4;
}

template <typename T>
int launch_qr_panel(void *A, int m, int n, int j0, void *Vall, void *Tout, void *tau,
                    hipStream_t s) {
    const int mp = m - j0;
    if (mp < 1 || mp > 4 * QR_NTH || j0 >= n) return -1;
    const int nbk = qr_panel_width(2 * sizeof(T), mp);
    auto *a = (cx<T> *)A;
    auto *v = (cx<T> *)Vall;
    auto *t = (cx<T> *)Tout;
    auto *u = (cx<T> *)tau;
#define EA_QRP(R, B) k_qr_panel<T, R, B><<<1, QR_NTH, 0, s>>>(a, m, n, j0, v, t, u)
    if constexpr (sizeof(T) == 4) {
        if (mp <= 1024) EA_QRP(1, 16);
        else if (mp <= 2048) EA_QRP(2, 8);
        else EA_QRP(4, 4);
    } else {
        if (mp <= 1024) EA_QRP(1, 8);
        else if (mp <= 2048) EA_QRP(2, 4);
        else EA_QRP(4, 2);
    }
#undef EA_QRP
    return nbk;
}

template <typename T>
void launch_qr_rh(const void *A, int m, int n, void *X, hipStream_t s) {
    const size_t tot = (size_t)n * n;
    if (tot) k_qr_rh<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((const cx<T> *)A, m, n, (cx<T> *)X);
}
template <typename T>
void launch_qr_finish(const void *Wx, void *Vx, const double *sv, int n, void *Vr, hipStream_t s) {
    const size_t tot = (size_t)n * n;
    if (tot)
        k_qr_finish<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((const cx<T> *)Wx, (cx<T> *)Vx,
                                                                     sv, n, (cx<T> *)Vr);
}
template <typename T>
void launch_qr_fill(const void *Y, int m, int n, void *C, hipStream_t s) {
    const size_t tot = (size_t)m * n;
    if (tot) k_qr_fill<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((const cx<T> *)Y, m, n, (cx<T> *)C);
}

#define EA_QR_INST(T)                                                                            \
    template int launch_qr_panel<T>(void *, int, int, int, void *, void *, void *, hipStream_t); \
    template void launch_qr_rh<T>(const void *, int, int, void *, hipStream_t);                 \
    template void launch_qr_finish<T>(const void *, void *, const double *, int, void *,        \
                                      hipStream_t);                                             \
    template void launch_qr_fill<T>(const void *, int, int, void *, hipStream_t);
EA_QR_INST(float)
EA_QR_INST(double)

// T (ob x ob, column-major, upper triangular) of the compact WY form of ob
// reflectors from their Gram matrix G = V^H V (ob x ob, column-major) and
// tau: T(i, j) = -tau_j sum_{i<=k<j} T(i, k) G(k, j), T(j, j) = tau_j.
// One wave; thread i owns row i of T, so no barrier is needed.
template <typename T>
__global__ __launch_bounds__(64) void k_qr_larft(const cx<T> *__restrict__ G,
                                                 const cx<T> *__restrict__ tau, int ob,
                                                 cx<T> *__restrict__ Tout) {
    __shared__ cx<T> Tl[64][65];
    const int i = threadIdx.x;
    for (int j = 0; j < ob; ++j) {
        if (i < j) {
            cx<T> s = zero_cx<T>();
            for (int k = i; k < j; ++k) cmac(s, Tl[i][k], G[(size_t)j * ob + k]);
            Tl[i][j] = zero_cx<T>() - tau[j] * s;
        } else if (i == j) {
            Tl[i][j] = tau[j];
        }
    }
    if (i < ob)
        for (int j = 0; j < ob; ++j) Tout[(size_t)j * ob + i] = j >= i ? Tl[i][j] : zero_cx<T>();
}

template <typename T>
void launch_qr_larft(const void *G, const void *tau, int ob, void *Tout, hipStream_t s) {
    if (ob > 0 && ob <= 64)
        k_qr_larft<T><<<1, 64, 0, s>>>((const cx<T> *)G, (const cx<T> *)tau, ob, (cx<T> *)Tout);
}
template void launch_qr_larft<float>(const void *, const void *, int, void *, hipStream_t);
template void launch_qr_larft<double>(const void *, const void *, int, void *, hipStream_t);

// out (k x ncols, column-major, ld k) = the upper trapezoid of A's first k
// rows (A column-major, ld lda), conjugated if conj_r; zero below the diagonal.
template <typename T>
__global__ void k_qr_r_extract(const cx<T> *__restrict__ A, int lda, int k, int ncols, int conj_r,
                               cx<T> *__restrict__ out) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)k * ncols) return;
    const int j = (int)(e / k), i = (int)(e % k);
    cx<T> v = zero_cx<T>();
    if (i <= j) {
        v = A[(size_t)j * lda + i];
        if (conj_r) v = conj(v);
    }
    out[e] = v;
}

// C (m x k, column-major) = [I_k; 0].
template <typename T>
__global__ void k_qr_eye(int m, int k, cx<T> *__restrict__ C) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)m * k) return;
    const int j = (int)(e / m), i = (int)(e % m);
    C[e] = mk<T>(i == j ? T(1) : T(0), T(0));
}

template <typename T>
void launch_qr_r_extract(const void *A, int lda, int k, int ncols, int conj_r, void *out,
                         hipStream_t s) {
    const size_t tot = (size_t)k * ncols;
    if (tot)
        k_qr_r_extract<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((const cx<T> *)A, lda, k,
                                                                        ncols, conj_r, (cx<T> *)out);
}
template <typename T>
void launch_qr_eye(int m, int k, void *C, hipStream_t s) {
    const size_t tot = (size_t)m * k;
    if (tot) k_qr_eye<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(m, k, (cx<T> *)C);
}
template void launch_qr_r_extract<float>(const void *, int, int, int, int, void *, hipStream_t);
template void launch_qr_r_extract<double>(const void *, int, int, int, int, void *, hipStream_t);
template void launch_qr_eye<float>(int, int, void *, hipStream_t);
template void launch_qr_eye<double>(int, int, void *, hipStream_t);
