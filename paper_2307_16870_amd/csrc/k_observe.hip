// Observables: overlaps for <O> at the orthogonality centre (Sec. III,
// Eq. 6), transfer vectors for Tr(rho O) of a matrix product operator, and
// the reshuffle of vec(rho) into a dense density matrix (Eq. 3).
#include "ea_dev.h"
#include "ea_kernels.h"

// partial[3*blk + {0,1,2}] = (Re, Im) of sum conj(a) b, and sum |a|^2.
template <typename T>
__global__ __launch_bounds__(256) void k_cdot(const cx<T> *__restrict__ a,
                                              const cx<T> *__restrict__ b, size_t len,
                                              double *__restrict__ partial) {
    __shared__ double r0[256], r1[256], r2[256];
    double sx = 0, sy = 0, sn = 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (size_t)gridDim.x * 256) {
        cx<T> u = a[i], v = b[i];
        double ux = u.x, uy = u.y, vx = v.x, vy = v.y;
        sx += ux * vx + uy * vy;
        sy += ux * vy - uy * vx;
        sn += ux * ux + uy * uy;
    }
    r0[threadIdx.x] = sx;
    r1[threadIdx.x] = sy;
    r2[threadIdx.x] = sn;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
            r2[threadIdx.x] += r2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = r0[0];
        partial[3 * blockIdx.x + 1] = r1[0];
        partial[3 * blockIdx.x + 2] = r2[0];
    }
}

template <typename T>
int launch_cdot(const void *a, const void *b, size_t len, double *partial, int max_blocks,
                hipStream_t s) {
    size_t want = (len + 255) / 256;
    int nblk = (int)(want < (size_t)max_blocks ? want : (size_t)max_blocks);
    if (nblk < 1) nblk = 1;
    k_cdot<T><<<nblk, 256, 0, s>>>((const cx<T> *)a, (const cx<T> *)b, len, partial);
    return nblk;
}

__global__ void k_cdot_final(const double *partial, int nblk, double *out) {
    if (threadIdx.x != 0) return;
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < nblk; ++i) {
        a += partial[3 * i];
        b += partial[3 * i + 1];
        c += partial[3 * i + 2];
    }
    out[0] = a;
    out[1] = b;
    out[2] = c;
}
void launch_cdot_final(const double *partial, int nblk, double *out, hipStream_t s) {
    k_cdot_final<<<1, 64, 0, s>>>(partial, nblk, out);
}

// out[r] = sum_{l,p} env[l] wgt[p] A[l,p,r]; one thread per r.
template <typename T>
__global__ __launch_bounds__(256) void k_env_left(const cx<T> *__restrict__ env,
                                                  const cx<T> *__restrict__ A,
                                                  const cx<T> *__restrict__ wgt,
                                                  cx<T> *__restrict__ out, int chiL, int d,
                                                  int chiR) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= chiR) return;
    cx<T> acc = zero_cx<T>();
    for (int l = 0; l < chiL; ++l) {
        cx<T> part = zero_cx<T>();
        for (int p = 0; p < d; ++p) cmac(part, wgt[p], A[((size_t)l * d + p) * chiR + r]);
        cmac(acc, env[l], part);
    }
    out[r] = acc;
}

// out[l] = sum_{p,r} A[l,p,r] wgt[p] env[r]; one workgroup per l.
template <typename T>
__global__ __launch_bounds__(256) void k_env_right(const cx<T> *__restrict__ A,
                                                   const cx<T> *__restrict__ wgt,
                                                   const cx<T> *__restrict__ env,
                                                   cx<T> *__restrict__ out, int d, int chiR) {
    __shared__ T rx[256], ry[256];
    const int l = blockIdx.x;
    const cx<T> *row = A + (size_t)l * d * chiR;
    cx<T> acc = zero_cx<T>();
    for (int i = threadIdx.x; i < d * chiR; i += 256) {
        const int p = i / chiR, r = i % chiR;
        cx<T> t = wgt[p] * row[i];
        cmac(acc, t, env[r]);
    }
    rx[threadIdx.x] = acc.x;
    ry[threadIdx.x] = acc.y;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            rx[threadIdx.x] += rx[threadIdx.x + o];
            ry[threadIdx.x] += ry[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[l] = mk<T>(rx[0], ry[0]);
}

// tmp[p, m] = sum_l env[l] A[l,p,m]
template <typename T>
__global__ __launch_bounds__(256) void k_env_raw(const cx<T> *__restrict__ env,
                                                 const cx<T> *__restrict__ A,
                                                 cx<T> *__restrict__ tmp, int chiL, int d,
                                                 int chiM) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= d * chiM) return;
    cx<T> acc = zero_cx<T>();
    for (int l = 0; l < chiL; ++l) cmac(acc, env[l], A[(size_t)l * d * chiM + i]);
    tmp[i] = acc;
}

// out[r] = sum_{p,m,q} tmp[p,m] W2[p,q] B[m,q,r]
template <typename T>
__global__ __launch_bounds__(256) void k_env_w2(const cx<T> *__restrict__ tmp,
                                                const cx<T> *__restrict__ W2,
                                                const cx<T> *__restrict__ B,
                                                cx<T> *__restrict__ out, int d, int chiM,
                                                int chiR) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= chiR) return;
    cx<T> acc = zero_cx<T>();
    for (int m = 0; m < chiM; ++m) {
        for (int q = 0; q < d; ++q) {
            cx<T> w = zero_cx<T>();
            for (int p = 0; p < d; ++p) cmac(w, tmp[(size_t)p * chiM + m], W2[p * d + q]);
            cmac(acc, w, B[((size_t)m * d + q) * chiR + r]);
        }
    }
    out[r] = acc;
}

template <typename T>
void launch_env_left(const void *env, const void *A, const void *wgt, void *out, int chiL,
                     int d, int chiR, hipStream_t s) {
    k_env_left<T><<<(chiR + 255) / 256, 256, 0, s>>>((const cx<T> *)env, (const cx<T> *)A,
                                                     (const cx<T> *)wgt, (cx<T> *)out, chiL, d,
                                                     chiR);
}
template <typename T>
void launch_env_right(const void *A, const void *wgt, const void *env, void *out, int chiL,
                      int d, int chiR, hipStream_t s) {
    k_env_right<T><<<chiL, 256, 0, s>>>((const cx<T> *)A, (const cx<T> *)wgt,
                                        (const cx<T> *)env, (cx<T> *)out, d, chiR);
}
template <typename T>
void launch_env_left2(const void *env, const void *A, const void *B, const void *W2,
                      void *tmp, void *out, int chiL, int d, int chiM, int chiR,
                      hipStream_t s) {
    k_env_raw<T><<<(d * chiM + 255) / 256, 256, 0, s>>>((const cx<T> *)env, (const cx<T> *)A,
                                                        (cx<T> *)tmp, chiL, d, chiM);
    k_env_w2<T><<<(chiR + 255) / 256, 256, 0, s>>>((const cx<T> *)tmp, (const cx<T> *)W2,
                                                   (const cx<T> *)B, (cx<T> *)out, d, chiM,
                                                   chiR);
}

// rho[row, col] = vec[interleave(row, col)]: site i contributes p_i = 2 s_i + s_i'
// with s_i, s_i' the i-th most significant bits of row and col.
template <typename T>
__global__ void k_vec_to_rho(const cx<T> *__restrict__ vec, cx<T> *__restrict__ rho, int n) {
    const size_t dim = (size_t)1 << n;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= dim * dim) return;
    const size_t row = idx / dim, col = idx % dim;
    size_t v = 0;
    for (int i = 0; i < n; ++i) {
        const size_t sb = (row >> (n - 1 - i)) & 1, cb = (col >> (n - 1 - i)) & 1;
        v = (v << 2) | (sb << 1) | cb;
    }
    rho[idx] = vec[v];
}
template <typename T>
void launch_vec_to_rho(const void *vec, void *rho, int n, hipStream_t s) {
    const size_t tot = ((size_t)1 << n) * ((size_t)1 << n);
    k_vec_to_rho<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>((const cx<T> *)vec,
                                                                  (cx<T> *)rho, n);
}

#define INST(T)                                                                               \
    template int launch_cdot<T>(const void *, const void *, size_t, double *, int, hipStream_t); \
    template void launch_env_left<T>(const void *, const void *, const void *, void *, int, int, \
                                     int, hipStream_t);                                       \
    template void launch_env_right<T>(const void *, const void *, const void *, void *, int,  \
                                      int, int, hipStream_t);                                 \
    template void launch_env_left2<T>(const void *, const void *, const void *, const void *, \
                                      void *, void *, int, int, int, int, hipStream_t);       \
    template void launch_vec_to_rho<T>(const void *, void *, int, hipStream_t);
INST(float)
INST(double)
