// Complex GEMM on the matrix cores, for the dense products around the
// factorisations: the absorb of a centre move's non-orthogonal factor into
// the neighbouring site (Sec. III), the FP64 re-orthogonalisation products,
// the Householder and Cholesky QR pieces and the products of the reverse
// pass.
//
//   C (M x N) = alpha op(A) op(B) + beta C,  row-major, leading dimensions
//   lda / ldb / ldc; op 0: the matrix as stored (A is M x K), 1: conjugate
//   transpose (A stored K x M), 2: transpose (A stored K x M), 3: conjugate
//   (A stored M x K).
//
// 64 x 64 output tile per workgroup of four waves (2 x 2 waves of 32 x 32,
// i.e. 2 x 2 MFMA tiles of 16 x 16 each), K in stages of 16.  Real and
// imaginary parts live in separate LDS planes; a complex product is four
// real MFMAs (Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br).  The next stage's
// operands are loaded into registers while the current stage's products run.
#include "ea_dev.h"
#include "ea_kernels.h"

namespace {

typedef float f4v_ __attribute__((ext_vector_type(4)));
typedef double d4v_ __attribute__((ext_vector_type(4)));

template <typename T>
struct ZM;
// 16x16x4 MFMA.  Inputs: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// Output: lane l, value v holds D[row(l, v)][l % 16].
template <>
struct ZM<float> {
    typedef f4v_ acc;
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct ZM<double> {
    typedef d4v_ acc;
    static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

constexpr int ZT = 64;   // output tile (rows and columns)
constexpr int ZK = 16;   // K per stage
constexpr int ZPER = ZT * ZK / 256;  // operand elements per thread and stage

// Stage of a 64-row x 16-k operand: element (r, k) is X[r ld + k] (cp = 0,
// contiguous in k) or X[k ld + r] (cp = 1, contiguous in r), conjugated if cj.
// The thread's elements are chosen so that consecutive threads read
// consecutive addresses.
template <typename T>
__device__ __forceinline__ void z_load(const cx<T> *__restrict__ X, bool cp, bool cj, int ld,
                                       int R, int K, int r0, int k0, cx<T> (&v)[ZPER],
                                       int (&rr)[ZPER], int (&kk)[ZPER], int tid) {
#pragma unroll
    for (int i = 0; i < ZPER; ++i) {
        const int e = tid + 256 * i;
        const int r = cp ? e % ZT : e / ZK, k = cp ? e / ZT : e % ZK;
        rr[i] = r;
        kk[i] = k;
        const int gr = r0 + r, gk = k0 + k;
        cx<T> x = zero_cx<T>();
        if (gr < R && gk < K) x = cp ? X[(size_t)gk * ld + gr] : X[(size_t)gr * ld + gk];
        if (cj) x.y = -x.y;
        v[i] = x;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zgemm(int opA, int opB, int M, int N, int K, cx<T> alpha,
                                               const cx<T> *__restrict__ A, int lda, size_t sA,
                                               const cx<T> *__restrict__ B, int ldb, size_t sB,
                                               cx<T> beta, cx<T> *__restrict__ C, int ldc,
                                               size_t sC) {
    using MF = ZM<T>;
    // batch entry blockIdx.z: operands offset by its strides
    A += sA * blockIdx.z;
    B += sB * blockIdx.z;
    C += sC * blockIdx.z;
    // operand planes [re/im][tile row or column][k]
    __shared__ T As[2][ZT][ZK + 1], Bs[2][ZT][ZK + 1];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * ZT, n0 = blockIdx.x * ZT;
    // op(A)[m][k]: A[m lda + k] (ops 0, 3) or A[k lda + m] (ops 1, 2); op(B)[k][n],
    // staged as its transpose: B[k ldb + n] (ops 0, 3) or B[n ldb + k] (ops 1, 2);
    // ops 1 and 3 conjugate
    const bool cpA = opA == 1 || opA == 2, cjA = opA == 1 || opA == 3;
    const bool cpB = opB == 0 || opB == 3, cjB = opB == 1 || opB == 3;
    typename MF::acc re[2][2], im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            re[a][b] = MF::zero();
            im[a][b] = MF::zero();
        }
    cx<T> va[ZPER], vb[ZPER];
    int ra[ZPER], ka[ZPER], rb[ZPER], kb[ZPER];
    z_load<T>(A, cpA, cjA, lda, M, K, m0, 0, va, ra, ka, tid);
    z_load<T>(B, cpB, cjB, ldb, N, K, n0, 0, vb, rb, kb, tid);
    const int li = lane % 16, lk = lane / 16;
    for (int k0 = 0; k0 < K; k0 += ZK) {
#pragma unroll
        for (int i = 0; i < ZPER; ++i) {
            As[0][ra[i]][ka[i]] = va[i].x;
            As[1][ra[i]][ka[i]] = va[i].y;
            Bs[0][rb[i]][kb[i]] = vb[i].x;
            Bs[1][rb[i]][kb[i]] = vb[i].y;
        }
        __syncthreads();
        if (k0 + ZK < K) {
            z_load<T>(A, cpA, cjA, lda, M, K, m0, k0 + ZK, va, ra, ka, tid);
            z_load<T>(B, cpB, cjB, ldb, N, K, n0, k0 + ZK, vb, rb, kb, tid);
        }
#pragma unroll
        for (int ks = 0; ks < ZK; ks += 4) {
            T ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int r = wm * 32 + a * 16 + li;
                ar[a] = As[0][r][ks + lk];
                ai[a] = As[1][r][ks + lk];
                nai[a] = -ai[a];
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int c = wn * 32 + b * 16 + li;
                br[b] = Bs[0][c][ks + lk];
                bi[b] = Bs[1][c][ks + lk];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    re[a][b] = MF::op(ar[a], br[b], re[a][b]);
                    re[a][b] = MF::op(nai[a], bi[b], re[a][b]);
                    im[a][b] = MF::op(ar[a], bi[b], im[a][b]);
                    im[a][b] = MF::op(ai[a], br[b], im[a][b]);
                }
        }
        __syncthreads();
    }
    const bool use_beta = beta.x != T(0) || beta.y != T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wm * 32 + a * 16 + MF::row(lane, v);
                const int gn = n0 + wn * 32 + b * 16 + li;
                if (gm < M && gn < N) {
                    cx<T> *c = C + (size_t)gm * ldc + gn;
                    cx<T> x = alpha * mk<T>(re[a][b][v], im[a][b][v]);
                    if (use_beta) x = x + beta * (*c);
                    *c = x;
                }
            }
}

}  // namespace

template <typename T>
void launch_zgemm_batched(int opA, int opB, int M, int N, int K, double ar, double ai,
                          const void *A, int lda, size_t sA, const void *B, int ldb, size_t sB,
                          double br, double bi, void *C, int ldc, size_t sC, int batch,
                          hipStream_t s) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    dim3 grid((N + ZT - 1) / ZT, (M + ZT - 1) / ZT, batch);
    k_zgemm<T><<<grid, 256, 0, s>>>(opA, opB, M, N, K, mk<T>((T)ar, (T)ai), (const cx<T> *)A, lda,
                                    sA, (const cx<T> *)B, ldb, sB, mk<T>((T)br, (T)bi),
                                    (cx<T> *)C, ldc, sC);
}

template <typename T>
void launch_zgemm(int opA, int opB, int M, int N, int K, double ar, double ai, const void *A,
                  int lda, const void *B, int ldb, double br, double bi, void *C, int ldc,
                  hipStream_t s) {
    launch_zgemm_batched<T>(opA, opB, M, N, K, ar, ai, A, lda, 0, B, ldb, 0, br, bi, C, ldc, 0, 1,
                            s);
}

template void launch_zgemm<float>(int, int, int, int, int, double, double, const void *, int,
                                  const void *, int, double, double, void *, int, hipStream_t);
template void launch_zgemm<double>(int, int, int, int, int, double, double, const void *, int,
                                   const void *, int, double, double, void *, int, hipStream_t);
template void launch_zgemm_batched<double>(int, int, int, int, int, double, double, const void *,
                                           int, size_t, const void *, int, size_t, double, double,
                                           void *, int, size_t, int, hipStream_t);
