// Two-site contraction (paper Sec. V, the contraction of two neighbouring
// site tensors followed by the gate) on the bf16 matrix cores, with each FP32
// operand split as x = x_hi + x_lo (x_hi = bf16(x), x_lo = bf16(x - x_hi)) and
// every real product taken as hi*hi + hi*lo + lo*hi with FP32 accumulation.
// The dropped lo*lo term and the rounding of x_lo leave a relative error of
// about 2^-16 per product, between bf16 (2^-8) and FP32 (2^-24).
//
// Output tile: 16 values of l by 16 values of r, i.e. a (16 D) x (16 D) tile
// of C[(l, t1), (t2, r)] = sum_m A[(l, t1), m] B[m, (t2, r)].  Complex
// products are split into real and imaginary parts:
//   Re C = Ar Br - Ai Bi,   Im C = Ar Bi + Ai Br,
// i.e. 12 bf16 MFMAs (16x16x32) per 16x16 sub-tile and 32-wide K step.
// The gate epilogue reads C back from LDS: one thread per (l, r) applies the
// D^2 x D^2 gate to all D^2 entries of its (t1, t2) block.
#include "ea_dev.h"
#include "ea_kernels.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int KS = 32;       // K per MFMA
constexpr int KPAD = KS + 8; // LDS row pitch in bf16 (keeps 16-byte alignment)

struct Split {
    __bf16 hi, lo;
};
__device__ __forceinline__ Split split(float x) {
    Split s;
    s.hi = (__bf16)x;
    s.lo = (__bf16)(x - (float)s.hi);
    return s;
}

template <int D>
__global__ __launch_bounds__(256) void k_theta_bf16x3(const cx<float> *__restrict__ A,
                                                      const cx<float> *__restrict__ B,
                                                      const cx<float> *__restrict__ G,
                                                      cx<float> *__restrict__ W, int chiL,
                                                      int chiM, int chiR, int orient) {
    constexpr int R = 16 * D;           // tile rows (l, t1) and columns (t2, r)
    constexpr int SUB = (D * D) / 4;    // 16x16 sub-tiles per wave (4 waves)
    // operand planes: [re/im][hi/lo][row][k]; B stored transposed ([col][k]).
    // The finished C tile reuses the operand space.
    union Smem {
        struct {
            __bf16 a[2][2][R][KPAD];
            __bf16 b[2][2][R][KPAD];
        } op;
        cx<float> c[R][R + 1];
    };
    __shared__ __attribute__((aligned(16))) Smem sm;
    __shared__ cx<float> Gs[D * D][D * D];
    auto &As = sm.op.a;
    auto &Bs = sm.op.b;
    auto &Cs = sm.c;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l0 = blockIdx.y * 16, r0 = blockIdx.x * 16;
    for (int e = tid; e < D * D * D * D; e += 256) Gs[e / (D * D)][e % (D * D)] = G[e];

    f32x4 crr[SUB], cii[SUB], cim[SUB];
#pragma unroll
    for (int u = 0; u < SUB; ++u)
        for (int v = 0; v < 4; ++v) crr[u][v] = cii[u][v] = cim[u][v] = 0.f;

    const size_t ldb = (size_t)D * chiR;
    for (int k0 = 0; k0 < chiM; k0 += KS) {
        // A tile: rows l0*D .. l0*D + R of the (chiL D) x chiM matrix
        for (int e = tid; e < R * KS; e += 256) {
            const int row = e / KS, kk = e % KS;
            const int gk = k0 + kk, l = l0 + row / D;
            cx<float> v = zero_cx<float>();
            if (l < chiL && gk < chiM) v = A[((size_t)l0 * D + row) * chiM + gk];
            const Split re = split(v.x), im = split(v.y);
            As[0][0][row][kk] = re.hi;
            As[0][1][row][kk] = re.lo;
            As[1][0][row][kk] = im.hi;
            As[1][1][row][kk] = im.lo;
        }
        // B tile: column c = t2 * 16 + rr is B column t2 * chiR + r0 + rr
        for (int e = tid; e < R * KS; e += 256) {
            const int kk = e / R, c = e % R;
            const int gk = k0 + kk, t2 = c / 16, r = r0 + c % 16;
            cx<float> v = zero_cx<float>();
            if (r < chiR && gk < chiM) v = B[(size_t)gk * ldb + (size_t)t2 * chiR + r];
            const Split re = split(v.x), im = split(v.y);
            Bs[0][0][c][kk] = re.hi;
            Bs[0][1][c][kk] = re.lo;
            Bs[1][0][c][kk] = im.hi;
            Bs[1][1][c][kk] = im.lo;
        }
        __syncthreads();
        const int kq = 8 * (lane >> 4), rl = lane & 15;
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            const int st = wave * SUB + u, ti = st / D, tj = st % D;
            bf16x8 a[2][2], b[2][2];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    a[p][h] = *(const bf16x8 *)&As[p][h][ti * 16 + rl][kq];
                    b[p][h] = *(const bf16x8 *)&Bs[p][h][tj * 16 + rl][kq];
                }
            // Re-Re, Im-Im and cross products, each as hi*hi + hi*lo + lo*hi
            crr[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], b[0][0], crr[u], 0, 0, 0);
            crr[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], b[0][1], crr[u], 0, 0, 0);
            crr[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][1], b[0][0], crr[u], 0, 0, 0);
            cii[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], b[1][0], cii[u], 0, 0, 0);
            cii[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], b[1][1], cii[u], 0, 0, 0);
            cii[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][1], b[1][0], cii[u], 0, 0, 0);
            cim[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], b[1][0], cim[u], 0, 0, 0);
            cim[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][0], b[1][1], cim[u], 0, 0, 0);
            cim[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][1], b[1][0], cim[u], 0, 0, 0);
            cim[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], b[0][0], cim[u], 0, 0, 0);
            cim[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][0], b[0][1], cim[u], 0, 0, 0);
            cim[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][1], b[0][0], cim[u], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulators -> LDS: lane holds rows 4 (lane / 16) + v, column lane % 16
#pragma unroll
    for (int u = 0; u < SUB; ++u) {
        const int st = wave * SUB + u, ti = st / D, tj = st % D;
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Cs[ti * 16 + 4 * (lane >> 4) + v][tj * 16 + (lane & 15)] =
                mk<float>(crr[u][v] - cii[u][v], cim[u][v]);
    }
    __syncthreads();
    // gate epilogue; the thread order follows the contiguous output index
    const int ll = orient == 0 ? (tid & 15) : (tid >> 4);
    const int rr = orient == 0 ? (tid >> 4) : (tid & 15);
    const int l = l0 + ll, r = r0 + rr;
    if (l >= chiL || r >= chiR) return;
    cx<float> c[D][D];
#pragma unroll
    for (int t1 = 0; t1 < D; ++t1)
#pragma unroll
        for (int t2 = 0; t2 < D; ++t2) c[t1][t2] = Cs[ll * D + t1][t2 * 16 + rr];
#pragma unroll
    for (int s1 = 0; s1 < D; ++s1)
#pragma unroll
        for (int s2 = 0; s2 < D; ++s2) {
            cx<float> th = zero_cx<float>();
#pragma unroll
            for (int t1 = 0; t1 < D; ++t1)
#pragma unroll
                for (int t2 = 0; t2 < D; ++t2) cmac(th, Gs[s1 * D + s2][t1 * D + t2], c[t1][t2]);
            const size_t row = (size_t)l * D + s1, col = (size_t)s2 * chiR + r;
            if (orient == 0)
                W[col * (size_t)(D * chiL) + row] = th;
            else
                W[row * (size_t)(D * chiR) + col] = conj(th);
        }
}

}  // namespace

void launch_theta_bf16x3(const void *A, const void *B, const void *G, void *W, int chiL,
                         int chiM, int chiR, int d, int orient, hipStream_t s) {
    dim3 grid((chiR + 15) / 16, (chiL + 15) / 16);
    if (d == 2)
        k_theta_bf16x3<2><<<grid, 256, 0, s>>>((const cx<float> *)A, (const cx<float> *)B,
                                               (const cx<float> *)G, (cx<float> *)W, chiL, chiM,
                                               chiR, orient);
    else
        k_theta_bf16x3<4><<<grid, 256, 0, s>>>((const cx<float> *)A, (const cx<float> *)B,
                                               (const cx<float> *)G, (cx<float> *)W, chiL, chiM,
                                               chiR, orient);
}

// ---------------------------------------------------------------------------
// The same contraction in FP32 or FP64 on the matching 16x16x4 matrix cores.
// A workgroup (4 waves) owns a 64 x 64 tile of C[(l, t1), (t2, r)], i.e.
// 64/D values of l by 64/D values of r with all D^2 (t1, t2) combinations, so
// the gate epilogue has every input it needs in LDS.  Each wave computes a
// 32 x 32 quarter as 2 x 2 MFMA tiles; complex products as four real MFMAs
// (Re += ar br - ai bi, Im += ar bi + ai br).  K advances in steps of 32;
// every thread issues all its loads of a step before writing LDS.
// ---------------------------------------------------------------------------
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaT;
template <>
struct MfmaT<float> {
    typedef f32x4 acc;
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
    static __device__ __forceinline__ acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct MfmaT<double> {
    typedef f64x4 acc;
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
    static __device__ __forceinline__ acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

constexpr int TT = 64;  // C tile edge
constexpr int TK = 32;  // K step

template <typename T, int D>
__global__ __launch_bounds__(256) void k_theta_mfma(const cx<T> *__restrict__ A,
                                                    const cx<T> *__restrict__ B,
                                                    const cx<T> *__restrict__ G,
                                                    cx<T> *__restrict__ W, int chiL, int chiM,
                                                    int chiR, int orient) {
    using MF = MfmaT<T>;
    constexpr int TL = TT / D, TR = TT / D;
    // operand planes: A as [row][k], B transposed as [col][k]; the finished C
    // tile reuses the space
    union Smem {
        struct {
            T ar[TT][TK + 1], ai[TT][TK + 1];
            T br[TT][TK + 1], bi[TT][TK + 1];
        } op;
        cx<T> c[TT][TT + 1];
    };
    __shared__ Smem sm;
    __shared__ cx<T> Gs[D * D][D * D];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l0 = blockIdx.y * TL, r0 = blockIdx.x * TR;
    for (int e = tid; e < D * D * D * D; e += 256) Gs[e / (D * D)][e % (D * D)] = G[e];
    typename MF::acc re[2][2], im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) re[a][b][v] = im[a][b][v] = T(0);
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;  // this wave's quarter
    const size_t ldb = (size_t)D * chiR;
    constexpr int PER = TT * TK / 256;
    for (int k0 = 0; k0 < chiM; k0 += TK) {
        cx<T> va[PER], vb[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            {  // A: row = e / TK, k = e % TK
                const int row = e / TK, kk = e % TK, gk = k0 + kk, l = l0 + row / D;
                va[u] = (l < chiL && gk < chiM) ? A[((size_t)l0 * D + row) * chiM + gk]
                                                : zero_cx<T>();
            }
            {  // B: k = e / TT, col = e % TT (col = t2 * TR + rr)
                const int kk = e / TT, c = e % TT, gk = k0 + kk, t2 = c / TR, r = r0 + c % TR;
                vb[u] = (r < chiR && gk < chiM) ? B[(size_t)gk * ldb + (size_t)t2 * chiR + r]
                                                : zero_cx<T>();
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            const int row = e / TK, kk = e % TK;
            sm.op.ar[row][kk] = va[u].x;
            sm.op.ai[row][kk] = va[u].y;
            const int kb = e / TT, c = e % TT;
            sm.op.br[c][kb] = vb[u].x;
            sm.op.bi[c][kb] = vb[u].y;
        }
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < TK; kk += 4) {
            const int kq = kk + (lane >> 4), rl = lane & 15;
            T ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                ar[a] = sm.op.ar[wr + 16 * a + rl][kq];
                ai[a] = sm.op.ai[wr + 16 * a + rl][kq];
                br[a] = sm.op.br[wc + 16 * a + rl][kq];
                bi[a] = sm.op.bi[wc + 16 * a + rl][kq];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    re[a][b] = MF::op(ar[a], br[b], re[a][b]);
                    re[a][b] = MF::op(-ai[a], bi[b], re[a][b]);
                    im[a][b] = MF::op(ar[a], bi[b], im[a][b]);
                    im[a][b] = MF::op(ai[a], br[b], im[a][b]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                sm.c[wr + 16 * a + MF::row(lane, v)][wc + 16 * b + (lane & 15)] =
                    mk<T>(re[a][b][v], im[a][b][v]);
    __syncthreads();
    // gate epilogue: one (l, r) per thread and pass; the fastest thread index
    // follows the contiguous output index
    for (int e = tid; e < TL * TR; e += 256) {
        const int ll = orient == 0 ? e % TL : e / TR;
        const int rr = orient == 0 ? e / TL : e % TR;
        const int l = l0 + ll, r = r0 + rr;
        if (l >= chiL || r >= chiR) continue;
        cx<T> c[D][D];
#pragma unroll
        for (int t1 = 0; t1 < D; ++t1)
#pragma unroll
            for (int t2 = 0; t2 < D; ++t2) c[t1][t2] = sm.c[ll * D + t1][t2 * TR + rr];
#pragma unroll
        for (int s1 = 0; s1 < D; ++s1)
#pragma unroll
            for (int s2 = 0; s2 < D; ++s2) {
                cx<T> th = zero_cx<T>();
#pragma unroll
                for (int t1 = 0; t1 < D; ++t1)
#pragma unroll
                    for (int t2 = 0; t2 < D; ++t2)
                        cmac(th, Gs[s1 * D + s2][t1 * D + t2], c[t1][t2]);
                const size_t row = (size_t)l * D + s1, col = (size_t)s2 * chiR + r;
                if (orient == 0)
                    W[col * (size_t)(D * chiL) + row] = th;
                else
                    W[row * (size_t)(D * chiR) + col] = conj(th);
            }
    }
}

}  // namespace

template <typename T>
void launch_theta_mfma(const void *A, const void *B, const void *G, void *W, int chiL, int chiM,
                       int chiR, int d, int orient, hipStream_t s) {
    if (d == 2) {
        dim3 grid((chiR + TT / 2 - 1) / (TT / 2), (chiL + TT / 2 - 1) / (TT / 2));
        k_theta_mfma<T, 2><<<grid, 256, 0, s>>>((const cx<T> *)A, (const cx<T> *)B,
                                                (const cx<T> *)G, (cx<T> *)W, chiL, chiM, chiR,
                                                orient);
    } else {
        dim3 grid((chiR + TT / 4 - 1) / (TT / 4), (chiL + TT / 4 - 1) / (TT / 4));
        k_theta_mfma<T, 4><<<grid, 256, 0, s>>>((const cx<T> *)A, (const cx<T> *)B,
                                                (const cx<T> *)G, (cx<T> *)W, chiL, chiM, chiR,
                                                orient);
    }
}
template void launch_theta_mfma<float>(const void *, const void *, const void *, void *, int, int,
                                       int, int, int, hipStream_t);
template void launch_theta_mfma<double>(const void *, const void *, const void *, void *, int,
                                        int, int, int, int, hipStream_t);
