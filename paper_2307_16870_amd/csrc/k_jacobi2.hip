// Multi-workgroup round of the block one-sided Jacobi SVD, split in three
// kernels so that the two dense contractions of a round run on MFMA over the
// whole chip and only the small rotation search is per block pair:
//
//   k_jgram : partial Gram matrices  G_c = W[rows_c, cols]^H W[rows_c, cols]
//             (block pair x row chunk workgroups, MFMA 16x16x4)
//   k_jeig  : G = sum_c G_c, two-sided Jacobi rotations on G accumulated in J
//             (one workgroup per block pair)
//   k_japply: W[rows, cols] <- W[rows, cols] J and V[rows, cols] <- V[rows, cols] J
//             (block pair x row chunk workgroups, MFMA 16x16x4)
//
// The rotation of a column pair is the Hestenes one-sided rotation expressed
// on the Gram matrix (symmetric 2x2 Schur rotation of [[a, |g|], [|g|, b]]
// after removing the phase of g).  Block pairs follow the round-robin
// (circle method) ordering of the blocks.  W, V are column-major.
#include "ea_dev.h"
#include "ea_kernels.h"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Output layout of one 16x16 tile: lane l, value v holds D[row(l, v)][l % 16]
// (measured on gfx950: f32 rows 4*(l/16)+v, f64 rows l/16+4v).  Inputs: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16].
template <>
struct Mfma<float> {
    typedef f4v acc;
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    typedef d4v acc;
    static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Columns owned by block pair `pair` in round `rnd` (blocks of width w).
__device__ __forceinline__ int pair_columns(int pair, int rnd, int nb, int w, int n, int *cols,
                                            int tid, int nth) {
    const int a = rr_player(pair, rnd, nb), b = rr_player(nb - 1 - pair, rnd, nb);
    const int a0 = a * w, a1 = min(a0 + w, n), b0 = b * w, b1 = min(b0 + w, n);
    const int na = max(0, a1 - a0), nbb = max(0, b1 - b0);
    for (int c = tid; c < na; c += nth) cols[c] = a0 + c;
    for (int c = tid; c < nbb; c += nth) cols[na + c] = b0 + c;
    return na + nbb;
}

// Change stamps of a factorisation (zero at its start): ver[b] (b < nb) counts
// the rounds that rotated column block b; seen[2 (rnd nb/2 + pair)] holds
// ver + 1 of the pair's two blocks when round rnd last examined the pair (0:
// never).  The pairing of a round is the same in every sweep, so a pair whose
// blocks are unchanged since that examination would form the same Gram
// matrix from bit-identical columns and again find no rotation (had it
// rotated, both stamps would have moved since): such a pair is skipped.
__device__ __forceinline__ bool pair_unchanged(const int *stamp, int nb, int rnd, int pair) {
    if (!stamp) return false;
    const int a = rr_player(pair, rnd, nb), b = rr_player(nb - 1 - pair, rnd, nb);
    const int *seen = stamp + nb + 2 * (rnd * (nb / 2) + pair);
    return seen[0] == stamp[a] + 1 && seen[1] == stamp[b] + 1;
}

constexpr int JRS = 64;  // rows staged in LDS per step

// True whenever jacobi_rotation would rotate the pair (it may also be true
// when it would not).  FP32 data: |g|^2 > tol^2 al be in FP64 with a relative
// margin of 1e-9 toward rotating, far wider than the error of the refined
// square roots of the exact test, and no square root or reciprocal on the
// way; squares of FP32 values neither overflow nor underflow in FP64.  FP64
// data take the exact test.
template <typename T>
__device__ __forceinline__ bool may_rotate(T al, T be, cx<T> ga, T tol) {
    if constexpr (sizeof(T) == 4) {
        const double gx = ga.x, gy = ga.y, g2 = gx * gx + gy * gy;
        const double ab = (double)al * (double)be, t = tol;
        return g2 > 0.0 && ab >= 0.0 && (ab == 0.0 || g2 > t * t * ab * (1.0 - 1e-9));
    } else {
        JRot<T> rt;
        return jacobi_rotation(al, be, ga, tol, rt);
    }
}

// A rotation as the block and J updates read it (16 bytes in FP32): gm < 0
// marks a pair that does not rotate (1 - cos is never negative).
template <typename T>
struct alignas(16) RotP {
    T s, gm;  // sin, 1 - cos
    cx<T> e;  // phase conj(g) / |g|
};
// The diagonal entries of the pair's columns before the step, the shift t |g|
// they take when it rotates, and whether it does.
template <typename T>
struct alignas(16) RotD {
    T al, be, tg;
    int on;
};

// Load rows [r0, r0+JRS) of the owned columns into split real/imag LDS planes,
// zero-padding rows >= r_end and columns >= nc.
// All loads of a thread are issued before the first LDS write, so their
// latencies overlap instead of adding up.
template <typename T, int NC>
__device__ __forceinline__ void stage_load(const cx<T> *__restrict__ X, int M, const int *cols,
                                           int nc, int r0, int r_end, cx<T> (&v)[JRS * NC / 256],
                                           int tid) {
    constexpr int PER = JRS * NC / 256;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + 256 * i, c = e / JRS, row = r0 + e % JRS;
        v[i] = (c < nc && row < r_end) ? X[(size_t)cols[c] * M + row] : zero_cx<T>();
    }
}
template <typename T, int NC>
__device__ __forceinline__ void stage_store(const cx<T> (&v)[JRS * NC / 256], T (*Sr)[NC + 1],
                                            T (*Si)[NC + 1], int tid) {
    constexpr int PER = JRS * NC / 256;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = tid + 256 * i, c = e / JRS, rr = e % JRS;
        Sr[rr][c] = v[i].x;
        Si[rr][c] = v[i].y;
    }
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_jgram(const cx<T> *__restrict__ W, int m, int n, int w,
                                               int nb, int rnd, int rpc,
                                               cx<T> *__restrict__ partial,
                                               const int *__restrict__ stamp) {
    using MF = Mfma<T>;
    constexpr int NT = NC / 16;
    constexpr int NU = NT * (NT + 1) / 2;  // upper-triangular 16x16 tiles
    constexpr int UPW = (NU + 3) / 4;       // tiles per wave
    // NU = 4 UPW - 2 (NC = 64: 10 tiles): the last two tiles are shared by
    // four waves, waves 0-1 taking the first half of every stage's rows and
    // waves 2-3 the second, so that each wave issues 2.5 tiles' products
    constexpr bool SPLIT = NU % 4 == 2;
    __shared__ T Sr[JRS][NC + 1], Si[JRS][NC + 1];
    __shared__ int cols[NC];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int pair = blockIdx.x, chunk = blockIdx.y, nchunks = gridDim.y;
    if (pair_unchanged(stamp, nb, rnd, pair)) return;
    const int nc = pair_columns(pair, rnd, nb, w, n, cols, tid, 256);
    const int r_begin = chunk * rpc, r_end = min(m, r_begin + rpc);
    int ti_[UPW], tj_[UPW];
#pragma unroll
    for (int u = 0; u < UPW; ++u) {
        int t = (SPLIT && u == UPW - 1 && wave >= 2) ? 4 * u + wave - 2 : wave + 4 * u;
        int ti = 0, tj = 0, k = 0;
        ti_[u] = -1;
        for (ti = 0; ti < NT; ++ti)
            for (tj = ti; tj < NT; ++tj, ++k)
                if (k == t) {
                    ti_[u] = ti;
                    tj_[u] = tj;
                }
    }
    typename MF::acc re[UPW], im[UPW];
#pragma unroll
    for (int u = 0; u < UPW; ++u) {
        re[u] = MF::zero();
        im[u] = MF::zero();
    }
    __syncthreads();
    // rows of the next step are loaded while this step's products run
    cx<T> v[JRS * NC / 256];
    if (r_begin < r_end) stage_load<T, NC>(W, m, cols, nc, r_begin, r_end, v, tid);
    for (int r0 = r_begin; r0 < r_end; r0 += JRS) {
        stage_store<T, NC>(v, Sr, Si, tid);
        __syncthreads();
        if (r0 + JRS < r_end) stage_load<T, NC>(W, m, cols, nc, r0 + JRS, r_end, v, tid);
#pragma unroll
        for (int u = 0; u < UPW; ++u) {
            if (ti_[u] < 0) continue;
            const int pc = ti_[u] * 16 + lane % 16, qc = tj_[u] * 16 + lane % 16;
            const bool half = SPLIT && u == UPW - 1;
            const int kb = (half && wave >= 2) ? JRS / 2 : 0;
            const int ke = (half && wave < 2) ? JRS / 2 : JRS;
#pragma unroll 4
            for (int k0 = kb; k0 < ke; k0 += 4) {
                const int kr = k0 + lane / 16;
                const T ar = Sr[kr][pc], ai = Si[kr][pc];
                const T br = Sr[kr][qc], bi = Si[kr][qc];
                re[u] = MF::op(ar, br, re[u]);
                re[u] = MF::op(ai, bi, re[u]);
                im[u] = MF::op(ar, bi, im[u]);
                im[u] = MF::op(-ai, br, im[u]);
            }
        }
        __syncthreads();
    }
    if constexpr (SPLIT) {
        // waves 2-3 hand their halves of the shared tiles to waves 0-1
        // through LDS (free: the stage loop ended with a barrier)
        T *hr = &Sr[0][0], *hi = &Si[0][0];
        if (wave >= 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                hr[(wave - 2) * 256 + v * 64 + lane] = re[UPW - 1][v];
                hi[(wave - 2) * 256 + v * 64 + lane] = im[UPW - 1][v];
            }
        }
        __syncthreads();
        if (wave < 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                re[UPW - 1][v] += hr[wave * 256 + v * 64 + lane];
                im[UPW - 1][v] += hi[wave * 256 + v * 64 + lane];
            }
        }
    }
    cx<T> *out = partial + ((size_t)pair * nchunks + chunk) * NC * NC;
#pragma unroll
    for (int u = 0; u < UPW; ++u) {
        if (ti_[u] < 0) continue;
        if (SPLIT && u == UPW - 1 && wave >= 2) continue;  // added into waves 0-1
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = ti_[u] * 16 + MF::row(lane, v), q = tj_[u] * 16 + lane % 16;
            out[p * NC + q] = mk<T>(re[u][v], im[u][v]);
        }
    }
}

template <typename T, int NC, int NTH, int INTER>
__global__ __launch_bounds__(NTH) void k_jeig(const cx<T> *__restrict__ partial, int nchunks,
                                              int n, int w, int nb, int rnd, T tol,
                                              int inner_max,
                                              cx<T> *__restrict__ Jout,
                                              int *__restrict__ rotflag,
                                              int *__restrict__ rot_counter,
                                              int *__restrict__ stamp) {
    constexpr int NP = NC / 2;
    __shared__ cx<T> G[NC][NC + 1];
    __shared__ cx<T> J[NC][NC + 1];
    static_assert((NP & (NP - 1)) == 0 && NP <= 256, "block pair width must be a power of 2");
    __shared__ RotP<T> rp_[2][NP];  // this step's rotations and the next step's
    __shared__ RotD<T> rd_[2][NP];
    __shared__ unsigned short tab_[NP * (NP + 1) / 2];  // packed (a, b), a <= b
    __shared__ int cols[NC];
    __shared__ int nrot_sh[2];
    const int tid = threadIdx.x, pair = blockIdx.x;
    if (pair_unchanged(stamp, nb, rnd, pair)) {
        if (tid == 0) rotflag[pair] = 0;
        return;
    }
    const int nc = pair_columns(pair, rnd, nb, w, n, cols, tid, NTH);
    // Sum the partial Gram tiles (upper triangle) in a fixed order per entry.
    // Rows r and NC - 1 - r together hold NC + 1 entries of the triangle, so
    // entry e of the NC/2 x (NC + 1) arrangement spreads the triangle evenly
    // over the threads; each thread issues the chunk loads of two entries
    // before summing either.
    const cx<T> *src = partial + (size_t)pair * nchunks * NC * NC;
    constexpr int NUT = (NC / 2) * (NC + 1);
    auto tri = [&](int e, int &p, int &q) {
        const int r = e / (NC + 1), c = e % (NC + 1);
        if (c < NC - r) {
            p = r;
            q = r + c;
        } else {
            p = NC - 1 - r;
            q = p + (c - (NC - r));
        }
    };
    auto put = [&](int p, int q, double sx, double sy) {
        if (p != q) {
            G[p][q] = mk<T>((T)sx, (T)sy);
            G[q][p] = mk<T>((T)sx, (T)-sy);
        } else {
            G[p][p] = mk<T>((T)sx, T(0));
        }
    };
    for (int e0 = tid; e0 < NUT; e0 += 2 * NTH) {
        const int e1 = e0 + NTH;
        const bool two = e1 < NUT;
        int p0, q0, p1 = 0, q1 = 0;
        tri(e0, p0, q0);
        if (two) tri(e1, p1, q1);
        const size_t o0 = (size_t)p0 * NC + q0, o1 = (size_t)p1 * NC + q1;
        double sx0 = 0.0, sy0 = 0.0, sx1 = 0.0, sy1 = 0.0;
        int c = 0;
        for (; c + 8 <= nchunks; c += 8) {
            cx<T> v0[8], v1[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v0[j] = src[(size_t)(c + j) * NC * NC + o0];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v1[j] = two ? src[(size_t)(c + j) * NC * NC + o1] : zero_cx<T>();
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sx0 += (double)v0[j].x;
                sy0 += (double)v0[j].y;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sx1 += (double)v1[j].x;
                sy1 += (double)v1[j].y;
            }
        }
        for (; c < nchunks; ++c) {
            const cx<T> v0 = src[(size_t)c * NC * NC + o0];
            sx0 += (double)v0.x;
            sy0 += (double)v0.y;
            if (two) {
                const cx<T> v1 = src[(size_t)c * NC * NC + o1];
                sx1 += (double)v1.x;
                sy1 += (double)v1.y;
            }
        }
        put(p0, q0, sx0, sy0);
        if (two) put(p1, q1, sx1, sy1);
    }
    for (int e = tid; e < NC * NC; e += NTH) {
        const int p = e / NC, q = e % NC;
        J[p][q] = mk<T>(p == q ? T(1) : T(0), T(0));
    }
    if (tid < 2) nrot_sh[tid] = 0;
    for (int e = tid; e < NP * NP; e += NTH) {
        const int a = e / NP, b = e % NP;
        if (a <= b) tab_[a * NP - a * (a - 1) / 2 + (b - a)] = (unsigned short)((a << 8) | b);
    }
    __syncthreads();
    const int nce = nc + (nc & 1);
    // inter = 0: every pair of the nc columns (round-robin over nce players,
    // nce - 1 steps of nce / 2 pairs).  inter = 1: only the na x nbb pairs
    // across the two blocks, step k pairing column i of block a with column
    // (i + k) mod w of block b (w steps of w pairs); the pairs inside a block
    // were rotated in the first round of the sweep.
    const int na = max(0, min(w, n - rr_player(pair, rnd, nb) * w));
    constexpr bool inter = INTER != 0;
    const int npairs = inter ? w : nce / 2;
    const int nsteps = inter ? w : nce - 1;
    // Columns (p, q) of pair slot `sl` at step `step`.  The p, q of all slots
    // partition the rows of G: in the inter-block order an idle slot of a
    // short block a takes a row past na + w (zero rows below NC).  Indices are
    // arithmetic, so the update threads need no lookup before their loads.
    auto slot_pq = [&](int sl, int step, int &pp, int &qq) -> bool {
        if (inter) {
            pp = sl < na ? sl : na + w + (sl - na);
            qq = na + (w == NP ? ((sl + step) & (NP - 1)) : (sl + step) % w);
            return sl < na && qq < nc;
        }
        pp = rr_player(sl, step, nce);
        qq = rr_player(nce - 1 - sl, step, nce);
        if (pp > qq) {
            const int t = pp;
            pp = qq;
            qq = t;
        }
        return qq < nc;
    };
    // rotation of pair slot `sl` at `step` from the diagonal entries al, be of
    // its columns p, q and the entry ga = G[p][q].  The record carries al and
    // be whether or not the pair rotates (the chained formation below follows
    // the diagonal through them).
    auto form_rot = [&](int sl, int step, T al, T be, cx<T> ga) -> RotRec<T> {
        int p, q;
        RotRec<T> r;
        r.s = r.gm = r.tg = T(0);
        r.al = al;
        r.be = be;
        r.e = mk<T>(T(1), T(0));
        r.on = 0;
        if (slot_pq(sl, step, p, q)) {
            JRot<T> rt;
            if (jacobi_rotation(al, be, ga, tol, rt)) {
                r.s = rt.s;
                r.gm = rt.gm;
                r.e = rt.e;
                r.tg = rt.tg;
                r.on = 1;
            }
        }
        return r;
    };
    // the same from the current G (p, q of every slot index rows of G)
    auto make_rot = [&](int sl, int step) -> RotRec<T> {
        int p, q;
        slot_pq(sl, step, p, q);
        return form_rot(sl, step, G[p][p].x, G[q][q].x, G[p][q]);
    };
    // Every caller of make_rot / form_rot is a thread tid < npairs <= 32, all
    // in the first wave: the rotations of a step are counted by one ballot.
    auto count_rot = [&](bool on, int cnt_slot) {
        const unsigned long long bal = __ballot(on);
        if (tid == 0) nrot_sh[cnt_slot] += __popcll(bal);
    };
    auto store_rot = [&](int buf, int sl, const RotRec<T> &r) {
        RotP<T> rp;
        rp.s = r.s;
        rp.gm = r.on ? r.gm : T(-1);
        rp.e = r.e;
        rp_[buf][sl] = rp;
        RotD<T> rd;
        rd.al = r.al;
        rd.be = r.be;
        rd.tg = r.tg;
        rd.on = r.on;
        rd_[buf][sl] = rd;
    };
    // G <- M^H G M on the 2x2 block (row pair a, column pair b), a <= b; block
    // (b, a) is its conjugate transpose, written alongside.  x01, x10 return
    // the block's entries (p_a, q_b) and (q_a, p_b) after the update.
    // Inter-block order: rows p (block a) against columns q (block b) are kept
    // in the upper-right quadrant only, an entry (q, p) being read as the
    // conjugate of (p, q), and the lower triangle of the block-a quadrant is
    // not written: no step and no rotation reads it (the p indices of a block
    // are increasing, and rotations read (p, p), (q, q) and (p, q)).
    auto block_update = [&](int a, int b, int step, int buf, cx<T> &x01, cx<T> &x10) {
        int pa, qa, pb, qb;
        slot_pq(a, step, pa, qa);
        slot_pq(b, step, pb, qb);
        const RotP<T> ra = rp_[buf][a], rb = rp_[buf][b];
        const bool ona = ra.gm >= T(0), onb = rb.gm >= T(0);
        cx<T> g00 = G[pa][pb], g01 = G[pa][qb], g11 = G[qa][qb];
        cx<T> g10 = inter ? conj(G[pb][qa]) : G[qa][pb];
        x01 = g01;
        x10 = g10;
        if (!ona && !onb) return;
        if (a == b) {  // rotated pair: exact diagonal
            const RotD<T> d = rd_[buf][a];
            G[pa][qa] = zero_cx<T>();
            if (!inter) G[qa][pa] = zero_cx<T>();
            G[pa][pa] = mk<T>(d.al - d.tg, T(0));
            G[qa][qa] = mk<T>(d.be + d.tg, T(0));
            x01 = x10 = zero_cx<T>();
            return;
        }
        const bool va = qa < nc, vb = qb < nc;
        if (!vb) g01 = g11 = zero_cx<T>();
        if (!va) g10 = g11 = zero_cx<T>();
        if (onb) {  // columns: [x0, x1] = [g0, g1] [[c, s], [-s e, c e]]
            rot_pair(g00, rb.e * g01, rb.s, rb.gm, g00, g01);
            rot_pair(g10, rb.e * g11, rb.s, rb.gm, g10, g11);
        }
        if (ona) {  // rows: [r0; r1] = [[c, -s e*], [s, c e*]] [g0; g1]
            const cx<T> ec = conj(ra.e);
            rot_pair(g00, ec * g10, ra.s, ra.gm, g00, g10);
            rot_pair(g01, ec * g11, ra.s, ra.gm, g01, g11);
        }
        x01 = g01;
        x10 = g10;
        G[pa][pb] = g00;
        if (!inter) G[pb][pa] = conj(g00);
        if (vb) {
            G[pa][qb] = g01;
            if (!inter) G[qb][pa] = conj(g01);
        }
        if (va) {
            if (!inter) G[qa][pb] = g10;
            G[pb][qa] = conj(g10);
        }
        if (va && vb) {
            G[qa][qb] = g11;
            G[qb][qa] = conj(g11);
        }
    };
    // Inter-block order: slot sl always rotates column sl of block a against
    // column na + (sl + step) mod w of block b, so J's columns are held in
    // registers: lane sl of a group of NP lanes keeps J[row][sl] (block a)
    // and the block-b column it meets at the current step, and after each
    // step takes the block-b values of slot (sl + 1) mod w.  After whole
    // inner sweeps (w steps each) every block-b value is back at its slot.
    // The first wave, which forms the rotations, holds no rows of J when the
    // other waves can hold them all at 4 rows per thread (FP32: in FP64 the
    // extra rows spill registers).
    constexpr int JG0 = (INTER != 0 && sizeof(T) == 4 && NTH >= 256 && NP <= 64 &&
                         (NC + NTH / NP - 64 / NP - 1) / (NTH / NP - 64 / NP) <= 4)
                            ? 64 / NP
                            : 0;
    constexpr int RGROUPS = NTH / NP - JG0;           // row groups of NP lanes
    constexpr int RI = (NC + RGROUPS - 1) / RGROUPS;  // rows per thread
    constexpr bool REGJ = INTER != 0 && NP <= 64 && RGROUPS >= 1 && RI <= 4;
    const int sl_j = tid % NP, grp_j = tid / NP - JG0;  // grp_j < 0: the first wave
    cx<T> ja[RI], jb[RI];
    int src_j = tid % 64;
    if constexpr (REGJ) {
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int row = grp_j < 0 ? -1 : grp_j + i * RGROUPS;
            ja[i] = mk<T>(sl_j < na && row == sl_j ? T(1) : T(0), T(0));
            jb[i] = mk<T>(sl_j < w && row == na + sl_j ? T(1) : T(0), T(0));
        }
        const int lane = tid % 64;
        src_j = (lane & ~(NP - 1)) | (sl_j < w ? (sl_j + 1) % w : sl_j);
    }
    // With skipping on, a pair none of whose column pairs is out of tolerance
    // runs no inner sweep: no rotation would change G, so every later step
    // would see exactly the values checked here and again rotate nothing.
    bool need = true;
    if (stamp) {
        bool any = false;
        for (int e = tid; e < NC * NC && !any; e += NTH) {
            const int p = e / NC, q = e % NC;
            const bool cand = inter ? (p < na && q >= na && q < nc) : (p < q && q < nc);
            if (cand) any = may_rotate(G[p][p].x, G[q][q].x, G[p][q], tol);
        }
        need = __syncthreads_or(any) != 0;
    }
    // J <- J M for the rotations of one step
    auto j_update = [&](int step, int buf) {
        if constexpr (REGJ) {
            if (grp_j < 0) return;  // uniform over the first wave
            const RotP<T> rb = rp_[buf][sl_j < npairs ? sl_j : 0];
            const bool on = sl_j < npairs && rb.gm >= T(0);
#pragma unroll
            for (int i = 0; i < RI; ++i) {
                if (on) rot_pair(ja[i], rb.e * jb[i], rb.s, rb.gm, ja[i], jb[i]);
                jb[i] = mk<T>(__shfl(jb[i].x, src_j), __shfl(jb[i].y, src_j));
            }
        } else {
            for (int e = tid; e < NP * NC; e += NTH) {
                const int b = e / NC, row = e % NC;
                if (b >= npairs || row >= nc) continue;
                int p, q;
                slot_pq(b, step, p, q);
                const RotP<T> rb = rp_[buf][b];
                const cx<T> jp = J[row][p], jq = J[row][q];
                if (rb.gm >= T(0)) rot_pair(jp, rb.e * jq, rb.s, rb.gm, J[row][p], J[row][q]);
            }
        }
    };
    // Chained formation (inter-block order with w = NP): at step k + 1 slot s
    // pairs column s of block a with the block-b column that slot s + 1 held
    // at step k.  Its entries are the diagonal of column s (al - tg if slot s
    // rotated at step k, else al), that of slot s + 1's block-b column (be +
    // tg, else be) and entry (p_s, q_{s+1}) of the 2x2 block (s, s + 1) just
    // updated.  The first wave owns the blocks (s, s + 1 mod w), so the
    // thread that updates block (s, s + 1) forms the next rotation of slot s
    // from values it holds (the diagonal values from the rotation records of
    // slots s and s + 1): one barrier per step, and
    // the inputs of every rotation are the values the unchained order reads
    // back from G.
    const bool chain = inter && w == NP && NP >= 4;
    constexpr int NU = NP * (NP + 1) / 2;
    constexpr int G0 = (2 * NP + 63) / 64 * 64;  // first thread of the other blocks
    // the diagonal blocks go to the last wave when it has nothing else to update
    constexpr int D0 = NTH >= G0 + NU + 64 ? NTH - 64 : NP;
    int first = 0;
    if (need && nc >= 2 && (!inter || (na > 0 && nc > na))) {
        for (int isw = 0; isw < inner_max; ++isw) {
            const int slot = isw & 1;
            if (tid < npairs) {
                const RotRec<T> r = make_rot(tid, 0);
                store_rot(0, tid, r);
                count_rot(r.on, slot);
            }
            __syncthreads();
            if (chain) {
                for (int step = 0; step < nsteps; ++step) {
                    const int buf = step & 1;
                    // one block per thread, chosen first, so that a wave runs a
                    // single copy of the update
                    int a = -1, b = -1;
                    if (tid < NP) {
                        const int s1 = tid + 1 == NP ? 0 : tid + 1;
                        a = s1 != 0 ? tid : 0;
                        b = s1 != 0 ? s1 : tid;
                    } else if (tid >= D0 && tid < D0 + NP) {
                        a = b = tid - D0;
                    } else if (tid >= G0 && tid - G0 < NU) {
                        const int ab = tab_[tid - G0];
                        a = ab >> 8;
                        b = ab & 255;
                        if (b <= a + 1 || (a == 0 && b == NP - 1)) a = -1;
                    }
                    cx<T> x01, x10;
                    if (a >= 0) block_update(a, b, step, buf, x01, x10);
                    if (tid < NP && step + 1 < nsteps) {
                        const int s = tid, s1 = s + 1 == NP ? 0 : s + 1;
                        const RotD<T> r0 = rd_[buf][s], r1 = rd_[buf][s1];
                        const T al = r0.on ? r0.al - r0.tg : r0.al;
                        const T be = r1.on ? r1.be + r1.tg : r1.be;
                        const RotRec<T> r =
                            form_rot(s, step + 1, al, be, s1 != 0 ? x01 : conj(x10));
                        store_rot(buf ^ 1, s, r);
                        count_rot(r.on, slot);
                    }
                    if constexpr (NTH < G0 + NU) {  // blocks beyond one per thread
                        for (int e = tid - G0 + NTH; e < NU; e += NTH) {
                            const int ab = tab_[e], a2 = ab >> 8, b2 = ab & 255;
                            if (b2 <= a2 + 1 || (a2 == 0 && b2 == NP - 1)) continue;
                            block_update(a2, b2, step, buf, x01, x10);
                        }
                    }
                    j_update(step, buf);
                    __syncthreads();
                }
            } else {
                for (int step = 0; step < nsteps; ++step) {
                    const int buf = step & 1;
                    // the a <= b blocks are packed (tab_) so that only as many
                    // waves as needed work
                    for (int e = tid; e < NU; e += NTH) {
                        const int ab = tab_[e], a = ab >> 8, b = ab & 255;
                        if (b >= npairs) continue;
                        cx<T> x01, x10;
                        block_update(a, b, step, buf, x01, x10);
                    }
                    __syncthreads();
                    // the next step's rotations need only the updated G: they are
                    // formed while this step's rotations are applied to J
                    if (step + 1 < nsteps && tid < npairs) {
                        const RotRec<T> r = make_rot(tid, step + 1);
                        store_rot(buf ^ 1, tid, r);
                        count_rot(r.on, slot);
                    }
                    j_update(step, buf);
                    __syncthreads();
                }
            }
            const int nr = nrot_sh[slot];
            if (isw == 0) first = nr;
            if (tid == 0) nrot_sh[slot ^ 1] = 0;  // counter of the next sweep
            __syncthreads();
            if (nr == 0) break;
        }
    }
    if constexpr (REGJ) {  // J from the registers (identity entries elsewhere)
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int row = grp_j + i * RGROUPS;
            if (grp_j < 0 || row >= NC) continue;
            if (sl_j < na) J[row][sl_j] = ja[i];
            if (sl_j < w && na + sl_j < NC) J[row][na + sl_j] = jb[i];
        }
        __syncthreads();
    }
    // J is read only for a pair that rotated (the apply kernel checks rotflag)
    cx<T> *jo = Jout + (size_t)pair * NC * NC;
    if (first > 0) {
        for (int e = tid; e < NC * NC; e += NTH) {
            const int p = e / NC, q = e % NC;
            jo[e] = (p < nc && q < nc) ? J[p][q] : zero_cx<T>();
        }
    }
    if (tid == 0) {
        rotflag[pair] = first > 0 ? 1 : 0;
        atomicAdd(rot_counter + 1, nc * nc);
        if (first > 0) {
            atomicAdd(rot_counter, first);
            atomicAdd(rot_counter + 2, nc * nc);
        }
        if (stamp) {
            const int a = rr_player(pair, rnd, nb), b = rr_player(nb - 1 - pair, rnd, nb);
            int *seen = stamp + nb + 2 * (rnd * (nb / 2) + pair);
            seen[0] = stamp[a] + 1;
            seen[1] = stamp[b] + 1;
            if (first > 0) {  // blocks a and b belong to this pair alone in this round
                stamp[a] += 1;
                stamp[b] += 1;
            }
        }
    }
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_japply(cx<T> *__restrict__ W, int m, cx<T> *__restrict__ V,
                                                int n, int w, int nb, int rnd, int nchW, int rpcW,
                                                int rpcV, const cx<T> *__restrict__ Jin,
                                                const int *__restrict__ rotflag) {
    using MF = Mfma<T>;
    constexpr int NT = NC / 16;
    constexpr int TPW = (4 * NT) / 4;  // (JRS/16 row tiles x NT col tiles) / 4 waves
    __shared__ T Sr[JRS][NC + 1], Si[JRS][NC + 1];
    __shared__ int cols[NC];
    const int pair = blockIdx.x;
    if (!rotflag[pair]) return;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const bool isW = (int)blockIdx.y < nchW;
    cx<T> *X = isW ? W : V;
    const int M = isW ? m : n;
    const int chunk = isW ? blockIdx.y : blockIdx.y - nchW;
    const int rpc = isW ? rpcW : rpcV;
    const int r_begin = chunk * rpc, r_end = min(M, r_begin + rpc);
    if (r_begin >= r_end) return;
    const int nc = pair_columns(pair, rnd, nb, w, n, cols, tid, 256);
    // Wave w's output tiles t = w + 4u all lie in column tile t % NT = w % NT
    // (NT divides 4), so each lane's MFMA B operands, J[4i + lane/16][bq] for
    // the NC/4 k-steps i, are the same for all its tiles: they are held in
    // registers (no LDS copy of J).
    static_assert(4 % NT == 0, "a wave's tiles share one column tile");
    const cx<T> *jin = Jin + (size_t)pair * NC * NC;
    T jr[NC / 4], ji[NC / 4];
    {
        const int bq = (wave % NT) * 16 + lane % 16;
#pragma unroll
        for (int i = 0; i < NC / 4; ++i) {
            const cx<T> v = jin[(size_t)(4 * i + lane / 16) * NC + bq];
            jr[i] = v.x;
            ji[i] = v.y;
        }
    }
    __syncthreads();  // cols[] is written by other waves in pair_columns
    // rows of the next step are loaded while this step's products run
    cx<T> sv[JRS * NC / 256];
    stage_load<T, NC>(X, M, cols, nc, r_begin, r_end, sv, tid);
    for (int r0 = r_begin; r0 < r_end; r0 += JRS) {
        __syncthreads();
        stage_store<T, NC>(sv, Sr, Si, tid);
        __syncthreads();
        if (r0 + JRS < r_end) stage_load<T, NC>(X, M, cols, nc, r0 + JRS, r_end, sv, tid);
        typename MF::acc re[TPW], im[TPW];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            re[u] = MF::zero();
            im[u] = MF::zero();
            const int ar_row = ((wave + 4 * u) / NT) * 16 + lane % 16;
#pragma unroll
            for (int i = 0; i < NC / 4; ++i) {
                const int kc = 4 * i + lane / 16;
                const T ar = Sr[ar_row][kc], ai = Si[ar_row][kc];
                re[u] = MF::op(ar, jr[i], re[u]);
                re[u] = MF::op(-ai, ji[i], re[u]);
                im[u] = MF::op(ar, ji[i], im[u]);
                im[u] = MF::op(ai, jr[i], im[u]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int t = wave + 4 * u;
            const int ti = t / NT, tj = t % NT;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = ti * 16 + MF::row(lane, v), cc = tj * 16 + lane % 16;
                Sr[rr][cc] = re[u][v];
                Si[rr][cc] = im[u][v];
            }
        }
        __syncthreads();
        for (int e = tid; e < JRS * NC; e += 256) {
            const int c = e / JRS, rr = e % JRS, row = r0 + rr;
            if (c < nc && row < r_end) X[(size_t)cols[c] * M + row] = mk<T>(Sr[rr][c], Si[rr][c]);
        }
    }
}

static int chunks_for(int rows, int npairs, int target) {
    int maxc = (rows + JRS - 1) / JRS;
    int c = (target + npairs - 1) / npairs;
    if (c > maxc) c = maxc;
    if (c < 1) c = 1;
    return c;
}
static int rows_per_chunk(int rows, int nch) {
    int steps = (rows + JRS - 1) / JRS;
    return JRS * ((steps + nch - 1) / nch);
}


template <typename T, int NC>
static void round_part(int part, void *W, int m, void *V, int n, int w, int nb, int rnd,
                       double tol, int inner_max, int inter, void *partial, void *J,
                       int *rotflag, int *rot_counter, int *stamp, int rot_threads, int wgs,
                       hipStream_t s) {
    const int npairs = nb / 2;
    const int nchG = chunks_for(m, npairs, wgs);
    const int rpcG = rows_per_chunk(m, nchG);
    const int nchG_eff = (m + rpcG - 1) / rpcG;
    if (part == 0) {
        k_jgram<T, NC><<<dim3(npairs, nchG_eff), 256, 0, s>>>((const cx<T> *)W, m, n, w, nb, rnd,
                                                            rpcG, (cx<T> *)partial, stamp);
    } else if (part == 1) {
#define EA_JEIG(NTH)                                                                          \
    do {                                                                                      \
        if (inter)                                                                            \
            k_jeig<T, NC, NTH, 1><<<npairs, NTH, 0, s>>>((const cx<T> *)partial, nchG_eff, n, \
                                                         w, nb, rnd, (T)tol, inner_max,       \
                                                         (cx<T> *)J, rotflag, rot_counter,    \
                                                         stamp);                              \
        else                                                                                  \
            k_jeig<T, NC, NTH, 0><<<npairs, NTH, 0, s>>>((const cx<T> *)partial, nchG_eff, n, \
                                                         w, nb, rnd, (T)tol, inner_max,       \
                                                         (cx<T> *)J, rotflag, rot_counter,    \
                                                         stamp);                              \
    } while (0)
        if (rot_threads <= 64) EA_JEIG(64);
        else if (rot_threads <= 128) EA_JEIG(128);
        else if (rot_threads <= 256) EA_JEIG(256);
        else if (rot_threads <= 512) EA_JEIG(512);
        else EA_JEIG(1024);
#undef EA_JEIG
    } else {
        const int nchW = chunks_for(m, npairs, wgs), rpcW = rows_per_chunk(m, nchW);
        const int nchV = chunks_for(n, npairs, 2 * wgs), rpcV = rows_per_chunk(n, nchV);
        const int nW = (m + rpcW - 1) / rpcW, nV = (n + rpcV - 1) / rpcV;
        k_japply<T, NC><<<dim3(npairs, nW + nV), 256, 0, s>>>((cx<T> *)W, m, (cx<T> *)V, n, w, nb,
                                                            rnd, nW, rpcW, rpcV,
                                                            (const cx<T> *)J, rotflag);
    }
}

// Workspace (in complex elements) needed by launch_jacobi_round3.
size_t jacobi_round3_partial_elems(int m, int n, int w, int wgs) {
    const int nc = 2 * w <= 32 ? 32 : 64;
    int nb = (n + w - 1) / w;
    nb += nb & 1;
    const int npairs = nb / 2;
    const int nchG = chunks_for(m, npairs, wgs);
    const int rpcG = rows_per_chunk(m, nchG);
    const int nchG_eff = (m + rpcG - 1) / rpcG;
    return (size_t)npairs * nchG_eff * nc * nc;
}
size_t jacobi_round3_j_elems(int n, int w) {
    const int nc = 2 * w <= 32 ? 32 : 64;
    int nb = (n + w - 1) / w;
    nb += nb & 1;
    return (size_t)(nb / 2) * nc * nc;
}

template <typename T>
void launch_jacobi_part(int part, void *W, int m, void *V, int n, int w, int nb, int rnd,
                        double tol, int inner_max, int inter, void *partial, void *J,
                        int *rotflag, int *rot_counter, int *stamp, int rot_threads, int wgs,
                        hipStream_t s) {
    if (2 * w <= 32)
        round_part<T, 32>(part, W, m, V, n, w, nb, rnd, tol, inner_max, inter, partial, J,
                          rotflag, rot_counter, stamp, rot_threads, wgs, s);
    else
        round_part<T, 64>(part, W, m, V, n, w, nb, rnd, tol, inner_max, inter, partial, J,
                          rotflag, rot_counter, stamp, rot_threads, wgs, s);
}

template void launch_jacobi_part<float>(int, void *, int, void *, int, int, int, int, double, int,
                                        int, void *, void *, int *, int *, int *, int, int,
                                        hipStream_t);
template void launch_jacobi_part<double>(int, void *, int, void *, int, int, int, int, double,
                                         int, int, void *, void *, int *, int *, int *, int, int,
                                         hipStream_t);
