// Device-resident two-site updates for small bonds (Sec. V-VI).  Every size
// is read from device memory, so one launch advances one circuit layer of
// many independent states: one workgroup per state walks the layer's gates in
// the order the host path uses (ascending if the orthogonality centre is
// nearer the lowest gate, else descending), moving the centre site by site
// with exact factorisations (Sec. III) and applying each update: contraction
// with the gate, one-sided Jacobi SVD, kept-rank rule in FP64, write-back,
// running fidelity estimate (Eq. 12) and the target schedule (Eq. 14).
// Valid while every matrix of the layer has at most SM_N^2 entries and every
// factorisation at most SM_N columns, which holds for a whole layer when every
// bond is at most SM_N / d when the layer starts (the host checks this).
// Factorisations with more than 64 columns run the block round-robin Jacobi
// (pairs of 32-column blocks) inside the workgroup.
#include "ea_dev.h"
#include "ea_kernels.h"
#include "jacobi_body.h"

#include <math.h>

namespace {

constexpr int NTH = 256;

struct Dec {  // one factorisation's decision
    int k, k_f, k_nz, capped, sweeps, converged, r;
    double total, disc, f, lnf, kept2, scale, s0;
};

template <typename T>
struct Work {
    cx<T> *W, *V, *X, *P;  // factor, right factor, gathered factor, products
    double *G64;           // re-orthogonalisation Gram (FP64, complex)
    cx<T> *Y, *R;          // re-orthogonalisation factors
};

template <typename T>
__device__ Work<T> work_of(const SmallDesc<T> &D) {
    Work<T> w;
    cx<T> *b = D.scratch;
    w.W = b;
    w.V = b + SM_ELEMS;
    w.X = w.V + SM_ELEMS;
    w.P = w.X + SM_ELEMS;
    w.Y = w.P + SM_ELEMS;
    w.R = w.Y + SM_ELEMS;
    w.G64 = reinterpret_cast<double *>(w.R + SM_ELEMS);
    return w;
}

__device__ double schedule_target_dev(int has_sched, int strategy, double f_min, long long n_total,
                                      long long g, double lnP) {
    if (!has_sched) return 1.0;
    const double n = (double)n_total, gg = (double)g;
    double ft;
    if (strategy == EA_NAIVE) {
        ft = pow(f_min, 1.0 / n);
    } else if (strategy == EA_GLOBAL) {
        const double left = n - gg;
        ft = left <= 0 ? 1.0 : exp((log(f_min) - lnP) / left);
    } else if (strategy == EA_NEAREST) {
        ft = exp(log(f_min) * (gg + 1) / n - lnP);
    } else {  // EA_FIXED: only the chi_max cap truncates
        ft = 1.0;
    }
    return fmin(1.0, fmax(ft, 1e-300));
}

// SVD of W (m x n column-major, m >= n) by the single-workgroup Jacobi, then
// s_j = ||w_j|| in FP64, order by decreasing s (ties by index), suffix sums
// D(k) from the smallest value up, and the kept rank: mode 0 the update rule
// k = min(k_f, k_nz, chi_max), mode 1 (centre move) k = k_nz.
template <typename T>
__device__ __noinline__ void factor(const SmallDesc<T> &D, const Work<T> &w, int m, int n, int mode,
                       double f_t, Dec &dec, double *s_raw, double *s_sorted, int *perm,
                       double *Dsuf, double *part, int *sw, int *cnt) {
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += NTH) {
        const int c = e / n, r = e % n;
        w.V[e] = mk<T>(r == c ? T(1) : T(0), T(0));
    }
    __syncthreads();
    const double tol = D.tol_user > 0 ? D.tol_user
                                      : (double)m * (sizeof(T) == 8 ? 0x1p-53 : 0x1p-24);
    if (n <= 64) {  // all columns in one Gram matrix
        jacobi_block_body<T, 64>(w.W, m, w.V, n, n, 1, 0, (T)tol, D.inner, 1, D.max_sweeps,
                                 nullptr, sw, 0);
    } else {  // blocks of 32 columns, round-robin over block pairs
        const int bw = 32;
        int nb = (n + bw - 1) / bw;
        nb += nb & 1;
        int sweeps = 0, conv = 0;
        for (int s = 0; s < D.max_sweeps; ++s) {
            if (tid == 0) cnt[0] = 0;
            __syncthreads();
            for (int rnd = 0; rnd < nb - 1; ++rnd)
                for (int pr = 0; pr < nb / 2; ++pr) {
                    jacobi_block_body<T, 64>(w.W, m, w.V, n, bw, nb, rnd, (T)tol, D.inner, 0, 1,
                                             cnt, nullptr, pr);
                    __syncthreads();
                }
            ++sweeps;
            const int c = cnt[0];
            __syncthreads();
            if (c == 0) {
                conv = 1;
                break;
            }
        }
        if (tid == 0) {
            sw[0] = sweeps;
            sw[1] = conv;
        }
    }
    __syncthreads();
    {  // tpc threads per column
        const int tpc = n <= 64 ? 4 : 2;
        const int j = tid / tpc, q = tid % tpc;
        double a = 0.0;
        if (j < n)
            for (int i = q; i < m; i += tpc) {
                const cx<T> v = w.W[(size_t)j * m + i];
                a += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            }
        part[tid] = a;
    }
    __syncthreads();
    if (tid < n) {
        const int tpc = n <= 64 ? 4 : 2;
        double a = 0.0;
        for (int u = 0; u < tpc; ++u) a += part[tpc * tid + u];
        s_raw[tid] = sqrt(a);
    }
    __syncthreads();
    if (tid < n) {
        const double sj = s_raw[tid];
        int r = 0;
        for (int i = 0; i < n; ++i) {
            const double si = s_raw[i];
            r += (si > sj) || (si == sj && i < tid);
        }
        perm[r] = tid;
        s_sorted[r] = sj;
    }
    __syncthreads();
    if (tid == 0) {
        const int r = n;
        Dsuf[r] = 0.0;
        for (int i = r - 1; i >= 0; --i) Dsuf[i] = Dsuf[i + 1] + s_sorted[i] * s_sorted[i];
        const double T0 = Dsuf[0], s0 = r > 0 ? s_sorted[0] : 0.0;
        const double thr = (1.0 - f_t) * T0;
        int k_f = r;
        for (int k = 1; k <= r; ++k)
            if (Dsuf[k] <= thr) {
                k_f = k;
                break;
            }
        int k_nz = 0;
        for (int i = 0; i < r; ++i) k_nz += s_sorted[i] > D.tau * s0;
        if (k_nz < 1) k_nz = 1;
        if (k_nz > r) k_nz = r;
        int k, capped = 0;
        if (mode == 1) {
            k = k_nz;
        } else {
            k = k_f < k_nz ? k_f : k_nz;
            if (D.chi_max > 0 && D.chi_max < k) {
                k = D.chi_max;
                capped = 1;
            }
        }
        const double disc = Dsuf[k], kept2 = T0 - disc;
        dec.k = k;
        dec.k_f = k_f;
        dec.k_nz = k_nz;
        dec.capped = capped;
        dec.sweeps = sw[0];
        dec.converged = sw[1];
        dec.r = r;
        dec.total = T0;
        dec.disc = disc;
        dec.f = T0 > 0 ? 1.0 - disc / T0 : 1.0;
        dec.lnf = T0 > 0 ? log1p(-disc / T0) : 0.0;
        dec.kept2 = kept2;
        dec.scale = (mode == 1 || kept2 <= 0.0) ? 1.0 : 1.0 / sqrt(kept2);
        dec.s0 = (s0 > 0.0 && isfinite(T0)) ? s0 : 0.0;
    }
    __syncthreads();
}

// out_j = a_j (conj) src[perm[j]] for the k kept columns of src (leading
// dimension ld); a_j = s_j (es = 1), 1/s_j (es = -1) or 1, times the update's
// renormalisation when ec.  Rows: out[j X + x]; transposed: out[x k + j].
template <typename T>
__device__ void gather(const cx<T> *src, int ld, const int *perm, const double *s_sorted,
                       const Dec &dec, int k, int X, int conj_src, int es, int ec, int transposed,
                       cx<T> *out) {
    for (int e = threadIdx.x; e < k * X; e += NTH) {
        const int j = e / X, x = e % X;
        double a = 1.0;
        if (es == 1) a *= s_sorted[j];
        if (es == -1) a /= s_sorted[j];
        if (ec) a *= dec.scale;
        cx<T> v = src[(size_t)perm[j] * ld + x];
        if (conj_src) v = conj(v);
        const cx<T> o = (T)a * v;
        if (transposed)
            out[(size_t)x * k + j] = o;
        else
            out[(size_t)j * X + x] = o;
    }
}

// C = A B, row-major (M x K)(K x N); then C is copied to `dst` (M x N).
template <typename T>
__device__ void gemm_copy(const cx<T> *A, const cx<T> *B, cx<T> *Ptmp, cx<T> *dst, int M, int N,
                          int K) {
    for (int e = threadIdx.x; e < M * N; e += NTH) {
        const int i = e / N, j = e % N;
        cx<T> acc = zero_cx<T>();
        for (int t = 0; t < K; ++t) cmac(acc, A[(size_t)i * K + t], B[(size_t)t * N + j]);
        Ptmp[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M * N; e += NTH) dst[e] = Ptmp[e];
    __syncthreads();
}

// FP64 re-orthogonalisation of an FP32 isometric factor (one Loewdin step).
// cols: X (rows x k) should have orthonormal columns, N (k x nother) absorbs
// (I + E/2) from the left; else X (k x rows) orthonormal rows, N (nother x k)
// absorbs it from the right.  G = X^H X (or X X^H) = I + E in FP64.
template <typename T>
__device__ void reorth(const Work<T> &w, bool cols, cx<T> *X, int rows, int k, cx<T> *N,
                       int nother) {
    for (int e = threadIdx.x; e < k * k; e += NTH) {
        const int a = e / k, b = e % k;
        double gr = 0.0, gi = 0.0;
        for (int r = 0; r < rows; ++r) {
            cx<T> xa, xb;
            if (cols) {
                xa = X[(size_t)r * k + a];
                xb = X[(size_t)r * k + b];
            } else {  // (X X^H)_ab = sum_r X[a][r] conj(X[b][r]) = conj(sum conj(X[a][r]) X[b][r])
                xa = conj(X[(size_t)b * rows + r]);
                xb = conj(X[(size_t)a * rows + r]);
            }
            const double ar = xa.x, ai = xa.y, br = xb.x, bi = xb.y;
            gr += ar * br + ai * bi;
            gi += ar * bi - ai * br;
        }
        const double d = a == b ? 1.0 : 0.0;
        w.G64[2 * e] = gr - d;
        w.G64[2 * e + 1] = gi;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += NTH) {
        const int a = e / k, b = e % k;
        const double d = a == b ? 1.0 : 0.0;
        const double er = w.G64[2 * e], ei = w.G64[2 * e + 1];
        w.Y[e] = mk<T>((T)(d - 0.5 * er), (T)(-0.5 * ei));
        w.R[e] = mk<T>((T)(d + 0.5 * er), (T)(0.5 * ei));
    }
    __syncthreads();
    if (cols) {
        gemm_copy<T>(X, w.Y, w.P, X, rows, k, k);
        gemm_copy<T>(w.R, N, w.P, N, k, nother, k);
    } else {
        gemm_copy<T>(w.Y, X, w.P, X, k, rows, k);
        gemm_copy<T>(N, w.R, w.P, N, nother, k, k);
    }
}

template <typename T>
__global__ __launch_bounds__(NTH) void k_layer_small(SmallDesc<T> *descs) {
    SmallDesc<T> &D = descs[blockIdx.x];
    const Work<T> w = work_of(D);
    __shared__ Dec dec;
    __shared__ double s_raw[SM_N], s_sorted[SM_N], Dsuf[SM_N + 1], part[NTH];
    __shared__ int perm[SM_N], order[SM_GATES], sw[2], cnt[1];
    __shared__ int center_sh, big_sh;
    const int tid = threadIdx.x, d = D.d;
    int *bond = D.bond;
    cx<T> *const *site = D.site;
    if (tid == 0) center_sh = D.center;
    __syncthreads();
    for (int L = 0; L < D.n_layers; ++L) {
        // a later layer runs here only while every bond is within the limit
        if (tid == 0) big_sh = 0;
        __syncthreads();
        for (int x = tid; x <= D.n; x += NTH)
            if (bond[x] > D.lim) big_sh = 1;
        __syncthreads();
        if (big_sh) break;
        const int g0 = D.layer_off[L], ng = D.layer_off[L + 1] - g0;
        if (tid == 0) {
            int lo = D.n, hi = -1;
            for (int j = 0; j < ng; ++j) {
                lo = min(lo, D.gsite[g0 + j]);
                hi = max(hi, D.gsite[g0 + j]);
                order[j] = g0 + j;
            }
            const bool asc = abs(center_sh - lo) <= abs(center_sh - hi);
            for (int a = 1; a < ng; ++a) {  // insertion sort by site
                const int v = order[a];
                int b = a - 1;
                while (b >= 0 &&
                       (asc ? D.gsite[order[b]] > D.gsite[v] : D.gsite[order[b]] < D.gsite[v])) {
                    order[b + 1] = order[b];
                    --b;
                }
                order[b + 1] = v;
            }
            D.asc = asc ? 1 : 0;
        }
        __syncthreads();
        const int asc = D.asc;
        for (int gi = 0; gi < ng; ++gi) {
            const int j = order[gi], i = D.gsite[j];
            // ---- centre moves (Sec. III) ----
            while (true) {
                const int c = center_sh;
                const int dir = c < i ? 1 : (c > i + 1 ? -1 : 0);
                if (dir == 0) break;
                if (dir > 0) {  // A_c = U (S V^H): A_c <- U, A_{c+1} <- (S V^H) A_{c+1}
                    const int M = bond[c] * d, N = bond[c + 1];
                    const int orient = M >= N ? 0 : 1, mw = max(M, N), nw = min(M, N);
                    for (int e = tid; e < M * N; e += NTH) {
                        const int r = e / N, cc = e % N;
                        const cx<T> v = site[c][e];
                        if (orient == 0) w.W[(size_t)cc * M + r] = v;
                        else w.W[e] = conj(v);
                    }
                    __syncthreads();
                    factor<T>(D, w, mw, nw, 1, 1.0, dec, s_raw, s_sorted, perm, Dsuf, part, sw, cnt);
                    if (!(dec.s0 > 0.0)) {
                        if (tid == 0) {
                            D.status = EA_EINVAL;
                            D.center = center_sh;
                        }
                        return;
                    }
                    const int k = dec.k, chi2 = bond[c + 2];
                    if (orient == 0) {
                        gather<T>(w.W, M, perm, s_sorted, dec, k, M, 0, -1, 0, 1, site[c]);
                        gather<T>(w.V, N, perm, s_sorted, dec, k, N, 1, 1, 0, 0, w.X);
                    } else {
                        gather<T>(w.V, M, perm, s_sorted, dec, k, M, 0, 0, 0, 1, site[c]);
                        gather<T>(w.W, N, perm, s_sorted, dec, k, N, 1, 0, 0, 0, w.X);
                    }
                    __syncthreads();
                    gemm_copy<T>(w.X, site[c + 1], w.P, site[c + 1], k, d * chi2, N);
                    if constexpr (sizeof(T) == 4)
                        if (D.reorth) reorth<T>(w, true, site[c], M, k, site[c + 1], d * chi2);
                    if (tid == 0) {
                        bond[c + 1] = k;
                        center_sh = c + 1;
                    }
                } else {  // A_c = (U S) V^H: A_c <- V^H, A_{c-1} <- A_{c-1} (U S)
                    const int M = bond[c], N = d * bond[c + 1];
                    const int orient = M >= N ? 0 : 1, mw = max(M, N), nw = min(M, N);
                    for (int e = tid; e < M * N; e += NTH) {
                        const int r = e / N, cc = e % N;
                        const cx<T> v = site[c][e];
                        if (orient == 0) w.W[(size_t)cc * M + r] = v;
                        else w.W[e] = conj(v);
                    }
                    __syncthreads();
                    factor<T>(D, w, mw, nw, 1, 1.0, dec, s_raw, s_sorted, perm, Dsuf, part, sw, cnt);
                    if (!(dec.s0 > 0.0)) {
                        if (tid == 0) {
                            D.status = EA_EINVAL;
                            D.center = center_sh;
                        }
                        return;
                    }
                    const int k = dec.k, rowsP = bond[c - 1] * d;
                    if (orient == 0) {
                        gather<T>(w.V, N, perm, s_sorted, dec, k, N, 1, 0, 0, 0, site[c]);
                        gather<T>(w.W, M, perm, s_sorted, dec, k, M, 0, 0, 0, 1, w.X);
                    } else {
                        gather<T>(w.W, N, perm, s_sorted, dec, k, N, 1, -1, 0, 0, site[c]);
                        gather<T>(w.V, M, perm, s_sorted, dec, k, M, 0, 1, 0, 1, w.X);
                    }
                    __syncthreads();
                    gemm_copy<T>(site[c - 1], w.X, w.P, site[c - 1], rowsP, k, M);
                    if constexpr (sizeof(T) == 4)
                        if (D.reorth) reorth<T>(w, false, site[c], N, k, site[c - 1], rowsP);
                    if (tid == 0) {
                        bond[c] = k;
                        center_sh = c - 1;
                    }
                }
                __syncthreads();
            }
            // ---- two-site update (Sec. V-VI) ----
            const double b = D.budget ? D.budget[j] : -1.0;
            double f_t = b >= 0 ? b : schedule_target_dev(D.has_sched, D.strategy, D.f_min, D.n_total, D.g, D.lnP);
            f_t = fmin(1.0, fmax(f_t, 1e-300));
            const int chiL = bond[i], chiM = bond[i + 1], chiR = bond[i + 2];
            const int M = d * chiL, N = d * chiR;
            const int orient = M >= N ? 0 : 1, mw = max(M, N), nw = min(M, N);
            const cx<T> *G = D.gmat + (size_t)j * d * d * d * d;
            // C[(l,t1),(t2,r)] = sum_m A_i[l,t1,m] A_{i+1}[m,t2,r] into P, then the gate
            for (int e = tid; e < M * N; e += NTH) {
                const int row = e / N, col = e % N;
                const int l = row / d, t1 = row % d, t2 = col / chiR, r = col % chiR;
                cx<T> acc = zero_cx<T>();
                const cx<T> *a = site[i] + ((size_t)l * d + t1) * chiM;
                const cx<T> *bb = site[i + 1] + (size_t)t2 * chiR + r;
                for (int mm = 0; mm < chiM; ++mm) cmac(acc, a[mm], bb[(size_t)mm * d * chiR]);
                w.P[e] = acc;
            }
            __syncthreads();
            for (int e = tid; e < M * N; e += NTH) {
                const int row = e / N, col = e % N;
                const int l = row / d, s1 = row % d, s2 = col / chiR, r = col % chiR;
                cx<T> th = zero_cx<T>();
                for (int t1 = 0; t1 < d; ++t1)
                    for (int t2 = 0; t2 < d; ++t2)
                        cmac(th, G[(s1 * d + s2) * d * d + t1 * d + t2],
                             w.P[((size_t)l * d + t1) * N + (size_t)t2 * chiR + r]);
                if (orient == 0)
                    w.W[(size_t)col * M + row] = th;
                else
                    w.W[(size_t)row * N + col] = conj(th);
            }
            __syncthreads();
            factor<T>(D, w, mw, nw, 0, f_t, dec, s_raw, s_sorted, perm, Dsuf, part, sw, cnt);
            if (!(dec.s0 > 0.0) || !isfinite(dec.total)) {
                if (tid == 0) {
                    D.status = EA_EINVAL;
                    D.center = center_sh;
                }
                return;
            }
            const int k = dec.k;
            const bool right = asc != 0;
            if (orient == 0) {
                gather<T>(w.W, M, perm, s_sorted, dec, k, M, 0, right ? -1 : 0, right ? 0 : 1, 1, site[i]);
                gather<T>(w.V, N, perm, s_sorted, dec, k, N, 1, right ? 1 : 0, right ? 1 : 0, 0, site[i + 1]);
            } else {
                gather<T>(w.V, M, perm, s_sorted, dec, k, M, 0, right ? 0 : 1, right ? 0 : 1, 1, site[i]);
                gather<T>(w.W, N, perm, s_sorted, dec, k, N, 1, right ? 0 : -1, right ? 1 : 0, 0, site[i + 1]);
            }
            __syncthreads();
            if constexpr (sizeof(T) == 4) {
                if (D.reorth) {
                    if (right)
                        reorth<T>(w, true, site[i], M, k, site[i + 1], N);
                    else
                        reorth<T>(w, false, site[i + 1], N, k, site[i], M);
                }
            }
            if (tid == 0) {
                bond[i + 1] = k;
                center_sh = right ? i + 1 : i;
                D.lnP += dec.lnf;
                if (D.kind == EA_MIXED && dec.kept2 > 0) D.lnS += 0.5 * log(dec.kept2);
                ea_gate_record &r = D.log[D.n_done];
                r.gate = D.g;
                r.site = i;
                r.chi_l = chiL;
                r.chi_m = chiM;
                r.chi_r = chiR;
                r.k = k;
                r.k_f = dec.k_f;
                r.sweeps = dec.sweeps;
                r.capped = dec.capped;
                r.subspace = 0;
                r.attempts = 0;
                r.f_t = f_t;
                r.f = dec.f;
                r.total = dec.total;
                r.lnP = D.lnP;
                r.lnS = D.lnS;
                D.g += 1;
                if (D.fout) D.fout[j] = dec.f;
                D.n_capped += dec.capped;
                D.n_noconv += dec.converged ? 0 : 1;
                D.n_done += 1;
            }
            __syncthreads();
        }

        if (tid == 0) D.layers_done = L + 1;
        __syncthreads();
    }
    if (tid == 0) D.center = center_sh;
}

}  // namespace

template <typename T>
void launch_layer_small(SmallDesc<T> *descs, int n_states, hipStream_t s) {
    if (n_states > 0) k_layer_small<T><<<n_states, NTH, 0, s>>>(descs);
}
template void launch_layer_small<float>(SmallDesc<float> *, int, hipStream_t);
template void launch_layer_small<double>(SmallDesc<double> *, int, hipStream_t);
