// Body of the one-sided block Jacobi workgroup (see k_jacobi.hip); shared by
// the per-round kernel and by the device-resident small-bond layer kernel.
// `pair` selects the block pair of round `rnd` when single = 0.
#pragma once
#include "ea_dev.h"

template <typename T, int NC>
__device__ __forceinline__ void jacobi_block_body(cx<T> *__restrict__ W, int m,
                                                      cx<T> *__restrict__ V, int n, int w,
                                                      int nb, int rnd, T tol, int inner_max,
                                                      int single, int max_outer,
                                                      int *__restrict__ rot_counter,
                                                      int *__restrict__ sweeps_out, int pair) {
    constexpr int RC = (NC >= 64 && sizeof(T) == 8) ? 16 : 32;
    constexpr int NP = NC / 2;
    constexpr int EPT = (NC * NC + 255) / 256;  // Gram entries per thread
    __shared__ cx<T> G[NC][NC + 1];
    __shared__ cx<T> J[NC][NC + 1];
    __shared__ cx<T> S[RC][NC + 1];
    __shared__ T rs_[NP], rgm_[NP], rtg_[NP], ra_[NP], rb_[NP];
    __shared__ cx<T> re_[NP];
    __shared__ int rp_[NP], rq_[NP], rdo_[NP];
    __shared__ int cols[NC];
    __shared__ int nrot_sh;
    const int tid = threadIdx.x, nth = blockDim.x;

    int nc;
    if (single) {
        nc = n;
        for (int c = tid; c < n; c += nth) cols[c] = c;
    } else {
        const int a = rr_player(pair, rnd, nb), b = rr_player(nb - 1 - pair, rnd, nb);
        const int a0 = a * w, a1 = min(a0 + w, n), b0 = b * w, b1 = min(b0 + w, n);
        const int na = max(0, a1 - a0), nbb = max(0, b1 - b0);
        nc = na + nbb;
        for (int c = tid; c < na; c += nth) cols[c] = a0 + c;
        for (int c = tid; c < nbb; c += nth) cols[na + c] = b0 + c;
    }
    __syncthreads();
    if (nc < 2) {
        if (single && tid == 0) {
            sweeps_out[0] = 1;
            sweeps_out[1] = 1;
        }
        return;
    }
    const int nce = nc + (nc & 1);
    const int npairs = nce / 2;
    int outer = 0;
    int converged = 0;
    for (; outer < max_outer; ++outer) {
        // ---- Gram matrix of the owned columns ----
        cx<T> gacc[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) gacc[u] = zero_cx<T>();
        for (int r0 = 0; r0 < m; r0 += RC) {
            const int rows = min(RC, m - r0);
            for (int e = tid; e < rows * nc; e += nth) {
                const int c = e / rows, rr = e % rows;
                S[rr][c] = W[(size_t)cols[c] * m + r0 + rr];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int e = tid + u * 256;
                if (e < nc * nc) {
                    const int p = e / nc, q = e % nc;
                    cx<T> acc = gacc[u];
                    for (int rr = 0; rr < rows; ++rr) cmacc(acc, S[rr][p], S[rr][q]);
                    gacc[u] = acc;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + u * 256;
            if (e < nc * nc) {
                const int p = e / nc, q = e % nc;
                G[p][q] = gacc[u];
                J[p][q] = mk<T>(p == q ? T(1) : T(0), T(0));
            }
        }
        __syncthreads();

        // ---- two-sided Jacobi on G, accumulated in J ----
        int first = 0;
        for (int isw = 0; isw < inner_max; ++isw) {
            if (tid == 0) nrot_sh = 0;
            __syncthreads();
            for (int step = 0; step < nce - 1; ++step) {
                if (tid < npairs) {
                    int p = rr_player(tid, step, nce), q = rr_player(nce - 1 - tid, step, nce);
                    if (p > q) {
                        int t = p;
                        p = q;
                        q = t;
                    }
                    int dd = 0;
                    if (q < nc) {
                        const T al = G[p][p].x, be = G[q][q].x;
                        const cx<T> ga = G[p][q];
                        JRot<T> rt;
                        if (jacobi_rotation(al, be, ga, tol, rt)) {
                            rs_[tid] = rt.s;
                            rgm_[tid] = rt.gm;
                            re_[tid] = rt.e;
                            rtg_[tid] = rt.tg;
                            ra_[tid] = al;
                            rb_[tid] = be;
                            dd = 1;
                            atomicAdd(&nrot_sh, 1);
                        }
                    }
                    rp_[tid] = p;
                    rq_[tid] = q;
                    rdo_[tid] = dd;
                }
                __syncthreads();
                // columns: G <- G M, J <- J M, M = [[c, s], [-s e, c e]]
                for (int e = tid; e < npairs * nc; e += nth) {
                    const int pi = e / nc, row = e % nc;
                    if (rdo_[pi]) {
                        const int p = rp_[pi], q = rq_[pi];
                        const T s = rs_[pi], gm = rgm_[pi];
                        const cx<T> ee = re_[pi];
                        rot_pair(G[row][p], ee * G[row][q], s, gm, G[row][p], G[row][q]);
                        rot_pair(J[row][p], ee * J[row][q], s, gm, J[row][p], J[row][q]);
                    }
                }
                __syncthreads();
                // rows: G <- M^H G
                for (int e = tid; e < npairs * nc; e += nth) {
                    const int pi = e / nc, col = e % nc;
                    if (rdo_[pi]) {
                        const int p = rp_[pi], q = rq_[pi];
                        const cx<T> ec = conj(re_[pi]);
                        rot_pair(G[p][col], ec * G[q][col], rs_[pi], rgm_[pi], G[p][col],
                                 G[q][col]);
                    }
                }
                __syncthreads();
                if (tid < npairs && rdo_[tid]) {
                    const int p = rp_[tid], q = rq_[tid];
                    G[p][q] = zero_cx<T>();
                    G[q][p] = zero_cx<T>();
                    G[p][p] = mk<T>(ra_[tid] - rtg_[tid], T(0));
                    G[q][q] = mk<T>(rb_[tid] + rtg_[tid], T(0));
                }
                __syncthreads();
            }
            const int nr = nrot_sh;
            __syncthreads();
            if (isw == 0) first = nr;
            if (nr == 0) break;
        }
        if (!single && tid == 0 && first > 0) atomicAdd(rot_counter, first);
        if (first == 0) {
            converged = 1;
            break;
        }

        // ---- apply J to the owned columns of W and V ----
        for (int pass = 0; pass < 2; ++pass) {
            cx<T> *X = pass == 0 ? W : V;
            const int M = pass == 0 ? m : n;
            for (int r0 = 0; r0 < M; r0 += RC) {
                const int rows = min(RC, M - r0);
                for (int e = tid; e < rows * nc; e += nth) {
                    const int c = e / rows, rr = e % rows;
                    S[rr][c] = X[(size_t)cols[c] * M + r0 + rr];
                }
                __syncthreads();
                for (int e = tid; e < rows * nc; e += nth) {
                    const int q = e / rows, rr = e % rows;
                    cx<T> acc = zero_cx<T>();
                    for (int c = 0; c < nc; ++c) cmac(acc, S[rr][c], J[c][q]);
                    X[(size_t)cols[q] * M + r0 + rr] = acc;
                }
                __syncthreads();
            }
        }
    }
    if (single && tid == 0) {
        sweeps_out[0] = converged ? outer + 1 : outer;
        sweeps_out[1] = converged;
    }
}

