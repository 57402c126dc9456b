// One-sided (Hestenes) block Jacobi SVD of a column-major matrix W (m x n,
// m >= n), accumulating the right rotations in V (n x n, column-major).
//
// A workgroup owns a set of nc <= NC columns (one block pair of the
// round-robin ordering, or all columns when n <= 64).  It forms their Gram
// matrix G = W_c^H W_c in LDS, diagonalises G by two-sided Jacobi rotations
// (each rotation is the one-sided rotation of the corresponding column pair
// expressed on the Gram matrix: the symmetric 2x2 Schur rotation of
// [[a, |g|], [|g|, b]] after removing the phase of g), accumulates them in J,
// and finally applies W_c <- W_c J and V_c <- V_c J.  The next Gram is
// formed from the rotated columns again, so the accuracy is that of
// one-sided Jacobi, not of an eigen-solve of a squared matrix.
// A pair (p, q) is rotated when |G_pq| > tol * sqrt(G_pp G_qq); the number of
// pairs rotated on the first inner sweep of a freshly formed Gram matrix is
// the convergence measure (0 over a full outer sweep = converged).
#include "ea_dev.h"
#include "ea_kernels.h"
#include "jacobi_body.h"

template <typename T, int NC>
__global__ __launch_bounds__(256) void k_jacobi_block(cx<T> *__restrict__ W, int m,
                                                      cx<T> *__restrict__ V, int n, int w,
                                                      int nb, int rnd, T tol, int inner_max,
                                                      int single, int max_outer,
                                                      int *__restrict__ rot_counter,
                                                      int *__restrict__ sweeps_out) {
    jacobi_block_body<T, NC>(W, m, V, n, w, nb, rnd, tol, inner_max, single, max_outer,
                             rot_counter, sweeps_out, blockIdx.x);
}

template <typename T>
void launch_jacobi_single(void *W, int m, void *V, int n, double tol, int inner_max,
                          int max_sweeps, int *sweeps_dev, hipStream_t s) {
    k_jacobi_block<T, 64><<<1, 256, 0, s>>>((cx<T> *)W, m, (cx<T> *)V, n, n, 1, 0, (T)tol,
                                            inner_max, 1, max_sweeps, nullptr, sweeps_dev);
}

template <typename T>
void launch_jacobi_round(void *W, int m, void *V, int n, int w, int nb, int rnd, double tol,
                         int inner_max, int ncmax, int *rot_counter, hipStream_t s) {
    const int grid = nb / 2;
    if (ncmax <= 16)
        k_jacobi_block<T, 16><<<grid, 256, 0, s>>>((cx<T> *)W, m, (cx<T> *)V, n, w, nb, rnd,
                                                   (T)tol, inner_max, 0, 1, rot_counter, nullptr);
    else if (ncmax <= 32)
        k_jacobi_block<T, 32><<<grid, 256, 0, s>>>((cx<T> *)W, m, (cx<T> *)V, n, w, nb, rnd,
                                                   (T)tol, inner_max, 0, 1, rot_counter, nullptr);
    else
        k_jacobi_block<T, 64><<<grid, 256, 0, s>>>((cx<T> *)W, m, (cx<T> *)V, n, w, nb, rnd,
                                                   (T)tol, inner_max, 0, 1, rot_counter, nullptr);
}

template void launch_jacobi_single<float>(void *, int, void *, int, double, int, int, int *,
                                          hipStream_t);
template void launch_jacobi_single<double>(void *, int, void *, int, double, int, int, int *,
                                           hipStream_t);
template void launch_jacobi_round<float>(void *, int, void *, int, int, int, int, double, int,
                                         int, int *, hipStream_t);
template void launch_jacobi_round<double>(void *, int, void *, int, int, int, int, double, int,
                                          int, int *, hipStream_t);
