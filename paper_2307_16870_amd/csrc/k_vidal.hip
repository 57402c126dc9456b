// Pieces of the two-site update in the layer-parallel gauge (Vidal form with
// Hastings' division-free update): the bond values Lambda_i scale the rows of
// the contracted block before its SVD, and the kept, renormalised singular
// values become the new bond's Lambda.
#include "ea_dev.h"
#include "ea_kernels.h"

// W (rows x cols, column-major) holds Theta (orient 0: rows = d chi_l) or
// Theta^H (orient 1: cols = d chi_l).  Row (l, s) of Theta is scaled by lam[l].
template <typename T>
__global__ void k_scale_lambda(cx<T> *__restrict__ W, int rows, int cols, int orient,
                               const double *__restrict__ lam, int d) {
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)rows * cols) return;
    const int c = (int)(idx / rows), r = (int)(idx % rows);
    const T a = (T)lam[(orient == 0 ? r : c) / d];
    W[idx] = a * W[idx];
}
template <typename T>
void launch_scale_lambda(void *W, int rows, int cols, int orient, const double *lam, int d,
                         hipStream_t s) {
    const size_t n = (size_t)rows * cols;
    if (n == 0) return;
    k_scale_lambda<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((cx<T> *)W, rows, cols, orient,
                                                                  lam, d);
}

// lam_out[j] = s_sorted[j] * scale (j < k): the kept values renormalised.
__global__ void k_vidal_lambda(const double *__restrict__ s_sorted,
                               const ea_dev_rec *__restrict__ rec, int k,
                               double *__restrict__ lam_out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < k) lam_out[j] = s_sorted[j] * rec->scale;
}
void launch_vidal_lambda(const double *s_sorted, const ea_dev_rec *rec, int k, double *lam_out,
                         hipStream_t s) {
    if (k > 0) k_vidal_lambda<<<(k + 255) / 256, 256, 0, s>>>(s_sorted, rec, k, lam_out);
}

template void launch_scale_lambda<float>(void *, int, int, int, const double *, int, hipStream_t);
template void launch_scale_lambda<double>(void *, int, int, int, const double *, int, hipStream_t);
