// Host-visible launchers of the HIP kernels (one instantiation per precision).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "ea_dev.h"
#include "ea_mps.h"

// Result of one truncation decision, written by the device, read by the host.
struct ea_dev_rec {
    int k;        // kept rank
    int k_f;      // rank asked for by the target alone
    int k_nz;     // number of singular values above tau * s_0
    int capped;   // chi_max bound
    int sweeps;   // Jacobi sweeps (Gram evaluations) used
    int converged;
    int r;        // number of singular values
    int pad;
    double total;    // T = sum s^2
    double disc;     // D(k) = sum_{j>=k} s_j^2
    double f;        // 1 - D(k)/T
    double lnf;      // log1p(-D(k)/T)
    double kept2;    // T - D(k)
    double scale;    // 1/sqrt(kept2) for an update, 1 for a centre move
    double s0;       // largest singular value
    double pad2;
};

// Largest number of singular values the single-workgroup sort handles.
constexpr int EA_SORT_MAX = 4096;

// ---- contraction / small dense kernels (T = float or double) -------------
// Theta[(l,s1),(s2,r)] = sum G[(s1 s2),(t1 t2)] sum_m A[l,t1,m] B[m,t2,r].
// orient 0: W column-major (dchiL x dchiR), W[col*dchiL+row] = Theta.
// orient 1: W = Theta^H column-major, W[row*dchiR+col] = conj(Theta).
template <typename T>
void launch_theta(const void *A, const void *B, const void *G, void *W, int chiL, int chiM,
                  int chiR, int d, int orient, hipStream_t s);
// FP32 operands split into bf16 hi/lo parts on the bf16 matrix cores
// (three products per real product, FP32 accumulation); same layout and
// The contraction on the FP32 / FP64 16x16x4 matrix cores (same layout and
// epilogue as launch_theta).
template <typename T>
void launch_theta_mfma(const void *A, const void *B, const void *G, void *W, int chiL, int chiM,
                       int chiR, int d, int orient, hipStream_t s);
// epilogue as launch_theta<float>.
void launch_theta_bf16x3(const void *A, const void *B, const void *G, void *W, int chiL,
                         int chiM, int chiR, int d, int orient, hipStream_t s);
// C (M x N) = alpha op(A) op(B) + beta C on the matrix cores (k_zgemm.hip),
// row-major with leading dimensions; op 0: as stored (A is M x K), 1:
// conjugate transpose (A stored K x M), 2: transpose (A stored K x M), 3:
// conjugate (A stored M x K).
template <typename T>
void launch_zgemm(int opA, int opB, int M, int N, int K, double ar, double ai, const void *A,
                  int lda, const void *B, int ldb, double br, double bi, void *C, int ldc,
                  hipStream_t s);
// Cholesky of a Hermitian positive definite complex FP64 matrix (k_chol.hip):
// G (n x n, row-major, overwritten) = R^H R, R upper triangular, and
// Rinv = R^{-1}; T1 is scratch of n x n complex; dmax receives the
// largest diagonal entry of G.  A pivot at or below rel_min * dmax sets *flag
// (which is not cleared) and is replaced by that bound.
constexpr int CHOL_NB = 32;
void launch_cholesky_inv(void *G, void *R, void *Rinv, void *T1, int n, double *dmax,
                         double rel_min, int *flag, hipStream_t s);
// ||G - I||_F^2 of an n x n complex FP64 matrix into *out (device); part is
// scratch of (n + 3) / 4 doubles.
void launch_offident_fro2(const void *G, int n, double *part, double *out, hipStream_t s);
// The same for `batch` independent products, entry b taking its operands at
// A + b sA, B + b sB, C + b sC (complex elements).
template <typename T>
void launch_zgemm_batched(int opA, int opB, int M, int N, int K, double ar, double ai,
                          const void *A, int lda, size_t sA, const void *B, int ldb, size_t sB,
                          double br, double bi, void *C, int ldc, size_t sC, int batch,
                          hipStream_t s);
// Layer-parallel gauge (k_vidal.hip): scale row (l, s) of Theta by lam[l],
// W holding Theta (orient 0, rows = d chi_l) or Theta^H (orient 1) column-major;
// lam_out[j] = s_sorted[j] * rec->scale for j < k.
template <typename T>
void launch_scale_lambda(void *W, int rows, int cols, int orient, const double *lam, int d,
                         hipStream_t s);
void launch_vidal_lambda(const double *s_sorted, const ea_dev_rec *rec, int k, double *lam_out,
                         hipStream_t s);
// C (M x N) = A (M x K) * B (K x N), row-major with leading dimensions.
template <typename T>
void launch_gemm(const void *A, const void *B, void *C, int M, int N, int K, int lda, int ldb,
                 int ldc, hipStream_t s);
// out[l,s,r] = sum_t g[s,t] in[l,t,r]  (in == out allowed).
template <typename T>
void launch_apply1(const void *in, void *out, const void *g, int chiL, int d, int chiR,
                   hipStream_t s);
// V = identity (n x n).
template <typename T>
void launch_eye(void *V, int n, hipStream_t s);
// out (column-major M x N) = in (row-major M x N), optionally conjugated
// elementwise without transposition (conj_copy = 1: out[i] = conj(in[i])).
template <typename T>
void launch_to_colmajor(const void *in, void *out, int M, int N, int conj_copy, hipStream_t s);
// s_out[j] = || column j || (FP64 accumulation), column-major m x n.
template <typename T>
void launch_colnorms(const void *W, int m, int n, double *s_out, hipStream_t s);
// Divides column j of V (n x n) and W (m x n), column-major, by |V_j| (FP64).
template <typename T>
void launch_unit_right(void *W, int m, void *V, int n, hipStream_t s);
// Write-back gather: for j < k, alpha_j = s_j^es * scale^ec;
//   rows_out:  out[j*X + x] = alpha_j * op(src[perm[j]*ld + x])
//   transposed: out[x*k + j] = alpha_j * op(src[perm[j]*ld + x])
template <typename T>
void launch_gather(const void *src, int ld, const int *perm, const double *s_sorted,
                   const ea_dev_rec *rec, int k, int X, int conj_src, int es, int ec,
                   int transposed, void *out, hipStream_t s);
// Convert T -> double complex.
template <typename T>
void launch_to_c128(const void *in, double *out, size_t n, hipStream_t s);
template <typename T>
void launch_from_c128(const double *in, void *out, size_t n, hipStream_t s);
// Fill n ints with a value (graph-capturable replacement of a memset).
void launch_fill_int(int *p, int n, int v, hipStream_t s);

// ---- truncation -----------------------------------------------------------
// mode 0: truncation rule of the two-site update; mode 1: centre move (keep
// all numerically non-zero values, no renormalisation).  forced_k > 0 forces
// the kept rank.  chi_max <= 0: no cap.  resid (device, may be null): a
// weight outside the r values (a partial factorisation) added to every
// discarded weight and to T; k_f = r + 1 when no k <= r meets the target.
void launch_sort_trunc(const double *s_raw, int r, double f_t, int chi_max, double tau,
                       int mode, int forced_k, const int *sweeps_dev, int *perm,
                       double *s_sorted, ea_dev_rec *rec, hipStream_t s,
                       const double *resid = nullptr);

// ---- partial (top-k) factorisation ------------------------------------------
// out[e] (n complex FP64) = (2u(base + 2e) - 1) + i (2u(base + 2e + 1) - 1),
// u(x) the top 53 bits of SplitMix64(seed) at counter x times 2^-53.
void launch_omega(unsigned long long seed, unsigned long long base, size_t n, double *out,
                  hipStream_t s);
// out[0] = sum of |x|^2 over n complex FP64 values (part: sumsq_part_doubles()
// doubles of scratch); the same bits on every run.
size_t sumsq_part_doubles();
void launch_sumsq(const double *x, size_t n, double *part, double *out, hipStream_t s);
// out[0] = max(0, a[0] - b[0]) on the device.
void launch_resid(const double *a, const double *b, double *out, hipStream_t s);
// G (n x n complex FP64): G_ii += rel * trace(G).
void launch_shift_diag(void *G, int n, double rel, hipStream_t s);

// ---- one-sided block Jacobi ----------------------------------------------
// Single-workgroup form for n <= 64 columns: iterates to convergence.
// sweeps_dev[0] = Gram evaluations, sweeps_dev[1] = converged flag.
template <typename T>
void launch_jacobi_single(void *W, int m, void *V, int n, double tol, int inner_max,
                          int max_sweeps, int *sweeps_dev, hipStream_t s);
// One round of the block round-robin ordering: nb blocks of width w,
// nb/2 workgroups; adds the number of rotated pairs to *rot_counter.
// ncmax selects the instantiation (2w <= ncmax).
template <typename T>
void launch_jacobi_round(void *W, int m, void *V, int n, int w, int nb, int rnd, double tol,
                         int inner_max, int ncmax, int *rot_counter, hipStream_t s);

// ---- observables ----------------------------------------------------------
// partial[blk] = (sum conj(a) b, sum |a|^2) over len elements; then
// launch_cdot_final sums the partials in fixed order into out[0..2]
// (re, im, norm).
template <typename T>
int launch_cdot(const void *a, const void *b, size_t len, double *partial, int max_blocks,
                hipStream_t s);
void launch_cdot_final(const double *partial, int nblk, double *out, hipStream_t s);
// Mixed-state transfer vectors.
// out[r] = sum_{l,p} env[l] wgt[p] A[l,p,r]
template <typename T>
void launch_env_left(const void *env, const void *A, const void *wgt, void *out, int chiL,
                     int d, int chiR, hipStream_t s);
// out[l] = sum_{p,r} A[l,p,r] wgt[p] env[r]
template <typename T>
void launch_env_right(const void *A, const void *wgt, const void *env, void *out, int chiL,
                      int d, int chiR, hipStream_t s);
// Two-site weighted transfer: out[r] = sum env[l] A[l,p,m] W[p,q] B[m,q,r]
// via tmp[p,m] = sum_l env[l] A[l,p,m].
template <typename T>
void launch_env_left2(const void *env, const void *A, const void *B, const void *W2,
                      void *tmp, void *out, int chiL, int d, int chiM, int chiR,
                      hipStream_t s);
// vec over (p_1..p_N), p = 2 s + s', to rho[s..., s'...] (2^N x 2^N).
template <typename T>
void launch_vec_to_rho(const void *vec, void *rho, int n, hipStream_t s);
// x[i] *= (re + i im), i < n.
template <typename T>
void launch_scale(void *x, size_t n, double re, double im, hipStream_t s);
// One part of a three-kernel round (2w <= 64): part 0 = MFMA partial Gram
// matrices, 1 = per-pair rotations, 2 = MFMA apply to W and V.
// rot_counter[0] += rotations, [1] += nc^2 of the pairs examined, [2] += nc^2
// of the pairs rotated.  stamp (nullable, jacobi_stamp_ints(nb) ints, zero at
// the start of a factorisation): change stamps that let a pair whose blocks
// are unchanged since it was last examined be skipped.  wgs: target number of
// workgroups of the Gram and W-apply launches (row chunks x block pairs; the
// V apply takes twice as many).
template <typename T>
void launch_jacobi_part(int part, void *W, int m, void *V, int n, int w, int nb, int rnd,
                        double tol, int inner_max, int inter, void *partial, void *J,
                        int *rotflag, int *rot_counter, int *stamp, int rot_threads, int wgs,
                        hipStream_t s);
inline size_t jacobi_stamp_ints(int nb) { return (size_t)nb + (size_t)(nb - 1) * nb; }
size_t jacobi_round3_partial_elems(int m, int n, int w, int wgs);
// ---- QR preconditioning (k_qr.hip) ----
// Columns of the next panel for a panel of mp rows (mp <= 4096).
int qr_panel_width(int elem_bytes, int mp);
// Factor the panel of columns j0.. (rows j0..m-1) of A (m x n, column-major)
// in place; writes its Householder vectors (unit lower trapezoidal) into the
// same columns of Vall, its T (nbk x nbk, column-major) to Tout and tau[j0..].
// Returns the panel width nbk used (columns j0 .. j0 + min(nbk, n - j0) - 1),
// or -1 if m - j0 is outside 1..4096 or j0 >= n.
template <typename T>
int launch_qr_panel(void *A, int m, int n, int j0, void *Vall, void *Tout, void *tau,
                    hipStream_t s);
template <typename T>
void launch_qr_rh(const void *A, int m, int n, void *X, hipStream_t s);
template <typename T>
void launch_qr_finish(const void *Wx, void *Vx, const double *sv, int n, void *Vr, hipStream_t s);
template <typename T>
void launch_qr_fill(const void *Y, int m, int n, void *C, hipStream_t s);
// out (k x ncols) = upper trapezoid of A's first k rows (conjugated if conj_r).
template <typename T>
void launch_qr_r_extract(const void *A, int lda, int k, int ncols, int conj_r, void *out,
                         hipStream_t s);
// C (m x k) = [I_k; 0].
template <typename T>
void launch_qr_eye(int m, int k, void *C, hipStream_t s);
// T (ob x ob) of the compact WY form of ob <= 64 reflectors from G = V^H V and tau.
template <typename T>
void launch_qr_larft(const void *G, const void *tau, int ob, void *Tout, hipStream_t s);
size_t jacobi_round3_j_elems(int n, int w);

// ---- reverse pass (k_adjoint.hip) ------------------------------------------
// C (M x N) = alpha op(A) op(B) + beta C, row-major; op 1 = conjugate transpose
// (the operand is then stored transposed).
template <typename T>
void launch_gemm_ex(int opA, int opB, int M, int N, int K, double ar, double ai, const void *A,
                    int lda, const void *B, int ldb, double br, double bi, void *C, int ldc,
                    hipStream_t s);
template <typename T>
void launch_axpby(size_t n, double ar, double ai, const void *X, double br, double bi, void *Y,
                  hipStream_t s);
// Y[j][i] = cst * scale_i^power * conj(X[i][j]) for i < rows_used, else 0.
template <typename T>
void launch_conjT_scaled(int rows, int rows_used, int cols, const void *X, int ldx,
                         const double *scale, int power, double cst, void *Y, int ldy,
                         hipStream_t s);
template <typename T>
void launch_scale_cols(int rows, int cols, void *X, int ld, const double *scale, int power,
                       hipStream_t s);
template <typename T>
void launch_rowdot_re(int k, int n, const void *X, int ldx, const void *Y, int ldy, double *out,
                      hipStream_t s);
template <typename T>
void launch_coldot_re(int rows, int cols, const void *A, const void *B, int ld, double *out,
                      hipStream_t s);
void launch_sbar_renorm(int k, int r, const double *stbar, const double *s, double sig,
                        double *sbar, hipStream_t st);
template <typename T>
void launch_svdvjp_P(int r, const void *J, const void *K, const double *s, const double *sbar,
                     double eta, void *P, hipStream_t st);
template <typename T>
void launch_gbar_grad(const void *Ab, const void *A, int chiL, int chiR, double *partial,
                      const double *dg, double *grad, int param, hipStream_t s);
// Y = I - E/2, R = I + E/2 from G = I + E (k x k, complex FP64); raises the
// double at rowsq_max (device, non-negative, cleared by the caller) to the
// largest squared row norm of E.
template <typename T>
void launch_reorth_factors(int k, const void *G, void *Y, void *R, void *rowsq_max,
                           hipStream_t s);
// C = (G2 - 2 G + 5 I) / 4 = I + E^2/4 from G = I + E and G2 = G G (k x k,
// complex FP64).
template <typename T>
void launch_reorth_corr(int k, const void *G2, const void *G, void *C, hipStream_t s);

// ---- device-resident small-bond layers (k_small.hip) ----
constexpr int SM_N = 128;      // columns of a factorisation (bonds <= SM_N / d)
constexpr int SM_GATES = 256;  // gates of one state's layer
// Every matrix of a small-bond layer (factor, right factor, products, site
// tensors) holds at most SM_N^2 complex entries.  Scratch per state: W, V,
// X, P, Y, R of SM_N^2 entries in the working precision, then an SM_N^2
// complex FP64 Gram.
constexpr size_t SM_ELEMS = (size_t)SM_N * SM_N;
inline size_t small_scratch_bytes(size_t csz) { return csz * 6 * SM_ELEMS + 16 * SM_ELEMS; }
// One state's consecutive small-bond layers; read and updated by its workgroup.
template <typename T>
struct SmallDesc {
    cx<T> *const *site;    // device array of n site pointers
    int *bond;             // device, n + 1 bond dimensions
    cx<T> *scratch;        // small_scratch_bytes
    const int *layer_off;  // n_layers + 1 offsets into the gate arrays
    const int *gsite;      // left sites of the gates (caller's order within a layer)
    const cx<T> *gmat;     // d^4 complex per gate
    const double *budget;  // per-gate target (< 0: schedule), or null
    ea_gate_record *log;   // one record per gate, in visiting order
    double *fout;          // per-gate f (caller's order), or null
    double tau, tol_user, f_min, lnP, lnS;
    long long n_total, g;
    int n, d, kind, n_gates, n_layers, lim, center, asc;  // lim: largest bond for a layer
    int chi_max, max_sweeps, inner, has_sched, strategy, reorth;
    int status, n_capped, n_noconv, n_done, layers_done;
};
template <typename T>
void launch_layer_small(SmallDesc<T> *descs, int n_states, hipStream_t s);
