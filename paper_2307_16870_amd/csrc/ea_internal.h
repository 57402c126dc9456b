// Internal declarations shared by the host sources of the library: the
// handle, device buffers, per-launch profiling and the templated steps of the
// two-site update that the forward API and the adjoint both use.
#pragma once
#include "ea_mps.h"
#include "ea_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

namespace ea {

extern thread_local std::string g_err;

// Launch shape of the three-kernel Jacobi for a factorisation of n columns
// from the process-wide tuning table (mps_set_tuning); false if no entry
// covers it.
bool tune_lookup(bool f64, int n, int *block, int *rot_threads, int *wgs);

inline int set_err(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// A device buffer.  `al` is the allocator it came from (NULL: hipMalloc) and
// `stream` the stream it was allocated for, so it can be released without
// its handle.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    const ea_allocator *al = nullptr;
    void *stream = nullptr;
};

}  // namespace ea

struct ea_mps {
    int n = 0, d = 2, kind = EA_PURE, prec = EA_C128, chi_max = 0;
    bool f64 = true;
    size_t csz = 16;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ea_allocator alloc{};    // device memory source (alloc.alloc NULL: hipMalloc / hipFree)
    std::vector<int> bond;  // n+1 entries, bond[0] = bond[n] = 1
    std::vector<ea::DevBuf> site;
    ea::DevBuf spare;
    int center = 0;
    double lnP = 0.0, lnS = 0.0;
    long g = 0;
    bool has_sched = false;
    double f_min = 1.0;
    long n_total = 1;
    int strategy = EA_GLOBAL;
    // workspace
    ea::DevBuf jpart, jmat, jflag, jstamp;
    // QR preconditioning: factored matrix, Householder vectors, T blocks,
    // tau, GEMM scratch, right vectors
    ea::DevBuf qr_a, qr_v, qr_t, qr_tau, qr_y, qr_z, qr_r, qr_s;
    int qr_min = 0;  // precondition factorisations of at least this many columns (0: off)
    // centre moves of the update path: 0 Jacobi SVD, 1 Householder QR, 2 Cholesky QR2
    int move_kind = 2;
    ea::DevBuf cq_x, cq_q, cq_g, cq_r1, cq_r2, cq_ri, cq_t, cq_misc;  // Cholesky QR workspace
    long n_chol_fallback = 0;  // Cholesky QR moves that fell back to the SVD move
    long n_cholqr_single = 0;  // Cholesky QR moves that needed one pass
    long n_topk = 0, n_topk_fallback = 0;  // partial factorisations accepted / abandoned
    // partial (top-k) factorisation of two-site updates (off by default)
    bool topk = false;
    int topk_p = 64, topk_q = 1, topk_min = 256;
    unsigned long long topk_seed = 0;
    ea::DevBuf tk_x, tk_om, tk_y, tk_w, tk_q1, tk_vj, tk_misc;
    // layer-parallel gauge (Vidal form, Hastings update): site tensors hold
    // B_i = Gamma_i Lambda_{i+1}; lam[b] the FP64 Schmidt values of bond b
    int gauge = 0;  // 0: one orthogonality centre; 1: layer-parallel
    std::vector<ea::DevBuf> lam;
    ea::DevBuf cbuf, ybuf;  // the unscaled two-site block; the kept right vectors
    std::vector<ea_mps *> workers;  // per-gate stream and workspace of a layer run side by side
    hipEvent_t ev = nullptr;        // orders a layer's streams
    bool vidal_parallel = true;     // run a layer's gates side by side
    // allocation-free calls: while `arena` is set, workspace buffers are carved
    // from it instead of allocated (see ensure); `arena_saved` keeps every
    // buffer's previous value, restored when the call ends
    char *arena = nullptr;
    size_t arena_cap = 0, arena_off = 0;
    std::vector<std::pair<ea::DevBuf *, ea::DevBuf>> arena_saved;
    int device = 0;  // device current when the handle was created
    bool jskip = true;  // skip block pairs unchanged since they were last examined
    ea::DevBuf ro_x64, ro_g, ro_y, ro_r, ro_t;  // re-orthogonalisation workspace
    bool reorth = true;
    int inner_round = 1, jkernel = 0, rot_threads = 0;  // 0: 16 per column of a block pair
    void *adj = nullptr;                 // adjoint buffers kept between calls
    void (*adj_free)(void *) = nullptr;
    int jorder = 1;  // 1: pairs inside a column block rotated in a sweep's first round only
    ea::DevBuf W, V, X, X2, s_raw, s_sorted, perm, rec, ints, partial, envb, tmp, out3, c128;
    // device-resident small-bond layers
    ea::DevBuf sm_scratch, sm_sites, sm_bond, sm_loff, sm_gsite, sm_gmat, sm_budget, sm_log,
        sm_fout, sm_descs;
    int small_cols = 64;  // device-resident layers: largest factorisation width (0: off)
    ea_dev_rec *rec_host = nullptr;
    int *int_host = nullptr;
    double *dbl_host = nullptr;
    char *stage_host = nullptr;
    size_t stage_cap = 0, stage_off = 0;
    ea::DevBuf stage_dev;
    // options
    double tol = 0.0;  // 0: m * eps
    int max_sweeps = 40;
    double tau = 1e-13;
    int block = 0;
    int inner_max = 12;
    std::vector<ea_gate_record> log;
    bool poisoned = false;
    // per-launch event timing (mps_profile)
    struct ProfRec {
        hipEvent_t a, b;
        int fam;
    };
    bool prof_on = false;
    int prof_every = 1;  // one launch in prof_every of each family is timed
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[EA_K_COUNT] = {0}, prof_flops[EA_K_COUNT] = {0}, prof_bytes[EA_K_COUNT] = {0};
    long prof_cnt[EA_K_COUNT] = {0}, prof_timed[EA_K_COUNT] = {0};
};


namespace ea {

#define HIPCHK(h, call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (h)->poisoned = true;                                                            \
            return set_err(EA_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
        }                                                                                    \
    } while (0)

#define LAUNCHCHK(h) HIPCHK(h, hipGetLastError())

#define TRY(x)                     \
    do {                           \
        int rc_ = (x);             \
        if (rc_ < 0) return rc_;   \
    } while (0)

// As TRY, returning fail(status) instead (clean-up on the error path).
#define TRY_OR(fail, x)                \
    do {                               \
        int rc_ = (x);                 \
        if (rc_ < 0) return fail(rc_); \
    } while (0)

template <typename T>
constexpr bool f64_of() {
    return sizeof(T) == 8;
}

inline hipEvent_t ev_get(ea_mps *h) {
    if (!h->prof_pool.empty()) {
        hipEvent_t e = h->prof_pool.back();
        h->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Counts the launches enqueued during its lifetime with their algorithmic
// flops and bytes, and times every prof_every-th of them per family with an
// event pair.
struct ProfScope {
    ea_mps *h;
    hipEvent_t a = nullptr;
    int fam;
    ProfScope(ea_mps *h_, int fam_, double fl, double by) : h(h_), fam(fam_) {
        if (!h->prof_on) return;
        const long k = h->prof_cnt[fam]++;
        h->prof_flops[fam] += fl;
        h->prof_bytes[fam] += by;
        if (k % h->prof_every == 0 && (a = ev_get(h)) != nullptr) (void)hipEventRecord(a, h->stream);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = ev_get(h);
        if (!b) return;
        (void)hipEventRecord(b, h->stream);
        h->prof_pending.push_back({a, b, fam});
    }
};

// Accumulate completed event pairs (call after a stream synchronisation).
inline void prof_harvest(ea_mps *h) {
    for (auto &r : h->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            h->prof_ms[r.fam] += ms;
            h->prof_timed[r.fam] += 1;
        }
        h->prof_pool.push_back(r.a);
        h->prof_pool.push_back(r.b);
    }
    h->prof_pending.clear();
}

// Tag of buffers carved from an allocation-free call's array: never freed.
inline ea_allocator *arena_tag() {
    static ea_allocator tag{};
    return &tag;
}

inline void free_buf(DevBuf &b) {
    if (b.p && b.al != arena_tag()) {
        if (b.al) b.al->free(b.al->ctx, b.p, b.stream);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.bytes = 0;
    b.al = nullptr;
}

inline bool is_site_buf(const ea_mps *h, const DevBuf &b) {
    return !h->site.empty() && &b >= &h->site.front() && &b <= &h->site.back();
}

// Grow b to at least `bytes` (x1.25 steps, contents not kept), from the
// handle's allocator if it has one, else hipMalloc.  During an
// allocation-free call nothing is allocated: a site tensor's buffer must
// already hold `bytes` (else EA_ETOOBIG), and any other (workspace) buffer is
// carved from the call's array in bump order, 256-byte aligned (EA_ETOOBIG
// when the array is exhausted), its previous value kept for the end of the call.
inline int ensure(ea_mps *h, DevBuf &b, size_t bytes) {
    if (h->arena) {
        if (is_site_buf(h, b)) {
            if (bytes <= b.bytes) return EA_OK;
            return set_err(EA_ETOOBIG,
                           "allocation-free call: a site tensor needs %zu bytes, its buffer holds "
                           "%zu (reserve bond capacity first)", bytes, b.bytes);
        }
        if (b.al == arena_tag() && bytes <= b.bytes) return EA_OK;
        const size_t want = (bytes + 255) & ~size_t(255);
        if (want > h->arena_cap - h->arena_off)
            return set_err(EA_ETOOBIG,
                           "allocation-free call: workspace beyond its %zu-byte device array",
                           h->arena_cap);
        h->arena_saved.push_back({&b, b});
        b.p = h->arena + h->arena_off;
        b.bytes = want;
        b.al = arena_tag();
        b.stream = nullptr;
        h->arena_off += want;
        return EA_OK;
    }
    if (bytes <= b.bytes) return EA_OK;
    const size_t old = b.bytes;
    if (b.p) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        free_buf(b);
    }
    size_t want = std::max(bytes, old + old / 4);
    want = (want + 255) & ~size_t(255);
    if (h->alloc.alloc) {
        b.p = h->alloc.alloc(h->alloc.ctx, want, (void *)h->stream);
        if (!b.p) return set_err(EA_ENOMEM, "allocator callback returned NULL for %zu bytes", want);
        b.al = &h->alloc;
        b.stream = (void *)h->stream;
    } else if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return set_err(EA_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    b.bytes = want;
    return EA_OK;
}

// Undo the carves made since (off, nsaved): the buffers get back their
// previous values and the array space is free again for later work of the
// same call (stream order keeps the earlier kernels' use of it first).
inline void arena_release(ea_mps *h, size_t off, size_t nsaved) {
    while (h->arena_saved.size() > nsaved) {
        *h->arena_saved.back().first = h->arena_saved.back().second;
        h->arena_saved.pop_back();
    }
    h->arena_off = off;
}

// A result computed into `spare` becomes the content of the site buffer
// dst: normally by exchanging the two buffers; during an allocation-free call
// (spare is then carved from the call's array) by a device copy into dst,
// which must hold `bytes`.
inline int commit_spare(ea_mps *h, DevBuf &dst, size_t bytes) {
    if (!h->arena) {
        std::swap(dst, h->spare);
        return EA_OK;
    }
    if (bytes > dst.bytes)
        return set_err(EA_ETOOBIG, "allocation-free call: site buffer too small (%zu < %zu)",
                       dst.bytes, bytes);
    HIPCHK(h, hipMemcpyAsync(dst.p, h->spare.p, bytes, hipMemcpyDeviceToDevice, h->stream));
    return EA_OK;
}

inline int check(const ea_mps *h) {
    if (!h) return set_err(EA_EINVAL, "null handle");
    if (h->poisoned) return set_err(EA_EHIP, "handle poisoned by an earlier HIP error");
    return EA_OK;
}

inline bool finite_cplx(const double *p, size_t n) {
    for (size_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// ||A^H A - I||_max for a k x k complex matrix given as interleaved doubles.
inline bool is_unitary(const double *a, int k) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double re = 0, im = 0;
            for (int r = 0; r < k; ++r) {
                double ar = a[2 * (r * k + i)], ai = -a[2 * (r * k + i) + 1];
                double br = a[2 * (r * k + j)], bi = a[2 * (r * k + j) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            if (std::fabs(re - (i == j ? 1.0 : 0.0)) > 1e-12 || std::fabs(im) > 1e-12) return false;
        }
    return true;
}

// Copy n complex doubles into the pinned staging ring, converted to T, and
// enqueue the upload on the handle's stream.  Slots are reused only after a
// stream synchronisation, so earlier kernels never see later operands.
template <typename T>
int stage(ea_mps *h, const double *src, size_t n, void **dev) {
    const size_t bytes = n * 2 * sizeof(T);
    size_t need = (bytes + 255) & ~size_t(255);
    if (need > h->stage_cap) return set_err(EA_ETOOBIG, "operand too large for staging");
    if (h->stage_off + need > h->stage_cap) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        h->stage_off = 0;
    }
    T *dst = reinterpret_cast<T *>(h->stage_host + h->stage_off);
    for (size_t i = 0; i < 2 * n; ++i) dst[i] = (T)src[i];
    char *d = (char *)h->stage_dev.p + h->stage_off;
    HIPCHK(h, hipMemcpyAsync(d, dst, bytes, hipMemcpyHostToDevice, h->stream));
    h->stage_off += need;
    *dev = d;
    return EA_OK;
}

inline double schedule_target(const ea_mps *h) {
    if (!h->has_sched) return 1.0;
    const double n = (double)h->n_total, g = (double)h->g;
    double ft;
    if (h->strategy == EA_NAIVE) {
        ft = std::pow(h->f_min, 1.0 / n);
    } else if (h->strategy == EA_GLOBAL) {
        double left = n - g;
        ft = left <= 0 ? 1.0 : std::exp((std::log(h->f_min) - h->lnP) / left);
    } else if (h->strategy == EA_NEAREST) {
        ft = std::exp(std::log(h->f_min) * (g + 1) / n - h->lnP);
    } else {  // EA_FIXED: only the chi_max cap truncates
        ft = 1.0;
    }
    return std::min(1.0, std::max(ft, 1e-300));
}

template <typename T>
double default_tol(int m) {
    return (double)m * (sizeof(T) == 8 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
}

// One-sided Jacobi on W (m x n, column-major, m >= n), V <- accumulated
// rotations.  Writes (sweeps, converged) to ints[0..1] on the device.
template <typename T>
int svd_core(ea_mps *h, int m, int n) {
    int *sweeps_dev = (int *)h->ints.p;
    int *counter = sweeps_dev + 2;
    const double tol = h->tol > 0 ? h->tol : default_tol<T>(m);
    const double c = (double)h->csz;
    {
        ProfScope ps(h, EA_K_OTHER, 0.0, c * n * (double)n);
        launch_eye<T>(h->V.p, n, h->stream);
    }
    if (n <= 64) {
        ProfScope ps(h, EA_K_JSMALL, 0.0, 2.0 * c * (m + n) * (double)n);
        launch_jacobi_single<T>(h->W.p, m, h->V.p, n, tol, h->inner_max, h->max_sweeps,
                                sweeps_dev, h->stream);
        LAUNCHCHK(h);
        return EA_OK;
    }
    const bool three = h->jkernel == 0;
    // launch shape: explicit options, else the tuning table, else built in
    int tb = 32, trt = 0, wgs = 256;
    const bool tuned = three && tune_lookup(h->f64, n, &tb, &trt, &wgs);
    int w = h->block > 0 ? h->block : (three ? tb : (n <= 256 ? 8 : 16));
    if (2 * w > 64) w = 32;
    const int ncmax = 2 * w <= 16 ? 16 : (2 * w <= 32 ? 32 : 64);
    const int rot_threads = h->rot_threads > 0 ? h->rot_threads
                            : (tuned && h->block == 0) ? trt
                                                       : (2 * w <= 32 ? 512 : 1024);
    int nb = (n + w - 1) / w;
    nb += nb & 1;
    if (three) {
        TRY(ensure(h, h->jpart, h->csz * jacobi_round3_partial_elems(m, n, w, wgs)));
        TRY(ensure(h, h->jmat, h->csz * jacobi_round3_j_elems(n, w)));
        TRY(ensure(h, h->jflag, sizeof(int) * (nb / 2 + 1)));
        if (h->jskip) {
            TRY(ensure(h, h->jstamp, sizeof(int) * jacobi_stamp_ints(nb)));
            launch_fill_int((int *)h->jstamp.p, (int)jacobi_stamp_ints(nb), 0, h->stream);
        }
    }
    int *stamp = three && h->jskip ? (int *)h->jstamp.p : nullptr;
    int sweeps = 0, conv = 0;
    for (int sw = 0; sw < h->max_sweeps; ++sw) {
        launch_fill_int(counter, 3, 0, h->stream);
        for (int rnd = 0; rnd < nb - 1; ++rnd) {
            // pairs inside a block are rotated in the sweep's first round only
            const int inter = (h->jorder == 1 && rnd > 0) ? 1 : 0;
            if (three) {
                // algorithmic work is counted per sweep from the pairs examined
                // and rotated (below)
                {
                    ProfScope ps(h, EA_K_JGRAM, 0.0, c * m * (double)n);
                    launch_jacobi_part<T>(0, h->W.p, m, h->V.p, n, w, nb, rnd, tol, h->inner_round,
                                          inter, h->jpart.p, h->jmat.p, (int *)h->jflag.p, counter,
                                          stamp, rot_threads, wgs, h->stream);
                }
                {
                    // per block pair: the Hermitian Gram matrix (upper triangle) in,
                    // the accumulated rotation J out
                    const double ncd = 2 * w <= 32 ? 32.0 : 64.0;
                    ProfScope ps(h, EA_K_JROT, 0.0, c * (nb / 2) * (ncd * (ncd + 1) / 2 + ncd * ncd));
                    launch_jacobi_part<T>(1, h->W.p, m, h->V.p, n, w, nb, rnd, tol, h->inner_round,
                                          inter, h->jpart.p, h->jmat.p, (int *)h->jflag.p, counter,
                                          stamp, rot_threads, wgs, h->stream);
                }
                {
                    ProfScope ps(h, EA_K_JAPPLY, 0.0, 2.0 * c * (m + n) * (double)n);
                    launch_jacobi_part<T>(2, h->W.p, m, h->V.p, n, w, nb, rnd, tol, h->inner_round,
                                          inter, h->jpart.p, h->jmat.p, (int *)h->jflag.p, counter,
                                          stamp, rot_threads, wgs, h->stream);
                }
            } else {
                // algorithmic work of one round: every column block pair forms its
                // Hermitian Gram matrix (4 m nc^2 flops) and rotates its nc columns
                // of W and V (8 (m + n) nc^2 flops)
                double fl2 = 0.0;
                for (int p = 0; p < nb / 2; ++p) {
                    const int a = p == 0 ? 0 : (p - 1 + rnd) % (nb - 1) + 1;
                    const int bq = nb - 1 - p;
                    const int b = bq == 0 ? 0 : (bq - 1 + rnd) % (nb - 1) + 1;
                    const int nc = std::max(0, std::min(w, n - a * w)) +
                                   std::max(0, std::min(w, n - b * w));
                    fl2 += (double)nc * nc;
                }
                ProfScope ps(h, EA_K_JFUSED, (4.0 * m + 8.0 * (m + n)) * fl2,
                             2.0 * c * (m + n) * (double)n);
                launch_jacobi_round<T>(h->W.p, m, h->V.p, n, w, nb, rnd, tol, 6, ncmax, counter,
                                       h->stream);
            }
        }
        LAUNCHCHK(h);
        HIPCHK(h, hipMemcpyAsync(h->int_host, counter, 3 * sizeof(int), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        ++sweeps;
        // algorithmic work of this sweep: each rotation updates two rows of the
        // Hermitian Gram matrix and two columns of J (48 nc flops); each pair
        // examined forms its Gram matrix (4 m nc^2 flops); each pair rotated
        // multiplies its nc columns of W and V by J (8 (m + n) nc^2 flops)
        if (h->prof_on && three) {
            h->prof_flops[EA_K_JROT] += 48.0 * 2 * w * (double)h->int_host[0];
            h->prof_flops[EA_K_JGRAM] += 4.0 * m * (double)h->int_host[1];
            h->prof_flops[EA_K_JAPPLY] += 8.0 * (m + n) * (double)h->int_host[2];
        }
        if (h->int_host[0] == 0) {
            conv = 1;
            break;
        }
    }
    if (sizeof(T) == 4 && h->reorth) {
        // FP32 right vectors carry a norm drift that grows with the rotations
        // applied to them; unit columns keep U S V^H (and the norm) exact.
        ProfScope ps(h, EA_K_NORMS, 4.0 * n * (double)n, c * (2.0 * m + 3.0 * n) * (double)n);
        launch_unit_right<T>(h->W.p, m, h->V.p, n, h->stream);
    }
    launch_fill_int(sweeps_dev, 1, sweeps, h->stream);
    launch_fill_int(sweeps_dev + 1, 1, conv, h->stream);
    return EA_OK;
}

// C = alpha op(A) op(B) + beta C on the state's stream (column-major;
// op 'N', 'T' = transpose or 'C' = conjugate transpose), complex FP32 or FP64,
// on the matrix-core GEMM.  A column-major matrix is the row-major array of
// its transpose, so the row-major kernel computes C^T = op(B)^T op(A)^T; the
// op codes carry over unchanged (op(B)^T of a column-major B is, on B's
// row-major view, the same kind of operation).
template <typename T>
int blas_gemm(ea_mps *h, char opa, char opb, int m, int n, int k, double alpha, const void *A,
              int lda, const void *B, int ldb, double beta, void *C, int ldc) {
    if (m <= 0 || n <= 0) return EA_OK;
    auto code = [](char o) { return o == 'C' ? 1 : (o == 'T' ? 2 : 0); };
    launch_zgemm<T>(code(opb), code(opa), n, m, k, alpha, 0.0, B, ldb, A, lda, beta, 0.0, C, ldc,
                    h->stream);
    LAUNCHCHK(h);
    return EA_OK;
}

constexpr int QR_NBK_MAX = 16, QR_OBW = 64;  // panel width <= 16; reflectors applied 64 at a time


// Householder QR of src (m x n, column-major, ld m; m <= 4096) with
// k = min(m, n) reflectors: the factored matrix (R in its upper trapezoid) in
// qr_a, the reflectors (unit lower trapezoidal) in qr_v, per 64-column block
// the T of Q_b = I - V_b T_b V_b^H in qr_t; Q = Q_1 Q_2 ... .
template <typename T>
int qr_factor(ea_mps *h, const void *src, int m, int n) {
    const size_t c = h->csz;
    const int k = std::min(m, n), nblk = (k + QR_OBW - 1) / QR_OBW;
    if (m > 4096) return set_err(EA_ETOOBIG, "the QR takes at most 4096 rows");
    TRY(ensure(h, h->qr_a, c * (size_t)m * n));
    TRY(ensure(h, h->qr_v, c * (size_t)m * k));
    TRY(ensure(h, h->qr_t, c * ((size_t)QR_OBW * QR_OBW * (nblk + 1) + QR_NBK_MAX * QR_NBK_MAX)));
    TRY(ensure(h, h->qr_tau, c * (size_t)k));
    TRY(ensure(h, h->qr_y, c * (size_t)QR_OBW * std::max(m, n)));
    TRY(ensure(h, h->qr_z, c * (size_t)QR_OBW * std::max(m, n)));
    char *A = (char *)h->qr_a.p, *Vall = (char *)h->qr_v.p, *Tb = (char *)h->qr_t.p;
    char *Tpanel = Tb + c * (size_t)QR_OBW * QR_OBW * nblk;  // the current panel's T
    ProfScope ps(h, EA_K_QR, 4.0 * (4.0 * m * (double)n * k - 2.0 * (double)(m + n) * k * k +
                                    4.0 / 3.0 * (double)k * k * k),
                 2.0 * c * (double)m * n);
    HIPCHK(h, hipMemcpyAsync(A, src, c * (size_t)m * n, hipMemcpyDeviceToDevice, h->stream));
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * QR_OBW, bend = std::min(k, b0 + QR_OBW), ob = bend - b0, mb = m - b0;
        char *Vb = Vall + c * ((size_t)b0 * m + b0);
        // the block's reflectors are zero above their diagonal
        HIPCHK(h, hipMemset2DAsync(Vb, c * (size_t)m, 0, c * (size_t)mb, ob, h->stream));
        for (int j0 = b0; j0 < bend;) {
            const int nbk = launch_qr_panel<T>(A, m, bend, j0, Vall, Tpanel, h->qr_tau.p, h->stream);
            if (nbk <= 0) return set_err(EA_EINVAL, "QR panel at column %d of %d x %d", j0, m, n);
            const int nc = std::min(nbk, bend - j0), mp = m - j0, nt = bend - j0 - nc;
            if (nt > 0) {  // the rest of the block: A2 <- A2 - V (T^H (V^H A2))
                const char *V = Vall + c * ((size_t)j0 * m + j0);
                char *A2 = A + c * ((size_t)(j0 + nc) * m + j0);
                TRY(blas_gemm<T>(h, 'C', 'N', nc, nt, mp, 1.0, V, m, A2, m, 0.0, h->qr_y.p, nc));
                TRY(blas_gemm<T>(h, 'C', 'N', nc, nt, nc, 1.0, Tpanel, nbk, h->qr_y.p, nc, 0.0,
                                 h->qr_z.p, nc));
                TRY(blas_gemm<T>(h, 'N', 'N', mp, nt, nc, -1.0, V, m, h->qr_z.p, nc, 1.0, A2, m));
            }
            j0 += nc;
        }
        // the block's T from G = V_b^H V_b, then every column right of the block
        char *Tblk = Tb + c * (size_t)QR_OBW * QR_OBW * b;
        TRY(blas_gemm<T>(h, 'C', 'N', ob, ob, mb, 1.0, Vb, m, Vb, m, 0.0, h->qr_z.p, ob));
        launch_qr_larft<T>(h->qr_z.p, (char *)h->qr_tau.p + c * (size_t)b0, ob, Tblk, h->stream);
        const int nt = n - bend;
        if (nt > 0) {
            char *A2 = A + c * ((size_t)bend * m + b0);
            TRY(blas_gemm<T>(h, 'C', 'N', ob, nt, mb, 1.0, Vb, m, A2, m, 0.0, h->qr_y.p, ob));
            TRY(blas_gemm<T>(h, 'C', 'N', ob, nt, ob, 1.0, Tblk, ob, h->qr_y.p, ob, 0.0, h->qr_z.p,
                             ob));
            TRY(blas_gemm<T>(h, 'N', 'N', mb, nt, ob, -1.0, Vb, m, h->qr_z.p, ob, 1.0, A2, m));
        }
    }
    LAUNCHCHK(h);
    return EA_OK;
}

// C (m x ncols, column-major, ld m) <- Q C with the Q of the last qr_factor
// of an m x n matrix (k = min(m, n) reflectors, applied block by block from
// the last).
template <typename T>
int qr_apply_q(ea_mps *h, void *C, int m, int n, int ncols) {
    const size_t c = h->csz;
    const int k = std::min(m, n), nblk = (k + QR_OBW - 1) / QR_OBW;
    TRY(ensure(h, h->qr_y, c * (size_t)QR_OBW * ncols));
    TRY(ensure(h, h->qr_z, c * (size_t)QR_OBW * ncols));
    ProfScope ps(h, EA_K_QR, 4.0 * (4.0 * m * (double)ncols * k - 2.0 * (double)ncols * k * k),
                 2.0 * c * (double)m * ncols);
    const char *Vall = (const char *)h->qr_v.p, *Tb = (const char *)h->qr_t.p;
    for (int b = nblk - 1; b >= 0; --b) {
        const int b0 = b * QR_OBW, ob = std::min(k, b0 + QR_OBW) - b0, mb = m - b0;
        const char *Vb = Vall + c * ((size_t)b0 * m + b0);
        const char *Tblk = Tb + c * (size_t)QR_OBW * QR_OBW * b;
        char *C2 = (char *)C + c * (size_t)b0;
        TRY(blas_gemm<T>(h, 'C', 'N', ob, ncols, mb, 1.0, Vb, m, C2, m, 0.0, h->qr_y.p, ob));
        TRY(blas_gemm<T>(h, 'N', 'N', ob, ncols, ob, 1.0, Tblk, ob, h->qr_y.p, ob, 0.0, h->qr_z.p,
                         ob));
        TRY(blas_gemm<T>(h, 'N', 'N', mb, ncols, ob, -1.0, Vb, m, h->qr_z.p, ob, 1.0, C2, m));
    }
    return EA_OK;
}

// SVD of W (m x n, m >= n, column-major) preconditioned by its Householder QR:
// W = Q R, one-sided Jacobi on X = R^H (X V_x = W_x = U_x S), then
// W <- Q [V_x S; 0] = U S and V <- W_x S^-1 = the right singular vectors, so
// the caller sees the same (W = U S, V) as from svd_core.
template <typename T>
int svd_precond(ea_mps *h, int m, int n) {
    const size_t c = h->csz;
    TRY(qr_factor<T>(h, h->W.p, m, n));
    launch_qr_rh<T>(h->qr_a.p, m, n, h->W.p, h->stream);  // W = R^H (n x n)
    LAUNCHCHK(h);
    TRY(svd_core<T>(h, n, n));  // W = W_x (n x n), V = V_x
    TRY(ensure(h, h->qr_r, c * (size_t)n * n));
    TRY(ensure(h, h->qr_s, sizeof(double) * n));
    launch_colnorms<T>(h->W.p, n, n, (double *)h->qr_s.p, h->stream);
    launch_qr_finish<T>(h->W.p, h->V.p, (const double *)h->qr_s.p, n, h->qr_r.p, h->stream);
    launch_qr_fill<T>(h->V.p, m, n, h->W.p, h->stream);  // W = [V_x S; 0]
    LAUNCHCHK(h);
    TRY(qr_apply_q<T>(h, h->W.p, m, n, n));
    std::swap(h->V, h->qr_r);  // V = W_x S^-1
    return EA_OK;
}

// Factor matrix X (rows x cols, currently in W as column-major after the
// caller's copy/contraction) and read back the decision record.
template <typename T>
int factor_and_decide(ea_mps *h, int mw, int nw, double f_t, int mode, int forced_k) {
    TRY(ensure(h, h->s_raw, sizeof(double) * nw));
    TRY(ensure(h, h->s_sorted, sizeof(double) * nw));
    TRY(ensure(h, h->perm, sizeof(int) * nw));
    if (h->qr_min > 0 && nw >= h->qr_min && nw > 64 && h->jkernel == 0)
        TRY(svd_precond<T>(h, mw, nw));
    else
        TRY(svd_core<T>(h, mw, nw));
    {
        ProfScope ps(h, EA_K_NORMS, 4.0 * mw * (double)nw, (double)h->csz * mw * (double)nw);
        launch_colnorms<T>(h->W.p, mw, nw, (double *)h->s_raw.p, h->stream);
    }
    {
        ProfScope ps(h, EA_K_TRUNC, (double)nw, 24.0 * nw);
        launch_sort_trunc((const double *)h->s_raw.p, nw, f_t, h->chi_max, h->tau, mode,
                          forced_k, (const int *)h->ints.p, (int *)h->perm.p,
                          (double *)h->s_sorted.p, (ea_dev_rec *)h->rec.p, h->stream);
    }
    LAUNCHCHK(h);
    HIPCHK(h, hipMemcpyAsync(h->rec_host, h->rec.p, sizeof(ea_dev_rec), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    return EA_OK;
}

template <typename T>
void gather(ea_mps *h, const void *src, int ld, int k, int X, int conj_src, int es, int ec,
            int transposed, void *out) {
    ProfScope ps(h, EA_K_GATHER, 0.0, 2.0 * (double)h->csz * k * (double)X);
    launch_gather<T>(src, ld, (const int *)h->perm.p, (const double *)h->s_sorted.p,
                     (const ea_dev_rec *)h->rec.p, k, X, conj_src, es, ec, transposed, out,
                     h->stream);
}

// FP64 re-orthogonalisation of the isometric factor written by an FP32
// factorisation (Loewdin steps).  cols = 1: X (rows x k, row-major) should
// have orthonormal columns and the neighbour N (k x ncols) absorbs R from the
// left; cols = 0: X (k x rows) should have orthonormal rows and N (nrows x k)
// absorbs R from the right.  With G = X^H X (or X X^H) = I + E formed in FP64,
// X <- X (I - E/2) and N <- (I + E/2) N leave X^H X - I = -(3/4) E^2 + O(E^3)
// and change the product by the factor I - E^2/4; the entries of E^2 are at
// most r, the largest squared row norm of E.  Two corrections hold both to
// 1e-6: once r/4 exceeds it, N also takes C = I + E^2/4 (product factor
// I - E^4/16; the loss E^2/4 falls on the heavy columns, whose rows of E
// collect the errors of the many light columns, and would bias the kept
// weights); while 3r/4 exceeds it, a further step runs (three at most).
// Well-conditioned factors need neither; wide ill-conditioned ones (thousands
// of kept columns over several decades of singular values) take both once.
// Workspace of reorth (taken before the caller's first write, so that an
// allocation-free call fails, if it must, while the state is still whole).
template <typename T>
int reorth_reserve(ea_mps *h, int rows, int k, int nother) {
    if (sizeof(T) == 8 || !h->reorth || k < 1) return EA_OK;
    const size_t nx = (size_t)rows * k;
    TRY(ensure(h, h->ro_x64, 16 * std::max(nx, (size_t)k * k)));
    TRY(ensure(h, h->ro_g, 16 * (size_t)k * k + 256));
    TRY(ensure(h, h->ro_y, h->csz * (size_t)k * k));
    TRY(ensure(h, h->ro_r, h->csz * (size_t)k * k));
    TRY(ensure(h, h->ro_t, h->csz * std::max(nx, (size_t)k * nother)));
    return EA_OK;
}

template <typename T>
int reorth(ea_mps *h, bool cols, void *X, int rows, int k, void *N, int nother) {
    if (sizeof(T) == 8 || !h->reorth || k < 1) return EA_OK;
    const size_t nx = (size_t)rows * k;
    TRY(reorth_reserve<T>(h, rows, k, nother));
    void *rowsq = (char *)h->ro_g.p + 16 * (size_t)k * k;
    // Row-major products through column-major GEMMs: the row-major C = A B
    // (m x n) is the column-major C^T = B^T A^T.
    // N <- F N (cols) or N F (rows) for a k x k factor F in T precision
    auto absorb = [&](const void *F) -> int {
        if (cols)
            TRY(blas_gemm<T>(h, 'N', 'N', nother, k, k, 1.0, N, nother, F, k, 0.0, h->ro_t.p,
                             nother));
        else
            TRY(blas_gemm<T>(h, 'N', 'N', k, nother, k, 1.0, F, k, N, k, 0.0, h->ro_t.p, k));
        HIPCHK(h, hipMemcpyAsync(N, h->ro_t.p, h->csz * (size_t)k * nother,
                                 hipMemcpyDeviceToDevice, h->stream));
        return EA_OK;
    };
    for (int step = 0; step < 3; ++step) {
        double r;
        {
            ProfScope ps(h, EA_K_OTHER, 8.0 * rows * (double)k * k * 2 + 8.0 * k * (double)k * nother,
                         (double)h->csz * (3.0 * nx + 2.0 * k * (double)nother));
            launch_to_c128<T>(X, (double *)h->ro_x64.p, nx, h->stream);
            // G = X^H X (cols) or X X^H (rows), row-major k x k, in FP64
            if (cols)
                TRY(blas_gemm<double>(h, 'N', 'C', k, k, rows, 1.0, h->ro_x64.p, k, h->ro_x64.p,
                                      k, 0.0, h->ro_g.p, k));
            else
                TRY(blas_gemm<double>(h, 'C', 'N', k, k, rows, 1.0, h->ro_x64.p, rows,
                                      h->ro_x64.p, rows, 0.0, h->ro_g.p, k));
            HIPCHK(h, hipMemsetAsync(rowsq, 0, sizeof(double), h->stream));
            launch_reorth_factors<T>(k, h->ro_g.p, h->ro_y.p, h->ro_r.p, rowsq, h->stream);
            HIPCHK(h, hipMemcpyAsync(h->dbl_host, rowsq, sizeof(double), hipMemcpyDeviceToHost,
                                     h->stream));
            // X <- X Y (cols) or Y X (rows)
            if (cols)
                TRY(blas_gemm<T>(h, 'N', 'N', k, rows, k, 1.0, h->ro_y.p, k, X, k, 0.0,
                                 h->ro_t.p, k));
            else
                TRY(blas_gemm<T>(h, 'N', 'N', rows, k, k, 1.0, X, rows, h->ro_y.p, k, 0.0,
                                 h->ro_t.p, rows));
            HIPCHK(h, hipMemcpyAsync(X, h->ro_t.p, h->csz * nx, hipMemcpyDeviceToDevice,
                                     h->stream));
            TRY(absorb(h->ro_r.p));
            LAUNCHCHK(h);
            HIPCHK(h, hipStreamSynchronize(h->stream));
            r = h->dbl_host[0];
        }
        if (0.25 * r > 1e-6) {
            ProfScope ps(h, EA_K_OTHER, 8.0 * k * (double)k * k + 8.0 * k * (double)k * nother,
                         16.0 * 3.0 * k * (double)k + (double)h->csz * 2.0 * k * (double)nother);
            TRY(blas_gemm<double>(h, 'N', 'N', k, k, k, 1.0, h->ro_g.p, k, h->ro_g.p, k, 0.0,
                                  h->ro_x64.p, k));
            launch_reorth_corr<T>(k, h->ro_x64.p, h->ro_g.p, h->ro_r.p, h->stream);
            TRY(absorb(h->ro_r.p));
            LAUNCHCHK(h);
        }
        if (0.75 * r <= 1e-6) break;
    }
    return EA_OK;
}

// Move the orthogonality centre one site right: SVD of A_c as
// (chi_l d) x chi_r; A_c <- U, A_{c+1} <- (S V^H) A_{c+1}.
template <typename T>
int move_right(ea_mps *h) {
    const int c = h->center, d = h->d;
    const int M = h->bond[c] * d, N = h->bond[c + 1];
    const int orient = M >= N ? 0 : 1, mw = std::max(M, N), nw = std::min(M, N);
    if (nw > EA_SORT_MAX) return set_err(EA_ETOOBIG, "bond too large for centre move");
    TRY(ensure(h, h->W, h->csz * (size_t)mw * nw));
    TRY(ensure(h, h->V, h->csz * (size_t)nw * nw));
    {
        ProfScope ps(h, EA_K_OTHER, 0.0, 2.0 * (double)h->csz * M * (double)N);
        launch_to_colmajor<T>(h->site[c].p, h->W.p, M, N, orient, h->stream);
    }
    TRY(factor_and_decide<T>(h, mw, nw, 1.0, 1, 0));
    const int k = h->rec_host->k;
    if (!(h->rec_host->s0 > 0.0)) return set_err(EA_EINVAL, "zero site tensor");
    const int chi2 = h->bond[c + 2];
    TRY(ensure(h, h->site[c], h->csz * (size_t)M * k));
    TRY(ensure(h, h->X, h->csz * (size_t)k * N));
    TRY(ensure(h, h->spare, h->csz * (size_t)k * d * chi2));
    TRY(reorth_reserve<T>(h, M, k, d * chi2));
    if (orient == 0) {
        gather<T>(h, h->W.p, M, k, M, 0, -1, 0, 1, h->site[c].p);
        gather<T>(h, h->V.p, N, k, N, 1, 1, 0, 0, h->X.p);
    } else {
        gather<T>(h, h->V.p, M, k, M, 0, 0, 0, 1, h->site[c].p);
        gather<T>(h, h->W.p, N, k, N, 1, 0, 0, 0, h->X.p);
    }
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * k * (double)(d * chi2) * N,
                     (double)h->csz * ((double)k * N + (double)N * d * chi2 + (double)k * d * chi2));
        launch_gemm<T>(h->X.p, h->site[c + 1].p, h->spare.p, k, d * chi2, N, N, d * chi2,
                       d * chi2, h->stream);
    }
    LAUNCHCHK(h);
    TRY(commit_spare(h, h->site[c + 1], h->csz * (size_t)k * d * chi2));
    TRY(reorth<T>(h, true, h->site[c].p, M, k, h->site[c + 1].p, d * chi2));
    h->bond[c + 1] = k;
    h->center = c + 1;
    return EA_OK;
}

// Move the centre one site left: SVD of A_c as chi_l x (d chi_r);
// A_c <- V^H, A_{c-1} <- A_{c-1} (U S).
template <typename T>
int move_left(ea_mps *h) {
    const int c = h->center, d = h->d;
    const int M = h->bond[c], N = d * h->bond[c + 1];
    const int orient = M >= N ? 0 : 1, mw = std::max(M, N), nw = std::min(M, N);
    if (nw > EA_SORT_MAX) return set_err(EA_ETOOBIG, "bond too large for centre move");
    TRY(ensure(h, h->W, h->csz * (size_t)mw * nw));
    TRY(ensure(h, h->V, h->csz * (size_t)nw * nw));
    {
        ProfScope ps(h, EA_K_OTHER, 0.0, 2.0 * (double)h->csz * M * (double)N);
        launch_to_colmajor<T>(h->site[c].p, h->W.p, M, N, orient, h->stream);
    }
    TRY(factor_and_decide<T>(h, mw, nw, 1.0, 1, 0));
    const int k = h->rec_host->k;
    if (!(h->rec_host->s0 > 0.0)) return set_err(EA_EINVAL, "zero site tensor");
    const int rowsP = h->bond[c - 1] * d;
    TRY(ensure(h, h->site[c], h->csz * (size_t)k * N));
    TRY(ensure(h, h->X, h->csz * (size_t)M * k));
    TRY(ensure(h, h->spare, h->csz * (size_t)rowsP * k));
    TRY(reorth_reserve<T>(h, N, k, rowsP));
    if (orient == 0) {
        gather<T>(h, h->V.p, N, k, N, 1, 0, 0, 0, h->site[c].p);
        gather<T>(h, h->W.p, M, k, M, 0, 0, 0, 1, h->X.p);
    } else {
        gather<T>(h, h->W.p, N, k, N, 1, -1, 0, 0, h->site[c].p);
        gather<T>(h, h->V.p, M, k, M, 0, 1, 0, 1, h->X.p);
    }
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * rowsP * (double)k * M,
                     (double)h->csz * ((double)rowsP * M + (double)M * k + (double)rowsP * k));
        launch_gemm<T>(h->site[c - 1].p, h->X.p, h->spare.p, rowsP, k, M, M, k, k, h->stream);
    }
    LAUNCHCHK(h);
    TRY(commit_spare(h, h->site[c - 1], h->csz * (size_t)rowsP * k));
    TRY(reorth<T>(h, false, h->site[c].p, N, k, h->site[c - 1].p, rowsP));
    h->bond[c] = k;
    h->center = c - 1;
    return EA_OK;
}

// Centre moves by Householder QR (Sec. III: A_c = Q R, Q left-normalised,
// R absorbed into the neighbour; no rank is dropped).  Right: A_c as
// (chi_l d) x chi_r = Q R, A_c <- Q, A_{c+1} <- R A_{c+1}.
template <typename T>
int move_right_qr(ea_mps *h) {
    const int c = h->center, d = h->d;
    const int M = h->bond[c] * d, N = h->bond[c + 1], k = std::min(M, N);
    const int P = d * h->bond[c + 2];
    if (M > 4096) return set_err(EA_ETOOBIG, "bond too large for a QR centre move");
    TRY(ensure(h, h->W, h->csz * (size_t)M * N));
    launch_to_colmajor<T>(h->site[c].p, h->W.p, M, N, 0, h->stream);
    TRY(qr_factor<T>(h, h->W.p, M, N));
    TRY(ensure(h, h->X, h->csz * (size_t)k * N));
    launch_qr_r_extract<T>(h->qr_a.p, M, k, N, 0, h->X.p, h->stream);  // R (k x N)
    launch_qr_eye<T>(M, k, h->W.p, h->stream);
    LAUNCHCHK(h);
    TRY(qr_apply_q<T>(h, h->W.p, M, N, k));  // Q (M x k)
    TRY(ensure(h, h->site[c], h->csz * (size_t)M * k));
    TRY(ensure(h, h->spare, h->csz * (size_t)k * P));
    TRY(reorth_reserve<T>(h, M, k, P));
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * k * (double)N * P,
                     (double)h->csz * ((double)k * N + (double)N * P + (double)k * P));
        launch_to_colmajor<T>(h->W.p, h->site[c].p, k, M, 0, h->stream);  // row-major (M, k)
        // (R A_{c+1})^T = A_{c+1}^T R^T in column-major terms: row-major (k, P)
        TRY(blas_gemm<T>(h, 'N', 'T', P, k, N, 1.0, h->site[c + 1].p, P, h->X.p, k, 0.0,
                         h->spare.p, P));
    }
    LAUNCHCHK(h);
    TRY(commit_spare(h, h->site[c + 1], h->csz * (size_t)k * P));
    TRY(reorth<T>(h, true, h->site[c].p, M, k, h->site[c + 1].p, P));
    h->bond[c + 1] = k;
    h->center = c + 1;
    return EA_OK;
}

// Left: A_c as chi_l x (d chi_r) = L Q_r through the QR of A_c^H = Q' R':
// A_c <- Q'^H (orthonormal rows), A_{c-1} <- A_{c-1} R'^H.
template <typename T>
int move_left_qr(ea_mps *h) {
    const int c = h->center, d = h->d;
    const int M = h->bond[c], N = d * h->bond[c + 1], k = std::min(M, N);
    const int P = h->bond[c - 1] * d;
    if (N > 4096) return set_err(EA_ETOOBIG, "bond too large for a QR centre move");
    TRY(ensure(h, h->W, h->csz * (size_t)M * N));
    launch_to_colmajor<T>(h->site[c].p, h->W.p, M, N, 1, h->stream);  // A^H, N x M
    TRY(qr_factor<T>(h, h->W.p, N, M));
    TRY(ensure(h, h->X, h->csz * (size_t)k * M));
    launch_qr_r_extract<T>(h->qr_a.p, N, k, M, 1, h->X.p, h->stream);  // conj(R') (k x M)
    launch_qr_eye<T>(N, k, h->W.p, h->stream);
    LAUNCHCHK(h);
    TRY(qr_apply_q<T>(h, h->W.p, N, M, k));  // Q' (N x k)
    TRY(ensure(h, h->site[c], h->csz * (size_t)k * N));
    TRY(ensure(h, h->spare, h->csz * (size_t)P * k));
    TRY(reorth_reserve<T>(h, N, k, P));
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * P * (double)M * k,
                     (double)h->csz * ((double)P * M + (double)M * k + (double)P * k));
        launch_to_colmajor<T>(h->W.p, h->site[c].p, k, N, 1, h->stream);  // Q'^H, row-major (k, N)
        // (A_{c-1} R'^H)^T = conj(R') A_{c-1}^T in column-major terms: row-major (P, k)
        TRY(blas_gemm<T>(h, 'N', 'N', k, P, M, 1.0, h->X.p, k, h->site[c - 1].p, M, 0.0,
                         h->spare.p, k));
    }
    LAUNCHCHK(h);
    TRY(commit_spare(h, h->site[c - 1], h->csz * (size_t)P * k));
    TRY(reorth<T>(h, false, h->site[c].p, N, k, h->site[c - 1].p, P));
    h->bond[c] = k;
    h->center = c - 1;
    return EA_OK;
}

// Centre moves by Cholesky QR2 (Sec. III: A_c = Q R, Q the new site, R
// absorbed into the neighbour; no rank dropped), in FP64 whatever the working
// precision.  With X the site matrix: G = X^H X = R1^H R1, Q1 = X R1^{-1};
// again on Q1: Q = Q1 R2^{-1}, R = R2 R1.  Every product is a matrix-core
// GEMM and the Cholesky factorisations are blocked (k_chol.hip).  A pivot
// below 1e-14 of the largest diagonal entry (a condition number of X above
// about 1e7, or a numerically rank-deficient site) abandons the move before
// the state is touched and the Jacobi SVD move runs instead.
constexpr double CHOLQR_PIVOT_REL = 1e-14;

// Orthogonality (||Q^H Q - I||_F) at which one Cholesky QR pass suffices: far
// below the working precision's rounding (Q is stored in it), 1e-8 for FP32
// sites and 1e-13 for FP64 sites.
template <typename T>
constexpr double cholqr_skip_tol() { return sizeof(T) == 4 ? 1e-8 : 1e-13; }

// Cholesky QR on the FP64 matrix X (rows x cols, row-major, rows >= cols)
// when `cols_orth` (Q has orthonormal columns, X = Q R), else on X (rows x
// cols, cols >= rows) with orthonormal rows (X = R^H Q).  The first pass's Q1
// is checked through the next pass's Gram matrix G2 = Q1^H Q1 (or Q1 Q1^H):
// when ||G2 - I||_F <= skip_tol, Q1 and R1 are kept (one pass, one Cholesky);
// otherwise G2 is factored as well (Cholesky QR2).  Q is left in cq_x, R in
// cq_g (cols x cols or rows x rows).  Returns 1 if a Cholesky broke down
// (state untouched), 0 on success, < 0 on error.
inline int cholqr2(ea_mps *h, const double *X, int rows, int cols, bool cols_orth,
                   double skip_tol) {
    const int n = cols_orth ? cols : rows;  // order of the Gram matrix
    const size_t nx = (size_t)rows * cols, nn = (size_t)n * n;
    TRY(ensure(h, h->cq_q, 16 * nx));
    TRY(ensure(h, h->cq_x, 16 * nx));
    TRY(ensure(h, h->cq_g, 16 * nn));
    TRY(ensure(h, h->cq_r1, 16 * nn));
    TRY(ensure(h, h->cq_r2, 16 * nn));
    TRY(ensure(h, h->cq_ri, 16 * nn));
    TRY(ensure(h, h->cq_t, 16 * nn));
    TRY(ensure(h, h->cq_misc, 256 + 8 * (size_t)((n + 3) / 4)));
    double *dmax = (double *)h->cq_misc.p;
    double *fro2 = dmax + 1;
    int *flag = (int *)((char *)h->cq_misc.p + 64);
    double *part = (double *)((char *)h->cq_misc.p + 256);
    launch_fill_int(flag, 1, 0, h->stream);
    const double fl_gram = 8.0 * (double)nx * n, fl_chol = 8.0 * (double)nn * n;
    auto gram = [&](const void *src) {
        if (cols_orth)  // G = X^H X
            launch_zgemm<double>(1, 0, n, n, rows, 1.0, 0.0, src, cols, src, cols, 0.0, 0.0,
                                 h->cq_g.p, n, h->stream);
        else  // G = X X^H
            launch_zgemm<double>(0, 1, n, n, cols, 1.0, 0.0, src, cols, src, cols, 0.0, 0.0,
                                 h->cq_g.p, n, h->stream);
    };
    auto factor_apply = [&](const void *src, void *Rk, void *dst) {
        launch_cholesky_inv(h->cq_g.p, Rk, h->cq_ri.p, h->cq_t.p, n, dmax, CHOLQR_PIVOT_REL,
                            flag, h->stream);
        if (cols_orth)  // Q = X R^{-1}
            launch_zgemm<double>(0, 0, rows, cols, n, 1.0, 0.0, src, cols, h->cq_ri.p, n, 0.0,
                                 0.0, dst, cols, h->stream);
        else  // Q = R^{-H} X
            launch_zgemm<double>(1, 0, rows, cols, n, 1.0, 0.0, h->cq_ri.p, n, src, cols, 0.0,
                                 0.0, dst, cols, h->stream);
    };
    {
        ProfScope ps(h, EA_K_QR, 2.0 * fl_gram + fl_chol, 16.0 * (3.0 * nx + 3.0 * nn));
        gram(X);
        factor_apply(X, h->cq_r1.p, h->cq_q.p);
        gram(h->cq_q.p);  // G2 of Q1
        launch_offident_fro2(h->cq_g.p, n, part, fro2, h->stream);
    }
    LAUNCHCHK(h);
    HIPCHK(h, hipMemcpyAsync(h->int_host, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->dbl_host, fro2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    if (h->int_host[0] != 0) return 1;
    if (std::sqrt(h->dbl_host[0]) <= skip_tol) {  // Q1 orthonormal enough: one pass
        std::swap(h->cq_q, h->cq_x);
        std::swap(h->cq_g, h->cq_r1);
        h->n_cholqr_single += 1;
        return 0;
    }
    {
        ProfScope ps(h, EA_K_QR, fl_gram + 2.0 * fl_chol, 16.0 * (2.0 * nx + 3.0 * nn));
        factor_apply(h->cq_q.p, h->cq_r2.p, h->cq_x.p);
        // R = R2 R1 (upper triangular products)
        launch_zgemm<double>(0, 0, n, n, n, 1.0, 0.0, h->cq_r2.p, n, h->cq_r1.p, n, 0.0, 0.0,
                             h->cq_g.p, n, h->stream);
    }
    LAUNCHCHK(h);
    HIPCHK(h, hipMemcpyAsync(h->int_host, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    return h->int_host[0] != 0 ? 1 : 0;
}

// Orthonormal basis of range(Y), Y (rows x cols, column-major FP64, rows >=
// cols): Cholesky QR2 when Y's condition number is below about 1e7; when a
// pivot breaks down, shifted Cholesky QR first (one pass on G + s I with
// s = 11 (rows cols + cols (cols + 1)) 2^-53 trace(G), trace(G) = ||Y||_F^2
// bounding ||Y||_2^2, which keeps the factorisation defined however
// ill-conditioned Y is and leaves a basis of condition number below about
// 1e4), then Cholesky QR2 on that (Fukaya et al., SIAM J. Sci. Comput. 42,
// 2020).  *Q points at the basis (rows x cols, column-major, in cq_x).
// Returns 1 when a pivot still breaks down (Y numerically rank-deficient),
// 0 on success.
inline int orth_cols(ea_mps *h, const double *Y, int rows, int cols, const double **Q) {
    // in the row-major terms of cholqr2: Y is cols x rows with orthonormal rows
    const int n = cols;
    const size_t nx = (size_t)rows * cols, nn = (size_t)n * n;
    int rc = cholqr2(h, Y, n, rows, false, 1e-13);  // ensures the cq_* workspace
    *Q = (const double *)h->cq_x.p;
    if (rc <= 0) return rc;
    TRY(ensure(h, h->tk_q1, 16 * nx));
    double *dmax = (double *)h->cq_misc.p;
    int *flag = (int *)((char *)h->cq_misc.p + 64);
    {
        ProfScope ps(h, EA_K_QR, 8.0 * (double)nx * n * 2 + 8.0 * (double)nn * n,
                     16.0 * (3.0 * nx + 3.0 * nn));
        launch_zgemm<double>(0, 1, n, n, rows, 1.0, 0.0, Y, rows, Y, rows, 0.0, 0.0, h->cq_g.p, n,
                             h->stream);
        const double rel = 11.0 * ((double)rows * cols + (double)cols * (cols + 1)) *
                           std::ldexp(1.0, -53);
        launch_shift_diag(h->cq_g.p, n, rel, h->stream);
        launch_cholesky_inv(h->cq_g.p, h->cq_r1.p, h->cq_ri.p, h->cq_t.p, n, dmax,
                            CHOLQR_PIVOT_REL, flag, h->stream);
        launch_zgemm<double>(1, 0, n, rows, n, 1.0, 0.0, h->cq_ri.p, n, Y, rows, 0.0, 0.0,
                             h->tk_q1.p, rows, h->stream);
    }
    LAUNCHCHK(h);
    rc = cholqr2(h, (const double *)h->tk_q1.p, n, rows, false, 1e-13);
    *Q = (const double *)h->cq_x.p;
    return rc;
}

// Partial (top-k) factorisation of X = W (mw x nw, column-major, mw >= nw,
// working precision) for a two-site update across a bond of dimension chiM:
// the reading taken and the acceptance rule are documented at EA_OPT_TOPK.
// Every product of the range finder runs in FP64 on the matrix cores:
//   T = ||X||_F^2;  Y = X^H Omega;  q times Y = X^H (X Y);  Q = orth(Y);
//   W64 = X Q (mw x l);  R = max(0, T - ||W64||_F^2);
// then the working-precision Jacobi SVD of W64 (W = U S, V_W), V = Q V_W, and
// the kept rank from the columns' norms with every discarded weight raised by
// R.  When an attempt is accepted, *used = l and W (mw x l), V (nw x l),
// s_raw, perm, s_sorted and the record hold what factor_and_decide leaves
// for a full factorisation; otherwise *used = 0 and W holds X again.
// *attempts counts the subspaces tried.
template <typename T>
int topk_factor(ea_mps *h, int mw, int nw, int chiM, double f_t, int *used, int *attempts) {
    *used = 0;
    *attempts = 0;
    const int p = h->topk_p;
    const int cap = h->chi_max > 0 ? std::min(h->chi_max, nw) : nw;
    long l = (long)std::min(cap, 2 * chiM) + p;
    if (4 * l > 3 * (long)nw) return EA_OK;
    const size_t nx = (size_t)mw * nw;
    const size_t nparts = sumsq_part_doubles();
    TRY(ensure(h, h->tk_x, 16 * nx));
    TRY(ensure(h, h->tk_misc, 8 * (nparts + 8)));
    TRY(ensure(h, h->s_raw, sizeof(double) * nw));
    TRY(ensure(h, h->s_sorted, sizeof(double) * nw));
    TRY(ensure(h, h->perm, sizeof(int) * nw));
    double *sums = (double *)h->tk_misc.p;  // T, ||W64||^2, R
    double *part = sums + 8;
    const double *X = (const double *)h->tk_x.p;
    {
        ProfScope ps(h, EA_K_TOPK, 4.0 * (double)nx, (double)(h->csz + 16) * nx + 16.0 * nx);
        launch_to_c128<T>(h->W.p, (double *)h->tk_x.p, nx, h->stream);
        launch_sumsq(X, nx, part, sums, h->stream);
    }
    for (int a = 0; 4 * l <= 3 * (long)nw; ++a) {
        const int L = (int)l;
        *attempts = a + 1;
        const size_t nml = (size_t)mw * L, nnl = (size_t)nw * L;
        TRY(ensure(h, h->tk_om, 16 * nml));
        TRY(ensure(h, h->tk_y, 16 * nnl));
        TRY(ensure(h, h->tk_w, 16 * nml));
        TRY(ensure(h, h->tk_vj, 16 * (size_t)L * L));
        const unsigned long long base =
            ((unsigned long long)((h->g & 0xFFFFF) * 16 + a)) << 40;
        {
            ProfScope ps(h, EA_K_TOPK, 8.0 * (double)nml * nw, 16.0 * (nx + nml + nnl));
            launch_omega(h->topk_seed, base, nml, (double *)h->tk_om.p, h->stream);
            // Y = X^H Omega (nw x L)
            TRY(blas_gemm<double>(h, 'C', 'N', nw, L, mw, 1.0, X, mw, h->tk_om.p, mw, 0.0,
                                  h->tk_y.p, nw));
        }
        // q times Y <- X^H (X Y), then Q = orth(Y): the power scheme spans the
        // same subspace as orthonormalising after every product; in FP64 the
        // growth of Y's condition number, (s_0 / s_L)^(2q+1), is left to the
        // shifted Cholesky QR, and a block it cannot resolve falls back to
        // the full factorisation
        for (int it = 0; it < h->topk_q; ++it) {
            ProfScope ps(h, EA_K_TOPK, 16.0 * (double)nml * nw,
                         16.0 * (2.0 * nx + 2.0 * nml + 2.0 * nnl));
            // Z = X Y (mw x L), Y = X^H Z (nw x L)
            TRY(blas_gemm<double>(h, 'N', 'N', mw, L, nw, 1.0, X, mw, h->tk_y.p, nw, 0.0,
                                  h->tk_om.p, mw));
            TRY(blas_gemm<double>(h, 'C', 'N', nw, L, mw, 1.0, X, mw, h->tk_om.p, mw, 0.0,
                                  h->tk_y.p, nw));
        }
        const double *Q = nullptr;
        const int rc = orth_cols(h, (const double *)h->tk_y.p, nw, L, &Q);
        if (rc < 0) return rc;
        if (rc == 1) {  // rank-deficient block: the full factorisation
            h->n_topk_fallback += 1;
            break;
        }
        // Q (nw x L, orthonormal, in cq_x) is kept until V = Q V_W
        {
            ProfScope ps(h, EA_K_TOPK, 8.0 * (double)nml * nw + 4.0 * (double)nml,
                         16.0 * (nx + 2.0 * nml + nnl) + (double)h->csz * nml);
            // W64 = X Q (mw x L), R = T - ||W64||^2, W = W64 in the working precision
            TRY(blas_gemm<double>(h, 'N', 'N', mw, L, nw, 1.0, X, mw, Q, nw, 0.0, h->tk_w.p,
                                  mw));
            launch_sumsq((const double *)h->tk_w.p, nml, part, sums + 1, h->stream);
            launch_resid(sums, sums + 1, sums + 2, h->stream);
            launch_from_c128<T>((const double *)h->tk_w.p, h->W.p, nml, h->stream);
        }
        TRY(svd_core<T>(h, mw, L));  // W = U S, V = V_W (L x L)
        {
            ProfScope ps(h, EA_K_TOPK, 8.0 * (double)nnl * L,
                         16.0 * (nnl * 2.0 + (double)L * L) +
                             (double)h->csz * (nnl + (double)L * L));
            // V = Q V_W (nw x L) in FP64, stored in the working precision
            launch_to_c128<T>(h->V.p, (double *)h->tk_vj.p, (size_t)L * L, h->stream);
            TRY(ensure(h, h->tk_q1, 16 * nnl));
            TRY(blas_gemm<double>(h, 'N', 'N', nw, L, L, 1.0, Q, nw, h->tk_vj.p, L, 0.0,
                                  h->tk_q1.p, nw));
            launch_from_c128<T>((const double *)h->tk_q1.p, h->V.p, nnl, h->stream);
        }
        {
            ProfScope ps(h, EA_K_NORMS, 4.0 * (double)nml, (double)h->csz * nml);
            launch_colnorms<T>(h->W.p, mw, L, (double *)h->s_raw.p, h->stream);
        }
        {
            ProfScope ps(h, EA_K_TRUNC, (double)L, 24.0 * L);
            launch_sort_trunc((const double *)h->s_raw.p, L, f_t, h->chi_max, h->tau, 0, 0,
                              (const int *)h->ints.p, (int *)h->perm.p, (double *)h->s_sorted.p,
                              (ea_dev_rec *)h->rec.p, h->stream, sums + 2);
        }
        LAUNCHCHK(h);
        HIPCHK(h, hipMemcpyAsync(h->rec_host, h->rec.p, sizeof(ea_dev_rec),
                                 hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        prof_harvest(h);
        if (h->rec_host->k <= L - p) {
            *used = L;
            h->n_topk += 1;
            return EA_OK;
        }
        l = std::min<long>(nw, 2 * l);
    }
    // the full factorisation runs on X again
    launch_from_c128<T>(X, h->W.p, nx, h->stream);
    LAUNCHCHK(h);
    return EA_OK;
}

// The site matrix of site c (n complex values) in FP64: the tensor itself
// when T is double, else a converted copy in cq_x.
template <typename T>
int site_c128(ea_mps *h, int c, size_t n, const double **out) {
    if (sizeof(T) == 8) {
        *out = (const double *)h->site[c].p;
        return EA_OK;
    }
    TRY(ensure(h, h->cq_x, 16 * n));
    launch_to_c128<T>(h->site[c].p, (double *)h->cq_x.p, n, h->stream);
    *out = (const double *)h->cq_x.p;
    return EA_OK;
}

// The factor R (n x n, FP64 in cq_g) in the working precision: cq_g itself
// for double, else converted into X.
template <typename T>
int r_working(ea_mps *h, int n, const void **out) {
    if (sizeof(T) == 8) {
        *out = h->cq_g.p;
        return EA_OK;
    }
    TRY(ensure(h, h->X, h->csz * (size_t)n * n));
    launch_from_c128<T>((const double *)h->cq_g.p, h->X.p, (size_t)n * n, h->stream);
    *out = h->X.p;
    return EA_OK;
}

// Right: A_c as (chi_l d) x chi_r = Q R; A_c <- Q, A_{c+1} <- R A_{c+1}.
template <typename T>
int move_right_cholqr(ea_mps *h) {
    const int c = h->center, d = h->d;
    const int M = h->bond[c] * d, N = h->bond[c + 1], P = d * h->bond[c + 2];
    if (M < N || N > EA_SORT_MAX) return move_right<T>(h);
    const size_t nx = (size_t)M * N;
    const double *X = nullptr;
    TRY(site_c128<T>(h, c, nx, &X));
    const int rc = cholqr2(h, X, M, N, true, cholqr_skip_tol<T>());
    if (rc < 0) return rc;
    if (rc == 1) {  // ill-conditioned: the SVD move
        h->n_chol_fallback += 1;
        return move_right<T>(h);
    }
    const void *R = nullptr;
    TRY(r_working<T>(h, N, &R));
    TRY(ensure(h, h->spare, h->csz * (size_t)N * P));
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * N * (double)N * P,
                     (double)h->csz * ((double)N * N + 2.0 * (double)N * P));
        launch_from_c128<T>((const double *)h->cq_x.p, h->site[c].p, nx, h->stream);
        launch_zgemm<T>(0, 0, N, P, N, 1.0, 0.0, R, N, h->site[c + 1].p, P, 0.0, 0.0,
                        h->spare.p, P, h->stream);
    }
    LAUNCHCHK(h);
    TRY(commit_spare(h, h->site[c + 1], h->csz * (size_t)N * P));
    h->center = c + 1;
    return EA_OK;
}

// Left: A_c as chi_l x (d chi_r) = R^H Q with orthonormal rows;
// A_c <- Q, A_{c-1} <- A_{c-1} R^H.
template <typename T>
int move_left_cholqr(ea_mps *h) {
    const int c = h->center, d = h->d;
    const int M = h->bond[c], N = d * h->bond[c + 1], P = h->bond[c - 1] * d;
    if (N < M || M > EA_SORT_MAX) return move_left<T>(h);
    const size_t nx = (size_t)M * N;
    const double *X = nullptr;
    TRY(site_c128<T>(h, c, nx, &X));
    const int rc = cholqr2(h, X, M, N, false, cholqr_skip_tol<T>());
    if (rc < 0) return rc;
    if (rc == 1) {
        h->n_chol_fallback += 1;
        return move_left<T>(h);
    }
    const void *R = nullptr;
    TRY(r_working<T>(h, M, &R));
    TRY(ensure(h, h->spare, h->csz * (size_t)P * M));
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * P * (double)M * M,
                     (double)h->csz * ((double)M * M + 2.0 * (double)P * M));
        launch_from_c128<T>((const double *)h->cq_x.p, h->site[c].p, nx, h->stream);
        launch_zgemm<T>(0, 1, P, M, M, 1.0, 0.0, h->site[c - 1].p, M, R, M, 0.0, 0.0,
                        h->spare.p, M, h->stream);
    }
    LAUNCHCHK(h);
    TRY(commit_spare(h, h->site[c - 1], h->csz * (size_t)P * M));
    h->center = c - 1;
    return EA_OK;
}

// Space of an allocation-free call's array used by one centre move is free
// again after it (stream order puts the move's kernels first).
struct ArenaMark {
    ea_mps *h;
    size_t off, nsaved;
    explicit ArenaMark(ea_mps *h_) : h(h_), off(h_->arena_off), nsaved(h_->arena_saved.size()) {}
    ~ArenaMark() {
        if (h->arena) arena_release(h, off, nsaved);
    }
};

template <typename T>
int move_center(ea_mps *h, int j) {
    while (h->center < j) {
        ArenaMark am(h);
        ProfScope ps(h, EA_K_MOVE, 0.0, 0.0);
        if (h->move_kind == 2) TRY(move_right_cholqr<T>(h));
        else if (h->move_kind == 1) TRY(move_right_qr<T>(h));
        else TRY(move_right<T>(h));
    }
    while (h->center > j) {
        ArenaMark am(h);
        ProfScope ps(h, EA_K_MOVE, 0.0, 0.0);
        if (h->move_kind == 2) TRY(move_left_cholqr<T>(h));
        else if (h->move_kind == 1) TRY(move_left_qr<T>(h));
        else TRY(move_left<T>(h));
    }
    return EA_OK;
}

// Two-site update on (i, i+1); dir = +1: centre ends on i+1, -1: on i.
template <typename T>
int apply_2q_impl(ea_mps *h, int i, const double *op, double budget, int dir, double *f_out,
                  int forced_k) {
    if (h->center < i) TRY(move_center<T>(h, i));
    if (h->center > i + 1) TRY(move_center<T>(h, i + 1));
    double f_t = budget >= 0 ? budget : schedule_target(h);
    f_t = std::min(1.0, std::max(f_t, 1e-300));
    const int d = h->d, chiL = h->bond[i], chiM = h->bond[i + 1], chiR = h->bond[i + 2];
    const int M = d * chiL, N = d * chiR;
    const int orient = M >= N ? 0 : 1, mw = std::max(M, N), nw = std::min(M, N);
    if (nw > EA_SORT_MAX) return set_err(EA_ETOOBIG, "two-site matrix too large (%d)", nw);
    TRY(ensure(h, h->W, h->csz * (size_t)mw * nw));
    TRY(ensure(h, h->V, h->csz * (size_t)nw * nw));
    void *G = nullptr;
    TRY(stage<T>(h, op, (size_t)d * d * d * d, &G));
    {
        const double dd = d;
        ProfScope ps(h, EA_K_THETA,
                     8.0 * dd * dd * chiL * (double)chiM * chiR + 8.0 * dd * dd * dd * dd * chiL * (double)chiR,
                     (double)h->csz * (dd * chiL * chiM + dd * chiM * (double)chiR +
                                       dd * dd * chiL * (double)chiR + dd * dd * dd * dd));
        if (sizeof(T) == 4 && h->prec == EA_C64_BF16X3)
            launch_theta_bf16x3(h->site[i].p, h->site[i + 1].p, G, h->W.p, chiL, chiM, chiR, d,
                                orient, h->stream);
        else
            launch_theta_mfma<T>(h->site[i].p, h->site[i + 1].p, G, h->W.p, chiL, chiM, chiR, d,
                                 orient, h->stream);
    }
    LAUNCHCHK(h);
    int sub = 0, att = 0;
    if (h->topk && forced_k <= 0 && nw >= h->topk_min && h->arena == nullptr)
        TRY(topk_factor<T>(h, mw, nw, chiM, f_t, &sub, &att));
    if (sub == 0) TRY(factor_and_decide<T>(h, mw, nw, f_t, 0, forced_k));
    const ea_dev_rec rec = *h->rec_host;
    const int k = rec.k;
    if (!(rec.s0 > 0.0) || !std::isfinite(rec.total))
        return set_err(EA_EINVAL, "the operator annihilates the state (all singular values 0)");
    TRY(ensure(h, h->site[i], h->csz * (size_t)M * k));
    TRY(ensure(h, h->site[i + 1], h->csz * (size_t)k * N));
    const bool right = dir > 0;
    if (right) TRY(reorth_reserve<T>(h, M, k, N));
    else TRY(reorth_reserve<T>(h, N, k, M));
    if (orient == 0) {
        gather<T>(h, h->W.p, M, k, M, 0, right ? -1 : 0, right ? 0 : 1, 1, h->site[i].p);
        gather<T>(h, h->V.p, N, k, N, 1, right ? 1 : 0, right ? 1 : 0, 0, h->site[i + 1].p);
    } else {
        gather<T>(h, h->V.p, M, k, M, 0, right ? 0 : 1, right ? 0 : 1, 1, h->site[i].p);
        gather<T>(h, h->W.p, N, k, N, 1, right ? 0 : -1, right ? 1 : 0, 0, h->site[i + 1].p);
    }
    LAUNCHCHK(h);
    if (right)
        TRY(reorth<T>(h, true, h->site[i].p, M, k, h->site[i + 1].p, N));
    else
        TRY(reorth<T>(h, false, h->site[i + 1].p, N, k, h->site[i].p, M));
    h->bond[i + 1] = k;
    h->center = right ? i + 1 : i;
    h->lnP += rec.lnf;
    if (h->kind == EA_MIXED && rec.kept2 > 0) h->lnS += 0.5 * std::log(rec.kept2);
    ea_gate_record r;
    r.gate = h->g;
    r.site = i;
    r.chi_l = chiL;
    r.chi_m = chiM;
    r.chi_r = chiR;
    r.k = k;
    r.k_f = rec.k_f;
    r.sweeps = rec.sweeps;
    r.capped = rec.capped;
    r.subspace = sub;
    r.attempts = att;
    r.f_t = f_t;
    r.f = rec.f;
    r.total = rec.total;
    r.lnP = h->lnP;
    r.lnS = h->lnS;
    h->log.push_back(r);
    h->g += 1;
    if (f_out) *f_out = rec.f;
    if (rec.capped) return set_err(EA_WARN_CAPPED, "chi_max bound at gate %ld", (long)r.gate);
    if (!rec.converged) return set_err(EA_WARN_NOCONV, "Jacobi did not converge");
    return EA_OK;
}

// Two-site update in the layer-parallel gauge (Vidal form, Hastings'
// division-free update; gates of one layer touch disjoint sites and bonds):
//   C = G (B_i B_{i+1}),  Theta = diag(Lambda_i) C = X S Y^H,  k kept (Sec. VI),
//   B_{i+1} <- Y_k^H,  B_i <- C Y_k / ||s_k||,  Lambda_{i+1} <- s_k / ||s_k||,
// f = sum_kept s^2 / sum s^2 (Eqs. 10-11; exact while the form is exact).
// The device work of one gate runs on the workspace and stream of `w` (the
// state's own, or a worker's for gates run side by side); it writes only
// sites i, i+1 and bond value i+1 of the state h.  The scalar bookkeeping
// (bond, estimate, log) is vidal_finish, applied in gate order.
struct VidalOut {
    ea_dev_rec rec{};
    int chi_l = 0, chi_m = 0, chi_r = 0;
    double f_t = 1.0;
};

template <typename T>
int vidal_gate(ea_mps *h, ea_mps *w, int i, const double *op, double f_t, int forced_k,
               VidalOut *out) {
    f_t = std::min(1.0, std::max(f_t, 1e-300));
    const int d = h->d, chiL = h->bond[i], chiM = h->bond[i + 1], chiR = h->bond[i + 2];
    const int M = d * chiL, N = d * chiR;
    const int orient = M >= N ? 0 : 1, mw = std::max(M, N), nw = std::min(M, N);
    if (nw > EA_SORT_MAX) return set_err(EA_ETOOBIG, "two-site matrix too large (%d)", nw);
    TRY(ensure(w, w->W, w->csz * (size_t)mw * nw));
    TRY(ensure(w, w->V, w->csz * (size_t)nw * nw));
    TRY(ensure(w, w->cbuf, w->csz * (size_t)mw * nw));
    void *G = nullptr;
    TRY(stage<T>(w, op, (size_t)d * d * d * d, &G));
    {
        const double dd = d;
        ProfScope ps(w, EA_K_THETA,
                     8.0 * dd * dd * chiL * (double)chiM * chiR + 8.0 * dd * dd * dd * dd * chiL * (double)chiR,
                     (double)w->csz * (dd * chiL * chiM + dd * chiM * (double)chiR +
                                       dd * dd * chiL * (double)chiR + dd * dd * dd * dd));
        if (sizeof(T) == 4 && w->prec == EA_C64_BF16X3)
            launch_theta_bf16x3(h->site[i].p, h->site[i + 1].p, G, w->W.p, chiL, chiM, chiR, d,
                                orient, w->stream);
        else
            launch_theta_mfma<T>(h->site[i].p, h->site[i + 1].p, G, w->W.p, chiL, chiM, chiR, d,
                                 orient, w->stream);
    }
    {
        ProfScope ps(w, EA_K_OTHER, 0.0, 3.0 * (double)w->csz * mw * (double)nw);
        HIPCHK(w, hipMemcpyAsync(w->cbuf.p, w->W.p, w->csz * (size_t)mw * nw,
                                 hipMemcpyDeviceToDevice, w->stream));
        launch_scale_lambda<T>(w->W.p, mw, nw, orient, (const double *)h->lam[i].p, d, w->stream);
    }
    LAUNCHCHK(w);
    TRY(factor_and_decide<T>(w, mw, nw, f_t, 0, forced_k));  // syncs w's stream
    const ea_dev_rec rec = *w->rec_host;
    const int k = rec.k;
    if (!(rec.s0 > 0.0) || !std::isfinite(rec.total))
        return set_err(EA_EINVAL, "the operator annihilates the state (all singular values 0)");
    // the state's buffers of sites i, i+1 were last read by this gate's
    // contraction, which has completed (w's stream was synchronised above)
    TRY(ensure(h, h->site[i], h->csz * (size_t)M * k));
    TRY(ensure(h, h->site[i + 1], h->csz * (size_t)k * N));
    TRY(ensure(h, h->lam[i + 1], sizeof(double) * (size_t)k));
    TRY(ensure(w, w->ybuf, w->csz * (size_t)N * k));
    TRY(reorth_reserve<T>(w, N, k, M));
    // Y_k (N x k, row-major) and B_{i+1} = Y_k^H: the right singular vectors
    // are V's columns (orient 0) or W's columns over s (orient 1, W = Theta^H)
    const void *ysrc = orient == 0 ? w->V.p : w->W.p;
    const int es = orient == 0 ? 0 : -1;
    gather<T>(w, ysrc, N, k, N, 0, es, 0, 1, w->ybuf.p);
    gather<T>(w, ysrc, N, k, N, 1, es, 0, 0, h->site[i + 1].p);
    {
        // B_i = C Y_k / ||s_k||; cbuf holds C column-major (orient 0: its
        // row-major view is C^T) or C^H column-major (orient 1: view conj(C))
        ProfScope ps(w, EA_K_GEMM, 8.0 * M * (double)N * k,
                     (double)w->csz * ((double)M * N + (double)N * k + (double)M * k));
        launch_zgemm<T>(orient == 0 ? 2 : 3, 0, M, k, N, rec.scale, 0.0, w->cbuf.p,
                        orient == 0 ? M : N, w->ybuf.p, k, 0.0, 0.0, h->site[i].p, k, w->stream);
    }
    launch_vidal_lambda((const double *)w->s_sorted.p, (const ea_dev_rec *)w->rec.p, k,
                        (double *)h->lam[i + 1].p, w->stream);
    LAUNCHCHK(w);
    TRY(reorth<T>(w, false, h->site[i + 1].p, N, k, h->site[i].p, M));
    out->rec = rec;
    out->chi_l = chiL;
    out->chi_m = chiM;
    out->chi_r = chiR;
    out->f_t = f_t;
    return EA_OK;
}

// Bookkeeping of one layer-parallel update (in gate order).
inline int vidal_finish(ea_mps *h, int i, const VidalOut &o, double *f_out) {
    const ea_dev_rec &rec = o.rec;
    h->bond[i + 1] = rec.k;
    h->lnP += rec.lnf;
    if (h->kind == EA_MIXED && rec.kept2 > 0) h->lnS += 0.5 * std::log(rec.kept2);
    ea_gate_record r;
    r.gate = h->g;
    r.site = i;
    r.chi_l = o.chi_l;
    r.chi_m = o.chi_m;
    r.chi_r = o.chi_r;
    r.k = rec.k;
    r.k_f = rec.k_f;
    r.sweeps = rec.sweeps;
    r.capped = rec.capped;
    r.subspace = 0;
    r.attempts = 0;
    r.f_t = o.f_t;
    r.f = rec.f;
    r.total = rec.total;
    r.lnP = h->lnP;
    r.lnS = h->lnS;
    h->log.push_back(r);
    h->g += 1;
    if (f_out) *f_out = rec.f;
    if (rec.capped) return set_err(EA_WARN_CAPPED, "chi_max bound at gate %ld", (long)r.gate);
    if (!rec.converged) return set_err(EA_WARN_NOCONV, "Jacobi did not converge");
    return EA_OK;
}

// One gate on the state's own stream.
template <typename T>
int vidal_2q_impl(ea_mps *h, int i, const double *op, double f_t, double *f_out, int forced_k) {
    VidalOut o;
    TRY(vidal_gate<T>(h, h, i, op, f_t, forced_k, &o));
    return vidal_finish(h, i, o, f_out);
}

// Bond values of a product state in the layer-parallel gauge: every bond 1.
inline int vidal_reset_lambdas(ea_mps *h) {
    h->lam.resize(h->n + 1);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const double one = 1.0;
    for (int b = 0; b <= h->n; ++b) {
        TRY(ensure(h, h->lam[b], sizeof(double)));
        HIPCHK(h, hipMemcpy(h->lam[b].p, &one, sizeof(double), hipMemcpyHostToDevice));
    }
    return EA_OK;
}

template <typename T>
int apply_1q_impl(ea_mps *h, int site, const double *op) {
    if (!is_unitary(op, h->d)) TRY(move_center<T>(h, site));
    void *g = nullptr;
    TRY(stage<T>(h, op, (size_t)h->d * h->d, &g));
    launch_apply1<T>(h->site[site].p, h->site[site].p, g, h->bond[site], h->d, h->bond[site + 1],
                     h->stream);
    LAUNCHCHK(h);
    return EA_OK;
}

// <O> for a pure state at the centre (Eq. 6).
template <typename T>
int expect_pure(ea_mps *h, int site, int width, const double *op, double *res3) {
    TRY(move_center<T>(h, site));
    const int d = h->d;
    double *dev3 = (double *)h->out3.p;
    double *partial = (double *)h->partial.p;
    int nblk;
    if (width == 1) {
        const size_t len = (size_t)h->bond[site] * d * h->bond[site + 1];
        TRY(ensure(h, h->X, h->csz * len));
        void *g = nullptr;
        TRY(stage<T>(h, op, (size_t)d * d, &g));
        launch_apply1<T>(h->site[site].p, h->X.p, g, h->bond[site], d, h->bond[site + 1],
                         h->stream);
        nblk = launch_cdot<T>(h->site[site].p, h->X.p, len, partial, 1024, h->stream);
    } else {
        const int chiL = h->bond[site], chiM = h->bond[site + 1], chiR = h->bond[site + 2];
        const size_t len = (size_t)d * chiL * d * chiR;
        TRY(ensure(h, h->X, h->csz * len));
        TRY(ensure(h, h->X2, h->csz * len));
        double eye[32] = {0};
        for (int a = 0; a < 4; ++a) eye[2 * (a * 4 + a)] = 1.0;
        void *gi = nullptr, *go = nullptr;
        TRY(stage<T>(h, eye, 16, &gi));
        TRY(stage<T>(h, op, 16, &go));
        launch_theta<T>(h->site[site].p, h->site[site + 1].p, gi, h->X.p, chiL, chiM, chiR, d, 0,
                        h->stream);
        launch_theta<T>(h->site[site].p, h->site[site + 1].p, go, h->X2.p, chiL, chiM, chiR, d, 0,
                        h->stream);
        nblk = launch_cdot<T>(h->X.p, h->X2.p, len, partial, 1024, h->stream);
    }
    launch_cdot_final(partial, nblk, dev3, h->stream);
    LAUNCHCHK(h);
    HIPCHK(h, hipMemcpyAsync(res3, dev3, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return EA_OK;
}

// All terms of a mixed state: Tr(rho O) / Tr(rho) with left/right transfer
// vectors built once (identity weights vec(I) = [1, 0, 0, 1]).
template <typename T>
int expect_mixed(ea_mps *h, int n_terms, const int *sites, const int *widths, const double *ops,
                 double *out) {
    const int n = h->n, d = h->d;
    std::vector<size_t> offL(n + 1), offR(n + 1);
    size_t tot = 0;
    for (int j = 0; j <= n; ++j) {
        offL[j] = tot;
        tot += h->bond[j];
    }
    for (int j = 0; j <= n; ++j) {
        offR[j] = tot;
        tot += h->bond[j];
    }
    const size_t term_off = tot;
    tot += (size_t)n_terms + 1;  // terms, then Tr(rho)
    int maxchi = *std::max_element(h->bond.begin(), h->bond.end());
    TRY(ensure(h, h->envb, h->csz * tot));
    TRY(ensure(h, h->tmp, h->csz * (size_t)d * maxchi + 64));
    TRY(ensure(h, h->X, h->csz * (size_t)maxchi + 64));
    char *E = (char *)h->envb.p;
    auto at = [&](size_t off) { return (void *)(E + off * h->csz); };
    const double one[2] = {1.0, 0.0};
    double vid[8] = {1, 0, 0, 0, 0, 0, 1, 0};
    void *d_one = nullptr, *d_vid = nullptr;
    TRY(stage<T>(h, one, 1, &d_one));
    TRY(stage<T>(h, vid, 4, &d_vid));
    HIPCHK(h, hipMemcpyAsync(at(offL[0]), d_one, 2 * sizeof(T), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(at(offR[n]), d_one, 2 * sizeof(T), hipMemcpyDeviceToDevice, h->stream));
    for (int j = 0; j < n; ++j)
        launch_env_left<T>(at(offL[j]), h->site[j].p, d_vid, at(offL[j + 1]), h->bond[j], d,
                           h->bond[j + 1], h->stream);
    for (int j = n - 1; j >= 0; --j)
        launch_env_right<T>(h->site[j].p, d_vid, at(offR[j + 1]), at(offR[j]), h->bond[j], d,
                            h->bond[j + 1], h->stream);
    LAUNCHCHK(h);
    size_t opoff = 0;
    for (int t = 0; t < n_terms; ++t) {
        const int s = sites[t], w = widths[t];
        const double *o = ops + 2 * opoff;
        opoff += w == 1 ? 4 : 16;
        void *e_out = h->X.p;
        if (w == 1) {
            double wg[8];  // weight at p = 2 s + s' is O[s', s]
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const int p = 2 * a + b;
                    wg[2 * p] = o[2 * (b * 2 + a)];
                    wg[2 * p + 1] = o[2 * (b * 2 + a) + 1];
                }
            void *dw = nullptr;
            TRY(stage<T>(h, wg, 4, &dw));
            launch_env_left<T>(at(offL[s]), h->site[s].p, dw, e_out, h->bond[s], d,
                               h->bond[s + 1], h->stream);
        } else {
            double w2[32];  // W2[p1, p2] = O[(s1' s2'), (s1 s2)]
            for (int s1 = 0; s1 < 2; ++s1)
                for (int s1p = 0; s1p < 2; ++s1p)
                    for (int s2 = 0; s2 < 2; ++s2)
                        for (int s2p = 0; s2p < 2; ++s2p) {
                            const int p1 = 2 * s1 + s1p, p2 = 2 * s2 + s2p;
                            const int src = (2 * s1p + s2p) * 4 + (2 * s1 + s2);
                            w2[2 * (p1 * 4 + p2)] = o[2 * src];
                            w2[2 * (p1 * 4 + p2) + 1] = o[2 * src + 1];
                        }
            void *dw = nullptr;
            TRY(stage<T>(h, w2, 16, &dw));
            launch_env_left2<T>(at(offL[s]), h->site[s].p, h->site[s + 1].p, dw, h->tmp.p, e_out,
                                h->bond[s], d, h->bond[s + 1], h->bond[s + 2], h->stream);
        }
        // plain dot with the right transfer vector: treat it as a chi x 1 x 1 tensor
        const int chi = h->bond[s + w];
        launch_env_left<T>(e_out, at(offR[s + w]), d_one, at(term_off + t), chi, 1, 1, h->stream);
    }
    LAUNCHCHK(h);
    // results: Tr(rho) = L_N[0]; terms
    const size_t nres = n_terms + 1;
    TRY(ensure(h, h->c128, sizeof(double) * 2 * nres));
    HIPCHK(h, hipMemcpyAsync(at(term_off + n_terms), at(offL[n]), h->csz, hipMemcpyDeviceToDevice,
                             h->stream));
    launch_to_c128<T>(at(term_off), (double *)h->c128.p, nres, h->stream);
    std::vector<double> host(2 * nres);
    HIPCHK(h, hipMemcpyAsync(host.data(), h->c128.p, sizeof(double) * 2 * nres,
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const double tr = host[2 * n_terms], ti = host[2 * n_terms + 1];
    const double den = tr * tr + ti * ti;
    for (int t = 0; t < n_terms; ++t) {
        const double a = host[2 * t], b = host[2 * t + 1];
        out[2 * t] = (a * tr + b * ti) / den;
        out[2 * t + 1] = (b * tr - a * ti) / den;
    }
    return EA_OK;
}

template <typename T>
int to_vector_impl(ea_mps *h, double *out, size_t out_len) {
    const int n = h->n, d = h->d;
    size_t total = 1;
    for (int j = 0; j < n; ++j) total *= (size_t)d;
    if (out_len < total) return set_err(EA_ETOOBIG, "output needs %zu complex entries", total);
    // chain contraction: cur (rows x chi_j) * A_j (chi_j x d chi_{j+1})
    size_t maxsz = total, rows_j = 1;
    for (int j = 0; j < n; ++j) {
        rows_j *= (size_t)d;
        maxsz = std::max(maxsz, rows_j * (size_t)h->bond[j + 1]);
    }
    TRY(ensure(h, h->X, h->csz * maxsz));
    TRY(ensure(h, h->X2, h->csz * maxsz));
    size_t rows = d;
    HIPCHK(h, hipMemcpyAsync(h->X.p, h->site[0].p, h->csz * d * h->bond[1],
                             hipMemcpyDeviceToDevice, h->stream));
    void *cur = h->X.p, *nxt = h->X2.p;
    for (int j = 1; j < n; ++j) {
        const int cl = h->bond[j], cr = h->bond[j + 1];
        launch_gemm<T>(cur, h->site[j].p, nxt, (int)rows, d * cr, cl, cl, d * cr, d * cr,
                       h->stream);
        rows *= d;
        std::swap(cur, nxt);
    }
    LAUNCHCHK(h);
    void *res = cur;
    if (h->kind == EA_MIXED) {
        // trace = sum over rows of rho's diagonal: use the transfer vectors
        launch_vec_to_rho<T>(cur, nxt, n, h->stream);
        res = nxt;
        const size_t dim = (size_t)1 << n;
        // Tr(rho) from the diagonal: diagonal entries have stride dim+1
        TRY(ensure(h, h->tmp, h->csz * dim));
        // gather the diagonal with a strided copy
        HIPCHK(h, hipMemcpy2DAsync(h->tmp.p, h->csz, res, h->csz * (dim + 1), h->csz, dim,
                                   hipMemcpyDeviceToDevice, h->stream));
        TRY(ensure(h, h->envb, h->csz * dim));
        std::vector<double> ones(2 * dim, 0.0);
        for (size_t i = 0; i < dim; ++i) ones[2 * i] = 1.0;
        void *d1 = nullptr;
        if (dim * 2 * sizeof(T) * 2 <= h->stage_cap) {
            TRY(stage<T>(h, ones.data(), dim, &d1));
        } else {
            return set_err(EA_ETOOBIG, "density matrix too large");
        }
        int nb = launch_cdot<T>(d1, h->tmp.p, dim, (double *)h->partial.p, 1024, h->stream);
        launch_cdot_final((double *)h->partial.p, nb, (double *)h->out3.p, h->stream);
        double tr[3];
        HIPCHK(h, hipMemcpyAsync(tr, h->out3.p, 3 * sizeof(double), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        const double den = tr[0] * tr[0] + tr[1] * tr[1];
        launch_scale<T>(res, total, tr[0] / den, -tr[1] / den, h->stream);
    }
    if (h->f64) {
        HIPCHK(h, hipMemcpyAsync(out, res, 16 * total, hipMemcpyDeviceToHost, h->stream));
    } else {
        TRY(ensure(h, h->c128, 16 * total));
        launch_to_c128<T>(res, (double *)h->c128.p, total, h->stream);
        HIPCHK(h, hipMemcpyAsync(out, h->c128.p, 16 * total, hipMemcpyDeviceToHost, h->stream));
    }
    LAUNCHCHK(h);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return EA_OK;
}

template <typename T>
int load_impl(ea_mps *h, const int *dims, const double *data, int center) {
    const int n = h->n, d = h->d;
    size_t off = 0;
    for (int j = 0; j < n; ++j) {
        const size_t sz = (size_t)dims[j] * d * dims[j + 1];
        TRY(ensure(h, h->site[j], h->csz * sz));
        TRY(ensure(h, h->c128, 16 * sz));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        HIPCHK(h, hipMemcpy(h->c128.p, data + 2 * off, 16 * sz, hipMemcpyHostToDevice));
        launch_from_c128<T>((const double *)h->c128.p, h->site[j].p, sz, h->stream);
        LAUNCHCHK(h);
        off += sz;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int j = 0; j <= n; ++j) h->bond[j] = dims[j];
    h->center = center;
    return EA_OK;
}

template <typename T>
int get_site_impl(ea_mps *h, int site, double *out) {
    const size_t sz = (size_t)h->bond[site] * h->d * h->bond[site + 1];
    TRY(ensure(h, h->c128, 16 * sz));
    launch_to_c128<T>(h->site[site].p, (double *)h->c128.p, sz, h->stream);
    LAUNCHCHK(h);
    HIPCHK(h, hipMemcpyAsync(out, h->c128.p, 16 * sz, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return EA_OK;
}

}  // namespace ea
