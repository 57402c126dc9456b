// Host side of the C ABI declared in include/ea_mps.h: handle, validation,
// device memory, orthogonality-centre bookkeeping, the target schedule and
// the orchestration of the kernels of one two-site update.
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

namespace {

thread_local std::string g_err;

int set_err(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct ea_mps {
    int n = 0, d = 2, kind = EA_PURE, prec = EA_C128, chi_max = 0;
    bool f64 = true;
    size_t csz = 16;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<int> bond;  // n+1 entries, bond[0] = bond[n] = 1
    std::vector<DevBuf> site;
    DevBuf spare;
    int center = 0;
    double lnP = 0.0, lnS = 0.0;
    long g = 0;
    bool has_sched = false;
    double f_min = 1.0;
    long n_total = 1;
    int strategy = EA_GLOBAL;
    // workspace
    DevBuf jpart, jmat, jflag;
    int inner_round = 1, jkernel = 0, rot_threads = 512;
    DevBuf W, V, X, X2, s_raw, s_sorted, perm, rec, ints, partial, envb, tmp, out3, c128;
    ea_dev_rec *rec_host = nullptr;
    int *int_host = nullptr;
    double *dbl_host = nullptr;
    char *stage_host = nullptr;
    size_t stage_cap = 0, stage_off = 0;
    DevBuf stage_dev;
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
        double flops, bytes;
    };
    bool prof_on = false;
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[EA_K_COUNT] = {0}, prof_flops[EA_K_COUNT] = {0}, prof_bytes[EA_K_COUNT] = {0};
    long prof_cnt[EA_K_COUNT] = {0};
};

namespace {

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

hipEvent_t ev_get(ea_mps *h) {
    if (!h->prof_pool.empty()) {
        hipEvent_t e = h->prof_pool.back();
        h->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Times the launches enqueued during its lifetime with an event pair.
struct ProfScope {
    ea_mps *h;
    hipEvent_t a = nullptr;
    int fam;
    double fl, by;
    ProfScope(ea_mps *h_, int fam_, double fl_, double by_) : h(h_), fam(fam_), fl(fl_), by(by_) {
        if (h->prof_on && (a = ev_get(h)) != nullptr) (void)hipEventRecord(a, h->stream);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = ev_get(h);
        if (!b) return;
        (void)hipEventRecord(b, h->stream);
        h->prof_pending.push_back({a, b, fam, fl, by});
    }
};

// Accumulate completed event pairs (call after a stream synchronisation).
void prof_harvest(ea_mps *h) {
    for (auto &r : h->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            h->prof_ms[r.fam] += ms;
            h->prof_cnt[r.fam] += 1;
            h->prof_flops[r.fam] += r.flops;
            h->prof_bytes[r.fam] += r.bytes;
        }
        h->prof_pool.push_back(r.a);
        h->prof_pool.push_back(r.b);
    }
    h->prof_pending.clear();
}

int ensure(ea_mps *h, DevBuf &b, size_t bytes) {
    if (bytes <= b.bytes) return EA_OK;
    if (b.p) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        HIPCHK(h, hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max(bytes, b.bytes + b.bytes / 4);
    want = (want + 255) & ~size_t(255);
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return set_err(EA_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    b.bytes = want;
    return EA_OK;
}

int check(const ea_mps *h) {
    if (!h) return set_err(EA_EINVAL, "null handle");
    if (h->poisoned) return set_err(EA_EHIP, "handle poisoned by an earlier HIP error");
    return EA_OK;
}

bool finite_cplx(const double *p, size_t n) {
    for (size_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// ||A^H A - I||_max for a k x k complex matrix given as interleaved doubles.
bool is_unitary(const double *a, int k) {
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

double schedule_target(const ea_mps *h) {
    if (!h->has_sched) return 1.0;
    const double n = (double)h->n_total, g = (double)h->g;
    double ft;
    if (h->strategy == EA_NAIVE) {
        ft = std::pow(h->f_min, 1.0 / n);
    } else if (h->strategy == EA_GLOBAL) {
        double left = n - g;
        ft = left <= 0 ? 1.0 : std::exp((std::log(h->f_min) - h->lnP) / left);
    } else {
        ft = std::exp(std::log(h->f_min) * (g + 1) / n - h->lnP);
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
    int w = h->block > 0 ? h->block : (three ? 16 : (n <= 256 ? 8 : 16));
    if (2 * w > 64) w = 32;
    const int ncmax = 2 * w <= 16 ? 16 : (2 * w <= 32 ? 32 : 64);
    int nb = (n + w - 1) / w;
    nb += nb & 1;
    if (three) {
        TRY(ensure(h, h->jpart, h->csz * jacobi_round3_partial_elems(m, n, w)));
        TRY(ensure(h, h->jmat, h->csz * jacobi_round3_j_elems(n, w)));
        TRY(ensure(h, h->jflag, sizeof(int) * (nb / 2 + 1)));
    }
    int sweeps = 0, conv = 0;
    for (int sw = 0; sw < h->max_sweeps; ++sw) {
        launch_fill_int(counter, 1, 0, h->stream);
        for (int rnd = 0; rnd < nb - 1; ++rnd) {
            // algorithmic work of one round: every column block pair forms its
            // Hermitian Gram matrix (4 m nc^2 flops) and rotates its nc columns of W
            // and V (8 (m + n) nc^2 flops)
            double fl2 = 0.0;
            for (int p = 0; p < nb / 2; ++p) {
                const int a = p == 0 ? 0 : (p - 1 + rnd) % (nb - 1) + 1;
                const int bq = nb - 1 - p;
                const int b = bq == 0 ? 0 : (bq - 1 + rnd) % (nb - 1) + 1;
                const int nc = std::max(0, std::min(w, n - a * w)) + std::max(0, std::min(w, n - b * w));
                fl2 += (double)nc * nc;
            }
            if (three) {
                {
                    ProfScope ps(h, EA_K_JGRAM, 4.0 * m * fl2, c * m * (double)n);
                    launch_jacobi_part<T>(0, h->W.p, m, h->V.p, n, w, nb, rnd, tol, h->inner_round,
                                          h->jpart.p, h->jmat.p, (int *)h->jflag.p, counter,
                                          h->rot_threads, h->stream);
                }
                {
                    ProfScope ps(h, EA_K_JROT, 0.0, c * (nb / 2) * 64.0 * 64.0);
                    launch_jacobi_part<T>(1, h->W.p, m, h->V.p, n, w, nb, rnd, tol, h->inner_round,
                                          h->jpart.p, h->jmat.p, (int *)h->jflag.p, counter,
                                          h->rot_threads, h->stream);
                }
                {
                    ProfScope ps(h, EA_K_JAPPLY, 8.0 * (m + n) * fl2, 2.0 * c * (m + n) * (double)n);
                    launch_jacobi_part<T>(2, h->W.p, m, h->V.p, n, w, nb, rnd, tol, h->inner_round,
                                          h->jpart.p, h->jmat.p, (int *)h->jflag.p, counter,
                                          h->rot_threads, h->stream);
                }
            } else {
                ProfScope ps(h, EA_K_JFUSED, (4.0 * m + 8.0 * (m + n)) * fl2,
                             2.0 * c * (m + n) * (double)n);
                launch_jacobi_round<T>(h->W.p, m, h->V.p, n, w, nb, rnd, tol, 6, ncmax, counter,
                                       h->stream);
            }
        }
        LAUNCHCHK(h);
        HIPCHK(h, hipMemcpyAsync(h->int_host, counter, sizeof(int), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        ++sweeps;
        // algorithmic work of the rotations of this sweep: each rotation updates
        // two rows of the Hermitian Gram matrix and two columns of J (48 nc flops)
        if (h->prof_on && three) h->prof_flops[EA_K_JROT] += 48.0 * 2 * w * (double)h->int_host[0];
        if (h->int_host[0] == 0) {
            conv = 1;
            break;
        }
    }
    launch_fill_int(sweeps_dev, 1, sweeps, h->stream);
    launch_fill_int(sweeps_dev + 1, 1, conv, h->stream);
    return EA_OK;
}

// Factor matrix X (rows x cols, currently in W as column-major after the
// caller's copy/contraction) and read back the decision record.
template <typename T>
int factor_and_decide(ea_mps *h, int mw, int nw, double f_t, int mode, int forced_k) {
    TRY(ensure(h, h->s_raw, sizeof(double) * nw));
    TRY(ensure(h, h->s_sorted, sizeof(double) * nw));
    TRY(ensure(h, h->perm, sizeof(int) * nw));
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
    if (orient == 0) {
        gather<T>(h, h->W.p, M, k, M, 0, -1, 0, 1, h->site[c].p);
        gather<T>(h, h->V.p, N, k, N, 1, 1, 0, 0, h->X.p);
    } else {
        gather<T>(h, h->V.p, M, k, M, 0, 0, 0, 1, h->site[c].p);
        gather<T>(h, h->W.p, N, k, N, 1, 0, 0, 0, h->X.p);
    }
    TRY(ensure(h, h->spare, h->csz * (size_t)k * d * chi2));
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * k * (double)(d * chi2) * N,
                     (double)h->csz * ((double)k * N + (double)N * d * chi2 + (double)k * d * chi2));
        launch_gemm<T>(h->X.p, h->site[c + 1].p, h->spare.p, k, d * chi2, N, N, d * chi2,
                       d * chi2, h->stream);
    }
    LAUNCHCHK(h);
    std::swap(h->site[c + 1], h->spare);
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
    if (orient == 0) {
        gather<T>(h, h->V.p, N, k, N, 1, 0, 0, 0, h->site[c].p);
        gather<T>(h, h->W.p, M, k, M, 0, 0, 0, 1, h->X.p);
    } else {
        gather<T>(h, h->W.p, N, k, N, 1, -1, 0, 0, h->site[c].p);
        gather<T>(h, h->V.p, M, k, M, 0, 1, 0, 1, h->X.p);
    }
    TRY(ensure(h, h->spare, h->csz * (size_t)rowsP * k));
    {
        ProfScope ps(h, EA_K_GEMM, 8.0 * rowsP * (double)k * M,
                     (double)h->csz * ((double)rowsP * M + (double)M * k + (double)rowsP * k));
        launch_gemm<T>(h->site[c - 1].p, h->X.p, h->spare.p, rowsP, k, M, M, k, k, h->stream);
    }
    LAUNCHCHK(h);
    std::swap(h->site[c - 1], h->spare);
    h->bond[c] = k;
    h->center = c - 1;
    return EA_OK;
}

template <typename T>
int move_center(ea_mps *h, int j) {
    while (h->center < j) {
        ProfScope ps(h, EA_K_MOVE, 0.0, 0.0);
        TRY(move_right<T>(h));
    }
    while (h->center > j) {
        ProfScope ps(h, EA_K_MOVE, 0.0, 0.0);
        TRY(move_left<T>(h));
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
        launch_theta<T>(h->site[i].p, h->site[i + 1].p, G, h->W.p, chiL, chiM, chiR, d, orient,
                        h->stream);
    }
    LAUNCHCHK(h);
    TRY(factor_and_decide<T>(h, mw, nw, f_t, 0, forced_k));
    const ea_dev_rec rec = *h->rec_host;
    const int k = rec.k;
    if (!(rec.s0 > 0.0) || !std::isfinite(rec.total))
        return set_err(EA_EINVAL, "the operator annihilates the state (all singular values 0)");
    TRY(ensure(h, h->site[i], h->csz * (size_t)M * k));
    TRY(ensure(h, h->site[i + 1], h->csz * (size_t)k * N));
    const bool right = dir > 0;
    if (orient == 0) {
        gather<T>(h, h->W.p, M, k, M, 0, right ? -1 : 0, right ? 0 : 1, 1, h->site[i].p);
        gather<T>(h, h->V.p, N, k, N, 1, right ? 1 : 0, right ? 1 : 0, 0, h->site[i + 1].p);
    } else {
        gather<T>(h, h->V.p, M, k, M, 0, right ? 0 : 1, right ? 0 : 1, 1, h->site[i].p);
        gather<T>(h, h->W.p, N, k, N, 1, right ? 0 : -1, right ? 1 : 0, 0, h->site[i + 1].p);
    }
    LAUNCHCHK(h);
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
    r.f_t = f_t;
    r.f = rec.f;
    r.total = rec.total;
    r.lnP = h->lnP;
    h->log.push_back(r);
    h->g += 1;
    if (f_out) *f_out = rec.f;
    if (rec.capped) return set_err(EA_WARN_CAPPED, "chi_max bound at gate %ld", (long)r.gate);
    if (!rec.converged) return set_err(EA_WARN_NOCONV, "Jacobi did not converge");
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

void free_buf(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *ea_last_error(void) { return g_err.c_str(); }

int mps_init_product(int n_sites, int kind, int prec, int chi_max, const double *local,
                     void *hip_stream, ea_mps **out) {
    if (!out) return set_err(EA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_sites < 2) return set_err(EA_EINVAL, "n_sites must be >= 2");
    if (kind != EA_PURE && kind != EA_MIXED) return set_err(EA_EINVAL, "bad kind %d", kind);
    if (prec != EA_C128 && prec != EA_C64 && prec != EA_C64_BF16X3)
        return set_err(EA_EINVAL, "bad precision %d", prec);
    if (chi_max < 0) return set_err(EA_EINVAL, "chi_max must be >= 0");
    const int d = kind == EA_PURE ? 2 : 4;
    if (local && !finite_cplx(local, (size_t)n_sites * d))
        return set_err(EA_EINVAL, "local state has non-finite entries");
    ea_mps *h = new ea_mps();
    h->n = n_sites;
    h->d = d;
    h->kind = kind;
    h->prec = prec;
    h->chi_max = chi_max;
    h->f64 = prec == EA_C128;
    h->csz = h->f64 ? 16 : 8;
    h->tau = h->f64 ? 1e-13 : 2e-6;
    h->stream = (hipStream_t)hip_stream;
    if (!h->stream) {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return set_err(EA_EHIP, "stream creation failed");
        }
        h->own_stream = true;
    }
    h->bond.assign(n_sites + 1, 1);
    h->site.resize(n_sites);
    auto bail = [&](int rc) {
        mps_free(h);
        return rc;
    };
    int rc;
    for (int i = 0; i < n_sites; ++i)
        if ((rc = ensure(h, h->site[i], h->csz * d)) < 0) return bail(rc);
    if ((rc = ensure(h, h->rec, sizeof(ea_dev_rec))) < 0) return bail(rc);
    if ((rc = ensure(h, h->ints, 64 * sizeof(int))) < 0) return bail(rc);
    if ((rc = ensure(h, h->partial, 3 * 1024 * sizeof(double))) < 0) return bail(rc);
    if ((rc = ensure(h, h->out3, 4 * sizeof(double))) < 0) return bail(rc);
    h->stage_cap = 8u << 20;
    if ((rc = ensure(h, h->stage_dev, h->stage_cap)) < 0) return bail(rc);
    if (hipHostMalloc((void **)&h->stage_host, h->stage_cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&h->rec_host, sizeof(ea_dev_rec), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&h->int_host, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&h->dbl_host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return bail(set_err(EA_ENOMEM, "pinned host allocation failed"));
    }
    std::vector<double> host(2 * (size_t)n_sites * d, 0.0);
    if (local) {
        std::memcpy(host.data(), local, host.size() * sizeof(double));
    } else {
        for (int i = 0; i < n_sites; ++i) host[2 * (size_t)i * d] = 1.0;
    }
    if ((rc = ensure(h, h->c128, host.size() * sizeof(double))) < 0) return bail(rc);
    if (hipMemcpy(h->c128.p, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice) !=
        hipSuccess)
        return bail(set_err(EA_EHIP, "upload of the product state failed"));
    for (int i = 0; i < n_sites; ++i) {
        if (h->f64)
            launch_from_c128<double>((const double *)h->c128.p + 2 * (size_t)i * d, h->site[i].p, d,
                                     h->stream);
        else
            launch_from_c128<float>((const double *)h->c128.p + 2 * (size_t)i * d, h->site[i].p, d,
                                    h->stream);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
        return bail(set_err(EA_EHIP, "initialisation kernels failed"));
    *out = h;
    return EA_OK;
}

void mps_free(ea_mps *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    prof_harvest(h);
    for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
    for (auto &b : h->site) free_buf(b);
    DevBuf *bufs[] = {&h->jpart, &h->jmat, &h->jflag, &h->spare, &h->W, &h->V, &h->X, &h->X2, &h->s_raw, &h->s_sorted, &h->perm,
                      &h->rec, &h->ints, &h->partial, &h->envb, &h->tmp, &h->out3, &h->c128,
                      &h->stage_dev};
    for (DevBuf *b : bufs) free_buf(*b);
    if (h->stage_host) (void)hipHostFree(h->stage_host);
    if (h->rec_host) (void)hipHostFree(h->rec_host);
    if (h->int_host) (void)hipHostFree(h->int_host);
    if (h->dbl_host) (void)hipHostFree(h->dbl_host);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int mps_set_option(ea_mps *h, int option, double value) {
    TRY(check(h));
    switch (option) {
    case EA_OPT_JACOBI_TOL:
        if (!(value >= 0) || value >= 1) return set_err(EA_EINVAL, "tol out of range");
        h->tol = value;
        return EA_OK;
    case EA_OPT_MAX_SWEEPS:
        if (!(value >= 1) || value > 1000) return set_err(EA_EINVAL, "max_sweeps out of range");
        h->max_sweeps = (int)value;
        return EA_OK;
    case EA_OPT_TAU:
        if (!(value >= 0) || value >= 1) return set_err(EA_EINVAL, "tau out of range");
        h->tau = value;
        return EA_OK;
    case EA_OPT_BLOCK:
        if (!(value >= 0) || value > 32) return set_err(EA_EINVAL, "block out of range");
        h->block = (int)value;
        return EA_OK;
    case EA_OPT_CHI_MAX:
        if (!(value >= 0) || value > 1e9) return set_err(EA_EINVAL, "chi_max out of range");
        h->chi_max = (int)value;
        return EA_OK;
    case EA_OPT_INNER_SWEEPS:
        if (!(value >= 1) || value > 50) return set_err(EA_EINVAL, "inner sweeps out of range");
        h->inner_round = (int)value;
        return EA_OK;
    case EA_OPT_JACOBI_KERNEL:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "jacobi kernel must be 0 or 1");
        h->jkernel = (int)value;
        return EA_OK;
    case EA_OPT_ROT_THREADS:
        if (value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
            return set_err(EA_EINVAL, "rotation threads must be 64, 128, 256, 512 or 1024");
        h->rot_threads = (int)value;
        return EA_OK;
    default:
        return set_err(EA_EINVAL, "unknown option %d", option);
    }
}

int mps_set_schedule(ea_mps *h, double f_min, long n_2q_total, int strategy) {
    TRY(check(h));
    if (!(f_min > 0.0 && f_min <= 1.0)) return set_err(EA_EINVAL, "F_min must be in (0, 1]");
    if (n_2q_total < 1) return set_err(EA_EINVAL, "n_2q_total must be >= 1");
    if (strategy < EA_NAIVE || strategy > EA_NEAREST) return set_err(EA_EINVAL, "bad strategy");
    h->has_sched = true;
    h->f_min = f_min;
    h->n_total = n_2q_total;
    h->strategy = strategy;
    return EA_OK;
}

int mps_apply_1q(ea_mps *h, int site, const double *op) {
    TRY(check(h));
    if (site < 0 || site >= h->n) return set_err(EA_ERANGE, "site %d out of range", site);
    if (!op || !finite_cplx(op, (size_t)h->d * h->d)) return set_err(EA_EINVAL, "bad operator");
    return h->f64 ? apply_1q_impl<double>(h, site, op) : apply_1q_impl<float>(h, site, op);
}

int mps_apply_2q(ea_mps *h, int site, const double *op, double fidelity_budget, double *f_out) {
    TRY(check(h));
    if (site < 0 || site + 1 >= h->n) return set_err(EA_ERANGE, "site %d out of range", site);
    const size_t nop = (size_t)h->d * h->d * h->d * h->d;
    if (!op || !finite_cplx(op, nop)) return set_err(EA_EINVAL, "bad operator");
    if (!(fidelity_budget < 0 || (fidelity_budget > 0 && fidelity_budget <= 1.0)))
        return set_err(EA_EINVAL, "fidelity budget must be in (0, 1] or negative");
    return h->f64 ? apply_2q_impl<double>(h, site, op, fidelity_budget, +1, f_out, 0)
                  : apply_2q_impl<float>(h, site, op, fidelity_budget, +1, f_out, 0);
}

int mps_apply_layer(ea_mps *h, int n_gates, const int *sites, const double *ops,
                    const double *budgets, double *f_out) {
    TRY(check(h));
    if (n_gates < 0) return set_err(EA_EINVAL, "n_gates < 0");
    if (n_gates == 0) return EA_OK;
    if (!sites || !ops) return set_err(EA_EINVAL, "null sites/ops");
    const size_t nop = (size_t)h->d * h->d * h->d * h->d;
    std::vector<char> used(h->n, 0);
    int lo = h->n, hi = -1;
    for (int j = 0; j < n_gates; ++j) {
        const int s = sites[j];
        if (s < 0 || s + 1 >= h->n) return set_err(EA_ERANGE, "site %d out of range", s);
        if (used[s] || used[s + 1]) return set_err(EA_EINVAL, "overlapping pairs in a layer");
        used[s] = used[s + 1] = 1;
        lo = std::min(lo, s);
        hi = std::max(hi, s);
        if (budgets && !(budgets[j] < 0 || (budgets[j] > 0 && budgets[j] <= 1.0)))
            return set_err(EA_EINVAL, "bad budget for gate %d", j);
    }
    if (!finite_cplx(ops, nop * n_gates)) return set_err(EA_EINVAL, "non-finite operator");
    std::vector<int> order(n_gates);
    for (int j = 0; j < n_gates; ++j) order[j] = j;
    const bool asc = std::abs(h->center - lo) <= std::abs(h->center - hi);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return asc ? sites[a] < sites[b] : sites[a] > sites[b];
    });
    int worst = EA_OK;
    for (int j : order) {
        double f = 1.0;
        const double b = budgets ? budgets[j] : -1.0;
        int rc = h->f64 ? apply_2q_impl<double>(h, sites[j], ops + 2 * nop * j, b, asc ? +1 : -1, &f, 0)
                        : apply_2q_impl<float>(h, sites[j], ops + 2 * nop * j, b, asc ? +1 : -1, &f, 0);
        if (rc < 0) return rc;
        if (rc > worst) worst = rc;
        if (f_out) f_out[j] = f;
    }
    if (worst > 0) g_err = "warning during layer";
    return worst;
}

int mps_apply_layer_batched(int n_states, ea_mps *const *hs, const int *n_gates,
                            const int *const *sites, const double *const *ops,
                            const double *const *budgets, double *const *f_out,
                            int *status_out) {
    if (n_states < 0) return set_err(EA_EINVAL, "n_states < 0");
    if (n_states == 0) return EA_OK;
    if (!hs || !n_gates || !sites || !ops) return set_err(EA_EINVAL, "null argument");
    for (int b = 0; b < n_states; ++b) {
        TRY(check(hs[b]));
        for (int c = 0; c < b; ++c)
            if (hs[c] == hs[b]) return set_err(EA_EINVAL, "a state appears twice in the batch");
    }
    std::vector<int> rc(n_states, EA_OK);
    std::vector<std::string> err(n_states);
    auto work = [&](int b) {
        rc[b] = mps_apply_layer(hs[b], n_gates[b], sites[b], ops[b], budgets ? budgets[b] : nullptr,
                                f_out ? f_out[b] : nullptr);
        if (rc[b] != EA_OK) err[b] = g_err;
    };
    std::vector<std::thread> pool;
    pool.reserve(n_states);
    for (int b = 1; b < n_states; ++b) pool.emplace_back(work, b);
    work(0);
    for (auto &t : pool) t.join();
    int worst = EA_OK, worst_b = -1;
    for (int b = 0; b < n_states; ++b) {
        if (status_out) status_out[b] = rc[b];
        if ((rc[b] < 0 && (worst >= 0 || rc[b] < worst)) || (worst >= 0 && rc[b] > worst)) {
            worst = rc[b];
            worst_b = b;
        }
    }
    if (worst_b >= 0) set_err(worst, "state %d: %s", worst_b, err[worst_b].c_str());
    return worst;
}

int mps_fidelity_estimate(const ea_mps *h, double *F_out, double *lnF_out) {
    TRY(check(h));
    if (F_out) *F_out = std::exp(h->lnP);
    if (lnF_out) *lnF_out = h->lnP;
    return EA_OK;
}

int mps_expect(ea_mps *h, int n_terms, const int *sites, const int *widths, const double *ops,
               double *out) {
    TRY(check(h));
    if (n_terms < 0 || (n_terms > 0 && (!sites || !widths || !ops || !out)))
        return set_err(EA_EINVAL, "bad arguments");
    size_t nops = 0;
    for (int t = 0; t < n_terms; ++t) {
        if (widths[t] != 1 && widths[t] != 2) return set_err(EA_EINVAL, "width must be 1 or 2");
        if (sites[t] < 0 || sites[t] + widths[t] > h->n) return set_err(EA_ERANGE, "bad site");
        nops += widths[t] == 1 ? 4 : 16;
    }
    if (!finite_cplx(ops, nops)) return set_err(EA_EINVAL, "non-finite operator");
    if (h->kind == EA_MIXED)
        return h->f64 ? expect_mixed<double>(h, n_terms, sites, widths, ops, out)
                      : expect_mixed<float>(h, n_terms, sites, widths, ops, out);
    size_t off = 0;
    for (int t = 0; t < n_terms; ++t) {
        double r3[3];
        int rc = h->f64 ? expect_pure<double>(h, sites[t], widths[t], ops + 2 * off, r3)
                        : expect_pure<float>(h, sites[t], widths[t], ops + 2 * off, r3);
        if (rc < 0) return rc;
        off += widths[t] == 1 ? 4 : 16;
        out[2 * t] = r3[0] / r3[2];
        out[2 * t + 1] = r3[1] / r3[2];
    }
    return EA_OK;
}

int mps_to_statevector(ea_mps *h, double *out, size_t out_complex_len) {
    TRY(check(h));
    if (!out) return set_err(EA_EINVAL, "out is NULL");
    if (h->kind == EA_PURE && h->n > 28) return set_err(EA_ETOOBIG, "N > 28");
    if (h->kind == EA_MIXED && h->n > 11) return set_err(EA_ETOOBIG, "N > 11 for a density matrix");
    return h->f64 ? to_vector_impl<double>(h, out, out_complex_len)
                  : to_vector_impl<float>(h, out, out_complex_len);
}

int mps_bond_dims(const ea_mps *h, int *out) {
    TRY(check(h));
    if (!out) return set_err(EA_EINVAL, "out is NULL");
    for (int j = 1; j < h->n; ++j) out[j - 1] = h->bond[j];
    return EA_OK;
}

int mps_center(const ea_mps *h, int *out) {
    TRY(check(h));
    if (!out) return set_err(EA_EINVAL, "out is NULL");
    *out = h->center;
    return EA_OK;
}

int mps_gate_log(const ea_mps *h, ea_gate_record *records, size_t cap, size_t *n_out) {
    TRY(check(h));
    if (n_out) *n_out = h->log.size();
    if (records) {
        const size_t m = std::min(cap, h->log.size());
        if (m) std::memcpy(records, h->log.data(), m * sizeof(ea_gate_record));
    }
    return EA_OK;
}

int mps_load(ea_mps *h, const int *bond_dims, const double *data, int center) {
    TRY(check(h));
    if (!bond_dims || !data) return set_err(EA_EINVAL, "null argument");
    if (bond_dims[0] != 1 || bond_dims[h->n] != 1) return set_err(EA_EINVAL, "end bonds must be 1");
    size_t tot = 0;
    for (int j = 0; j <= h->n; ++j) {
        if (bond_dims[j] < 1 || bond_dims[j] > (1 << 20)) return set_err(EA_EINVAL, "bad bond");
        if (j < h->n) tot += (size_t)bond_dims[j] * h->d * bond_dims[j + 1];
    }
    if (center < 0 || center >= h->n) return set_err(EA_ERANGE, "bad centre");
    if (!finite_cplx(data, tot)) return set_err(EA_EINVAL, "non-finite data");
    return h->f64 ? load_impl<double>(h, bond_dims, data, center)
                  : load_impl<float>(h, bond_dims, data, center);
}

int mps_get_site(ea_mps *h, int site, double *out, size_t out_complex_len, int *dims) {
    TRY(check(h));
    if (site < 0 || site >= h->n) return set_err(EA_ERANGE, "bad site");
    const size_t sz = (size_t)h->bond[site] * h->d * h->bond[site + 1];
    if (dims) {
        dims[0] = h->bond[site];
        dims[1] = h->d;
        dims[2] = h->bond[site + 1];
    }
    if (!out) return EA_OK;
    if (out_complex_len < sz) return set_err(EA_ETOOBIG, "need %zu entries", sz);
    return h->f64 ? get_site_impl<double>(h, site, out) : get_site_impl<float>(h, site, out);
}

int mps_reset_product(ea_mps *h, const double *local) {
    TRY(check(h));
    const int n = h->n, d = h->d;
    if (local && !finite_cplx(local, (size_t)n * d))
        return set_err(EA_EINVAL, "local state has non-finite entries");
    std::vector<double> host(2 * (size_t)n * d, 0.0);
    if (local)
        std::memcpy(host.data(), local, host.size() * sizeof(double));
    else
        for (int i = 0; i < n; ++i) host[2 * (size_t)i * d] = 1.0;
    std::vector<int> dims(n + 1, 1);
    int rc = h->f64 ? load_impl<double>(h, dims.data(), host.data(), 0)
                    : load_impl<float>(h, dims.data(), host.data(), 0);
    if (rc < 0) return rc;
    h->lnP = h->lnS = 0.0;
    h->g = 0;
    h->has_sched = false;
    h->log.clear();
    return EA_OK;
}

int mps_profile(ea_mps *h, int enable) {
    TRY(check(h));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    if (enable) {
        for (int f = 0; f < EA_K_COUNT; ++f) {
            h->prof_ms[f] = h->prof_flops[f] = h->prof_bytes[f] = 0.0;
            h->prof_cnt[f] = 0;
        }
    }
    h->prof_on = enable != 0;
    return EA_OK;
}

int mps_profile_read(ea_mps *h, int family, double *ms_total, long *launches, double *flops,
                     double *bytes) {
    TRY(check(h));
    if (family < 0 || family >= EA_K_COUNT) return set_err(EA_EINVAL, "bad kernel family");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    if (ms_total) *ms_total = h->prof_ms[family];
    if (launches) *launches = h->prof_cnt[family];
    if (flops) *flops = h->prof_flops[family];
    if (bytes) *bytes = h->prof_bytes[family];
    return EA_OK;
}

}  // extern "C"
