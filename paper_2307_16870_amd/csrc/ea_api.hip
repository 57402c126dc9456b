// Host side of the C ABI declared in include/ea_mps.h: handle, validation,
// device memory, orthogonality-centre bookkeeping, the target schedule and
// the orchestration of the kernels of one two-site update.
#include "ea_internal.h"

#include <mutex>

namespace ea {
thread_local std::string g_err;

// Process-wide tuning table (mps_set_tuning), entries sorted by (f64, n_max).
static std::mutex g_tune_mu;
static std::vector<ea_tune_entry> g_tune;

bool tune_lookup(bool f64, int n, int *block, int *rot_threads, int *wgs) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &e : g_tune)
        if ((e.f64 != 0) == f64 && n <= e.n_max) {
            *block = e.block;
            *rot_threads = e.rot_threads;
            *wgs = e.chunk_wgs;
            return true;
        }
    return false;
}
}  // namespace ea

using namespace ea;

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *ea_last_error(void) { return g_err.c_str(); }

int mps_set_tuning(int n_entries, const ea_tune_entry *entries) {
    if (n_entries < 0) return set_err(EA_EINVAL, "n_entries < 0");
    if (n_entries > 0 && !entries) return set_err(EA_EINVAL, "entries is NULL");
    std::vector<ea_tune_entry> t(entries, entries + n_entries);
    for (int i = 0; i < n_entries; ++i) {
        const ea_tune_entry &e = t[i];
        const int rt = e.rot_threads;
        if ((e.f64 != 0 && e.f64 != 1) || e.n_max < 1 || (e.block != 16 && e.block != 32) ||
            (rt != 64 && rt != 128 && rt != 256 && rt != 512 && rt != 1024) ||
            e.chunk_wgs < 64 || e.chunk_wgs > 4096)
            return set_err(EA_EINVAL, "tuning entry %d out of range", i);
        for (int j = 0; j < i; ++j)
            if (t[j].f64 == e.f64 && t[j].n_max == e.n_max)
                return set_err(EA_EINVAL, "tuning entries %d and %d cover the same sizes", j, i);
    }
    std::sort(t.begin(), t.end(), [](const ea_tune_entry &a, const ea_tune_entry &b) {
        return a.f64 != b.f64 ? a.f64 < b.f64 : a.n_max < b.n_max;
    });
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(t);
    return EA_OK;
}

int mps_get_tuning(int capacity, ea_tune_entry *out) {
    if (capacity < 0 || (capacity > 0 && !out)) return set_err(EA_EINVAL, "bad output buffer");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int n = (int)g_tune.size();
    for (int i = 0; i < n && i < capacity; ++i) out[i] = g_tune[i];
    return n;
}

int mps_init_product(int n_sites, int kind, int prec, int chi_max, const double *local,
                     const ea_allocator *alloc, void *hip_stream, ea_mps **out) {
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
    if (alloc && (!alloc->alloc || !alloc->free))
        return set_err(EA_EINVAL, "allocator needs both alloc and free");
    ea_mps *h = new ea_mps();
    if (alloc) h->alloc = *alloc;
    if (hipGetDevice(&h->device) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return set_err(EA_EHIP, "hipGetDevice failed");
    }
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
        const hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return set_err(EA_EHIP, "stream creation failed: %s", hipGetErrorString(e));
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
    for (ea_mps *w : h->workers) mps_free(w);
    h->workers.clear();
    if (h->ev) (void)hipEventDestroy(h->ev);
    if (h->adj_free) h->adj_free(h->adj);
    h->adj = nullptr;
    for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
    for (auto &b : h->site) free_buf(b);
    DevBuf *bufs[] = {&h->ro_x64, &h->ro_g, &h->ro_y, &h->ro_r, &h->ro_t, &h->jpart, &h->jmat, &h->jflag, &h->jstamp, &h->qr_a, &h->qr_v, &h->qr_t, &h->qr_tau, &h->qr_y, &h->qr_z, &h->qr_r, &h->qr_s, &h->spare, &h->W, &h->V, &h->X, &h->X2, &h->s_raw, &h->s_sorted, &h->perm,
                      &h->rec, &h->ints, &h->partial, &h->envb, &h->tmp, &h->out3, &h->c128,
                      &h->stage_dev, &h->sm_scratch, &h->sm_sites, &h->sm_bond, &h->sm_loff, &h->sm_gsite,
                      &h->sm_gmat, &h->sm_budget, &h->sm_log, &h->sm_fout, &h->sm_descs,
                      &h->cq_x, &h->cq_q, &h->cq_g, &h->cq_r1, &h->cq_r2, &h->cq_ri, &h->cq_t,
                      &h->cq_misc, &h->cbuf, &h->ybuf, &h->tk_x, &h->tk_om, &h->tk_y,
                      &h->tk_w, &h->tk_q1, &h->tk_vj, &h->tk_misc};
    for (DevBuf *b : bufs) free_buf(*b);
    for (auto &b : h->lam) free_buf(b);
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
    case EA_OPT_REORTH:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "reorth must be 0 or 1");
        h->reorth = value != 0;
        return EA_OK;
    case EA_OPT_SMALL_LAYERS:
        if (value != 0 && value != 64 && value != SM_N)
            return set_err(EA_EINVAL, "small layers must be 0, 64 or %d", SM_N);
        h->small_cols = (int)value;
        return EA_OK;
    case EA_OPT_JACOBI_ORDER:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "jacobi order must be 0 or 1");
        h->jorder = (int)value;
        return EA_OK;
    case EA_OPT_QR_MOVES:
        if (value != 0 && value != 1 && value != 2)
            return set_err(EA_EINVAL, "centre-move kind must be 0, 1 or 2");
        h->move_kind = (int)value;
        return EA_OK;
    case EA_OPT_RESERVE_BOND: {
        if (!(value >= 1) || value > 65536) return set_err(EA_EINVAL, "reserve bond out of range");
        const size_t chi = (size_t)value, want = h->csz * chi * h->d * chi;
        for (int i = 0; i < h->n; ++i) {
            if (h->site[i].bytes >= want) continue;
            // a larger buffer holding the current tensor
            DevBuf nb;
            TRY(ensure(h, nb, want));
            const size_t used = h->csz * (size_t)h->bond[i] * h->d * h->bond[i + 1];
            HIPCHK(h, hipMemcpyAsync(nb.p, h->site[i].p, used, hipMemcpyDeviceToDevice,
                                     h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
            free_buf(h->site[i]);
            h->site[i] = nb;
        }
        return EA_OK;
    }
    case EA_OPT_TOPK:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "must be 0 or 1");
        h->topk = value != 0;
        return EA_OK;
    case EA_OPT_TOPK_OVERSAMPLE:
        if (!(value >= 1 && value <= 512) || value != std::floor(value))
            return set_err(EA_EINVAL, "oversampling must be an integer in 1..512");
        h->topk_p = (int)value;
        return EA_OK;
    case EA_OPT_TOPK_POWER:
        if (!(value >= 0 && value <= 4) || value != std::floor(value))
            return set_err(EA_EINVAL, "subspace iterations must be an integer in 0..4");
        h->topk_q = (int)value;
        return EA_OK;
    case EA_OPT_TOPK_SEED:
        if (!(value >= 0 && value < 9007199254740992.0) || value != std::floor(value))
            return set_err(EA_EINVAL, "seed must be an integer in [0, 2^53)");
        h->topk_seed = (unsigned long long)value;
        return EA_OK;
    case EA_OPT_TOPK_MIN:
        if (!(value >= 2 && value <= EA_SORT_MAX) || value != std::floor(value))
            return set_err(EA_EINVAL, "minimum width must be an integer in 2..4096");
        h->topk_min = (int)value;
        return EA_OK;
    case EA_OPT_GAUGE_PARALLEL:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "must be 0 or 1");
        h->vidal_parallel = value != 0;
        return EA_OK;
    case EA_OPT_GAUGE:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "gauge must be 0 or 1");
        if (value == 1 && !h->gauge) {
            for (int b = 1; b < h->n; ++b)
                if (h->bond[b] != 1)
                    return set_err(EA_EINVAL, "the layer-parallel gauge starts from a product state");
            TRY(vidal_reset_lambdas(h));
            h->gauge = 1;
        } else if (value == 0 && h->gauge) {
            // B_0 .. B_{N-1} contract to the state; exact moves from the last
            // site to the first leave sites 1 .. N-1 right-normalised and the
            // orthogonality centre on site 0
            h->gauge = 0;
            h->center = h->n - 1;
            TRY(h->f64 ? move_center<double>(h, 0) : move_center<float>(h, 0));
        }
        return EA_OK;
    case EA_OPT_QR_PRECOND:
        if (!(value >= 0) || value > 4096) return set_err(EA_EINVAL, "QR width out of range");
        h->qr_min = (int)value;
        return EA_OK;
    case EA_OPT_JACOBI_SKIP:
        if (value != 0 && value != 1) return set_err(EA_EINVAL, "jacobi skip must be 0 or 1");
        h->jskip = value != 0;
        return EA_OK;
    case EA_OPT_ROT_THREADS:
        if (value != 0 && value != 64 && value != 128 && value != 256 && value != 512 &&
            value != 1024)
            return set_err(EA_EINVAL, "rotation threads must be 0, 64, 128, 256, 512 or 1024");
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
    if (strategy < EA_NAIVE || strategy > EA_FIXED) return set_err(EA_EINVAL, "bad strategy");
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
    if (h->gauge) {  // layer-parallel gauge: B_i <- g B_i, no centre to move
        void *g = nullptr;
        if (h->f64) {
            TRY(stage<double>(h, op, (size_t)h->d * h->d, &g));
            launch_apply1<double>(h->site[site].p, h->site[site].p, g, h->bond[site], h->d,
                                  h->bond[site + 1], h->stream);
        } else {
            TRY(stage<float>(h, op, (size_t)h->d * h->d, &g));
            launch_apply1<float>(h->site[site].p, h->site[site].p, g, h->bond[site], h->d,
                                 h->bond[site + 1], h->stream);
        }
        LAUNCHCHK(h);
        return EA_OK;
    }
    return h->f64 ? apply_1q_impl<double>(h, site, op) : apply_1q_impl<float>(h, site, op);
}

int mps_apply_2q(ea_mps *h, int site, const double *op, double fidelity_budget, double *f_out) {
    TRY(check(h));
    if (site < 0 || site + 1 >= h->n) return set_err(EA_ERANGE, "site %d out of range", site);
    const size_t nop = (size_t)h->d * h->d * h->d * h->d;
    if (!op || !finite_cplx(op, nop)) return set_err(EA_EINVAL, "bad operator");
    if (!(fidelity_budget < 0 || (fidelity_budget > 0 && fidelity_budget <= 1.0)))
        return set_err(EA_EINVAL, "fidelity budget must be in (0, 1] or negative");
    if (h->gauge) {
        const double ft = fidelity_budget >= 0 ? fidelity_budget : schedule_target(h);
        return h->f64 ? vidal_2q_impl<double>(h, site, op, ft, f_out, 0)
                      : vidal_2q_impl<float>(h, site, op, ft, f_out, 0);
    }
    return h->f64 ? apply_2q_impl<double>(h, site, op, fidelity_budget, +1, f_out, 0)
                  : apply_2q_impl<float>(h, site, op, fidelity_budget, +1, f_out, 0);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free two-site update.  Its workspace lives in `scratch`, one
// array per device for the life of the process.  In host code the array's
// name is only a stand-in: its device address on each device is taken once,
// with that device current, by hipGetSymbolAddress and kept in
// g_scratch_ptr; kernels and copies only ever see that address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[EA_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<char *> g_scratch_ptr;  // device address of `scratch`, per device

// Device address of `scratch` on the current device `dev` (looked up once).
int scratch_address(int dev, char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0) return set_err(EA_EINVAL, "bad device %d", dev);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_err(EA_EHIP, "hipGetSymbolAddress(scratch) failed: %s",
                           hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return EA_OK;
}
}  // namespace

extern "C" {

int mps_apply_2q_noalloc(ea_mps *h, int site, const double *op, double fidelity_budget,
                         double *f_out) {
    TRY(check(h));
    if (h->gauge) return set_err(EA_EINVAL, "the allocation-free update needs the single-centre gauge");
    if (site < 0 || site + 1 >= h->n) return set_err(EA_ERANGE, "site %d out of range", site);
    const size_t nop = (size_t)h->d * h->d * h->d * h->d;
    if (!op || !finite_cplx(op, nop)) return set_err(EA_EINVAL, "bad operator");
    if (!(fidelity_budget < 0 || (fidelity_budget > 0 && fidelity_budget <= 1.0)))
        return set_err(EA_EINVAL, "fidelity budget must be in (0, 1] or negative");
    char *base = nullptr;
    {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
            (void)hipGetLastError();
            return set_err(EA_EINVAL, "the handle's device (%d) is not the current device",
                           h->device);
        }
    }
    TRY(scratch_address(h->device, &base));
    // event timing would create events on demand: suspended for the call
    const bool prof = h->prof_on;
    h->prof_on = false;
    h->arena = base;
    h->arena_cap = EA_NOALLOC_SCRATCH_BYTES;
    h->arena_off = 0;
    h->arena_saved.clear();
    const int rc = h->f64 ? apply_2q_impl<double>(h, site, op, fidelity_budget, +1, f_out, 0)
                          : apply_2q_impl<float>(h, site, op, fidelity_budget, +1, f_out, 0);
    arena_release(h, 0, 0);  // every workspace buffer back to its own memory
    h->arena = nullptr;
    h->arena_cap = 0;
    h->prof_on = prof;
    return rc;
}

}  // extern "C"

namespace {
// Argument checks of one layer; lo/hi receive the lowest and highest left site.
int validate_layer(ea_mps *h, int n_gates, const int *sites, const double *ops,
                   const double *budgets, int *lo_out, int *hi_out) {
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
    if (lo_out) *lo_out = lo;
    if (hi_out) *hi_out = hi;
    return EA_OK;
}

// Layer-parallel gauge: a worker is a handle used only for its stream, pinned
// staging and workspace, configured like the state so that a gate gives the
// same bits on a worker as on the state's own stream.
void copy_config(ea_mps *w, const ea_mps *h) {
    w->n = h->n;
    w->d = h->d;
    w->kind = h->kind;
    w->prec = h->prec;
    w->chi_max = h->chi_max;
    w->f64 = h->f64;
    w->csz = h->csz;
    w->tol = h->tol;
    w->max_sweeps = h->max_sweeps;
    w->tau = h->tau;
    w->block = h->block;
    w->inner_max = h->inner_max;
    w->inner_round = h->inner_round;
    w->jkernel = h->jkernel;
    w->rot_threads = h->rot_threads;
    w->jorder = h->jorder;
    w->jskip = h->jskip;
    w->qr_min = h->qr_min;
    w->reorth = h->reorth;
    w->prof_on = h->prof_on;
    w->prof_every = h->prof_every;
}

ea_mps *make_worker(ea_mps *h, int *rc_out) {
    ea_mps *w = new ea_mps();
    w->alloc = h->alloc;
    w->device = h->device;
    copy_config(w, h);
    *rc_out = EA_OK;
    auto fail = [&](int rc) {
        *rc_out = rc;
        mps_free(w);
        return nullptr;
    };
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete w;
        *rc_out = set_err(EA_EHIP, "worker stream creation failed");
        return nullptr;
    }
    w->own_stream = true;
    if (hipEventCreateWithFlags(&w->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_err(EA_EHIP, "worker event creation failed"));
    }
    int rc;
    if ((rc = ensure(w, w->rec, sizeof(ea_dev_rec))) < 0) return fail(rc);
    if ((rc = ensure(w, w->ints, 64 * sizeof(int))) < 0) return fail(rc);
    w->stage_cap = 1u << 20;
    if ((rc = ensure(w, w->stage_dev, w->stage_cap)) < 0) return fail(rc);
    if (hipHostMalloc((void **)&w->stage_host, w->stage_cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&w->rec_host, sizeof(ea_dev_rec), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&w->int_host, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&w->dbl_host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_err(EA_ENOMEM, "pinned host allocation failed"));
    }
    return w;
}

// The gates of one layer in the layer-parallel gauge, each on its own worker
// (stream and host thread), ordered after the state's pending work; the
// state's stream then waits for all of them, and the bookkeeping is applied
// in gate order.
template <typename T>
int vidal_layer_parallel(ea_mps *h, const std::vector<int> &order, const int *sites,
                         const double *ops, size_t nop, const double *fts, const int *ranks,
                         double *f_out) {
    const int ng = (int)order.size();
    while ((int)h->workers.size() < ng) {
        int rc = EA_OK;
        ea_mps *w = make_worker(h, &rc);
        if (!w) return rc;
        h->workers.push_back(w);
    }
    if (!h->ev) HIPCHK(h, hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
    HIPCHK(h, hipEventRecord(h->ev, h->stream));
    for (int u = 0; u < ng; ++u) {
        copy_config(h->workers[u], h);
        HIPCHK(h, hipStreamWaitEvent(h->workers[u]->stream, h->ev, 0));
    }
    std::vector<VidalOut> outs(ng);
    std::vector<int> rcs(ng, EA_OK);
    std::vector<std::string> errs(ng);
    auto work = [&](int u) {
        const int j = order[u];
        ea_mps *w = h->workers[u];
        rcs[u] = vidal_gate<T>(h, w, sites[j], ops + 2 * nop * j, fts[j], ranks ? ranks[j] : 0,
                               &outs[u]);
        if (rcs[u] < 0) errs[u] = g_err;
        if (hipEventRecord(w->ev, w->stream) != hipSuccess) {
            (void)hipGetLastError();
            if (rcs[u] >= 0) {
                rcs[u] = EA_EHIP;
                errs[u] = "event record failed";
            }
        }
    };
    std::vector<std::thread> pool;
    pool.reserve(ng);
    for (int u = 1; u < ng; ++u) pool.emplace_back(work, u);
    work(0);
    for (auto &t : pool) t.join();
    for (int u = 0; u < ng; ++u) HIPCHK(h, hipStreamWaitEvent(h->stream, h->workers[u]->ev, 0));
    if (h->prof_on) {
        for (int u = 0; u < ng; ++u) {
            ea_mps *w = h->workers[u];
            prof_harvest(w);
            for (int f = 0; f < EA_K_COUNT; ++f) {
                h->prof_ms[f] += w->prof_ms[f];
                h->prof_flops[f] += w->prof_flops[f];
                h->prof_bytes[f] += w->prof_bytes[f];
                h->prof_cnt[f] += w->prof_cnt[f];
                h->prof_timed[f] += w->prof_timed[f];
                w->prof_ms[f] = w->prof_flops[f] = w->prof_bytes[f] = 0.0;
                w->prof_cnt[f] = w->prof_timed[f] = 0;
            }
        }
    }
    int worst = EA_OK;
    for (int u = 0; u < ng; ++u) {
        const int j = order[u];
        if (rcs[u] < 0) {
            g_err = errs[u];
            return rcs[u];
        }
        double f = 1.0;
        const int rc = vidal_finish(h, sites[j], outs[u], &f);
        if (rc > worst) worst = rc;
        if (f_out) f_out[j] = f;
    }
    if (worst > 0) g_err = "warning during layer";
    return worst;
}

// A layer qualifies for the device-resident path when every bond is at most
// small_cols / d: then every factorisation of the layer has at most small_cols
// (<= SM_N) columns.
bool small_eligible(const ea_mps *h, int n_gates) {
    if (h->gauge || h->small_cols <= 0 || n_gates < 1 || n_gates > SM_GATES) return false;
    const int lim = h->small_cols / h->d;
    for (int b : h->bond)
        if (b > lim) return false;
    return true;
}

// One state's share of a device-resident launch: consecutive layers of
// two-qubit gates (layer L holds gates off[L] .. off[L+1]-1).
struct SmallJob {
    int b = 0;                       // index of the state in the caller's arrays
    std::vector<int> off;            // n_layers + 1 gate offsets
    const int *sites = nullptr;      // all gates' left sites
    const double *ops = nullptr;     // all gates' operators (complex d^4 each)
    const double *budgets = nullptr; // per gate, single-layer calls only
    double *f_out = nullptr;         // per gate, single-layer calls only
    int layers_done = 0;
};

// Grow every site buffer to the small-path capacity, keeping its tensor, and
// size the state's scratch (synchronises the state's stream).
int small_grow_sites(ea_mps *h) {
    const size_t cap = SM_ELEMS;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->n; ++i) {
        if (h->site[i].bytes >= h->csz * cap) continue;
        DevBuf nb;
        TRY(ensure(h, nb, h->csz * cap));
        const size_t used = h->csz * (size_t)h->bond[i] * h->d * h->bond[i + 1];
        if (used > 0 && h->site[i].p)
            HIPCHK(h, hipMemcpy(nb.p, h->site[i].p, used, hipMemcpyDeviceToDevice));
        free_buf(h->site[i]);
        h->site[i] = nb;
    }
    return ensure(h, h->sm_scratch, small_scratch_bytes(h->csz));
}

// The state's scalars in a small-path descriptor (pointers are the caller's).
template <typename T>
void small_fill_scalars(const ea_mps *h, int total, int n_layers, SmallDesc<T> &D) {
    D.tau = h->tau;
    D.tol_user = h->tol;
    D.f_min = h->f_min;
    D.lnP = h->lnP;
    D.lnS = h->lnS;
    D.n_total = h->n_total;
    D.g = h->g;
    D.n = h->n;
    D.d = h->d;
    D.kind = h->kind;
    D.n_gates = total;
    D.n_layers = n_layers;
    D.lim = h->small_cols / h->d;
    D.center = h->center;
    D.chi_max = h->chi_max;
    D.max_sweeps = h->max_sweeps;
    D.inner = h->inner_max;
    D.has_sched = h->has_sched ? 1 : 0;
    D.strategy = h->strategy;
    D.reorth = h->reorth ? 1 : 0;
}

// Apply a finished descriptor's results to the handle: records, bonds,
// centre, fidelity and scale logs, gate counter.  Returns the state's status.
template <typename T>
int small_apply_results(ea_mps *h, const SmallDesc<T> &D, const int *bond,
                        const ea_gate_record *recs) {
    std::copy(bond, bond + h->n + 1, h->bond.begin());
    for (int r = 0; r < D.n_done; ++r) h->log.push_back(recs[r]);
    h->center = D.center;
    h->lnP = D.lnP;
    h->lnS = D.lnS;
    h->g = D.g;
    if (D.status < 0)
        return set_err(D.status, "the operator annihilates the state (all singular values 0)");
    int rc = EA_OK;
    if (D.n_noconv > 0) rc = std::max(rc, (int)EA_WARN_NOCONV);
    if (D.n_capped > 0) rc = std::max(rc, (int)EA_WARN_CAPPED);
    return rc;
}

// Upload one state's layers and fill its descriptor (host copy).
template <typename T>
int small_prepare(ea_mps *h, const SmallJob &job, SmallDesc<T> &D) {
    const int d = h->d, n_layers = (int)job.off.size() - 1, total = job.off.back();
    TRY(small_grow_sites(h));
    const size_t nop = (size_t)d * d * d * d;
    TRY(ensure(h, h->sm_sites, sizeof(void *) * h->n));
    TRY(ensure(h, h->sm_bond, sizeof(int) * (h->n + 1)));
    TRY(ensure(h, h->sm_loff, sizeof(int) * (n_layers + 1)));
    TRY(ensure(h, h->sm_gsite, sizeof(int) * std::max(1, total)));
    TRY(ensure(h, h->sm_gmat, h->csz * nop * std::max(1, total)));
    TRY(ensure(h, h->sm_budget, sizeof(double) * std::max(1, total)));
    TRY(ensure(h, h->sm_log, sizeof(ea_gate_record) * std::max(1, total)));
    TRY(ensure(h, h->sm_fout, sizeof(double) * std::max(1, total)));
    std::vector<void *> ptrs(h->n);
    for (int i = 0; i < h->n; ++i) ptrs[i] = h->site[i].p;
    std::vector<T> g(2 * nop * total);
    for (size_t e = 0; e < g.size(); ++e) g[e] = (T)job.ops[e];
    HIPCHK(h, hipMemcpy(h->sm_sites.p, ptrs.data(), sizeof(void *) * h->n, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->sm_bond.p, h->bond.data(), sizeof(int) * (h->n + 1),
                        hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->sm_loff.p, job.off.data(), sizeof(int) * (n_layers + 1),
                        hipMemcpyHostToDevice));
    if (total > 0) {
        HIPCHK(h, hipMemcpy(h->sm_gsite.p, job.sites, sizeof(int) * total, hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->sm_gmat.p, g.data(), sizeof(T) * g.size(), hipMemcpyHostToDevice));
    }
    if (job.budgets)
        HIPCHK(h, hipMemcpy(h->sm_budget.p, job.budgets, sizeof(double) * total,
                            hipMemcpyHostToDevice));
    D = SmallDesc<T>{};
    D.site = (cx<T> *const *)h->sm_sites.p;
    D.bond = (int *)h->sm_bond.p;
    D.scratch = (cx<T> *)h->sm_scratch.p;
    D.layer_off = (const int *)h->sm_loff.p;
    D.gsite = (const int *)h->sm_gsite.p;
    D.gmat = (const cx<T> *)h->sm_gmat.p;
    D.budget = job.budgets ? (const double *)h->sm_budget.p : nullptr;
    D.log = (ea_gate_record *)h->sm_log.p;
    D.fout = job.f_out ? (double *)h->sm_fout.p : nullptr;
    small_fill_scalars(h, total, n_layers, D);
    return EA_OK;
}

// Read back one state; returns its status.
template <typename T>
int small_finish(ea_mps *h, const SmallDesc<T> &D, SmallJob &job) {
    HIPCHK(h, hipMemcpy(h->bond.data(), h->sm_bond.p, sizeof(int) * (h->n + 1),
                        hipMemcpyDeviceToHost));
    std::vector<ea_gate_record> recs(D.n_done);
    if (D.n_done > 0)
        HIPCHK(h, hipMemcpy(recs.data(), h->sm_log.p, sizeof(ea_gate_record) * D.n_done,
                            hipMemcpyDeviceToHost));
    if (job.f_out && D.n_gates > 0)
        HIPCHK(h, hipMemcpy(job.f_out, h->sm_fout.p, sizeof(double) * D.n_gates,
                            hipMemcpyDeviceToHost));
    job.layers_done = D.layers_done;
    const std::vector<int> bond(h->bond);
    return small_apply_results<T>(h, D, bond.data(), recs.data());
}

// All jobs of one precision in one launch (one workgroup per state).
template <typename T>
void small_batch(std::vector<SmallJob> &jobs, ea_mps *const *hs, std::vector<int> &rc,
                 std::vector<std::string> &err) {
    if (jobs.empty()) return;
    std::vector<SmallDesc<T>> run;
    std::vector<int> run_u;
    for (size_t u = 0; u < jobs.size(); ++u) {
        SmallDesc<T> D;
        const int r = small_prepare<T>(hs[jobs[u].b], jobs[u], D);
        if (r < 0) {
            rc[jobs[u].b] = r;
            err[jobs[u].b] = g_err;
        } else {
            run.push_back(D);
            run_u.push_back((int)u);
        }
    }
    if (run.empty()) return;
    ea_mps *h0 = hs[jobs[run_u[0]].b];
    auto fail_all = [&](int r) {
        for (int u : run_u) {
            rc[jobs[u].b] = r;
            err[jobs[u].b] = g_err;
        }
    };
    int r = ensure(h0, h0->sm_descs, sizeof(SmallDesc<T>) * run.size());
    if (r < 0) return fail_all(r);
    if (hipMemcpy(h0->sm_descs.p, run.data(), sizeof(SmallDesc<T>) * run.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
        return fail_all(set_err(EA_EHIP, "descriptor upload failed"));
    launch_layer_small<T>((SmallDesc<T> *)h0->sm_descs.p, (int)run.size(), h0->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h0->stream);
    if (e != hipSuccess) return fail_all(set_err(EA_EHIP, "small layer: %s", hipGetErrorString(e)));
    if (hipMemcpy(run.data(), h0->sm_descs.p, sizeof(SmallDesc<T>) * run.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return fail_all(set_err(EA_EHIP, "descriptor read-back failed"));
    for (size_t v = 0; v < run.size(); ++v) {
        SmallJob &job = jobs[run_u[v]];
        rc[job.b] = small_finish<T>(hs[job.b], run[v], job);
        if (rc[job.b] != EA_OK) err[job.b] = g_err;
    }
}
}  // namespace

extern "C" {

int mps_apply_layer(ea_mps *h, int n_gates, const int *sites, const double *ops,
                    const double *budgets, double *f_out) {
    int lo = 0, hi = 0;
    TRY(validate_layer(h, n_gates, sites, ops, budgets, &lo, &hi));
    if (n_gates == 0) return EA_OK;
    if (small_eligible(h, n_gates)) {  // the whole layer in one device-resident launch
        std::vector<SmallJob> jobs(1);
        jobs[0].off = {0, n_gates};
        jobs[0].sites = sites;
        jobs[0].ops = ops;
        jobs[0].budgets = budgets;
        jobs[0].f_out = f_out;
        std::vector<int> rc1(1, EA_OK);
        std::vector<std::string> err1(1);
        ea_mps *hs1[1] = {h};
        if (h->f64)
            small_batch<double>(jobs, hs1, rc1, err1);
        else
            small_batch<float>(jobs, hs1, rc1, err1);
        if (rc1[0] != EA_OK) g_err = err1[0];
        return rc1[0];
    }
    const size_t nop = (size_t)h->d * h->d * h->d * h->d;
    std::vector<int> order(n_gates);
    for (int j = 0; j < n_gates; ++j) order[j] = j;
    if (h->gauge) {
        // layer-parallel gauge: every gate's target from the estimate before
        // the layer; gates in increasing site order (they are independent)
        std::sort(order.begin(), order.end(), [&](int a, int b) { return sites[a] < sites[b]; });
        const double ft_layer = schedule_target(h);
        if (h->vidal_parallel && n_gates > 1) {
            std::vector<double> fts(n_gates);
            for (int j = 0; j < n_gates; ++j)
                fts[j] = budgets && budgets[j] >= 0 ? budgets[j] : ft_layer;
            return h->f64 ? vidal_layer_parallel<double>(h, order, sites, ops, nop, fts.data(),
                                                         nullptr, f_out)
                          : vidal_layer_parallel<float>(h, order, sites, ops, nop, fts.data(),
                                                        nullptr, f_out);
        }
        int worst = EA_OK;
        for (int j : order) {
            double f = 1.0;
            const double ft = budgets && budgets[j] >= 0 ? budgets[j] : ft_layer;
            int rc = h->f64 ? vidal_2q_impl<double>(h, sites[j], ops + 2 * nop * j, ft, &f, 0)
                            : vidal_2q_impl<float>(h, sites[j], ops + 2 * nop * j, ft, &f, 0);
            if (rc < 0) return rc;
            if (rc > worst) worst = rc;
            if (f_out) f_out[j] = f;
        }
        if (worst > 0) g_err = "warning during layer";
        return worst;
    }
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

int mps_apply_layer_ranks(ea_mps *h, int n_gates, const int *sites, const double *ops,
                          const int *ranks, double *f_out) {
    int lo = 0, hi = 0;
    TRY(validate_layer(h, n_gates, sites, ops, nullptr, &lo, &hi));
    if (n_gates == 0) return EA_OK;
    if (!ranks) return set_err(EA_EINVAL, "ranks is NULL");
    for (int j = 0; j < n_gates; ++j)
        if (ranks[j] < 1) return set_err(EA_EINVAL, "rank %d of gate %d must be >= 1", ranks[j], j);
    const size_t nop = (size_t)h->d * h->d * h->d * h->d;
    std::vector<int> order(n_gates);
    for (int j = 0; j < n_gates; ++j) order[j] = j;
    if (h->gauge) {
        std::sort(order.begin(), order.end(), [&](int a, int b) { return sites[a] < sites[b]; });
        const double ft_layer = schedule_target(h);
        if (h->vidal_parallel && n_gates > 1) {
            std::vector<double> fts(n_gates, ft_layer);
            return h->f64 ? vidal_layer_parallel<double>(h, order, sites, ops, nop, fts.data(),
                                                         ranks, f_out)
                          : vidal_layer_parallel<float>(h, order, sites, ops, nop, fts.data(),
                                                        ranks, f_out);
        }
        int worst = EA_OK;
        for (int j : order) {
            double f = 1.0;
            int rc = h->f64 ? vidal_2q_impl<double>(h, sites[j], ops + 2 * nop * j, ft_layer, &f, ranks[j])
                            : vidal_2q_impl<float>(h, sites[j], ops + 2 * nop * j, ft_layer, &f, ranks[j]);
            if (rc < 0) return rc;
            if (rc > worst) worst = rc;
            if (f_out) f_out[j] = f;
        }
        if (worst > 0) g_err = "warning during layer";
        return worst;
    }
    const bool asc = std::abs(h->center - lo) <= std::abs(h->center - hi);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return asc ? sites[a] < sites[b] : sites[a] > sites[b];
    });
    int worst = EA_OK;
    for (int j : order) {
        double f = 1.0;
        int rc = h->f64 ? apply_2q_impl<double>(h, sites[j], ops + 2 * nop * j, -1.0, asc ? +1 : -1, &f, ranks[j])
                        : apply_2q_impl<float>(h, sites[j], ops + 2 * nop * j, -1.0, asc ? +1 : -1, &f, ranks[j]);
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
    // states whose bonds are all small: one device-resident launch per
    // precision; the others: one host thread and stream each
    std::vector<SmallJob> small32, small64;
    std::vector<int> big;
    for (int b = 0; b < n_states; ++b) {
        if (n_gates[b] > 0 && small_eligible(hs[b], n_gates[b])) {
            int r = validate_layer(hs[b], n_gates[b], sites[b], ops[b],
                                   budgets ? budgets[b] : nullptr, nullptr, nullptr);
            if (r < 0) {
                rc[b] = r;
                err[b] = g_err;
                continue;
            }
            SmallJob job;
            job.b = b;
            job.off = {0, n_gates[b]};
            job.sites = sites[b];
            job.ops = ops[b];
            job.budgets = budgets ? budgets[b] : nullptr;
            job.f_out = f_out ? f_out[b] : nullptr;
            (hs[b]->f64 ? small64 : small32).push_back(job);
        } else {
            big.push_back(b);
        }
    }
    auto work = [&](int b) {
        rc[b] = mps_apply_layer(hs[b], n_gates[b], sites[b], ops[b], budgets ? budgets[b] : nullptr,
                                f_out ? f_out[b] : nullptr);
        if (rc[b] != EA_OK) err[b] = g_err;
    };
    std::vector<std::thread> pool;
    pool.reserve(big.size());
    for (size_t u = 1; u < big.size(); ++u) pool.emplace_back(work, big[u]);
    small_batch<float>(small32, hs, rc, err);
    small_batch<double>(small64, hs, rc, err);
    if (!big.empty()) work(big[0]);
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

int mps_run_layers_batched(int n_states, ea_mps *const *hs, const int *n_layers,
                           const int *const *layer_gates, const int *const *sites,
                           const double *const *ops, int *layers_done, int *status_out) {
    if (n_states < 0) return set_err(EA_EINVAL, "n_states < 0");
    if (n_states == 0) return EA_OK;
    if (!hs || !n_layers || !layer_gates || !sites || !ops || !layers_done)
        return set_err(EA_EINVAL, "null argument");
    for (int b = 0; b < n_states; ++b) {
        TRY(check(hs[b]));
        if (hs[b]->gauge) return set_err(EA_EINVAL, "state %d is in the layer-parallel gauge", b);
        for (int c = 0; c < b; ++c)
            if (hs[c] == hs[b]) return set_err(EA_EINVAL, "a state appears twice in the batch");
        if (n_layers[b] < 0) return set_err(EA_EINVAL, "n_layers < 0");
    }
    std::vector<int> rc(n_states, EA_OK);
    std::vector<std::string> err(n_states);
    std::vector<SmallJob> small32, small64;
    for (int b = 0; b < n_states; ++b) {
        layers_done[b] = 0;
        ea_mps *h = hs[b];
        const size_t nop = (size_t)h->d * h->d * h->d * h->d;
        SmallJob job;
        job.b = b;
        job.off.assign(1, 0);
        int maxg = 0, r = EA_OK;
        for (int L = 0; L < n_layers[b] && r == EA_OK; ++L) {
            const int ng = layer_gates[b][L];
            if (ng < 0) r = set_err(EA_EINVAL, "negative gate count in layer %d", L);
            else
                r = validate_layer(h, ng, sites[b] + job.off.back(), ops[b] + 2 * nop * job.off.back(),
                                   nullptr, nullptr, nullptr);
            maxg = std::max(maxg, ng);
            job.off.push_back(job.off.back() + std::max(0, ng));
        }
        if (r < 0) {
            rc[b] = r;
            err[b] = g_err;
            continue;
        }
        if (n_layers[b] == 0 || !small_eligible(h, std::max(1, maxg)) || maxg > SM_GATES) continue;
        job.sites = sites[b];
        job.ops = ops[b];
        (h->f64 ? small64 : small32).push_back(job);
    }
    small_batch<float>(small32, hs, rc, err);
    small_batch<double>(small64, hs, rc, err);
    for (auto *jobs : {&small32, &small64})
        for (auto &j : *jobs) layers_done[j.b] = j.layers_done;
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
    if (h->gauge) return set_err(EA_EINVAL, "mps_expect needs the single-centre gauge (EA_OPT_GAUGE 0)");
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
    h->gauge = 0;  // loaded tensors: one orthogonality centre
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
    if (h->gauge) TRY(vidal_reset_lambdas(h));  // the gauge is kept; every bond value 1
    return EA_OK;
}

int mps_profile(ea_mps *h, int every) {
    TRY(check(h));
    if (every < 0) return set_err(EA_EINVAL, "profile period < 0");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    if (every) {
        for (int f = 0; f < EA_K_COUNT; ++f) {
            h->prof_ms[f] = h->prof_flops[f] = h->prof_bytes[f] = 0.0;
            h->prof_cnt[f] = h->prof_timed[f] = 0;
        }
        h->prof_every = every;
    }
    h->prof_on = every != 0;
    return EA_OK;
}

int mps_profile_read(ea_mps *h, int family, double *ms_timed, long *launches, double *flops,
                     double *bytes, long *timed) {
    TRY(check(h));
    if (family < 0 || family >= EA_K_COUNT) return set_err(EA_EINVAL, "bad kernel family");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    prof_harvest(h);
    if (ms_timed) *ms_timed = h->prof_ms[family];
    if (timed) *timed = h->prof_timed[family];
    if (launches) *launches = h->prof_cnt[family];
    if (flops) *flops = h->prof_flops[family];
    if (bytes) *bytes = h->prof_bytes[family];
    return EA_OK;
}

}  // extern "C"

// ============================================================================
// Captured programs: the device-resident small-bond launch of many circuits
// as one replayable HIP graph
// ============================================================================
struct ea_program {
    std::vector<ea_mps *> hs;
    std::vector<int> f64, slot, total;        // per state
    std::vector<std::vector<int>> off;        // per state: layer offsets
    std::vector<void *> loff, gsite, gmat, log;  // per state, device, owned
    // staging block (pinned in, device, pinned out) with the same layout:
    // FP32 descriptors | FP64 descriptors | per state: site pointers, bonds
    size_t at_d32 = 0, at_d64 = 0, bytes = 0;
    std::vector<size_t> at_ptr, at_bond;
    int n32 = 0, n64 = 0;
    char *in = nullptr, *out = nullptr;
    void *dev = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void program_release(ea_program *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (auto *v : {&p->loff, &p->gsite, &p->gmat, &p->log})
        for (void *q : *v)
            if (q) (void)hipFree(q);
    if (p->dev) (void)hipFree(p->dev);
    if (p->in) (void)hipHostFree(p->in);
    if (p->out) (void)hipHostFree(p->out);
    delete p;
}

int dev_upload(void **dst, const void *src, size_t bytes) {
    if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return set_err(EA_ENOMEM, "hipMalloc(%zu) failed", bytes);
    }
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return set_err(EA_EHIP, "program upload failed");
    return EA_OK;
}

// The descriptor of state b for the next replay, in the pinned block.
template <typename T>
int program_stage(ea_program *p, int b) {
    ea_mps *h = p->hs[b];
    TRY(small_grow_sites(h));
    void **ptrs = (void **)(p->in + p->at_ptr[b]);
    for (int i = 0; i < h->n; ++i) ptrs[i] = h->site[i].p;
    std::copy(h->bond.begin(), h->bond.end(), (int *)(p->in + p->at_bond[b]));
    const size_t at = (f64_of<T>() ? p->at_d64 : p->at_d32) + sizeof(SmallDesc<T>) * p->slot[b];
    SmallDesc<T> D{};
    D.site = (cx<T> *const *)((char *)p->dev + p->at_ptr[b]);
    D.bond = (int *)((char *)p->dev + p->at_bond[b]);
    D.scratch = (cx<T> *)h->sm_scratch.p;
    D.layer_off = (const int *)p->loff[b];
    D.gsite = (const int *)p->gsite[b];
    D.gmat = (const cx<T> *)p->gmat[b];
    D.budget = nullptr;
    D.log = (ea_gate_record *)p->log[b];
    D.fout = nullptr;
    small_fill_scalars(h, p->total[b], (int)p->off[b].size() - 1, D);
    std::memcpy(p->in + at, &D, sizeof D);
    return EA_OK;
}

// Results of state b after a replay; returns its status.
template <typename T>
int program_finish(ea_program *p, int b, int *layers_done) {
    ea_mps *h = p->hs[b];
    SmallDesc<T> D;
    std::memcpy(&D, p->out + (f64_of<T>() ? p->at_d64 : p->at_d32) + sizeof(D) * p->slot[b],
                sizeof D);
    std::vector<ea_gate_record> recs(std::max(0, D.n_done));
    if (D.n_done > 0)
        HIPCHK(h, hipMemcpy(recs.data(), p->log[b], sizeof(ea_gate_record) * D.n_done,
                            hipMemcpyDeviceToHost));
    *layers_done = D.layers_done;
    return small_apply_results<T>(h, D, (const int *)(p->out + p->at_bond[b]), recs.data());
}

}  // namespace

extern "C" {

int mps_program_capture(int n_states, ea_mps *const *hs, const int *n_layers,
                        const int *const *layer_gates, const int *const *sites,
                        const double *const *ops, ea_program **out) {
    if (!out) return set_err(EA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_states < 1) return set_err(EA_EINVAL, "n_states < 1");
    if (!hs || !n_layers || !layer_gates || !sites || !ops)
        return set_err(EA_EINVAL, "null argument");
    for (int b = 0; b < n_states; ++b) {
        TRY(check(hs[b]));
        if (hs[b]->gauge) return set_err(EA_EINVAL, "state %d is in the layer-parallel gauge", b);
        for (int c = 0; c < b; ++c)
            if (hs[c] == hs[b]) return set_err(EA_EINVAL, "a state appears twice in the program");
        if (n_layers[b] < 0) return set_err(EA_EINVAL, "n_layers < 0");
        if (hs[b]->small_cols == 0)
            return set_err(EA_EINVAL, "state %d has device-resident layers switched off", b);
    }
    ea_program *p = new ea_program();
    auto bail = [&](int rc) {
        program_release(p);
        return rc;
    };
    p->hs.assign(hs, hs + n_states);
    p->f64.resize(n_states);
    p->slot.resize(n_states);
    p->total.resize(n_states);
    p->off.resize(n_states);
    p->loff.assign(n_states, nullptr);
    p->gsite.assign(n_states, nullptr);
    p->gmat.assign(n_states, nullptr);
    p->log.assign(n_states, nullptr);
    for (int b = 0; b < n_states; ++b) {
        ea_mps *h = hs[b];
        const size_t nop = (size_t)h->d * h->d * h->d * h->d;
        std::vector<int> &off = p->off[b];
        off.assign(1, 0);
        for (int L = 0; L < n_layers[b]; ++L) {
            const int ng = layer_gates[b][L];
            if (ng < 0 || ng > SM_GATES)
                return bail(set_err(EA_EINVAL, "state %d layer %d: %d gates", b, L, ng));
            TRY_OR(bail, validate_layer(h, ng, sites[b] + off.back(), ops[b] + 2 * nop * off.back(),
                                        nullptr, nullptr, nullptr));
            off.push_back(off.back() + ng);
        }
        const int total = off.back();
        p->total[b] = total;
        p->f64[b] = h->f64 ? 1 : 0;
        p->slot[b] = h->f64 ? p->n64++ : p->n32++;
        TRY_OR(bail, dev_upload(&p->loff[b], off.data(), sizeof(int) * off.size()));
        TRY_OR(bail, dev_upload(&p->gsite[b], sites[b], sizeof(int) * total));
        const size_t ne = 2 * nop * total;
        if (h->f64) {
            TRY_OR(bail, dev_upload(&p->gmat[b], ops[b], sizeof(double) * ne));
        } else {
            std::vector<float> g(ne);
            for (size_t e = 0; e < ne; ++e) g[e] = (float)ops[b][e];
            TRY_OR(bail, dev_upload(&p->gmat[b], g.data(), sizeof(float) * ne));
        }
        std::vector<char> zero(sizeof(ea_gate_record) * std::max(1, total), 0);
        TRY_OR(bail, dev_upload(&p->log[b], zero.data(), zero.size()));
    }
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    p->at_d32 = 0;
    p->at_d64 = align(sizeof(SmallDesc<float>) * p->n32);
    size_t at = align(p->at_d64 + sizeof(SmallDesc<double>) * p->n64);
    p->at_ptr.resize(n_states);
    p->at_bond.resize(n_states);
    for (int b = 0; b < n_states; ++b) {
        p->at_ptr[b] = at;
        at = align(at + sizeof(void *) * hs[b]->n);
        p->at_bond[b] = at;
        at = align(at + sizeof(int) * (hs[b]->n + 1));
    }
    p->bytes = at;
    if (hipHostMalloc((void **)&p->in, p->bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&p->out, p->bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&p->dev, p->bytes) != hipSuccess) {
        (void)hipGetLastError();
        return bail(set_err(EA_ENOMEM, "program staging (%zu bytes) failed", p->bytes));
    }
    std::memset(p->in, 0, p->bytes);
    std::memset(p->out, 0, p->bytes);
    // capture: staged descriptors in, one persistent launch per precision,
    // results out (no memset nodes)
    p->stream = hs[0]->stream;
    for (int b = 0; b < n_states; ++b) HIPCHK(hs[b], hipStreamSynchronize(hs[b]->stream));
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->dev, p->in, p->bytes, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess && p->n32)
        launch_layer_small<float>((SmallDesc<float> *)((char *)p->dev + p->at_d32), p->n32,
                                  p->stream);
    if (e == hipSuccess && p->n64)
        launch_layer_small<double>((SmallDesc<double> *)((char *)p->dev + p->at_d64), p->n64,
                                   p->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->out, p->dev, p->bytes, hipMemcpyDeviceToHost, p->stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(p->stream, &g);
    p->graph = g;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return bail(set_err(EA_EHIP, "graph capture failed: %s", hipGetErrorString(e)));
    }
    *out = p;
    return EA_OK;
}

int mps_program_launch(ea_program *p, int *layers_done, int *status_out) {
    if (!p || !p->exec) return set_err(EA_EINVAL, "null program");
    const int n_states = (int)p->hs.size();
    for (int b = 0; b < n_states; ++b) TRY(check(p->hs[b]));
    std::vector<int> rc(n_states, EA_OK);
    std::vector<std::string> err(n_states);
    for (int b = 0; b < n_states; ++b) {
        const int r = p->f64[b] ? program_stage<double>(p, b) : program_stage<float>(p, b);
        if (r < 0) return r;  // nothing launched: the states are unchanged
    }
    hipError_t e = hipGraphLaunch(p->exec, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        for (ea_mps *h : p->hs) h->poisoned = true;
        return set_err(EA_EHIP, "program launch failed: %s", hipGetErrorString(e));
    }
    int worst = EA_OK, worst_b = -1;
    for (int b = 0; b < n_states; ++b) {
        int done = 0;
        rc[b] = p->f64[b] ? program_finish<double>(p, b, &done) : program_finish<float>(p, b, &done);
        if (rc[b] != EA_OK) err[b] = g_err;
        if (layers_done) layers_done[b] = done;
        if (status_out) status_out[b] = rc[b];
        if ((rc[b] < 0 && (worst >= 0 || rc[b] < worst)) || (worst >= 0 && rc[b] > worst)) {
            worst = rc[b];
            worst_b = b;
        }
    }
    if (worst_b >= 0) set_err(worst, "state %d: %s", worst_b, err[worst_b].c_str());
    return worst;
}

void mps_program_free(ea_program *p) {
    if (p && p->stream) (void)hipStreamSynchronize(p->stream);
    program_release(p);
}

}  // extern "C"
