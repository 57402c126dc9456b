// Reverse pass of the entanglement-aware simulation: energy and gradient
// with respect to one-qubit rotation angles, kept ranks frozen.
//
// Forward: ops are applied layer by layer with a checkpoint of the state at
// each layer start; the energy terms are then evaluated with a tape.
// Reverse: the energy tape is undone, then for each layer (last first) the
// checkpoint is restored, the layer is recomputed while recording, for every
// step, copies of its inputs and the full singular triplets of its
// factorisation, and the vector-Jacobian products are applied in reverse.
//
// Adjoint convention: dL = Re sum(conj(Xbar) dX).  Step VJPs (pure states):
//   A' = g A                       Abar = g^H A'bar,  gbar = sum A'bar conj(A)
//   Theta = G (A B)                Cbar = G^H Thetabar, Abar = Cbar B^H, Bbar = A^H Cbar
//   Theta = U S V^H, k kept,       A' = U_k, B' = (s_k/||s_k||) V_k^H
//   truncated SVD adjoint          Thetabar = U P V^H + (I-UU^H) Ubar S^-1 V^H
//                                             + U S^-1 Vbar^H (I-VV^H)
//     with J = U^H Ubar, K = V^H Vbar, P_ij = F_ij (s_j (J-J^H)_ij + s_i (K-K^H)_ij),
//     P_ii = sbar_i + i (Im J_ii - Im K_ii)/(2 s_i), F_ij = 1/(s_j^2 - s_i^2)
//     (Lorentzian-broadened), over the numerically non-zero singular values.
//   centre moves M = U (S V^H): the same SVD adjoint without truncation.
//   <O> = <Theta|O Theta>/<Theta|Theta>: Thetabar = c ((O+O^H) Theta - 2 Re<O> Theta)/N.
#include "ea_internal.h"

using namespace ea;

namespace {

enum { R_1Q = 0, R_2Q = 1, R_MR = 2, R_ML = 3, R_EX = 4 };

struct Rec {
    int kind = 0, site = 0, param = -1, width = 1;
    int d0 = 0, d1 = 0, d2 = 0;  // shapes: 1q (chiL, chiR); 2q (chiL, chiM, chiR); moves (cl, cr, other)
    int m = 0, n = 0, r = 0, k = 0;
    double sig = 1.0, coef = 0.0, val = 0.0, nrm = 1.0, s0 = 0.0;
    double gH[8] = {0}, dg[8] = {0};
    double op[32] = {0};  // 2q: G^H; ex: O + O^H (width 1: 2x2, width 2: 4x4)
    void *A = nullptr, *B = nullptr, *U = nullptr, *V = nullptr;
    double *s = nullptr;
};

// Device bump allocator made of chunks; reset() keeps the chunks.
struct Arena {
    std::vector<DevBuf> chunks;
    size_t off = 0;
    size_t cur = 0;
    void reset() {
        cur = 0;
        off = 0;
    }
    int alloc(ea_mps *h, size_t bytes, void **out) {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        while (true) {
            if (cur < chunks.size() && off + bytes <= chunks[cur].bytes) {
                *out = (char *)chunks[cur].p + off;
                off += bytes;
                return EA_OK;
            }
            if (cur < chunks.size() && off > 0) {
                ++cur;
                off = 0;
                continue;
            }
            if (cur == chunks.size()) chunks.emplace_back();
            if (chunks[cur].bytes < bytes) TRY(ensure(h, chunks[cur], std::max(bytes, size_t(64) << 20)));
        }
    }
    void release() {
        for (auto &b : chunks) free_buf(b);
        chunks.clear();
    }
};

struct Checkpoint {
    std::vector<int> bond;
    int center = 0;
    double lnP = 0.0, lnS = 0.0;
    long g = 0;
    std::vector<DevBuf> site;
};

struct Ctx {
    ea_mps *h;
    Arena tape, ws;
    std::vector<DevBuf> Ab;  // adjoint of each site tensor
    DevBuf gradbuf, partbuf;
    double *grad = nullptr;  // device
    double *partial = nullptr;
    double eta_rel = 0.0;
};

struct AdjCache {
    Ctx x;
    std::vector<Checkpoint> cps;
    void release() {
        x.tape.release();
        x.ws.release();
        free_buf(x.gradbuf);
        free_buf(x.partbuf);
        for (auto &b : x.Ab) free_buf(b);
        x.Ab.clear();
        for (auto &c : cps)
            for (auto &b : c.site) free_buf(b);
        cps.clear();
    }
};

void cplx_mul2(const double *a, const double *b, double *c) {  // 2x2 complex, row-major
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double re = 0, im = 0;
            for (int k = 0; k < 2; ++k) {
                const double ar = a[2 * (2 * i + k)], ai = a[2 * (2 * i + k) + 1];
                const double br = b[2 * (2 * k + j)], bi = b[2 * (2 * k + j) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            c[2 * (2 * i + j)] = re;
            c[2 * (2 * i + j) + 1] = im;
        }
}

// g and dg/dt for RY/RZ (or a fixed gate with dg = 0).
void rotation(int kind, double t, const double *mat, double *g, double *dg) {
    std::memset(dg, 0, 8 * sizeof(double));
    if (kind == EA_DOP_GATE1) {
        std::memcpy(g, mat, 8 * sizeof(double));
        return;
    }
    const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
    double P[8] = {0};  // -i/2 * (Y or Z)
    if (kind == EA_DOP_RY) {
        const double gg[8] = {c, 0, -s, 0, s, 0, c, 0};
        std::memcpy(g, gg, sizeof gg);
        // Y = [[0, -i], [i, 0]];  -i/2 Y = [[0, -1/2], [1/2, 0]]
        P[2] = -0.5;
        P[4] = 0.5;
    } else {
        const double gg[8] = {c, -s, 0, 0, 0, 0, c, s};
        std::memcpy(g, gg, sizeof gg);
        // -i/2 Z = diag(-i/2, i/2)
        P[1] = -0.5;
        P[7] = 0.5;
    }
    cplx_mul2(P, g, dg);
}

void herm_conj(const double *a, int k, double *out) {  // out = a^H (k x k)
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            out[2 * (i * k + j)] = a[2 * (j * k + i)];
            out[2 * (i * k + j) + 1] = -a[2 * (j * k + i) + 1];
        }
}

template <typename T>
int save_copy(Ctx &x, const void *src, size_t elems, void **dst) {
    TRY(x.tape.alloc(x.h, x.h->csz * elems, dst));
    HIPCHK(x.h, hipMemcpyAsync(*dst, src, x.h->csz * elems, hipMemcpyDeviceToDevice, x.h->stream));
    return EA_OK;
}

// Copies of U (M x r) and V (N x r), row-major, and s (r) from the last
// factorisation held in the handle's workspace (orient as chosen there).
template <typename T>
int save_triplets(Ctx &x, Rec &rc, int M, int N, int r) {
    ea_mps *h = x.h;
    const int orient = M >= N ? 0 : 1;
    TRY(x.tape.alloc(h, h->csz * (size_t)M * r, &rc.U));
    TRY(x.tape.alloc(h, h->csz * (size_t)N * r, &rc.V));
    void *sp = nullptr;
    TRY(x.tape.alloc(h, sizeof(double) * r, &sp));
    rc.s = (double *)sp;
    if (orient == 0) {
        gather<T>(h, h->W.p, M, r, M, 0, -1, 0, 1, rc.U);
        gather<T>(h, h->V.p, N, r, N, 0, 0, 0, 1, rc.V);
    } else {
        gather<T>(h, h->V.p, M, r, M, 0, 0, 0, 1, rc.U);
        gather<T>(h, h->W.p, N, r, N, 0, -1, 0, 1, rc.V);
    }
    HIPCHK(h, hipMemcpyAsync(rc.s, h->s_sorted.p, sizeof(double) * r, hipMemcpyDeviceToDevice,
                             h->stream));
    LAUNCHCHK(h);
    rc.m = M;
    rc.n = N;
    rc.r = r;
    rc.s0 = h->rec_host->s0;
    return EA_OK;
}

template <typename T>
int tape_move(Ctx &x, std::vector<Rec> *tape, bool right) {
    ea_mps *h = x.h;
    const int c = h->center, d = h->d;
    Rec rc;
    rc.kind = right ? R_MR : R_ML;
    rc.site = c;
    const int cl = h->bond[c], cr = h->bond[c + 1];
    const int nb = right ? c + 1 : c - 1;
    const size_t na = (size_t)cl * d * cr;
    const size_t nbe = (size_t)h->bond[nb] * d * h->bond[nb + 1];
    if (tape) {
        TRY(save_copy<T>(x, h->site[c].p, na, &rc.A));
        TRY(save_copy<T>(x, h->site[nb].p, nbe, &rc.B));
    }
    rc.d0 = cl;
    rc.d1 = cr;
    rc.d2 = right ? h->bond[c + 2] : h->bond[c - 1];
    if (right)
        TRY(move_right<T>(h));
    else
        TRY(move_left<T>(h));
    if (tape) {
        const int M = right ? cl * d : cl, N = right ? cr : d * cr;
        TRY(save_triplets<T>(x, rc, M, N, h->rec_host->k));
        tape->push_back(rc);
    }
    return EA_OK;
}

template <typename T>
int tape_center(Ctx &x, std::vector<Rec> *tape, int j) {
    while (x.h->center < j) TRY(tape_move<T>(x, tape, true));
    while (x.h->center > j) TRY(tape_move<T>(x, tape, false));
    return EA_OK;
}

template <typename T>
int tape_1q(Ctx &x, std::vector<Rec> *tape, const ea_dop &op, const double *params) {
    ea_mps *h = x.h;
    Rec rc;
    rc.kind = R_1Q;
    rc.site = op.site;
    double g[8];
    rotation(op.kind, op.kind == EA_DOP_GATE1 ? 0.0 : params[op.param], op.mat, g, rc.dg);
    rc.param = op.kind == EA_DOP_GATE1 ? -1 : op.param;
    herm_conj(g, 2, rc.gH);
    rc.d0 = h->bond[op.site];
    rc.d1 = h->bond[op.site + 1];
    if (tape) TRY(save_copy<T>(x, h->site[op.site].p, (size_t)rc.d0 * 2 * rc.d1, &rc.A));
    void *gd = nullptr;
    TRY(stage<T>(h, g, 4, &gd));
    launch_apply1<T>(h->site[op.site].p, h->site[op.site].p, gd, rc.d0, 2, rc.d1, h->stream);
    LAUNCHCHK(h);
    if (tape) tape->push_back(rc);
    return EA_OK;
}

template <typename T>
int tape_2q(Ctx &x, std::vector<Rec> *tape, const ea_dop &op, int forced_k, int *k_out) {
    ea_mps *h = x.h;
    const int i = op.site;
    if (h->center < i) TRY(tape_center<T>(x, tape, i));
    if (h->center > i + 1) TRY(tape_center<T>(x, tape, i + 1));
    Rec rc;
    rc.kind = R_2Q;
    rc.site = i;
    rc.d0 = h->bond[i];
    rc.d1 = h->bond[i + 1];
    rc.d2 = h->bond[i + 2];
    if (tape) {
        TRY(save_copy<T>(x, h->site[i].p, (size_t)rc.d0 * 2 * rc.d1, &rc.A));
        TRY(save_copy<T>(x, h->site[i + 1].p, (size_t)rc.d1 * 2 * rc.d2, &rc.B));
    }
    herm_conj(op.mat, 4, rc.op);
    double f = 0.0;
    const int st = apply_2q_impl<T>(h, i, op.mat, -1.0, +1, &f, forced_k);
    if (st < 0) return st;
    rc.k = h->rec_host->k;
    rc.sig = std::sqrt(h->rec_host->kept2);
    if (k_out) *k_out = rc.k;
    if (tape) {
        TRY(save_triplets<T>(x, rc, 2 * rc.d0, 2 * rc.d2, h->rec_host->k_nz));
        tape->push_back(rc);
    }
    return EA_OK;
}

template <typename T>
int tape_expect(Ctx &x, std::vector<Rec> *tape, int site, int width, const double *opm,
                double coef, double *val_out) {
    ea_mps *h = x.h;
    TRY(tape_center<T>(x, tape, site));
    Rec rc;
    rc.kind = R_EX;
    rc.site = site;
    rc.width = width;
    rc.coef = coef;
    const int k = width == 1 ? 2 : 4;
    for (int i = 0; i < k; ++i)  // O + O^H
        for (int j = 0; j < k; ++j) {
            rc.op[2 * (i * k + j)] = opm[2 * (i * k + j)] + opm[2 * (j * k + i)];
            rc.op[2 * (i * k + j) + 1] = opm[2 * (i * k + j) + 1] - opm[2 * (j * k + i) + 1];
        }
    rc.d0 = h->bond[site];
    rc.d1 = h->bond[site + 1];
    rc.d2 = width == 2 ? h->bond[site + 2] : 0;
    if (tape) {
        TRY(save_copy<T>(x, h->site[site].p, (size_t)rc.d0 * 2 * rc.d1, &rc.A));
        if (width == 2) TRY(save_copy<T>(x, h->site[site + 1].p, (size_t)rc.d1 * 2 * rc.d2, &rc.B));
    }
    double r3[3];
    TRY(expect_pure<T>(h, site, width, opm, r3));
    rc.val = r3[0] / r3[2];
    rc.nrm = r3[2];
    *val_out = coef * rc.val;
    if (tape) tape->push_back(rc);
    return EA_OK;
}

// ---------------------------------------------------------------- reverse

template <typename T>
int set_adjoint(Ctx &x, int site, void *src, size_t elems) {
    ea_mps *h = x.h;
    TRY(ensure(h, x.Ab[site], h->csz * elems));
    HIPCHK(h, hipMemcpyAsync(x.Ab[site].p, src, h->csz * elems, hipMemcpyDeviceToDevice, h->stream));
    return EA_OK;
}

template <typename T>
int wsalloc(Ctx &x, size_t elems, void **p) {
    return x.ws.alloc(x.h, x.h->csz * std::max<size_t>(elems, 1), p);
}

// out (m x n) = SVD adjoint for A = U diag(s) V^H (U m x r, V n x r row-major).
template <typename T>
int svd_vjp_dev(Ctx &x, const Rec &rc, const void *Ub, const double *sbar, const void *Vb,
                void *out) {
    ea_mps *h = x.h;
    hipStream_t st = h->stream;
    const int m = rc.m, n = rc.n, r = rc.r;
    void *J, *K, *P, *T1, *X1, *Q, *Z1;
    TRY(wsalloc<T>(x, (size_t)r * r, &J));
    TRY(wsalloc<T>(x, (size_t)r * r, &K));
    TRY(wsalloc<T>(x, (size_t)r * r, &P));
    TRY(wsalloc<T>(x, (size_t)r * r, &Q));
    TRY(wsalloc<T>(x, (size_t)m * r, &T1));
    TRY(wsalloc<T>(x, (size_t)m * r, &X1));
    TRY(wsalloc<T>(x, (size_t)n * r, &Z1));
    launch_gemm_ex<T>(1, 0, r, r, m, 1, 0, rc.U, r, Ub, r, 0, 0, J, r, st);
    launch_gemm_ex<T>(1, 0, r, r, n, 1, 0, rc.V, r, Vb, r, 0, 0, K, r, st);
    const double eta = x.eta_rel * rc.s0 * rc.s0 * rc.s0 * rc.s0;
    launch_svdvjp_P<T>(r, J, K, rc.s, sbar, eta, P, st);
    launch_gemm_ex<T>(0, 0, m, r, r, 1, 0, rc.U, r, P, r, 0, 0, T1, r, st);
    launch_gemm_ex<T>(0, 1, m, n, r, 1, 0, T1, r, rc.V, r, 0, 0, out, n, st);
    // (I - U U^H) Ubar S^-1 V^H
    HIPCHK(h, hipMemcpyAsync(X1, Ub, h->csz * (size_t)m * r, hipMemcpyDeviceToDevice, st));
    launch_scale_cols<T>(m, r, X1, r, rc.s, -1, st);
    launch_gemm_ex<T>(1, 0, r, r, m, 1, 0, rc.U, r, X1, r, 0, 0, Q, r, st);
    launch_gemm_ex<T>(0, 0, m, r, r, -1, 0, rc.U, r, Q, r, 1, 0, X1, r, st);
    launch_gemm_ex<T>(0, 1, m, n, r, 1, 0, X1, r, rc.V, r, 1, 0, out, n, st);
    // U S^-1 Vbar^H (I - V V^H) = U [(I - V V^H) Vbar S^-1]^H
    HIPCHK(h, hipMemcpyAsync(Z1, Vb, h->csz * (size_t)n * r, hipMemcpyDeviceToDevice, st));
    launch_scale_cols<T>(n, r, Z1, r, rc.s, -1, st);
    launch_gemm_ex<T>(1, 0, r, r, n, 1, 0, rc.V, r, Z1, r, 0, 0, Q, r, st);
    launch_gemm_ex<T>(0, 0, n, r, r, -1, 0, rc.V, r, Q, r, 1, 0, Z1, r, st);
    launch_gemm_ex<T>(0, 1, m, n, r, 1, 0, rc.U, r, Z1, r, 1, 0, out, n, st);
    LAUNCHCHK(h);
    return EA_OK;
}

template <typename T>
int rev_1q(Ctx &x, const Rec &rc) {
    ea_mps *h = x.h;
    if (rc.param >= 0) {
        double *dgd = nullptr;
        void *p = nullptr;
        TRY(stage<double>(h, rc.dg, 4, &p));  // 4 complex doubles
        dgd = (double *)p;
        launch_gbar_grad<T>(x.Ab[rc.site].p, rc.A, rc.d0, rc.d1, x.partial, dgd, x.grad, rc.param,
                            h->stream);
    }
    void *gH = nullptr;
    TRY(stage<T>(h, rc.gH, 4, &gH));
    launch_apply1<T>(x.Ab[rc.site].p, x.Ab[rc.site].p, gH, rc.d0, 2, rc.d1, h->stream);
    LAUNCHCHK(h);
    return EA_OK;
}

template <typename T>
int rev_ex(Ctx &x, const Rec &rc) {
    ea_mps *h = x.h;
    hipStream_t st = h->stream;
    const double a = rc.coef / rc.nrm, b = -2.0 * rc.coef * rc.val / rc.nrm;
    void *oh = nullptr;
    if (rc.width == 1) {
        const size_t ne = (size_t)rc.d0 * 2 * rc.d1;
        void *X;
        TRY(wsalloc<T>(x, ne, &X));
        TRY(stage<T>(h, rc.op, 4, &oh));
        launch_apply1<T>(rc.A, X, oh, rc.d0, 2, rc.d1, st);
        launch_axpby<T>(ne, b, 0, rc.A, a, 0, X, st);
        launch_axpby<T>(ne, 1, 0, X, 1, 0, x.Ab[rc.site].p, st);
    } else {
        const int M = 2 * rc.d0, K = rc.d1, N = 2 * rc.d2;
        const size_t ne = (size_t)M * N;
        void *Th, *X;
        TRY(wsalloc<T>(x, ne, &Th));
        TRY(wsalloc<T>(x, ne, &X));
        TRY(stage<T>(h, rc.op, 16, &oh));
        launch_gemm<T>(rc.A, rc.B, Th, M, N, K, K, N, N, st);
        launch_apply1<T>(Th, X, oh, rc.d0, 4, rc.d2, st);
        launch_axpby<T>(ne, b, 0, Th, a, 0, X, st);
        // Abar_s += X B^H ; Abar_{s+1} += A^H X
        launch_gemm_ex<T>(0, 1, M, K, N, 1, 0, X, N, rc.B, N, 1, 0, x.Ab[rc.site].p, K, st);
        launch_gemm_ex<T>(1, 0, K, N, M, 1, 0, rc.A, K, X, N, 1, 0, x.Ab[rc.site + 1].p, N, st);
    }
    LAUNCHCHK(h);
    return EA_OK;
}

template <typename T>
int rev_2q(Ctx &x, const Rec &rc) {
    ea_mps *h = x.h;
    hipStream_t st = h->stream;
    const int m = rc.m, n = rc.n, r = rc.r, k = rc.k;
    const int chiL = rc.d0, chiM = rc.d1, chiR = rc.d2;
    void *Ub, *Vb, *Thb, *Cb, *newA, *newB, *tmp;
    double *stbar, *sbar;
    TRY(wsalloc<T>(x, (size_t)m * r, &Ub));
    TRY(wsalloc<T>(x, (size_t)n * r, &Vb));
    TRY(wsalloc<T>(x, (size_t)m * n, &Thb));
    TRY(wsalloc<T>(x, (size_t)m * n, &Cb));
    TRY(wsalloc<T>(x, (size_t)m * chiM, &newA));
    TRY(wsalloc<T>(x, (size_t)chiM * n, &newB));
    TRY(x.ws.alloc(h, sizeof(double) * r, &tmp));
    stbar = (double *)tmp;
    TRY(x.ws.alloc(h, sizeof(double) * r, &tmp));
    sbar = (double *)tmp;
    // Ubar = [A_i'bar | 0]  (m x r)
    HIPCHK(h, hipMemsetAsync(Ub, 0, h->csz * (size_t)m * r, st));
    HIPCHK(h, hipMemcpy2DAsync(Ub, h->csz * r, x.Ab[rc.site].p, h->csz * k, h->csz * k, m,
                               hipMemcpyDeviceToDevice, st));
    // A_{i+1}' = diag(s_k / sig) V_k^H:
    //   stbar_j = Re sum_c Bbar[j][c] V[c][j];  Vbar[c][j] = (s_j / sig) conj(Bbar[j][c])
    launch_rowdot_re<T>(k, n, x.Ab[rc.site + 1].p, n, rc.V, r, stbar, st);
    launch_conjT_scaled<T>(r, k, n, x.Ab[rc.site + 1].p, n, rc.s, 1, 1.0 / rc.sig, Vb, r, st);
    launch_sbar_renorm(k, r, stbar, rc.s, rc.sig, sbar, st);
    TRY(svd_vjp_dev<T>(x, rc, Ub, sbar, Vb, Thb));
    // Cbar = G^H Thetabar (Theta viewed as (chiL, 4, chiR))
    void *gh = nullptr;
    TRY(stage<T>(h, rc.op, 16, &gh));
    launch_apply1<T>(Thb, Cb, gh, chiL, 4, chiR, st);
    // Abar = Cbar B^H (m x chiM); Bbar = A^H Cbar (chiM x n)
    launch_gemm_ex<T>(0, 1, m, chiM, n, 1, 0, Cb, n, rc.B, n, 0, 0, newA, chiM, st);
    launch_gemm_ex<T>(1, 0, chiM, n, m, 1, 0, rc.A, chiM, Cb, n, 0, 0, newB, n, st);
    LAUNCHCHK(h);
    TRY(set_adjoint<T>(x, rc.site, newA, (size_t)m * chiM));
    TRY(set_adjoint<T>(x, rc.site + 1, newB, (size_t)chiM * n));
    return EA_OK;
}

template <typename T>
int rev_move(Ctx &x, const Rec &rc) {
    ea_mps *h = x.h;
    hipStream_t st = h->stream;
    const int m = rc.m, n = rc.n, r = rc.r;
    const int c = rc.site;
    void *Ub, *Vb, *Mb, *tmp;
    double *sbar;
    TRY(wsalloc<T>(x, (size_t)m * r, &Ub));
    TRY(wsalloc<T>(x, (size_t)n * r, &Vb));
    TRY(wsalloc<T>(x, (size_t)m * n, &Mb));
    TRY(x.ws.alloc(h, sizeof(double) * r, &tmp));
    sbar = (double *)tmp;
    if (rc.kind == R_MR) {
        // A_c' = U (m x r); A_{c+1}' = X B with X = S V^H (r x n), B (n x q)
        const int q = 2 * rc.d2;
        void *X, *Xb, *newB;
        TRY(wsalloc<T>(x, (size_t)r * n, &X));
        TRY(wsalloc<T>(x, (size_t)r * n, &Xb));
        TRY(wsalloc<T>(x, (size_t)n * q, &newB));
        {  // X = S V^H = (V S)^H
            void *Vs;
            TRY(wsalloc<T>(x, (size_t)n * r, &Vs));
            HIPCHK(h, hipMemcpyAsync(Vs, rc.V, h->csz * (size_t)n * r, hipMemcpyDeviceToDevice, st));
            launch_scale_cols<T>(n, r, Vs, r, rc.s, 1, st);              // V S (n x r)
            launch_conjT_scaled<T>(n, n, r, Vs, r, rc.s, 0, 1.0, X, n, st);  // (V S)^H = S V^H
        }
        // Xbar = A_{c+1}'bar B^H (r x n); new Bbar = X^H A_{c+1}'bar (n x q)
        launch_gemm_ex<T>(0, 1, r, n, q, 1, 0, x.Ab[c + 1].p, q, rc.B, q, 0, 0, Xb, n, st);
        launch_gemm_ex<T>(1, 0, n, q, r, 1, 0, X, n, x.Ab[c + 1].p, q, 0, 0, newB, q, st);
        // sbar_j = Re sum_c Xbar[j][c] V[c][j]; Vbar[c][j] = s_j conj(Xbar[j][c])
        launch_rowdot_re<T>(r, n, Xb, n, rc.V, r, sbar, st);
        launch_conjT_scaled<T>(r, r, n, Xb, n, rc.s, 1, 1.0, Vb, r, st);
        HIPCHK(h, hipMemcpyAsync(Ub, x.Ab[c].p, h->csz * (size_t)m * r, hipMemcpyDeviceToDevice, st));
        TRY(svd_vjp_dev<T>(x, rc, Ub, sbar, Vb, Mb));
        LAUNCHCHK(h);
        TRY(set_adjoint<T>(x, c, Mb, (size_t)m * n));
        TRY(set_adjoint<T>(x, c + 1, newB, (size_t)n * q));
    } else {
        // A_c' = V^H (r x n); A_{c-1}' = P Y with Y = U S (m x r), P (p x m)
        const int p = 2 * rc.d2;
        void *Y, *Yb, *newP;
        TRY(wsalloc<T>(x, (size_t)m * r, &Y));
        TRY(wsalloc<T>(x, (size_t)m * r, &Yb));
        TRY(wsalloc<T>(x, (size_t)p * m, &newP));
        HIPCHK(h, hipMemcpyAsync(Y, rc.U, h->csz * (size_t)m * r, hipMemcpyDeviceToDevice, st));
        launch_scale_cols<T>(m, r, Y, r, rc.s, 1, st);
        // Ybar = P^H A_{c-1}'bar (m x r); new Pbar = A_{c-1}'bar Y^H (p x m)
        launch_gemm_ex<T>(1, 0, m, r, p, 1, 0, rc.B, m, x.Ab[c - 1].p, r, 0, 0, Yb, r, st);
        launch_gemm_ex<T>(0, 1, p, m, r, 1, 0, x.Ab[c - 1].p, r, Y, r, 0, 0, newP, m, st);
        // Ubar = Ybar S; sbar_j = Re sum_i conj(U[i][j]) Ybar[i][j]; Vbar[c][j] = conj(A_c'bar[j][c])
        launch_coldot_re<T>(m, r, rc.U, Yb, r, sbar, st);
        HIPCHK(h, hipMemcpyAsync(Ub, Yb, h->csz * (size_t)m * r, hipMemcpyDeviceToDevice, st));
        launch_scale_cols<T>(m, r, Ub, r, rc.s, 1, st);
        launch_conjT_scaled<T>(r, r, n, x.Ab[c].p, n, rc.s, 0, 1.0, Vb, r, st);
        TRY(svd_vjp_dev<T>(x, rc, Ub, sbar, Vb, Mb));
        LAUNCHCHK(h);
        TRY(set_adjoint<T>(x, c, Mb, (size_t)m * n));
        TRY(set_adjoint<T>(x, c - 1, newP, (size_t)p * m));
    }
    return EA_OK;
}

template <typename T>
int reverse_tape(Ctx &x, const std::vector<Rec> &tape) {
    for (auto it = tape.rbegin(); it != tape.rend(); ++it) {
        x.ws.reset();
        switch (it->kind) {
        case R_1Q: TRY(rev_1q<T>(x, *it)); break;
        case R_2Q: TRY(rev_2q<T>(x, *it)); break;
        case R_EX: TRY(rev_ex<T>(x, *it)); break;
        default: TRY(rev_move<T>(x, *it)); break;
        }
        // the workspace is reused by the next record; all kernels are on one
        // stream, so the next record's kernels start after this record's
    }
    return EA_OK;
}

template <typename T>
int snapshot(ea_mps *h, Checkpoint &cp) {
    cp.bond = h->bond;
    cp.center = h->center;
    cp.lnP = h->lnP;
    cp.lnS = h->lnS;
    cp.g = h->g;
    cp.site.resize(h->n);
    for (int i = 0; i < h->n; ++i) {
        const size_t b = h->csz * (size_t)h->bond[i] * h->d * h->bond[i + 1];
        TRY(ensure(h, cp.site[i], b));
        HIPCHK(h, hipMemcpyAsync(cp.site[i].p, h->site[i].p, b, hipMemcpyDeviceToDevice, h->stream));
    }
    return EA_OK;
}

template <typename T>
int restore(ea_mps *h, const Checkpoint &cp) {
    for (int i = 0; i < h->n; ++i) {
        const size_t b = h->csz * (size_t)cp.bond[i] * h->d * cp.bond[i + 1];
        TRY(ensure(h, h->site[i], b));
        HIPCHK(h, hipMemcpyAsync(h->site[i].p, cp.site[i].p, b, hipMemcpyDeviceToDevice, h->stream));
    }
    h->bond = cp.bond;
    h->center = cp.center;
    h->lnP = cp.lnP;
    h->lnS = cp.lnS;
    h->g = cp.g;
    return EA_OK;
}

template <typename T>
int energy_grad_impl(ea_mps *h, int n_ops, const ea_dop *ops, const double *params, int n_params,
                     int n_terms, const int *sites, const int *widths, const double *term_ops,
                     const double *coefs, double f_min, double eta_rel, double *E_out,
                     double *grad_out, double *lnP_out) {
    // device buffers (tape, workspace, adjoints, checkpoints) persist in the
    // handle between calls and are released by mps_free
    if (!h->adj) {
        h->adj = new AdjCache();
        h->adj_free = [](void *p) {
            AdjCache *c = static_cast<AdjCache *>(p);
            c->release();
            delete c;
        };
    }
    AdjCache &cache = *static_cast<AdjCache *>(h->adj);
    Ctx &x = cache.x;
    x.h = h;
    x.eta_rel = eta_rel;
    x.tape.reset();
    x.ws.reset();
    std::vector<Checkpoint> &cps = cache.cps;
    struct Cleanup {
        ea_mps *h;
        ~Cleanup() {
            if (h->stream) (void)hipStreamSynchronize(h->stream);
        }
    } cleanup{h};

    TRY(mps_reset_product(h, nullptr));
    long n2 = 0;
    for (int j = 0; j < n_ops; ++j) n2 += ops[j].kind == EA_DOP_GATE2;
    if (f_min < 1.0 && n2 > 0) TRY(mps_set_schedule(h, f_min, n2, EA_GLOBAL));
    // layers: [begin, end) op ranges
    std::vector<std::pair<int, int>> layers;
    int b0 = 0;
    for (int j = 0; j < n_ops; ++j)
        if (ops[j].layer_end || j == n_ops - 1) {
            layers.emplace_back(b0, j + 1);
            b0 = j + 1;
        }
    // device gradient and the partial sums of the angle derivatives
    TRY(ensure(h, x.gradbuf, sizeof(double) * std::max(1, n_params)));
    TRY(ensure(h, x.partbuf, sizeof(double) * 8 * 256));
    x.grad = (double *)x.gradbuf.p;
    x.partial = (double *)x.partbuf.p;
    HIPCHK(h, hipMemsetAsync(x.grad, 0, sizeof(double) * std::max(1, n_params), h->stream));

    // forward with checkpoints; the kept ranks are recorded
    std::vector<int> ranks;
    cps.resize(layers.size() + 1);
    for (size_t l = 0; l < layers.size(); ++l) {
        TRY(snapshot<T>(h, cps[l]));
        for (int j = layers[l].first; j < layers[l].second; ++j) {
            if (ops[j].kind == EA_DOP_GATE2) {
                int k = 0;
                TRY(tape_2q<T>(x, nullptr, ops[j], 0, &k));
                ranks.push_back(k);
            } else {
                TRY(tape_1q<T>(x, nullptr, ops[j], params));
            }
        }
    }
    const double lnP = h->lnP;
    const size_t log_size = h->log.size();  // recomputation below must not add records
    // energy with a tape
    std::vector<Rec> tape;
    double E = 0.0;
    size_t off = 0;
    for (int t = 0; t < n_terms; ++t) {
        double v = 0.0;
        TRY(tape_expect<T>(x, &tape, sites[t], widths[t], term_ops + 2 * off, coefs[t], &v));
        off += widths[t] == 1 ? 4 : 16;
        E += v;
    }
    TRY(snapshot<T>(h, cps.back()));
    // adjoints of the final tensors start at zero
    x.Ab.resize(h->n);
    for (int i = 0; i < h->n; ++i) {
        const size_t ne = (size_t)h->bond[i] * h->d * h->bond[i + 1];
        TRY(ensure(h, x.Ab[i], h->csz * ne));
        HIPCHK(h, hipMemsetAsync(x.Ab[i].p, 0, h->csz * ne, h->stream));
    }
    TRY(reverse_tape<T>(x, tape));
    // layers in reverse: restore, recompute with a tape, reverse
    size_t rank_pos = ranks.size();
    for (size_t l = layers.size(); l-- > 0;) {
        int n2l = 0;
        for (int j = layers[l].first; j < layers[l].second; ++j) n2l += ops[j].kind == EA_DOP_GATE2;
        rank_pos -= n2l;
        size_t rp = rank_pos;
        TRY(restore<T>(h, cps[l]));
        x.tape.reset();
        tape.clear();
        for (int j = layers[l].first; j < layers[l].second; ++j) {
            if (ops[j].kind == EA_DOP_GATE2)
                TRY(tape_2q<T>(x, &tape, ops[j], ranks[rp++], nullptr));
            else
                TRY(tape_1q<T>(x, &tape, ops[j], params));
        }
        TRY(reverse_tape<T>(x, tape));
    }
    TRY(restore<T>(h, cps.back()));
    h->log.resize(log_size);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (n_params > 0)
        HIPCHK(h, hipMemcpy(grad_out, x.grad, sizeof(double) * n_params, hipMemcpyDeviceToHost));
    h->lnP = lnP;
    if (E_out) *E_out = E;
    if (lnP_out) *lnP_out = lnP;
    return EA_OK;
}

}  // namespace

extern "C" int mps_energy_grad(ea_mps *h, int n_ops, const ea_dop *ops, const double *params,
                               int n_params, int n_terms, const int *sites, const int *widths,
                               const double *term_ops, const double *coefs, double f_min,
                               double eta_rel, double *E_out, double *grad_out,
                               double *lnP_out) {
    TRY(check(h));
    if (h->kind != EA_PURE) return set_err(EA_EINVAL, "mps_energy_grad supports pure states");
    if (h->gauge) return set_err(EA_EINVAL, "gradients need the single-centre gauge");
    if (n_ops < 1 || !ops) return set_err(EA_EINVAL, "no ops");
    if (n_params < 0 || (n_params > 0 && (!params || !grad_out)))
        return set_err(EA_EINVAL, "bad params");
    if (!(f_min > 0.0 && f_min <= 1.0)) return set_err(EA_EINVAL, "f_min must be in (0, 1]");
    if (!(eta_rel >= 0.0)) return set_err(EA_EINVAL, "eta_rel must be >= 0");
    for (int j = 0; j < n_ops; ++j) {
        const ea_dop &o = ops[j];
        const int w = o.kind == EA_DOP_GATE2 ? 2 : 1;
        if (o.kind < EA_DOP_GATE1 || o.kind > EA_DOP_GATE2)
            return set_err(EA_EINVAL, "op %d: bad kind", j);
        if (o.site < 0 || o.site + w > h->n) return set_err(EA_ERANGE, "op %d: bad site", j);
        if ((o.kind == EA_DOP_RY || o.kind == EA_DOP_RZ) &&
            (o.param < 0 || o.param >= n_params || !std::isfinite(params[o.param])))
            return set_err(EA_EINVAL, "op %d: bad parameter", j);
        if (o.kind == EA_DOP_GATE1 && (!finite_cplx(o.mat, 4) || !is_unitary(o.mat, 2)))
            return set_err(EA_EINVAL, "op %d: fixed one-qubit gates must be unitary", j);
        if (o.kind == EA_DOP_GATE2 && !finite_cplx(o.mat, 16))
            return set_err(EA_EINVAL, "op %d: bad gate", j);
    }
    if (n_terms < 0 || (n_terms > 0 && (!sites || !widths || !term_ops || !coefs)))
        return set_err(EA_EINVAL, "bad terms");
    size_t nop = 0;
    for (int t = 0; t < n_terms; ++t) {
        if (widths[t] != 1 && widths[t] != 2) return set_err(EA_EINVAL, "width must be 1 or 2");
        if (sites[t] < 0 || sites[t] + widths[t] > h->n) return set_err(EA_ERANGE, "bad term site");
        if (!std::isfinite(coefs[t])) return set_err(EA_EINVAL, "bad coefficient");
        nop += widths[t] == 1 ? 4 : 16;
    }
    if (!finite_cplx(term_ops, nop)) return set_err(EA_EINVAL, "non-finite term operator");
    // the adjoint differentiates the full factorisation of every update: the
    // partial one is off for the call and restored after it
    struct TopkOff {
        ea_mps *h;
        bool saved;
        ~TopkOff() { h->topk = saved; }
    } topk_off{h, h->topk};
    h->topk = false;
    return h->f64 ? energy_grad_impl<double>(h, n_ops, ops, params, n_params, n_terms, sites,
                                             widths, term_ops, coefs, f_min, eta_rel, E_out,
                                             grad_out, lnP_out)
                  : energy_grad_impl<float>(h, n_ops, ops, params, n_params, n_terms, sites,
                                            widths, term_ops, coefs, f_min, eta_rel, E_out,
                                            grad_out, lnP_out);
}
