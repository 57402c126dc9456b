/*
 * ea_mps.h -- C ABI of the entanglement-aware MPS / MPO gate-update library
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: M. Oliva, "An entanglement-aware quantum computer simulation
 * algorithm" (arXiv:2307.16870).  A pure state is a matrix product state
 * (Sec. II, Eq. 2); a mixed state is a matrix product operator (Sec. II,
 * Eq. 4).  The state is kept in mixed canonical form with one orthogonality
 * centre (Sec. III).  A two-qubit gate contracts the two neighbouring site
 * tensors with the gate, takes the SVD, keeps the fewest singular values
 * whose kept weight sum_kept s^2 / sum_all s^2 reaches the bond's target
 * truncation fidelity (Sec. V, Eqs. 10-11; rule of Sec. VI), and multiplies
 * the achieved truncation fidelity into the running estimate of the state
 * fidelity (Sec. VI, Eq. 12).  Targets come from F_min (Eq. 14 and the
 * adaptive updates of Sec. VI); an optional cap on the bond dimension
 * overrides them (end of Sec. VI).
 *
 * Conventions
 *   - Sites are 0-based; qubit 0 is the most significant bit of a state-vector
 *     index.  Site tensor i has shape (chi_i, d, chi_{i+1}), row-major,
 *     chi_0 = chi_N = 1; d = 2 (EA_PURE) or d = 4 (EA_MIXED, p = 2s + s' for
 *     |s><s'|).
 *   - Every complex number crossing this ABI is two doubles (re, im),
 *     interleaved, layout-compatible with C99 `double _Complex`.
 *   - One-site operators are d x d, row-major.  Two-site operators on
 *     (i, i+1) are d^2 x d^2, row-major, indexed [d*s_i + s_{i+1},
 *     d*t_i + t_{i+1}]; for EA_MIXED that is the 16x16 superoperator with
 *     p_i = 2 s_i + s_i'.
 *   - All pointers in this header are HOST pointers unless stated otherwise.
 *     The caller owns them; the library copies what it needs before the call
 *     returns.  Device memory of the state is owned by the library.
 *
 * Errors
 *   Return value 0 (EA_OK) is success, > 0 a warning (the update was applied),
 *   < 0 an error.  Arguments are validated on the host before anything is
 *   enqueued; on an error the state is unchanged, except after EA_EHIP (a HIP
 *   runtime failure), which poisons the handle: every later call on it
 *   returns EA_EHIP.  ea_last_error() returns a thread-local message for the
 *   last non-zero status.
 *
 * Threading: one handle must not be used from two threads at once; distinct
 * handles are independent.  Calls are enqueued on the handle's HIP stream;
 * calls that return host data synchronise that stream.
 */
#ifndef EA_MPS_H
#define EA_MPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ea_mps ea_mps; /* opaque handle, owned by the library */

enum ea_kind { EA_PURE = 0, EA_MIXED = 1 };

/* Arithmetic of the state and of the update.
 * EA_C128: complex FP64 everywhere.
 * EA_C64:  complex FP32 storage, contraction and Jacobi rotations; singular
 *          values, the kept-weight search and the fidelity product in FP64.
 * EA_C64_BF16X3: as EA_C64, with the two-site contraction done as three
 *          BF16 products per real product (x = hi + lo; hi*hi + hi*lo +
 *          lo*hi) with FP32 accumulation. */
enum ea_prec { EA_C128 = 0, EA_C64 = 1, EA_C64_BF16X3 = 2 };

enum ea_status {
    EA_OK = 0,
    EA_WARN_CAPPED = 1, /* chi_max bound: target truncation fidelity not met */
    EA_WARN_NOCONV = 2, /* Jacobi stopped at max_sweeps */
    EA_EINVAL = -1,     /* bad argument */
    EA_ERANGE = -2,     /* site index out of range */
    EA_ENOMEM = -3,     /* device allocation failed */
    EA_EHIP = -4,       /* HIP runtime error; handle poisoned */
    EA_ETOOBIG = -5     /* output buffer too small / N too large */
};

/* Target schedules (Sec. VI).  EA_FIXED is the standard fixed-bond-dimension
 * simulation the paper compares against (Sec. VI, Fig. 4): every target is 1,
 * so only numerically zero values and the chi_max cap truncate. */
enum ea_strategy { EA_NAIVE = 0, EA_GLOBAL = 1, EA_NEAREST = 2, EA_FIXED = 3 };

/* Device-memory source of a handle.  alloc(ctx, bytes, stream) returns device
 * memory usable by work enqueued on `stream` (a hipStream_t), or NULL;
 * free(ctx, ptr, stream) releases it (the library has synchronised the
 * stream first, or frees only memory that no pending work uses).  Both may be
 * called from the thread that calls into the library, including the host
 * workers of mps_apply_layer_batched.  Used, for example, to draw the state's
 * memory from a framework's caching allocator.  Not part of the paper. */
typedef struct ea_allocator {
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
    void *ctx;
} ea_allocator;

enum ea_option {
    EA_OPT_JACOBI_TOL = 0,   /* rotate a pair if |g| > tol*sqrt(a b); default m*eps */
    EA_OPT_MAX_SWEEPS = 1,   /* default 40 */
    EA_OPT_TAU = 2,          /* numerical-zero cutoff tau*s_0; 1e-13 (FP64), 2e-6 (FP32) */
    EA_OPT_BLOCK = 3,        /* Jacobi column-block width (0 = automatic: 32 for the
                                three-kernel form) */
    EA_OPT_CHI_MAX = 4,      /* cap on kept rank; 0 = none */
    EA_OPT_INNER_SWEEPS = 5, /* rotation sweeps over a block pair's Gram per round (default 1) */
    EA_OPT_JACOBI_KERNEL = 6,/* 0: Gram / rotations / apply as three kernels (MFMA);
                                1: one fused kernel per round (vector ALU) */
    EA_OPT_ROT_THREADS = 7,  /* threads of the per-pair rotation kernel: 64, 128, 256, 512,
                                1024, or 0 (default: 16 per column of a block pair) */
    EA_OPT_REORTH = 8,       /* FP32 precisions: 1 (default) divides the right singular
                                vectors of every factorisation by their FP64 norms (the
                                rotations leave a norm drift) and re-orthogonalises every
                                isometric factor in FP64 (Loewdin steps, the neighbour
                                absorbing the inverse factor), holding X^H X - I and the
                                change of the product within 1e-6; 0: neither */
    EA_OPT_JACOBI_ORDER = 9, /* three-kernel Jacobi: 1 (default) rotates the column pairs
                                inside a block in the first round of a sweep only, later
                                rounds rotate only pairs across the two blocks (every pair
                                once per sweep); 0 rotates all pairs of the block pair in
                                every round */
    EA_OPT_SMALL_LAYERS = 10, /* c = 64 (default) or 128: a layer whose every bond is at
                                most c / d runs as one device-resident launch (one
                                workgroup per state walks the layer, sizes read on the
                                device, no host synchronisation between its gates;
                                mps_apply_layer and mps_apply_layer_batched, where all
                                such states share one launch); 0: host-orchestrated */
    EA_OPT_JACOBI_SKIP = 11, /* three-kernel Jacobi: 1 (default) skips a column block pair
                                whose two blocks are unchanged since the pair was last
                                examined (it would find the same Gram matrix and no
                                rotation, so results are bit-identical); 0 examines every
                                pair in every sweep */
    EA_OPT_QR_MOVES = 13,    /* centre moves of the update path (Sec. III): 2 (default):
                                Cholesky QR in FP64 (A_c = Q R, Q the new site, R absorbed
                                into the neighbour; matrix-core GEMMs and a blocked
                                Cholesky; a second pass when the first Q is not orthonormal
                                to 1e-8 for FP32 sites or 1e-13 for FP64), no rank dropped; a site whose condition number
                                exceeds about 1e7 (a Cholesky pivot below 1e-14 of the
                                largest diagonal entry), or whose matrix is wider than
                                tall, moves by the Jacobi SVD instead.  1: Householder QR,
                                no rank dropped.  0: the Jacobi SVD, dropping numerically
                                zero singular values.  The gradient path (mps_energy_grad)
                                always moves by SVD. */
    EA_OPT_GAUGE_PARALLEL = 16, /* layer-parallel gauge: 1 (default) runs the gates of a layer
                                side by side, each on a stream and host thread of its own
                                (the same bits as one after another); 0: one after another
                                on the state's stream. */
    EA_OPT_GAUGE = 15,       /* 1: from a product state, switch to the layer-parallel gauge
                                (Vidal's form, B_i = Gamma_i Lambda_{i+1} and each bond's
                                Schmidt values; Hastings' update, no division by Lambda):
                                the two-site updates of a layer are independent of each
                                other (no centre moves), every gate of a layer takes its
                                target from the estimate before the layer, and f is the
                                kept weight of diag(Lambda_i) G (B_i B_{i+1}), exact while
                                no truncation has happened and approximate after.  Not
                                in the paper, which keeps one orthogonality centre
                                (Sec. III, VI).  mps_expect, gradients, the batched small-
                                bond launches and the allocation-free update refuse a
                                state in this gauge (EA_EINVAL).  0: back to one centre
                                (exact moves from the last site to the first: the centre
                                ends on site 0). */
    EA_OPT_RESERVE_BOND = 14,/* chi > 0: grow every site tensor's buffer now to hold a
                                (chi, d, chi) tensor (never shrunk), so that later updates up
                                to bond chi need no new site memory, as the allocation-free
                                entry point requires.  Allocates; EA_ENOMEM on failure. */
    EA_OPT_TOPK = 17,        /* 1: a two-site update whose matrix X (Theta, or Theta^H when
                                it is wider than tall; mw x nw, mw >= nw) has at least
                                EA_OPT_TOPK_MIN columns takes a partial factorisation when
                                a subspace of l = min(chi_max, 2 chi_m) + p columns (p =
                                EA_OPT_TOPK_OVERSAMPLE) satisfies 4 l <= 3 nw: randomized
                                subspace iteration in FP64 (Y = X^H Omega, then q =
                                EA_OPT_TOPK_POWER times Y = X^H (X Y), Q = orth(Y) by
                                Cholesky QR2, shifted first if ill-conditioned; Omega from
                                SplitMix64, seed EA_OPT_TOPK_SEED, counters from the gate
                                index and attempt), the Jacobi
                                SVD of X Q (mw x l) in the working precision, and the kept
                                rank of Sec. VI from its singular values with every
                                discarded weight raised by R = ||X||_F^2 - ||X Q||_F^2 (so
                                f is the exact fidelity of the state kept).  Accepted when
                                the kept rank is at most l - p, else l doubles; when 4 l >
                                3 nw, or orth meets a rank-deficient block, the full
                                factorisation runs.  Not in the paper (Sec. V takes the
                                full SVD); k may exceed the full SVD's, and a capped update
                                may keep less weight.  Off (0) by default; never used by
                                forced ranks, the layer-parallel gauge, the small-bond
                                launches, gradients (mps_energy_grad differentiates the
                                full factorisation) or the allocation-free entry point. */
    EA_OPT_TOPK_OVERSAMPLE = 18, /* p, 1..512 (default 64) */
    EA_OPT_TOPK_POWER = 19,  /* q, 0..4 subspace iterations (default 1); Y's condition
                                number grows as (s_0 / s_l)^(2q+1), and a block that the
                                shifted Cholesky QR cannot resolve takes the full
                                factorisation */
    EA_OPT_TOPK_SEED = 20,   /* seed of the start block, an integer in [0, 2^53) (default 0) */
    EA_OPT_TOPK_MIN = 21,    /* smallest nw that tries the partial factorisation (default 256) */
    EA_OPT_QR_PRECOND = 12   /* w > 0: a factorisation of at least w columns on the
                                three-kernel Jacobi first takes the Householder QR of its
                                matrix (Theta = Q R, panels on one workgroup each, trailing
                                updates and products with Q as matrix-core GEMMs) and runs the
                                Jacobi on R^H, whose columns are nearer orthogonal (fewer
                                sweeps); the SVD of Theta is then (Q V_x) S U_x^H.  0: off */
};

/* ---- Captured programs (HIP graph of the device-resident launch) ---- */

typedef struct ea_program ea_program; /* opaque, library-owned */

/* Capture the two-qubit-gate layers of n_states circuits (arguments as for
 * mps_run_layers_batched) as one HIP graph: an upload of the states'
 * descriptors from pinned host memory, the persistent device-resident launch
 * of each precision present (one workgroup per state walks its layers; Sec.
 * V-VI per gate, global/naive/nearest schedule only), and a read-back.  The
 * layers and gates are copied to device memory owned by the program; no
 * state is changed.  Every state needs EA_OPT_SMALL_LAYERS != 0, at most 256
 * gates per layer, and must outlive the program.  EA_EINVAL on bad arguments
 * or a state given twice; EA_ENOMEM; EA_EHIP if the capture fails. */
int mps_program_capture(int n_states, ea_mps *const *hs, const int *n_layers,
                        const int *const *layer_gates, const int *const *sites,
                        const double *const *ops, ea_program **out);

/* Replay the program on the states' current content: each state's
 * descriptor (site pointers, bonds, centre, fidelity log, schedule, options)
 * is refreshed on the host, then the graph runs on the first state's stream
 * (the other states' streams are synchronised first) and the results are
 * applied to the handles as by mps_run_layers_batched.  layers_done (may be
 * NULL): layers each state completed; a state stops before the first layer
 * at which one of its bonds exceeds the small limit, and the caller goes on
 * from there.  Returns the worst status, per state in status_out (may be
 * NULL).  Launches of one program, or of programs sharing a state, must not
 * overlap. */
int mps_program_launch(ea_program *p, int *layers_done, int *status_out);

/* Release the program (waits for its stream).  NULL is a no-op. */
void mps_program_free(ea_program *p);

/* ---- Launch-shape tuning (written by the package's autotuner) ---- */

/* One entry of the process-wide tuning table of the three-kernel Jacobi. */
typedef struct ea_tune_entry {
    int32_t f64;         /* 0: FP32 working data (EA_C64, EA_C64_BF16X3); 1: EA_C128 */
    int32_t n_max;       /* covers factorisations of n <= n_max columns not covered
                            by an entry of the same f64 with a smaller n_max */
    int32_t block;       /* column-block width: 16 or 32 */
    int32_t rot_threads; /* threads of the rotation kernel: 64, 128, 256, 512, 1024 */
    int32_t chunk_wgs;   /* workgroups targeted by the Gram and apply launches, 64..4096 */
} ea_tune_entry;

/* Replace the process-wide tuning table (copied; n_entries = 0 clears it).
 * A factorisation of n > 64 columns on the three-kernel Jacobi takes the
 * entry of its precision with the smallest n_max >= n: its row-chunk target
 * always, its block width when the handle's EA_OPT_BLOCK is 0, and its
 * rotation threads when EA_OPT_BLOCK and EA_OPT_ROT_THREADS are both 0 (a set
 * option wins).  Without an entry: block 32, 1024 rotation threads (512 at
 * block 16), 256 workgroups.  Results depend on
 * the block width only through rounding.  EA_EINVAL, table unchanged, on a
 * malformed entry or two entries with the same (f64, n_max).  Host only (no
 * device call); safe to call from any thread, a factorisation already
 * running keeps the shape it chose. */
int mps_set_tuning(int n_entries, const ea_tune_entry *entries);

/* Copies up to `capacity` entries of the table, sorted by (f64, n_max), into
 * out; returns the number of entries (or EA_EINVAL). */
int mps_get_tuning(int capacity, ea_tune_entry *out);

/* One record per two-site update (Sec. VI bookkeeping; Figs. 1-4 plot these). */
typedef struct ea_gate_record {
    int64_t gate;    /* 0-based index among two-qubit updates */
    int32_t site;    /* left site */
    int32_t chi_l, chi_m, chi_r; /* bonds before the update */
    int32_t k;       /* kept rank = new chi_m */
    int32_t k_f;     /* rank asked for by the target alone */
    int32_t sweeps;  /* Jacobi sweeps used */
    int32_t capped;  /* 1 if chi_max bound */
    int32_t subspace;/* EA_OPT_TOPK: dimension l of the subspace the kept values came
                        from; 0 for a full factorisation */
    int32_t attempts;/* EA_OPT_TOPK: subspace attempts made (the last one accepted
                        when subspace > 0); 0 when none was tried */
    double f_t;      /* target truncation fidelity */
    double f;        /* achieved truncation fidelity 1 - D(k)/T */
    double total;    /* T = sum of all s^2 */
    double lnP;      /* running log fidelity estimate after this update */
    double lnS;      /* EA_MIXED: running log of the scale removed by renormalising the
                        kept values (the unnormalised truncated state is exp(lnS) times
                        the stored one); 0 for EA_PURE */
} ea_gate_record;

/* Create a product state (Sec. VI: simulations start from a product state;
 * Sec. II, Eq. 2 with every bond dimension 1).
 *  n_sites >= 2; kind: ea_kind; prec: ea_prec; chi_max: cap on the kept rank
 *  (0 = no cap, end of Sec. VI).
 *  local: NULL for |0...0> (pure) or |0><0|^N (mixed), else n_sites*d complex
 *  numbers, the d-vector of each site (vec(rho_i) for EA_MIXED).
 *  alloc: NULL = hipMalloc / hipFree, else the source of all of the handle's
 *  device memory (copied; its ctx must stay valid until mps_free).  Pinned
 *  host staging buffers always come from hipHostMalloc.
 *  hip_stream: hipStream_t on which all work is enqueued; NULL = a private
 *  non-blocking stream created (default priority) and destroyed with the
 *  handle.
 *  out: receives the handle.  Returns EA_EINVAL on bad arguments, EA_ENOMEM if
 *  device memory cannot be allocated. */
int mps_init_product(int n_sites, int kind, int prec, int chi_max,
                     const double *local, const ea_allocator *alloc, void *hip_stream,
                     ea_mps **out);

/* Release the handle and all its device memory (library bookkeeping, not
 * part of the paper).  Synchronises the handle's stream first.  NULL is
 * ignored. */
void mps_free(ea_mps *h);

/* Tuning and numerical options (ea_option).  EA_EINVAL on unknown option or
 * out-of-range value. */
int mps_set_option(ea_mps *h, int option, double value);

/* Target schedule (Sec. VI): F_min in (0, 1], n_2q_total >= 1 two-qubit gates
 * to come, strategy ea_strategy: naive f_t = F_min^(1/n) (Eq. 14); global
 * f_t = (F_min / P)^(1/(n - g)) before gate g; nearest f_t = F_min^((g+1)/n)
 * / P; fixed f_t = 1 (only the cap truncates).  Targets are clamped to
 * (0, 1].  Without a schedule every target is 1 (only numerically zero
 * singular values are dropped). */
int mps_set_schedule(ea_mps *h, double f_min, long n_2q_total, int strategy);

/* One-site operator (Sec. II: one-qubit gates do not change bond dimensions).
 *  op: d x d complex (2x2 unitary, or 4x4 superoperator for EA_MIXED).
 *  A non-unitary operator first moves the orthogonality centre to `site`. */
int mps_apply_1q(ea_mps *h, int site, const double *op);

/* Two-site update on (site, site+1) (Sec. V-VI).
 *  op: d^2 x d^2 complex gate / superoperator.
 *  fidelity_budget: target truncation fidelity f_t in (0, 1]; a negative
 *  value takes the next target from the schedule.
 *  f_out: if non-NULL receives the achieved truncation fidelity.
 *  The centre ends on site+1.  Returns EA_WARN_CAPPED if chi_max bound. */
int mps_apply_2q(ea_mps *h, int site, const double *op, double fidelity_budget,
                 double *f_out);

/* Size of the device array that holds the workspace of mps_apply_2q_noalloc:
 * one per GPU the library runs on, held until the process ends. */
#define EA_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* mps_apply_2q without any device allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, update, result and
 * warnings as mps_apply_2q, except:
 *  - no device memory is allocated or freed (no hipMalloc / hipFree, no
 *    allocator callback, no library routine that allocates): the update's
 *    workspace (two-site matrix, Jacobi buffers, centre-move and FP64
 *    re-orthogonalisation buffers) is carved from one library-owned device
 *    array of EA_NOALLOC_SCRATCH_BYTES per GPU, and every site tensor's
 *    buffer must already hold its result (grown by earlier updates, or
 *    reserved with EA_OPT_RESERVE_BOND);
 *  - EA_ETOOBIG when the workspace would exceed the array (about bond 1024 for
 *    a pure state in complex FP32 or FP64) or a site buffer is too small; the
 *    state is then unchanged except that the orthogonality centre may have
 *    moved (an exact re-gauging of the same state);
 *  - all calls on one GPU share the array, which keeps the last call's
 *    contents (nothing in it is assumed to start at zero): calls that overlap
 *    on one GPU race (other threads, or another stream before this call's
 *    work has finished); calls on one stream are ordered;
 *  - the calling thread's current device must be the handle's (EA_EINVAL);
 *  - event timing (mps_profile) is suspended for the call.
 * The host-side gate log still grows by one record. */
int mps_apply_2q_noalloc(ea_mps *h, int site, const double *op, double fidelity_budget,
                         double *f_out);

/* A layer of two-site updates on disjoint pairs (sites[j], sites[j]+1): the
 * update of Sec. V-VI applied to each gate of one circuit layer.  The paper
 * applies gates one at a time with the canonical form kept (Sec. III, VI);
 * the visiting order below is this library's choice (the centre walks the
 * layer once, serpentine over a brickwork circuit).
 *  ops: n_gates consecutive d^2 x d^2 complex matrices.
 *  budgets: NULL (schedule) or n_gates targets, one per gate in the order
 *  given.  Gates are visited in increasing site order if the centre is
 *  nearer the lowest site, else in decreasing order; the centre follows.
 *  f_out: NULL or n_gates achieved fidelities, in the order given.
 *  EA_EINVAL if two pairs overlap; then nothing is applied. */
int mps_apply_layer(ea_mps *h, int n_gates, const int *sites, const double *ops,
                    const double *budgets, double *f_out);

/* Kept ranks forced (Sec. V-VI update with the truncation rule replaced):
 * as mps_apply_layer with the schedule's targets, except that gate j keeps
 * exactly min(ranks[j], r) singular values, r the number of singular values
 * of its two-site matrix, renormalised as usual; f and the estimate are those
 * of the rank kept, and no update is flagged as capped.  Replays a run with
 * given kept ranks (comparison with a reference whose rank decision sits
 * within rounding of the threshold) and runs fixed-rank schedules.  The
 * schedule's gate counter advances as usual.  ranks[j] >= 1, else EA_EINVAL
 * and nothing is applied.  Always host-orchestrated. */
int mps_apply_layer_ranks(ea_mps *h, int n_gates, const int *sites, const double *ops,
                          const int *ranks, double *f_out);

/* One layer on each of several independent states.  The paper does not batch
 * circuits; independent circuits share nothing, so each state receives the
 * Sec. V-VI updates exactly as from mps_apply_layer.  State b applies
 * n_gates[b] two-site updates given, as for mps_apply_layer, by sites[b],
 * ops[b] and budgets[b]
 * (budgets may be NULL, or budgets[b] NULL, for the schedule); f_out may be
 * NULL or hold n_states pointers (each NULL or n_gates[b] doubles).  The
 * states advance concurrently, one host worker per state, each enqueuing on
 * its own handle's stream, so their kernels overlap on the GPU; pass states
 * created with distinct streams (or NULL streams, which give each handle a
 * private stream).  status_out (n_states ints, may be NULL) receives each
 * state's status.  Returns the most severe status (errors < warnings). */
int mps_apply_layer_batched(int n_states, ea_mps *const *hs, const int *n_gates,
                            const int *const *sites, const double *const *ops,
                            const double *const *budgets, double *const *f_out,
                            int *status_out);

/* Leading layers of many independent circuits in ONE device-resident launch
 * (Sec. V-VI; the same updates as repeated mps_apply_layer calls with the
 * schedule of mps_set_schedule, no per-gate targets).  One workgroup per
 * state walks its layers in order (centre moves, contraction, SVD, kept-rank
 * rule, write-back, fidelity product) with every size read on the device, and
 * stops before the first layer at which some bond exceeds the small-layer
 * limit (EA_OPT_SMALL_LAYERS c: bonds <= c / d; c = 0 runs nothing).  A state
 * that does not qualify when the call starts is left untouched.
 *   n_layers[b]       layers offered for state b
 *   layer_gates[b][L] number of two-qubit gates in layer L of state b
 *   sites[b]          left sites of all its gates, layer after layer
 *   ops[b]            their operators, complex d^2 x d^2 row-major each
 *                     (interleaved re, im doubles), in the same order
 *   layers_done[b]    out: layers applied; the caller continues from there
 *                     (for example with mps_apply_layer_batched)
 *   status_out[b]     out (may be NULL): each state's status
 * Host arrays are read during the call only.  The states synchronise their
 * streams first.  Returns the most severe status (errors < warnings). */
int mps_run_layers_batched(int n_states, ea_mps *const *hs, const int *n_layers,
                           const int *const *layer_gates, const int *const *sites,
                           const double *const *ops, int *layers_done, int *status_out);

/* Running estimate of the state fidelity, prod_i f_i (Eq. 12; Eq. 13 for
 * noisy runs, where it is a lower estimate).  Either pointer may be NULL. */
int mps_fidelity_estimate(const ea_mps *h, double *F_out, double *lnF_out);

/* Expectation values (Sec. III, Eqs. 5-6).  Term j acts on sites[j]
 * (widths[j] = 1, d x d operator) or (sites[j], sites[j]+1) (widths[j] = 2,
 * 4x4 operator on the two qubits, NOT a superoperator).  ops: the operators
 * concatenated.  out: n_terms complex values.  Pure: <psi|O|psi>/<psi|psi>
 * from the centre block (the centre is moved).  Mixed: Tr(rho O)/Tr(rho). */
int mps_expect(ea_mps *h, int n_terms, const int *sites, const int *widths,
               const double *ops, double *out);

/* Dense output (Eq. 1 / Eq. 3).  Pure: the 2^N amplitudes (N <= 28),
 * out_complex_len >= 2^N.  Mixed: rho / Tr(rho) as a row-major 2^N x 2^N
 * matrix (N <= 13), out_complex_len >= 4^N.  EA_ETOOBIG otherwise. */
int mps_to_statevector(ea_mps *h, double *out, size_t out_complex_len);

/* Bond dimensions chi_1 .. chi_{N-1} (Sec. II, Eq. 2; plotted in Figs. 2-4)
 * into out (n_sites - 1 ints). */
int mps_bond_dims(const ea_mps *h, int *out);

/* Current orthogonality centre (site index). */
int mps_center(const ea_mps *h, int *out);

/* Copy the per-update records (oldest first).  n_out receives the number of
 * records available; at most `cap` are written. */
int mps_gate_log(const ea_mps *h, ea_gate_record *records, size_t cap, size_t *n_out);

/* Replace the whole state by explicit site tensors (checkpoint restore and
 * tests).  bond_dims: n_sites+1 ints with both ends 1.  data: the site
 * tensors concatenated, complex, each (chi_i, d, chi_{i+1}) row-major.
 * center: orthogonality centre the caller vouches for.  The fidelity log,
 * estimate and gate counter are left as they are. */
int mps_load(ea_mps *h, const int *bond_dims, const double *data, int center);

/* Copy site tensor `site` (chi_l*d*chi_r complex) into out; dims receives
 * (chi_l, d, chi_r).  EA_ETOOBIG if out_complex_len is too small. */
int mps_get_site(ea_mps *h, int site, double *out, size_t out_complex_len, int *dims);

/* Reset the handle to a product state exactly as mps_init_product would
 * create it (local as there), keeping its device buffers.  Clears the
 * fidelity estimate, the gate counter, the schedule and the gate log. */
int mps_reset_product(ea_mps *h, const double *local);

/* Kernel families timed by mps_profile (tracing aid, Sec. VI bookkeeping is
 * unaffected). */
enum ea_kfamily {
    EA_K_THETA = 0,        /* two-site contraction + gate */
    EA_K_JGRAM = 1,        /* Jacobi round, part 1: MFMA partial Gram matrices */
    EA_K_JROT = 2,         /* Jacobi round, part 2: rotations of each block pair */
    EA_K_JAPPLY = 3,       /* Jacobi round, part 3: MFMA apply to W and V */
    EA_K_JFUSED = 4,       /* Jacobi round as one fused kernel (vector ALU) */
    EA_K_JSMALL = 5,       /* single-workgroup Jacobi (<= 64 columns) */
    EA_K_NORMS = 6,        /* singular values as column norms */
    EA_K_TRUNC = 7,        /* sort + kept-rank search */
    EA_K_GATHER = 8,       /* write-back of the new site tensors */
    EA_K_GEMM = 9,         /* absorb products (centre moves, chain contraction) */
    EA_K_OTHER = 10,
    EA_K_MOVE = 11,        /* whole centre moves (overlaps the families above) */
    EA_K_QR = 12,          /* QR: preconditioning panels and products, Cholesky QR passes */
    EA_K_TOPK = 13,        /* partial factorisation: start block, range-finder products,
                              the weight outside the subspace, right vectors */
    EA_K_COUNT = 14
};

/* every >= 1: reset the counters and start counting every kernel launch of
 * this handle with its algorithmic flops and bytes, and timing one launch in
 * `every` of each family (the 1st, (every+1)th, ...) with a pair of HIP events
 * on its stream; every = 1 times all launches (each event pair adds host and
 * device overhead to the run).  0: stop.  EA_EINVAL if every < 0. */
int mps_profile(ea_mps *h, int every);

/* For one family: the device time (ms) of the timed launches and their
 * number, the number of all launches and their algorithmic floating-point
 * operations and bytes.  The average launch time is ms_timed / timed.
 * Synchronises the handle's stream.  Any output pointer may be NULL. */
int mps_profile_read(ea_mps *h, int family, double *ms_timed, long *launches,
                     double *flops, double *bytes, long *timed);

/* ---- Differentiation (adjoint of the update with kept ranks frozen) ---- */

enum ea_dop_kind {
    EA_DOP_GATE1 = 0, /* fixed one-qubit unitary (mat: 2x2) */
    EA_DOP_RY = 1,    /* RY(params[param]) = exp(-i t Y / 2) */
    EA_DOP_RZ = 2,    /* RZ(params[param]) = exp(-i t Z / 2) */
    EA_DOP_GATE2 = 3  /* fixed two-qubit gate on (site, site+1) (mat: 4x4) */
};

/* One operation of a differentiable circuit. */
typedef struct ea_dop {
    int32_t kind;      /* ea_dop_kind */
    int32_t site;
    int32_t param;     /* index into params (RY/RZ), else ignored */
    int32_t layer_end; /* non-zero: a per-layer checkpoint follows this op */
    double mat[32];    /* fixed gate, row-major complex: 2x2 (GATE1) or 4x4 (GATE2) */
} ea_dop;

/* Energy and gradient through the entanglement-aware simulation (pure
 * states, EA_PURE handles of any precision).  Starting from |0...0>, applies
 * the ops in order (two-site updates as mps_apply_2q, Sec. V-VI, with the
 * global schedule for f_min if f_min < 1, else only numerically zero
 * singular values are dropped), then evaluates
 *     E = sum_t coefs[t] Re <O_t>
 * with <O_t> as in mps_expect (Eq. 6), and the gradient dE/dparams with every
 * kept rank frozen to the forward pass's choice: reverse passes through the
 * one-qubit gates, the contraction (products with G^H), the truncated complex
 * SVD (kept/discarded coupling through 1/(s_j^2 - s_i^2), broadened to
 * (s_j^2 - s_i^2)/((s_j^2 - s_i^2)^2 + eta_rel s_0^4), phase term,
 * renormalisation) and the centre moves.  The state is checkpointed at every
 * layer end and each layer is recomputed once during the reverse pass.
 * Outputs: E_out, grad_out (n_params doubles), lnP_out (ln of the fidelity
 * estimate; any may be NULL except grad_out when n_params > 0).  On return the
 * handle holds the final state of the circuit. */
int mps_energy_grad(ea_mps *h, int n_ops, const ea_dop *ops, const double *params,
                    int n_params, int n_terms, const int *sites, const int *widths,
                    const double *term_ops, const double *coefs, double f_min,
                    double eta_rel, double *E_out, double *grad_out, double *lnP_out);

/* Message for the last non-zero status returned on this thread. */
const char *ea_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EA_MPS_H */
