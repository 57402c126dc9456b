"""ctypes binding of ``libeamps.so`` (declared in include/ea_mps.h).

Argument marshalling only: every function forwards to the C entry point of
the same name, converting NumPy arrays to interleaved complex doubles.  All
arithmetic of the gate update runs in the library's HIP kernels; if the
library is missing this module raises at import time.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# EA_MPS_LIB may name another build of the same library (for example one
# built with different tuning constants); default: the in-tree build.
LIB_PATH = os.environ.get("EA_MPS_LIB") or os.path.join(_HERE, "_lib", "libeamps.so")

EA_PURE, EA_MIXED = 0, 1
EA_C128, EA_C64, EA_C64_BF16X3 = 0, 1, 2
EA_OK, EA_WARN_CAPPED, EA_WARN_NOCONV = 0, 1, 2
EA_EINVAL, EA_ERANGE, EA_ENOMEM, EA_EHIP, EA_ETOOBIG = -1, -2, -3, -4, -5
EA_NAIVE, EA_GLOBAL, EA_NEAREST, EA_FIXED = 0, 1, 2, 3
EA_OPT_JACOBI_TOL, EA_OPT_MAX_SWEEPS, EA_OPT_TAU, EA_OPT_BLOCK, EA_OPT_CHI_MAX = 0, 1, 2, 3, 4
EA_OPT_INNER_SWEEPS, EA_OPT_JACOBI_KERNEL, EA_OPT_ROT_THREADS, EA_OPT_REORTH = 5, 6, 7, 8
EA_OPT_JACOBI_ORDER, EA_OPT_SMALL_LAYERS, EA_OPT_JACOBI_SKIP, EA_OPT_QR_PRECOND = 9, 10, 11, 12
EA_OPT_QR_MOVES, EA_OPT_RESERVE_BOND, EA_OPT_GAUGE, EA_OPT_GAUGE_PARALLEL = 13, 14, 15, 16
EA_OPT_TOPK, EA_OPT_TOPK_OVERSAMPLE, EA_OPT_TOPK_POWER, EA_OPT_TOPK_SEED = 17, 18, 19, 20
EA_OPT_TOPK_MIN = 21
EA_NOALLOC_SCRATCH_BYTES = 256 << 20

SYMBOLS = [
    "mps_init_product", "mps_free", "mps_set_option", "mps_set_schedule", "mps_apply_1q",
    "mps_apply_2q", "mps_apply_layer", "mps_fidelity_estimate", "mps_expect",
    "mps_to_statevector", "mps_bond_dims", "mps_center", "mps_gate_log", "mps_load",
    "mps_get_site", "mps_reset_product", "mps_profile", "mps_profile_read",
    "mps_apply_layer_batched", "mps_run_layers_batched", "mps_energy_grad", "ea_last_error",
    "mps_set_tuning", "mps_get_tuning", "mps_program_capture", "mps_program_launch",
    "mps_program_free", "mps_apply_layer_ranks", "mps_apply_2q_noalloc",
]

# Lorentzian broadening of the SVD adjoint's 1/(s_j^2 - s_i^2) factors,
# relative to s_0^4: F = D / (D^2 + ETA_REL_DEFAULT s_0^4), D = s_j^2 - s_i^2.
# Pairs with |D| >> 1e-6 s_0^2 keep 1/D to a relative 1e-12; closer pairs are
# damped instead of amplified without bound.
ETA_REL_DEFAULT = 1e-12

K_FAMILY_NAMES = ["theta", "jacobi_gram", "jacobi_rot", "jacobi_apply", "jacobi_fused",
                  "jacobi_small", "norms", "trunc", "gather", "gemm", "other", "centre_move", "qr",
                  "topk"]
(EA_K_THETA, EA_K_JGRAM, EA_K_JROT, EA_K_JAPPLY, EA_K_JFUSED, EA_K_JSMALL, EA_K_NORMS,
 EA_K_TRUNC, EA_K_GATHER, EA_K_GEMM, EA_K_OTHER, EA_K_MOVE, EA_K_QR, EA_K_TOPK) = range(14)
EA_K_COUNT = 14


class EAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


EA_DOP_GATE1, EA_DOP_RY, EA_DOP_RZ, EA_DOP_GATE2 = 0, 1, 2, 3


class DOp(ct.Structure):
    """One op of a differentiable circuit (ea_dop)."""
    _fields_ = [("kind", ct.c_int32), ("site", ct.c_int32), ("param", ct.c_int32),
                ("layer_end", ct.c_int32), ("mat", ct.c_double * 32)]


class TuneEntry(ct.Structure):
    """One entry of the process-wide Jacobi launch-shape table (ea_tune_entry)."""
    _fields_ = [("f64", ct.c_int32), ("n_max", ct.c_int32), ("block", ct.c_int32),
                ("rot_threads", ct.c_int32), ("chunk_wgs", ct.c_int32)]


class GateRecord(ct.Structure):
    _fields_ = [("gate", ct.c_int64), ("site", ct.c_int32), ("chi_l", ct.c_int32),
                ("chi_m", ct.c_int32), ("chi_r", ct.c_int32), ("k", ct.c_int32),
                ("k_f", ct.c_int32), ("sweeps", ct.c_int32), ("capped", ct.c_int32),
                ("subspace", ct.c_int32), ("attempts", ct.c_int32), ("f_t", ct.c_double),
                ("f", ct.c_double), ("total", ct.c_double), ("lnP", ct.c_double),
                ("lnS", ct.c_double)]


_ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p)
_FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p, ct.c_void_p)


class Allocator(ct.Structure):
    """ea_allocator: the device-memory source of a handle."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ct.c_void_p)]


def load_library(path: str = LIB_PATH) -> ct.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python paper_2307_16870_amd/_build.py`")
    lib = ct.CDLL(path)
    P, I, D, L, S = ct.c_void_p, ct.c_int, ct.c_double, ct.c_long, ct.c_size_t
    dp, ip = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)
    sig = {
        "mps_init_product": (I, [I, I, I, I, dp, ct.POINTER(Allocator), P, ct.POINTER(P)]),
        "mps_free": (None, [P]),
        "mps_set_option": (I, [P, I, D]),
        "mps_set_schedule": (I, [P, D, L, I]),
        "mps_apply_1q": (I, [P, I, dp]),
        "mps_apply_2q": (I, [P, I, dp, D, dp]),
        "mps_apply_2q_noalloc": (I, [P, I, dp, D, dp]),
        "mps_apply_layer": (I, [P, I, ip, dp, dp, dp]),
        "mps_apply_layer_ranks": (I, [P, I, ip, dp, ip, dp]),
        "mps_fidelity_estimate": (I, [P, dp, dp]),
        "mps_expect": (I, [P, I, ip, ip, dp, dp]),
        "mps_to_statevector": (I, [P, dp, S]),
        "mps_bond_dims": (I, [P, ip]),
        "mps_center": (I, [P, ip]),
        "mps_gate_log": (I, [P, ct.POINTER(GateRecord), S, ct.POINTER(S)]),
        "mps_load": (I, [P, ip, dp, I]),
        "mps_get_site": (I, [P, I, dp, S, ip]),
        "mps_reset_product": (I, [P, dp]),
        "mps_profile": (I, [P, I]),
        "mps_profile_read": (I, [P, I, dp, ct.POINTER(ct.c_long), dp, dp, ct.POINTER(ct.c_long)]),
        "mps_apply_layer_batched": (I, [I, ct.POINTER(P), ip, ct.POINTER(ip), ct.POINTER(dp),
                                        ct.POINTER(dp), ct.POINTER(dp), ip]),
        "mps_run_layers_batched": (I, [I, ct.POINTER(P), ip, ct.POINTER(ip), ct.POINTER(ip),
                                       ct.POINTER(dp), ip, ip]),
        "mps_energy_grad": (I, [P, I, ct.POINTER(DOp), dp, I, I, ip, ip, dp, dp, D, D, dp, dp, dp]),
        "ea_last_error": (ct.c_char_p, []),
        "mps_set_tuning": (I, [I, ct.POINTER(TuneEntry)]),
        "mps_program_capture": (I, [I, ct.POINTER(P), ip, ct.POINTER(ip), ct.POINTER(ip),
                                    ct.POINTER(dp), ct.POINTER(P)]),
        "mps_program_launch": (I, [P, ip, ip]),
        "mps_program_free": (None, [P]),
        "mps_get_tuning": (I, [I, ct.POINTER(TuneEntry)]),
    }
    for name, (res, args) in sig.items():
        try:
            fn = getattr(lib, name)
        except AttributeError as e:
            raise ImportError(f"{path} lacks {name}: rebuild with "
                              "`python paper_2307_16870_amd/_build.py`") from e
        fn.restype = res
        fn.argtypes = args
    return lib


# PyTorch bundles its own HIP runtime.  Loaded after this library, it becomes a
# second runtime in the process, and whichever initialises second sees no
# device; importing torch first makes this library bind to torch's runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = load_library()


def _c(a) -> np.ndarray:
    """Interleaved complex128 view (contiguous copy if needed)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _ip(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int))


def _chk(rc: int) -> int:
    if rc < 0:
        raise EAError(rc, _lib.ea_last_error().decode())
    return rc


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):  # torch.cuda.Stream
        return ct.c_void_p(stream.cuda_stream)
    return ct.c_void_p(int(stream))


def ea_last_error() -> str:
    return _lib.ea_last_error().decode()


def _torch_alloc(ctx, nbytes, stream):
    import torch
    return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))


def _torch_free(ctx, ptr, stream):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


# One process-wide instance: the callbacks must outlive every handle using it.
_TORCH_ALLOCATOR = Allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)


def torch_allocator():
    """An ea_allocator drawing device memory from torch's caching allocator
    (on the stream the library passes: the handle's stream)."""
    return _TORCH_ALLOCATOR


def mps_init_product(n_sites, kind=EA_PURE, prec=EA_C128, chi_max=0, local=None, stream=None,
                     allocator=None):
    """allocator: None (hipMalloc), "torch" (torch's caching allocator) or an
    :class:`Allocator` that outlives the handle."""
    h = ct.c_void_p()
    loc = None
    if local is not None:
        loc = _c(local)
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError(f"unknown allocator {allocator!r}")
        allocator = _TORCH_ALLOCATOR
    _chk(_lib.mps_init_product(int(n_sites), int(kind), int(prec), int(chi_max),
                               _dp(loc) if loc is not None else None,
                               ct.byref(allocator) if allocator is not None else None,
                               _stream_handle(stream), ct.byref(h)))
    return h


def mps_free(h):
    _lib.mps_free(h)


def mps_set_option(h, option, value):
    return _chk(_lib.mps_set_option(h, int(option), float(value)))


def mps_set_schedule(h, f_min, n_2q_total, strategy=EA_GLOBAL):
    return _chk(_lib.mps_set_schedule(h, float(f_min), int(n_2q_total), int(strategy)))


def mps_apply_1q(h, site, op):
    o = _c(op)
    return _chk(_lib.mps_apply_1q(h, int(site), _dp(o)))


def mps_apply_2q(h, site, op, fidelity_budget=-1.0):
    """Returns (status, achieved f)."""
    o = _c(op)
    f = ct.c_double(0.0)
    rc = _chk(_lib.mps_apply_2q(h, int(site), _dp(o), float(fidelity_budget), ct.byref(f)))
    return rc, f.value


def mps_apply_2q_noalloc(h, site, op, fidelity_budget=-1.0):
    """mps_apply_2q with its workspace in the library's fixed device array
    (no device allocation).  Returns (status, achieved f)."""
    o = _c(op)
    f = ct.c_double(0.0)
    rc = _chk(_lib.mps_apply_2q_noalloc(h, int(site), _dp(o), float(fidelity_budget),
                                        ct.byref(f)))
    return rc, f.value


def mps_apply_layer(h, sites, ops, budgets=None):
    """Returns (status, achieved f per gate in the order given)."""
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int32))
    if len(s) == 0:  # an empty layer: nothing to pass
        o = _c(np.zeros((1, 4, 4)))
    else:
        o = _c(np.stack([np.asarray(x) for x in ops]) if isinstance(ops, (list, tuple)) else ops)
    b = None if budgets is None else np.ascontiguousarray(np.asarray(budgets, dtype=np.float64))
    f = np.zeros(len(s))
    rc = _chk(_lib.mps_apply_layer(h, len(s), _ip(s), _dp(o), _dp(b) if b is not None else None,
                                   _dp(f)))
    return rc, f


def mps_apply_layer_ranks(h, sites, ops, ranks):
    """A layer with every kept rank given.  Returns (status, achieved f per
    gate in the order given)."""
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int32))
    if len(s) == 0:
        o = _c(np.zeros((1, 4, 4)))
    else:
        o = _c(np.stack([np.asarray(x) for x in ops]) if isinstance(ops, (list, tuple)) else ops)
    r = np.ascontiguousarray(np.asarray(ranks, dtype=np.int32))
    if r.size != s.size:
        raise ValueError("one rank per gate")
    f = np.zeros(len(s))
    rc = _chk(_lib.mps_apply_layer_ranks(h, len(s), _ip(s), _dp(o), _ip(r) if r.size else None,
                                         _dp(f)))
    return rc, f


def mps_fidelity_estimate(h):
    F, lnF = ct.c_double(), ct.c_double()
    _chk(_lib.mps_fidelity_estimate(h, ct.byref(F), ct.byref(lnF)))
    return F.value, lnF.value


def mps_expect(h, sites, widths, ops):
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int32))
    w = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    o = _c(np.concatenate([np.asarray(x, dtype=np.complex128).ravel() for x in ops]))
    out = np.zeros(len(s), dtype=np.complex128)
    _chk(_lib.mps_expect(h, len(s), _ip(s), _ip(w), _dp(o), _dp(out)))
    return out


def mps_to_statevector(h, n_complex):
    out = np.zeros(n_complex, dtype=np.complex128)
    _chk(_lib.mps_to_statevector(h, _dp(out), out.size))
    return out


def mps_bond_dims(h, n_sites):
    out = np.zeros(n_sites - 1, dtype=np.int32)
    _chk(_lib.mps_bond_dims(h, _ip(out)))
    return out.tolist()


def mps_center(h):
    c = ct.c_int()
    _chk(_lib.mps_center(h, ct.byref(c)))
    return c.value


def mps_gate_log(h):
    n = ct.c_size_t()
    _chk(_lib.mps_gate_log(h, None, 0, ct.byref(n)))
    recs = (GateRecord * max(1, n.value))()
    _chk(_lib.mps_gate_log(h, recs, n.value, ct.byref(n)))
    return [{f: getattr(r, f) for f, _ in GateRecord._fields_} for r in recs[: n.value]]


def mps_load(h, tensors, center):
    dims = [tensors[0].shape[0]] + [t.shape[2] for t in tensors]
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    data = _c(np.concatenate([np.asarray(t, dtype=np.complex128).ravel() for t in tensors]))
    return _chk(_lib.mps_load(h, _ip(d), _dp(data), int(center)))


def mps_get_site(h, site):
    dims = np.zeros(3, dtype=np.int32)
    _chk(_lib.mps_get_site(h, int(site), None, 0, _ip(dims)))
    out = np.zeros(int(np.prod(dims)), dtype=np.complex128)
    _chk(_lib.mps_get_site(h, int(site), _dp(out), out.size, _ip(dims)))
    return out.reshape(tuple(int(x) for x in dims))


def mps_reset_product(h, local=None):
    loc = None if local is None else _c(local)
    return _chk(_lib.mps_reset_product(h, _dp(loc) if loc is not None else None))


def mps_profile(h, every):
    """every: 0 stops; k >= 1 times one launch in k per family (True = 1)."""
    return _chk(_lib.mps_profile(h, int(every)))


def mps_profile_read(h, family):
    """One kernel family: dict(ms, ms_timed, timed, avg_ms, launches, flops,
    bytes); ms = avg_ms * launches estimates the device time of all launches
    from the timed ones."""
    ms, n, fl, by, nt = ct.c_double(), ct.c_long(), ct.c_double(), ct.c_double(), ct.c_long()
    _chk(_lib.mps_profile_read(h, int(family), ct.byref(ms), ct.byref(n), ct.byref(fl),
                               ct.byref(by), ct.byref(nt)))
    avg = ms.value / nt.value if nt.value else 0.0
    return {"ms": avg * n.value, "ms_timed": ms.value, "timed": nt.value, "avg_ms": avg,
            "launches": n.value, "flops": fl.value, "bytes": by.value}


def mps_apply_layer_batched(handles, sites_list, ops_list, budgets_list=None):
    """One layer on each state.  Returns (worst status, per-state statuses,
    per-state achieved fidelities)."""
    nb = len(handles)
    hs = (ct.c_void_p * nb)(*[h.value if isinstance(h, ct.c_void_p) else h for h in handles])
    keep = []
    ng = np.ascontiguousarray([len(s) for s in sites_list], dtype=np.int32)
    sp = (ct.POINTER(ct.c_int) * nb)()
    op = (ct.POINTER(ct.c_double) * nb)()
    bp = (ct.POINTER(ct.c_double) * nb)()
    fp = (ct.POINTER(ct.c_double) * nb)()
    fs = []
    for b in range(nb):
        s = np.ascontiguousarray(np.asarray(sites_list[b], dtype=np.int32))
        o = _c(ops_list[b])
        keep += [s, o]
        sp[b] = _ip(s)
        op[b] = _dp(o)
        if budgets_list is not None and budgets_list[b] is not None:
            bb = np.ascontiguousarray(np.asarray(budgets_list[b], dtype=np.float64))
            keep.append(bb)
            bp[b] = _dp(bb)
        f = np.zeros(len(s))
        fs.append(f)
        fp[b] = _dp(f)
    st = np.zeros(nb, dtype=np.int32)
    rc = _lib.mps_apply_layer_batched(nb, hs, _ip(ng), sp, op,
                                      bp if budgets_list is not None else None, fp, _ip(st))
    _chk(rc)
    return rc, st.tolist(), fs


def _layer_arrays(handles, layers_list):
    """ctypes arrays of a multi-circuit layer program (and the numpy arrays
    they point into, which the caller keeps alive)."""
    nb = len(handles)
    hs = (ct.c_void_p * nb)(*[h.value if isinstance(h, ct.c_void_p) else h for h in handles])
    keep = []
    nl = np.ascontiguousarray([len(L) for L in layers_list], dtype=np.int32)
    gp = (ct.POINTER(ct.c_int) * nb)()
    sp = (ct.POINTER(ct.c_int) * nb)()
    op = (ct.POINTER(ct.c_double) * nb)()
    for b in range(nb):
        counts = np.ascontiguousarray([len(layer) for layer in layers_list[b]], dtype=np.int32)
        sites = np.ascontiguousarray([g[0] for layer in layers_list[b] for g in layer],
                                     dtype=np.int32)
        mats = [np.asarray(g[1], dtype=np.complex128) for layer in layers_list[b] for g in layer]
        o = _c(np.stack(mats)) if mats else _c(np.zeros((1, 4, 4), complex))
        if sites.size == 0:
            sites = np.zeros(1, dtype=np.int32)
        if counts.size == 0:
            counts = np.zeros(1, dtype=np.int32)
        keep += [counts, sites, o]
        gp[b] = _ip(counts)
        sp[b] = _ip(sites)
        op[b] = _dp(o)
    return hs, nl, gp, sp, op, keep


def mps_run_layers_batched(handles, layers_list):
    """Leading layers of every state in one device-resident launch.
    ``layers_list[b]`` is a list of layers, each a list of (site, 4x4 or 16x16
    operator).  Returns (worst status, per-state statuses, per-state number
    of layers applied)."""
    nb = len(handles)
    hs, nl, gp, sp, op, keep = _layer_arrays(handles, layers_list)
    done = np.zeros(nb, dtype=np.int32)
    st = np.zeros(nb, dtype=np.int32)
    rc = _lib.mps_run_layers_batched(nb, hs, _ip(nl), gp, sp, op, _ip(done), _ip(st))
    _chk(rc)
    return rc, st.tolist(), done.tolist()


class Program:
    """A captured multi-circuit layer program (``mps_program_capture``)."""

    def __init__(self, ptr, n_states):
        self.ptr, self.n = ptr, n_states

    def close(self):
        if self.ptr:
            _lib.mps_program_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mps_program_capture(handles, layers_list):
    """Capture the layers of every state (as for mps_run_layers_batched) as
    one replayable HIP graph; returns a Program."""
    hs, nl, gp, sp, op, keep = _layer_arrays(handles, layers_list)
    out = ct.c_void_p()
    _chk(_lib.mps_program_capture(len(handles), hs, _ip(nl), gp, sp, op, ct.byref(out)))
    return Program(out, len(handles))


def mps_program_launch(prog):
    """Replay a Program on its states' current content.  Returns (worst
    status, per-state statuses, per-state number of layers applied)."""
    done = np.zeros(prog.n, dtype=np.int32)
    st = np.zeros(prog.n, dtype=np.int32)
    rc = _lib.mps_program_launch(prog.ptr, _ip(done), _ip(st))
    _chk(rc)
    return rc, st.tolist(), done.tolist()


def mps_program_free(prog):
    """Release a Program (also done when it is garbage-collected)."""
    prog.close()


def make_dops(ops):
    """ops: list of (kind, site, param, layer_end, mat or None) -> ctypes array."""
    arr = (DOp * len(ops))()
    for j, (kind, site, param, layer_end, mat) in enumerate(ops):
        arr[j].kind = kind
        arr[j].site = site
        arr[j].param = -1 if param is None else param
        arr[j].layer_end = int(bool(layer_end))
        if mat is not None:
            m = _c(mat).view(np.float64).ravel()
            for q in range(m.size):
                arr[j].mat[q] = m[q]
    return arr


def hea_dops(n_qubits, n_layers):
    """Hardware-efficient ansatz: per layer RY, RZ on every qubit (angles
    2*(l*n+q) and 2*(l*n+q)+1), then CZ on brickwork pairs."""
    cz = np.diag([1, 1, 1, -1]).astype(np.complex128)
    ops = []
    for l in range(n_layers):
        for q in range(n_qubits):
            ops.append((EA_DOP_RY, q, 2 * (l * n_qubits + q), False, None))
            ops.append((EA_DOP_RZ, q, 2 * (l * n_qubits + q) + 1, False, None))
        for i in range(l % 2, n_qubits - 1, 2):
            ops.append((EA_DOP_GATE2, i, None, False, cz))
        last = ops[-1]
        ops[-1] = (last[0], last[1], last[2], True, last[4])
    return ops


def mps_energy_grad(h, dops, params, terms, f_min=1.0, eta_rel=ETA_REL_DEFAULT):
    """E = sum_t c_t Re <O_t> after the circuit, and dE/dparams.  ``dops`` is
    a list for make_dops or its result; ``terms`` a list of (site, width, op,
    coef).  Returns (E, grad, lnP)."""
    arr = dops if not isinstance(dops, list) else make_dops(dops)
    prm = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
    sites = np.ascontiguousarray([t[0] for t in terms], dtype=np.int32)
    widths = np.ascontiguousarray([t[1] for t in terms], dtype=np.int32)
    ops = _c(np.concatenate([np.asarray(t[2], dtype=np.complex128).ravel() for t in terms]))
    coefs = np.ascontiguousarray([t[3] for t in terms], dtype=np.float64)
    grad = np.zeros(prm.size)
    E, lnP = ct.c_double(), ct.c_double()
    _chk(_lib.mps_energy_grad(h, len(arr), arr, _dp(prm), prm.size, len(terms), _ip(sites),
                              _ip(widths), _dp(ops), _dp(coefs), float(f_min), float(eta_rel),
                              ct.byref(E), _dp(grad), ct.byref(lnP)))
    return E.value, grad, lnP.value


_TUNE_KEYS = ("f64", "n_max", "block", "rot_threads", "chunk_wgs")


def mps_set_tuning(entries):
    """Replace the process-wide Jacobi launch-shape table; entries: dicts with
    keys f64, n_max, block, rot_threads, chunk_wgs ([] clears it)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        for k in _TUNE_KEYS:
            setattr(arr[i], k, int(e[k]))
    return _chk(_lib.mps_set_tuning(len(entries), arr))


def mps_get_tuning():
    """The current table as a list of dicts sorted by (f64, n_max)."""
    n = _chk(_lib.mps_get_tuning(0, None))
    arr = (TuneEntry * max(1, n))()
    _chk(_lib.mps_get_tuning(n, arr))
    return [{k: getattr(arr[i], k) for k in _TUNE_KEYS} for i in range(n)]


def load_tuning(path):
    """Install the table stored by the autotuner (JSON with an "entries" list)."""
    import json
    with open(path) as fh:
        return mps_set_tuning(json.load(fh)["entries"])

