"""Precision variants of the update: complex FP32 with FP64 re-orthogonalised
isometric factors, and the BF16x3 contraction (FP32 operands split into bf16
hi/lo parts, three products each, FP32 accumulation).  Tolerances follow the
arithmetic: BF16x3 products carry a relative error of about 2^-16, FP32
products 2^-24, both far below the truncation errors the method tolerates."""
import sys

import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.mps import OracleMPS
from tests.gpu_util import gauge_free_pair, protected

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_bf16x3_config1_exact():
    """12 qubits, depth 8, no truncation: amplitudes against brute force."""
    _say("case: bf16x3 config1")
    prog, c = C.config_program(1)
    with P.EAState(prog.n_sites, "pure", "bf16x3", chi_max=c["chi_max"]) as st:
        st.run(prog, 1.0)
        psi = st.statevector()
        F, _ = st.fidelity_estimate()
    ref = brute.run_statevector(prog)
    err = np.abs(psi - ref).max() / np.abs(ref).max()
    _say("bf16x3 amplitude max relative error", err)
    assert err < 1e-3
    assert abs(F - 1.0) < 1e-4
    assert abs(brute.fidelity_pure(ref, psi) - 1.0) < 1e-5


_CACHE = {}


@pytest.mark.parametrize("kind,chis,prec", [
    ("pure", (300, 260, 333), "bf16x3"),
    ("pure", (300, 260, 333), "c64"),
    ("mixed", (70, 90, 65), "bf16x3"),
])
def test_reduced_precision_single_update(kind, chis, prec):
    """One update across several contraction tiles with ragged edges (pure
    d = 2 and MPO d = 4): total weight, fidelity, rank and the gauge-free
    truncated product against the FP64 oracle."""
    _say("case: reduced precision update", kind, chis, prec)
    d = 2 if kind == "pure" else 4
    chiL, chiM, chiR = chis
    tens = C.random_mps_tensors([1, chiL, chiM, chiR, 1], d, seed=sum(chis) + d)
    rng = np.random.default_rng(9)
    u = C.haar_unitary(rng)
    G = u if d == 2 else C.depolarizing2_superop(2e-3) @ C.unitary_superop(u)
    f_t = 0.99
    key = (kind, chis)
    if key not in _CACHE:
        o = OracleMPS(4, kind, keep_spectra=True, svd="lapack")
        o.load(tens, 1)
        _CACHE[key] = (o, o.apply_2q(1, G, f_t))
    o, rec = _CACHE[key]
    with P.EAState(4, kind, prec) as st:
        st.load(tens, 1)
        rc, f = st.apply_2q(1, G, f_t)
        g = st.gate_log()[0]
        a1, a2 = st.site(1), st.site(2)
    T = float(np.sum(rec.s ** 2))
    rel = 2e-4 if prec == "bf16x3" else 2e-5
    _say("total rel err", abs(g["total"] - T) / T, "f err", abs(f - rec.f))
    assert abs(g["total"] - T) < rel * T
    assert abs(f - rec.f) < rel
    assert g["k"] == rec.k or not protected(rec, f_t, 10 * rel)
    if g["k"] == rec.k:
        got = gauge_free_pair(a1, a2)
        ref = gauge_free_pair(o.A[1], o.A[2])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say("A_1 A_2 relative Frobenius error", err)
        assert err < (5e-3 if prec == "bf16x3" else 5e-4)


@pytest.mark.parametrize("prec", ["c64", "bf16x3"])
def test_reorthogonalisation_keeps_canonical_form(prec):
    """After a truncating 24-qubit run the FP32 isometries are orthonormal to
    near FP32 roundoff with the FP64 re-orthogonalisation, and measurably less
    so without it."""
    _say("case: reorth canonical form", prec)
    prog, c = C.config_program(2, n=24, depth=12)

    def worst_dev(reorth):
        with P.EAState(prog.n_sites, "pure", prec, chi_max=256) as st:
            st.set_option(P.EA_OPT_REORTH, reorth)
            st.run(prog, 0.999)
            center = st.center()
            worst = 0.0
            for i in range(prog.n_sites):
                a = st.site(i).astype(np.complex128)
                cl, dd, cr = a.shape
                if i < center:
                    m = a.reshape(cl * dd, cr)
                    worst = max(worst, np.abs(m.conj().T @ m - np.eye(cr)).max())
                elif i > center:
                    m = a.reshape(cl, dd * cr)
                    worst = max(worst, np.abs(m @ m.conj().T - np.eye(cl)).max())
            return worst
    on, off = worst_dev(1), worst_dev(0)
    _say("max |X^H X - I|: reorth on", on, "off", off)
    assert on < 2e-6
    assert on < off
