"""Parity at the benchmark's full sizes.

* One two-site update at chi = 1024 (Theta 2048 x 2048, the bond cap of the
  50-qubit workload) in FP64 and in mixed precision, against the oracle whose
  SVD step here is numpy's LAPACK routine (pinned to the oracle's own Jacobi by
  the CPU tests); and one MPO update at d = 4, chi = 512.
* The whole 50-qubit depth-20 circuit in mixed precision (the launch
  configuration bench.py times), checked through properties that hold at any
  size: canonical form of every site, the fidelity estimate equal to the
  product of the logged truncation fidelities, bond dimensions within the cap.
"""
import json
import math
import os

import numpy as np
import pytest

import circuits as C
from oracle.mps import OracleMPS
from tests.gpu_util import gauge_free_pair, protected

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")


def _single(prec, d, chi, f_t, seed):
    dims = [1, chi, chi, chi, 1]
    tens = C.random_mps_tensors(dims, d, seed=seed)
    rng = np.random.default_rng(seed)
    u = C.haar_unitary(rng)
    G = u if d == 2 else C.depolarizing2_superop(1e-3) @ C.unitary_superop(u)
    kind = "pure" if d == 2 else "mixed"
    o = OracleMPS(4, kind, svd="lapack", keep_spectra=True)
    o.load(tens, 1)
    rec = o.apply_2q(1, G, f_t)
    with P.EAState(4, kind, prec) as st:
        st.load(tens, 1)
        rc, f = st.apply_2q(1, G, f_t)
        g = st.gate_log()[0]
        assert st.center() == 2
        a1, a2 = st.site(1), st.site(2)
    return rec, g, f, a1, a2, o


UNIT = {"c128": 2.0 ** -53, "c64": 2.0 ** -24}


def _check_update(prec, rec, g, f, a1, a2, o, f_t):
    """Kept rank, fidelity and total weight; the kept spectrum (well
    conditioned: |ds| <= ||E||_2); and the truncated product A_1 A_2 within a
    first-order perturbation bound.  Each column of the one-sided Jacobi
    receives about n rotations per sweep, each adding an independent rounding
    of relative size u, so the backward error is modelled as
    ||E||_2 ~ u sqrt(n sweeps) s_0.  With the gap delta = s_{k-1} - s_k at the
    cut the kept subspace turns by at most ||E|| / delta (Wedin), so the
    renormalised product moves by at most ||E|| (1 + 2 s_{k-1} / delta) / sigma
    in Frobenius norm, sigma the kept norm."""
    u = UNIT[prec]
    s = rec.s
    T = float(np.sum(s ** 2))
    nw = s.size
    E = u * np.sqrt(nw * max(g["sweeps"], 1)) * s[0]
    # Total weight: the same per-column model without credit for averaging
    # over columns.  In FP32 the rotations accumulated in J shrink unit-size
    # entries by amounts below their half-ulp, so column norms drift upward
    # by up to that much; f and k are ratios of such sums and are unaffected.
    assert abs(g["total"] - T) < 8 * u * np.sqrt(nw * max(g["sweeps"], 1)) * T
    tol_w = 1e-12 if prec == "c128" else 1e-6
    assert g["k"] == rec.k or not protected(rec, f_t, tol_w)
    assert abs(f - rec.f) < (1e-10 if prec == "c128" else 1e-5)
    if g["k"] != rec.k:
        return
    k = rec.k
    sigma = np.sqrt(np.sum(s[:k] ** 2))
    # the centre site holds diag(s_kept) V^H / sigma: its row norms are the spectrum
    got_s = np.linalg.norm(a2.reshape(k, -1), axis=1)
    ds = np.abs(got_s - s[:k] / sigma).max()
    print("kept spectrum max error (units of s_0/sigma):", ds / (s[0] / sigma), flush=True)
    assert ds <= 8 * E / sigma
    got = gauge_free_pair(a1, a2)
    ref = gauge_free_pair(o.A[1], o.A[2])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    bound = E * (1 + 2 * s[k - 1] / (s[k - 1] - s[k])) / sigma
    print(f"A_1 A_2 relative Frobenius error {err:.3e}, perturbation bound {bound:.3e}", flush=True)
    assert err < 2 * bound


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_full_size_update_chi1024(prec):
    print("case: full-size update chi=1024", prec, flush=True)
    f_t = 1 - 2.05e-3
    _check_update(prec, *_single(prec, 2, 1024, f_t, seed=2024), f_t)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_full_size_mpo_update(prec):
    print("case: full-size MPO update chi=512", prec, flush=True)
    f_t = 1 - 8.77e-4
    _check_update(prec, *_single(prec, 4, 512, f_t, seed=3030), f_t)


def test_full_size_mpo_update_chi1024_cross_precision():
    """The largest factorisation the workloads reach: one MPO update at
    chi = 1024, d = 4 (Theta 4096 x 4096).  The CPU oracle cannot take this
    SVD within a test, so the FP64 GPU path (pinned to the oracle up to
    2048 x 2048) is the reference for FP32: kept rank, f and total weight.
    Both: the new left site is an isometry, and f T equals the weight of the
    kept spectrum carried by the centre site (its row norms)."""
    print("case: full-size MPO update chi=1024 (Theta 4096 x 4096)", flush=True)
    chi, d, f_t = 1024, 4, 1 - 8.77e-4
    tens = C.random_mps_tensors([1, chi, chi, chi, 1], d, seed=4096)
    u = C.haar_unitary(np.random.default_rng(4096))
    G = C.depolarizing2_superop(1e-3) @ C.unitary_superop(u)
    out = {}
    for prec in ("c128", "c64"):
        with P.EAState(4, "mixed", prec) as st:
            st.load(tens, 1)
            rc, f = st.apply_2q(1, G, f_t)
            g = st.gate_log()[0]
            a1, a2 = st.site(1), st.site(2)
        k = g["k"]
        A = a1.reshape(-1, k).astype(np.complex128)  # measured in FP64
        iso = np.abs(A.conj().T @ A - np.eye(k)).max()
        s_kept = np.linalg.norm(a2.reshape(k, -1), axis=1)  # diag(s) V^H / sigma
        print(prec, "k", k, "f", f, "sweeps", g["sweeps"], "isometry", iso, flush=True)
        assert iso < (1e-12 if prec == "c128" else 1e-6)
        assert abs(np.sum(s_kept ** 2) - 1.0) < (1e-10 if prec == "c128" else 1e-5)
        assert f >= f_t - (1e-12 if prec == "c128" else 1e-5) or g["capped"]
        out[prec] = (k, f, g["total"])
    (k64, f64, T64), (k32, f32, T32) = out["c128"], out["c64"]
    assert abs(k32 - k64) <= max(2, k64 // 500)
    assert abs(f32 - f64) < 1e-5
    assert abs(T32 - T64) < 1e-4 * T64


def test_factorisation_above_the_size_limit_is_rejected():
    """A two-site matrix of more than 4096 columns (d = 4, chi = 1025 on both
    sides: Theta 4100 x 4100) is refused with EA_ETOOBIG before any kernel
    runs; the state, its log and its bonds are unchanged."""
    print("case: size limit (Theta 4100 x 4100)", flush=True)
    chi, d = 1025, 4
    tens = C.random_mps_tensors([1, chi, chi, chi, 1], d, seed=4100)
    G = C.unitary_superop(C.haar_unitary(np.random.default_rng(4100)))
    with P.EAState(4, "mixed", "c64") as st:
        st.load(tens, 1)
        before = [st.site(i) for i in range(4)]
        with pytest.raises(P.EAError) as e:
            st.apply_2q(1, G, 0.999)
        assert e.value.code == P.EA_ETOOBIG
        assert st.gate_log() == [] and st.bond_dims() == [chi, chi, chi]
        for i in range(4):
            np.testing.assert_array_equal(st.site(i), before[i])


def test_full_circuit_bench_config_invariants():
    """50 qubits, depth 20, F_min 0.99, chi <= 1024, mixed precision."""
    print("case: full circuit invariants", flush=True)
    prog, c = C.config_program(2)
    with P.EAState(prog.n_sites, "pure", "c64", chi_max=c["chi_max"]) as st:
        st.run(prog, c["f_min"])
        F, lnF = st.fidelity_estimate()
        glog = st.gate_log()
        bonds = st.bond_dims()
        center = st.center()
        worst = 0.0
        for i in range(prog.n_sites):
            a = st.site(i).astype(np.complex128)  # measured in FP64
            cl, d, cr = a.shape
            if i < center:
                m = a.reshape(cl * d, cr)
                worst = max(worst, np.abs(m.conj().T @ m - np.eye(cr)).max())
            elif i > center:
                m = a.reshape(cl, d * cr)
                worst = max(worst, np.abs(m @ m.conj().T - np.eye(cl)).max())
        a = st.site(center)
        nrm = np.vdot(a, a).real
    print("canonical-form max deviation:", worst, "P:", F, flush=True)
    assert len(glog) == prog.n_2q
    assert max(bonds) <= c["chi_max"]
    assert abs(lnF - sum(math.log(r["f"]) for r in glog)) < 1e-9
    assert all(r["k"] <= c["chi_max"] for r in glog)
    assert worst < 1e-4
    assert abs(nrm - 1.0) < 1e-4


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "brickwork50_depth20_oracle.json")
_OPS = {"Z": np.diag([1.0, -1.0]).astype(complex),
        "X": np.array([[0, 1], [1, 0]], dtype=complex)}
_OPS["ZZ"] = np.kron(_OPS["Z"], _OPS["Z"])
# per precision: decision margin (relative to T) under which a kept-rank
# decision counts as protected, and tolerances on f, ln P and observables
_BAR = {"c128": (1e-12, 1e-10, 1e-9, 1e-8),
        "c64": (1e-6, 5e-6, 4e-5, 4e-5),
        "bf16x3": (1e-5, 5e-6, 4e-5, 4e-5)}


@pytest.mark.parametrize("prec", ["c128", "c64", "bf16x3"])
def test_brickwork50_against_oracle_record(prec):
    """The whole 50-qubit depth-20 workload against the oracle's stored record
    (written by tests/golden/make_brickwork50_reference.py): every kept rank
    whose decision is protected by the margin, every truncation fidelity, the
    final ln P and one- and two-site observables.  Prints the per-result error
    of this precision against the FP64 oracle."""
    print("case: brickwork50 vs oracle record", prec, flush=True)
    with open(GOLD) as fh:
        ref = json.load(fh)
    tol_w, tol_f, tol_lnp, tol_obs = _BAR[prec]
    prog, c = C.config_program(2)
    assert ref["workload"]["n"] == prog.n_sites and ref["workload"]["seed"] == c["seed"]
    with P.EAState(prog.n_sites, "pure", prec, chi_max=c["chi_max"]) as st:
        st.run(prog, c["f_min"])
        glog = st.gate_log()
        F, lnF = st.fidelity_estimate()
        got_obs = st.expect([o["site"] for o in ref["observables"]],
                            [o["width"] for o in ref["observables"]],
                            [_OPS[o["name"]] for o in ref["observables"]])
    gates = ref["gates"]
    assert len(glog) == len(gates)
    n_prot = n_mismatch_unprot = 0
    df = 0.0
    for g, r in zip(glog, gates):
        assert g["site"] == r["site"]
        prot = abs(r["margin_k"]) > tol_w and abs(r["margin_km1"]) > tol_w
        if prot:
            n_prot += 1
            assert g["k"] == r["k"], (g["gate"], g["k"], r["k"])
        elif g["k"] != r["k"]:
            n_mismatch_unprot += 1
        df = max(df, abs(g["f"] - r["f"]))
    dlnp = abs(lnF - ref["lnP"])
    dobs = max(abs(complex(o["re"], o["im"]) - v) for o, v in zip(ref["observables"], got_obs))
    print(f"error table [{prec}]: protected ranks {n_prot}/{len(gates)} equal, "
          f"unprotected rank differences {n_mismatch_unprot}, max |df| {df:.2e}, "
          f"|d ln P| {dlnp:.2e}, max |d<O>| {dobs:.2e}", flush=True)
    assert df < tol_f
    assert dlnp < tol_lnp
    assert dobs < tol_obs


def test_brickwork50_forced_rank_replay_c64():
    """Gap rule of the parity protocol: the whole 50-qubit workload replayed
    in complex FP32 with the oracle record's kept ranks forced
    (mps_apply_layer_ranks), so every update truncates exactly as the oracle
    did; every f and the final ln P then agree within the FP32 bar whether or
    not a rank decision sat inside the rounding margin."""
    print("case: brickwork50 forced-rank replay c64", flush=True)
    with open(GOLD) as fh:
        ref = json.load(fh)
    prog, c = C.config_program(2)
    gates = ref["gates"]
    with P.EAState(prog.n_sites, "pure", "c64", chi_max=c["chi_max"]) as st:
        st.replay(prog, [r["k"] for r in gates], c["f_min"])
        glog = st.gate_log()
        F, lnF = st.fidelity_estimate()
    assert [g["k"] for g in glog] == [r["k"] for r in gates]
    assert [g["site"] for g in glog] == [r["site"] for r in gates]
    df = max(abs(g["f"] - r["f"]) for g, r in zip(glog, gates))
    print(f"replay c64: max |df| {df:.2e}, |d ln P| {abs(lnF - ref['lnP']):.2e}", flush=True)
    assert df < 5e-6
    assert abs(lnF - ref["lnP"]) < 4e-5
