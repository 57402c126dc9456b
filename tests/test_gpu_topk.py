"""GPU parity of the partial (top-k) factorisation (EA_OPT_TOPK) through the
C ABI against the oracle's partial mode, on the same SplitMix64 start blocks:
single updates in both orientations, capped, grown to a second attempt and on
an MPO (kept rank, f, subspace size, attempts, the kept state), a capped
circuit, the fall-back on a rank-deficient block (bit-identical to the full
path), a full-size capped update, and option checks.  FP64 within 1e-10,
FP32 within the stated bounds."""
import math
import sys

import numpy as np
import pytest

import circuits as C
from oracle.mps import OracleMPS
from oracle import topk as K

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2307_16870_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _canonical(bonds, d, seed, kind):
    n = len(bonds) - 1
    o = OracleMPS(n, kind)
    o.load(C.random_mps_tensors(bonds, d, seed), n - 1)
    o.move_center(0)
    o.A[0] = o.A[0] / np.linalg.norm(o.A[0])
    return o


def _vector(sites):
    v = sites[0].reshape(sites[0].shape[1], -1)
    for a in sites[1:]:
        v = (v @ a.reshape(a.shape[0], -1)).reshape(-1, a.shape[2])
    return v.reshape(-1)


def _options(st, p, q, seed, tmin):
    st.set_option(P.EA_OPT_TOPK, 1)
    st.set_option(P.EA_OPT_TOPK_OVERSAMPLE, p)
    st.set_option(P.EA_OPT_TOPK_POWER, q)
    st.set_option(P.EA_OPT_TOPK_SEED, seed)
    st.set_option(P.EA_OPT_TOPK_MIN, tmin)


# (bonds, d, kind, site, chi_max, f_t, p, q): the update acts on (site, site+1)
CASES = {
    "capped": ([1, 2, 4, 8, 16, 32, 64, 128, 64, 32, 16, 8, 4, 2, 1], 2, "pure", 6, 16, 0.97, 8, 1),
    "target": ([1, 2, 4, 8, 16, 32, 48, 24, 48, 32, 16, 8, 4, 2, 1], 2, "pure", 6, None, 0.97, 8, 1),
    "wide": ([1, 2, 4, 8, 16, 32, 40, 24, 48, 32, 16, 8, 4, 2, 1], 2, "pure", 6, None, 0.97, 8, 0),
    "grown": ([1, 4, 16, 8, 16, 4, 1], 4, "mixed", 2, None, 0.95, 3, 0),
}


def _single(case, prec):
    """Both sides start from the same tensors with the centre already on the
    left site of the pair, so that no centre move (whose gauge conventions
    differ between the two sides) precedes the update: the start block then
    multiplies the same matrix on both sides."""
    bonds, d, kind, site, chi_max, ft, p, q = CASES[case]
    n = len(bonds) - 1
    o = _canonical(bonds, d, 17, kind)
    o.move_center(site)
    G = C.haar_unitary(np.random.default_rng(5), d * d)
    tens = [a.copy() for a in o.A]
    t = K.OracleTopK(n, kind, chi_max=chi_max, p=p, q=q, seed=77, topk_min=16,
                     keep_spectra=True)
    t.load([a.copy() for a in tens], o.center)
    rec = t.apply_2q(site, G, ft)
    with P.EAState(n, kind, prec, chi_max=chi_max or 0) as st:
        _options(st, p, q, 77, 16)
        st.load(tens, o.center)
        st.apply_2q(site, G, ft)
        g = st.gate_log()[0]
        sites = [st.site(i) for i in range(n)]
    return rec, g, _vector(sites), t.to_vector(), t


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("case", list(CASES))
def test_single_update_vs_oracle(case, prec):
    _say("case: topk single", case, prec)
    rec, g, vec, ref, t = _single(case, prec)
    assert hasattr(rec, "subspace")
    assert g["subspace"] == rec.subspace and g["attempts"] == rec.attempts
    s = rec.s
    gap = (s[rec.k - 1] - s[rec.k]) / s[0] if rec.k < len(s) else 1.0
    assert gap > 1e-3, "seed must leave a gap at the cut"
    assert g["k"] == rec.k and g["capped"] == rec.capped
    tol = 1e-10 if prec == "c128" else 2e-5
    assert abs(g["f"] - rec.f) < tol
    assert abs(g["lnP"] - t.lnP) < tol
    # the kept state (unique for distinct values at the cut), up to one phase
    ph = np.vdot(vec, ref)
    ph = ph / abs(ph)
    err = np.linalg.norm(vec * ph - ref) / np.linalg.norm(ref)
    rel_gap = (s[rec.k - 1] - s[rec.k]) / s[rec.k - 1] if rec.k < len(s) else 1.0
    assert err < (1e-9 if prec == "c128" else 1e-5 * (1 + 2 / rel_gap)), err


def _apply_pair(psi, n, i, G):
    v = psi.reshape(2 ** i, 4, 2 ** (n - i - 2))
    return np.einsum("ab,xby->xay", G, v).reshape(-1)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_capped_circuit_properties(prec):
    """12 qubits, depth 10, chi <= 8, F_min 0.95, p = 4, q = 1, updates of
    >= 8 columns partial (host-orchestrated layers).  Over a circuit the
    centre moves fix each bond's gauge by each side's own conventions, and
    the start block multiplies the rows of X, so the two sides' subspaces
    differ from the first move on: the circuit is checked by properties
    that hold for any subspace.  Gate by gate, f equals the overlap of the
    state kept with G applied to the state before (Eqs. 10-11), ln P is the
    sum of ln f, every partial update keeps at most l - p values and meets
    its target unless capped; and the estimate and true fidelity stay near
    the oracle's full-SVD run of the same circuit (soft)."""
    _say("case: topk capped circuit", prec)
    n = 12
    prog = C.brickwork_program(n, 10, 21)
    tol = 1e-10 if prec == "c128" else 2e-5
    n_part = 0
    with P.EAState(n, "pure", prec, chi_max=8) as st:
        st.set_option(P.EA_OPT_SMALL_LAYERS, 0)
        _options(st, 4, 1, 1, 8)
        st.set_schedule(0.95, prog.n_2q)
        for layer in prog.layers:
            for op in layer:
                if op.width == 1:
                    st.apply_1q(op.site, op.mat)
                    continue
                before = st.statevector()
                st.apply_2q(op.site, op.mat)
                after = st.statevector()
                g = st.gate_log()[-1]
                ref = _apply_pair(before, n, op.site, op.mat)
                fid = abs(np.vdot(ref, after)) ** 2 / (np.vdot(ref, ref).real *
                                                       np.vdot(after, after).real)
                assert abs(fid - g["f"]) < tol, (g, fid)
                if g["subspace"]:
                    n_part += 1
                    assert g["k"] <= g["subspace"] - 4
                if not g["capped"]:
                    assert g["f"] >= g["f_t"] - tol
        glog = st.gate_log()
        F, lnF = st.fidelity_estimate()
        psi = st.statevector()
    assert n_part >= 10
    assert abs(lnF - sum(math.log(g["f"]) for g in glog)) < 1e-9
    o = OracleMPS(n, "pure", chi_max=8).run(prog, 0.95)
    assert abs(F - o.fidelity_estimate()[0]) < 0.05


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_rank_deficient_block_falls_back_bit_identically(prec):
    """A gate without entangling power (I x I) leaves Theta of rank chi_m =
    24 < l = 56.  In FP64 the orthonormalisation meets a rank-deficient
    block, the full factorisation runs, and the result is bit-identical to a
    run with the partial path off.  In FP32 the rounding of Theta leaves the
    block of full numerical rank (the null directions at about 1e-7 of the
    largest), so the partial path may be accepted: then it captures the
    rank-24 range and agrees with the full path in k and f."""
    _say("case: topk fallback", prec)
    bonds = CASES["target"][0]
    o = _canonical(bonds, 2, 17, "pure")
    G = np.eye(4, dtype=complex)
    out = []
    for on in (1, 0):
        with P.EAState(len(bonds) - 1, "pure", prec) as st:
            if on:
                _options(st, 8, 1, 77, 16)
            st.load([a.copy() for a in o.A], o.center)
            st.apply_2q(6, G, 0.97)
            g = st.gate_log()[0]
            out.append((g, [st.site(i) for i in (6, 7)]))
    (g1, s1), (g0, s0) = out
    assert g1["attempts"] >= 1 and g0["attempts"] == 0 and g0["subspace"] == 0
    if prec == "c128" or g1["subspace"] == 0:
        assert g1["subspace"] == 0
        assert (g1["k"], g1["f"], g1["sweeps"]) == (g0["k"], g0["f"], g0["sweeps"])
        assert all(np.array_equal(a, b) for a, b in zip(s1, s0))
    else:
        assert g1["k"] == g0["k"] and abs(g1["f"] - g0["f"]) < 1e-5


def test_full_size_capped_update_fp32():
    """chi = 1024 around the pair, cap 1024 (Theta 2048 x 2048, the 50-qubit
    workload's capped updates), the library's default oversampling (64):
    l = 1088, one attempt.  Against the oracle's
    partial mode with LAPACK as its SVD step: kept rank, f within 1e-5 and
    the kept values within FP32 bounds; the left site is an isometry."""
    _say("case: topk full size chi=1024 c64")
    chi, f_t = 1024, 1 - 2.05e-3
    dims = [1, chi, chi, chi, 1]
    tens = C.random_mps_tensors(dims, 2, seed=2024)
    G = C.haar_unitary(np.random.default_rng(2024))
    t = K.OracleTopK(4, "pure", chi_max=chi, p=64, q=1, seed=0, topk_min=256, svd="lapack",
                     keep_spectra=True)
    t.load([a.copy() for a in tens], 1)
    rec = t.apply_2q(1, G, f_t)
    assert rec.subspace == 1088 and rec.capped
    with P.EAState(4, "pure", "c64", chi_max=chi) as st:
        st.set_option(P.EA_OPT_TOPK, 1)  # every other setting at its default
        st.load(tens, 1)
        st.apply_2q(1, G, f_t)
        g = st.gate_log()[0]
        a1, a2 = st.site(1), st.site(2)
    assert g["subspace"] == 1088 and g["attempts"] == 1
    assert g["k"] == rec.k == 1024 and g["capped"]
    assert abs(g["f"] - rec.f) < 1e-5
    k = rec.k
    sig = math.sqrt(float(np.sum(rec.s[:k] ** 2)))
    got_s = np.linalg.norm(a2.reshape(k, -1), axis=1)
    assert np.abs(got_s - rec.s[:k] / sig).max() < 1e-4 * rec.s[0] / sig
    q = a1.reshape(-1, k)
    assert np.abs(q.conj().T @ q - np.eye(k)).max() < 1e-5


def test_options_checked_and_off_by_default():
    _say("case: topk options")
    with P.EAState(4, "pure", "c64") as st:
        for opt, bad in [(P.EA_OPT_TOPK, 2), (P.EA_OPT_TOPK_OVERSAMPLE, 0),
                         (P.EA_OPT_TOPK_OVERSAMPLE, 1.5), (P.EA_OPT_TOPK_POWER, 5),
                         (P.EA_OPT_TOPK_SEED, -1), (P.EA_OPT_TOPK_MIN, 1)]:
            with pytest.raises(P.EAError):
                st.set_option(opt, bad)
        st.apply_2q(1, C.haar_unitary(np.random.default_rng(0)), 1.0)
        assert st.gate_log()[0]["subspace"] == 0 and st.gate_log()[0]["attempts"] == 0


def test_full_size_mpo_capped_update_fp32():
    """The largest partial factorisation of the workloads: an MPO update at
    chi = 1024, d = 4 (Theta 4096 x 4096, the 40-qubit noisy circuit's capped
    updates), default oversampling: l = 1088 of 4096 columns.  Against the
    oracle's partial mode (LAPACK SVD step): kept rank, f within 1e-5, the
    kept values within FP32 bounds; the left site is an isometry."""
    _say("case: topk full size MPO chi=1024 c64")
    chi, d, f_t = 1024, 4, 1 - 8.77e-4
    tens = C.random_mps_tensors([1, chi, chi, chi, 1], d, seed=4097)
    u = C.haar_unitary(np.random.default_rng(4097))
    G = C.depolarizing2_superop(1e-3) @ C.unitary_superop(u)
    t = K.OracleTopK(4, "mixed", chi_max=chi, seed=0, topk_min=256, svd="lapack",
                     keep_spectra=True)
    t.load([a.copy() for a in tens], 1)
    rec = t.apply_2q(1, G, f_t)
    assert rec.subspace == 1088 and rec.capped and rec.k == chi
    with P.EAState(4, "mixed", "c64", chi_max=chi) as st:
        st.set_option(P.EA_OPT_TOPK, 1)
        st.load(tens, 1)
        st.apply_2q(1, G, f_t)
        g = st.gate_log()[0]
        a1, a2 = st.site(1), st.site(2)
    assert g["subspace"] == 1088 and g["attempts"] == 1
    assert g["k"] == rec.k and g["capped"]
    assert abs(g["f"] - rec.f) < 1e-5
    k = rec.k
    sig = math.sqrt(float(np.sum(rec.s[:k] ** 2)))
    got_s = np.linalg.norm(a2.reshape(k, -1), axis=1)
    assert np.abs(got_s - rec.s[:k] / sig).max() < 1e-4 * rec.s[0] / sig
    q = a1.reshape(-1, k)
    assert np.abs(q.conj().T @ q - np.eye(k)).max() < 1e-5


def test_gradients_take_the_full_factorisation():
    """mps_energy_grad differentiates the full factorisation: with the
    partial one switched on (and eligible from 8 columns) the energy, the
    gradient and ln P are bit-identical to a run without it, and the option
    is still on afterwards."""
    _say("case: topk off for gradients")
    n, L = 12, 4
    angles = C.hea_angles(n, L, seed=9)
    terms = C.hea_hamiltonian(n)
    res = []
    for on in (0, 1):
        with P.EAState(n, "pure", "c64") as st:
            if on:
                _options(st, 4, 1, 0, 8)
            res.append(P.mps_energy_grad(st.h, P.hea_dops(n, L), angles, terms,
                                         f_min=0.99))
            if on:  # the option survives the call: a circuit then takes it
                st.reset()
                st.set_option(P.EA_OPT_CHI_MAX, 8)
                st.set_option(P.EA_OPT_SMALL_LAYERS, 0)
                st.run(C.brickwork_program(n, 10, 21), 0.95)
                assert any(g["subspace"] > 0 for g in st.gate_log())
    (E0, g0, l0), (E1, g1, l1) = res
    assert E0 == E1 and l0 == l1 and np.array_equal(g0, g1)
