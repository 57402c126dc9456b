"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64 bar: amplitudes, per-update f and the estimate within 1e-10, identical
kept ranks wherever the decision is protected by a gap (discarded weight
farther than 1e-12 T from the threshold on both sides of k).
"""
import math
import sys

import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.mps import OracleMPS
from tests.gpu_util import oracle_run, protected, gauge_free_pair

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2307_16870_amd")

X, Y, Z = C.pauli_matrices()[1:]
H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare_logs(glog, olog, tol=1e-10, tol_w=1e-12):
    assert len(glog) == len(olog)
    for g, o in zip(glog, olog):
        assert g["site"] == o.site
        if protected(o, o.f_t, tol_w):
            assert g["k"] == o.k, (g, o.k)
        assert abs(g["f"] - o.f) < tol
        assert abs(g["f_t"] - o.f_t) < tol


def test_config1_fp64_exact_vs_bruteforce():
    """12 qubits, depth 8, Haar brickwork, F_min = 1: all 4096 amplitudes."""
    _say("case: config1 fp64")
    prog, c = C.config_program(1)
    with P.EAState(prog.n_sites, "pure", "c128", chi_max=c["chi_max"]) as st:
        st.run(prog, 1.0)
        psi = st.statevector()
        F, lnF = st.fidelity_estimate()
        glog = st.gate_log()
        bonds = st.bond_dims()
    ref = brute.run_statevector(prog)
    np.testing.assert_allclose(psi, ref, atol=1e-10)
    assert abs(F - 1.0) < 1e-12
    o = oracle_run(prog, 1.0, chi_max=c["chi_max"])
    _compare_logs(glog, o.log)
    assert bonds == o.bond_dims()


@pytest.mark.parametrize("f_min,seed", [(0.95, 21), (0.9, 22)])
def test_truncating_run_fp64(f_min, seed):
    """Truncating runs: per-update k, f, the estimate and amplitudes."""
    _say("case: truncating fp64", f_min, seed)
    prog = C.brickwork_program(12, 12, seed)
    with P.EAState(12, "pure", "c128") as st:
        st.run(prog, f_min)
        psi = st.statevector()
        F, _ = st.fidelity_estimate()
        glog = st.gate_log()
    o = oracle_run(prog, f_min)
    _compare_logs(glog, o.log)
    assert all(g["k"] == r.k for g, r in zip(glog, o.log)), "unprotected rank flip"
    np.testing.assert_allclose(psi, o.to_statevector(), atol=1e-10)
    assert abs(F - o.fidelity_estimate()[0]) < 1e-10
    assert F >= f_min * (1 - 1e-12)


_SINGLE_CACHE = {}


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("chis", [(37, 70, 45), (100, 128, 90), (160, 150, 129), (300, 260, 333)])
def test_single_update_multiworkgroup(chis, kernel):
    """One update on loaded random tensors large enough for the multi-
    workgroup Jacobi (2*chi > 64) with a ragged tail; compares f, T, k and the
    gauge-free product A_i A_{i+1} after truncation.  kernel 0: three-kernel
    MFMA round; 1: fused round."""
    chiL, chiM, chiR = chis
    _say("case: single update", chis, "kernel", kernel)
    n = 4
    dims = [1, chiL, chiM, chiR, 1]
    # outer sites must be able to carry the bonds: give them d = 2 only in
    # shape, the update never reads them
    tens = C.random_mps_tensors(dims, 2, seed=sum(chis))
    rng = np.random.default_rng(5)
    G = C.haar_unitary(rng)
    if chis not in _SINGLE_CACHE:
        o = OracleMPS(n, "pure", keep_spectra=True)
        o.load(tens, 1)
        _SINGLE_CACHE[chis] = (o, o.apply_2q(1, G, 0.98))
    o, rec = _SINGLE_CACHE[chis]
    with P.EAState(n, "pure", "c128") as st:
        st.set_option(P.EA_OPT_JACOBI_KERNEL, kernel)
        st.load(tens, 1)
        rc, f = st.apply_2q(1, G, 0.98)
        glog = st.gate_log()
        a1, a2 = st.site(1), st.site(2)
    g = glog[0]
    assert abs(g["total"] - float(np.sum(rec.s ** 2))) < 1e-10 * g["total"]
    assert abs(f - rec.f) < 1e-10
    assert g["k"] == rec.k
    got = gauge_free_pair(a1, a2)
    ref = gauge_free_pair(o.A[1], o.A[2])
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("chis", [(160, 150, 129), (300, 260, 333)])
def test_jacobi_pair_skip_is_bit_identical(chis, prec):
    """Skipping block pairs whose columns are unchanged since they were last
    examined removes only examinations that would repeat on bit-identical
    columns: every output bit, the sweep count included, must match the run
    that examines every pair in every sweep."""
    chiL, chiM, chiR = chis
    _say("case: pair skip", chis, prec)
    tens = C.random_mps_tensors([1, chiL, chiM, chiR, 1], 2, seed=7 + sum(chis))
    G = C.haar_unitary(np.random.default_rng(6))
    out = []
    for skip in (1, 0):
        with P.EAState(4, "pure", prec) as st:
            st.set_option(P.EA_OPT_JACOBI_SKIP, skip)
            st.load(tens, 1)
            st.apply_2q(1, G, 0.98)
            out.append((st.gate_log()[0], st.site(1), st.site(2)))
    (g1, a1, b1), (g0, a0, b0) = out
    for key in ("k", "k_f", "f", "total", "sweeps", "capped"):
        assert g1[key] == g0[key], key
    assert np.array_equal(a1, a0) and np.array_equal(b1, b0)


def test_jacobi_pair_skip_circuit_bit_identical():
    """A 16-qubit depth-12 truncating circuit in mixed precision on the
    host-orchestrated path, with and without pair skipping."""
    _say("case: pair skip circuit")
    prog = C.brickwork_program(16, 12, 41)
    res = []
    for skip in (1, 0):
        with P.EAState(prog.n_sites, "pure", "c64") as st:
            st.set_option(P.EA_OPT_SMALL_LAYERS, 0)
            st.set_option(P.EA_OPT_JACOBI_SKIP, skip)
            st.run(prog, 0.97)
            res.append((st.statevector(), [(r["k"], r["sweeps"]) for r in st.gate_log()]))
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])


@pytest.mark.parametrize("block,threads,wgs", [(16, 256, 128), (32, 512, 512)])
def test_tuning_table_launch_shape_vs_oracle(block, threads, wgs):
    """A tuning-table entry sets the Jacobi launch shape (seen in the number
    of Gram launches: one per round, nb - 1 rounds per sweep) and the update
    still meets the FP64 bar against the oracle."""
    chis = (300, 260, 333)
    _say("case: tuning", block, threads, wgs)
    tens = C.random_mps_tensors([1, *chis, 1], 2, seed=sum(chis))
    G = C.haar_unitary(np.random.default_rng(5))
    if chis not in _SINGLE_CACHE:
        o = OracleMPS(4, "pure", keep_spectra=True)
        o.load(tens, 1)
        _SINGLE_CACHE[chis] = (o, o.apply_2q(1, G, 0.98))
    o, rec = _SINGLE_CACHE[chis]
    saved = P.mps_get_tuning()
    try:
        P.mps_set_tuning([{"f64": 1, "n_max": 1 << 30, "block": block, "rot_threads": threads,
                           "chunk_wgs": wgs}])
        with P.EAState(4, "pure", "c128") as st:
            st.load(tens, 1)
            st.profile(1)
            rc, f = st.apply_2q(1, G, 0.98)
            g = st.gate_log()[0]
            grams = st.profile_read(P.EA_K_JGRAM)["launches"]
            a1, a2 = st.site(1), st.site(2)
    finally:
        P.mps_set_tuning(saved)
    n = min(2 * chis[0], 2 * chis[2])
    nb = -(-n // block)
    nb += nb & 1
    assert grams == (nb - 1) * g["sweeps"]
    assert g["k"] == rec.k
    assert abs(f - rec.f) < 1e-10
    got, ref = gauge_free_pair(a1, a2), gauge_free_pair(o.A[1], o.A[2])
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("block,threads", [(20, 1024), (12, 128), (32, 256), (8, 64)])
def test_rotation_kernel_shapes_vs_oracle(block, threads):
    """Block widths below half the rotation kernel's tile (20 of 32 slots, 12
    of 16: the block-b values of J cycle over w slots, not the tile's) and
    thread counts that give each thread up to four J rows in registers (1024,
    128) or too many, where J stays in LDS (256 at 64 columns, 64 at 32), set
    through the options; every update meets the FP64 bar against the oracle."""
    chis = (300, 260, 333)
    _say("case: rotation kernel shape", block, threads)
    tens = C.random_mps_tensors([1, *chis, 1], 2, seed=sum(chis))
    G = C.haar_unitary(np.random.default_rng(5))
    if chis not in _SINGLE_CACHE:
        o = OracleMPS(4, "pure", keep_spectra=True)
        o.load(tens, 1)
        _SINGLE_CACHE[chis] = (o, o.apply_2q(1, G, 0.98))
    o, rec = _SINGLE_CACHE[chis]
    with P.EAState(4, "pure", "c128") as st:
        st.set_option(P.EA_OPT_BLOCK, block)
        st.set_option(P.EA_OPT_ROT_THREADS, threads)
        st.load(tens, 1)
        rc, f = st.apply_2q(1, G, 0.98)
        g = st.gate_log()[0]
        a1, a2 = st.site(1), st.site(2)
    assert g["k"] == rec.k
    assert abs(f - rec.f) < 1e-10
    got, ref = gauge_free_pair(a1, a2), gauge_free_pair(o.A[1], o.A[2])
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("chis", [(37, 70, 45), (160, 150, 129), (300, 260, 333)])
def test_qr_preconditioned_update_vs_oracle(chis):
    """SVD through the Householder QR (Jacobi on R^H, left vectors Q V_x):
    the FP64 bar against the oracle, with ragged panels and blocks."""
    _say("case: qr preconditioned", chis)
    tens = C.random_mps_tensors([1, *chis, 1], 2, seed=sum(chis))
    G = C.haar_unitary(np.random.default_rng(5))
    if chis not in _SINGLE_CACHE:
        o = OracleMPS(4, "pure", keep_spectra=True)
        o.load(tens, 1)
        _SINGLE_CACHE[chis] = (o, o.apply_2q(1, G, 0.98))
    o, rec = _SINGLE_CACHE[chis]
    with P.EAState(4, "pure", "c128") as st:
        st.set_option(P.EA_OPT_QR_PRECOND, 65)
        st.load(tens, 1)
        st.profile(1)
        rc, f = st.apply_2q(1, G, 0.98)
        g = st.gate_log()[0]
        qr_launches = st.profile_read(P.EA_K_QR)["launches"]
        a1, a2 = st.site(1), st.site(2)
    assert qr_launches > 0
    assert abs(g["total"] - float(np.sum(rec.s ** 2))) < 1e-10 * g["total"]
    assert g["k"] == rec.k
    assert abs(f - rec.f) < 1e-10
    got, ref = gauge_free_pair(a1, a2), gauge_free_pair(o.A[1], o.A[2])
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_qr_preconditioned_circuit(prec):
    """A 16-qubit depth-12 truncating circuit with every factorisation above
    64 columns preconditioned, against the same circuit without."""
    _say("case: qr preconditioned circuit", prec)
    prog = C.brickwork_program(16, 12, 43)
    res = []
    for qr in (0, 65):
        with P.EAState(prog.n_sites, "pure", prec) as st:
            st.set_option(P.EA_OPT_SMALL_LAYERS, 0)
            st.set_option(P.EA_OPT_QR_PRECOND, qr)
            st.run(prog, 0.97)
            res.append((st.statevector(), [r["k"] for r in st.gate_log()], st.fidelity_estimate()[0]))
    (psi0, k0, F0), (psi1, k1, F1) = res
    if prec == "c128":
        assert k0 == k1
        np.testing.assert_allclose(psi1, psi0, atol=1e-10)
        assert abs(F1 - F0) < 1e-12
    else:
        assert np.abs(psi1 - psi0).max() < 2e-4
        assert abs(F1 - F0) < 1e-5


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_qr_centre_moves_vs_oracle(prec, kind):
    """Centre moves by QR (the oracle's own move; kind 1 Householder, kind 2
    Cholesky QR2, the default): kept ranks, bond dimensions and amplitudes
    against the oracle on a 14-qubit truncating circuit."""
    _say("case: qr moves", prec, kind)
    prog = C.brickwork_program(14, 12, 11)
    o = oracle_run(prog, 0.97)
    with P.EAState(prog.n_sites, "pure", prec) as st:
        st.set_option(P.EA_OPT_SMALL_LAYERS, 0)
        st.set_option(P.EA_OPT_QR_MOVES, kind)
        st.profile(1)
        st.run(prog, 0.97)
        qr_launches = st.profile_read(P.EA_K_QR)["launches"]
        psi, glog, bonds = st.statevector(), st.gate_log(), st.bond_dims()
    assert qr_launches > 0
    tol_w = 1e-12 if prec == "c128" else 1e-6
    for g, r in zip(glog, o.log):
        if protected(r, r.f_t, tol_w):
            assert g["k"] == r.k
    assert bonds == o.bond_dims()
    np.testing.assert_allclose(psi, o.to_statevector(), atol=1e-10 if prec == "c128" else 2e-4)


def test_ghz_chain_gpu():
    _say("case: ghz")
    n = 10
    with P.EAState(n, "pure", "c128") as st:
        st.apply_1q(0, H)
        for i in range(n - 1):
            st.apply_2q(i, CNOT, 1.0)
        assert st.bond_dims() == [2] * (n - 1)
        psi = st.statevector()
        zz = st.expect([0, 3, 7], [2, 2, 2], [np.kron(Z, Z)] * 3)
        xs = st.expect([0, 5], [1, 1], [X, X])
    ref = np.zeros(2 ** n, complex)
    ref[0] = ref[-1] = 2 ** -0.5
    np.testing.assert_allclose(psi, ref, atol=1e-12)
    np.testing.assert_allclose(zz, 1.0, atol=1e-12)
    np.testing.assert_allclose(xs, 0.0, atol=1e-12)


def test_expect_pure_vs_oracle():
    _say("case: expect pure")
    prog = C.brickwork_program(10, 6, 8)
    rng = np.random.default_rng(1)
    ops1 = [C.haar_unitary(rng, 2) for _ in range(3)]
    ops1 = [o + o.conj().T for o in ops1]
    ops2 = [C.haar_unitary(rng, 4) for _ in range(3)]
    with P.EAState(10, "pure", "c128") as st:
        st.run(prog, 0.97)
        got = st.expect([0, 4, 9, 0, 5, 8], [1, 1, 1, 2, 2, 2], ops1 + ops2)
    o = oracle_run(prog, 0.97)
    ref = [o.expect(s, w, op) for s, w, op in zip([0, 4, 9, 0, 5, 8], [1, 1, 1, 2, 2, 2], ops1 + ops2)]
    np.testing.assert_allclose(got, ref, atol=1e-10)


def test_mpo_noisy_fp64_vs_bruteforce():
    """MPO with fused unitary + depolarising superoperators, F_min = 1:
    density matrix and <Z_i>, <Z_i Z_{i+1}> against brute force."""
    _say("case: mpo fp64")
    n = 5
    rng = np.random.default_rng(9)
    gates = []
    with P.EAState(n, "mixed", "c128") as st:
        for t in range(4):
            for i in C.brickwork_pairs(n, t):
                u = C.haar_unitary(rng)
                st.apply_2q(i, C.depolarizing2_superop(0.05) @ C.unitary_superop(u), 1.0)
                gates.append((i, 2, u, 0.05))
        rho_g = st.density()
        ev = st.expect(list(range(n)) + list(range(n - 1)), [1] * n + [2] * (n - 1),
                       [Z] * n + [np.kron(Z, Z)] * (n - 1))
    rho = brute.run_density(n, gates)
    np.testing.assert_allclose(rho_g, rho, atol=1e-10)
    ref = [brute.expect_rho(rho, n, i, 1, Z) for i in range(n)] + \
          [brute.expect_rho(rho, n, i, 2, np.kron(Z, Z)) for i in range(n - 1)]
    np.testing.assert_allclose(ev, ref, atol=1e-10)


def test_mpo_truncating_vs_oracle():
    _say("case: mpo truncating")
    prog = C.brickwork_program(6, 6, 33, kind="mixed", noise_p=1e-2)
    with P.EAState(6, "mixed", "c128") as st:
        st.run(prog, 0.95)
        glog = st.gate_log()
        F, _ = st.fidelity_estimate()
        ev = st.expect(list(range(6)), [1] * 6, [Z] * 6)
    o = oracle_run(prog, 0.95)
    _compare_logs(glog, o.log)
    assert abs(F - o.fidelity_estimate()[0]) < 1e-10
    ref = [o.expect(i, 1, Z) for i in range(6)]
    np.testing.assert_allclose(ev, ref, atol=1e-10)


def test_fp32_path_config1():
    """Complex FP32 storage / contraction / Jacobi: stated tolerances."""
    _say("case: fp32 config1")
    prog, c = C.config_program(1)
    with P.EAState(prog.n_sites, "pure", "c64", chi_max=c["chi_max"]) as st:
        st.run(prog, 1.0)
        psi = st.statevector()
        F, _ = st.fidelity_estimate()
    ref = brute.run_statevector(prog)
    err = np.abs(psi - ref).max()
    _say("fp32 amplitude max error", err)
    assert err < 1e-4
    assert abs(F - 1.0) < 1e-4
    assert abs(brute.fidelity_pure(ref, psi) - 1.0) < 1e-4


def test_error_paths_leave_state_unchanged():
    _say("case: error paths")
    with P.EAState(6, "pure", "c128") as st:
        st.apply_2q(0, C.haar_unitary(np.random.default_rng(0)), 1.0)
        before = st.statevector()
        with pytest.raises(P.EAError) as e:
            st.apply_layer([0, 1], np.stack([np.eye(4)] * 2))
        assert e.value.code == P.EA_EINVAL
        with pytest.raises(P.EAError) as e:
            st.apply_2q(5, np.eye(4))
        assert e.value.code == P.EA_ERANGE
        bad = np.eye(4, dtype=complex)
        bad[0, 0] = np.nan
        with pytest.raises(P.EAError):
            st.apply_2q(0, bad)
        with pytest.raises(P.EAError):
            st.apply_2q(0, np.eye(4), 1.5)
        np.testing.assert_allclose(st.statevector(), before, atol=0)


def test_cap_flags_warning():
    _say("case: cap")
    prog = C.brickwork_program(8, 6, 3)
    with P.EAState(8, "pure", "c128", chi_max=2) as st:
        st.run(prog, 0.99)
        F, _ = st.fidelity_estimate()
        assert max(st.bond_dims()) <= 2
        assert any(r["capped"] for r in st.gate_log())
    o = oracle_run(prog, 0.99, chi_max=2)
    assert abs(F - o.fidelity_estimate()[0]) < 1e-10


@pytest.mark.parametrize("small", [0, 64])
def test_empty_layer_is_a_no_op(small):
    _say("case: empty layer", small)
    prog = C.brickwork_program(8, 4, 17)
    with P.EAState(8, "pure", "c128") as st:
        st.set_option(P.EA_OPT_SMALL_LAYERS, small)
        st.run(prog, 0.99)
        psi, log, bonds = st.statevector(), st.gate_log(), st.bond_dims()
        rc, f = st.apply_layer([], [])
        assert rc == P.EA_OK and f.size == 0
        assert st.gate_log() == log and st.bond_dims() == bonds
        np.testing.assert_array_equal(st.statevector(), psi)


def test_zero_operator_is_rejected_and_state_kept():
    """An operator that annihilates the state (Theta = 0) is an error; the
    state is left as it was (the centre may have moved, which does not
    change it)."""
    _say("case: zero operator")
    prog = C.brickwork_program(8, 4, 18)
    with P.EAState(8, "pure", "c128") as st:
        st.set_option(P.EA_OPT_SMALL_LAYERS, 0)
        st.run(prog, 0.99)
        psi, n_log = st.statevector(), len(st.gate_log())
        with pytest.raises(P.EAError) as e:
            st.apply_2q(4, np.zeros((4, 4), complex))
        assert e.value.code == P.EA_EINVAL
        assert len(st.gate_log()) == n_log
        np.testing.assert_allclose(st.statevector(), psi, atol=1e-12)

