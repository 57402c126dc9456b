"""Pins of oracle branches that the basic pins leave open: non-unitary
one-site operators away from the centre, forced kept ranks, the MPO log-scale
and the fixed-bond-dimension schedule (CPU only).  Each test names the passage
it pins; the pins are brute force or closed forms, never the oracle's own
formulas retyped."""
import math

import numpy as np

import circuits as C
from oracle import brute
from oracle.mps import OracleMPS, FIXED, GLOBAL

X, Y, Z = C.pauli_matrices()[1:]


class _NoMoveMPS(OracleMPS):
    """Planted mistake: a non-unitary one-site operator applied without first
    moving the centre to its site."""

    def apply_1q(self, i, g):
        g = np.asarray(g, dtype=np.complex128)
        self.A[i] = np.einsum("st,atb->asb", g, self.A[i])


def _pure_nonunitary_case(cls):
    """Exact 10-qubit state, a non-unitary filter on site 0 while the centre
    sits far right, then one truncating gate on (4, 5): returns the true
    fidelity (brute force) and the truncation fidelity the update records."""
    n = 10
    prog = C.brickwork_program(n, 6, 71)
    mps = cls(n, "pure")
    for layer in prog.layers:
        mps.apply_layer(layer)
    mps.move_center(8)
    rng = np.random.default_rng(3)
    filt = np.diag([1.0, 0.35]).astype(complex) @ C.haar_unitary(rng, 2)
    mps.apply_1q(0, filt)
    u = C.haar_unitary(rng, 4)
    rec = mps.apply_2q(4, u, 0.97)
    psi = brute.run_statevector(prog)
    psi = brute.apply_1q(psi, n, 0, filt)
    psi = brute.apply_2q(psi, n, 4, u)
    return brute.fidelity_pure(psi, mps.to_statevector()), rec.f


def test_nonunitary_1q_offcentre_keeps_eq10_exact():
    """Sec. II one-site operators with the canonical form of Sec. III: a
    non-unitary operator on a site the centre is far from, then one
    truncation elsewhere; the true fidelity equals the recorded f (Eq. 10)
    only if the centre was moved to the operator's site first."""
    true_f, f = _pure_nonunitary_case(OracleMPS)
    assert f < 1.0 - 1e-3
    assert abs(true_f - f) < 1e-12


def test_nonunitary_1q_pin_catches_a_skipped_move():
    true_f, f = _pure_nonunitary_case(_NoMoveMPS)
    assert abs(true_f - f) > 1e-4


def _mixed_nonunitary_case(cls):
    """6-qubit MPO with noisy two-site superoperators, a one-qubit
    depolarising superoperator on site 0 while the centre is at site 4, then
    one truncation on (3, 4)."""
    n = 6
    rng = np.random.default_rng(19)
    mpo = cls(n, "mixed")
    gates = []
    for t in range(4):
        for i in C.brickwork_pairs(n, t):
            u = C.haar_unitary(rng)
            mpo.apply_2q(i, C.depolarizing2_superop(0.02) @ C.unitary_superop(u), 1.0)
            gates.append((i, 2, u, 0.02))
    mpo.move_center(4)
    u1 = C.haar_unitary(rng, 2)
    mpo.apply_1q(0, C.depolarizing1_superop(0.1) @ C.unitary_superop(u1))
    gates.append((0, 1, u1, 0.1))
    u = C.haar_unitary(rng)
    rec = mpo.apply_2q(3, C.depolarizing2_superop(0.02) @ C.unitary_superop(u), 0.99)
    gates.append((3, 2, u, 0.02))
    rho = brute.run_density(n, gates)
    rho_t = mpo.to_density()
    num = abs(np.trace(rho @ rho_t)) ** 2
    den = abs(np.trace(rho @ rho)) * abs(np.trace(rho_t @ rho_t))
    return num / den, rec.f


def test_nonunitary_superop_offcentre_keeps_eq11_exact():
    """Eq. (11) with Eq. (9): after a one-qubit depolarising superoperator
    away from the centre, one MPO truncation has (Tr rho rho~)^2 /
    (Tr rho^2 Tr rho~^2) equal to the recorded f."""
    w, f = _mixed_nonunitary_case(OracleMPS)
    assert f < 1.0 - 1e-5
    assert abs(w - f) < 1e-12


def test_nonunitary_superop_pin_catches_a_skipped_move():
    w, f = _mixed_nonunitary_case(_NoMoveMPS)
    assert abs(w - f) > 1e-6


def test_noisy_program_with_one_qubit_channels_vs_density():
    """Sec. VI, Fig. 2(b) workload structure: one- and two-qubit depolarising
    noise fused after every gate.  With F_min = 1 the MPO equals the dense
    density matrix, whose channels are applied in Pauli-sum form (pins the
    4x4 superoperator layout and the non-unitary branch in a chain)."""
    prog = C.noisy_program(5, 6, 8, eps1=0.05, eps2=0.05)
    mpo = OracleMPS(5, "mixed").run(prog, 1.0)
    rho = brute.run_density(5, prog.units)
    np.testing.assert_allclose(mpo.to_density(), rho, atol=1e-12)
    assert abs(mpo.fidelity_estimate()[0] - 1.0) < 1e-12


def test_depolarizing1_closed_form():
    """(1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z) shrinks the Bloch vector
    by 1 - 4p/3 and preserves the trace."""
    p = 0.05
    s = C.depolarizing1_superop(p)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(3)
    r = 0.9 * r / np.linalg.norm(r)
    rho = 0.5 * (np.eye(2) + r[0] * X + r[1] * Y + r[2] * Z)
    out = (s @ rho.reshape(4)).reshape(2, 2)  # vec index 2 s + s'
    bloch = [np.trace(out @ P).real for P in (X, Y, Z)]
    np.testing.assert_allclose(bloch, (1 - 4 * p / 3) * r, atol=1e-15)
    assert abs(np.trace(out) - 1) < 1e-15


def test_forced_rank_bookkeeping_vs_bruteforce():
    """Forced kept ranks (replay / fixed-rank runs): one truncation forced
    below and one above the rule's choice; the true fidelity equals the
    recorded f, and exp(ln P) equals f (Eq. 10 for the kept rank, Eq. 12
    with one factor)."""
    n = 10
    prog = C.brickwork_program(n, 7, 90)
    psi_ref = brute.run_statevector(prog)
    ops = list(prog.ops())
    target = len(ops) - 4
    probe = OracleMPS(n, "pure", keep_spectra=True)
    for j, op in enumerate(ops):
        probe.apply_2q(op.site, op.mat, 0.95 if j == target else 1.0)
    k_rule = probe.log[target].k
    assert k_rule >= 4
    for k_forced in (k_rule - 3, k_rule + 2):
        mps = OracleMPS(n, "pure")
        for j, op in enumerate(ops):
            if j == target:
                rec = mps.apply_2q(op.site, op.mat, 0.95, forced_k=k_forced)
            else:
                mps.apply_2q(op.site, op.mat, 1.0)
        assert rec.k == k_forced and not rec.capped
        true_f = brute.fidelity_pure(psi_ref, mps.to_statevector())
        assert abs(true_f - rec.f) < 1e-12
        assert abs(math.exp(mps.lnP) - rec.f) < 1e-13
        if k_forced < k_rule:
            assert rec.f < 0.95  # below the target: the rule would keep more
        else:
            assert rec.f > probe.log[target].f


def _vec_rho(rho, n):
    """vec(rho) over (p_1 .. p_N), p = 2 sigma + sigma'."""
    perm = [q for i in range(n) for q in (i, n + i)]
    return rho.reshape([2] * (2 * n)).transpose(perm).reshape(-1)


def test_lnS_scale_exact_mpo():
    """Renormalisation reading (kept values to unit norm, removed scale in
    lnS): without truncation, exp(lnS) times the stored MPO is the exact
    density matrix, trace 1, under trace-preserving but purity-reducing
    noise."""
    n = 5
    prog = C.noisy_program(n, 5, 4, eps1=0.05, eps2=0.1)
    mpo = OracleMPS(n, "mixed").run(prog, 1.0)
    rho = brute.run_density(n, prog.units)
    assert mpo.lnS < -0.1  # the noise removed Hilbert-Schmidt norm
    np.testing.assert_allclose(math.exp(mpo.lnS) * mpo.to_vector(), _vec_rho(rho, n), atol=1e-12)
    assert abs(mpo.log[-1].lnS - mpo.lnS) < 1e-15


def test_lnS_scale_single_truncation_is_the_projection():
    """One MPO truncation (the last gate, on (2, 3)): exp(lnS) times the stored
    state equals the exact vec(rho) projected onto its k largest Schmidt
    components across that bond (dense SVD of the reshaped exact vector)."""
    n = 6
    prog = C.noisy_program(n, 5, 12, eps1=0.02, eps2=0.05)
    mpo = OracleMPS(n, "mixed")
    mpo.set_schedule(1.0, prog.n_2q)
    for layer in prog.layers:
        for op in layer:
            if op.width == 1:
                mpo.apply_1q(op.site, op.mat)
        mpo.apply_layer([op for op in layer if op.width == 2])
    rng = np.random.default_rng(5)
    u = C.haar_unitary(rng)
    rec = mpo.apply_2q(2, C.depolarizing2_superop(0.05) @ C.unitary_superop(u), 0.995)
    units = list(prog.units) + [(2, 2, u, 0.05)]
    assert rec.k < min(rec.chi_l, rec.chi_r) * 4 and rec.f < 1.0
    v = _vec_rho(brute.run_density(n, units), n).reshape(4 ** 3, 4 ** 3)
    uu, s, vh = np.linalg.svd(v)
    k = rec.k
    proj = (uu[:, :k] * s[:k]) @ vh[:k]
    np.testing.assert_allclose(math.exp(mpo.lnS) * mpo.to_vector(), proj.reshape(-1),
                               atol=1e-11)
    w = np.sum(s[:k] ** 2) / np.sum(s ** 2)
    assert abs(w - rec.f) < 1e-12


def test_fixed_strategy_is_the_standard_capped_simulation():
    """Sec. VI, Fig. 4 comparison: the fixed schedule targets f_t = 1, so each
    update keeps min(chi_max, number of non-zero values); without a cap the
    run is exact (all amplitudes, P = 1)."""
    prog = C.brickwork_program(10, 8, 55)
    exact = OracleMPS(10, "pure").run(prog, 0.9, FIXED)
    np.testing.assert_allclose(exact.to_statevector(), brute.run_statevector(prog), atol=1e-12)
    assert exact.fidelity_estimate()[0] == 1.0
    assert all(r.f_t == 1.0 for r in exact.log)
    capped = OracleMPS(10, "pure", chi_max=6, keep_spectra=True).run(prog, 0.9, FIXED)
    for r in capped.log:
        nz = int(np.count_nonzero(r.s > 1e-13 * r.s[0]))
        assert r.k == min(6, nz)
        assert r.capped == (nz > 6)
    assert max(capped.bond_dims()) == 6
    ea = OracleMPS(10, "pure").run(prog, 0.9, GLOBAL)
    assert sum(r.k for r in ea.log) < sum(r.k for r in exact.log)
