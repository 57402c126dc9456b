"""Pins of the oracle MPS/MPO simulator against brute force, closed forms and
invariants (CPU only).  Each test names the passage of the paper it pins."""
import math

import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.mps import OracleMPS, truncation_rule, NAIVE, GLOBAL, NEAREST

H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
X, Y, Z = C.pauli_matrices()[1:]


# --------------------------------------------------------------- truncation

def test_truncation_rule_schmidt_pair():
    """cos(t)|00> + sin(t)|11>: s = (cos t, sin t); k = 1 iff f_t <= cos^2 t,
    and then f = cos^2 t (Eq. 10 with the kept-weight reading, Sec. VI rule)."""
    t = 0.3
    s = np.array([np.cos(t), np.sin(t)])
    c2 = np.cos(t) ** 2
    d = truncation_rule(s, c2 - 1e-9, None, 1e-13)
    assert d.k == 1 and abs(d.f - c2) < 1e-15
    d = truncation_rule(s, c2 + 1e-9, None, 1e-13)
    assert d.k == 2 and d.f == 1.0
    d = truncation_rule(s, 1.0, 1, 1e-13)
    assert d.k == 1 and d.capped and abs(d.f - c2) < 1e-15


def test_truncation_rule_brute_force_minimal():
    """k is the smallest k >= 1 whose kept weight reaches f_t (exhaustive)."""
    rng = np.random.default_rng(0)
    for trial in range(200):
        r = int(rng.integers(1, 12))
        s = np.sort(rng.random(r))[::-1]
        ft = float(rng.uniform(0.5, 1.0))
        d = truncation_rule(s, ft, None, 0.0)
        w = s ** 2 / np.sum(s ** 2)
        ok = [k for k in range(1, r + 1) if 1.0 - np.sum(w[k:]) >= ft - 1e-15]
        assert d.k == min(ok)
        assert d.f >= ft - 1e-12


def test_truncation_zero_values_dropped():
    s = np.array([1.0, 0.5, 1e-15, 0.0])
    d = truncation_rule(s, 1.0, None, 1e-13)
    assert d.k == 2 and d.k_nz == 2


# ------------------------------------------------------------- exact runs

def test_fmin1_matches_statevector_config1():
    """F_min = 1 on the 12-qubit depth-8 Haar brickwork workload: every
    amplitude equals brute force and the estimate is exactly 1 (Eq. 2, 12)."""
    prog, c = C.config_program(1)
    mps = OracleMPS(prog.n_sites, "pure", chi_max=c["chi_max"]).run(prog, 1.0)
    ref = brute.run_statevector(prog)
    np.testing.assert_allclose(mps.to_statevector(), ref, atol=1e-12)
    assert abs(mps.fidelity_estimate()[0] - 1.0) < 1e-12
    assert max(mps.bond_dims()) <= 64
    assert not mps.any_capped


def test_single_truncation_pure_fidelity():
    """Eq. (10): one truncating gate in an otherwise exact run; the true
    fidelity |<psi|psi~>|^2 equals the kept weight f."""
    n = 10
    prog = C.brickwork_program(n, 6, 123)
    ref = brute.run_statevector(prog)
    ops = list(prog.ops())
    mps = OracleMPS(n, "pure")
    target_gate = len(ops) - 3  # a late gate: large spectrum
    for j, op in enumerate(ops):
        ft = 0.97 if j == target_gate else 1.0
        mps.apply_2q(op.site, op.mat, ft)
    f = mps.log[target_gate].f
    assert f < 1.0 - 1e-4 and f >= 0.97
    # gates after the truncating one are unitary, so they keep the overlap
    got = brute.fidelity_pure(ref, mps.to_statevector())
    assert abs(got - f) < 1e-12
    assert abs(mps.fidelity_estimate()[0] - f) < 1e-13


def test_single_truncation_mixed_fidelity():
    """Eq. (11) / Eq. (9): one truncation of an MPO; (Tr rho rho~)^2 /
    (Tr rho^2 Tr rho~^2) equals the kept weight f, i.e. F_Wang = sqrt(f)."""
    n = 5
    rng = np.random.default_rng(5)
    gates = []
    mpo = OracleMPS(n, "mixed")
    sched = [(0, 0.0), (2, 1e-2), (1, 0.0), (3, 1e-2), (0, 0.0), (2, 0.0), (1, 0.0)]
    for j, (site, p) in enumerate(sched):
        u = C.haar_unitary(rng)
        s = C.unitary_superop(u)
        if p:
            s = C.depolarizing2_superop(p) @ s
        gates.append((site, 2, u, p))
        ft = 0.98 if j == len(sched) - 1 else 1.0
        mpo.apply_2q(site, s, ft)
    rho = brute.run_density(n, gates)
    f = mpo.log[-1].f
    assert f < 1.0 - 1e-6
    rho_t = mpo.to_density()
    num = abs(np.trace(rho @ rho_t)) ** 2
    den = abs(np.trace(rho @ rho)) * abs(np.trace(rho_t @ rho_t))
    assert abs(num / den - f) < 1e-12
    assert abs(brute.fidelity_wang(rho, rho_t) - math.sqrt(f)) < 1e-12


def test_mpo_exact_matches_density_with_noise():
    """F_min = 1 MPO with fused unitary + depolarising superoperators equals
    the brute-force density matrix (Eq. 3, 4); Hermitian with unit trace."""
    n = 5
    rng = np.random.default_rng(9)
    gates, mpo = [], OracleMPS(n, "mixed")
    for t in range(4):
        for i in C.brickwork_pairs(n, t):
            u = C.haar_unitary(rng)
            mpo.apply_2q(i, C.depolarizing2_superop(0.05) @ C.unitary_superop(u), 1.0)
            gates.append((i, 2, u, 0.05))
    rho = brute.run_density(n, gates)
    got = mpo.to_density()
    np.testing.assert_allclose(got, rho, atol=1e-12)
    assert np.linalg.norm(got - got.conj().T) < 1e-12
    for i in range(n):
        assert abs(mpo.expect(i, 1, Z) - brute.expect_rho(rho, n, i, 1, Z)) < 1e-12
    for i in range(n - 1):
        zz = np.kron(Z, X)
        assert abs(mpo.expect(i, 2, zz) - brute.expect_rho(rho, n, i, 2, zz)) < 1e-12


def test_mps_vs_mpo_consistency():
    """A noiseless circuit as an MPO (F_min = 1) is |psi><psi| and its bond
    spectra are the pairwise products s_a s_b of the MPS spectra."""
    n = 6
    prog = C.brickwork_program(n, 4, 77)
    mps = OracleMPS(n, "pure", keep_spectra=True)
    mpo = OracleMPS(n, "mixed", keep_spectra=True)
    for op in prog.ops():
        mps.apply_2q(op.site, op.mat, 1.0)
        mpo.apply_2q(op.site, C.unitary_superop(op.mat), 1.0)
    psi = mps.to_statevector()
    np.testing.assert_allclose(mpo.to_density(), np.outer(psi, psi.conj()), atol=1e-12)
    for ra, rb in zip(mps.log, mpo.log):
        sa = ra.s[ra.s > 1e-10]
        outer = np.sort(np.outer(sa, sa).ravel())[::-1]
        sb = rb.s[: outer.size]
        np.testing.assert_allclose(sb / sb[0], outer / outer[0], atol=1e-10)


def test_ghz_chain():
    """GHZ: chi = 2 on every bond, s = (1/sqrt2, 1/sqrt2), two amplitudes
    1/sqrt2, <Z_i Z_j> = 1, <X_i> = 0 (closed form)."""
    n = 8
    mps = OracleMPS(n, "pure", keep_spectra=True)
    mps.apply_1q(0, H)
    for i in range(n - 1):
        mps.apply_2q(i, CNOT, 1.0)
    assert mps.bond_dims() == [2] * (n - 1)
    for r in mps.log:
        np.testing.assert_allclose(r.s[:2], [2 ** -0.5] * 2, atol=1e-14)
    psi = mps.to_statevector()
    ref = np.zeros(2 ** n, dtype=complex)
    ref[0] = ref[-1] = 2 ** -0.5
    np.testing.assert_allclose(psi, ref, atol=1e-14)
    for i in range(n - 1):
        assert abs(mps.expect(i, 2, np.kron(Z, Z)) - 1.0) < 1e-13
    for i in range(n):
        assert abs(mps.expect(i, 1, X)) < 1e-13


def test_product_gates_keep_chi_one():
    """Tensor-product two-qubit gates and one-qubit gates keep chi = 1, f = 1."""
    n = 7
    rng = np.random.default_rng(2)
    mps = OracleMPS(n, "pure")
    for t in range(6):
        for i in C.brickwork_pairs(n, t):
            g = np.kron(C.haar_unitary(rng, 2), C.haar_unitary(rng, 2))
            mps.apply_2q(i, g, 0.9)
        mps.apply_1q(t % n, C.haar_unitary(rng, 2))
    assert mps.bond_dims() == [1] * (n - 1)
    assert all(r.f == 1.0 for r in mps.log)


def test_mirror_circuit_returns_to_product():
    """Fig. 2(a) analogue: a Haar circuit followed by its adjoint returns to
    |0..0> with chi = 1 on every bond (F_min = 1)."""
    n = 8
    prog = C.brickwork_program(n, 6, 31)
    mps = OracleMPS(n, "pure")
    ops = list(prog.ops())
    for op in ops:
        mps.apply_2q(op.site, op.mat, 1.0)
    assert max(mps.bond_dims()) > 4
    for op in reversed(ops):
        mps.apply_2q(op.site, op.mat.conj().T, 1.0)
    assert mps.bond_dims() == [1] * (n - 1)
    psi = mps.to_statevector()
    assert abs(abs(psi[0]) - 1.0) < 1e-12


def test_expectation_eq6_vs_bruteforce():
    """Eq. (6): <O> from the centre block equals the dense <psi|O|psi>."""
    n = 9
    prog = C.brickwork_program(n, 5, 8)
    mps = OracleMPS(n, "pure").run(prog, 1.0)
    psi = brute.run_statevector(prog)
    rng = np.random.default_rng(4)
    for i in [0, 3, 8]:
        o = C.haar_unitary(rng, 2)
        o = o + o.conj().T
        assert abs(mps.expect(i, 1, o) - brute.expect_pure(psi, n, i, 1, o)) < 1e-12
    for i in [0, 4, 7]:
        o = C.haar_unitary(rng, 4)
        assert abs(mps.expect(i, 2, o) - brute.expect_pure(psi, n, i, 2, o)) < 1e-12


def test_norm_and_canonical_form_invariants():
    """Unit norm, and the canonical form of Sec. III holds after every update."""
    n = 10
    prog = C.brickwork_program(n, 6, 12)
    mps = OracleMPS(n, "pure").run(prog, 0.95)
    psi = mps.to_statevector()
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    c = mps.center
    for i, a in enumerate(mps.A):
        cl, d, cr = a.shape
        if i < c:
            m = a.reshape(cl * d, cr)
            assert np.linalg.norm(m.conj().T @ m - np.eye(cr)) < 1e-12
        elif i > c:
            m = a.reshape(cl, d * cr)
            assert np.linalg.norm(m @ m.conj().T - np.eye(cl)) < 1e-12


@pytest.mark.parametrize("strategy", [NAIVE, GLOBAL])
@pytest.mark.parametrize("f_min", [0.9, 0.99])
def test_fmin_guarantee(strategy, f_min):
    """Sec. VI: without a cap, the product of truncation fidelities never
    falls below F_min (naive and global targets)."""
    prog = C.brickwork_program(12, 10, 5)
    mps = OracleMPS(12, "pure").run(prog, f_min, strategy)
    P = mps.fidelity_estimate()[0]
    assert P >= f_min * (1 - 1e-12)
    assert any(r.k < r.chi_l * 2 and r.k < r.chi_r * 2 and r.f < 1.0 for r in mps.log)
    if strategy == GLOBAL:
        assert P < 0.5 * (1 + f_min) + 0.5  # adaptive: spends the budget
    # the estimate tracks the true fidelity (Eq. 12 is an approximation: soft)
    true_f = brute.fidelity_pure(brute.run_statevector(prog), mps.to_statevector())
    assert abs(true_f - P) < 0.5 * (1 - P) + 1e-3


def test_lower_fmin_truncates_more():
    """Sec. VI: a smaller F_min gives smaller (never larger) bond dimensions."""
    prog = C.brickwork_program(12, 10, 6)
    tot = []
    for f_min in [0.999, 0.99, 0.9]:
        mps = OracleMPS(12, "pure").run(prog, f_min)
        tot.append(sum(r.k for r in mps.log))
    assert tot[0] > tot[1] > tot[2]


def test_cap_binds_and_flags():
    """End of Sec. VI: chi_max = 1 enforces truncation, flags it and the
    estimate drops below F_min."""
    prog = C.brickwork_program(6, 4, 3)
    mps = OracleMPS(6, "pure", chi_max=1).run(prog, 0.99)
    assert mps.any_capped
    assert mps.bond_dims() == [1] * 5
    assert mps.fidelity_estimate()[0] < 0.99


def test_schedules_values():
    """Eq. (14) and the adaptive targets: values at the first gate and the
    global target after a known loss."""
    m = OracleMPS(4, "pure")
    m.set_schedule(0.99, 490, NAIVE)
    assert abs(m.target() - 0.99 ** (1 / 490)) < 1e-16
    m.set_schedule(0.99, 490, GLOBAL)
    assert abs(m.target() - 0.99 ** (1 / 490)) < 1e-15
    m.lnP, m.g = math.log(0.995), 100
    assert abs(m.target() - (0.99 / 0.995) ** (1 / 390)) < 1e-15
    m.set_schedule(0.99, 490, NEAREST)
    m.lnP = math.log(0.999)
    assert abs(m.target() - 0.99 ** (101 / 490) / 0.999) < 1e-15
    m.lnP = math.log(0.995)  # ahead of the nearest milestone: no truncation
    assert m.target() == 1.0


def test_depolarizing_closed_form():
    """Pauli-form channel on |00><00|: diag(1 - 4p/5, 4p/15, 4p/15, 4p/15),
    trace preserved (input generator check)."""
    p = 1e-3
    s = C.depolarizing2_superop(p)
    rho = np.zeros((4, 4), complex)
    rho[0, 0] = 1
    # vec in the site-interleaved layout: p_i = 2 s_i + s_i'
    v = rho.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(16)
    out = (s @ v).reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
    np.testing.assert_allclose(np.diag(out).real, [1 - 4 * p / 5] + [4 * p / 15] * 3, atol=1e-16)
    assert abs(np.trace(out) - 1) < 1e-15
    rng = np.random.default_rng(0)
    u = C.haar_unitary(rng)
    r = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    r = r @ r.conj().T
    v = r.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(16)
    out = (C.unitary_superop(u) @ v).reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
    np.testing.assert_allclose(out, u @ r @ u.conj().T, atol=1e-12)


def test_haar_generator_unitary_and_seeded():
    rng = np.random.default_rng(1)
    u = C.haar_unitary(rng)
    assert np.linalg.norm(u.conj().T @ u - np.eye(4)) < 1e-14
    p1 = C.brickwork_program(12, 8, 1)
    p2 = C.brickwork_program(12, 8, 1)
    assert p1.n_2q == 44
    assert all(np.array_equal(a.mat, b.mat) for a, b in zip(p1.ops(), p2.ops()))
    assert C.config_program(2)[0].n_2q == 490
    assert C.config_program(3)[0].n_2q == 585


def test_forced_rank_replay_reproduces():
    """Replaying a run with its own kept ranks forced reproduces it exactly."""
    prog = C.brickwork_program(8, 6, 44)
    a = OracleMPS(8, "pure").run(prog, 0.95)
    b = OracleMPS(8, "pure")
    # replay in the same visiting order
    b.set_schedule(0.95, prog.n_2q)
    ks = iter([r.k for r in a.log])
    for layer in prog.layers:
        sites = [op.site for op in layer]
        lo, hi = min(sites), max(sites)
        asc = abs(b.center - lo) <= abs(b.center - hi)
        for op in sorted(layer, key=lambda o: o.site, reverse=not asc):
            b.apply_2q(op.site, op.mat, None, "right" if asc else "left", forced_k=next(ks))
    np.testing.assert_allclose(a.to_statevector(), b.to_statevector(), atol=1e-13)
