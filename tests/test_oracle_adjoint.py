"""Pins of the FP64 adjoint oracle (CPU only): central finite differences with
the kept ranks frozen, the parameter-shift rule on brute-force state vectors
(no truncation), and directional derivatives of the SVD adjoint alone."""
import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.adjoint import svd_vjp, hea_energy_and_grad, AdjointMPS
from oracle.jacobi import jacobi_svd
from oracle.mps import OracleMPS


def _terms(n, hx=0.5):
    return C.hea_hamiltonian(n, hx)


def test_svd_vjp_directional_derivative():
    """Loss = Re<W, U_k diag(s_k/||s_k||) V_k^H> + Re<X, U_k> ... gauge-free
    combination: truncated, renormalised product; checked along random
    complex directions by central differences (k < rank: kept/discarded
    coupling is exercised)."""
    rng = np.random.default_rng(0)
    m, n, k = 9, 7, 4
    A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Wt = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Wq = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))

    def f(A):
        r = jacobi_svd(A)
        U, s, Vh = r.u[:, :k], r.s[:k], r.vh[:k]
        T = (U * (s / np.linalg.norm(s))) @ Vh
        P = U @ U.conj().T  # projector, gauge free
        return float(np.real(np.vdot(Wt, T)) + np.real(np.vdot(Wq, P)))

    r = jacobi_svd(A)
    U, s, Vh = r.u, r.s, r.vh
    V = Vh.conj().T
    sig = np.linalg.norm(s[:k])
    # adjoints of (U, s, V) for this loss
    Tbar = Wt
    Ubar = np.zeros_like(U)
    Vbar = np.zeros_like(V)
    st = s[:k] / sig
    # T = U_k diag(st) V_k^H
    Ubar[:, :k] = Tbar @ V[:, :k] * st[None, :]
    Vbar[:, :k] = Tbar.conj().T @ U[:, :k] * st[None, :]
    stbar = np.real(np.einsum("ij,ij->j", U[:, :k].conj(), Tbar @ V[:, :k]))
    sbar = np.zeros(s.size)
    sbar[:k] = stbar / sig - s[:k] * np.dot(stbar, s[:k]) / sig ** 3
    # P = U_k U_k^H
    Ubar[:, :k] += (Wq + Wq.conj().T) @ U[:, :k]
    Abar = svd_vjp(U, s, Vh, Ubar, sbar, Vbar)
    for _ in range(4):
        D = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
        h = 1e-5
        fd = (f(A + h * D) - f(A - h * D)) / (2 * h)
        an = float(np.real(np.vdot(Abar, D)))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("n,L,f_min", [(6, 3, 0.999), (5, 4, 0.99)])
def test_hea_gradient_vs_central_differences(n, L, f_min):
    """Ranks frozen to the base run; h = 1e-4; |g - g_FD| <= 1e-6 max(1,|g|)."""
    angles = C.hea_angles(n, L, seed=7)
    terms = _terms(n)
    E, g, ranks, lnP = hea_energy_and_grad(angles, terms, f_min=f_min)
    assert lnP < 0  # the run truncates
    h = 1e-4
    flat = angles.reshape(-1)
    gflat = g.reshape(-1)
    rng = np.random.default_rng(3)
    idx = rng.choice(flat.size, size=min(flat.size, 16), replace=False)
    for j in idx:
        ap = flat.copy()
        ap[j] += h
        am = flat.copy()
        am[j] -= h
        Ep = hea_energy_and_grad(ap.reshape(angles.shape), terms, f_min=f_min, forced_ranks=ranks)[0]
        Em = hea_energy_and_grad(am.reshape(angles.shape), terms, f_min=f_min, forced_ranks=ranks)[0]
        fd = (Ep - Em) / (2 * h)
        assert abs(gflat[j] - fd) <= 1e-6 * max(1.0, abs(gflat[j])), (j, gflat[j], fd)


def test_hea_exact_gradient_parameter_shift():
    """Without truncation the gradient equals the parameter-shift rule
    dE/dt = (E(t + pi/2) - E(t - pi/2)) / 2 on brute-force state vectors."""
    n, L = 5, 3
    angles = C.hea_angles(n, L, seed=11)
    terms = _terms(n)

    def exact_energy(a):
        psi = brute.run_statevector(C.hea_program(a))
        return sum(c * brute.expect_pure(psi, n, s, w, op).real for s, w, op, c in terms)

    E, g, ranks, lnP = hea_energy_and_grad(angles, terms, f_min=None)
    assert abs(E - exact_energy(angles)) < 1e-12
    assert abs(lnP) < 1e-14
    flat = angles.reshape(-1)
    for j in range(flat.size):
        ap, am = flat.copy(), flat.copy()
        ap[j] += np.pi / 2
        am[j] -= np.pi / 2
        ps = (exact_energy(ap.reshape(angles.shape)) - exact_energy(am.reshape(angles.shape))) / 2
        assert abs(g.reshape(-1)[j] - ps) < 1e-10, j


def test_adjoint_forward_matches_oracle_energy():
    """The tape forward (SVD centre moves) gives the oracle's energy and
    fidelity estimate (QR centre moves) for the same gate order."""
    n, L = 7, 4
    angles = C.hea_angles(n, L, seed=2)
    terms = _terms(n)
    E, g, ranks, lnP = hea_energy_and_grad(angles, terms, f_min=0.999)
    o = OracleMPS(n, "pure")
    prog = C.hea_program(angles)
    o.set_schedule(0.999, prog.n_2q)
    for op in prog.ops():
        if op.width == 1:
            o.apply_1q(op.site, op.mat)
        else:
            o.apply_2q(op.site, op.mat)
    assert [r.k for r in o.log] == ranks
    assert abs(o.lnP - lnP) < 1e-12
    E_o = sum(c * o.expect(s, w, op).real for s, w, op, c in terms)
    assert abs(E - E_o) < 1e-12


@pytest.mark.parametrize("mistake", ["drop_projection", "wrong_F_sign", "drop_phase_term"])
def test_planted_mistakes_are_caught(mistake, monkeypatch):
    """A plausible mistake planted in the oracle's SVD adjoint makes the
    finite-difference pin fail (the pins have teeth)."""
    import oracle.adjoint as adj
    real = adj.svd_vjp

    def broken(U, s, Vh, Ubar, sbar, Vbar, eta=0.0, eta_rel=0.0):
        if mistake == "drop_projection":
            V = Vh.conj().T
            J = U.conj().T @ Ubar
            K = V.conj().T @ Vbar
            s2 = s * s
            D = s2[None, :] - s2[:, None]
            F = np.where(D != 0, 1.0 / np.where(D != 0, D, 1.0), 0.0)
            np.fill_diagonal(F, 0.0)
            P = F * (s[None, :] * (J - J.conj().T) + s[:, None] * (K - K.conj().T))
            P[np.diag_indices(s.size)] = sbar + 1j * (np.imag(np.diag(J)) - np.imag(np.diag(K))) / (2 * s)
            return U @ P @ Vh
        if mistake == "wrong_F_sign":
            return real(U, s, Vh, Ubar, sbar, Vbar, eta, eta_rel) - 2 * (
                real(U, s, Vh, Ubar, sbar, Vbar, eta, eta_rel)
                - real(U, s, Vh, np.zeros_like(Ubar), sbar, np.zeros_like(Vbar), eta, eta_rel))
        if mistake == "drop_phase_term":
            V = Vh.conj().T
            J = U.conj().T @ Ubar
            K = V.conj().T @ Vbar
            extra = U @ np.diag(1j * (np.imag(np.diag(J)) - np.imag(np.diag(K))) / (2 * s)) @ Vh
            return real(U, s, Vh, Ubar, sbar, Vbar, eta, eta_rel) - extra
        raise ValueError(mistake)

    monkeypatch.setattr(adj, "svd_vjp", broken)
    n, L = 5, 3
    angles = C.hea_angles(n, L, seed=7)
    terms = _terms(n)
    E, g, ranks, lnP = adj.hea_energy_and_grad(angles, terms, f_min=0.99)
    h = 1e-4
    flat = angles.reshape(-1)
    worst = 0.0
    for j in range(flat.size):
        ap, am = flat.copy(), flat.copy()
        ap[j] += h
        am[j] -= h
        Ep = adj.hea_energy_and_grad(ap.reshape(angles.shape), terms, f_min=0.99, forced_ranks=ranks)[0]
        Em = adj.hea_energy_and_grad(am.reshape(angles.shape), terms, f_min=0.99, forced_ranks=ranks)[0]
        worst = max(worst, abs(g.reshape(-1)[j] - (Ep - Em) / (2 * h)))
    assert worst > 1e-4, f"planted mistake {mistake} not detected (worst {worst})"


def test_svd_vjp_near_degenerate_lorentzian():
    """A spectrum with two kept singular values 1e-5 apart (D = s_1^2 - s_2^2
    = 1.2e-5 s_0^2).  Exact branch (eta = 0): the gauge-free loss's
    derivative matches central differences.  Broadened branch: the only term
    that eta changes appreciably is the near-degenerate pair's, scaled by
    D^2 / (D^2 + eta), so the bias g_eta - g_FD along one direction must
    follow eta / (D^2 + eta) between two broadenings (the next-closest pair
    has D = 0.05 s_0^2, whose change is below 1e-9 relative)."""
    rng = np.random.default_rng(4)
    m, n, k = 9, 7, 4

    def haar(n_):
        Z = rng.standard_normal((n_, n_)) + 1j * rng.standard_normal((n_, n_))
        Q, R = np.linalg.qr(Z)
        return Q * (np.diag(R) / abs(np.diag(R)))

    s_true = np.array([1.0, 0.6 + 1e-5, 0.6, 0.3, 0.2, 0.1, 0.05])
    A = (haar(m)[:, :n] * s_true) @ haar(n).conj().T
    Wt = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Wq = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))

    def f(A):
        r = jacobi_svd(A)
        U, s, Vh = r.u[:, :k], r.s[:k], r.vh[:k]
        T = (U * (s / np.linalg.norm(s))) @ Vh
        return float(np.real(np.vdot(Wt, T)) + np.real(np.vdot(Wq, U @ U.conj().T)))

    r = jacobi_svd(A)
    U, s, Vh = r.u, r.s, r.vh
    V = Vh.conj().T
    sig = np.linalg.norm(s[:k])
    st = s[:k] / sig
    Ubar = np.zeros_like(U)
    Vbar = np.zeros_like(V)
    Ubar[:, :k] = Wt @ V[:, :k] * st[None, :] + (Wq + Wq.conj().T) @ U[:, :k]
    Vbar[:, :k] = Wt.conj().T @ U[:, :k] * st[None, :]
    stbar = np.real(np.einsum("ij,ij->j", U[:, :k].conj(), Wt @ V[:, :k]))
    sbar = np.zeros(s.size)
    sbar[:k] = stbar / sig - s[:k] * np.dot(stbar, s[:k]) / sig ** 3
    D = s[1] ** 2 - s[2] ** 2
    assert 1.1e-5 < D < 1.3e-5
    etas = (1e-14, 1e-12)
    g0 = svd_vjp(U, s, Vh, Ubar, sbar, Vbar)
    ge = [svd_vjp(U, s, Vh, Ubar, sbar, Vbar, eta_rel=e) for e in etas]
    for _ in range(3):
        Dd = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
        h = 1e-7
        fd = (f(A + h * Dd) - f(A - h * Dd)) / (2 * h)
        a0 = float(np.real(np.vdot(g0, Dd)))
        assert abs(a0 - fd) < 1e-6 * max(1.0, abs(a0)), (a0, fd)
        bias = [float(np.real(np.vdot(g, Dd))) - a0 for g in ge]
        law = [e / (D * D + e) for e in etas]  # s_0 = 1
        assert abs(bias[0] / bias[1] - law[0] / law[1]) < 1e-3 * law[0] / law[1], (bias, law)
        # and the broadened value stays within that bias of the finite difference
        assert abs(a0 + bias[1] - fd) <= abs(bias[1]) + 1e-6 * max(1.0, abs(a0))


def test_svd_vjp_lorentzian_bounded_at_a_cut_inside_a_degenerate_pair():
    """Exactly equal singular values on both sides of the cut: the exact
    F = 1/D is unbounded (taken as 0 at D = 0 exactly), the broadened one is
    bounded by 1 / (2 sqrt(eta)).  With D at rounding level the broadened
    adjoint stays finite and within that bound times the numerators."""
    rng = np.random.default_rng(8)
    m, n = 6, 5
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    s_true = np.array([1.0, 0.5, 0.5 * (1 + 1e-15), 0.2, 0.1])
    A = (Q1[:, :n] * s_true) @ Q2.conj().T
    r = jacobi_svd(A)
    U, s, Vh = r.u, r.s, r.vh
    Ubar = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    Vbar = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    sbar = rng.standard_normal(n)
    eta_rel = 1e-12
    g = svd_vjp(U, s, Vh, Ubar, sbar, Vbar, eta_rel=eta_rel)
    assert np.all(np.isfinite(g))
    # every F entry is at most 1/(2 sqrt(eta)) = 5e5; numerators are O(10)
    assert np.abs(g).max() < 1e8
