"""Reverse-mode gradient of an energy through the EA-MPS simulation (FP64).

Test infrastructure only (see the package header).

The loss is E = sum_t c_t Re <O_t> evaluated on the final state of a circuit
of one-qubit rotations and two-qubit gates run by the entanglement-aware MPS
algorithm (Sec. V-VI), with every kept rank frozen to the value the forward
pass chose.  With the ranks frozen the simulation is a smooth map, and its
gradient is obtained by applying, in reverse order, the vector-Jacobian
product of every step:

* one-site gate A' = g A;
* two-site contraction Theta = G (A B) (Sec. V);
* SVD Theta = U S V^H with the first k triplets kept, renormalised
  s~ = s_k / ||s_k|| and written back (Sec. V-VI);
* centre moves, done here by an SVD M = U (S V^H) with the non-isometric
  factor absorbed into the neighbour (exact re-gauging, Sec. III);
* <O> at the orthogonality centre (Eq. 6).

Adjoint convention: for a real loss L and complex X, Xbar is defined by
dL = Re sum(conj(Xbar) * dX).

SVD adjoint (derived from d(U^H A V) = dOmega_U S + dS - S dOmega_V with
dOmega skew-Hermitian): with J = U^H Ubar, K = V^H Vbar (r x r, r = number of
numerically non-zero singular values), F_ij = 1 / (s_j^2 - s_i^2) (i != j),
  P_ij = F_ij (s_j (J - J^H)_ij + s_i (K - K^H)_ij),
  P_ii = sbar_i + i (Im J_ii - Im K_ii) / (2 s_i),
  Abar = U P V^H + (I - U U^H) Ubar S^-1 V^H + U S^-1 Vbar^H (I - V V^H).
Kept-discarded couplings enter through F_ij with one kept and one discarded
index; the full spectrum comes from the Jacobi SVD.  A broadening eta > 0
replaces F by the Lorentzian (s_j^2 - s_i^2) / ((s_j^2 - s_i^2)^2 + eta), with
eta = eta_abs + eta_rel s_0^4 (s_0 the largest singular value of the factored
matrix), so that a relative broadening means the same for every update.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .jacobi import jacobi_svd
from .mps import truncation_rule


def svd_vjp(U, s, Vh, Ubar, sbar, Vbar, eta: float = 0.0, eta_rel: float = 0.0):
    """Adjoint of A for A = U diag(s) Vh (all r columns non-zero).

    U: (m, r), s: (r,), Vh: (r, n); Ubar: (m, r), sbar: (r,), Vbar: (n, r).
    eta (absolute) and eta_rel (relative to s_0^4) broaden F; both 0: exact.
    """
    eta = eta + eta_rel * float(np.max(s)) ** 4
    V = Vh.conj().T
    r = s.size
    J = U.conj().T @ Ubar
    K = V.conj().T @ Vbar
    s2 = s * s
    D = s2[None, :] - s2[:, None]  # D_ij = s_j^2 - s_i^2
    with np.errstate(divide="ignore", invalid="ignore"):
        F = D / (D * D + eta) if eta > 0 else np.where(D != 0, 1.0 / np.where(D != 0, D, 1.0), 0.0)
    np.fill_diagonal(F, 0.0)
    Js = J - J.conj().T
    Ks = K - K.conj().T
    P = F * (s[None, :] * Js + s[:, None] * Ks)
    P[np.diag_indices(r)] = sbar + 1j * (np.imag(np.diag(J)) - np.imag(np.diag(K))) / (2.0 * s)
    Abar = U @ P @ Vh
    m, n = U.shape[0], Vh.shape[1]
    UbS = Ubar / s[None, :]
    Abar = Abar + (UbS - U @ (U.conj().T @ UbS)) @ Vh
    VbS = Vbar / s[None, :]
    Abar = Abar + U @ (VbS - V @ (V.conj().T @ VbS)).conj().T
    return Abar


def _svd_r(M, tau):
    """Jacobi SVD restricted to the numerically non-zero singular values."""
    res = jacobi_svd(M)
    s = res.s
    r = max(1, int(np.count_nonzero(s > tau * s[0])))
    return res.u[:, :r], s[:r].copy(), res.vh[:r, :], res.s


class AdjointMPS:
    """Pure-state EA-MPS with a tape, for E and dE/d(angles)."""

    def __init__(self, n_sites, chi_max=None, tau=1e-13, eta=0.0, eta_rel=0.0):
        self.n = n_sites
        self.chi_max = chi_max
        self.tau = tau
        self.eta = eta
        self.eta_rel = eta_rel
        self.A: List[np.ndarray] = []
        for _ in range(n_sites):
            a = np.zeros((1, 2, 1), dtype=np.complex128)
            a[0, 0, 0] = 1.0
            self.A.append(a)
        self.center = 0
        self.lnP = 0.0
        self.g = 0
        self.tape = []
        self.ranks: List[int] = []
        self.f_min = None
        self.n_total = None

    # ------------------------------------------------------------ forward
    def _move_right(self):
        c = self.center
        a, b = self.A[c], self.A[c + 1]
        cl, d, cr = a.shape
        U, s, Vh, _ = _svd_r(a.reshape(cl * d, cr), self.tau)
        self.tape.append(("mr", c, a, b, U, s, Vh))
        self.A[c] = U.reshape(cl, d, s.size)
        self.A[c + 1] = np.einsum("ij,jsk->isk", s[:, None] * Vh, b)
        self.center = c + 1

    def _move_left(self):
        c = self.center
        a, b = self.A[c], self.A[c - 1]
        cl, d, cr = a.shape
        U, s, Vh, _ = _svd_r(a.reshape(cl, d * cr), self.tau)
        self.tape.append(("ml", c, a, b, U, s, Vh))
        self.A[c] = Vh.reshape(s.size, d, cr)
        self.A[c - 1] = np.einsum("isj,jk->isk", b, U * s[None, :])
        self.center = c - 1

    def move_center(self, j):
        while self.center < j:
            self._move_right()
        while self.center > j:
            self._move_left()

    def target(self):
        """Global target of Sec. VI (1 without a schedule)."""
        if self.f_min is None:
            return 1.0
        left = self.n_total - self.g
        return 1.0 if left <= 0 else min(1.0, math.exp((math.log(self.f_min) - self.lnP) / left))

    def apply_1q(self, i, g, angle_index=None, kind=None):
        """Unitary one-site gate; (angle_index, kind) tags an RY/RZ angle."""
        a = self.A[i]
        self.tape.append(("1q", i, a, g, angle_index, kind))
        self.A[i] = np.einsum("st,atb->asb", g, a)

    def apply_2q(self, i, G, forced_k=None):
        """Two-site update (Sec. V-VI); the centre ends on i+1."""
        if not (self.center == i or self.center == i + 1):
            self.move_center(i if self.center < i else i + 1)
        f_t = self.target()
        a, b = self.A[i], self.A[i + 1]
        chi_l, chi_r = a.shape[0], b.shape[2]
        C = np.einsum("ljm,mkr->ljkr", a, b)
        th = np.einsum("stuv,luvr->lstr", G.reshape(2, 2, 2, 2), C).reshape(chi_l * 2, 2 * chi_r)
        U, s, Vh, s_all = _svd_r(th, self.tau)
        dec = truncation_rule(s_all, f_t, self.chi_max, self.tau)
        k = dec.k if forced_k is None else forced_k
        self.ranks.append(k)
        sig = math.sqrt(float(np.sum((s[:k] ** 2)[::-1])))
        disc = float(np.sum((s_all[k:] ** 2)[::-1]))
        self.lnP += math.log1p(-disc / dec.total)
        self.g += 1
        self.tape.append(("2q", i, a, b, G, U, s, Vh, k, sig))
        self.A[i] = U[:, :k].reshape(chi_l, 2, k)
        self.A[i + 1] = ((s[:k] / sig)[:, None] * Vh[:k]).reshape(k, 2, chi_r)
        self.center = i + 1

    def expect_term(self, site, width, op, coef):
        """coef * Re <O> at the orthogonality centre (Eq. 6)."""
        self.move_center(site)
        a = self.A[site]
        if width == 1:
            th = a
            oth = np.einsum("st,ltr->lsr", op, th)
            b = None
        else:
            b = self.A[site + 1]
            th = np.einsum("ljm,mkr->ljkr", a, b)
            oth = np.einsum("stuv,luvr->lstr", op.reshape(2, 2, 2, 2), th)
        nrm = np.vdot(th, th).real
        val = np.vdot(th, oth) / nrm
        self.tape.append(("ex", site, width, op, coef, th, val, nrm, a, b))
        return coef * val.real

    # ----------------------------------------------------------- backward
    def backward(self, n_angles):
        """Reverse pass over the tape; returns dE/d(angles) (flat)."""
        Ab = [np.zeros_like(a) for a in self.A]
        grad = np.zeros(n_angles)
        for rec in reversed(self.tape):
            _reverse_record(rec, Ab, grad, self.eta, self.eta_rel)
        return grad


def _dgate(kind, g):
    """d g / d angle for RY(t) = exp(-i t Y/2) and RZ(t) = exp(-i t Z/2)."""
    if kind == "ry":
        y = np.array([[0, -1j], [1j, 0]])
        return -0.5j * (y @ g)
    if kind == "rz":
        z = np.diag([1.0, -1.0]).astype(complex)
        return -0.5j * (z @ g)
    raise ValueError(kind)


def _reverse_record(rec, Ab, grad, eta, eta_rel):
    """Vector-Jacobian product of one recorded step, in place on the site
    adjoints ``Ab`` (and ``grad`` for tagged angles)."""
    kind = rec[0]
    if kind == "ex":
        _, site, width, op, coef, th, val, nrm, a, b = rec
        oh = op + op.conj().T
        if width == 1:
            thb = coef * (np.einsum("st,ltr->lsr", oh, th) - 2.0 * val.real * th) / nrm
            Ab[site] = Ab[site] + thb
        else:
            thb = coef * (np.einsum("stuv,luvr->lstr", oh.reshape(2, 2, 2, 2), th)
                          - 2.0 * val.real * th) / nrm
            Ab[site] = Ab[site] + np.einsum("ljkr,mkr->ljm", thb, b.conj())
            Ab[site + 1] = Ab[site + 1] + np.einsum("ljm,ljkr->mkr", a.conj(), thb)
    elif kind == "1q":
        _, i, a, g, idx, gk = rec
        abar_out = Ab[i]
        Ab[i] = np.einsum("ts,atb->asb", g.conj(), abar_out)  # g^H applied
        if idx is not None:
            gbar = np.einsum("asb,atb->st", abar_out, a.conj())
            grad[idx] += float(np.real(np.sum(gbar.conj() * _dgate(gk, g))))
    elif kind == "2q":
        _, i, a, b, G, U, s, Vh, k, sig = rec
        chi_l, chi_r = a.shape[0], b.shape[2]
        r = s.size
        V = Vh.conj().T
        abar = Ab[i].reshape(chi_l * 2, k)
        bbar = Ab[i + 1].reshape(k, 2 * chi_r)
        st = s[:k] / sig
        Ubar = np.zeros((U.shape[0], r), complex)
        Vbar = np.zeros((V.shape[0], r), complex)
        Ubar[:, :k] = abar                                  # A_i' = U_k
        stbar = np.real(np.einsum("jc,cj->j", bbar, V[:, :k]))  # A_{i+1}' = s~ V_k^H
        Vbar[:, :k] = st[None, :] * bbar.T.conj()
        sbar = np.zeros(r)                                  # s~ = s_k / ||s_k||
        sbar[:k] = stbar / sig - s[:k] * np.dot(stbar, s[:k]) / sig ** 3
        thbar = svd_vjp(U, s, Vh, Ubar, sbar, Vbar, eta, eta_rel)
        # Theta = G (A B):  Cbar = G^H Thetabar, Abar = Cbar B^H, Bbar = A^H Cbar
        Cb = np.einsum("stuv,lstr->luvr", G.reshape(2, 2, 2, 2).conj(),
                       thbar.reshape(chi_l, 2, 2, chi_r))
        Ab[i] = np.einsum("ljkr,mkr->ljm", Cb, b.conj())
        Ab[i + 1] = np.einsum("ljm,ljkr->mkr", a.conj(), Cb)
    elif kind == "mr":
        _, c, a, b, U, s, Vh = rec
        cl, d, cr = a.shape
        r = s.size
        X = s[:, None] * Vh
        bbar_out = Ab[c + 1].reshape(r, -1)
        Xbar = bbar_out @ b.reshape(cr, -1).conj().T         # A_{c+1}' = X A_{c+1}
        Ab[c + 1] = (X.conj().T @ bbar_out).reshape(b.shape)
        V = Vh.conj().T
        sbar = np.real(np.einsum("jc,cj->j", Xbar, V))       # X = S V^H
        Vbar = s[None, :] * Xbar.T.conj()
        Ab[c] = svd_vjp(U, s, Vh, Ab[c].reshape(cl * d, r), sbar, Vbar, eta, eta_rel).reshape(a.shape)
    elif kind == "ml":
        _, c, a, b, U, s, Vh = rec
        cl, d, cr = a.shape
        r = s.size
        Y = U * s[None, :]
        pbar_out = Ab[c - 1].reshape(-1, r)
        Ybar = b.reshape(-1, cl).conj().T @ pbar_out          # A_{c-1}' = A_{c-1} Y
        Ab[c - 1] = (pbar_out @ Y.conj().T).reshape(b.shape)
        Ubar = Ybar * s[None, :]                              # Y = U S
        sbar = np.real(np.einsum("rj,rj->j", U.conj(), Ybar))
        Vbar = Ab[c].reshape(r, d * cr).T.conj()               # A_c' = V^H
        Ab[c] = svd_vjp(U, s, Vh, Ubar, sbar, Vbar, eta, eta_rel).reshape(a.shape)
    else:
        raise ValueError(kind)


def hea_energy_and_grad(angles, terms, f_min=None, chi_max=None, forced_ranks=None, eta=0.0,
                        tau=1e-13, eta_rel=0.0):
    """E = sum_t c_t Re <O_t> after the hardware-efficient ansatz (per layer:
    RY then RZ on every qubit, then CZ on brickwork pairs) run by EA-MPS with
    the global schedule for F_min, and dE/d(angles).

    Returns (E, grad shaped like angles, kept ranks, ln of the estimate).
    """
    from circuits import ry, rz, CZ, brickwork_pairs
    L, n, _ = angles.shape
    sim = AdjointMPS(n, chi_max=chi_max, tau=tau, eta=eta, eta_rel=eta_rel)
    if f_min is not None:
        sim.f_min = f_min
        sim.n_total = sum(len(brickwork_pairs(n, l)) for l in range(L))
    ranks = iter(forced_ranks) if forced_ranks is not None else None
    for l in range(L):
        for q in range(n):
            sim.apply_1q(q, ry(angles[l, q, 0]), (l * n + q) * 2, "ry")
            sim.apply_1q(q, rz(angles[l, q, 1]), (l * n + q) * 2 + 1, "rz")
        for i in brickwork_pairs(n, l):
            sim.apply_2q(i, CZ, None if ranks is None else next(ranks))
    E = 0.0
    for site, width, op, coef in terms:
        E += sim.expect_term(site, width, op, coef)
    grad = sim.backward(angles.size).reshape(angles.shape)
    return E, grad, list(sim.ranks), sim.lnP
