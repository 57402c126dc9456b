"""One-sided (Hestenes) Jacobi SVD, complex128, written out.

Test infrastructure only (see the package header).

The paper needs M = U Lambda V^dagger with Lambda sorted in decreasing order
(Sec. III; Sec. V takes the SVD of the contracted two-site tensor).  The
method used here is Hestenes' one-sided Jacobi: columns of W = M are rotated
pairwise until mutually orthogonal; then s_j = ||w_j||, u_j = w_j / s_j and
V is the product of the rotations.

For each column pair (p, q) with alpha = ||w_p||^2, beta = ||w_q||^2 and
gamma = w_p^H w_q: if |gamma| > tol * sqrt(alpha * beta) the pair is rotated
by  [w_p, w_q] <- [w_p, w_q] diag(1, e^{-i phi}) [[c, s], [-s, c]],
phi = arg(gamma), where (c, s) is the symmetric 2x2 Schur rotation of the real
matrix [[alpha, |gamma|], [|gamma|, beta]] (Golub & Van Loan's sym.schur2):
zeta = (beta - alpha) / (2 |gamma|), t = sign(zeta) / (|zeta| + sqrt(1 +
zeta^2)), c = 1 / sqrt(1 + t^2), s = c t.  The same rotation is applied to
the columns of V.  A sweep visits every pair once; iteration stops after a
sweep that rotates nothing (tol = m * 2^-53 by default).

Two visiting orders are provided, both the same algorithm:
``cyclic``  -- the row-cyclic order (p = 0..n-2, q = p+1..n-1), one pair at a
               time; the textbook statement.
``rr``      -- the round-robin ("circle method") order, in which the n/2
               disjoint pairs of a round are rotated together (vectorised over
               pairs with NumPy); needed for the larger matrices.
``lapack``  -- not Jacobi: ``numpy.linalg.svd`` called as a library step, for
               sizes at which the Python loops take minutes.  Pinned against
               the Jacobi orders by the tests.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

EPS64 = 2.0 ** -53


@dataclass
class JacobiResult:
    u: np.ndarray      # (m, r) left singular vectors, r = min(m, n)
    s: np.ndarray      # (r,) singular values, decreasing
    vh: np.ndarray     # (r, n)
    sweeps: int
    converged: bool


def _rotation(alpha, beta, gamma, tol):
    """Return (do, c, s, e) for one pair; e = e^{-i arg gamma}."""
    g = abs(gamma)
    if not (g > tol * np.sqrt(alpha * beta)) or g == 0.0:
        return False, 1.0, 0.0, 1.0
    zeta = (beta - alpha) / (2.0 * g)
    t = (1.0 if zeta >= 0 else -1.0) / (abs(zeta) + np.hypot(1.0, zeta))
    c = 1.0 / np.sqrt(1.0 + t * t)
    return True, c, c * t, np.conj(gamma) / g


def _sweeps_cyclic(w, v, tol, max_sweeps):
    n = w.shape[1]
    for sweep in range(1, max_sweeps + 1):
        rotated = 0
        for p in range(n - 1):
            for q in range(p + 1, n):
                wp, wq = w[:, p], w[:, q]
                alpha = np.vdot(wp, wp).real
                beta = np.vdot(wq, wq).real
                gamma = np.vdot(wp, wq)
                do, c, s, e = _rotation(alpha, beta, gamma, tol)
                if not do:
                    continue
                rotated += 1
                wq_e = e * wq
                w[:, p], w[:, q] = c * wp - s * wq_e, s * wp + c * wq_e
                vp, vq_e = v[:, p].copy(), e * v[:, q]
                v[:, p], v[:, q] = c * vp - s * vq_e, s * vp + c * vq_e
        if rotated == 0:
            return sweep, True
    return max_sweeps, False


def round_robin_pairs(n_even: int, rnd: int):
    """Pairs of round ``rnd`` of the circle method over ``n_even`` players.

    Player 0 stays in slot 0; the others rotate by one slot per round; slot i
    plays slot n_even-1-i.  Over n_even-1 rounds every pair meets once.
    """
    def player(slot):
        if slot == 0:
            return 0
        return (slot - 1 + rnd) % (n_even - 1) + 1
    return [(player(i), player(n_even - 1 - i)) for i in range(n_even // 2)]


def _sweeps_rr(w, v, tol, max_sweeps):
    n = w.shape[1]
    n_even = n + (n % 2)
    rounds = []
    for r in range(n_even - 1):
        pr = [(a, b) for a, b in round_robin_pairs(n_even, r) if a < n and b < n]
        if pr:
            a = np.array([min(x) for x in pr])
            b = np.array([max(x) for x in pr])
            rounds.append((a, b))
    for sweep in range(1, max_sweeps + 1):
        rotated = 0
        for a, b in rounds:
            wp, wq = w[:, a], w[:, b]
            alpha = np.einsum("ij,ij->j", wp.conj(), wp).real
            beta = np.einsum("ij,ij->j", wq.conj(), wq).real
            gamma = np.einsum("ij,ij->j", wp.conj(), wq)
            g = np.abs(gamma)
            do = (g > tol * np.sqrt(alpha * beta)) & (g > 0.0)
            if not np.any(do):
                continue
            rotated += int(np.count_nonzero(do))
            gs = np.where(do, g, 1.0)
            zeta = (beta - alpha) / (2.0 * gs)
            t = np.where(zeta >= 0, 1.0, -1.0) / (np.abs(zeta) + np.hypot(1.0, zeta))
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            e = np.conj(gamma) / gs
            c = np.where(do, c, 1.0)
            s = np.where(do, s, 0.0)
            e = np.where(do, e, 1.0)
            wq_e = wq * e[None, :]
            w[:, a] = c * wp - s * wq_e
            w[:, b] = s * wp + c * wq_e
            vp, vq_e = v[:, a], v[:, b] * e[None, :]
            v[:, a] = c * vp - s * vq_e
            v[:, b] = s * vp + c * vq_e
        if rotated == 0:
            return sweep, True
    return max_sweeps, False


def jacobi_svd(m: np.ndarray, order: str = "auto", tol: float | None = None,
               max_sweeps: int = 40) -> JacobiResult:
    """Thin SVD M = U diag(s) V^H of a complex matrix, s decreasing.

    If M has fewer rows than columns, the one-sided iteration runs on M^H and
    the roles of U and V are swapped.
    """
    m = np.asarray(m, dtype=np.complex128)
    rows, cols = m.shape
    if order == "lapack":
        u, s, vh = np.linalg.svd(m, full_matrices=False)
        return JacobiResult(u, s, vh, 0, True)
    transposed = rows < cols
    w = (m.conj().T if transposed else m).copy()
    mw, nw = w.shape
    if tol is None:
        tol = mw * EPS64
    v = np.eye(nw, dtype=np.complex128)
    if order == "auto":
        order = "cyclic" if nw <= 8 else "rr"
    if order == "cyclic":
        sweeps, conv = _sweeps_cyclic(w, v, tol, max_sweeps)
    elif order == "rr":
        sweeps, conv = _sweeps_rr(w, v, tol, max_sweeps)
    else:
        raise ValueError(order)
    s = np.sqrt(np.einsum("ij,ij->j", w.conj(), w).real)
    perm = np.argsort(-s, kind="stable")
    s = s[perm]
    w = w[:, perm]
    v = v[:, perm]
    u = np.zeros_like(w)
    nz = s > 0
    u[:, nz] = w[:, nz] / s[nz]
    if transposed:
        # M^H = U' S V'^H  ->  M = V' S U'^H
        return JacobiResult(v, s, u.conj().T, sweeps, conv)
    return JacobiResult(u, s, v.conj().T, sweeps, conv)
