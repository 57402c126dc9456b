"""Entanglement-aware MPS / MPO simulator, complex128, one step at a time.

Test infrastructure only (see the package header).

State (paper Sec. II): N site tensors A[i] of shape (chi_i, d, chi_{i+1}),
chi_0 = chi_N = 1, row-major; d = 2 for a pure state (Eq. 2) and d = 4 for a
mixed state stored as a matrix product operator (Eq. 4) with the per-site
index p = 2 sigma + sigma'.

Canonical form (Sec. III): a single orthogonality centre c; sites left of c
are left-normalised (sum_{l,s} conj(A[l,s,r]) A[l,s,r'] = delta), sites right
of c right-normalised.  It is moved by exact QR / LQ factorisations, one site
at a time, and kept at all times, which is what makes the truncation fidelity
a function of the bond's singular values alone (Sec. V, Sec. VI).

Two-site update (Sec. V, Sec. VI): contract A[i] and A[i+1] over their shared
bond, apply the 4x4 gate (16x16 superoperator), reshape to
Theta[(l, s1), (s2, r)], take its SVD, keep the fewest singular values whose
kept weight meets the target truncation fidelity (Eqs. (10)/(11) read as
f = sum_kept s^2 / sum_all s^2), capped by chi_max, renormalise, and multiply
f into the running estimate of Eq. (12) (kept as a log in FP64).

Readings of the paper taken here (each also listed in the design notes):
* Eq. (10) and Eq. (11) print a garbled numerator; both are read as
  f = w = sum_{j<k} s_j^2 / sum_j s_j^2 (for the pure state this is exactly
  |<psi|psi_trunc>|^2 with psi_trunc renormalised; for the mixed state it is
  the square of the Eq. (9) fidelity between rho and its truncation).
* Target rule (Sec. VI): the fewest kept values with f >= f_t, equality
  meeting the target, decided in discarded-weight form D(k) <= (1 - f_t) T.
* Numerically zero singular values (s_j <= tau * s_0) are never kept; at
  least one value is always kept.
* Targets: naive f_t = F_min^(1/n) (Eq. 14, n = number of two-qubit gates);
  global f_t = (F_min / P_g)^(1/(n - g)) before gate g; nearest
  f_t = F_min^((g+1)/n) / P_g; all clamped to (0, 1].  The fixed strategy
  is the standard fixed-bond-dimension simulation the paper compares against
  (Sec. VI, Fig. 4): every target is 1, so only the chi_max cap truncates.
* A chi_max cap (end of Sec. VI) overrides the target; the achieved f is then
  recorded and the update is flagged as capped.
* After truncation the kept values are renormalised to unit norm; for the MPO
  the logarithm of the removed scale is accumulated in ``lnS``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .jacobi import jacobi_svd

NAIVE, GLOBAL, NEAREST, FIXED = 0, 1, 2, 3


@dataclass
class TruncDecision:
    k: int          # kept rank
    k_f: int        # rank the target alone asks for
    k_nz: int       # number of numerically non-zero values
    total: float    # T = sum_j s_j^2
    discarded: float  # D(k) = sum_{j>=k} s_j^2
    f: float        # 1 - D(k)/T
    capped: bool


def truncation_rule(s: np.ndarray, f_t: float, chi_max: Optional[int],
                    tau: float) -> TruncDecision:
    """Kept rank for decreasing singular values ``s`` (Sec. VI; Eqs. 10/11).

    T = sum s^2 (summed from the smallest value up), D(k) = sum_{j>=k} s_j^2
    (suffix sums accumulated from the smallest value up),
    k_f = min{k >= 1 : D(k) <= (1 - f_t) T}, k_nz = max(1, #{s_j > tau s_0}),
    k = min(k_f, k_nz, chi_max) and f = 1 - D(k) / T.
    """
    s = np.asarray(s, dtype=np.float64)
    r = s.size
    w = s * s
    # suffix[j] = sum_{i >= j} w_i, accumulated from the tail (smallest first)
    suffix = np.zeros(r + 1)
    acc = 0.0
    for j in range(r - 1, -1, -1):
        acc += w[j]
        suffix[j] = acc
    total = suffix[0]
    thr = (1.0 - f_t) * total
    k_f = r
    for k in range(1, r + 1):
        if suffix[k] <= thr:
            k_f = k
            break
    k_nz = max(1, int(np.count_nonzero(s > tau * s[0]))) if r else 1
    k = min(k_f, k_nz)
    capped = False
    if chi_max is not None and chi_max < k:
        k = chi_max
        capped = True
    disc = suffix[k]
    f = 1.0 - disc / total if total > 0 else 1.0
    return TruncDecision(k, k_f, k_nz, total, disc, f, capped)


@dataclass
class GateRecord:
    gate: int
    site: int
    chi_l: int
    chi_m: int
    chi_r: int
    k: int
    f_t: float
    f: float
    lnP: float
    sweeps: int
    capped: bool
    s: Optional[np.ndarray] = None
    lnS: float = 0.0  # MPO log-scale after this update (0 for pure states)


class OracleMPS:
    """Plain CPU EA-MPS (kind='pure') / EA-MPO (kind='mixed')."""

    def __init__(self, n_sites: int, kind: str = "pure", chi_max: Optional[int] = None,
                 local: Optional[List[np.ndarray]] = None, tau: float = 1e-13,
                 svd: str = "auto", keep_spectra: bool = False):
        if kind not in ("pure", "mixed"):
            raise ValueError(kind)
        self.n = n_sites
        self.kind = kind
        self.d = 2 if kind == "pure" else 4
        self.chi_max = chi_max
        self.tau = tau
        self.svd = svd
        self.keep_spectra = keep_spectra
        self.A: List[np.ndarray] = []
        for i in range(n_sites):
            v = np.zeros(self.d, dtype=np.complex128)
            if local is None:
                v[0] = 1.0  # |0> or vec(|0><0|) = [1, 0, 0, 0]
            else:
                v[:] = local[i]
            self.A.append(v.reshape(1, self.d, 1))
        self.center = 0
        self.lnP = 0.0
        self.lnS = 0.0
        self.g = 0
        self.f_min = None
        self.n_total = None
        self.strategy = GLOBAL
        self.log: List[GateRecord] = []
        self.any_capped = False

    # ----------------------------------------------------------------- state

    def load(self, tensors: List[np.ndarray], center: int):
        """Replace the state by explicit site tensors (no normalisation)."""
        assert len(tensors) == self.n
        for i, a in enumerate(tensors):
            assert a.ndim == 3 and a.shape[1] == self.d
            if i > 0:
                assert tensors[i - 1].shape[2] == a.shape[0]
        assert tensors[0].shape[0] == 1 and tensors[-1].shape[2] == 1
        self.A = [np.array(a, dtype=np.complex128) for a in tensors]
        self.center = center

    def bond_dims(self) -> List[int]:
        return [a.shape[2] for a in self.A[:-1]]

    def set_schedule(self, f_min: float, n_total: int, strategy: int = GLOBAL):
        self.f_min = f_min
        self.n_total = n_total
        self.strategy = strategy

    def target(self) -> float:
        """Target truncation fidelity of the next two-qubit gate (Eq. 14 and
        the adaptive updates of Sec. VI)."""
        if self.f_min is None:
            return 1.0
        n, g = self.n_total, self.g
        if self.strategy == NAIVE:
            ft = self.f_min ** (1.0 / n)
        elif self.strategy == GLOBAL:
            left = n - g
            ft = 1.0 if left <= 0 else math.exp((math.log(self.f_min) - self.lnP) / left)
        elif self.strategy == NEAREST:
            ft = math.exp(math.log(self.f_min) * (g + 1) / n - self.lnP)
        elif self.strategy == FIXED:
            ft = 1.0
        else:
            raise ValueError(self.strategy)
        return min(1.0, max(ft, 1e-300))

    # -------------------------------------------------------- canonical form

    def _move_right(self):
        """QR of the centre site as (chi_l d) x chi_r; R goes right (Sec. III)."""
        c = self.center
        a = self.A[c]
        cl, d, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl * d, cr))
        self.A[c] = q.reshape(cl, d, q.shape[1])
        self.A[c + 1] = np.einsum("ij,jsk->isk", r, self.A[c + 1])
        self.center = c + 1

    def _move_left(self):
        """LQ of the centre site as chi_l x (d chi_r); L goes left (Sec. III)."""
        c = self.center
        a = self.A[c]
        cl, d, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl, d * cr).conj().T)  # M^H = Q R
        # M = R^H Q^H: Q^H is right-normalised, R^H goes left
        self.A[c] = q.conj().T.reshape(q.shape[1], d, cr)
        self.A[c - 1] = np.einsum("isj,jk->isk", self.A[c - 1], r.conj().T)
        self.center = c - 1

    def move_center(self, j: int):
        while self.center < j:
            self._move_right()
        while self.center > j:
            self._move_left()

    # ------------------------------------------------------------- one-site

    def apply_1q(self, i: int, g: np.ndarray):
        """A[i][l,s,r] <- sum_t g[s,t] A[i][l,t,r].  A non-unitary operator
        first brings the centre to i so the canonical form survives."""
        g = np.asarray(g, dtype=np.complex128)
        assert g.shape == (self.d, self.d)
        if np.linalg.norm(g.conj().T @ g - np.eye(self.d)) > 1e-12:
            self.move_center(i)
        self.A[i] = np.einsum("st,atb->asb", g, self.A[i])

    # ------------------------------------------------------------- two-site

    def theta(self, i: int, G: np.ndarray) -> np.ndarray:
        """Theta[(l,s1),(s2,r)] = sum_{t1,t2} G[(s1 s2),(t1 t2)]
        sum_m A[i][l,t1,m] A[i+1][m,t2,r]."""
        d = self.d
        a, b = self.A[i], self.A[i + 1]
        c = np.einsum("ljm,mkr->ljkr", a, b)
        g4 = np.asarray(G, dtype=np.complex128).reshape(d, d, d, d)
        th = np.einsum("stuv,luvr->lstr", g4, c)
        return th.reshape(a.shape[0] * d, d * b.shape[2])

    def apply_2q(self, i: int, G: np.ndarray, f_t: Optional[float] = None,
                 direction: str = "right", forced_k: Optional[int] = None) -> GateRecord:
        """Two-site update on (i, i+1) (Sec. V-VI).  Returns the gate record."""
        d = self.d
        if not (self.center == i or self.center == i + 1):
            self.move_center(i if self.center < i else i + 1)
        if f_t is None or f_t < 0:
            f_t = self.target()
        chi_l, chi_m, chi_r = self.A[i].shape[0], self.A[i].shape[2], self.A[i + 1].shape[2]
        th = self.theta(i, G)
        res = jacobi_svd(th, order=self.svd)
        s = res.s
        dec = truncation_rule(s, f_t, self.chi_max, self.tau)
        k = dec.k if forced_k is None else forced_k
        disc = float(np.sum((s[k:] ** 2)[::-1])) if forced_k is not None else dec.discarded
        kept2 = float(np.sum((s[:k] ** 2)[::-1]))
        st = s[:k] / math.sqrt(kept2)
        if self.kind == "mixed":
            self.lnS += 0.5 * math.log(kept2)
        u = res.u[:, :k]
        vh = res.vh[:k, :]
        if direction == "right":
            self.A[i] = u.reshape(chi_l, d, k)
            self.A[i + 1] = (st[:, None] * vh).reshape(k, d, chi_r)
            self.center = i + 1
        else:
            self.A[i] = (u * st[None, :]).reshape(chi_l, d, k)
            self.A[i + 1] = vh.reshape(k, d, chi_r)
            self.center = i
        f = 1.0 - disc / dec.total if dec.total > 0 else 1.0
        self.lnP += math.log1p(-disc / dec.total) if dec.total > 0 else 0.0
        capped = dec.capped if forced_k is None else False
        self.any_capped |= capped
        rec = GateRecord(self.g, i, chi_l, chi_m, chi_r, k, f_t, f, self.lnP,
                         res.sweeps, capped, s.copy() if self.keep_spectra else None,
                         self.lnS)
        self.g += 1
        self.log.append(rec)
        return rec

    def apply_layer(self, ops, budgets=None):
        """Apply disjoint two-qubit ops of one layer.  Visiting order follows
        the centre: ascending if the centre is nearer the lowest site, else
        descending; write-back follows the visiting direction."""
        ops = list(ops)
        if not ops:
            return []
        sites = [op.site for op in ops]
        lo, hi = min(sites), max(sites)
        asc = abs(self.center - lo) <= abs(self.center - hi)
        order = sorted(range(len(ops)), key=lambda j: sites[j], reverse=not asc)
        recs = []
        for j in order:
            b = None if budgets is None else budgets[j]
            recs.append(self.apply_2q(ops[j].site, ops[j].mat, b,
                                      direction="right" if asc else "left"))
        return recs

    def run(self, program, f_min: float = 1.0, strategy: int = GLOBAL):
        """Run a :class:`circuits.Program`: per layer, one-qubit ops in order,
        then the two-qubit ops as one layer."""
        self.set_schedule(f_min, program.n_2q, strategy)
        for layer in program.layers:
            ones = [op for op in layer if op.width == 1]
            twos = [op for op in layer if op.width == 2]
            for op in ones:
                self.apply_1q(op.site, op.mat)
            self.apply_layer(twos)
        return self

    # -------------------------------------------------------------- outputs

    def fidelity_estimate(self):
        return math.exp(self.lnP), self.lnP

    def to_vector(self) -> np.ndarray:
        """Contract the chain: the 2^N state vector (pure) or the 4^N vector
        vec(rho) over (p_1..p_N) (mixed), without the ``lnS`` scale."""
        v = self.A[0].reshape(self.d, -1)
        for a in self.A[1:]:
            cl = a.shape[0]
            v = (v @ a.reshape(cl, -1)).reshape(-1, a.shape[2])
        return v.reshape(-1)

    def to_statevector(self) -> np.ndarray:
        assert self.kind == "pure"
        return self.to_vector()

    def to_density(self) -> np.ndarray:
        """Dense rho / Tr(rho) (mixed states only)."""
        assert self.kind == "mixed"
        n = self.n
        v = self.to_vector().reshape([2, 2] * n)  # s1 s1' s2 s2' ...
        perm = list(range(0, 2 * n, 2)) + list(range(1, 2 * n, 2))
        rho = v.transpose(perm).reshape(2 ** n, 2 ** n)
        return rho / np.trace(rho)

    def expect(self, site: int, width: int, op: np.ndarray) -> complex:
        """<O> for an operator on ``site`` (width 1) or (site, site+1).

        Pure (Eq. 6): the centre is moved to ``site`` and only the centre
        block is contracted, normalised by its norm.  Mixed: Tr(rho O) /
        Tr(rho) by a transfer contraction with the identity vector
        vec(I) = [1, 0, 0, 1] on the other sites.
        """
        op = np.asarray(op, dtype=np.complex128)
        if self.kind == "pure":
            self.move_center(site)
            if width == 1:
                a = self.A[site]
                oa = np.einsum("st,ltr->lsr", op, a)
                return complex(np.vdot(a, oa) / np.vdot(a, a))
            th = self.theta(site, np.eye(4))
            oth = self.theta(site, op)
            return complex(np.vdot(th, oth) / np.vdot(th, th))
        return self._mixed_trace(site, width, op) / self._mixed_trace(None, 0, None)

    def _mixed_trace(self, site, width, op) -> complex:
        ident = np.array([1, 0, 0, 1], dtype=np.complex128)
        env = np.ones(1, dtype=np.complex128)
        j = 0
        while j < self.n:
            if site is not None and j == site:
                if width == 1:
                    # Tr(rho O) weight: O[s', s] at p = 2 s + s'
                    wgt = np.array([op[sp, s] for s in range(2) for sp in range(2)])
                    env = np.einsum("l,lpr,p->r", env, self.A[j], wgt)
                    j += 1
                    continue
                o4 = op.reshape(2, 2, 2, 2)  # [s1' s2', s1 s2] as (a1 a2 b1 b2)
                wgt = np.zeros((4, 4), dtype=np.complex128)
                for s1 in range(2):
                    for s1p in range(2):
                        for s2 in range(2):
                            for s2p in range(2):
                                wgt[2 * s1 + s1p, 2 * s2 + s2p] = o4[s1p, s2p, s1, s2]
                env = np.einsum("l,lpm,mqr,pq->r", env, self.A[j], self.A[j + 1], wgt)
                j += 2
                continue
            env = np.einsum("l,lpr,p->r", env, self.A[j], ident)
            j += 1
        return complex(env[0])
