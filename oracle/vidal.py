"""Layer-parallel EA-MPS in the Vidal gauge, with Hastings' division-free
update.  Test infrastructure only (see the package header).

Reading taken (not in the paper).  Sec. III asks for the canonical form to be
kept; the exact way, one orthogonality centre moved site by site, makes the
gates of a layer sequential.  The alternative kept here stores the state in
Vidal's form, the site tensors B_i = Gamma_i Lambda_{i+1} (right-normalised
when the form is exact) and the Schmidt values Lambda_i of every bond, so that
all disjoint gates of a layer can be updated independently:

  C      = G (B_i B_{i+1})                      reshaped (chi_i d) x (d chi_{i+2})
  Theta  = diag(Lambda_i) C                     the two-site block in canonical form
  Theta  = X S Y^H                               SVD; k kept by the Sec. VI rule
  B_{i+1} <- Y_k^H,  B_i <- C Y_k / ||s_k||,  Lambda_{i+1} <- s_k / ||s_k||

B_i is obtained from C, not by dividing X S by Lambda_i, which would amplify
the rounding of small Schmidt values (Hastings, Phys. Rev. B 79, 2009).  The
truncation fidelity is f = sum_kept s^2 / sum s^2 as in the exact mode (Eqs.
10-11).  While no truncation has happened the form is exact and so is f; after
truncations the bonds' Lambda are Schmidt values only approximately, and f and
the running estimate of Eq. (12) approximate the exact-centre values.

All gates of a layer take their target from the estimate before the layer
(the schedule of Sec. VI evaluated once per layer: global f_t =
(F_min/P)^(1/(n-g)) with g the gates before the layer; naive F_min^(1/n)).
Gates of one layer act on disjoint sites and bonds, so applying them one after
another in site order is the same as applying them at once.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .jacobi import jacobi_svd
from .mps import OracleMPS, GateRecord, truncation_rule, GLOBAL, NAIVE, NEAREST, FIXED


class OracleVidal(OracleMPS):
    """EA-MPS (pure) / EA-MPO (mixed) in the Vidal gauge: ``A[i]`` holds B_i,
    ``lam[i]`` the Schmidt values of bond i (between sites i-1 and i;
    lam[0] = lam[N] = [1])."""

    def __init__(self, n_sites: int, kind: str = "pure", chi_max: Optional[int] = None,
                 tau: float = 1e-13, svd: str = "auto", keep_spectra: bool = False):
        super().__init__(n_sites, kind, chi_max=chi_max, tau=tau, svd=svd,
                         keep_spectra=keep_spectra)
        self.lam: List[np.ndarray] = [np.ones(1) for _ in range(n_sites + 1)]

    def layer_targets(self, n_gates: int) -> List[float]:
        """Targets of the next layer's gates, all from the estimate before it."""
        if self.f_min is None:
            return [1.0] * n_gates
        n, g = self.n_total, self.g
        if self.strategy == NAIVE:
            ft = self.f_min ** (1.0 / n)
        elif self.strategy == GLOBAL:
            left = n - g
            ft = 1.0 if left <= 0 else math.exp((math.log(self.f_min) - self.lnP) / left)
        elif self.strategy == FIXED:
            ft = 1.0
        else:
            raise ValueError("strategy not defined for the layer-parallel gauge")
        return [min(1.0, max(ft, 1e-300))] * n_gates

    def apply_1q(self, i: int, g: np.ndarray):
        """B_i <- g B_i (unitary g keeps the form exact)."""
        g = np.asarray(g, dtype=np.complex128)
        self.A[i] = np.einsum("st,atb->asb", g, self.A[i])

    def apply_2q(self, i: int, G: np.ndarray, f_t: Optional[float] = None,
                 direction: str = "right", forced_k: Optional[int] = None) -> GateRecord:
        d = self.d
        if f_t is None or f_t < 0:
            f_t = self.layer_targets(1)[0]
        chi_l, chi_m, chi_r = self.A[i].shape[0], self.A[i].shape[2], self.A[i + 1].shape[2]
        C = self.theta(i, G)  # (chi_l d) x (d chi_r), rows (l, s1)
        th = np.repeat(self.lam[i], d)[:, None] * C
        res = jacobi_svd(th, order=self.svd)
        s = res.s
        dec = truncation_rule(s, f_t, self.chi_max, self.tau)
        k = dec.k if forced_k is None else forced_k
        disc = float(np.sum((s[k:] ** 2)[::-1])) if forced_k is not None else dec.discarded
        kept2 = float(np.sum((s[:k] ** 2)[::-1]))
        norm = math.sqrt(kept2)
        yk = res.vh[:k, :].conj().T  # (d chi_r) x k
        self.A[i + 1] = res.vh[:k, :].reshape(k, d, chi_r)
        self.A[i] = (C @ yk / norm).reshape(chi_l, d, k)
        self.lam[i + 1] = s[:k] / norm
        if self.kind == "mixed":
            self.lnS += 0.5 * math.log(kept2)
        f = 1.0 - disc / dec.total if dec.total > 0 else 1.0
        self.lnP += math.log1p(-disc / dec.total) if dec.total > 0 else 0.0
        capped = dec.capped if forced_k is None else False
        self.any_capped |= capped
        rec = GateRecord(self.g, i, chi_l, chi_m, chi_r, k, f_t, f, self.lnP, res.sweeps,
                         capped, s.copy() if self.keep_spectra else None, self.lnS)
        self.g += 1
        self.log.append(rec)
        return rec

    def apply_layer(self, ops, budgets=None):
        """All disjoint two-qubit ops of one layer, targets from the estimate
        before the layer, applied in increasing site order."""
        ops = list(ops)
        if not ops:
            return []
        fts = self.layer_targets(len(ops)) if budgets is None else list(budgets)
        order = sorted(range(len(ops)), key=lambda j: ops[j].site)
        return [self.apply_2q(ops[j].site, ops[j].mat, fts[j]) for j in order]

    def right_normalisation_error(self) -> float:
        """max_i || B_i B_i^H - 1 || over sites (0 while the form is exact)."""
        err = 0.0
        for b in self.A:
            m = b.reshape(b.shape[0], -1)
            err = max(err, float(np.abs(m @ m.conj().T - np.eye(m.shape[0])).max()))
        return err
