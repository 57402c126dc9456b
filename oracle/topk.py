"""Partial (top-k) SVD of the two-site matrix by randomized subspace
iteration, the kept rank decided from the Ritz values plus the weight outside
the subspace.  Test infrastructure only (see the package header).

Reading taken (not in the paper, which takes the full SVD of the two-site
matrix, Sec. V).  The truncation rule of Sec. VI needs the leading singular
values only until their weight reaches f_t T, and T = ||Theta||_F^2 is known
without any SVD.  So the factorisation may stop at a subspace of dimension
l < n that holds that weight:

  X       = Theta if it has at least as many rows as columns, else Theta^H
            (mw x nw, mw >= nw; the same orientation as the full path)
  Omega   = mw x l, entries (2u - 1) + i (2u' - 1) from SplitMix64 (below)
  Q       = orth(X^H Omega)                              range finder
  q times:  Q <- orth(X^H orth(X Q))                     subspace iteration
  W       = X Q = U_W S V_W^H                            SVD of an mw x l matrix
  R       = T - ||W||_F^2                                weight outside span(Q)

(Halko, Martinsson & Tropp, SIAM Rev. 53, 2011, Algs. 4.3/4.4.)  The Ritz
values s (of W) decide the kept rank as in Sec. VI with every discarded
weight raised by R: D(k) = R + sum_{j >= k} s_j^2, T = D(0), k_f = min{k >=
1: D(k) <= (1 - f_t) T} (l + 1 when no k <= l qualifies), k = min(k_f, k_nz,
chi_max).  The kept state X ~ U_W S_k (Q V_W)_k^H is the projection of the
exact one onto a rank-k subspace, so its fidelity with the untruncated state
is exactly 1 - D(k)/T (Eqs. 10-11 stay exact bookkeeping); k may exceed the
full SVD's, and a capped update may keep less weight than the full SVD's.

Subspace size: l = min(chi_max, 2 chi_m) + p (chi_m the bond the gate acts
across, p the oversampling); an attempt is accepted when k <= l - p, else l
doubles.  Whenever 4 l > 3 nw, or when the orthonormalisation meets a rank-
deficient block, the full factorisation runs instead.

SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based generator:
output(x) = mix(seed + (x + 1) gamma mod 2^64), gamma = 0x9E3779B97F4A7C15,
mix(z): z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9; z = (z ^ (z >> 27)) *
0x94D049BB133111EB; z ^ (z >> 31).  u(x) = (output(x) >> 11) 2^-53.  Entry
(row r, column c) of Omega for gate g, attempt a: e = c mw + r, counters
base + 2e (real part) and base + 2e + 1 (imaginary), base = ((g mod 2^20) 16
+ a) 2^40.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .jacobi import jacobi_svd
from .mps import OracleMPS, GateRecord, TruncDecision

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB


def splitmix64(seed: int, counters) -> np.ndarray:
    """SplitMix64 output at each counter (uint64 arithmetic, mod 2^64)."""
    x = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % 2 ** 64) + (x + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
    return z ^ (z >> np.uint64(31))


def uniform_pm1(seed: int, counters) -> np.ndarray:
    """2 u - 1 in [-1, 1), u = top 53 bits of the output times 2^-53."""
    u = (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return 2.0 * u - 1.0


def omega(seed: int, gate: int, attempt: int, rows: int, cols: int) -> np.ndarray:
    """The rows x cols starting block of one attempt (column-major counters)."""
    assert 0 <= attempt < 16 and rows * cols * 2 < 2 ** 40
    base = ((gate % 2 ** 20) * 16 + attempt) << 40
    e = np.arange(rows * cols, dtype=np.uint64)  # e = c * rows + r
    re = uniform_pm1(seed, np.uint64(base) + np.uint64(2) * e)
    im = uniform_pm1(seed, np.uint64(base) + np.uint64(2) * e + np.uint64(1))
    return (re + 1j * im).reshape(cols, rows).T


def truncation_rule_residual(s: np.ndarray, resid: float, f_t: float,
                             chi_max: Optional[int], tau: float) -> TruncDecision:
    """Sec. VI's rule on Ritz values ``s`` (decreasing) when a weight
    ``resid`` lies outside the subspace: D(k) = resid + sum_{j>=k} s_j^2
    (the suffix summed from the smallest value up, then resid added), T =
    D(0); k_f = l + 1 when no k <= l meets the target."""
    s = np.asarray(s, dtype=np.float64)
    r = s.size
    w = s * s
    suffix = np.zeros(r + 1)
    acc = 0.0
    for j in range(r - 1, -1, -1):
        acc += w[j]
        suffix[j] = acc
    suffix = suffix + resid
    total = suffix[0]
    thr = (1.0 - f_t) * total
    k_f = r + 1
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


def orth(Y: np.ndarray) -> np.ndarray:
    """An orthonormal basis of range(Y) (Householder QR as a library step)."""
    return np.linalg.qr(Y, mode="reduced")[0]


@dataclass
class TopkResult:
    l: int            # subspace dimension of the accepted attempt
    attempts: int
    s: np.ndarray     # (l,) Ritz values, decreasing
    u: np.ndarray     # (mw, l) left vectors of X
    v: np.ndarray     # (nw, l) right vectors of X
    resid: float      # R = T - ||X Q||_F^2
    dec: TruncDecision
    sweeps: int


def start_size(nw: int, chi_m: int, chi_max: Optional[int], p: int) -> int:
    cap = nw if chi_max is None else min(chi_max, nw)
    return min(cap, 2 * chi_m) + p


def topk_factor(X: np.ndarray, f_t: float, chi_max: Optional[int], tau: float, chi_m: int,
                p: int = 64, q: int = 1, seed: int = 0, gate: int = 0,
                svd: str = "auto") -> Optional[TopkResult]:
    """The accepted attempt for X (mw x nw, mw >= nw), or None when the full
    factorisation is to run (subspace too large for a gain)."""
    X = np.asarray(X, dtype=np.complex128)
    mw, nw = X.shape
    assert mw >= nw and p >= 1
    T = float(np.sum(X.real ** 2 + X.imag ** 2))
    l = start_size(nw, chi_m, chi_max, p)
    a = 0
    while 4 * l <= 3 * nw:
        Q = orth(X.conj().T @ omega(seed, gate, a, mw, l))
        for _ in range(q):
            Q = orth(X.conj().T @ orth(X @ Q))
        W = X @ Q
        resid = max(0.0, T - float(np.sum(W.real ** 2 + W.imag ** 2)))
        res = jacobi_svd(W, order=svd)
        dec = truncation_rule_residual(res.s, resid, f_t, chi_max, tau)
        if dec.k <= l - p:
            return TopkResult(l, a + 1, res.s, res.u, Q @ res.vh.conj().T, resid, dec,
                              res.sweeps)
        l = min(nw, 2 * l)
        a += 1
    return None


class OracleTopK(OracleMPS):
    """OracleMPS whose two-site updates of at least ``topk_min`` columns (in
    the orientation above) take the partial factorisation."""

    def __init__(self, n_sites: int, kind: str = "pure", chi_max: Optional[int] = None,
                 tau: float = 1e-13, svd: str = "auto", keep_spectra: bool = False,
                 p: int = 64, q: int = 1, seed: int = 0, topk_min: int = 256):
        super().__init__(n_sites, kind, chi_max=chi_max, tau=tau, svd=svd,
                         keep_spectra=keep_spectra)
        self.p, self.q, self.seed, self.topk_min = p, q, seed, topk_min

    def apply_2q(self, i: int, G: np.ndarray, f_t: Optional[float] = None,
                 direction: str = "right", forced_k: Optional[int] = None) -> GateRecord:
        d = self.d
        if not (self.center == i or self.center == i + 1):
            self.move_center(i if self.center < i else i + 1)
        chi_l, chi_m, chi_r = self.A[i].shape[0], self.A[i].shape[2], self.A[i + 1].shape[2]
        M, N = chi_l * d, d * chi_r
        if forced_k is not None or min(M, N) < self.topk_min:
            return super().apply_2q(i, G, f_t, direction, forced_k)
        th = self.theta(i, G)
        tall = M >= N
        X = th if tall else th.conj().T
        if f_t is None or f_t < 0:
            f_t = self.target()
        res = topk_factor(X, f_t, self.chi_max, self.tau, chi_m, self.p, self.q, self.seed,
                          self.g, self.svd)
        if res is None:
            # the full path recomputes Theta from the unchanged tensors
            return super().apply_2q(i, G, f_t, direction, forced_k)
        dec = res.dec
        k = dec.k
        s = res.s
        if tall:  # Theta ~ U_W S (Q V_W)^H
            u, vh = res.u, res.v.conj().T
        else:     # Theta = X^H ~ (Q V_W) S U_W^H
            u, vh = res.v, res.u.conj().T
        kept2 = float(np.sum((s[:k] ** 2)[::-1]))
        st = s[:k] / math.sqrt(kept2)
        if self.kind == "mixed":
            self.lnS += 0.5 * math.log(kept2)
        if direction == "right":
            self.A[i] = u[:, :k].reshape(chi_l, d, k)
            self.A[i + 1] = (st[:, None] * vh[:k, :]).reshape(k, d, chi_r)
            self.center = i + 1
        else:
            self.A[i] = (u[:, :k] * st[None, :]).reshape(chi_l, d, k)
            self.A[i + 1] = vh[:k, :].reshape(k, d, chi_r)
            self.center = i
        f = 1.0 - dec.discarded / dec.total if dec.total > 0 else 1.0
        self.lnP += math.log1p(-dec.discarded / dec.total) if dec.total > 0 else 0.0
        self.any_capped |= dec.capped
        rec = GateRecord(self.g, i, chi_l, chi_m, chi_r, k, f_t, f, self.lnP, res.sweeps,
                         dec.capped, s.copy() if self.keep_spectra else None, self.lnS)
        rec.subspace, rec.attempts, rec.resid = res.l, res.attempts, res.resid
        self.g += 1
        self.log.append(rec)
        return rec
