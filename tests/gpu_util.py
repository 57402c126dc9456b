"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np

from oracle.mps import OracleMPS


def oracle_run(program, f_min=1.0, chi_max=None, strategy=1, svd="auto", kind=None):
    o = OracleMPS(program.n_sites, kind or program.kind, chi_max=chi_max, svd=svd,
                  keep_spectra=True)
    o.run(program, f_min, strategy)
    return o


def protected(rec_o, ft, tol_w):
    """A kept-rank decision is protected when the discarded weight at k and
    at k-1 are both farther than tol_w * T from the threshold (1 - f_t) T."""
    s = rec_o.s
    w = s * s
    T = w.sum()
    thr = (1.0 - ft) * T
    k = rec_o.k
    d_k = w[k:].sum()
    d_km1 = w[k - 1:].sum()
    return abs(d_k - thr) > tol_w * T and abs(d_km1 - thr) > tol_w * T


def gauge_free_pair(a, b):
    """A_i A_{i+1} as a (chiL d) x (d chiR) matrix."""
    cl, d, _ = a.shape
    _, d2, cr = b.shape
    return np.einsum("lsm,mtr->lstr", a, b).reshape(cl * d, d2 * cr)
