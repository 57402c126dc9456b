"""Pins of the oracle's one-sided Jacobi SVD (CPU only).

The SVD has a plain definition, so the pin is the special case that reduces
to a library routine: singular values against ``numpy.linalg.svd`` and the
defining identities M = U S V^H, U^H U = I, V V^H = I.
"""
import numpy as np
import pytest

from oracle.jacobi import jacobi_svd, round_robin_pairs


def _rand(rng, m, n):
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def _graded(rng, m, n, lo=1e-12):
    r = min(m, n)
    u, _ = np.linalg.qr(_rand(rng, m, r))
    v, _ = np.linalg.qr(_rand(rng, n, r))
    s = np.logspace(0, np.log10(lo), r)
    return (u * s) @ v.conj().T


def _rank_def(rng, m, n, rank):
    return _rand(rng, m, rank) @ _rand(rng, rank, n)


CASES = [(1, 1), (2, 1), (1, 3), (4, 4), (7, 3), (3, 7), (16, 16), (33, 20), (20, 33), (64, 64)]


@pytest.mark.parametrize("order", ["cyclic", "rr"])
@pytest.mark.parametrize("shape", CASES)
def test_random_matches_lapack(order, shape):
    rng = np.random.default_rng(hash(shape) % 2**32)
    m = _rand(rng, *shape)
    res = jacobi_svd(m, order=order)
    s_ref = np.linalg.svd(m, compute_uv=False)
    s0 = s_ref[0]
    assert res.converged
    np.testing.assert_allclose(res.s, s_ref, rtol=0, atol=1e-13 * s0 * max(shape))
    rec = (res.u * res.s) @ res.vh
    assert np.linalg.norm(rec - m) <= 1e-13 * np.linalg.norm(m) * max(shape)
    r = min(shape)
    assert np.linalg.norm(res.u.conj().T @ res.u - np.eye(r)) < 1e-12
    assert np.linalg.norm(res.vh @ res.vh.conj().T - np.eye(r)) < 1e-12
    assert np.all(np.diff(res.s) <= 0)


@pytest.mark.parametrize("shape", [(40, 40), (50, 30), (30, 50)])
def test_graded_spectrum(shape):
    rng = np.random.default_rng(7)
    m = _graded(rng, *shape)
    res = jacobi_svd(m)
    s_ref = np.linalg.svd(m, compute_uv=False)
    np.testing.assert_allclose(res.s, s_ref, rtol=0, atol=1e-13 * s_ref[0] * 50)
    rec = (res.u * res.s) @ res.vh
    assert np.linalg.norm(rec - m) <= 1e-12 * np.linalg.norm(m)


def test_rank_deficient():
    rng = np.random.default_rng(3)
    m = _rank_def(rng, 48, 40, 5)
    res = jacobi_svd(m)
    s_ref = np.linalg.svd(m, compute_uv=False)
    np.testing.assert_allclose(res.s, s_ref, rtol=0, atol=1e-12 * s_ref[0])
    assert np.all(res.s[5:] < 1e-12 * res.s[0])
    rec = (res.u[:, :5] * res.s[:5]) @ res.vh[:5]
    assert np.linalg.norm(rec - m) <= 1e-12 * np.linalg.norm(m)


def test_zero_and_real_diagonal():
    z = np.zeros((5, 3), dtype=complex)
    res = jacobi_svd(z)
    assert np.all(res.s == 0)
    d = np.diag([3.0, -5.0, 1.0]).astype(complex)
    res = jacobi_svd(d)
    np.testing.assert_allclose(res.s, [5, 3, 1], atol=1e-15)


@pytest.mark.slow
def test_larger_rr():
    rng = np.random.default_rng(11)
    m = _rand(rng, 200, 160)
    res = jacobi_svd(m, order="rr")
    s_ref = np.linalg.svd(m, compute_uv=False)
    np.testing.assert_allclose(res.s, s_ref, rtol=0, atol=1e-12 * s_ref[0])


@pytest.mark.parametrize("n", [2, 4, 6, 10, 16])
def test_round_robin_covers_all_pairs_once(n):
    seen = []
    for r in range(n - 1):
        pr = round_robin_pairs(n, r)
        flat = [x for p in pr for x in p]
        assert sorted(flat) == list(range(n))  # disjoint, complete round
        seen += [tuple(sorted(p)) for p in pr]
    assert sorted(seen) == sorted((a, b) for a in range(n) for b in range(a + 1, n))
