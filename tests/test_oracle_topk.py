"""Pins of the partial (top-k) factorisation oracle, CPU only: SplitMix64
against its published outputs, the Ritz values against the exact singular
values (interlacing, exact capture of a low-rank matrix), the residual
weight, the rule with a residual against the plain rule, and the key
property that the recorded truncation fidelity is the brute-force overlap of
the truncated state (Eqs. 10-11) however rough the subspace.  Planted
mistakes must fail these pins."""
import math

import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.mps import OracleMPS, truncation_rule
from oracle import topk as K


def test_splitmix64_published_outputs():
    """The first three outputs of SplitMix64 seeded with 0 (the reference
    implementation's sequence: state advanced by gamma before each mix)."""
    out = K.splitmix64(0, [0, 1, 2])
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                     0x06C45D188009454F]


def test_uniform_range_and_moments():
    x = K.uniform_pm1(7, np.arange(200000, dtype=np.uint64))
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0 / 3.0) < 0.01


def test_omega_layout_is_column_major_counters():
    om = K.omega(3, 5, 2, 7, 4)
    base = ((5 * 16) + 2) << 40
    r, c = 6, 3
    e = c * 7 + r
    assert om[r, c].real == K.uniform_pm1(3, [base + 2 * e])[0]
    assert om[r, c].imag == K.uniform_pm1(3, [base + 2 * e + 1])[0]


def test_rule_with_zero_residual_is_the_plain_rule():
    rng = np.random.default_rng(1)
    for _ in range(100):
        r = int(rng.integers(1, 30))
        s = np.sort(rng.random(r))[::-1]
        ft = float(rng.uniform(0.3, 0.999))
        cap = int(rng.integers(1, 40))
        a = truncation_rule(s, ft, cap, 1e-13)
        b = K.truncation_rule_residual(s, 0.0, ft, cap, 1e-13)
        assert (a.k, a.k_nz, a.capped) == (b.k, b.k_nz, b.capped)
        assert a.f == b.f and a.total == b.total


def test_rule_residual_raises_every_discarded_weight():
    """Ritz values s plus a weight R outside: the rule equals the plain rule
    on the spectrum s extended by values carrying R (any split of R), as long
    as k stays inside s."""
    s = np.array([1.0, 0.6, 0.3, 0.1])
    R = 0.05
    d = K.truncation_rule_residual(s, R, 0.9, None, 1e-13)
    ext = np.concatenate([s, [math.sqrt(R / 2)] * 2])
    p = truncation_rule(ext, 0.9, None, 1e-13)
    assert d.k == p.k and abs(d.f - p.f) < 1e-15 and abs(d.total - p.total) < 1e-15
    # a target the subspace cannot meet: k_f = l + 1
    d = K.truncation_rule_residual(s, R, 0.999, None, 1e-13)
    assert d.k_f == len(s) + 1 and d.k == len(s)


def _lowrank(m, n, r, seed, decay=0.7):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
    b = rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n))
    u, _ = np.linalg.qr(a)
    v, _ = np.linalg.qr(b.conj().T)
    s = decay ** np.arange(r)
    return (u * s) @ v.conj().T, s


@pytest.mark.parametrize("q", [0, 1])
def test_exact_capture_of_a_low_rank_matrix(q):
    """rank r <= l - p: span(Q) holds the whole row space, so the Ritz values
    are the singular values, R = 0, and the decision is the full SVD's."""
    X, s = _lowrank(96, 80, 12, 3)
    res = K.topk_factor(X, 0.999, None, 1e-13, chi_m=10, p=8, q=q)
    assert res is not None and res.l == 28
    np.testing.assert_allclose(res.s[:12], s, atol=1e-13)
    assert np.all(res.s[12:] < 1e-13) and abs(res.resid) < 1e-13
    full = truncation_rule(np.linalg.svd(X, compute_uv=False), 0.999, None, 1e-13)
    assert res.dec.k == full.k and abs(res.dec.f - full.f) < 1e-13
    Xk = (res.u[:, :res.dec.k] * res.s[:res.dec.k]) @ res.v[:, :res.dec.k].conj().T
    u, sv, vh = np.linalg.svd(X)
    k = full.k
    np.testing.assert_allclose(Xk, (u[:, :k] * sv[:k]) @ vh[:k], atol=1e-12)


def test_ritz_values_interlace_and_residual_bounds():
    """s_j(X Q) <= s_j(X); R = sum s(X)^2 - sum s(XQ)^2 >= sum_{j>=l} s_j(X)^2;
    the kept weight at any k never exceeds the full SVD's."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((120, 100)) + 1j * rng.standard_normal((120, 100))
    X = X * (0.97 ** np.arange(100))[None, :]
    sx = np.linalg.svd(X, compute_uv=False)
    res = K.topk_factor(X, 0.5, 30, 1e-13, chi_m=15, p=10, q=0)
    assert res is not None and res.l == 40
    assert np.all(res.s <= sx[:res.l] * (1 + 1e-12))
    tail = np.sum(sx[res.l:] ** 2)
    assert res.resid >= tail * (1 - 1e-12)
    assert abs(res.resid - (np.sum(sx ** 2) - np.sum(res.s ** 2))) < 1e-10
    for k in range(1, res.l + 1):
        assert np.sum(res.s[:k] ** 2) <= np.sum(sx[:k] ** 2) * (1 + 1e-12)


def test_subspace_iteration_approaches_the_full_svd():
    """More power iterations bring the leading Ritz values to the singular
    values (a spectrum with a gap after the cap)."""
    rng = np.random.default_rng(5)
    s = np.concatenate([np.linspace(1.0, 0.5, 20), 0.05 * np.linspace(1, 0.5, 60)])
    u, _ = np.linalg.qr(rng.standard_normal((90, 80)) + 1j * rng.standard_normal((90, 80)))
    v, _ = np.linalg.qr(rng.standard_normal((80, 80)) + 1j * rng.standard_normal((80, 80)))
    X = (u * s) @ v.conj().T
    errs = []
    for q in (0, 1, 3):
        res = K.topk_factor(X, 1.0, 20, 1e-13, chi_m=10, p=4, q=q)
        errs.append(np.abs(res.s[:20] - s[:20]).max())
    assert errs[2] < 1e-9 and errs[2] < errs[1] < errs[0]


def _canonical_random(bonds, d, seed, kind):
    n = len(bonds) - 1
    o = OracleMPS(n, kind)
    o.load(C.random_mps_tensors(bonds, d, seed), n - 1)
    o.move_center(0)
    o.A[0] = o.A[0] / np.linalg.norm(o.A[0])
    return o


def _apply_pair(vec, n, d, i, G):
    """G (d^2 x d^2) on sites (i, i+1) of a length d^n vector."""
    v = vec.reshape(d ** i, d * d, d ** (n - i - 2))
    return np.einsum("ab,xby->xay", G, v).reshape(-1)


# (bonds, d, kind, site, chi_max, f_t): chi_l, chi_m, chi_r around the pair
CASES = {
    "capped": ([1, 2, 4, 8, 16, 32, 16, 8, 4, 2, 1], 2, "pure", 4, 6, 0.97),
    "target": ([1, 2, 4, 8, 12, 6, 12, 8, 4, 2, 1], 2, "pure", 4, None, 0.97),
    "wide": ([1, 2, 4, 8, 10, 6, 12, 8, 4, 2, 1], 2, "pure", 4, None, 0.97),
    "grown": ([1, 4, 16, 8, 16, 4, 1], 4, "mixed", 2, None, 0.95),
}


def _one_update(case, factor=None):
    bonds, d, kind, site, chi_max, ft = CASES[case]
    o = _canonical_random(bonds, d, 11, kind)
    vec = o.to_vector()
    rng = np.random.default_rng(2)
    G = C.haar_unitary(rng, d * d)
    t = K.OracleTopK(len(bonds) - 1, kind, chi_max=chi_max, p=3, q=0, seed=9, topk_min=8)
    t.A = [a.copy() for a in o.A]
    t.center = o.center
    rec = t.apply_2q(site, G, ft)
    ref = _apply_pair(vec, len(bonds) - 1, d, site, G)
    phi = t.to_vector()
    fid = abs(np.vdot(ref, phi)) ** 2 / (np.vdot(phi, phi).real * np.vdot(ref, ref).real)
    return rec, fid, ft


@pytest.mark.parametrize("case", list(CASES))
def test_recorded_fidelity_is_the_brute_force_overlap(case):
    """One truncating update of an exact state (pure, or an MPO as its
    vectorisation) with a rough subspace (q = 0, oversampling 3): f =
    |<G psi|psi_t>|^2 / (<G psi|G psi> <psi_t|psi_t>) exactly (Eqs. 10-11),
    and the estimate is ln f; both orientations, a capped update and an
    accepted second attempt."""
    rec, fid, ft = _one_update(case)
    assert hasattr(rec, "subspace"), "the partial path must have run"
    assert (rec.attempts >= 2) == (case == "grown")
    if case == "capped":
        assert rec.capped and rec.k == 6
    if case == "wide":
        assert rec.chi_l < rec.chi_r
    assert abs(fid - rec.f) < 1e-12
    assert abs(rec.lnP - math.log(rec.f)) < 1e-12
    if not rec.capped:
        assert rec.f >= ft - 1e-12


def test_capped_circuit_bookkeeping_and_true_fidelity():
    """12 qubits, depth 10, chi <= 8, F_min 0.95, updates of >= 8 columns
    partial: the cap binds, so the partial path runs on the capped updates;
    ln P is the sum of ln f, uncapped updates meet their targets, and P is
    near the true fidelity (the product over many truncations is parity
    unpinned, as in the full mode: soft check)."""
    prog = C.brickwork_program(12, 10, 21)
    o = K.OracleTopK(12, "pure", chi_max=8, p=4, q=1, seed=1, topk_min=8).run(prog, 0.95)
    part = [r for r in o.log if hasattr(r, "subspace")]
    assert len(part) >= 10 and all(r.subspace == 12 for r in part)
    assert abs(o.lnP - sum(math.log(r.f) for r in o.log)) < 1e-12
    assert all(r.f >= r.f_t - 1e-12 for r in o.log if not r.capped)
    F = o.fidelity_estimate()[0]
    true = brute.fidelity_pure(brute.run_statevector(prog), o.to_statevector())
    assert abs(true - F) < 0.5 * (1 - F) + 0.05


@pytest.mark.parametrize("mistake", ["no_residual", "transpose", "right_vectors"])
@pytest.mark.parametrize("case", ["target", "wide"])
def test_planted_mistakes_fail_the_overlap_pin(mistake, case, monkeypatch):
    real = K.topk_factor

    def broken(X, *a, **kw):
        if mistake == "transpose":  # the conjugate dropped (Theta^T for Theta^H)
            return real(np.asarray(X).conj(), *a, **kw)
        res = real(X, *a, **kw)
        if res is None:
            return res
        if mistake == "no_residual":
            res.dec = K.truncation_rule_residual(res.s, 0.0, a[0], a[1], a[2])
        else:
            res.v = res.v.conj()
        return res

    monkeypatch.setattr(K, "topk_factor", broken)
    rec, fid, _ = _one_update(case)
    assert abs(fid - rec.f) > 1e-8
