"""Pins of the layer-parallel (Vidal gauge, Hastings update) oracle mode,
CPU only: exactness without truncation against brute force (amplitudes,
Schmidt values of every bond, right-normalised tensors), the first truncation
of an exact form against the brute-force overlap (Eq. 10), closed forms (GHZ),
the per-layer targets, and planted mistakes.  The product of truncation
fidelities over many truncations is parity unpinned here as in the exact
mode (soft check only)."""
import math

import numpy as np
import pytest

import circuits as C
from oracle import brute
from oracle.vidal import OracleVidal
from oracle.mps import OracleMPS

H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)


def _schmidt(psi, n, cut):
    s = np.linalg.svd(psi.reshape(2 ** cut, -1), compute_uv=False)
    return s[s > 1e-12 * s[0]]


def test_exact_without_truncation():
    """12 qubits, depth 8, F_min = 1: amplitudes, every bond's Lambda equal to
    the exact Schmidt values, right-normalised B, P = 1."""
    prog, _ = C.config_program(1)
    o = OracleVidal(prog.n_sites, "pure").run(prog, 1.0)
    psi = brute.run_statevector(prog)
    np.testing.assert_allclose(o.to_statevector(), psi, atol=1e-12)
    for cut in range(1, prog.n_sites):
        ref = _schmidt(psi, prog.n_sites, cut)
        lam = o.lam[cut][o.lam[cut] > 1e-12 * o.lam[cut][0]]
        np.testing.assert_allclose(lam, ref, atol=1e-12)
    assert o.right_normalisation_error() < 1e-12
    assert abs(o.fidelity_estimate()[0] - 1.0) < 1e-14


def test_equals_exact_centre_mode_without_truncation():
    prog = C.brickwork_program(10, 7, 3)
    a = OracleVidal(10, "pure").run(prog, 1.0).to_statevector()
    b = OracleMPS(10, "pure").run(prog, 1.0).to_statevector()
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_first_truncation_of_an_exact_form_is_eq10():
    """Exact layers, then one layer whose middle gate truncates to f_t = 0.9:
    f = |<psi_exact|psi_trunc>|^2 (renormalised), to 1e-12."""
    n = 10
    prog = C.brickwork_program(n, 7, 5)
    o = OracleVidal(n, "pure")
    for layer in prog.layers[:-1]:
        o.apply_layer(layer, budgets=[1.0] * len(layer))
    last = prog.layers[-1]
    mid = len(last) // 2
    budgets = [1.0] * len(last)
    budgets[mid] = 0.9
    recs = o.apply_layer(last, budgets=budgets)
    rec = [r for r in recs if r.site == last[mid].site][0]
    assert rec.k < min(rec.chi_l, rec.chi_r) * 2  # it truncated
    psi = brute.run_statevector(prog)
    phi = o.to_statevector()
    fid = abs(np.vdot(psi, phi)) ** 2 / (np.vdot(phi, phi).real * np.vdot(psi, psi).real)
    assert abs(fid - rec.f) < 1e-12
    assert abs(math.exp(o.lnP) - rec.f) < 1e-12


def test_ghz_lambdas():
    n = 8
    o = OracleVidal(n, "pure")
    o.apply_1q(0, H)
    for i in range(n - 1):
        o.apply_2q(i, CNOT, 1.0)
    for b in range(1, n):
        np.testing.assert_allclose(o.lam[b], [2 ** -0.5, 2 ** -0.5], atol=1e-14)
    ref = np.zeros(2 ** n, complex)
    ref[0] = ref[-1] = 2 ** -0.5
    np.testing.assert_allclose(o.to_statevector(), ref, atol=1e-14)


def test_layer_targets_from_the_estimate_before_the_layer():
    prog = C.brickwork_program(12, 10, 9)
    o = OracleVidal(12, "pure")
    o.set_schedule(0.95, prog.n_2q)
    for layer in prog.layers:
        g0, lnP0 = o.g, o.lnP
        recs = o.apply_layer(layer)
        want = min(1.0, math.exp((math.log(0.95) - lnP0) / (prog.n_2q - g0)))
        assert all(abs(r.f_t - want) < 1e-15 for r in recs)
    F = o.fidelity_estimate()[0]
    assert F >= 0.95 * (1 - 1e-12)  # the F_min guarantee holds layer by layer
    # soft: the estimate against the true fidelity after many truncations
    psi = brute.run_statevector(prog)
    true = brute.fidelity_pure(psi, o.to_statevector())
    assert abs(true - F) < 0.5 * (1 - F) + 0.05


def test_mixed_state_without_truncation_is_exact():
    prog = C.brickwork_program(5, 4, 8, kind="mixed", noise_p=1e-2)
    o = OracleVidal(5, "mixed").run(prog, 1.0)
    rho = brute.run_density(5, prog.units) if prog.units else None
    ref = OracleMPS(5, "mixed").run(prog, 1.0)
    np.testing.assert_allclose(o.to_density(), ref.to_density(), atol=1e-12)
    assert rho is None or np.abs(o.to_density() - rho).max() < 1e-12


@pytest.mark.parametrize("mistake", ["no_lambda", "left_vectors"])
def test_planted_mistakes_are_caught(mistake, monkeypatch):
    """Forgetting Lambda_i in Theta, or building B_i from X S instead of
    C Y_k, must fail the exact-form pins."""
    import oracle.vidal as V
    real = V.OracleVidal.apply_2q

    def broken(self, i, G, f_t=None, direction="right", forced_k=None):
        if mistake == "no_lambda":
            saved = self.lam[i]
            self.lam[i] = np.ones_like(saved)
            rec = real(self, i, G, f_t, direction, forced_k)
            return rec
        rec = real(self, i, G, f_t, direction, forced_k)
        b = self.A[i]
        self.A[i] = b * np.repeat(self.lam[i], self.d).reshape(b.shape[0], self.d, 1)
        return rec

    monkeypatch.setattr(V.OracleVidal, "apply_2q", broken)
    prog, _ = C.config_program(1)
    o = OracleVidal(prog.n_sites, "pure").run(prog, 1.0)
    psi = brute.run_statevector(prog)
    bad_amp = np.abs(o.to_statevector() - psi).max() > 1e-6
    bad_lam = any(
        np.abs(np.sort(o.lam[c])[::-1][: len(_schmidt(psi, prog.n_sites, c))]
               - _schmidt(psi, prog.n_sites, c)).max() > 1e-6 if len(o.lam[c]) >= len(
            _schmidt(psi, prog.n_sites, c)) else True
        for c in range(1, prog.n_sites))
    assert bad_amp or bad_lam
