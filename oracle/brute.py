"""Brute-force state-vector and density-matrix simulators and fidelities.

Test infrastructure only (see the package header).

* Pure states: the 2^N amplitude vector of Eq. (1), qubit 0 most significant.
* Mixed states: the 2^N x 2^N density matrix of Eq. (3).
* Fidelities: Eq. (7) |<psi|phi>|^2 (normalised) and Eq. (9), the
  alternative mixed-state fidelity |Tr(rho sigma)| / sqrt(Tr rho^2 Tr sigma^2).

Gates act directly on the dense objects (reshape to (2^i, 4, 2^(N-i-2)));
channels act by their Kraus/Pauli form, never through the superoperator
matrices handed to the MPS/MPO code, so these simulators also pin the
superoperator layout.
"""
from __future__ import annotations

import numpy as np

from circuits import pauli_matrices


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply_1q(psi: np.ndarray, n: int, i: int, g: np.ndarray) -> np.ndarray:
    v = psi.reshape(2 ** i, 2, 2 ** (n - i - 1))
    return np.einsum("st,atb->asb", g, v).reshape(-1)


def apply_2q(psi: np.ndarray, n: int, i: int, g: np.ndarray) -> np.ndarray:
    v = psi.reshape(2 ** i, 4, 2 ** (n - i - 2))
    return np.einsum("st,atb->asb", g, v).reshape(-1)


def run_statevector(program) -> np.ndarray:
    """Exact final state of a pure :class:`circuits.Program`."""
    n = program.n_sites
    psi = zero_state(n)
    for op in program.ops():
        psi = apply_1q(psi, n, op.site, op.mat) if op.width == 1 else \
            apply_2q(psi, n, op.site, op.mat)
    return psi


def _full_op(n: int, i: int, width: int, g: np.ndarray) -> np.ndarray:
    return np.kron(np.kron(np.eye(2 ** i), g), np.eye(2 ** (n - i - width)))


def apply_unitary_rho(rho, n, i, width, u):
    full = _full_op(n, i, width, u)
    return full @ rho @ full.conj().T


def apply_depolarizing2_rho(rho, n, i, p):
    """(1-p) rho + p/15 sum_{P != II} P rho P on qubits (i, i+1)."""
    paulis = pauli_matrices()
    out = (1.0 - p) * rho
    for a in range(4):
        for b in range(4):
            if a == 0 and b == 0:
                continue
            full = _full_op(n, i, 2, np.kron(paulis[a], paulis[b]))
            out = out + (p / 15.0) * (full @ rho @ full.conj().T)
    return out


def apply_depolarizing1_rho(rho, n, i, p):
    """(1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z) on qubit i."""
    paulis = pauli_matrices()
    out = (1.0 - p) * rho
    for a in range(1, 4):
        full = _full_op(n, i, 1, paulis[a])
        out = out + (p / 3.0) * (full @ rho @ full.conj().T)
    return out


def apply_kraus_rho(rho, n, i, width, kraus):
    """sum_K K rho K^dagger for Kraus operators on (i) or (i, i+1)."""
    out = np.zeros_like(rho)
    for k in kraus:
        full = _full_op(n, i, width, k)
        out = out + full @ rho @ full.conj().T
    return out


def run_density(n: int, gates) -> np.ndarray:
    """Exact final density matrix.  ``gates`` is a list of
    (site, width, unitary, depolarising_p) applied in order to |0><0|^n; the
    depolarising channel of the gate's width follows each gate with p > 0."""
    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    rho[0, 0] = 1.0
    for site, width, u, p in gates:
        rho = apply_unitary_rho(rho, n, site, width, u)
        if p:
            rho = apply_depolarizing2_rho(rho, n, site, p) if width == 2 else \
                apply_depolarizing1_rho(rho, n, site, p)
    return rho


def fidelity_pure(psi: np.ndarray, phi: np.ndarray) -> float:
    """Eq. (7), with both states normalised first."""
    ov = np.vdot(psi, phi)
    return float(abs(ov) ** 2 / (np.vdot(psi, psi).real * np.vdot(phi, phi).real))


def fidelity_wang(rho: np.ndarray, sigma: np.ndarray) -> float:
    """Eq. (9): |Tr(rho sigma)| / sqrt(Tr(rho^2) Tr(sigma^2))."""
    num = abs(np.trace(rho @ sigma))
    den = np.sqrt(abs(np.trace(rho @ rho)) * abs(np.trace(sigma @ sigma)))
    return float(num / den)


def expect_pure(psi: np.ndarray, n: int, site: int, width: int, op: np.ndarray) -> complex:
    opsi = apply_1q(psi, n, site, op) if width == 1 else apply_2q(psi, n, site, op)
    return complex(np.vdot(psi, opsi) / np.vdot(psi, psi))


def expect_rho(rho: np.ndarray, n: int, site: int, width: int, op: np.ndarray) -> complex:
    full = _full_op(n, site, width, op)
    return complex(np.trace(rho @ full) / np.trace(rho))
