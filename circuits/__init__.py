"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *draws* inputs: random two-qubit unitaries, gate lists of
brickwork circuits, channel matrices handed to the simulator as its gate
operands, random site tensors and random angles.  It holds none of the
entanglement-aware update itself (no contraction, SVD, truncation or
fidelity bookkeeping), so the oracle and the GPU path can both read from it
without sharing any of the method's arithmetic.

Conventions used throughout the project
---------------------------------------
* Sites are 0-based; qubit 0 is the most significant bit of a state-vector
  index.
* A two-qubit operator on sites (i, i+1) is a 4x4 matrix indexed
  ``[2*s_i + s_{i+1}, 2*t_i + t_{i+1}]``.
* Mixed states are vectorised per site with ``p = 2*sigma + sigma'`` for
  ``|sigma><sigma'|`` (ket index major), so a one-site superoperator is 4x4
  and a two-site superoperator is 16x16 indexed ``[4*p_i + p_{i+1},
  4*q_i + q_{i+1}]``.
* The synthetic random circuits stand in for the paper's random circuits
  (Sec. VI, benchmarks of Figs. 1-4), whose exact definition the paper defers
  to another work: they keep its structure (Haar-random two-qubit gates,
  nearest-neighbour layout, product initial state).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

__all__ = [
    "haar_unitary", "brickwork_pairs", "Program", "Op", "brickwork_program",
    "unitary_superop", "depolarizing1_superop", "depolarizing2_superop", "pauli_matrices",
    "ry", "rz", "CZ", "hea_angles", "hea_program", "hea_hamiltonian",
    "random_mps_tensors", "config_program", "batched_programs", "noisy_program",
    "mirror_program",
]

# ---------------------------------------------------------------------------
# Single matrices
# ---------------------------------------------------------------------------


def haar_unitary(rng: np.random.Generator, n: int = 4) -> np.ndarray:
    """Haar-random n x n unitary (Mezzadri's QR recipe with phase fix).

    Z has i.i.d. standard complex Gaussian entries (real parts drawn first,
    then imaginary parts); Z = QR and U = Q diag(R_jj/|R_jj|).
    """
    re = rng.standard_normal((n, n))
    im = rng.standard_normal((n, n))
    z = (re + 1j * im) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def pauli_matrices() -> List[np.ndarray]:
    """[I, X, Y, Z] as complex128 2x2 arrays."""
    i2 = np.eye(2, dtype=np.complex128)
    x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    return [i2, x, y, z]


def ry(theta: float) -> np.ndarray:
    """RY(theta) = exp(-i theta Y / 2)."""
    c, s = np.cos(theta / 2.0), np.sin(theta / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(phi: float) -> np.ndarray:
    """RZ(phi) = exp(-i phi Z / 2)."""
    return np.array([[np.exp(-0.5j * phi), 0.0], [0.0, np.exp(0.5j * phi)]],
                    dtype=np.complex128)


CZ = np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128)


def unitary_superop(u: np.ndarray) -> np.ndarray:
    """Superoperator of rho -> U rho U^dagger in the site-interleaved layout.

    For a one-qubit U this is kron(U, conj(U)) indexed [2s+s', 2t+t'].  For a
    two-qubit U the rows/columns are re-ordered from (s1 s2 s1' s2') to
    (s1 s1' s2 s2').
    """
    u = np.asarray(u, dtype=np.complex128)
    k = np.kron(u, u.conj())
    if u.shape == (2, 2):
        return k
    assert u.shape == (4, 4)
    k = k.reshape(2, 2, 2, 2, 2, 2, 2, 2)  # s1 s2 s1' s2' | t1 t2 t1' t2'
    k = k.transpose(0, 2, 1, 3, 4, 6, 5, 7)
    return k.reshape(16, 16)


def depolarizing1_superop(p: float) -> np.ndarray:
    """One-qubit depolarising channel in Pauli form, as a 4x4 superoperator.

    rho -> (1-p) rho + p/3 * (X rho X + Y rho Y + Z rho Z), the one-qubit
    counterpart of :func:`depolarizing2_superop` (the paper names the noise
    parameters of one- and two-qubit gates without a formula).
    """
    paulis = pauli_matrices()
    s = (1.0 - p) * np.eye(4, dtype=np.complex128)
    for a in range(1, 4):
        s = s + (p / 3.0) * unitary_superop(paulis[a])
    return s


def depolarizing2_superop(p: float) -> np.ndarray:
    """Two-qubit depolarising channel in Pauli form, as a 16x16 superoperator.

    rho -> (1-p) rho + p/15 * sum over the 15 non-identity two-qubit Paulis P
    of P rho P.  (The paper names depolarising noise without a formula; this
    is the reading used for the noisy mixed-state workload.)
    """
    paulis = pauli_matrices()
    s = (1.0 - p) * np.eye(16, dtype=np.complex128)
    for a in range(4):
        for b in range(4):
            if a == 0 and b == 0:
                continue
            s = s + (p / 15.0) * unitary_superop(np.kron(paulis[a], paulis[b]))
    return s


# ---------------------------------------------------------------------------
# Programs
# ---------------------------------------------------------------------------


@dataclass
class Op:
    """One gate: ``width`` 1 or 2, acting on (site) or (site, site+1)."""
    width: int
    site: int
    mat: np.ndarray
    tag: str = ""


@dataclass
class Program:
    """A circuit as a list of layers; each layer is a list of :class:`Op`.

    Two-qubit ops inside one layer act on disjoint pairs.
    """
    n_sites: int
    kind: str  # "pure" (d=2) or "mixed" (d=4)
    layers: List[List[Op]] = field(default_factory=list)
    # noisy programs: the unitaries and noise strengths behind the fused
    # operands, as (site, width, U, p) in program order
    units: list = field(default_factory=list)

    @property
    def n_2q(self) -> int:
        return sum(1 for layer in self.layers for op in layer if op.width == 2)

    def ops(self):
        for layer in self.layers:
            for op in layer:
                yield op


def brickwork_pairs(n_sites: int, layer: int) -> List[int]:
    """Left sites of the pairs of brickwork sub-layer ``layer``.

    Sub-layer t uses pairs (t mod 2 + 2j, t mod 2 + 2j + 1).
    """
    start = layer % 2
    return list(range(start, n_sites - 1, 2))


def brickwork_program(n_sites: int, depth: int, seed, kind: str = "pure",
                      noise_p: float = 0.0) -> Program:
    """Brickwork circuit of Haar-random U(4) gates.

    Gates are drawn in program order (layer, then pair left to right) from
    ``numpy.random.default_rng(seed)``.  For ``kind == "mixed"`` each gate is
    handed over as its 16x16 superoperator, followed (fused, one operand) by
    the two-qubit depolarising channel of strength ``noise_p``.
    """
    rng = np.random.default_rng(seed)
    prog = Program(n_sites=n_sites, kind=kind)
    dep = depolarizing2_superop(noise_p) if (kind == "mixed" and noise_p > 0) else None
    for t in range(depth):
        layer = []
        for i in brickwork_pairs(n_sites, t):
            u = haar_unitary(rng, 4)
            if kind == "mixed":
                m = unitary_superop(u)
                if dep is not None:
                    m = dep @ m
            else:
                m = u
            layer.append(Op(2, i, m, "haar"))
        prog.layers.append(layer)
    return prog


def noisy_program(n_sites: int, depth: int, seed, eps1: float, eps2: float) -> Program:
    """Noisy mixed-state circuit with one- and two-qubit noise.

    Each layer t first applies a Haar-random one-qubit unitary to every site,
    each followed (fused, one 4x4 operand) by the one-qubit depolarising
    channel of strength ``eps1``, then Haar-random two-qubit gates on the
    brickwork pairs of sub-layer t, each followed (fused, one 16x16 operand) by
    the two-qubit depolarising channel of strength ``eps2``.  Gates are drawn
    in program order from ``numpy.random.default_rng(seed)``.  The unitaries
    and strengths behind the fused operands are listed in ``Program.units``
    as (site, width, U, p), for references that apply the channels directly.
    """
    rng = np.random.default_rng(seed)
    prog = Program(n_sites=n_sites, kind="mixed")
    dep1 = depolarizing1_superop(eps1)
    dep2 = depolarizing2_superop(eps2)
    units = []
    for t in range(depth):
        layer = []
        for q in range(n_sites):
            u = haar_unitary(rng, 2)
            layer.append(Op(1, q, dep1 @ unitary_superop(u), "haar1+dep1"))
            units.append((q, 1, u, eps1))
        for i in brickwork_pairs(n_sites, t):
            u = haar_unitary(rng, 4)
            layer.append(Op(2, i, dep2 @ unitary_superop(u), "haar+dep2"))
            units.append((i, 2, u, eps2))
        prog.layers.append(layer)
    prog.units = units
    return prog


def mirror_program(n_sites: int, depth: int, seed) -> Program:
    """A brickwork Haar circuit of ``depth`` sub-layers followed by its
    adjoint: the same layers in reverse order with every gate replaced by its
    conjugate transpose, so the whole circuit is the identity."""
    fwd = brickwork_program(n_sites, depth, seed)
    prog = Program(n_sites=n_sites, kind="pure")
    prog.layers = [list(layer) for layer in fwd.layers]
    for layer in reversed(fwd.layers):
        prog.layers.append([Op(2, op.site, op.mat.conj().T.copy(), "haar-adjoint")
                            for op in layer])
    return prog


def hea_angles(n_qubits: int = 32, n_layers: int = 10, seed=5) -> np.ndarray:
    """Angles of the hardware-efficient ansatz, shape (layers, qubits, 2),
    uniform in [0, 2 pi): [..., 0] = RY angle, [..., 1] = RZ angle."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * np.pi, size=(n_layers, n_qubits, 2))


def hea_program(angles: np.ndarray) -> Program:
    """Per layer: RY then RZ on every qubit, then CZ on brickwork pairs."""
    n_layers, n_qubits, _ = angles.shape
    prog = Program(n_sites=n_qubits, kind="pure")
    for l in range(n_layers):
        layer = []
        for q in range(n_qubits):
            layer.append(Op(1, q, ry(angles[l, q, 0]), f"ry:{l}:{q}"))
            layer.append(Op(1, q, rz(angles[l, q, 1]), f"rz:{l}:{q}"))
        for i in brickwork_pairs(n_qubits, l):
            layer.append(Op(2, i, CZ.copy(), "cz"))
        prog.layers.append(layer)
    return prog


def hea_hamiltonian(n_qubits: int = 32, hx: float = 0.5):
    """Terms of H = sum_i Z_i Z_{i+1} + hx * sum_i X_i on an open chain, as a
    list of (site, width, matrix, coefficient)."""
    _, x, _, z = pauli_matrices()
    terms = []
    for i in range(n_qubits - 1):
        terms.append((i, 2, np.kron(z, z), 1.0))
    for i in range(n_qubits):
        terms.append((i, 1, x.copy(), hx))
    return terms


# ---------------------------------------------------------------------------
# Random states (for single-update tests at full size)
# ---------------------------------------------------------------------------


def random_mps_tensors(bond_dims, d: int, seed) -> List[np.ndarray]:
    """Random complex Gaussian site tensors for the given bond profile.

    ``bond_dims`` has length n_sites + 1 with both ends equal to 1; site i gets
    shape (bond_dims[i], d, bond_dims[i+1]).  Entries are scaled by
    1/sqrt(size) so every tensor has unit expected Frobenius norm.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(len(bond_dims) - 1):
        shp = (bond_dims[i], d, bond_dims[i + 1])
        a = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
        out.append(a / np.sqrt(2.0 * a.size))
    return out


# ---------------------------------------------------------------------------
# The five benchmark workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    1: dict(n=12, depth=8, kind="pure", f_min=1.0, chi_max=64, seed=1),
    2: dict(n=50, depth=20, kind="pure", f_min=0.99, chi_max=1024, seed=2),
    3: dict(n=40, depth=30, kind="mixed", f_min=0.95, chi_max=1024, seed=3, noise_p=1e-3),
}


def config_program(cfg: int, **over) -> Tuple[Program, dict]:
    """Program and parameters of benchmark workload ``cfg`` (1, 2 or 3)."""
    c = dict(CONFIGS[cfg])
    c.update(over)
    prog = brickwork_program(c["n"], c["depth"], c["seed"], kind=c["kind"],
                             noise_p=c.get("noise_p", 0.0))
    return prog, c


def batched_programs(n_circuits: int = 64, seed: int = 4, n_range=(20, 80),
                     depth_range=(10, 40)) -> List[Program]:
    """Independent brickwork circuits with random sizes and depths.

    Circuit c draws N_c ~ U{n_range} and D_c ~ U{depth_range} (inclusive) and
    then its gates, all from the c-th child of SeedSequence(seed).
    """
    children = np.random.SeedSequence(seed).spawn(n_circuits)
    progs = []
    for ch in children:
        rng = np.random.default_rng(ch)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        dep = int(rng.integers(depth_range[0], depth_range[1] + 1))
        sub = int(rng.integers(0, 2**62))
        progs.append(brickwork_program(n, dep, sub))
    return progs
