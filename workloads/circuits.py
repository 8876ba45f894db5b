"""Seeded random quantum circuits and their tensor networks.

The circuits follow the random-circuit family the paper verifies on (a
Sycamore-style circuit: single-qubit gates drawn from {sqrt X, sqrt Y, sqrt W}
and two-qubit fSim gates on a 2D grid, Section V).  The exact Sycamore circuit
files are not used: circuits here are synthetic stand-ins drawn from a seed.

Conventions (the paper leaves them open):
  * qubit q sits at row q // cols, column q % cols of the grid;
  * qubit 0 is the most significant bit of a basis-state index;
  * a cycle is a layer of single-qubit gates on every qubit followed by fSim
    gates on coupler pattern (cycle mod 4): 0 = horizontal pairs starting at an
    even column, 1 = horizontal pairs starting at an odd column, 2 = vertical
    pairs starting at an even row, 3 = vertical pairs starting at an odd row;
    one more single-qubit layer closes the circuit;
  * a two-qubit gate on (a, b) has matrix index 2*bit_a + bit_b.

Tensor networks (Section II.A): a wire segment is a bond label; the initial
state of each qubit is the vector |0>, a one-qubit gate is the rank-2 tensor
T[out, in] = M[out, in], a two-qubit gate the rank-4 tensor
T[oa, ob, ia, ib] = M[2*oa + ob, 2*ia + ib], and an amplitude <x|U|0> closes
each wire with the basis vector e_{x_q}.  This module builds these tensors by
copying matrix entries; it performs no contraction.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .rng import SplitMix64

_S2 = 1.0 / math.sqrt(2.0)

SQRT_X = _S2 * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)
SQRT_Y = _S2 * np.array([[1, -1], [1, 1]], dtype=np.complex128)
SQRT_W = _S2 * np.array([[1, -np.exp(1j * math.pi / 4)],
                         [np.exp(-1j * math.pi / 4), 1]], dtype=np.complex128)
HADAMARD = _S2 * np.array([[1, 1], [1, -1]], dtype=np.complex128)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                dtype=np.complex128)
ONE_QUBIT_SET = (SQRT_X, SQRT_Y, SQRT_W)


def fsim(theta: float, phi: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1
    m[1, 1] = c
    m[1, 2] = -1j * s
    m[2, 1] = -1j * s
    m[2, 2] = c
    m[3, 3] = np.exp(-1j * phi)
    return m


FSIM = fsim(math.pi / 2, math.pi / 6)


@dataclass
class Gate:
    qubits: tuple
    matrix: np.ndarray  # 2x2 or 4x4 complex128


@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)


def grid_shape(n_sites: int) -> tuple[int, int]:
    """Columns = ceil(sqrt(n)), rows as needed; the last row may be partial."""
    cols = int(math.ceil(math.sqrt(n_sites)))
    rows = (n_sites + cols - 1) // cols
    return rows, cols


def coupler_pairs(rows: int, cols: int, pattern: int, n_sites: int | None = None):
    n_sites = rows * cols if n_sites is None else n_sites
    pairs = []
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            if q >= n_sites:
                continue
            if pattern in (0, 1) and c % 2 == pattern and c + 1 < cols:
                p = q + 1
            elif pattern in (2, 3) and r % 2 == pattern - 2 and r + 1 < rows:
                p = q + cols
            else:
                continue
            if p < n_sites:
                pairs.append((q, p))
    return pairs


def random_circuit(rows: int, cols: int, cycles: int, seed: int,
                   n_sites: int | None = None) -> Circuit:
    n = rows * cols if n_sites is None else n_sites
    rng = SplitMix64(seed)
    circ = Circuit(n)
    for t in range(cycles):
        for q in range(n):
            circ.gates.append(Gate((q,), ONE_QUBIT_SET[rng.below(3)]))
        for a, b in coupler_pairs(rows, cols, t % 4, n):
            circ.gates.append(Gate((a, b), FSIM))
    for q in range(n):
        circ.gates.append(Gate((q,), ONE_QUBIT_SET[rng.below(3)]))
    return circ


def ghz_circuit(n: int) -> Circuit:
    circ = Circuit(n)
    circ.gates.append(Gate((0,), HADAMARD))
    for q in range(n - 1):
        circ.gates.append(Gate((q, q + 1), CNOT))
    return circ


def random_bitstring(n: int, seed: int) -> list[int]:
    rng = SplitMix64(seed)
    return [rng.below(2) for _ in range(n)]


@dataclass
class Network:
    """Tensors with integer bond labels.  Every label of dimension 2.

    tensors[i] is a complex128 ndarray whose axis j carries labels[i][j].
    A label shared by two tensors is a bond; a label carried once is open.
    """
    tensors: list
    labels: list
    open_labels: list = field(default_factory=list)

    def copy(self) -> "Network":
        return Network([t.copy() for t in self.tensors],
                       [list(l) for l in self.labels], list(self.open_labels))


def circuit_network(circ: Circuit, bitstring: list[int] | None) -> Network:
    """Tensor network of <x|U|0> (bitstring given) or of U|0> (open legs).

    With open legs the network's open labels are listed in qubit order.
    """
    tensors, labels = [], []
    next_label = 0
    wire = []
    for _ in range(circ.n):
        tensors.append(np.array([1.0, 0.0], dtype=np.complex128))
        labels.append([next_label])
        wire.append(next_label)
        next_label += 1
    for g in circ.gates:
        if len(g.qubits) == 1:
            (q,) = g.qubits
            tensors.append(np.array(g.matrix, dtype=np.complex128).reshape(2, 2).copy())
            labels.append([next_label, wire[q]])
            wire[q] = next_label
            next_label += 1
        else:
            a, b = g.qubits
            tensors.append(np.array(g.matrix, dtype=np.complex128).reshape(2, 2, 2, 2).copy())
            labels.append([next_label, next_label + 1, wire[a], wire[b]])
            wire[a], wire[b] = next_label, next_label + 1
            next_label += 2
    open_labels = []
    if bitstring is None:
        open_labels = list(wire)
    else:
        for q in range(circ.n):
            v = np.zeros(2, dtype=np.complex128)
            v[bitstring[q]] = 1.0
            tensors.append(v)
            labels.append([wire[q]])
    return Network(tensors, labels, open_labels)
