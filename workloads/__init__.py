"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws random numbers and lays them out as plain arrays
(letter strings, gate lists, angles, coefficients).  It performs none of the
simulation method's arithmetic: no Pauli products, no frame updates, no
amplitude updates.  Both the CPU oracle and the HIP path consume its output and
each interprets it on its own.

Conventions (interface, not arithmetic):
  * A Pauli string is a row of ``n`` uint8 letter codes, column ``j`` = qubit ``j``:
    0 = I, 1 = X, 2 = Y, 3 = Z.
  * A Clifford gate is a row ``(code, q0, q1)`` of int32 with codes
    0 = H, 1 = S, 2 = S^dagger, 3 = X, 4 = Y, 5 = Z, 6 = CNOT(q0 -> q1),
    7 = CZ, 8 = SWAP; ``q1 = -1`` for one-qubit gates.  Circuits add the
    one-qubit rotations 9 = RX, 10 = RY, 11 = RZ (exp(-i theta/2 sigma_q)) with
    one angle per gate row.
  * Qubit ``j`` is bit ``j`` of a basis-state index (least significant bit =
    qubit 0), following the paper's computer-science bit order (Sec. 3).
"""
from .jw import (  # noqa: F401
    LETTER_I, LETTER_X, LETTER_Y, LETTER_Z,
    GATE_H, GATE_S, GATE_SDG, GATE_X, GATE_Y, GATE_Z, GATE_CNOT, GATE_CZ, GATE_SWAP,
    GATE_RX, GATE_RY, GATE_RZ,
    Workload, jw_strings, clifford_prefix, random_klocal_strings, make_workload,
    klocal_hamiltonian, staircase_circuit, klocal_trotter_circuit,
    config, batched_configs, letters_to_str, pauli_weight,
)
