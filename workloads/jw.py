"""Jordan-Wigner-shaped Pauli strings, random Clifford prefixes and the five
workload configurations of the rotation hot path.

The paper evaluates Trotterised chemistry Hamiltonians taken from a public
library in the Jordan-Wigner encoding (Sec. 5.3, Table of chemistry
Hamiltonians) and random k-local Hamiltonians (Sec. 5.2).  That library is not
available here, so these generators produce synthetic stand-ins with the same
structure: one-body strings X Z..Z X / Y Z..Z Y and two-body 4-index strings with
an even number of Y letters and Z fill between the index pairs.  At 24 qubits
the Pauli-weight statistics of these strings (mean about 11.6, std about 4.8)
are close to the ones the paper tabulates for its 24-qubit molecules.

Nothing here is simulation arithmetic; see the package docstring.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

LETTER_I, LETTER_X, LETTER_Y, LETTER_Z = 0, 1, 2, 3
GATE_H, GATE_S, GATE_SDG, GATE_X, GATE_Y, GATE_Z, GATE_CNOT, GATE_CZ, GATE_SWAP = range(9)
GATE_RX, GATE_RY, GATE_RZ = 9, 10, 11  # exp(-i theta/2 sigma_q), the angle beside the gate row

# The eight two-body letter patterns at (a, b, c, d) with an even number of Y.
_TWO_BODY_PATTERNS = np.array(
    [[1, 1, 1, 1], [1, 1, 2, 2], [1, 2, 1, 2], [1, 2, 2, 1],
     [2, 1, 1, 2], [2, 1, 2, 1], [2, 2, 1, 1], [2, 2, 2, 2]], dtype=np.uint8)


@dataclass
class Workload:
    """One seeded problem instance.

    ``prefix``   int32 (g, 3) Clifford gates applied before the rotations.
    ``rot``      uint8 (K, n) letter strings of the rotations, in circuit order.
    ``theta``    float64 (K,) rotation angles: R_k = exp(-i theta_k / 2 * P_k).
    ``ham``      uint8 (m, n) letter strings of the observable H.
    ``coeff``    float64 (m,) real coefficients of H.
    ``init``     basis-state index of the initial state.
    """
    name: str
    n: int
    init: int
    prefix: np.ndarray
    rot: np.ndarray
    theta: np.ndarray
    ham: np.ndarray
    coeff: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_rot(self) -> int:
        return int(self.rot.shape[0])


def letters_to_str(row: np.ndarray) -> str:
    """Human-readable form, qubit 0 first."""
    return "".join("IXYZ"[int(v)] for v in row)


def pauli_weight(rows: np.ndarray) -> np.ndarray:
    """Number of non-identity letters per row (the paper's locality measure)."""
    return (np.asarray(rows) != LETTER_I).sum(axis=-1)


def _one_body(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    out = np.zeros((m, n), dtype=np.uint8)
    for r in range(m):
        i, j = np.sort(rng.choice(n, size=2, replace=False))
        letter = LETTER_X if rng.integers(2) == 0 else LETTER_Y
        out[r, i] = letter
        out[r, j] = letter
        out[r, i + 1:j] = LETTER_Z
    return out


def _two_body(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    if n < 4:
        raise ValueError("two-body JW strings need n >= 4")
    out = np.zeros((m, n), dtype=np.uint8)
    for r in range(m):
        a, b, c, d = np.sort(rng.choice(n, size=4, replace=False))
        pat = _TWO_BODY_PATTERNS[rng.integers(8)]
        out[r, a + 1:b] = LETTER_Z
        out[r, c + 1:d] = LETTER_Z
        out[r, a], out[r, b], out[r, c], out[r, d] = pat
    return out


def jw_strings(rng: np.random.Generator, n: int, m: int, frac_one_body: float = 0.2) -> np.ndarray:
    """``m`` JW-shaped strings: exactly round(frac*m) one-body, the rest
    two-body, in a seeded random order.  Duplicates are allowed."""
    n1 = int(round(frac_one_body * m))
    n2 = m - n1
    rows = np.concatenate([_one_body(rng, n, n1), _two_body(rng, n, n2)], axis=0)
    perm = rng.permutation(m)
    return np.ascontiguousarray(rows[perm])


def random_klocal_strings(rng: np.random.Generator, n: int, k: int, m: int) -> np.ndarray:
    """``m`` distinct strings of weight exactly ``k`` with letters uniform in
    {X, Y, Z} on a uniformly drawn support (Sec. 5.2, random Hamiltonians)."""
    seen = set()
    out = []
    while len(out) < m:
        supp = np.sort(rng.choice(n, size=k, replace=False))
        row = np.zeros(n, dtype=np.uint8)
        row[supp] = rng.integers(1, 4, size=k)
        key = row.tobytes()
        if key in seen:
            continue
        seen.add(key)
        out.append(row)
    return np.stack(out)


def klocal_hamiltonian(n: int, k: int, n_terms: int, seed: int = 0):
    """Random k-local Hamiltonian of Sec. 5.2: ``n_terms`` distinct weight-k
    strings and real coefficients drawn uniformly from [0, 1), normalized to
    unit 2-norm.  Returns (letters, coeff)."""
    rng = np.random.default_rng(seed)
    letters = random_klocal_strings(rng, n, k, n_terms)
    c = rng.uniform(0.0, 1.0, size=n_terms)
    return letters, c / np.linalg.norm(c)


def staircase_circuit(letters: np.ndarray, theta: np.ndarray):
    """Gate rows for the rotations exp(-i theta_j/2 P_j), one after the other,
    each compiled as in Sec. 5.1 (Fig. cnot_ladder): a one-qubit basis change
    on every qubit of the support (H for X; S^dagger then H for Y), a CNOT
    staircase that gathers the parity of the support on its last qubit, RZ
    there, then the staircase and the basis changes undone.  Returns (gates,
    angles) with one angle per gate row (0 for Clifford rows)."""
    gates, angles = [], []
    for row, th in zip(np.asarray(letters, np.uint8), np.asarray(theta, np.float64)):
        supp = np.flatnonzero(row)
        if supp.size == 0:
            continue
        for q in supp:
            if row[q] == LETTER_X:
                gates.append((GATE_H, q, -1))
            elif row[q] == LETTER_Y:
                gates.append((GATE_SDG, q, -1))
                gates.append((GATE_H, q, -1))
        for a, b in zip(supp[:-1], supp[1:]):
            gates.append((GATE_CNOT, a, b))
        gates.append((GATE_RZ, supp[-1], -1))
        angles_here = len(gates) - 1
        for a, b in reversed(list(zip(supp[:-1], supp[1:]))):
            gates.append((GATE_CNOT, a, b))
        for q in supp:
            if row[q] == LETTER_X:
                gates.append((GATE_H, q, -1))
            elif row[q] == LETTER_Y:
                gates.append((GATE_H, q, -1))
                gates.append((GATE_S, q, -1))
        angles.extend([0.0] * (len(gates) - len(angles)))
        angles[angles_here] = float(th)
    return np.array(gates, np.int32).reshape(-1, 3), np.array(angles, np.float64)


def klocal_trotter_circuit(n: int, k: int, n_terms: int, seed: int = 0, t: float = 1.0, steps: int = 1):
    """The first-order Trotter circuit (Eq. trotter) of a random k-local
    Hamiltonian, compiled to H, S, S^dagger, CNOT and RZ rows: every step
    applies exp(-i c_j t/steps P_j) for j in order, i.e. theta_j = 2 c_j t /
    steps.  Returns (gates, angles, letters, coeff)."""
    letters, coeff = klocal_hamiltonian(n, k, n_terms, seed)
    th = 2.0 * coeff * t / steps
    g, a = staircase_circuit(np.tile(letters, (steps, 1)), np.tile(th, steps))
    return g, a, letters, coeff


def clifford_prefix(rng: np.random.Generator, n: int, g: int) -> np.ndarray:
    """``g`` gates uniform over {H, S, CNOT}; one-qubit targets uniform; CNOT on a
    uniformly drawn ordered pair of distinct qubits."""
    out = np.full((g, 3), -1, dtype=np.int32)
    for r in range(g):
        t = rng.integers(3)
        if t == 0:
            out[r] = (GATE_H, rng.integers(n), -1)
        elif t == 1:
            out[r] = (GATE_S, rng.integers(n), -1)
        else:
            c, tq = rng.choice(n, size=2, replace=False)
            out[r] = (GATE_CNOT, c, tq)
    return out


def make_workload(name: str, n: int, *, seed: int, n_prefix: int = 0, n_rot: int = 0,
                  n_ham: int = 0, theta: str = "uniform", coeff_sigma: float = 1.0,
                  dt: Optional[float] = None, trotter_steps: int = 1,
                  n_occupied: Optional[int] = None, frac_one_body: float = 0.2,
                  ham_is_rotations: bool = False) -> Workload:
    """Generic generator.  Draw order: prefix, rotation strings, angles or
    coefficients, observable.

    ``theta="uniform"``: theta ~ U[-pi, pi].  ``theta="trotter"``: one
    coefficient c_j ~ N(0, coeff_sigma^2) per string and theta_j = 2 dt c_j,
    repeated ``trotter_steps`` times in identical order; the observable is then
    the same strings with the same coefficients (``ham_is_rotations``).
    """
    rng = np.random.default_rng(seed)
    ne = n // 2 if n_occupied is None else n_occupied
    init = (1 << ne) - 1
    prefix = clifford_prefix(rng, n, n_prefix)
    base = jw_strings(rng, n, n_rot, frac_one_body) if n_rot else np.zeros((0, n), np.uint8)
    meta = {"seed": seed, "n_prefix": n_prefix, "trotter_steps": trotter_steps}
    if theta == "trotter":
        c = rng.normal(0.0, coeff_sigma, size=n_rot)
        th1 = 2.0 * dt * c
        rot = np.ascontiguousarray(np.tile(base, (trotter_steps, 1)))
        th = np.tile(th1, trotter_steps)
        meta.update(dt=dt, coeff_sigma=coeff_sigma)
        if ham_is_rotations:
            ham, coeff = base.copy(), c.copy()
        else:
            ham = jw_strings(rng, n, n_ham, frac_one_body) if n_ham else np.zeros((0, n), np.uint8)
            coeff = rng.normal(0.0, 1.0, size=n_ham)
    else:
        rot = base
        th = rng.uniform(-np.pi, np.pi, size=n_rot)
        ham = jw_strings(rng, n, n_ham, frac_one_body) if n_ham else np.zeros((0, n), np.uint8)
        coeff = rng.normal(0.0, coeff_sigma, size=n_ham)
    return Workload(name=name, n=n, init=init, prefix=prefix, rot=rot,
                    theta=np.ascontiguousarray(th, dtype=np.float64),
                    ham=np.ascontiguousarray(ham, dtype=np.uint8),
                    coeff=np.ascontiguousarray(coeff, dtype=np.float64), meta=meta)


def config(i: int, seed: int = 0, *, n: Optional[int] = None, n_rot: Optional[int] = None,
           n_ham: Optional[int] = None, trotter_steps: Optional[int] = None) -> Workload:
    """The five benchmark workloads (index 0..3; index 4 is ``batched_configs``).

    Keyword overrides shrink a configuration while keeping its recipe (used by
    tests that must finish in seconds).
      0: n=10, HF |1^5 0^5>, 50-gate Clifford prefix, 200 JW rotations, theta ~ U[-pi,pi];
         a 100-term observable with N(0,1) coefficients.
      1: n=24, 500-gate prefix, one Trotter step of 5,000 JW rotations, c ~ N(0, 0.1^2),
         dt = 0.1; observable = the same 5,000 terms.
      2: n=28, no prefix, 2,000 JW terms, c ~ N(0, 0.1^2), dt = 0.05, 10 Trotter steps
         (20,000 rotations); observable = the same 2,000 terms.
      3: n=20, 1,000 JW rotations theta ~ U[-pi,pi] on HF; H = 500 JW terms, c ~ N(0,1).
    """
    if i == 0:
        return make_workload("jw_n10_prefix50_r200", n or 10, seed=seed, n_prefix=50,
                             n_rot=n_rot or 200, n_ham=n_ham or 100, n_occupied=5)
    if i == 1:
        nn = n or 24
        return make_workload(f"jw_n{nn}_prefix500_trotter1", nn, seed=seed, n_prefix=500,
                             n_rot=n_rot or 5000, theta="trotter", coeff_sigma=0.1, dt=0.1,
                             trotter_steps=1, ham_is_rotations=True)
    if i == 2:
        nn = n or 28
        st = trotter_steps or 10
        return make_workload(f"jw_n{nn}_terms{n_rot or 2000}_trotter{st}", nn, seed=seed,
                             n_rot=n_rot or 2000, theta="trotter", coeff_sigma=0.1, dt=0.05,
                             trotter_steps=st, ham_is_rotations=True)
    if i == 3:
        nn = n or 20
        return make_workload(f"jw_n{nn}_ansatz{n_rot or 1000}", nn, seed=seed,
                             n_rot=n_rot or 1000, n_ham=n_ham or 500)
    raise ValueError(f"config {i}: use batched_configs() for the batched workload")


def batched_configs(seed: int = 0, count: int = 256, n_range=(12, 20), r_range=(500, 3000),
                    n_ham: int = 200) -> List[Workload]:
    """256 independent circuits: n ~ U{12..20}, R ~ U{500..3000} from the base
    seed; circuit i uses seed 1000 + i for its strings, theta ~ U[-pi, pi] and a
    200-term observable with N(0,1) coefficients; half-filling initial state."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    rs = rng.integers(r_range[0], r_range[1] + 1, size=count)
    return [make_workload(f"batch{i}", int(ns[i]), seed=1000 + i, n_rot=int(rs[i]), n_ham=n_ham)
            for i in range(count)]
