"""ctypes front end of the C oracle (``cfh_oracle.c``).  Test infrastructure.

The physical circuit of a workload is: the initial basis state, the Clifford
prefix C as explicit gates, then R_k = exp(-i theta_k/2 P_k) for k = 1..K in
order (Sec. 4.2: the hybrid simulator reaches exactly this state).  The hybrid
representation keeps Phi = C^dag psi next to a frame for C (Eq. cfhsstate), so
``simulate`` returns both psi and Phi_ref = C^dag psi.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        # CFH_ORACLE_LIB selects another build of the oracle (the host sanitizer run uses one)
        path = os.environ.get("CFH_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.orc_apply_gate.argtypes = [_c128p, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_apply_gates.argtypes = [_c128p, C.c_int, _i32p, C.c_int64, C.c_int]
        L.orc_rotation_ladder.argtypes = [_c128p, C.c_int, _u8p, C.c_int, C.c_double]
        L.orc_rotations_ladder.argtypes = [_c128p, C.c_int, _u8p, C.c_void_p, _f64p, C.c_int64]
        L.orc_heisenberg.argtypes = [_i32p, C.c_int64, _u8p, C.c_int, C.POINTER(C.c_int)]
        L.orc_conj_table1.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.orc_expval.argtypes = [_c128p, C.c_int, _u8p, C.c_int, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]
        L.orc_energy.argtypes = [_c128p, C.c_int, _u8p, C.c_void_p, _f64p, C.c_int64]
        L.orc_energy.restype = C.c_double
        L.orc_apply_pauli_sum.argtypes = [_c128p, C.c_int, _u8p, C.c_void_p, _f64p, C.c_int64, _c128p]
        L.orc_sparse_rotations.argtypes = [C.c_int, _u64p, _c128p, C.c_int64, _u8p, C.c_void_p,
                                           _f64p, C.c_int64, _u64p, _c128p, C.c_int64]
        L.orc_sparse_rotations.restype = C.c_int64
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _LIB = L
    return _LIB


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Threads the oracle's parallel loops use from now on (k >= 1)."""
    lib().orc_set_num_threads(int(k))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} failed ({rc})")


def basis_state(n: int, index: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def apply_gate(psi: np.ndarray, n: int, g: int, q0: int, q1: int = -1) -> None:
    _check(lib().orc_apply_gate(psi, n, g, q0, q1), "apply_gate")


def apply_gates(psi: np.ndarray, n: int, gates: np.ndarray, inverse: bool = False) -> None:
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 3)
    _check(lib().orc_apply_gates(psi, n, g, g.shape[0], int(inverse)), "apply_gates")


def measure_z(psi: np.ndarray, n: int, q: int, u: float) -> Tuple[int, float]:
    """In place: measure Z_q with the uniform number u (outcome +1 when
    u < P(+1)), then collapse and renormalize.  Returns (outcome, P(+1))."""
    bit = (np.arange(1 << n, dtype=np.int64) >> q) & 1
    p_plus = float(np.sum(np.abs(psi[bit == 0]) ** 2))
    s = 1 if u < p_plus else -1
    keep = bit == (0 if s > 0 else 1)
    psi[~keep] = 0.0
    psi /= np.sqrt(p_plus if s > 0 else 1.0 - p_plus)
    return s, p_plus


def measure_pauli(psi: np.ndarray, n: int, letters: np.ndarray, u: float, phase: int = 0) -> Tuple[int, float]:
    """In place: measure the Hermitian i^phase P with the uniform number u:
    P(+1) = (1 + <P>)/2, psi <- (psi + s P psi) / (2 sqrt(P(s)))."""
    p_plus = min(1.0, max(0.0, 0.5 * (1.0 + expval(psi, n, letters, phase).real)))
    s = 1 if u < p_plus else -1
    ps = p_plus if s > 0 else 1.0 - p_plus
    ppsi = apply_pauli_sum(psi, n, np.asarray(letters, np.uint8).reshape(1, n), np.array([1.0]),
                           np.array([phase]))
    psi[:] = (psi + s * ppsi) / (2.0 * np.sqrt(ps))
    return s, p_plus


def apply_circuit(psi: np.ndarray, n: int, gates: np.ndarray, angles: np.ndarray,
                  probs: Optional[list] = None) -> np.ndarray:
    """In place, gate by gate: Clifford rows as apply_gate, rows 9/10/11 as the
    one-qubit rotations exp(-i theta/2 X_q / Y_q / Z_q), row 12 a Z_q
    measurement and row 13 a reset to |0> (measure, then X_q on -1), both with
    the row's angle as their uniform number (the gate-level simulation a
    circuit simulator performs, with no frame).  Returns the outcomes (+1/-1
    at measurement and reset rows, else 0); ``probs``, if given, receives the
    probability P(s) of each outcome drawn, in row order."""
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(g.shape[0], np.int32)
    for i, ((code, q0, q1), th) in enumerate(zip(g, np.asarray(angles, np.float64))):
        if code in (9, 10, 11):
            letters = np.zeros(n, np.uint8)
            letters[q0] = {9: 1, 10: 2, 11: 3}[int(code)]
            rotation(psi, n, letters, float(th))
        elif code in (12, 13):
            out[i], p_plus = measure_z(psi, n, int(q0), float(th))
            if probs is not None:
                probs.append(p_plus if out[i] > 0 else 1.0 - p_plus)
            if code == 13 and out[i] < 0:
                apply_gate(psi, n, 3, int(q0), -1)
        else:
            apply_gate(psi, n, int(code), int(q0), int(q1))
    return out


def rotation(psi: np.ndarray, n: int, letters: np.ndarray, theta: float, sign: int = 1) -> None:
    """In place: psi <- exp(-i theta/2 * sign * P) psi via basis change, CNOT ladder, RZ."""
    l = np.ascontiguousarray(letters, dtype=np.uint8)
    _check(lib().orc_rotation_ladder(psi, n, l, int(sign), float(theta)), "rotation")


def rotations(psi: np.ndarray, n: int, letters: np.ndarray, theta: np.ndarray,
              signs: Optional[np.ndarray] = None) -> None:
    l = np.ascontiguousarray(letters, dtype=np.uint8).reshape(-1, n)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    sp = None
    if signs is not None:
        s = np.ascontiguousarray(signs, dtype=np.int32)
        sp = s.ctypes.data
    _check(lib().orc_rotations_ladder(psi, n, l, sp, th, l.shape[0]), "rotations")


def heisenberg(gates: np.ndarray, letters: np.ndarray, phase: int = 0) -> Tuple[np.ndarray, int]:
    """C^dag Q C for Q = i^phase * letters, C the gate list (first row acts first)."""
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 3)
    l = np.array(letters, dtype=np.uint8, copy=True)
    ph = C.c_int(phase)
    _check(lib().orc_heisenberg(g, g.shape[0], l, l.shape[0], C.byref(ph)), "heisenberg")
    return l, int(ph.value)


def heisenberg_many(gates: np.ndarray, rows: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    rows = np.asarray(rows, dtype=np.uint8)
    out = np.empty_like(rows)
    ph = np.empty(rows.shape[0], dtype=np.int32)
    for i in range(rows.shape[0]):
        out[i], ph[i] = heisenberg(gates, rows[i])
    return out, ph


def frame_rows(gates: np.ndarray, n: int):
    """Backward-interpretation frame of C: effZ_q = C^dag Z_q C, effX_q = C^dag X_q C.
    Returns (zl, zph, xl, xph): letters (n, n) and phases (n,)."""
    zl = np.zeros((n, n), np.uint8)
    xl = np.zeros((n, n), np.uint8)
    zph = np.zeros(n, np.int32)
    xph = np.zeros(n, np.int32)
    for q in range(n):
        z = np.zeros(n, np.uint8)
        z[q] = 3
        x = np.zeros(n, np.uint8)
        x[q] = 1
        zl[q], zph[q] = heisenberg(gates, z)
        xl[q], xph[q] = heisenberg(gates, x)
    return zl, zph, xl, xph


def expval(psi: np.ndarray, n: int, letters: np.ndarray, phase: int = 0) -> complex:
    re, im = C.c_double(), C.c_double()
    l = np.ascontiguousarray(letters, dtype=np.uint8)
    _check(lib().orc_expval(psi, n, l, int(phase), C.byref(re), C.byref(im)), "expval")
    return complex(re.value, im.value)


def energy(psi: np.ndarray, n: int, ham: np.ndarray, coeff: np.ndarray,
           phases: Optional[np.ndarray] = None) -> float:
    h = np.ascontiguousarray(ham, dtype=np.uint8).reshape(-1, n)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    pp = None
    if phases is not None:
        p = np.ascontiguousarray(phases, dtype=np.int32)
        pp = p.ctypes.data
    return float(lib().orc_energy(psi, n, h, pp, c, h.shape[0]))


def apply_pauli_sum(psi: np.ndarray, n: int, ham: np.ndarray, coeff: np.ndarray,
                    phases: Optional[np.ndarray] = None) -> np.ndarray:
    """H psi with H = sum_j coeff_j i^phase_j P_j, letter by letter."""
    h = np.ascontiguousarray(ham, dtype=np.uint8).reshape(-1, n)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    pp = None
    if phases is not None:
        p = np.ascontiguousarray(phases, dtype=np.int32)
        pp = p.ctypes.data
    out = np.empty_like(psi)
    _check(lib().orc_apply_pauli_sum(psi, n, h, pp, c, h.shape[0], out), "apply_pauli_sum")
    return out


def simulate(w, n_rot: Optional[int] = None, theta: Optional[np.ndarray] = None):
    """Physical psi = R_K..R_1 C |init> and Phi_ref = C^dag psi."""
    K = w.n_rot if n_rot is None else n_rot
    th = w.theta[:K] if theta is None else np.asarray(theta, np.float64)[:K]
    psi = basis_state(w.n, w.init)
    apply_gates(psi, w.n, w.prefix)
    rotations(psi, w.n, w.rot[:K], th)
    phi = psi.copy()
    apply_gates(phi, w.n, w.prefix, inverse=True)
    return psi, phi


def energy_of(w, theta: np.ndarray, n_rot: Optional[int] = None) -> float:
    psi, _ = simulate(w, n_rot, theta)
    return energy(psi, w.n, w.ham, w.coeff)


def param_shift_grad(w, indices: Optional[Sequence[int]] = None) -> np.ndarray:
    """Two-term parameter-shift rule, exact because P_k^2 = I:
    dE/dtheta_k = [E(theta + pi/2 e_k) - E(theta - pi/2 e_k)] / 2."""
    idx = range(w.n_rot) if indices is None else indices
    out = []
    for k in idx:
        tp = w.theta.copy()
        tm = w.theta.copy()
        tp[k] += np.pi / 2
        tm[k] -= np.pi / 2
        out.append(0.5 * (energy_of(w, tp) - energy_of(w, tm)))
    return np.array(out)


def finite_diff_grad(w, h: float = 1e-6, indices: Optional[Sequence[int]] = None) -> np.ndarray:
    idx = range(w.n_rot) if indices is None else indices
    out = []
    for k in idx:
        tp = w.theta.copy()
        tm = w.theta.copy()
        tp[k] += h
        tm[k] -= h
        out.append((energy_of(w, tp) - energy_of(w, tm)) / (2 * h))
    return np.array(out)


def sparse_rotations(n: int, idx: np.ndarray, amp: np.ndarray, letters: np.ndarray,
                     theta: np.ndarray, signs: Optional[np.ndarray] = None,
                     max_out: int = 1 << 20) -> Tuple[np.ndarray, np.ndarray]:
    """Rotations by definition on a sparse state; returns (indices, amplitudes) sorted."""
    i_in = np.ascontiguousarray(idx, dtype=np.uint64)
    a_in = np.ascontiguousarray(amp, dtype=np.complex128)
    l = np.ascontiguousarray(letters, dtype=np.uint8).reshape(-1, n)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    sp = None
    if signs is not None:
        s = np.ascontiguousarray(signs, dtype=np.int32)
        sp = s.ctypes.data
    io = np.empty(max_out, np.uint64)
    ao = np.empty(max_out, np.complex128)
    cnt = lib().orc_sparse_rotations(n, i_in, a_in, i_in.shape[0], l, sp, th, l.shape[0],
                                     io, ao, max_out)
    if cnt < 0:
        raise ValueError("oracle: sparse support overflow")
    order = np.argsort(io[:cnt])
    return io[:cnt][order], ao[:cnt][order]
