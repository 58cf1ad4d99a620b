"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: matrices
printed in the paper (golden fixtures), scipy matrix exponentials of explicit
Kronecker products, textbook gate identities, closed forms stated in the paper,
and brute force on tiny inputs.  A plausible mistake in the oracle (a dropped
letter, a wrong sign, a swapped qubit order, a wrong ladder direction) fails at
least one of them.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import dense, sim
from conftest import load_golden_matrices
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def rand_state(n, rng=RNG):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def oracle_gate_matrix(code, q0, q1, n):
    N = 1 << n
    M = np.zeros((N, N), complex)
    for c in range(N):
        v = sim.basis_state(n, c)
        sim.apply_gate(v, n, code, q0, q1)
        M[:, c] = v
    return M


def oracle_rotation_matrix(letters, theta, n, sign=1):
    N = 1 << n
    M = np.zeros((N, N), complex)
    for c in range(N):
        v = sim.basis_state(n, c)
        sim.rotation(v, n, np.asarray(letters, np.uint8), theta, sign)
        M[:, c] = v
    return M


# ------------------------------------------------------------ gate matrices

def test_gate_matrices_match_paper_golden():
    """Sec. 2.1: the oracle's X, Y, Z, H, S, CNOT equal the printed matrices."""
    g = load_golden_matrices(os.path.join(GOLDEN, "paper_gates.txt"))
    for code, name in [(3, "X"), (4, "Y"), (5, "Z"), (0, "H"), (1, "S")]:
        assert np.allclose(oracle_gate_matrix(code, 0, -1, 1), g[name], atol=1e-15), name
    # control = qubit 1 (the more significant bit), target = qubit 0
    assert np.allclose(oracle_gate_matrix(6, 1, 0, 2), g["CNOT"], atol=0)
    assert np.allclose(oracle_gate_matrix(2, 0, -1, 1), g["S"].conj().T)


def test_pauli_identities_from_paper():
    """Sec. 2.1: XYZ = iI and sigma_j^2 = I, on random states via the oracle."""
    psi = rand_state(3)
    for q in range(3):
        v = psi.copy()
        for code in (5, 4, 3):  # apply Z, then Y, then X: X Y Z psi
            sim.apply_gate(v, 3, code, q)
        assert np.allclose(v, 1j * psi, atol=1e-14)
        for code in (3, 4, 5):
            v = psi.copy()
            sim.apply_gate(v, 3, code, q)
            sim.apply_gate(v, 3, code, q)
            assert np.allclose(v, psi, atol=1e-14)


def test_two_qubit_gates_against_dense_permutations():
    for n in (2, 3):
        for q0, q1 in itertools.permutations(range(n), 2):
            for code in (6, 7, 8):
                assert np.allclose(oracle_gate_matrix(code, q0, q1, n),
                                   dense.embed2(code, q0, q1, n), atol=0)


# ----------------------------------------------------------- ladder rotation

def test_ladder_equals_expm_all_strings_n2():
    """Every 2-qubit string (both signs) against scipy expm(-i theta/2 P)."""
    for letters in itertools.product(range(4), repeat=2):
        for theta in (0.37, -2.1, np.pi):
            for sign, phase in ((1, 0), (-1, 2)):
                ref = dense.rotation(letters, theta, phase)
                got = oracle_rotation_matrix(letters, theta, 2, sign)
                assert np.abs(got - ref).max() < 1e-13, (letters, theta, sign)


@pytest.mark.parametrize("n", [1, 3, 4, 5, 6])
def test_ladder_equals_expm_random(n):
    rng = np.random.default_rng(n)
    for _ in range(12):
        letters = rng.integers(0, 4, size=n).astype(np.uint8)
        theta = rng.uniform(-7, 7)
        psi = rand_state(n, rng)
        v = psi.copy()
        sim.rotation(v, n, letters, theta)
        assert np.abs(v - dense.rotation(letters, theta) @ psi).max() < 1e-13


def test_single_qubit_rotations_textbook():
    """RX, RY, RZ in their textbook closed forms (Sec. 3 with P a single letter)."""
    for th in (0.3, 1.7, -2.9):
        c, s = np.cos(th / 2), np.sin(th / 2)
        assert np.allclose(oracle_rotation_matrix([1], th, 1), [[c, -1j * s], [-1j * s, c]])
        assert np.allclose(oracle_rotation_matrix([2], th, 1), [[c, -s], [s, c]])
        assert np.allclose(oracle_rotation_matrix([3], th, 1),
                           np.diag([np.exp(-1j * th / 2), np.exp(1j * th / 2)]))


def test_rotation_special_angles_and_inverse():
    n = 6
    rng = np.random.default_rng(7)
    for _ in range(10):
        letters = rng.integers(0, 4, size=n).astype(np.uint8)
        psi = rand_state(n, rng)
        v = psi.copy()
        sim.rotation(v, n, letters, 0.0)
        assert np.abs(v - psi).max() < 1e-14                  # theta = 0 -> I
        v = psi.copy()
        sim.rotation(v, n, letters, 2 * np.pi)
        assert np.abs(v + psi).max() < 1e-13                  # theta = 2 pi -> -I
        th = rng.uniform(-3, 3)
        v = psi.copy()
        sim.rotation(v, n, letters, th)
        assert abs(np.linalg.norm(v) - 1) < 1e-14             # unitary
        sim.rotation(v, n, letters, -th)
        assert np.abs(v - psi).max() < 1e-13                  # R(-t) R(t) = I


def test_pauli_action_on_basis_closed_form():
    """Sec. 3: P|k> = i^|mY| (-1)^(|mY & k| + |mZ & k|) |k ^ mX ^ mY>, the
    bitwise product inside the phase read as AND (the paper's symbol there is
    defined as XOR, which would give Z|1> = +|1>)."""
    n = 4
    for letters in itertools.product(range(4), repeat=n):
        mx = sum(1 << j for j in range(n) if letters[j] == 1)
        my = sum(1 << j for j in range(n) if letters[j] == 2)
        mz = sum(1 << j for j in range(n) if letters[j] == 3)
        for k in range(1 << n):
            v = sim.basis_state(n, k)
            for q in range(n):
                if letters[q]:
                    sim.apply_gate(v, n, 2 + letters[q], q)   # X=3, Y=4, Z=5
            expect = np.zeros(1 << n, complex)
            sgn = (-1) ** (bin(my & k).count("1") + bin(mz & k).count("1"))
            expect[k ^ mx ^ my] = (1j ** bin(my).count("1")) * sgn
            assert np.allclose(v, expect, atol=1e-15), (letters, k)


def test_pair_update_rule_appendix_b():
    """App. B: the amplitude pair (a_k, a_f(k)) transforms by
    [[c, -i s e^{i phi(f(k))}], [-i s e^{i phi(k)}, c]]."""
    n = 4
    rng = np.random.default_rng(3)
    for _ in range(20):
        letters = rng.integers(0, 4, size=n).astype(np.uint8)
        if not any(l in (1, 2) for l in letters):
            continue
        th = rng.uniform(-3, 3)
        psi = rand_state(n, rng)
        v = psi.copy()
        sim.rotation(v, n, letters, th)
        mx = sum(1 << j for j in range(n) if letters[j] == 1)
        my = sum(1 << j for j in range(n) if letters[j] == 2)
        mz = sum(1 << j for j in range(n) if letters[j] == 3)
        ephi = lambda k: (1j ** bin(my).count("1")) * (-1) ** (bin(my & k).count("1") + bin(mz & k).count("1"))
        c, s = np.cos(th / 2), np.sin(th / 2)
        for k in range(1 << n):
            f = k ^ mx ^ my
            assert abs(v[k] - (c * psi[k] - 1j * s * ephi(f) * psi[f])) < 1e-13


def test_diagonal_rotation_branches():
    """App. B diagonal case, with the branches as Eq. for R_P|k> gives them:
    even parity of (mZ & k) -> e^{-i theta/2}, odd -> e^{+i theta/2}."""
    n = 5
    letters = np.array([3, 0, 3, 3, 0], np.uint8)
    mz = 0b01101
    th = 0.81
    for k in range(1 << n):
        v = sim.basis_state(n, k)
        sim.rotation(v, n, letters, th)
        odd = bin(mz & k).count("1") % 2
        assert abs(v[k] - np.exp((1j if odd else -1j) * th / 2)) < 1e-14


def test_clifford_pauli_rotation_note():
    """App. A, Note: with R(Q) = exp(-i pi/4 Q), R P R^dag = P if [P,Q] = 0 and
    -iQP if {P,Q} = 0; and for general angle, exp(-i t Q) P exp(i t Q) =
    i P Q sin 2t + P cos 2t in the anticommuting case."""
    n = 3
    rng = np.random.default_rng(11)
    for _ in range(25):
        lp = rng.integers(0, 4, size=n)
        lq = rng.integers(0, 4, size=n)
        P, Q = dense.pauli(lp), dense.pauli(lq)
        R = oracle_rotation_matrix(lq, np.pi / 2, n)
        conj = R @ P @ R.conj().T
        if np.allclose(P @ Q, Q @ P):
            assert np.allclose(conj, P, atol=1e-13)
        else:
            assert np.allclose(conj, -1j * Q @ P, atol=1e-13)
            t = rng.uniform(-2, 2)
            Rt = oracle_rotation_matrix(lq, 2 * t, n)   # exp(-i t Q) = R_Q(2t)
            assert np.allclose(Rt @ P @ Rt.conj().T, 1j * P @ Q * np.sin(2 * t) + P * np.cos(2 * t),
                               atol=1e-13)


def test_swap_from_three_pi4_rotations():
    """App. A footnote: SWAP of qubits 0 and 1 by pi/4 rotations about XX, YY, ZZ
    (exp(-i pi/4 P) = R_P(pi/2)); equal to SWAP up to the global phase e^{-i pi/4}."""
    n = 2
    M = (oracle_rotation_matrix([3, 3], np.pi / 2, n) @ oracle_rotation_matrix([2, 2], np.pi / 2, n)
         @ oracle_rotation_matrix([1, 1], np.pi / 2, n))
    assert np.allclose(M, np.exp(-1j * np.pi / 4) * oracle_gate_matrix(8, 0, 1, n), atol=1e-14)


# ----------------------------------------------------------- Heisenberg walk

def test_heisenberg_tables_textbook():
    """Textbook conjugations G^dag sigma G (one-qubit gates)."""
    expect = {
        (0, 1): (3, 0), (0, 3): (1, 0), (0, 2): (2, 2),        # H: X<->Z, Y->-Y
        (1, 1): (2, 2), (1, 2): (1, 0), (1, 3): (3, 0),        # S^dag X S = -Y, S^dag Y S = X
        (2, 1): (2, 0), (2, 2): (1, 2),                        # S X S^dag = Y, S Y S^dag = -X
        (3, 3): (3, 2), (3, 2): (2, 2), (3, 1): (1, 0),        # X: Z->-Z, Y->-Y
        (5, 1): (1, 2), (5, 2): (2, 2), (4, 1): (1, 2), (4, 3): (3, 2), (4, 2): (2, 0),
    }
    for (g, l), (l2, ph) in expect.items():
        p = np.zeros(1, np.int32)
        import ctypes
        out_ph = ctypes.c_int()
        got = sim.lib().orc_conj_table1(g, l, ctypes.byref(out_ph))
        assert (got, out_ph.value) == (l2, ph), (g, l)


def test_heisenberg_cnot_textbook():
    """CNOT (c -> t): X_c -> X_c X_t, Z_t -> Z_c Z_t, Z_c -> Z_c, X_t -> X_t."""
    gates = np.array([[6, 0, 1]], np.int32)
    cases = {(1, 0): ((1, 1), 0), (0, 3): ((3, 3), 0), (3, 0): ((3, 0), 0), (0, 1): ((0, 1), 0),
             (2, 0): ((2, 1), 0), (0, 2): ((3, 2), 0)}
    for inp, (out, ph) in cases.items():
        l, p = sim.heisenberg(gates, np.array(inp, np.uint8))
        assert tuple(l) == out and p == ph, (inp, l, p)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_heisenberg_equals_dense_conjugation(n):
    """C^dag Q C through the walk equals the explicit dense product, for random
    Clifford circuits over all nine gate codes."""
    rng = np.random.default_rng(100 + n)
    for _ in range(30):
        gates = []
        for _ in range(rng.integers(1, 15)):
            g = int(rng.integers(0, 9))
            q0, q1 = (int(v) for v in rng.choice(n, 2, replace=False))
            gates.append((g, q0, q1 if g >= 6 else -1))
        gates = np.array(gates, np.int32)
        U = dense.circuit_unitary(gates, n)
        letters = rng.integers(0, 4, size=n).astype(np.uint8)
        ph0 = int(rng.integers(0, 4))
        l2, ph = sim.heisenberg(gates, letters, ph0)
        assert np.allclose(U.conj().T @ dense.pauli(letters, ph0) @ U, dense.pauli(l2, ph), atol=1e-12)


def test_frame_rows_satisfy_frame_relations():
    """Sec. 4.1: lambda(effZ_i, effZ_j) = lambda(effX_i, effX_j) = 0 and
    lambda(effZ_i, effX_j) = delta_ij, checked with dense commutators."""
    n = 4
    rng = np.random.default_rng(5)
    gates = W.clifford_prefix(rng, n, 40)
    zl, zph, xl, xph = sim.frame_rows(gates, n)
    Z = [dense.pauli(zl[i], zph[i]) for i in range(n)]
    X = [dense.pauli(xl[i], xph[i]) for i in range(n)]
    anti = lambda A, B: np.allclose(A @ B, -B @ A)
    for i in range(n):
        for j in range(n):
            assert not anti(Z[i], Z[j]) and not anti(X[i], X[j])
            assert anti(Z[i], X[j]) == (i == j)
    for i in range(n):
        assert zph[i] % 2 == 0 and xph[i] % 2 == 0   # Hermitian rows


def test_single_to_multi_rotation_identity():
    """Eq. single_to_multirot: R_Z(i, theta) U = U R_{effZ_i}(theta)."""
    n = 4
    rng = np.random.default_rng(9)
    gates = W.clifford_prefix(rng, n, 30)
    U = dense.circuit_unitary(gates, n)
    zl, zph, _, _ = sim.frame_rows(gates, n)
    for i in range(n):
        th = rng.uniform(-3, 3)
        e = np.zeros(n, np.uint8)
        e[i] = 3
        lhs = dense.rotation(e, th) @ U
        sign = 1 if zph[i] == 0 else -1
        rhs = U @ oracle_rotation_matrix(zl[i], th, n, sign)
        assert np.allclose(lhs, rhs, atol=1e-12)


# ---------------------------------------------------------- expectation

def test_expval_closed_forms_on_basis_states():
    """<k|Z^z|k> = (-1)^|z & k|; <k|P|k> = 0 whenever P has an X or Y letter."""
    n = 4
    for letters in itertools.product(range(4), repeat=n):
        mz = sum(1 << j for j in range(n) if letters[j] == 3)
        off = any(l in (1, 2) for l in letters)
        for k in (0, 5, 11, 15):
            v = sim.expval(sim.basis_state(n, k), n, np.array(letters, np.uint8))
            expect = 0.0 if off else (-1) ** bin(mz & k).count("1")
            assert abs(v - expect) < 1e-15


def test_expval_equals_dense():
    n = 5
    rng = np.random.default_rng(21)
    psi = rand_state(n, rng)
    for _ in range(30):
        letters = rng.integers(0, 4, size=n).astype(np.uint8)
        ph = int(rng.integers(0, 4))
        assert abs(sim.expval(psi, n, letters, ph) - np.vdot(psi, dense.pauli(letters, ph) @ psi)) < 1e-13


@pytest.mark.parametrize("n", [1, 3, 5])
def test_apply_pauli_sum_equals_dense_weighted_sum(n):
    """Sec. 4.4, Eq. chfsexp with H = sum_j c_j i^{ph_j} P_j: the oracle's H psi
    against the dense sum of explicit Kronecker products, several terms at once,
    random real weights and every phase.  A dropped or mis-indexed weight, a
    wrong power of i or a lost accumulation across terms changes the result."""
    rng = np.random.default_rng(300 + n)
    psi = rand_state(n, rng)
    m = 7
    letters = rng.integers(0, 4, size=(m, n)).astype(np.uint8)
    coeff = rng.normal(size=m)
    phases = np.array([j % 4 for j in range(m)], np.int32)
    rng.shuffle(phases)
    dense_h = sum(c * dense.pauli(l, int(p)) for l, c, p in zip(letters, coeff, phases))
    out = sim.apply_pauli_sum(psi, n, letters, coeff, phases)
    assert np.abs(out - dense_h @ psi).max() < 1e-13
    # without phases every term is c_j P_j
    dense_0 = sum(c * dense.pauli(l) for l, c in zip(letters, coeff))
    assert np.abs(sim.apply_pauli_sum(psi, n, letters, coeff) - dense_0 @ psi).max() < 1e-13
    # linear in the weights: doubling one term's weight adds exactly that term once more
    c2 = coeff.copy()
    c2[3] *= 2
    extra = coeff[3] * dense.pauli(letters[3], int(phases[3])) @ psi
    assert np.abs(sim.apply_pauli_sum(psi, n, letters, c2, phases) - (dense_h @ psi + extra)).max() < 1e-13


def test_energy_with_phases_equals_dense():
    """E = sum_j c_j Re <psi| i^{ph_j} P_j |psi> against the dense quadratic form,
    with phases 1 and 3 (anti-Hermitian terms contribute Re of an imaginary
    number only through their Y and sign content) and several weighted terms."""
    n = 4
    rng = np.random.default_rng(77)
    psi = rand_state(n, rng)
    m = 9
    letters = rng.integers(0, 4, size=(m, n)).astype(np.uint8)
    coeff = rng.normal(size=m)
    phases = rng.integers(0, 4, size=m).astype(np.int32)
    want = sum(c * np.vdot(psi, dense.pauli(l, int(p)) @ psi).real for l, c, p in zip(letters, coeff, phases))
    assert abs(sim.energy(psi, n, letters, coeff, phases) - want) < 1e-13
    # the energy of a sum is the real part of <psi|H psi> built from the weighted sum
    hpsi = sim.apply_pauli_sum(psi, n, letters, coeff, phases)
    assert abs(np.vdot(psi, hpsi).real - want) < 1e-13


def test_expval_through_frame_equation():
    """Eq. chfsexp: <psi|P|psi> = <Phi|F(P)|Phi> with psi = C Phi and F(P) = C^dag P C."""
    w = W.config(0)
    psi, phi = sim.simulate(w, n_rot=40)
    rng = np.random.default_rng(4)
    for _ in range(10):
        letters = rng.integers(0, 4, size=w.n).astype(np.uint8)
        fl, fph = sim.heisenberg(w.prefix, letters)
        assert abs(sim.expval(psi, w.n, letters) - sim.expval(phi, w.n, fl, fph)) < 1e-12


# ------------------------------------------------------------- gradients

def test_param_shift_closed_form_single_qubit():
    """|0>, R_X(theta), H = Z: E = cos(theta), dE/dtheta = -sin(theta)."""
    w = W.Workload("t", 1, 0, np.zeros((0, 3), np.int32), np.array([[1]], np.uint8),
                   np.array([0.7]), np.array([[3]], np.uint8), np.array([1.0]))
    assert abs(sim.energy_of(w, w.theta) - np.cos(0.7)) < 1e-15
    assert abs(sim.param_shift_grad(w)[0] + np.sin(0.7)) < 1e-15
    assert abs(sim.finite_diff_grad(w)[0] + np.sin(0.7)) < 1e-9


def test_param_shift_vs_dense_finite_difference():
    """Parameter shift on a small JW circuit against a dense-matrix (scipy expm)
    central finite difference computed independently of the ladder."""
    w = W.config(0, n=5, n_rot=8, n_ham=6)
    def dense_energy(theta):
        U = dense.circuit_unitary(w.prefix, w.n)
        v = U @ sim.basis_state(w.n, w.init)
        for k in range(w.n_rot):
            v = dense.rotation(w.rot[k], theta[k]) @ v
        H = sum(c * dense.pauli(h) for c, h in zip(w.coeff, w.ham))
        return float(np.real(np.vdot(v, H @ v)))
    assert abs(dense_energy(w.theta) - sim.energy_of(w, w.theta)) < 1e-12
    g = sim.param_shift_grad(w)
    h = 1e-5
    for k in range(w.n_rot):
        tp, tm = w.theta.copy(), w.theta.copy()
        tp[k] += h
        tm[k] -= h
        assert abs(g[k] - (dense_energy(tp) - dense_energy(tm)) / (2 * h)) < 1e-8


# ------------------------------------------------------------ sparse path

def test_sparse_definition_equals_ladder():
    """The sparse by-definition simulator and the ladder agree (two routes)."""
    w = W.config(0)
    p = sim.basis_state(w.n, w.init)
    sim.rotations(p, w.n, w.rot, w.theta)
    io, ao = sim.sparse_rotations(w.n, np.array([w.init]), np.array([1 + 0j]), w.rot, w.theta)
    d = np.zeros(1 << w.n, complex)
    d[io.astype(np.int64)] = ao
    assert np.abs(d - p).max() < 1e-12


def test_sparse_equals_expm_small():
    n = 4
    rng = np.random.default_rng(8)
    letters = rng.integers(0, 4, size=(6, n)).astype(np.uint8)
    th = rng.uniform(-3, 3, size=6)
    signs = np.array([1, -1, 1, 1, -1, 1], np.int32)
    io, ao = sim.sparse_rotations(n, np.array([3]), np.array([1 + 0j]), letters, th, signs)
    v = sim.basis_state(n, 3)
    for k in range(6):
        v = dense.rotation(letters[k], th[k], 0 if signs[k] > 0 else 2) @ v
    d = np.zeros(1 << n, complex)
    d[io.astype(np.int64)] = ao
    assert np.abs(d - v).max() < 1e-13


# ------------------------------------------------------- workload shape

def test_jw_weight_statistics_match_paper_table():
    """The synthetic JW strings at 24 qubits have Pauli-weight mean and spread
    within the range of the paper's 24-qubit chemistry rows (Table tab:scores)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_table_24q.txt"))
            if l.strip() and not l.startswith("#")]
    means = [float(r[3]) for r in rows]
    stds = [float(r[4]) for r in rows]
    w = W.make_workload("s", 24, seed=0, n_rot=5000)
    wt = W.pauli_weight(w.rot)
    assert min(means) - 0.3 < wt.mean() < max(means) + 0.3
    assert min(stds) - 0.3 < wt.std() < max(stds) + 0.3
    assert wt.max() <= 24
    # every string Hermitian: X/Y count even per string (JW shape)
    assert np.all(((w.rot == 1) | (w.rot == 2)).sum(1) % 2 == 0)
