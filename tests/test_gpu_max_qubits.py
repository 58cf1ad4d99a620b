"""The largest states the library accepts, against the sparse oracle.

A state of 2^33 or 2^34 amplitudes has indices beyond 32 bits, so these runs
check the 64-bit index arithmetic of state set-up, the rotation passes and the
read-only measurement passes at the maximum size (n = 34 at complex64 and
n = 33 at complex128, 128 GiB each).  The rotations' x masks are drawn from a
10-dimensional span whose vectors reach the top index bits, so from a basis
state the run stays on at most 2^10 amplitudes, which the oracle computes by
definition; every other amplitude must stay zero, which the norm checks.  The
rotations interfere (24 of them on 10 dimensions), so the observable's terms,
whose x masks come from the same span, have non-zero expectation values.  (With
independent masks every <P> of this kind is exactly zero.)

<P> for a Hermitian Pauli P follows from the oracle's own rotation: with
R_P(theta) = cos(theta/2) - i sin(theta/2) P, R_P(pi) = -i P (up to the
rounding of cos(pi/2), about 6e-17), so <a|P|a> = i <a|R_P(pi) a>.
"""
import numpy as np
import pytest
import torch

from oracle import sim
from paper_2602_09020_amd import cfh, hybrid

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _letters(x, z, n):
    """(x, z) bit masks -> letters (0 I, 1 X, 2 Y, 3 Z)."""
    row = np.zeros(n, np.uint8)
    for j in range(n):
        xb, zb = (x >> j) & 1, (z >> j) & 1
        row[j] = 2 if (xb and zb) else 1 if xb else 3 if zb else 0
    return row


def _inputs(n):
    """Seeded rotations (x masks from a 10-dimensional span), angles, start
    index (bits 31 and n - 2 set) and an observable with masks from the span."""
    rng = np.random.default_rng(3400 + n)
    D, K, M = 10, 24, 16
    full = (1 << n) - 1
    base = [int(rng.integers(0, 1 << 62)) & full | (1 << (n - 1 - i % 3)) for i in range(D)]

    def comb(allow_zero):
        while True:
            c, x = int(rng.integers(0, 1 << D)), 0
            for i in range(D):
                if (c >> i) & 1:
                    x ^= base[i]
            if x or allow_zero:
                return x

    rows = np.array([_letters(comb(False), int(rng.integers(0, 1 << 62)) & full, n) for _ in range(K)])
    terms = np.array([_letters(comb(True), int(rng.integers(0, 1 << 62)) & full, n) for _ in range(M)])
    theta = rng.uniform(-np.pi, np.pi, size=K)
    init = (1 << (n - 2)) | (1 << 31) | int(rng.integers(0, 1 << 31))
    return rows, theta, init, terms, rng.normal(size=M)


def _sparse_expval(n, idx, amp, row):
    """<a|P|a> of the sparse state (idx, amp) by the oracle's R_P(pi)."""
    io, ao = sim.sparse_rotations(n, idx, amp, row[None, :], np.array([np.pi]))
    _, ia, ib = np.intersect1d(idx, io, assume_unique=True, return_indices=True)
    return 1j * np.sum(np.conj(amp[ia]) * ao[ib])


def _norm2(psi):
    """sum |psi|^2 in float64, a 2^28-amplitude chunk at a time."""
    tot = 0.0
    for ch in psi.split(1 << 28):
        tot += float(torch.view_as_real(ch).double().pow(2).sum().item())
    return tot


@pytest.mark.parametrize("dtype,n", [(torch.complex64, 34), (torch.complex128, 33)])
def test_max_qubits_rotations_and_expval_vs_sparse_oracle(dtype, n):
    torch.cuda.empty_cache()
    need = (1 << n) * (8 if dtype == torch.complex64 else 16)
    free, _ = torch.cuda.mem_get_info()
    assert free >= need + (4 << 30), f"{free / 2**30:.1f} GiB free, {need / 2**30:.0f} GiB needed"
    rows, theta, init, terms, coeff = _inputs(n)
    io, ao = sim.sparse_rotations(n, np.array([init], np.uint64), np.array([1 + 0j]), rows, theta)
    assert io.max() >= (1 << 32) and io.min() < (1 << 31)
    vals = np.array([_sparse_expval(n, io, ao, r) for r in terms])
    assert np.count_nonzero(np.abs(vals.real) > 1e-3) >= len(terms) // 2
    e_ref = complex(np.dot(coeff, vals))

    psi = hybrid.new_state(n, dtype, index=init)
    try:
        plan = hybrid.Plan(n, dtype, cfh.cfh_pauli_encode(rows))
        plan.apply(psi, torch.tensor(theta, device=DEV))
        ham = hybrid.Hamiltonian(n, dtype, cfh.cfh_pauli_encode(terms), coeff)
        e = ham.expval(psi)
        got = psi[torch.from_numpy(io.astype(np.int64)).to(DEV)].cpu().to(torch.complex128).numpy()
        norm = _norm2(psi)
    finally:
        del psi
        torch.cuda.empty_cache()
    print(f"n={n} {dtype}: support {io.size}, passes {plan.info()['n_passes']}, "
          f"<H> {e.real:.15f} vs {e_ref.real:.15f}", flush=True)
    tol = 1e-12 if dtype == torch.complex128 else 1e-4
    assert np.abs(got - ao).max() <= tol
    ntol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert abs(norm - 1) <= ntol
    assert abs(norm - float(np.sum(np.abs(got) ** 2))) <= ntol
    scale = np.abs(coeff).sum()
    assert abs(e.real - e_ref.real) <= tol * scale and abs(e.imag) <= tol * scale
    assert abs(e_ref.imag) <= 1e-12 * scale


def _sparse_energy(n, init, rows, theta, terms, coeff):
    """E(theta) = sum_k c_k <a|P_k|a> on the oracle's sparse state."""
    io, ao = sim.sparse_rotations(n, np.array([init], np.uint64), np.array([1 + 0j]), rows, theta)
    return float(np.real(sum(c * _sparse_expval(n, io, ao, r) for c, r in zip(coeff, terms))))


@pytest.mark.parametrize("dtype,n", [(torch.complex64, 33), (torch.complex128, 32)])
def test_max_qubits_adjoint_gradients_vs_sparse_parameter_shift(dtype, n):
    """The adjoint sweep holds psi and lambda (2 x 64 GiB here).  Every
    gradient against the parameter-shift rule on the sparse oracle,
    dE/dtheta_j = (E(theta + pi/2 e_j) - E(theta - pi/2 e_j)) / 2 for
    R_P(theta) = exp(-i theta P / 2); the sweep must also rewind psi to the
    start state.  complex64: amplitude errors within 1e-4 on unit-norm states
    move a gradient or the energy by at most about 1e-4 * sum |c_j|."""
    torch.cuda.empty_cache()
    need = 2 * (1 << n) * (8 if dtype == torch.complex64 else 16)
    free, _ = torch.cuda.mem_get_info()
    assert free >= need + (4 << 30), f"{free / 2**30:.1f} GiB free, {need / 2**30:.0f} GiB needed"
    rows, theta, init, terms, coeff = _inputs(n)
    e_ref = _sparse_energy(n, init, rows, theta, terms, coeff)
    g_ref = np.zeros(len(theta))
    for j in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += np.pi / 2
        tm[j] -= np.pi / 2
        g_ref[j] = 0.5 * (_sparse_energy(n, init, rows, tp, terms, coeff) -
                          _sparse_energy(n, init, rows, tm, terms, coeff))
    assert np.count_nonzero(np.abs(g_ref) > 1e-3) >= len(theta) // 2

    psi = hybrid.new_state(n, dtype, index=init)
    lam = None
    try:
        plan = hybrid.Plan(n, dtype, cfh.cfh_pauli_encode(rows))
        ham = hybrid.Hamiltonian(n, dtype, cfh.cfh_pauli_encode(terms), coeff)
        th = torch.tensor(theta, device=DEV)
        plan.apply(psi, th)
        e = ham.expval(psi)
        lam = torch.empty_like(psi)
        grad = torch.empty_like(th)
        cfh.cfh_adjoint_grad(plan.h, ham.h, psi, lam, th, grad)
        g = grad.cpu().numpy()
        back = psi[torch.tensor([init, init ^ 1, init ^ (1 << (n - 1))], device=DEV)].cpu()
        back = back.to(torch.complex128).numpy()
        norm = _norm2(psi)
    finally:
        del psi, lam
        torch.cuda.empty_cache()
    scale = np.abs(coeff).sum()
    tol = (1e-10 if dtype == torch.complex128 else 1e-4 * scale)
    etol = (1e-12 if dtype == torch.complex128 else 1e-4) * scale
    print(f"n={n} {dtype}: max |g - shift| {np.abs(g - g_ref).max():.2e}, E {e.real:.12f} vs {e_ref:.12f}",
          flush=True)
    assert abs(e.real - e_ref) <= etol
    assert np.abs(g - g_ref).max() <= tol
    rtol = 1e-11 if dtype == torch.complex128 else 1e-4
    assert abs(back[0] - 1) <= rtol and np.abs(back[1:]).max() <= rtol
    assert abs(norm - 1) <= (1e-11 if dtype == torch.complex128 else 1e-5)
