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
from functools import lru_cache
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from oracle import sim
from paper_2602_09020_amd import cfh, hybrid

pytestmark = pytest.mark.gpu
DEV = "cuda"
# the runs stay on at most 2^10 amplitudes; the oracle raises past this bound
_SUPPORT = 1 << 12


def _letters(x, z, n):
    """(x, z) bit masks -> letters (0 I, 1 X, 2 Y, 3 Z)."""
    row = np.zeros(n, np.uint8)
    for j in range(n):
        xb, zb = (x >> j) & 1, (z >> j) & 1
        row[j] = 2 if (xb and zb) else 1 if xb else 3 if zb else 0
    return row


def _inputs(n):
    """Seeded rotations (x masks from a 10-dimensional span), angles, start
    index (bits n - 2 and min(31, n - 1) set) and an observable with masks
    from the span."""
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
    k = min(31, n - 1)
    init = (1 << (n - 2)) | (1 << k) | int(rng.integers(0, 1 << k))
    return rows, theta, init, terms, rng.normal(size=M)


def _sparse_expval(n, idx, amp, row):
    """<a|P|a> of the sparse state (idx, amp) by the oracle's R_P(pi)."""
    io, ao = sim.sparse_rotations(n, idx, amp, row[None, :], np.array([np.pi]), max_out=_SUPPORT)
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
    io, ao = sim.sparse_rotations(n, np.array([init], np.uint64), np.array([1 + 0j]), rows, theta, max_out=_SUPPORT)
    return float(np.real(sum(c * _sparse_expval(n, io, ao, r) for c, r in zip(coeff, terms))))


@lru_cache(maxsize=None)
def _sparse_reference(n):
    """(energy, parameter-shift gradients) of the seeded circuit on n qubits."""
    rows, theta, init, terms, coeff = _inputs(n)
    e = _sparse_energy(n, init, rows, theta, terms, coeff)
    g = np.zeros(len(theta))
    for j in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += np.pi / 2
        tm[j] -= np.pi / 2
        g[j] = 0.5 * (_sparse_energy(n, init, rows, tp, terms, coeff) - _sparse_energy(n, init, rows, tm, terms, coeff))
    return e, g


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
    e_ref, g_ref = _sparse_reference(n)
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


def _with_diagonal(n, rows, theta):
    """The rotations with three diagonal (Z-only) rotations spliced in."""
    rng = np.random.default_rng(77 + n)
    diag = np.where(rng.integers(0, 2, size=(3, n)) == 1, 3, 0).astype(np.uint8)
    diag[:, n - 1] = 3
    r = np.concatenate([rows[:8], diag[:2], rows[8:16], diag[2:], rows[16:]])
    t = np.concatenate([theta[:8], rng.uniform(-np.pi, np.pi, 2), theta[8:16], rng.uniform(-np.pi, np.pi, 1),
                        theta[16:]])
    return r, t


@pytest.mark.parametrize("tuning", [{"unfused": 1}, {"variant": 1, "tile_bits": 10, "low_bits": 3}],
                         ids=["unfused", "lds_b10"])
def test_max_qubits_unfused_and_small_lds_tiles_vs_sparse_oracle(tuning):
    """n = 34 at complex64 through the paths whose launches grow with the
    state: one rotation per launch (2^34 amplitudes for a diagonal rotation),
    and LDS-staged passes on 2^10 tiles (2^24 workgroups of 256 threads, more
    work-items than one launch holds), with <H> on the same tiles.  The unfused
    run then measures a Z-type Pauli and checks the collapsed state: the
    amplitudes of the drawn eigenspace, divided by sqrt(P(s))."""
    n, dtype = 34, torch.complex64
    torch.cuda.empty_cache()
    rows, theta, init, terms, coeff = _inputs(n)
    rows, theta = _with_diagonal(n, rows, theta)
    io, ao = sim.sparse_rotations(n, np.array([init], np.uint64), np.array([1 + 0j]), rows, theta)
    e_ref = complex(np.dot(coeff, [_sparse_expval(n, io, ao, r) for r in terms]))
    zrow = np.where(np.random.default_rng(5).integers(0, 2, size=n) == 1, 3, 0).astype(np.uint8)
    zrow[n - 1] = zrow[0] = 3
    zmask = sum(1 << j for j in range(n) if zrow[j] == 3)
    ev_z = float(np.real(_sparse_expval(n, io, ao, zrow)))
    assert abs(ev_z) < 0.9
    psi = hybrid.new_state(n, dtype, index=init)
    try:
        plan = hybrid.Plan(n, dtype, cfh.cfh_pauli_encode(rows), tuning)
        plan.apply(psi, torch.tensor(theta, device=DEV))
        ham = hybrid.Hamiltonian(n, dtype, cfh.cfh_pauli_encode(terms), coeff,
                                 None if "unfused" in tuning else tuning)
        e = ham.expval(psi)
        sel = torch.from_numpy(io.astype(np.int64)).to(DEV)
        got = psi[sel].cpu().to(torch.complex128).numpy()
        norm = _norm2(psi)
        meas = None
        if "unfused" in tuning:
            s, pp = cfh.cfh_measure_pauli(psi, n, 0, zmask, 0, 0.5)
            after = psi[sel].cpu().to(torch.complex128).numpy()
            meas = (s, pp, after, _norm2(psi))
    finally:
        del psi
        torch.cuda.empty_cache()
    print(f"{tuning}: passes {plan.info()['n_passes']}, max |d| {np.abs(got - ao).max():.2e}, "
          f"<H> {e.real:.9f} vs {e_ref.real:.9f}", flush=True)
    scale = np.abs(coeff).sum()
    assert np.abs(got - ao).max() <= 1e-4
    assert abs(norm - 1) <= 1e-5 and abs(norm - float(np.sum(np.abs(got) ** 2))) <= 1e-5
    assert abs(e.real - e_ref.real) <= 1e-4 * scale and abs(e.imag) <= 1e-4 * scale
    if meas is not None:
        s, pp, after, norm2 = meas
        p_ref = 0.5 * (1 + ev_z)
        assert abs(pp - p_ref) <= 1e-4 and s == (1 if 0.5 < p_ref else -1)
        par = np.array([bin(int(y) & zmask).count("1") & 1 for y in io])
        keep = (1 - 2 * par) == s
        want = np.where(keep, ao / np.sqrt(pp if s == 1 else 1 - pp), 0)
        assert np.abs(after - want).max() <= 1e-4 and abs(norm2 - 1) <= 1e-5


@pytest.mark.parametrize("tuning", [None, {"variant": 1, "tile_bits": 9, "low_bits": 3}], ids=["reg", "lds_b9"])
def test_max_qubits_ham_apply_vs_sparse_oracle(tuning):
    """H psi at n = 33, complex64 (psi and the output 64 GiB each): the
    register-tiled passes, and LDS-staged passes on 2^9 tiles (2^24 workgroups
    of 256 threads: several launches).  Expected: sum_k c_k P_k a with
    P_k a = i R_{P_k}(pi) a from the sparse oracle; the output must carry no
    weight outside those amplitudes."""
    n, dtype = 33, torch.complex64
    torch.cuda.empty_cache()
    rows, theta, init, terms, coeff = _inputs(n)
    io, ao = sim.sparse_rotations(n, np.array([init], np.uint64), np.array([1 + 0j]), rows, theta)
    parts_i, parts_a = [], []
    for c, r in zip(coeff, terms):
        i2, a2 = sim.sparse_rotations(n, io, ao, r[None, :], np.array([np.pi]))
        parts_i.append(i2)
        parts_a.append(1j * c * a2)
    idx, inv = np.unique(np.concatenate(parts_i), return_inverse=True)
    want = np.zeros(idx.size, np.complex128)
    np.add.at(want, inv, np.concatenate(parts_a))
    psi = hybrid.new_state(n, dtype, index=init)
    out = None
    try:
        hybrid.Plan(n, dtype, cfh.cfh_pauli_encode(rows)).apply(psi, torch.tensor(theta, device=DEV))
        ham = hybrid.Hamiltonian(n, dtype, cfh.cfh_pauli_encode(terms), coeff, tuning)
        out = torch.empty_like(psi)
        ham.apply(psi, out)
        got = out[torch.from_numpy(idx.astype(np.int64)).to(DEV)].cpu().to(torch.complex128).numpy()
        onorm = _norm2(out)
    finally:
        del psi, out
        torch.cuda.empty_cache()
    scale = np.abs(coeff).sum()
    print(f"{tuning}: {idx.size} amplitudes, max |d| {np.abs(got - want).max():.2e}", flush=True)
    assert np.abs(got - want).max() <= 1e-4 * scale
    assert abs(onorm - float(np.sum(np.abs(want) ** 2))) <= 1e-4 * scale * scale


def test_max_state_empty_observable_and_calibration_kernel():
    """n = 32 at complex128 (64 GiB): H psi of an observable without terms
    zeroes all 2^33 doubles of the output, and the calibration kernel, in
    launches of at most 2^31 threads, turns every amplitude exactly once, in
    index order and in the scattered order: two calls multiply each amplitude
    by exp(0.5 i)."""
    n, dtype = 32, torch.complex128
    torch.cuda.empty_cache()
    psi = hybrid.new_state(n, dtype, index=(1 << 31) + 5)
    out = None
    try:
        h0 = hybrid.Hamiltonian(n, dtype, np.zeros(0, cfh.PAULI_DTYPE), np.zeros(0))
        out = torch.ones_like(psi)
        h0.apply(psi, out)
        zmax = max(float(ch.abs().max().item()) for ch in out.split(1 << 28))
        out.fill_(1.0)
        cfh.cfh_calib_rmw(out, n, -1)
        cfh.cfh_calib_rmw(out, n, 3)
        want = torch.tensor(np.exp(0.5j), dtype=dtype, device=DEV)
        dmax = max(float((ch - want).abs().max().item()) for ch in out.split(1 << 28))
    finally:
        del psi, out
        torch.cuda.empty_cache()
    assert zmax == 0
    assert dmax <= 1e-15


def _circuit(n):
    """The seeded circuit on n qubits as a batch workload (no Clifford prefix)."""
    rows, theta, init, terms, coeff = _inputs(n)
    return SimpleNamespace(n=n, prefix=np.zeros((0, 3), np.int32), init=init, rot=rows, theta=theta, ham=terms,
                           coeff=coeff, n_rot=len(theta))


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("variant", [0, 1], ids=["levels", "persistent"])
def test_batch_largest_circuits_vs_sparse_oracle(dtype, variant):
    """A batch with the largest circuits it accepts (30 and 29 qubits, beside
    a 12-qubit one; 48 GiB of states and lambda vectors at complex128), under
    level launches and the persistent kernel: energies and every gradient
    against the sparse oracle (parameter shift), within 1e-12 * sum |c_j|
    and 1e-10 at complex128, 1e-4 * sum |c_j| at complex64."""
    torch.cuda.empty_cache()
    ws = [_circuit(n) for n in (30, 29, 12)]
    B = hybrid.Batch(ws, dtype, {"variant": 1} if variant else None)
    try:
        B.run(True)
        r = B.results()
    finally:
        del B
        torch.cuda.empty_cache()
    for i, w in enumerate(ws):
        e_ref, g_ref = _sparse_reference(w.n)
        scale = np.abs(w.coeff).sum()
        etol = (1e-12 if dtype == torch.complex128 else 1e-4) * scale
        gtol = 1e-10 if dtype == torch.complex128 else 1e-4 * scale
        print(f"n={w.n}: |dE| {abs(r['energy'][i] - e_ref):.2e}, max |dg| {np.abs(r['grad'][i] - g_ref).max():.2e}",
              flush=True)
        assert abs(r["energy"][i] - e_ref) <= etol, i
        assert np.abs(r["grad"][i] - g_ref).max() <= gtol, i


def test_batch_items_of_a_large_circuit_cover_at_most_64_tiles():
    """A pass is cut into batch_items work items, or into more when an item
    would cover more than 64 tiles, so a large circuit's passes spread over
    the GPU.  One 26-qubit circuit (2^14 register tiles per pass): 256 items
    per pass at batch_items = 8 and 4,096 at batch_items = 4,096, the same
    passes, so exactly 16 times as many items in a gradient run; both against
    the sparse oracle at the complex128 bounds."""
    torch.cuda.empty_cache()
    w = _circuit(26)
    e_ref, g_ref = _sparse_reference(26)
    scale = np.abs(w.coeff).sum()
    items = {}
    for k in (8, 4096):
        B = hybrid.Batch([w], torch.complex128, {"batch_items": k})
        items[k] = B.info()["n_items_grad"]
        B.run(True)
        r = B.results()
        del B
        assert abs(r["energy"][0] - e_ref) <= 1e-12 * scale
        assert np.abs(r["grad"][0] - g_ref).max() <= 1e-10
    torch.cuda.empty_cache()
    assert items[8] * 16 == items[4096], items
