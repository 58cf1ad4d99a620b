"""GPU test of the allocation-free expectation value (cfh_expval_noalloc)
against cfh_expval, through the C ABI: two calls in a row on one device, the
second with a smaller state and fewer terms, so the shared partial-sum array
keeps nothing from the first call that the second would read."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2602_09020_amd import cfh, hybrid

pytestmark = pytest.mark.gpu


def _state(n, dtype, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    return torch.from_numpy(v).to(dtype).to("cuda")


def _terms(n, m, seed):
    w = W.make_workload("na", n, seed=seed, n_prefix=3 * n, n_rot=0, n_ham=m)
    frame = hybrid.Frame(n)
    frame.apply_gates(w.prefix)
    return frame.conjugate(cfh.cfh_pauli_encode(w.ham)), w.coeff


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_expval_noalloc_matches_expval_on_two_calls(dtype):
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    # first call: 2^16 amplitudes, 150 terms (three launches of terms)
    # second call: 2^9 amplitudes (one workgroup), 7 terms
    for n, m, seed in ((16, 150, 1), (9, 7, 2)):
        psi = _state(n, dtype, seed)
        terms, coeff = _terms(n, m, seed)
        cfh.cfh_expval_noalloc(psi, n, terms, coeff, out)
        torch.cuda.synchronize()
        got = complex(float(out[0]), float(out[1]))
        ref = cfh.cfh_expval(psi, n, terms, coeff)
        # both sum the same double products of the same stored amplitudes in
        # different orders: the difference is rounding, far below 1e-12 per
        # unit of total weight
        tol = 1e-12 * np.abs(coeff).sum()
        assert abs(got - ref) <= tol, (n, got, ref)
    # no terms: exactly zero, even after the calls above left partial sums behind
    psi = _state(10, dtype, 3)
    cfh.cfh_expval_noalloc(psi, 10, np.zeros(0, cfh.PAULI_DTYPE), np.zeros(0), out)
    torch.cuda.synchronize()
    assert float(out[0]) == 0.0 and float(out[1]) == 0.0


def test_expval_noalloc_errors():
    psi = _state(6, torch.complex128, 4)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    bad = np.zeros(1, cfh.PAULI_DTYPE)
    bad["x"] = 1 << 6                                   # mask bit at n
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_expval_noalloc(psi, 6, bad, np.ones(1), out)
    assert e.value.code == cfh.CFH_E_RANGE
    odd = np.zeros(1, cfh.PAULI_DTYPE)
    odd["x"], odd["e"] = 1, 1                           # odd phase: not Hermitian
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_expval_noalloc(psi, 6, odd, np.ones(1), out)
    assert e.value.code == cfh.CFH_E_NOT_HERMITIAN
