"""Host planning of the register-tiled <H> passes (cfh_ham_dry_run, no GPU).

Eq. chfsexp is summed pass by pass: a pass reads every coset of its tile once
and adds the terms whose x masks lie in the tile's span.  For the plan to be
that sum, every term must sit in exactly one pass, inside its pass's span,
with at most 32 terms per pass (the kernel's descriptor slots); the tile must
be spanned by independent masks that include the low index bits (the
contiguous runs the kernel reads).  Checked on the 28-qubit JW observable and
on the 24-qubit one after its 500-gate Clifford prefix (dense masks), at both
storage types and several tile sizes, with a guard on the pass counts the
greedy planner reaches.
"""
import numpy as np
import pytest

import workloads as W
from paper_2602_09020_amd import cfh, hybrid


def _reduce(x, piv):
    """x reduced against a GF(2) basis kept as {pivot bit: vector}."""
    for p in sorted(piv, reverse=True):
        if (x >> p) & 1:
            x ^= piv[p]
    return x


def _span(vectors):
    piv = {}
    for v in vectors:
        r = _reduce(int(v), piv)
        if r:
            piv[r.bit_length() - 1] = r
    return piv


def _check_plan(n, terms, plan, low_bits):
    ps, order, bits, basis = plan
    m = terms.shape[0]
    P = len(ps) - 1
    assert sorted(order.tolist()) == list(range(m))          # each term exactly once
    assert ps[0] == 0 and ps[-1] == m and np.all(np.diff(ps) >= 1)
    assert np.all(np.diff(ps) <= 32)
    for p in range(P):
        b = int(bits[p])
        vecs = [int(v) for v in basis[p, :b]]
        assert all(int(v) == 0 for v in basis[p, b:])
        piv = _span(vecs)
        assert len(piv) == b                                   # independent
        assert all(v < (1 << n) for v in vecs)
        for j in range(min(low_bits, b)):
            assert _reduce(1 << j, piv) == 0                   # the contiguous low bits
        for t in order[ps[p]:ps[p + 1]]:
            assert _reduce(int(terms[t]["x"]), piv) == 0        # the term's partner lies in the tile
    return P


def _observable(cfg):
    w = W.config(cfg)
    f = hybrid.Frame(w.n)
    f.apply_gates(w.prefix)
    return w.n, f.conjugate(cfh.cfh_pauli_encode(w.ham))


@pytest.mark.parametrize("dtype,tuning,low", [
    (cfh.CFH_C128, None, 3), (cfh.CFH_C64, None, 4),
    (cfh.CFH_C128, {"tile_bits": 12, "low_bits": 3}, 3), (cfh.CFH_C128, {"tile_bits": 14, "low_bits": 4}, 4),
    (cfh.CFH_C64, {"tile_bits": 10, "low_bits": 2}, 2), (cfh.CFH_C128, {"variant": 5, "tile_bits": 13, "low_bits": 3}, 3),
])
def test_trotter_observable_plan_is_a_partition_into_tile_spans(dtype, tuning, low):
    n, terms = _observable(2)
    P = _check_plan(n, terms, cfh.cfh_ham_dry_run(n, dtype, terms, tuning), low)
    if tuning is None and dtype == cfh.CFH_C128:
        assert P <= 99, P      # 2^11 tiles: 99 passes; whole-qubit covering needed 105 on larger tiles


@pytest.mark.parametrize("dtype,low", [(cfh.CFH_C128, 3), (cfh.CFH_C64, 4)])
def test_prefixed_observable_plan_is_a_partition_into_tile_spans(dtype, low):
    """After the Clifford prefix the masks are dense (mean weight 12)."""
    n, terms = _observable(1)
    P = _check_plan(n, terms, cfh.cfh_ham_dry_run(n, dtype, terms), low)
    if dtype == cfh.CFH_C128:
        assert P <= 280, P     # whole-qubit covering needed 1,647 passes on 2^13 tiles


def test_large_x_groups_split_and_diagonal_terms():
    """40 terms sharing one x mask (more than one pass holds) and 20 diagonal
    terms (x = 0, in every tile's span) beside random dense strings."""
    n = 16
    rng = np.random.default_rng(3)
    same = np.where(rng.integers(0, 2, size=(40, n)) == 1, 3, 0).astype(np.uint8)
    same[:, 0] = 1
    same[:, 3] = 2
    diag = np.where(rng.integers(0, 2, size=(20, n)) == 1, 3, 0).astype(np.uint8)
    dense = rng.integers(0, 4, size=(60, n)).astype(np.uint8)
    terms = cfh.cfh_pauli_encode(np.concatenate([dense, same, diag]))
    plan = cfh.cfh_ham_dry_run(n, cfh.CFH_C128, terms)
    _check_plan(n, terms, plan, 3)
    ps, order = plan[0], plan[1]
    where = {int(t): p for p in range(len(ps) - 1) for t in order[ps[p]:ps[p + 1]]}
    assert len({where[60 + k] for k in range(40)}) >= 2


def test_dry_run_errors_and_empty():
    n = 12
    ps, order, bits, basis = cfh.cfh_ham_dry_run(n, cfh.CFH_C128, np.zeros(0, cfh.PAULI_DTYPE))
    assert len(ps) == 1 and ps[0] == 0
    t = cfh.cfh_pauli_encode(np.array([[1] + [0] * (n - 1)], np.uint8))
    for tuning, terms, code in [({"variant": 1}, t, cfh.CFH_E_UNSUPPORTED),       # LDS-staged <H>
                                ({"tile_bits": 8}, t, cfh.CFH_E_UNSUPPORTED)]:
        with pytest.raises(cfh.CfhError) as e:
            cfh.cfh_ham_dry_run(n, cfh.CFH_C128, terms, tuning)
        assert e.value.code == code
    bad = t.copy()
    bad["e"] = 1                                                                   # i * X: not Hermitian
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_ham_dry_run(n, cfh.CFH_C128, bad)
    assert e.value.code == cfh.CFH_E_NOT_HERMITIAN
    far = t.copy()
    far["x"] = 1 << n                                                              # a qubit past n
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_ham_dry_run(n, cfh.CFH_C128, far)
    assert e.value.code == cfh.CFH_E_RANGE
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_ham_dry_run(35, cfh.CFH_C128, t)
    assert e.value.code == cfh.CFH_E_UNSUPPORTED
