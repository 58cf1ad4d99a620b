"""CPU tests of the libcfh boundary and its host logic (no device calls).

* the library loads and exports every function include/cfh.h declares, and
  the Python binding declares the same set;
* the frame tracker is bit-exact (x, z and sign) against the oracle's
  independent Heisenberg walk, whose letter tables come from gate matrices;
* the fusion planner's schedules keep every rotation once, keep the relative
  order of anticommuting rotations, and fit each pass into a tile subspace;
* error paths return the documented status codes.
"""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2602_09020_amd import cfh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfh.h")


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:cfh_status|int|const char \*)\s*(cfh_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    declared = header_functions()
    assert len(declared) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", cfh.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (cfh_\w+)$", out, re.M))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    lib = cfh.lib()
    for f in declared:
        assert hasattr(lib, f)
    assert sorted(cfh.declared_symbols()) == declared


def test_version_and_device_count():
    assert cfh.cfh_version() == 1
    assert cfh.cfh_device_count() >= 0


def letters_to_pauli(rows, phases=None):
    rows = np.asarray(rows)
    out = np.zeros(rows.shape[0], cfh.PAULI_DTYPE)
    for i, r in enumerate(rows):
        x = sum(1 << j for j, l in enumerate(r) if l in (1, 2))
        z = sum(1 << j for j, l in enumerate(r) if l in (2, 3))
        out[i] = (x, z, 0 if phases is None else int(phases[i]) & 3, 0)
    return out


def test_encode_matches_mask_definition():
    rng = np.random.default_rng(0)
    rows = rng.integers(0, 4, size=(50, 37)).astype(np.uint8)
    assert np.array_equal(cfh.cfh_pauli_encode(rows), letters_to_pauli(rows))
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_pauli_encode(np.array([[0, 4]], np.uint8))
    assert e.value.code == cfh.CFH_E_INVAL


def random_gates(rng, n, m):
    g = []
    for _ in range(m):
        code = int(rng.integers(0, 9))
        q0, q1 = (int(v) for v in rng.choice(n, 2, replace=False))
        g.append((code, q0, q1 if code >= 6 else -1))
    return np.array(g, np.int32)


@pytest.mark.parametrize("n,m,seed", [(2, 30, 0), (5, 200, 1), (10, 50, 2), (24, 500, 3), (63, 400, 4)])
def test_frame_rows_bit_exact_vs_heisenberg_walk(n, m, seed):
    rng = np.random.default_rng(seed)
    gates = random_gates(rng, n, m)
    f = cfh.cfh_frame_create(n)
    try:
        cfh.cfh_frame_apply_gates(f, gates)
        zl, zph, xl, xph = sim.frame_rows(gates, n)
        ez, ex = letters_to_pauli(zl, zph), letters_to_pauli(xl, xph)
        for q in range(n):
            rz, rx = cfh.cfh_frame_row(f, q)
            assert rz == (int(ez[q]["x"]), int(ez[q]["z"]), int(ez[q]["e"])), q
            assert rx == (int(ex[q]["x"]), int(ex[q]["z"]), int(ex[q]["e"])), q
    finally:
        cfh.cfh_frame_destroy(f)


@pytest.mark.parametrize("cfg", [0, 1])
def test_frame_conjugation_bit_exact_on_workloads(cfg):
    """F(P) for every rotation and observable term of configurations 0 and 1
    (10 qubits / 50-gate prefix, 24 qubits / 500-gate prefix)."""
    w = W.config(cfg, n_rot=300 if cfg == 1 else None)
    f = cfh.cfh_frame_create(w.n)
    try:
        cfh.cfh_frame_apply_gates(f, w.prefix)
        for rows in (w.rot, w.ham[:200]):
            got = cfh.cfh_frame_conjugate_many(f, cfh.cfh_pauli_encode(rows))
            ol, oph = sim.heisenberg_many(w.prefix, rows)
            assert np.array_equal(got, letters_to_pauli(ol, oph))
            assert np.all(got["e"] % 2 == 0)
    finally:
        cfh.cfh_frame_destroy(f)


def test_frame_conjugation_all_phases_and_letters():
    """Every one- and two-letter string with every phase, through random circuits."""
    rng = np.random.default_rng(9)
    n = 4
    for _ in range(20):
        gates = random_gates(rng, n, 25)
        f = cfh.cfh_frame_create(n)
        cfh.cfh_frame_apply_gates(f, gates)
        for _ in range(30):
            row = rng.integers(0, 4, size=n).astype(np.uint8)
            ph = int(rng.integers(0, 4))
            ol, oph = sim.heisenberg(gates, row, ph)
            p = letters_to_pauli([row], [ph])[0]
            got = cfh.cfh_frame_conjugate(f, int(p["x"]), int(p["z"]), ph)
            e = letters_to_pauli([ol], [oph])[0]
            assert got == (int(e["x"]), int(e["z"]), int(e["e"]))
        cfh.cfh_frame_destroy(f)


def test_frame_error_codes():
    f = cfh.cfh_frame_create(3)
    try:
        for args in [(cfh.CFH_GATE_H, 3, -1), (cfh.CFH_GATE_CNOT, 0, 0), (cfh.CFH_GATE_H, 0, 1), (99, 0, -1)]:
            with pytest.raises(cfh.CfhError) as e:
                cfh.cfh_frame_apply_clifford(f, *args)
            assert e.value.code == cfh.CFH_E_INVAL
        with pytest.raises(cfh.CfhError) as e:
            cfh.cfh_frame_conjugate(f, 1 << 3, 0)
        assert e.value.code == cfh.CFH_E_RANGE
    finally:
        cfh.cfh_frame_destroy(f)
    with pytest.raises(cfh.CfhError):
        cfh.cfh_frame_create(0)
    with pytest.raises(cfh.CfhError):
        cfh.cfh_frame_create(64)


# ------------------------------------------------------------------ planner

def anticommute(a, b):
    return (bin(int(a["x"]) & int(b["z"])).count("1") + bin(int(a["z"]) & int(b["x"])).count("1")) % 2 == 1


def gf2_rank(vectors):
    basis = []
    for v in vectors:
        for b in basis:
            v = min(v, v ^ b)
        if v:
            basis.append(v)
    return len(basis)


@pytest.mark.parametrize("cfg,n,tb,lb", [(2, 28, 12, 5), (2, 20, 10, 4), (1, 16, 12, 5), (3, 20, 11, 5),
                                         (0, 10, 6, 3), (2, 14, 13, 6)])
def test_planner_schedule_invariants(cfg, n, tb, lb):
    kw = {"n": n}
    if cfg == 2:
        kw.update(n_rot=400, trotter_steps=2)
    elif cfg == 1:
        kw.update(n_rot=400)
    w = W.config(cfg, **kw)
    f = cfh.cfh_frame_create(n)
    cfh.cfh_frame_apply_gates(f, w.prefix)
    rot = cfh.cfh_frame_conjugate_many(f, cfh.cfh_pauli_encode(w.rot))
    cfh.cfh_frame_destroy(f)
    ps, order = cfh.cfh_plan_dry_run(n, cfh.CFH_C128, rot, {"tile_bits": tb, "low_bits": lb})
    m = rot.shape[0]
    assert sorted(order.tolist()) == list(range(m))          # each rotation exactly once
    pos = np.empty(m, np.int64)
    pos[order] = np.arange(m)
    # anticommuting pairs keep their order (commuting ones may swap)
    for i in range(m):
        for j in range(i + 1, min(m, i + 200)):
            if pos[j] < pos[i]:
                assert not anticommute(rot[i], rot[j]), (i, j)
    lowv = [1 << j for j in range(min(lb, tb))]
    for p in range(len(ps) - 1):
        xs = [int(rot[k]["x"]) for k in order[ps[p]:ps[p + 1]]]
        assert 1 <= len(xs) <= 32
        assert gf2_rank(lowv + xs) <= tb                    # fits one tile subspace
    # fusion actually fuses: at least b - c rotations per pass on average (JW x masks)
    if cfg in (2, 3):
        assert m / (len(ps) - 1) >= tb - lb


def test_planner_in_order_mode_and_unfused():
    w = W.config(2, n=20, n_rot=100, trotter_steps=1)
    rot = cfh.cfh_pauli_encode(w.rot)
    ps, order = cfh.cfh_plan_dry_run(20, cfh.CFH_C64, rot, {"lookahead": -1})
    assert order.tolist() == list(range(100))
    ps, order = cfh.cfh_plan_dry_run(20, cfh.CFH_C64, rot, {"unfused": 1})
    assert len(ps) == 101


def test_planner_rejects_bad_input():
    p = np.zeros(1, cfh.PAULI_DTYPE)
    p[0] = (1, 0, 1, 0)
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_plan_dry_run(4, cfh.CFH_C128, p)
    assert e.value.code == cfh.CFH_E_NOT_HERMITIAN
    p[0] = (1 << 4, 0, 0, 0)
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_plan_dry_run(4, cfh.CFH_C128, p)
    assert e.value.code == cfh.CFH_E_RANGE
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_plan_dry_run(35, cfh.CFH_C128, np.zeros(0, cfh.PAULI_DTYPE))
    assert e.value.code == cfh.CFH_E_UNSUPPORTED


def test_batch_rejects_persistent_variant_below_register_tile_without_device_work():
    """A persistent batch (variant 1) runs register-tiled passes only: a
    circuit below the register tile fails in argument checking, before any
    device allocation."""
    import ctypes as C
    rot = cfh.cfh_pauli_encode(np.array([[1, 3, 1, 0, 0, 0, 0, 0]], np.uint8))
    circ = [{"n": 8, "init_index": 0, "rot": rot, "theta": np.array([0.3]), "terms": rot, "coeff": np.array([1.0])}]
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_batch_create(circ, cfh.CFH_C128, {"variant": 1})
    assert e.value.code == cfh.CFH_E_UNSUPPORTED


def test_autotune_candidates_respect_kernel_limits():
    import torch
    from paper_2602_09020_amd import autotune
    for n in (10, 16, 20, 28):
        for dt in (torch.complex128, torch.complex64):
            for tu in autotune.plan_candidates(n, dt):
                assert tu["low_bits"] < tu["tile_bits"] <= n
                if tu["variant"] in (3, 4):
                    assert 10 <= tu["tile_bits"] <= 13
                if tu["variant"] == 5:
                    assert 10 <= tu["tile_bits"] <= 14
                if dt == torch.complex128 and tu["variant"] == 1:
                    assert tu["tile_bits"] <= 13
