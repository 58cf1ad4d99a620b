"""GPU tests of the persistent batched schedule (tuning variant 1: one
persistent kernel per run, items claimed from a device counter, bounded
dependency waits).  The first test forces every wait to give up from the
host, so the kernel's own bound ends the run."""
import time

import numpy as np
import pytest
import torch

import workloads as W
from oracle import sim
from paper_2602_09020_amd import cfh, hybrid

pytestmark = pytest.mark.gpu


def _batch(seed=0, count=6, n_range=(12, 14), r_range=(40, 120), n_ham=20):
    return W.batched_configs(seed=seed, count=count, n_range=n_range, r_range=r_range, n_ham=n_ham)


def _run(B, with_grad, stream=None):
    B.run(with_grad=with_grad, stream=stream)
    r = B.results(stream=stream)
    return r, [B.state(i, stream=stream).cpu() for i in range(B.count)]


def test_persistent_run_gives_up_through_its_bounded_wait():
    """hold = 1: every dependency wait needs a ready value no workgroup ever
    writes, so each wait runs out (5 ms), raises the abort word, and every
    workgroup leaves; the results call reports CFH_E_TIMEOUT.  With the hold
    released the same batch then runs to the level launches' results."""
    ws = _batch(seed=11)
    B = hybrid.Batch(ws, torch.complex128, {"variant": 1, "batch_items": 4})
    print("persistent give-up: forward run, 6 circuits, hold", flush=True)
    cfh.cfh_batch_persist_config(B.h, max_wait_s=0.005, hold=True)
    for with_grad in (False, True):
        t0 = time.perf_counter()
        B.run(with_grad=with_grad)
        with pytest.raises(cfh.CfhError) as e:
            B.results()
        assert e.value.code == cfh.CFH_E_TIMEOUT
        assert time.perf_counter() - t0 < 10.0
    print("persistent give-up: released", flush=True)
    cfh.cfh_batch_persist_config(B.h, max_wait_s=2.0, hold=False)
    ref = hybrid.Batch(ws, torch.complex128, {"variant": 0, "batch_items": 4})
    for with_grad in (False, True):
        r, st = _run(B, with_grad)
        r0, st0 = _run(ref, with_grad)
        assert np.array_equal(r["energy"], r0["energy"])
        if with_grad:
            for a, b in zip(r["grad"], r0["grad"]):
                assert np.array_equal(a, b)
        for a, b in zip(st, st0):
            assert torch.equal(a, b)
    info = cfh.cfh_batch_persist_info(B.h)
    assert info["grid"] > 0 and info["tickets_grad"] > info["tickets_fwd"] > 0


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-4)])
def test_persistent_matches_level_launches_and_oracle(dtype, tol):
    """The same work items and the same fixed-order reductions as the level
    launches: states, energies and gradients bitwise equal; states and
    energies against the oracle, gradients against its parameter shift
    (complex64: 1e-4 times the observable's coefficient sum, as for the level
    launches)."""
    ws = _batch(seed=12, count=7, n_range=(12, 15), r_range=(60, 160), n_ham=24)
    out = {}
    for variant in (0, 1):
        B = hybrid.Batch(ws, dtype, {"variant": variant, "batch_items": 4})
        print(f"variant {variant} {dtype}", flush=True)
        out[variant] = (_run(B, False), _run(B, True))
    for k in (0, 1):
        (r1, s1), (r0, s0) = out[1][k], out[0][k]
        assert np.array_equal(r1["energy"], r0["energy"]), k
        for a, b in zip(s1, s0):
            assert torch.equal(a, b), k
        if k:
            for a, b in zip(r1["grad"], r0["grad"]):
                assert np.array_equal(a, b)
        assert np.all(r1["t_end"] >= r1["t_start"]) and np.all(r1["t_start"] > 0)
    (rf, sf), (rg, _) = out[1]
    for i, w in enumerate(ws[:4]):
        psi, phi = sim.simulate(w)
        scale = np.abs(w.coeff).sum()
        assert np.abs(sf[i].to(torch.complex128).numpy() - phi).max() <= tol, i
        assert abs(rf["energy"][i] - sim.energy(psi, w.n, w.ham, w.coeff)) <= tol * scale, i
    gtol = 1e-10 if dtype == torch.complex128 else None
    for i, w in enumerate(ws[:2]):
        ps = sim.param_shift_grad(w)
        bound = gtol if gtol is not None else 1e-4 * np.abs(w.coeff).sum()
        assert np.abs(rg["grad"][i] - ps).max() <= bound, i


@pytest.mark.parametrize("max_grid", [1, 3])
def test_persistent_completes_on_few_workgroups(max_grid):
    """Items go only to running workgroups, in the claim order, so the run
    needs no particular number of resident workgroups: one workgroup, or
    three, runs every item and gets the full grid's results bitwise."""
    ws = _batch(seed=13, count=5, n_range=(12, 13), r_range=(30, 80), n_ham=12)
    B = hybrid.Batch(ws, torch.complex128, {"variant": 1, "batch_items": 3})
    full = (_run(B, False), _run(B, True))
    print(f"persistent grid capped at {max_grid}", flush=True)
    cfh.cfh_batch_persist_config(B.h, max_wait_s=2.0, hold=False, max_grid=max_grid)
    few = (_run(B, False), _run(B, True))
    assert cfh.cfh_batch_persist_info(B.h)["grid"] == max_grid
    for k in (0, 1):
        assert np.array_equal(few[k][0]["energy"], full[k][0]["energy"])
        for a, b in zip(few[k][1], full[k][1]):
            assert torch.equal(a, b)
    for a, b in zip(few[1][0]["grad"], full[1][0]["grad"]):
        assert np.array_equal(a, b)


def test_persistent_hipgraph_replays():
    """Reset kernel + persistent kernel captured once and replayed, with eager
    work between replays: every replay equals the eager run."""
    ws = _batch(seed=14, count=8, n_range=(12, 15), r_range=(60, 200), n_ham=30)
    B = hybrid.Batch(ws, torch.complex128, {"variant": 1})
    s = torch.cuda.Stream()
    for with_grad in (True, False):
        B.run(with_grad=with_grad, stream=s)
        ref = B.results(stream=s)
        for rep in range(3):
            B.graph_launch(with_grad, s)
            got = B.results(stream=s)
            assert np.array_equal(got["energy"], ref["energy"]), rep
            for a, b in zip(got["grad"], ref["grad"]):
                assert np.array_equal(a, b), rep
            x = torch.randn(1 << 16, device="cuda")
            (x * 2).sum().item()


def test_persistent_config_replaces_captured_graphs():
    """A captured graph holds the persistent kernel's arguments: changing the
    wait limit or the hold drops the graphs, so the next graph launch captures
    the new arguments (hold: the replay gives up; released: the eager results
    again).  Bad arguments are rejected."""
    ws = _batch(seed=16, count=5, n_range=(12, 13), r_range=(30, 80), n_ham=12)
    B = hybrid.Batch(ws, torch.complex128, {"variant": 1, "batch_items": 4})
    s = torch.cuda.Stream()
    B.run(with_grad=True, stream=s)
    ref = B.results(stream=s)
    B.graph_launch(True, s)
    assert np.array_equal(B.results(stream=s)["energy"], ref["energy"])
    cfh.cfh_batch_persist_config(B.h, max_wait_s=0.005, hold=True)
    B.graph_launch(True, s)
    with pytest.raises(cfh.CfhError) as e:
        B.results(stream=s)
    assert e.value.code == cfh.CFH_E_TIMEOUT
    cfh.cfh_batch_persist_config(B.h, max_wait_s=2.0, hold=False)
    B.graph_launch(True, s)
    got = B.results(stream=s)
    assert np.array_equal(got["energy"], ref["energy"])
    for a, b in zip(got["grad"], ref["grad"]):
        assert np.array_equal(a, b)
    for bad in ((0.0, False, 0), (601.0, False, 0), (1.0, False, -1)):
        with pytest.raises(cfh.CfhError) as e:
            cfh.cfh_batch_persist_config(B.h, *bad)
        assert e.value.code == cfh.CFH_E_INVAL


def test_persistent_rejects_circuits_below_the_register_tile():
    ws = _batch(seed=15, count=3, n_range=(11, 13))
    ws[0] = W.make_workload("small", 11, seed=1, n_rot=20, n_ham=5)
    with pytest.raises(cfh.CfhError) as e:
        hybrid.Batch(ws, torch.complex128, {"variant": 1})
    assert e.value.code == cfh.CFH_E_UNSUPPORTED
    B = hybrid.Batch(ws[1:], torch.complex128, {"variant": 0})
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_batch_persist_config(B.h, 1.0, False, 0)
    assert e.value.code == cfh.CFH_E_UNSUPPORTED


@pytest.fixture(scope="module")
def full_batch():
    """The 256-circuit workload the bench times, with three sampled circuits
    (the 12-qubit one with the fewest rotations, a 16-qubit one, the 20-qubit
    one with the fewest rotations), their oracle energies, and the oracle's
    parameter-shift gradient of the 12-qubit one at four seeded indices."""
    ws = W.batched_configs()
    ns = np.array([w.n for w in ws])
    rs = np.array([w.n_rot for w in ws])
    sample = [int(np.where(ns == 12)[0][np.argmin(rs[ns == 12])]), int(np.where(ns == 16)[0][0]),
              int(np.where(ns == 20)[0][np.argmin(rs[ns == 20])])]
    energies = {i: sim.energy_of(ws[i], ws[i].theta) for i in sample}
    g_idx = np.sort(np.random.default_rng(21).choice(ws[sample[0]].n_rot, size=4, replace=False))
    grads = sim.param_shift_grad(ws[sample[0]], g_idx)
    return ws, sample, energies, g_idx, grads


@pytest.mark.parametrize("dtype,tol,max_run", [(torch.complex128, 1e-12, 32), (torch.complex64, 1e-4, 8)])
def test_full_batch_both_schedules_vs_oracle(full_batch, dtype, tol, max_run):
    """The bench's 256-circuit batch on 2^12 register tiles: the level
    launches at the bench's 128 items per pass, and both schedules at 32
    items per pass, which give bitwise the same energies and gradients (the
    same items and reductions).  For every run: sampled circuits' energies
    against the oracle (tol times the coefficient sum) and four gradients of
    the 12-qubit circuit against the oracle's parameter shift (1e-10 at
    complex128; 1e-4 times the coefficient sum at complex64)."""
    ws, sample, energies, g_idx, grads = full_batch
    out = {}
    for variant, items in ((0, 128), (0, 32), (1, 32)):
        print(f"full batch variant {variant} {dtype}", flush=True)
        B = hybrid.Batch(ws, dtype, {"variant": variant, "reg_tile_bits": 12, "max_run": max_run,
                                     "batch_items": items})
        B.run(with_grad=False)
        rf = B.results()
        B.run(with_grad=True)
        out[variant, items] = (rf, B.results())
        del B
        torch.cuda.empty_cache()
    for k in (0, 1):
        r0, r1 = out[0, 32][k], out[1, 32][k]
        assert np.array_equal(r0["energy"], r1["energy"]), k
        assert np.all(r1["t_end"] >= r1["t_start"]) and np.all(r1["t_start"] > 0)
    for a, b in zip(out[0, 32][1]["grad"], out[1, 32][1]["grad"]):
        assert np.array_equal(a, b)
    i0 = sample[0]
    bound = 1e-10 if dtype == torch.complex128 else 1e-4 * np.abs(ws[i0].coeff).sum()
    for key, (rf, rg) in out.items():
        for i in sample:
            scale = np.abs(ws[i].coeff).sum()
            assert abs(rf["energy"][i] - energies[i]) <= tol * scale, (key, i)
            assert abs(rg["energy"][i] - energies[i]) <= tol * scale, (key, i)
        assert np.abs(rg["grad"][i0][g_idx] - grads).max() <= bound, key
