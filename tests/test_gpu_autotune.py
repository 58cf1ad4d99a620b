"""The autotuner picks a tuning that the library accepts and that is no
slower than the default it was compared with; it caches per device/size."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from paper_2602_09020_amd import autotune, cfh, hybrid

pytestmark = pytest.mark.gpu


def test_tune_plan_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("CFH_TUNING_CACHE", str(tmp_path / "tune.json"))
    w = W.config(2, n=20, n_rot=300, trotter_steps=1)
    rot = hybrid.Frame(w.n).conjugate(cfh.cfh_pauli_encode(w.rot))
    cands = [{"variant": 1, "tile_bits": 11, "low_bits": 4}, {"variant": 3, "tile_bits": 11, "low_bits": 4},
             {"variant": 4, "tile_bits": 13, "low_bits": 3}]
    best = autotune.tune_plan(w.n, torch.complex128, rot, w.theta, candidates=cands)
    assert best in cands
    d = json.load(open(tmp_path / "tune.json"))
    assert any(v["tuning"] == best for v in d.values())
    # second call is served from the cache
    assert autotune.tune_plan(w.n, torch.complex128, rot, w.theta, candidates=[]) == best


def test_tune_batch_returns_accepted_tuning(tmp_path, monkeypatch):
    monkeypatch.setenv("CFH_TUNING_CACHE", str(tmp_path / "tune.json"))
    ws = W.batched_configs(seed=1, count=6, n_range=(12, 14), r_range=(50, 100), n_ham=20)
    cands = [{"tile_bits": 9, "batch_items": 8}, {"tile_bits": 10, "batch_items": 32}]
    best = autotune.tune_batch(ws, torch.complex128, candidates=cands)
    assert best in cands


def test_batch_candidates_change_the_schedule():
    """The batch autotuner's axes are live: the register tile changes how many
    cosets (work items) a pass has and how far rotations fuse, and the fusion
    depth cap changes the pass count."""
    ws = W.batched_configs(seed=2, count=4, n_range=(13, 15), r_range=(200, 300), n_ham=20)
    info = {}
    for rb in (11, 12, 13):
        for mr in (8, 32):
            B = hybrid.Batch(ws, torch.complex128, {"reg_tile_bits": rb, "max_run": mr})
            info[rb, mr] = B.info()
    for rb in (11, 12, 13):
        assert info[rb, 8]["n_passes"] > info[rb, 32]["n_passes"]
    assert len({info[rb, 32]["n_passes"] for rb in (11, 12, 13)}) == 3
    assert len({info[rb, 32]["bytes_fwd"] for rb in (11, 12, 13)}) == 3
    cands = autotune.batch_candidates(torch.complex128)
    assert {c["reg_tile_bits"] for c in cands} == {11, 12, 13} and {c["max_run"] for c in cands} == {8, 32}
    assert {c["variant"] for c in cands} == {0, 1}
    with pytest.raises(cfh.CfhError):
        hybrid.Batch(ws, torch.complex128, {"reg_tile_bits": 14})


def test_tune_batch_skips_schedules_the_batch_cannot_take(tmp_path, monkeypatch):
    """A persistent candidate needs every circuit on the register tile: with
    an 11-qubit circuit in the batch it is skipped, and the level launches win."""
    monkeypatch.setenv("CFH_TUNING_CACHE", str(tmp_path / "tune.json"))
    ws = W.batched_configs(seed=3, count=3, n_range=(12, 13), r_range=(40, 60), n_ham=10)
    ws.append(W.make_workload("n11", 11, seed=4, n_rot=30, n_ham=8))
    cands = [{"variant": 1, "reg_tile_bits": 12, "batch_items": 32}, {"variant": 0, "reg_tile_bits": 12}]
    assert autotune.tune_batch(ws, torch.complex128, candidates=cands, use_cache=False) == cands[1]
