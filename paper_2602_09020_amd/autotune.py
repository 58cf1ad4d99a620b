"""Autotuner for the fused rotation passes and the batched path.

Candidates are timed on the device with the library's own entry points
(``cfh_apply_plan`` / ``cfh_batch_graph_launch``); the fastest one is kept in a
JSON cache keyed by device name, qubit count, storage type and kind, so later
runs reuse it without timing.  The cache lives at ``$CFH_TUNING_CACHE`` or
``~/.cache/cfh_tuning.json``.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional

import numpy as np
import torch

from . import cfh as _c
from . import hybrid

_CACHE_ENV = "CFH_TUNING_CACHE"


def cache_path() -> str:
    return os.environ.get(_CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "cfh_tuning.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _key(kind: str, n: int, dtype) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{kind}|n{n}|{'c128' if hybrid.state_dtype(dtype) == _c.CFH_C128 else 'c64'}"


def plan_candidates(n: int, dtype) -> List[dict]:
    """Kernel variant x tile bits x contiguous low bits, within each kernel's limits."""
    c128 = hybrid.state_dtype(dtype) == _c.CFH_C128
    out = []
    tb_max = min(n, 14)
    for tb in range(max(8, min(n, 10)), tb_max + 1):
        for lb in (3, 4, 5, 6):
            if lb >= tb:
                continue
            if tb <= (13 if c128 else 14):
                out.append({"variant": 1, "tile_bits": tb, "low_bits": lb})
            if 10 <= tb <= 13:
                out.append({"variant": 4, "tile_bits": tb, "low_bits": lb})
            if 10 <= tb <= 14:
                out.append({"variant": 5, "tile_bits": tb, "low_bits": lb})
    return out


def _time_plan(n: int, dtype, rot: np.ndarray, theta: torch.Tensor, psi: torch.Tensor, tuning: dict,
               reps: int) -> float:
    plan = hybrid.Plan(n, dtype, rot, tuning)
    plan.apply(psi, theta)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.apply(psi, theta)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_plan(n: int, dtype, rot: np.ndarray, theta: np.ndarray, candidates: Optional[Iterable[dict]] = None,
              reps: int = 2, use_cache: bool = True, verbose: bool = False) -> dict:
    """Fastest tuning for applying ``rot`` (a representative sample of the
    rotations, already conjugated) on an n-qubit state."""
    key = _key("plan", n, dtype)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]["tuning"]
    psi = hybrid.new_state(n, dtype)
    th = torch.tensor(np.asarray(theta, np.float64), device="cuda")
    best, best_ms = None, float("inf")
    for tu in (candidates if candidates is not None else plan_candidates(n, dtype)):
        try:
            ms = _time_plan(n, dtype, rot, th, psi, tu, reps)
        except _c.CfhError:
            continue
        if verbose:
            print(f"autotune plan n={n} {tu}: {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = tu, ms
    if best is None:
        raise RuntimeError("autotune: no candidate tuning ran")
    if use_cache:
        cache = _load()
        cache[key] = {"tuning": best, "ms": best_ms, "rotations": int(rot.shape[0])}
        _store(cache)
    return best


def batch_candidates(dtype) -> List[dict]:
    """Schedule x register tile x fusion depth x work items per pass.  Level
    launches (variant 0): register tile 2^11..2^13 amplitudes (for circuits
    with at least that many qubits) x fusion depth (the most rotations one
    pass may carry) x work items per pass, the LDS tile of the smaller
    circuits at its default.  One persistent kernel per run (variant 1, only
    where every circuit fits the register tile): 2^12 tiles, both depths, 32
    items per pass (fewer, larger items: each one costs a claim and a
    device-scope release)."""
    c128 = hybrid.state_dtype(dtype) == _c.CFH_C128
    lb = 10 if c128 else 11
    levels = [{"variant": 0, "tile_bits": lb, "reg_tile_bits": rb, "max_run": mr, "batch_items": it, "group_mib": 0}
              for rb in (11, 12, 13) for mr in (8, 32) for it in (64, 128)]
    persistent = [{"variant": 1, "tile_bits": lb, "reg_tile_bits": 12, "max_run": mr, "batch_items": 32,
                   "group_mib": 0} for mr in (8, 32)]
    return levels + persistent


def _time_batch(B, with_grad: bool, s, reps: int) -> float:
    """Median over reps replays of the captured graph (one warm-up replay first)."""
    B.graph_launch(with_grad, s)
    B.results(stream=s)
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        B.graph_launch(with_grad, s)
        b.record(s)
        B.results(stream=s)
        ms.append(a.elapsed_time(b))
    return float(np.median(ms))


def tune_batch(workloads, dtype, candidates: Optional[Iterable[dict]] = None, with_grad: bool = True,
               use_cache: bool = True, verbose: bool = False, reps: int = 3) -> Dict:
    """Fastest batch tuning (schedule, register tile, fusion depth, items per
    pass, LDS tile, cache groups) for a batch of circuits, each candidate
    timed as the median of ``reps`` replays of its captured graph; candidates
    the batch cannot take (a persistent schedule with circuits below the
    register tile) are skipped."""
    key = _key(f"batch{len(workloads)}", max(w.n for w in workloads), dtype)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]["tuning"]
    s = torch.cuda.Stream()
    best, best_ms = None, float("inf")
    for tu in (candidates if candidates is not None else batch_candidates(dtype)):
        try:
            B = hybrid.Batch(workloads, dtype, tu)
        except _c.CfhError:
            continue
        ms = _time_batch(B, with_grad, s, reps)
        del B
        if verbose:
            print(f"autotune batch {tu}: {ms:.2f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = tu, ms
    if best is None:
        raise RuntimeError("autotune: no candidate tuning ran")
    if use_cache:
        cache = _load()
        cache[key] = {"tuning": best, "ms": best_ms}
        _store(cache)
    return best
