"""Calls from several host threads at once.

Four threads, each with its own plan, observable, state and stream, apply
their rotations, H psi and <H> concurrently, ten times over; the binding
releases the interpreter lock inside every library call, so the launches
really overlap on the host.  The tile sizes differ per thread, so different
kernel instantiations start at the same time.  Every final state, H psi and
energy must equal, bit for bit, the same calls made one after another (the
kernels reduce in a fixed order).
"""
import threading

import numpy as np
import pytest
import torch

import workloads as W
from paper_2602_09020_amd import cfh, hybrid

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _jobs(dtype):
    jobs = []
    for k, (n, tb, mt) in enumerate([(16, 10, 10), (17, 12, 11), (18, 13, 12), (19, 11, 13)]):
        w = W.make_workload(f"thr{k}", n, seed=70 + k, n_prefix=2 * n, n_rot=300, n_ham=60)
        _, _, _, plan, ham = hybrid.prepare(w, dtype, {"tile_bits": tb}, {"tile_bits": mt})
        jobs.append((w, plan, ham, torch.tensor(w.theta, device=DEV)))
    return jobs


def _run(job, dtype, stream, reps):
    w, plan, ham, theta = job
    with torch.cuda.stream(stream):  # torch's fills go to the thread's stream too
        psi = torch.empty(1 << w.n, dtype=dtype, device=DEV)
        out = torch.zeros(2, dtype=torch.float64, device=DEV)
        hpsi = torch.empty_like(psi)
    for _ in range(reps):
        cfh.cfh_state_set_basis(psi, w.n, w.init, stream=stream)
        plan.apply(psi, theta, stream=stream)
        ham.apply(psi, hpsi, stream=stream)
        ham.expval_async(psi, out, stream=stream)
    return psi, hpsi, out


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_concurrent_threads_match_serial_calls(dtype):
    jobs = _jobs(dtype)
    torch.cuda.synchronize()  # angles copied to the device before the threads start
    got = [None] * len(jobs)
    errors = []
    streams = [torch.cuda.Stream() for _ in jobs]

    def worker(i):
        try:
            r = _run(jobs[i], dtype, streams[i], 10)
            streams[i].synchronize()
            got[i] = r
        except Exception as e:  # reported below, on the main thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    torch.cuda.synchronize()
    for i, job in enumerate(jobs):
        s = torch.cuda.Stream()
        psi, hpsi, out = _run(job, dtype, s, 1)
        s.synchronize()
        assert torch.equal(got[i][0], psi), i
        assert torch.equal(got[i][1], hpsi), i
        assert torch.equal(got[i][2], out), i
        assert np.isfinite(out.cpu().numpy()).all()
