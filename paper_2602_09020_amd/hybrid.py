"""Handle classes over the libcfh C ABI and the adjoint autograd Function.

Each method forwards to one C entry point (argument marshalling only).  The
hybrid state (F, Phi) of Sec. 4.2 is a ``Frame`` next to a device tensor.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import cfh as _c


def state_dtype(dtype) -> int:
    return _c.CFH_C128 if dtype in (torch.complex128, _c.CFH_C128) else _c.CFH_C64


class Frame:
    """Pauli frame in the backward interpretation (Sec. 4.1)."""

    def __init__(self, n: int):
        self.n = n
        self.h = _c.cfh_frame_create(n)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _c is not None:  # None once the interpreter tears modules down
            _c.cfh_frame_destroy(h)
            self.h = None

    def apply_clifford(self, gate: int, q0: int, q1: int = -1) -> None:
        _c.cfh_frame_apply_clifford(self.h, gate, q0, q1)

    def apply_gates(self, gates: np.ndarray) -> None:
        _c.cfh_frame_apply_gates(self.h, gates)

    def row(self, q: int):
        return _c.cfh_frame_row(self.h, q)

    def conjugate(self, paulis: np.ndarray) -> np.ndarray:
        return _c.cfh_frame_conjugate_many(self.h, paulis)

    def conjugate_device(self, paulis_dev: torch.Tensor, out_dev: torch.Tensor, m: int, stream=None) -> None:
        _c.cfh_frame_conjugate_device(self.h, paulis_dev, out_dev, m, stream)

    def flush_rotations(self):
        """(paulis, theta) whose rotations, applied in order, take Phi to U Phi."""
        return _c.cfh_frame_flush_rotations(self.h, self.n)

    def translate(self, gates: np.ndarray, angles: Optional[np.ndarray] = None):
        """Absorb the circuit's Cliffords; return its rotations on Phi (paulis, theta)."""
        return _c.cfh_circuit_translate(self.h, gates, angles)

    def run_circuit(self, gates: np.ndarray, angles: Optional[np.ndarray], psi: torch.Tensor,
                    tuning: Optional[dict] = None, stream=None) -> np.ndarray:
        """Cliffords into the frame, rotations onto psi as fused plans between
        measurements (synchronous); returns the measurement/reset outcomes."""
        return _c.cfh_circuit_run(self.h, gates, angles, psi, tuning, stream)

    def flush(self, psi: torch.Tensor, stream=None) -> None:
        """psi <- U psi (up to a global phase) on the device; the frame becomes the identity."""
        _c.cfh_frame_flush(self.h, psi, stream)


class Plan:
    """Fused (or unfused) schedule of a rotation sequence on n qubits."""

    def __init__(self, n: int, dtype, rot: np.ndarray, tuning: Optional[dict] = None):
        self.n = n
        self.dtype = state_dtype(dtype)
        self.m = int(rot.shape[0])
        self.h = _c.cfh_plan_create(n, self.dtype, rot, tuning)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _c is not None:  # None once the interpreter tears modules down
            _c.cfh_plan_destroy(h)
            self.h = None

    def info(self) -> dict:
        return _c.cfh_plan_info(self.h)

    def schedule(self):
        return _c.cfh_plan_schedule(self.h, self.m, self.info()["n_passes"])

    def apply(self, psi: torch.Tensor, theta_dev: torch.Tensor, inverse: bool = False, stream=None) -> None:
        _c.cfh_apply_plan(self.h, psi, theta_dev, inverse, stream)


class Hamiltonian:
    """H = sum_j c_j P_j (terms already conjugated through the frame)."""

    def __init__(self, n: int, dtype, terms: np.ndarray, coeff: np.ndarray, tuning: Optional[dict] = None):
        self.n = n
        self.dtype = state_dtype(dtype)
        self.h = _c.cfh_ham_create(n, self.dtype, terms, coeff, tuning)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _c is not None:  # None once the interpreter tears modules down
            _c.cfh_ham_destroy(h)
            self.h = None

    def info(self) -> dict:
        return _c.cfh_ham_info(self.h)

    def expval_async(self, psi: torch.Tensor, out_dev: torch.Tensor, stream=None) -> None:
        _c.cfh_expval_async(self.h, psi, out_dev, stream)

    def expval(self, psi: torch.Tensor) -> complex:
        out = torch.zeros(2, dtype=torch.float64, device=psi.device)
        self.expval_async(psi, out)
        v = out.cpu()
        return complex(float(v[0]), float(v[1]))

    def apply(self, psi: torch.Tensor, out: torch.Tensor, stream=None) -> None:
        _c.cfh_ham_apply(self.h, psi, out, stream)


def new_state(n: int, dtype=torch.complex128, device="cuda", index: int = 0) -> torch.Tensor:
    psi = torch.empty(1 << n, dtype=dtype, device=device)
    _c.cfh_state_set_basis(psi, n, index)
    return psi


class PauliEnergy(torch.autograd.Function):
    """E(theta) = <Phi|H|Phi> with Phi = R_{m-1}..R_0 Phi_0 (rotations of ``plan``).

    Forward runs the plan and the expectation value in the library; backward
    runs the library's adjoint sweep (rewinding the state by the inverse
    rotations, so no intermediate states are stored)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, plan: Plan, ham: Hamiltonian, psi0: torch.Tensor):
        psi = psi0.clone()
        plan.apply(psi, theta)
        out = torch.zeros(2, dtype=torch.float64, device=psi.device)
        ham.expval_async(psi, out)
        ctx.plan, ctx.ham = plan, ham
        ctx.save_for_backward(theta, psi)
        return out[0].clone()

    @staticmethod
    def backward(ctx, grad_e: torch.Tensor):
        theta, psi = ctx.saved_tensors
        psi = psi.clone()
        lam = torch.empty_like(psi)
        grad = torch.empty_like(theta)
        _c.cfh_adjoint_grad(ctx.plan.h, ctx.ham.h, psi, lam, theta, grad)
        return grad * grad_e, None, None, None


def prepare(w, dtype=torch.complex128, tuning: Optional[dict] = None, ham_tuning: Optional[dict] = None):
    """Frame-track a workload's Clifford prefix, conjugate its rotations and
    observable, and build the plan and Hamiltonian (steps a1-a4 of the path)."""
    frame = Frame(w.n)
    frame.apply_gates(w.prefix)
    rot = frame.conjugate(_c.cfh_pauli_encode(w.rot)) if w.n_rot else np.zeros(0, _c.PAULI_DTYPE)
    terms = frame.conjugate(_c.cfh_pauli_encode(w.ham)) if w.ham.shape[0] else np.zeros(0, _c.PAULI_DTYPE)
    plan = Plan(w.n, dtype, rot, tuning)
    ham = Hamiltonian(w.n, dtype, terms, w.coeff, ham_tuning) if terms.shape[0] else None
    return frame, rot, terms, plan, ham


class Batch:
    """Many independent circuits run together (cfh_batch_*): by default one
    kernel launch per pass level and kernel kind, all items of a level in one
    grid; with tuning {"variant": 1}, one persistent kernel per run."""

    def __init__(self, workloads, dtype=torch.complex128, tuning: Optional[dict] = None):
        self.dtype = state_dtype(dtype)
        circuits = []
        self.m = []
        for w in workloads:
            frame = Frame(w.n)
            frame.apply_gates(w.prefix)
            circuits.append({"n": w.n, "init_index": w.init,
                             "rot": frame.conjugate(_c.cfh_pauli_encode(w.rot)),
                             "theta": w.theta, "terms": frame.conjugate(_c.cfh_pauli_encode(w.ham)),
                             "coeff": w.coeff})
            self.m.append(w.n_rot)
        self.count = len(circuits)
        self.total_rot = int(sum(self.m))
        self.n = [c["n"] for c in circuits]
        self.h = _c.cfh_batch_create(circuits, self.dtype, tuning)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _c is not None:  # None once the interpreter tears modules down
            _c.cfh_batch_destroy(h)
            self.h = None

    def info(self) -> dict:
        return _c.cfh_batch_info(self.h)

    def set_theta(self, theta: np.ndarray) -> None:
        _c.cfh_batch_set_theta(self.h, theta)

    def run(self, with_grad: bool = True, stream=None) -> None:
        _c.cfh_batch_run(self.h, with_grad, stream)

    def graph_launch(self, with_grad: bool, stream) -> None:
        _c.cfh_batch_graph_launch(self.h, with_grad, stream)

    def results(self, stream=None) -> dict:
        e, g, t0, t1, hz = _c.cfh_batch_results(self.h, self.count, self.total_rot, stream)
        off = np.concatenate([[0], np.cumsum(self.m)])
        return {"energy": e, "grad": [g[off[i]:off[i + 1]] for i in range(self.count)],
                "t_start": t0, "t_end": t1, "tick_hz": hz}

    def state(self, i: int, stream=None) -> torch.Tensor:
        out = torch.empty(1 << self.n[i], dtype=torch.complex128 if self.dtype == _c.CFH_C128 else torch.complex64,
                          device="cuda")
        _c.cfh_batch_state(self.h, i, out, stream)
        return out
