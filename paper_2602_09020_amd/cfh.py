"""ctypes binding of libcfh (include/cfh.h).

Argument marshalling only: every step of the hot path runs inside the HIP
library.  Functions carry the C names; torch tensors supply device memory
(``tensor.data_ptr()``) and streams (``torch.cuda.current_stream()``).  If the
library is not built this module raises on first use: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CFH_LIB_PATH selects another build of the library (the host sanitizer run uses one)
LIB_PATH = os.environ.get("CFH_LIB_PATH") or os.path.join(_HERE, "libcfh.so")

CFH_OK, CFH_E_INVAL, CFH_E_RANGE, CFH_E_NOT_HERMITIAN = 0, -1, -2, -3
CFH_E_NOMEM, CFH_E_HIP, CFH_E_UNSUPPORTED, CFH_E_TIMEOUT = -4, -5, -6, -7
CFH_C64, CFH_C128 = 0, 1
(CFH_GATE_H, CFH_GATE_S, CFH_GATE_SDG, CFH_GATE_X, CFH_GATE_Y, CFH_GATE_Z,
 CFH_GATE_CNOT, CFH_GATE_CZ, CFH_GATE_SWAP, CFH_GATE_RX, CFH_GATE_RY, CFH_GATE_RZ,
 CFH_GATE_MEASURE, CFH_GATE_RESET) = range(14)

PAULI_DTYPE = np.dtype([("x", "<u8"), ("z", "<u8"), ("e", "<i4"), ("reserved", "<i4")])


class cfh_pauli(C.Structure):
    _fields_ = [("x", C.c_uint64), ("z", C.c_uint64), ("e", C.c_int32), ("reserved", C.c_int32)]


class cfh_tuning(C.Structure):
    _fields_ = [("tile_bits", C.c_int32), ("low_bits", C.c_int32), ("max_run", C.c_int32),
                ("lookahead", C.c_int32), ("unfused", C.c_int32), ("block_threads", C.c_int32),
                ("variant", C.c_int32), ("batch_items", C.c_int32),
                ("group_mib", C.c_int32), ("tile_order", C.c_int32), ("reg_tile_bits", C.c_int32)]


class cfh_circuit_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("reserved", C.c_int32), ("init_index", C.c_uint64),
                ("rot", C.c_void_p), ("theta", C.c_void_p), ("m", C.c_int64),
                ("terms", C.c_void_p), ("coeff", C.c_void_p), ("mh", C.c_int64)]


class CfhError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_L = None
_vp = C.c_void_p
_P = C.POINTER

# name -> (restype, argtypes); the declarations of include/cfh.h
_SIGS = {
    "cfh_version": (C.c_int, []),
    "cfh_last_error": (C.c_char_p, []),
    "cfh_device_count": (C.c_int, []),
    "cfh_pauli_encode": (C.c_int32, [_vp, C.c_int, C.c_size_t, _vp]),
    "cfh_frame_create": (C.c_int32, [C.c_int, _P(_vp)]),
    "cfh_frame_destroy": (C.c_int32, [_vp]),
    "cfh_frame_apply_clifford": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int]),
    "cfh_frame_apply_gates": (C.c_int32, [_vp, _vp, C.c_size_t]),
    "cfh_frame_row": (C.c_int32, [_vp, C.c_int, _P(cfh_pauli), _P(cfh_pauli)]),
    "cfh_frame_conjugate": (C.c_int32, [_vp, _P(cfh_pauli), _P(cfh_pauli)]),
    "cfh_frame_conjugate_many": (C.c_int32, [_vp, _vp, _vp, C.c_size_t]),
    "cfh_frame_conjugate_device": (C.c_int32, [_vp, _vp, _vp, C.c_size_t, _vp]),
    "cfh_frame_flush_rotations": (C.c_int32, [_vp, _vp, _vp, C.c_size_t, _P(C.c_size_t)]),
    "cfh_frame_flush": (C.c_int32, [_vp, _vp, C.c_int, _vp]),
    "cfh_circuit_translate": (C.c_int32, [_vp, _vp, _vp, C.c_size_t, _vp, _vp, C.c_size_t, _P(C.c_size_t)]),
    "cfh_circuit_run": (C.c_int32, [_vp, _vp, _vp, C.c_size_t, _vp, C.c_int, _P(cfh_tuning), _vp, _vp]),
    "cfh_measure_pauli": (C.c_int32, [_vp, C.c_int, C.c_int, _P(cfh_pauli), C.c_double, _P(C.c_int32),
                                      _P(C.c_double), _vp]),
    "cfh_state_set_basis": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_uint64, _vp]),
    "cfh_apply_pauli_rotation": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_uint64, C.c_uint64, C.c_int,
                                             C.c_double, _vp]),
    "cfh_plan_create": (C.c_int32, [C.c_int, C.c_int, _vp, C.c_size_t, _P(cfh_tuning), _P(_vp)]),
    "cfh_plan_destroy": (C.c_int32, [_vp]),
    "cfh_plan_dry_run": (C.c_int32, [C.c_int, C.c_int, _vp, C.c_size_t, _P(cfh_tuning), _P(C.c_int64), _vp, _vp]),
    "cfh_ham_dry_run": (C.c_int32, [C.c_int, C.c_int, _vp, C.c_size_t, _P(cfh_tuning), _P(C.c_int64), _vp, _vp,
                                    _vp, _vp]),
    "cfh_plan_info": (C.c_int32, [_vp, _P(C.c_int64), _P(C.c_int64), _P(C.c_int32), _P(C.c_double),
                                  _P(C.c_int32)]),
    "cfh_plan_schedule": (C.c_int32, [_vp, _vp, _vp]),
    "cfh_plan_leaf_counts": (C.c_int32, [_vp, _vp, C.c_int, _vp]),
    "cfh_apply_plan": (C.c_int32, [_vp, _vp, _vp, C.c_int, _vp]),
    "cfh_ham_create": (C.c_int32, [C.c_int, C.c_int, _vp, _vp, C.c_size_t, _P(cfh_tuning), _P(_vp)]),
    "cfh_ham_destroy": (C.c_int32, [_vp]),
    "cfh_ham_info": (C.c_int32, [_vp, _P(C.c_int64), _P(C.c_int64), _P(C.c_double)]),
    "cfh_expval_async": (C.c_int32, [_vp, _vp, _vp, _vp]),
    "cfh_expval": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp, C.c_size_t, _vp, _vp]),
    "cfh_expval_noalloc": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp, C.c_size_t, _vp, _vp]),
    "cfh_ham_apply": (C.c_int32, [_vp, _vp, _vp, _vp]),
    "cfh_adjoint_grad": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cfh_calib_rmw": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp]),
    "cfh_batch_create": (C.c_int32, [_vp, C.c_int, C.c_int, _P(cfh_tuning), _P(_vp)]),
    "cfh_batch_destroy": (C.c_int32, [_vp]),
    "cfh_batch_info": (C.c_int32, [_vp, _P(C.c_int64), _P(C.c_int64), _P(C.c_int64), _P(C.c_double),
                                   _P(C.c_double), _P(C.c_double), _P(C.c_int32)]),
    "cfh_batch_set_theta": (C.c_int32, [_vp, _vp]),
    "cfh_batch_run": (C.c_int32, [_vp, C.c_int, _vp]),
    "cfh_batch_graph_launch": (C.c_int32, [_vp, C.c_int, _vp]),
    "cfh_batch_results": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _P(C.c_double), _vp]),
    "cfh_batch_state": (C.c_int32, [_vp, C.c_int, _vp, _vp]),
    "cfh_batch_persist_config": (C.c_int32, [_vp, C.c_double, C.c_int, C.c_int]),
    "cfh_batch_persist_info": (C.c_int32, [_vp, _P(C.c_int32), _P(C.c_int64), _P(C.c_int64)]),
    "cfh_batch_order": (C.c_int32, [C.c_int, _vp, _vp, _vp, _vp, _vp, _vp]),
}


def lib() -> C.CDLL:
    """Load libcfh.so (raises if it has not been built)."""
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _L = L
    return _L


def declared_symbols() -> Sequence[str]:
    return tuple(_SIGS)


def _call(name: str, *args) -> None:
    rc = getattr(lib(), name)(*args)
    if rc != CFH_OK:
        raise CfhError(name, rc, cfh_last_error())


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.complex128:
        return CFH_C128
    if t.dtype == torch.complex64:
        return CFH_C64
    raise TypeError(f"state tensors must be complex64 or complex128, got {t.dtype}")


def _dev_ptr(t, what: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def _paulis(p) -> np.ndarray:
    a = np.ascontiguousarray(p)
    if a.dtype != PAULI_DTYPE:
        raise TypeError("Pauli arrays must have PAULI_DTYPE (x, z, e, reserved)")
    return a


def _tuning(t) -> Optional[cfh_tuning]:
    if t is None:
        return None
    if isinstance(t, cfh_tuning):
        return t
    return cfh_tuning(**{k: int(v) for k, v in dict(t).items()})


# ------------------------------------------------------------------ misc

def cfh_version() -> int:
    return int(lib().cfh_version())


def cfh_last_error() -> str:
    return (lib().cfh_last_error() or b"").decode()


def cfh_device_count() -> int:
    return int(lib().cfh_device_count())


# ------------------------------------------------------------------ a1

def cfh_pauli_encode(letters: np.ndarray) -> np.ndarray:
    l = np.ascontiguousarray(letters, dtype=np.uint8)
    if l.ndim == 1:
        l = l[None, :]
    m, n = l.shape
    out = np.zeros(m, dtype=PAULI_DTYPE)
    _call("cfh_pauli_encode", l.ctypes.data, n, m, out.ctypes.data)
    return out


# ------------------------------------------------------------------ a2, a3

def cfh_frame_create(n: int) -> int:
    h = C.c_void_p()
    _call("cfh_frame_create", n, C.byref(h))
    return h.value


def cfh_frame_destroy(f: int) -> None:
    _call("cfh_frame_destroy", f)


def cfh_frame_apply_clifford(f: int, gate: int, q0: int, q1: int = -1) -> None:
    _call("cfh_frame_apply_clifford", f, gate, q0, q1)


def cfh_frame_apply_gates(f: int, gates: np.ndarray) -> None:
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 3)
    _call("cfh_frame_apply_gates", f, g.ctypes.data, g.shape[0])


def _pauli_tuple(p: cfh_pauli) -> Tuple[int, int, int]:
    return int(p.x), int(p.z), int(p.e)


def cfh_frame_row(f: int, q: int):
    z, x = cfh_pauli(), cfh_pauli()
    _call("cfh_frame_row", f, q, C.byref(z), C.byref(x))
    return _pauli_tuple(z), _pauli_tuple(x)


def cfh_frame_conjugate(f: int, x: int, z: int, e: int = 0) -> Tuple[int, int, int]:
    src, dst = cfh_pauli(x, z, e, 0), cfh_pauli()
    _call("cfh_frame_conjugate", f, C.byref(src), C.byref(dst))
    return _pauli_tuple(dst)


def cfh_frame_conjugate_many(f: int, paulis: np.ndarray) -> np.ndarray:
    a = _paulis(paulis)
    out = np.zeros_like(a)
    _call("cfh_frame_conjugate_many", f, a.ctypes.data, out.ctypes.data, a.shape[0])
    return out


def cfh_frame_conjugate_device(f: int, in_dev, out_dev, m: int, stream=None) -> None:
    _call("cfh_frame_conjugate_device", f, _dev_ptr(in_dev, "in"), _dev_ptr(out_dev, "out"), m, _stream(stream))


def cfh_frame_flush_rotations(f: int, n: int):
    """(paulis, theta): the rotations that flush the frame into Phi (host only)."""
    cap = 9 * n + 8
    rot = np.zeros(cap, PAULI_DTYPE)
    theta = np.zeros(cap, np.float64)
    m = C.c_size_t()
    _call("cfh_frame_flush_rotations", f, rot.ctypes.data, theta.ctypes.data, cap, C.byref(m))
    return rot[:m.value].copy(), theta[:m.value].copy()


def cfh_frame_flush(f: int, psi, stream=None) -> None:
    _call("cfh_frame_flush", f, _dev_ptr(psi, "psi"), _dtype_code(psi), _stream(stream))


def _gate_rows(gates, angles):
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 3)
    a = None if angles is None else np.ascontiguousarray(angles, dtype=np.float64).reshape(-1)
    if a is not None and a.shape[0] != g.shape[0]:
        raise ValueError("one angle per gate row")
    return g, a


def cfh_circuit_translate(f: int, gates, angles=None):
    """(paulis, theta) of the circuit's rotations on Phi; the frame absorbs its Cliffords."""
    g, a = _gate_rows(gates, angles)
    cap = max(1, int(np.isin(g[:, 0], (CFH_GATE_RX, CFH_GATE_RY, CFH_GATE_RZ)).sum()))
    rot = np.zeros(cap, PAULI_DTYPE)
    theta = np.zeros(cap, np.float64)
    m = C.c_size_t()
    _call("cfh_circuit_translate", f, g.ctypes.data, a.ctypes.data if a is not None else None, g.shape[0],
          rot.ctypes.data, theta.ctypes.data, cap, C.byref(m))
    return rot[:m.value].copy(), theta[:m.value].copy()


def cfh_circuit_run(f: int, gates, angles, psi, tuning=None, stream=None) -> np.ndarray:
    """Runs the circuit; returns the outcomes array (+1/-1 at measurement and reset rows, else 0)."""
    g, a = _gate_rows(gates, angles)
    t = _tuning(tuning)
    out = np.zeros(max(1, g.shape[0]), np.int32)
    _call("cfh_circuit_run", f, g.ctypes.data, a.ctypes.data if a is not None else None, g.shape[0],
          _dev_ptr(psi, "psi"), _dtype_code(psi), C.byref(t) if t is not None else None, out.ctypes.data,
          _stream(stream))
    return out[:g.shape[0]]


def cfh_measure_pauli(psi, n: int, x: int, z: int, e: int, u: float, stream=None):
    """(outcome, P(+1)) of measuring the Pauli (x, z, e) on psi, which collapses in place."""
    p = cfh_pauli(x, z, e, 0)
    o, pp = C.c_int32(), C.c_double()
    _call("cfh_measure_pauli", _dev_ptr(psi, "psi"), n, _dtype_code(psi), C.byref(p), float(u), C.byref(o),
          C.byref(pp), _stream(stream))
    return int(o.value), float(pp.value)


# ------------------------------------------------------------------ state

def cfh_state_set_basis(psi, n: int, index: int, stream=None) -> None:
    _call("cfh_state_set_basis", _dev_ptr(psi, "psi"), n, _dtype_code(psi), index, _stream(stream))


def cfh_apply_pauli_rotation(psi, n: int, x: int, z: int, e: int, theta: float, stream=None) -> None:
    _call("cfh_apply_pauli_rotation", _dev_ptr(psi, "psi"), n, _dtype_code(psi), x, z, e, float(theta),
          _stream(stream))


# ------------------------------------------------------------------ plans

def cfh_plan_create(n: int, dtype: int, rot: np.ndarray, tuning=None) -> int:
    a = _paulis(rot)
    h = C.c_void_p()
    t = _tuning(tuning)
    _call("cfh_plan_create", n, dtype, a.ctypes.data if a.size else None, a.shape[0],
          C.byref(t) if t is not None else None, C.byref(h))
    return h.value


def cfh_plan_destroy(p: int) -> None:
    _call("cfh_plan_destroy", p)


def cfh_ham_dry_run(n: int, dtype: int, terms: np.ndarray, tuning=None):
    """Host-only planning of the register-tiled <H> passes: returns
    (pass_start, order, pass_bits, basis) with basis of shape (P, 16)."""
    a = _paulis(terms)
    m = a.shape[0]
    ps = np.zeros(m + 1, np.int64)
    order = np.zeros(max(m, 1), np.int64)
    bits = np.zeros(max(m, 1), np.int32)
    basis = np.zeros((max(m, 1), 16), np.uint64)
    cnt = C.c_int64()
    t = _tuning(tuning)
    _call("cfh_ham_dry_run", n, dtype, a.ctypes.data if m else None, m, C.byref(t) if t is not None else None,
          C.byref(cnt), ps.ctypes.data, order.ctypes.data, bits.ctypes.data, basis.ctypes.data)
    P = cnt.value
    return ps[:P + 1].copy(), order[:m].copy(), bits[:P].copy(), basis[:P].copy()


def cfh_plan_dry_run(n: int, dtype: int, rot: np.ndarray, tuning=None):
    """Host-only planning: returns (pass_start, order)."""
    a = _paulis(rot)
    m = a.shape[0]
    ps = np.zeros(m + 1, np.int64)
    order = np.zeros(max(m, 1), np.int64)
    cnt = C.c_int64()
    t = _tuning(tuning)
    _call("cfh_plan_dry_run", n, dtype, a.ctypes.data if m else None, m, C.byref(t) if t is not None else None,
          C.byref(cnt), ps.ctypes.data, order.ctypes.data)
    return ps[:cnt.value + 1].copy(), order[:m].copy()


def cfh_plan_info(p: int) -> dict:
    np_, nr, tb, hb, var = C.c_int64(), C.c_int64(), C.c_int32(), C.c_double(), C.c_int32()
    _call("cfh_plan_info", p, C.byref(np_), C.byref(nr), C.byref(tb), C.byref(hb), C.byref(var))
    return {"n_passes": np_.value, "n_rot": nr.value, "tile_bits": tb.value, "hbm_bytes": hb.value,
            "variant": var.value}


def cfh_plan_schedule(p: int, m: int, n_passes: int):
    ps = np.zeros(n_passes + 1, np.int64)
    order = np.zeros(m, np.int64)
    _call("cfh_plan_schedule", p, ps.ctypes.data, order.ctypes.data)
    return ps, order


def cfh_plan_leaf_counts(p: int, theta: np.ndarray, inverse: bool = False) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros(512, np.int64)
    _call("cfh_plan_leaf_counts", p, th.ctypes.data, int(bool(inverse)), out.ctypes.data)
    return out


def cfh_apply_plan(p: int, psi, theta_dev, inverse: bool = False, stream=None) -> None:
    _call("cfh_apply_plan", p, _dev_ptr(psi, "psi"), _dev_ptr(theta_dev, "theta"), int(bool(inverse)),
          _stream(stream))


# ------------------------------------------------------------ Hamiltonians

def cfh_ham_create(n: int, dtype: int, terms: np.ndarray, coeff: np.ndarray, tuning=None) -> int:
    a = _paulis(terms)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    if c.shape[0] != a.shape[0]:
        raise ValueError("one coefficient per term")
    h = C.c_void_p()
    t = _tuning(tuning)
    _call("cfh_ham_create", n, dtype, a.ctypes.data if a.size else None, c.ctypes.data if c.size else None,
          a.shape[0], C.byref(t) if t is not None else None, C.byref(h))
    return h.value


def cfh_ham_destroy(h: int) -> None:
    _call("cfh_ham_destroy", h)


def cfh_ham_info(h: int) -> dict:
    np_, ng, hb = C.c_int64(), C.c_int64(), C.c_double()
    _call("cfh_ham_info", h, C.byref(np_), C.byref(ng), C.byref(hb))
    return {"n_passes": np_.value, "n_groups": ng.value, "hbm_bytes": hb.value}


def cfh_expval_async(h: int, psi, out_dev, stream=None) -> None:
    _call("cfh_expval_async", h, _dev_ptr(psi, "psi"), _dev_ptr(out_dev, "out"), _stream(stream))


def cfh_expval(psi, n: int, terms: np.ndarray, coeff: np.ndarray, stream=None) -> complex:
    a = _paulis(terms)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    out = np.zeros(2, np.float64)
    _call("cfh_expval", _dev_ptr(psi, "psi"), n, _dtype_code(psi), a.ctypes.data, c.ctypes.data, a.shape[0],
          out.ctypes.data, _stream(stream))
    return complex(out[0], out[1])


def cfh_expval_noalloc(psi, n: int, terms: np.ndarray, coeff: np.ndarray, out_dev, stream=None) -> None:
    a = _paulis(terms)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    _call("cfh_expval_noalloc", _dev_ptr(psi, "psi"), n, _dtype_code(psi), a.ctypes.data, c.ctypes.data,
          a.shape[0], _dev_ptr(out_dev, "out"), _stream(stream))


def cfh_calib_rmw(buf, n: int, chunk_bits: int = -1, nontemporal: bool = False, stream=None) -> None:
    _call("cfh_calib_rmw", _dev_ptr(buf, "buf"), n, _dtype_code(buf), int(chunk_bits), int(bool(nontemporal)),
          _stream(stream))


def cfh_ham_apply(h: int, psi, out, stream=None) -> None:
    _call("cfh_ham_apply", h, _dev_ptr(psi, "psi"), _dev_ptr(out, "out"), _stream(stream))


def cfh_adjoint_grad(p: int, h: int, psi, lam, theta_dev, grad_dev, stream=None) -> None:
    _call("cfh_adjoint_grad", p, h, _dev_ptr(psi, "psi"), _dev_ptr(lam, "lam"), _dev_ptr(theta_dev, "theta"),
          _dev_ptr(grad_dev, "grad"), _stream(stream))


# ------------------------------------------------------------------ batches

def cfh_batch_create(circuits, dtype: int, tuning=None) -> int:
    """circuits: sequence of dicts with n, init_index, rot (PAULI_DTYPE), theta,
    terms (PAULI_DTYPE), coeff.  The arrays are copied by the library."""
    keep = []
    descs = (cfh_circuit_desc * len(circuits))()
    for i, c in enumerate(circuits):
        rot = _paulis(c["rot"])
        th = np.ascontiguousarray(c["theta"], dtype=np.float64)
        terms = _paulis(c["terms"])
        coeff = np.ascontiguousarray(c["coeff"], dtype=np.float64)
        keep += [rot, th, terms, coeff]
        descs[i] = cfh_circuit_desc(int(c["n"]), 0, int(c["init_index"]), rot.ctypes.data, th.ctypes.data,
                                    rot.shape[0], terms.ctypes.data, coeff.ctypes.data, terms.shape[0])
    h = C.c_void_p()
    t = _tuning(tuning)
    _call("cfh_batch_create", C.addressof(descs), len(circuits), dtype, C.byref(t) if t is not None else None,
          C.byref(h))
    del keep
    return h.value


def cfh_batch_destroy(b: int) -> None:
    _call("cfh_batch_destroy", b)


def cfh_batch_info(b: int) -> dict:
    it, np_, nr, sb = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
    bf, bg, ng = C.c_double(), C.c_double(), C.c_int32()
    _call("cfh_batch_info", b, C.byref(it), C.byref(np_), C.byref(nr), C.byref(sb), C.byref(bf), C.byref(bg),
          C.byref(ng))
    return {"n_items_grad": it.value, "n_passes": np_.value, "n_rot": nr.value, "state_bytes": sb.value,
            "bytes_fwd": bf.value, "bytes_grad": bg.value, "n_groups": ng.value}


def cfh_batch_set_theta(b: int, theta: np.ndarray) -> None:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    _call("cfh_batch_set_theta", b, th.ctypes.data)


def cfh_batch_run(b: int, with_grad: bool, stream=None) -> None:
    _call("cfh_batch_run", b, int(bool(with_grad)), _stream(stream))


def cfh_batch_graph_launch(b: int, with_grad: bool, stream) -> None:
    _call("cfh_batch_graph_launch", b, int(bool(with_grad)), _stream(stream))


def cfh_batch_results(b: int, count: int, total_rot: int, stream=None):
    e = np.zeros(count, np.float64)
    g = np.zeros(max(total_rot, 1), np.float64)
    t0 = np.zeros(count, np.uint64)
    t1 = np.zeros(count, np.uint64)
    hz = C.c_double()
    _call("cfh_batch_results", b, e.ctypes.data, g.ctypes.data, t0.ctypes.data, t1.ctypes.data, C.byref(hz),
          _stream(stream))
    return e, g[:total_rot], t0, t1, hz.value


def cfh_batch_state(b: int, i: int, dst_dev, stream=None) -> None:
    _call("cfh_batch_state", b, i, _dev_ptr(dst_dev, "dst"), _stream(stream))


def cfh_batch_persist_config(b: int, max_wait_s: float = 2.0, hold: bool = False, max_grid: int = 0) -> None:
    _call("cfh_batch_persist_config", b, float(max_wait_s), int(bool(hold)), int(max_grid))


def cfh_batch_persist_info(b: int) -> dict:
    g, tf, tg = C.c_int32(), C.c_int64(), C.c_int64()
    _call("cfh_batch_persist_info", b, C.byref(g), C.byref(tf), C.byref(tg))
    return {"grid": g.value, "tickets_fwd": tf.value, "tickets_grad": tg.value}


def cfh_batch_order(chain_len, pass_items, circ_amps):
    """Claim order of a persistent run on the host: (ticket_pass, ticket_item, prev)."""
    cl = np.ascontiguousarray(chain_len, dtype=np.int32)
    pi = np.ascontiguousarray(pass_items, dtype=np.int32)
    ca = np.ascontiguousarray(circ_amps, dtype=np.float64)
    nt = int(pi.sum())
    tp = np.zeros(max(nt, 1), dtype=np.int32)
    ti = np.zeros(max(nt, 1), dtype=np.int32)
    pv = np.zeros(max(len(pi), 1), dtype=np.int32)
    _call("cfh_batch_order", len(cl), cl.ctypes.data, pi.ctypes.data, ca.ctypes.data, tp.ctypes.data,
          ti.ctypes.data, pv.ctypes.data)
    return tp[:nt], ti[:nt], pv[:len(pi)]
