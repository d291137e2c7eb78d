"""Schroedinger-style FP64 simulation (Sec. II-A; oracle, test-only).

`run(circuit)` applies every gate in list order to |0...0> with the plain C
core in sv.c.  `dense_unitary(circuit)` builds the full 2^n x 2^n operator
entry by entry (brute force, n <= 10), an independent check of the core.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import gates as G

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv.c")
_LIB = os.path.join(_HERE, "liboracle_sv.so")
_lib = None


def build(force=False):
    """Compile sv.c with gcc (OpenMP, -O2).  Called by the repo's build step
    and on first use when the library is missing."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.sv_apply.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P]
        lib.sv_run.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P, P, P]
        lib.sv_run_many.argtypes = [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, P, P, P, P, P]
        lib.sv_braket.argtypes = [P, P, ctypes.c_int, P, ctypes.c_int, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def apply(psi, n, qubits, m):
    """In place: psi <- (m on qubits) psi.  psi is complex128 of length 2^n."""
    lib = _load()
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    q = np.asarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(m, dtype=np.complex128)
    rc = lib.sv_apply(_ptr(psi), n, _ptr(q), len(q), _ptr(m))
    if rc:
        raise ValueError(f"sv_apply failed ({rc})")


def braket(lam, psi, n, qubits, m):
    """<lam| (m on qubits) |psi> without copying either state."""
    lib = _load()
    for v in (lam, psi):
        assert v.dtype == np.complex128 and v.flags.c_contiguous and v.size == 1 << n
    q = np.asarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(m, dtype=np.complex128)
    out = np.zeros(2, dtype=np.float64)
    rc = lib.sv_braket(_ptr(lam), _ptr(psi), n, _ptr(q), len(q), _ptr(m), _ptr(out))
    if rc:
        raise ValueError(f"sv_braket failed ({rc})")
    return complex(out[0], out[1])


def run_ops(n, ops, psi=None):
    """ops: list of (qubits, matrix).  Starts from |0...0> unless psi given."""
    lib = _load()
    if psi is None:
        psi = np.zeros(1 << n, dtype=np.complex128)
        psi[0] = 1.0
    if not ops:
        return psi
    qs = np.concatenate([np.asarray(q, dtype=np.int32) for q, _ in ops])
    ks = np.array([len(q) for q, _ in ops], dtype=np.int32)
    mats = [np.ascontiguousarray(m, dtype=np.complex128).ravel() for _, m in ops]
    moff = np.zeros(len(mats), dtype=np.int64)
    moff[1:] = np.cumsum([m.size for m in mats])[:-1]
    flat = np.concatenate(mats)
    rc = lib.sv_run(_ptr(psi), n, len(ops), _ptr(qs), _ptr(ks), _ptr(moff), _ptr(flat))
    if rc:
        raise ValueError(f"sv_run failed ({rc})")
    return psi


def run_many(n, ops, selections):
    """Independent states, one per row of `selections`.  ops: list of
    (qubits, [matrix, ...]); state s applies ops[g][1][selections[s, g]]."""
    lib = _load()
    selections = np.asarray(selections, dtype=np.int64)
    count = selections.shape[0]
    psi = np.zeros((count, 1 << n), dtype=np.complex128)
    psi[:, 0] = 1.0
    if not ops:
        return psi
    qs = np.concatenate([np.asarray(q, dtype=np.int32) for q, _ in ops])
    ks = np.array([len(q) for q, _ in ops], dtype=np.int32)
    mats, first = [], []
    for _, ms in ops:
        first.append(len(mats))
        mats.extend(np.ascontiguousarray(m, dtype=np.complex128).ravel() for m in ms)
    moff = np.zeros(len(mats), dtype=np.int64)
    moff[1:] = np.cumsum([m.size for m in mats])[:-1]
    sel = (selections + np.asarray(first, dtype=np.int64)[None, :]).astype(np.int64)
    sel = np.ascontiguousarray(sel)
    flat = np.concatenate(mats)
    rc = lib.sv_run_many(_ptr(psi), n, count, len(ops), _ptr(qs), _ptr(ks), _ptr(moff),
                         _ptr(sel), _ptr(flat))
    if rc:
        raise ValueError(f"sv_run_many failed ({rc})")
    return psi


def run(circuit):
    """Final state U_circuit |0...0> (plain definition, Sec. II-A)."""
    return run_ops(circuit["n"], [(g["q"], G.matrix(g)) for g in circuit["gates"]])


def embed(n, qubits, m):
    """Full 2^n x 2^n matrix of a gate, entry by entry (brute force)."""
    k = len(qubits)
    dim = 1 << n
    idx = np.arange(dim)
    loc = np.zeros(dim, dtype=np.int64)
    mask = 0
    for j, q in enumerate(qubits):
        loc |= ((idx >> q) & 1) << (k - 1 - j)
        mask |= 1 << q
    rest = idx & ~mask
    same = rest[:, None] == rest[None, :]
    return np.where(same, m[loc[:, None], loc[None, :]], 0.0)


def dense_unitary(circuit):
    n = circuit["n"]
    assert n <= 10
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circuit["gates"]:
        u = embed(n, g["q"], G.matrix(g)) @ u
    return u
