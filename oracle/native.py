"""ctypes front of the oracle's plain C float64 twin (oracle/capply.c).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.  The C file computes
the same two things as ``oracle.apply`` -- the term-by-term scatter from
source configurations and the ungrouped gather at selected targets -- from
the letter-form action of each string, with OpenMP threads, so that
full-size workloads (28 and 32 qubits) can be checked whole rows at a time
and timed on the host cores.  It is compiled with gcc into
``oracle/libcapply.so`` (``build()``), on first use when it is not there.
"""

import ctypes
import os
import subprocess

import numpy as np

from .apply import term_action

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "capply.c")
LIB = os.path.join(HERE, "libcapply.so")


def build():
    """Compiles capply.c (gcc, -O2, OpenMP, no floating-point contraction)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-Wall", SRC, "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, LIB)
    return LIB


class _Space(ctypes.Structure):
    _fields_ = [
        ("sector", ctypes.c_int32),
        ("n_bits", ctypes.c_int32),
        ("dim", ctypes.c_uint64),
        ("dim_b", ctypes.c_uint64),
        ("pos_a", ctypes.c_void_p),
        ("pos_b", ctypes.c_void_p),
        ("str_a", ctypes.c_void_p),
        ("str_b", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        sig = [ctypes.POINTER(_Space), ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
               ctypes.POINTER(ctypes.c_int)]
        for name in ("orc_apply_scatter", "orc_apply_targets"):
            fn = getattr(lib, name)
            fn.argtypes = sig
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class _Prepared:
    """Term arrays and space tables in the layout the C code reads (kept
    alive for the duration of a call)."""

    def __init__(self, op, space):
        flip, sign, n_y = term_action(op.letters)
        self.n_terms = op.n_terms
        self.flip = np.ascontiguousarray(flip, dtype=np.uint64)
        self.sign = np.ascontiguousarray(sign, dtype=np.uint64)
        self.n_y = np.ascontiguousarray(np.asarray(n_y) % 4, dtype=np.uint8)
        self.coeff = np.ascontiguousarray(np.asarray(op.coeff, dtype=np.complex128))
        sp = _Space()
        sp.dim = space.dim
        if hasattr(space, "alpha"):
            n_orb = space.n_orb
            self.str_a = np.ascontiguousarray(space.alpha, dtype=np.uint64)
            self.str_b = np.ascontiguousarray(space.beta, dtype=np.uint64)
            # position tables from the enumerated ascending lists
            self.pos_a = np.full(1 << n_orb, -1, dtype=np.int32)
            self.pos_a[self.str_a.astype(np.int64)] = np.arange(len(self.str_a), dtype=np.int32)
            self.pos_b = np.full(1 << n_orb, -1, dtype=np.int32)
            self.pos_b[self.str_b.astype(np.int64)] = np.arange(len(self.str_b), dtype=np.int32)
            sp.sector, sp.n_bits, sp.dim_b = 1, n_orb, len(self.str_b)
            sp.pos_a, sp.pos_b = _ptr(self.pos_a), _ptr(self.pos_b)
            sp.str_a, sp.str_b = _ptr(self.str_a), _ptr(self.str_b)
        else:
            sp.sector, sp.n_bits, sp.dim_b = 0, space.n_qubits, 0
        self.space = sp

    def args(self):
        return (ctypes.byref(self.space), self.n_terms, _ptr(self.flip), _ptr(self.sign), _ptr(self.n_y),
                _ptr(self.coeff))


def prepare(op, space):
    """Reusable term and space tables for repeated calls on one operator."""
    return _Prepared(op, space)


def apply_scatter(op, space, psi, sources=None, threads=0, prepared=None):
    """(P H P psi) from the listed source indices (all when None), float64,
    term by term in scatter order.  Returns (out, threads used)."""
    lib = _load()
    prep = prepared or _Prepared(op, space)
    psi = np.ascontiguousarray(np.asarray(psi).astype(np.complex128, copy=False))
    assert psi.shape == (space.dim,)
    src = None if sources is None else np.ascontiguousarray(sources, dtype=np.int64)
    out = np.empty(space.dim, dtype=np.complex128)
    used = ctypes.c_int(0)
    rc = lib.orc_apply_scatter(*prep.args(), _ptr(psi), 0 if src is None else len(src), _ptr(src), _ptr(out),
                               int(threads), ctypes.byref(used))
    if rc != 0:
        raise MemoryError("orc_apply_scatter: out of host memory")
    return out, used.value


def apply_targets(op, space, psi, targets, threads=0, prepared=None):
    """(P H P psi)[t] for the listed target indices, float64, each target
    summed over the terms in their order.  Returns (values, threads used)."""
    lib = _load()
    prep = prepared or _Prepared(op, space)
    psi = np.ascontiguousarray(np.asarray(psi).astype(np.complex128, copy=False))
    assert psi.shape == (space.dim,)
    tgt = np.ascontiguousarray(targets, dtype=np.int64)
    assert tgt.size == 0 or (tgt.min() >= 0 and tgt.max() < space.dim)
    out = np.empty(len(tgt), dtype=np.complex128)
    used = ctypes.c_int(0)
    rc = lib.orc_apply_targets(*prep.args(), _ptr(psi), len(tgt), _ptr(tgt), _ptr(out), int(threads),
                               ctypes.byref(used))
    if rc != 0:
        raise MemoryError("orc_apply_targets: out of host memory")
    return out, used.value
