"""Python access to the plain CPU oracle (hp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the library.  Each routine is
the definition from the paper's problem formulation (Sec. 2.1 permutation,
Sec. 2.2 extraction, Sec. 2.3 assignment with the Add step of Sec. 4.7),
written out directly in C; see hp_oracle.c.

Two routines per operation: the literal ones (permute, spref, spref_dcsc)
search every (i, j) pair of the definition; permute_map and spref_map reach
the same result from the stored entries through inverse index tables (the
column renaming qinv, the column multimap list[c]), at a cost proportional
to the entries read, so they finish whole outputs at full benchmark sizes.
The assignment (spasgn) is a merge of stored entries.  The map routines and
the assignment take a thread count (rows are independent).

Parity status: every routine, and the sampled-row mode of each, is pinned by
the CPU tests in tests/ against dense brute force, SciPy indexing, the
selection-matrix products of Sec. 2, hand-worked examples and invariants,
and planted mistakes in each must fail a pin (nothing here is "parity
unpinned").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "INDEX_RANGE", 3: "NOT_PERMUTATION",
          4: "DUPLICATE_INDEX", 5: "NOT_CANONICAL", 6: "SHAPE"}
OPS = {"second": 0, "plus": 1, "replace": 2}


class OracleError(RuntimeError):
    def __init__(self, code):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"oracle status {code} ({self.name})")


def build(force: bool = False, extra_flags=()) -> str:
    """Compile hp_oracle.c into liboracle.so with gcc (no GPU code)."""
    out = _LIB if not extra_flags else os.path.join(_HERE, "liboracle_variant.so")
    if force or extra_flags or not os.path.exists(out) or \
            os.path.getmtime(out) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", *extra_flags, _SRC, "-o", out]
        subprocess.check_call(cmd)
    return out


_lib = None


def _load(path=None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        _lib = _bind(ctypes.CDLL(build()))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.orc_check_csr.argtypes = [I64, I64, P, P]
    lib.orc_permute.argtypes = [I64, I64, P, P, P, ctypes.c_int, P, P, P, I64, P, P, P, I64, P]
    lib.orc_spref.argtypes = [I64, I64, P, P, P, ctypes.c_int, P, I64, P, I64, P, I64, P, P, P, I64, P]
    lib.orc_spasgn.argtypes = [I64, I64, P, P, P, ctypes.c_int, I64, I64, P, P, P,
                               P, I64, P, I64, ctypes.c_int, P, I64, P, P, P, I64, P, ctypes.c_int]
    lib.orc_spref_dcsc.argtypes = [I64, I64, I64, P, P, P, P, ctypes.c_int, P, I64, P, I64, P, I64, P, P, P,
                                   I64, P]
    lib.orc_permute_map.argtypes = [I64, I64, P, P, P, ctypes.c_int, P, P, P, I64, P, P, P, I64, P,
                                    ctypes.c_int]
    lib.orc_spref_map.argtypes = [I64, I64, P, P, P, ctypes.c_int, P, I64, P, I64, P, I64, P, P, P, I64, P,
                                  ctypes.c_int]
    for f in (lib.orc_check_csr, lib.orc_permute, lib.orc_spref, lib.orc_spasgn, lib.orc_spref_dcsc,
              lib.orc_permute_map, lib.orc_spref_map):
        f.restype = ctypes.c_int
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr(A):
    """(m, n, rowptr int64, col int32, val) as contiguous numpy arrays."""
    if hasattr(A, "rowptr"):
        m, n = A.nrows, A.ncols
        rp, c, v = A.rowptr, A.col, A.val
    else:
        m, n, rp, c, v = A
    conv = lambda t: t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    rp = np.ascontiguousarray(conv(rp), dtype=np.int64)
    c = np.ascontiguousarray(conv(c), dtype=np.int32)
    v = np.ascontiguousarray(conv(v))
    assert v.dtype in (np.float32, np.float64, np.uint32, np.uint64, np.int32, np.int64)
    return m, n, rp, c, v


def _ivec(x):
    if x is None:
        return None
    if hasattr(x, "cpu"):
        x = x.cpu().numpy()
    return np.ascontiguousarray(x, dtype=np.int32)


def _rows(rows):
    if rows is None:
        return None, 0
    r = np.ascontiguousarray(rows.cpu().numpy() if hasattr(rows, "cpu") else rows, dtype=np.int64)
    return r, len(r)


def _two_call(fn, nout, vdtype):
    ptr = np.zeros(nout + 1, dtype=np.int64)
    need = ctypes.c_int64(0)
    st = fn(ptr, None, None, 0, need)
    if st != 0:
        raise OracleError(st)
    cap = need.value
    col = np.empty(max(cap, 1), dtype=np.int32)
    val = np.empty(max(cap, 1), dtype=vdtype)
    st = fn(ptr, col, val, cap, need)
    if st != 0:
        raise OracleError(st)
    return ptr, col[:cap], val[:cap]


def check_csr(A) -> str:
    m, n, rp, c, _ = _csr(A)
    return STATUS[_load().orc_check_csr(m, n, _ptr(rp), _ptr(c))]


def permute(A, p, q=None, rows=None, lib=None):
    """Rows of A' with A'[i, j] = A[p[i], q[j]] (q=None: symmetric, q = p).

    Returns (rowptr int64 [len(rows)+1], col int32, val) for the requested
    output rows (all rows when rows is None)."""
    lib = lib or _load()
    m, n, rp, c, v = _csr(A)
    p = _ivec(p)
    q = _ivec(q)
    r, ns = _rows(rows)
    nout = ns if r is not None else m

    def fn(ptr, oc, ov, cap, need):
        return lib.orc_permute(m, n, _ptr(rp), _ptr(c), _ptr(v), v.itemsize, _ptr(p), _ptr(q),
                               _ptr(r), ns, _ptr(ptr), _ptr(oc), _ptr(ov), cap, ctypes.byref(need))
    return _two_call(fn, nout, v.dtype)


def spref(A, I, J, rows=None, lib=None):
    """Rows of C with C[i, j] = A[I[i], J[j]] over I x J."""
    lib = lib or _load()
    m, n, rp, c, v = _csr(A)
    I = _ivec(I)
    J = _ivec(J)
    r, ns = _rows(rows)
    nout = ns if r is not None else len(I)

    def fn(ptr, oc, ov, cap, need):
        return lib.orc_spref(m, n, _ptr(rp), _ptr(c), _ptr(v), v.itemsize, _ptr(I), len(I),
                             _ptr(J), len(J), _ptr(r), ns, _ptr(ptr), _ptr(oc), _ptr(ov), cap,
                             ctypes.byref(need))
    return _two_call(fn, nout, v.dtype)


def permute_map(A, p, q=None, rows=None, lib=None, threads=1):
    """As permute(), through the inverse column map: row i is row p[i] of A
    with every column c renamed qinv[c], then sorted."""
    lib = lib or _load()
    m, n, rp, c, v = _csr(A)
    p = _ivec(p)
    q = _ivec(q)
    r, ns = _rows(rows)
    nout = ns if r is not None else m

    def fn(ptr, oc, ov, cap, need):
        return lib.orc_permute_map(m, n, _ptr(rp), _ptr(c), _ptr(v), v.itemsize, _ptr(p), _ptr(q),
                                   _ptr(r), ns, _ptr(ptr), _ptr(oc), _ptr(ov), cap, ctypes.byref(need),
                                   int(threads))
    return _two_call(fn, nout, v.dtype)


def spref_map(A, I, J, rows=None, lib=None, threads=1):
    """As spref(), through the column multimap list[c] = {j : J[j] = c}:
    every stored entry (I[i], c) is emitted at each j of list[c], then the
    row is sorted."""
    lib = lib or _load()
    m, n, rp, c, v = _csr(A)
    I = _ivec(I)
    J = _ivec(J)
    r, ns = _rows(rows)
    nout = ns if r is not None else len(I)

    def fn(ptr, oc, ov, cap, need):
        return lib.orc_spref_map(m, n, _ptr(rp), _ptr(c), _ptr(v), v.itemsize, _ptr(I), len(I),
                                 _ptr(J), len(J), _ptr(r), ns, _ptr(ptr), _ptr(oc), _ptr(ov), cap,
                                 ctypes.byref(need), int(threads))
    return _two_call(fn, nout, v.dtype)


def spasgn(A, B, I, J, op="second", rows=None, lib=None, threads=1):
    """Rows of A_new = A (+) B' with B'[I[i], J[j]] = B[i, j] for stored B entries."""
    lib = lib or _load()
    m, n, rp, c, v = _csr(A)
    bm, bn, brp, bc, bv = _csr(B)
    if bv.dtype != v.dtype:
        raise OracleError(1)
    I = _ivec(I)
    J = _ivec(J)
    r, ns = _rows(rows)
    nout = ns if r is not None else m

    def fn(ptr, oc, ov, cap, need):
        return lib.orc_spasgn(m, n, _ptr(rp), _ptr(c), _ptr(v), v.itemsize, bm, bn, _ptr(brp),
                              _ptr(bc), _ptr(bv), _ptr(I), len(I), _ptr(J), len(J), OPS[op],
                              _ptr(r), ns, _ptr(ptr), _ptr(oc), _ptr(ov), cap, ctypes.byref(need),
                              int(threads))
    return _two_call(fn, nout, v.dtype)


def _dcsc(A):
    """(m, n, nzc, jc or None, colptr int64, row int32, val) as numpy arrays;
    A has attributes nrows, ncols, jc (None for CSC), colptr, row, val, or is
    that tuple."""
    if hasattr(A, "colptr"):
        m, n, jc, cp, r, v = A.nrows, A.ncols, A.jc, A.colptr, A.row, A.val
    else:
        m, n, jc, cp, r, v = A
    conv = lambda t: t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    cp = np.ascontiguousarray(conv(cp), dtype=np.int64)
    r = np.ascontiguousarray(conv(r), dtype=np.int32)
    v = np.ascontiguousarray(conv(v))
    jc = None if jc is None else np.ascontiguousarray(conv(jc), dtype=np.int32)
    nzc = len(cp) - 1
    return m, n, nzc, jc, cp, r, v


def spref_dcsc(A, I, J, cols=None, lib=None):
    """C = A(I, J) for column-compressed A (CSC, or DCSC with jc): returns
    the CSC of C, (colptr int64 [len(cols)+1], row int32, val), for the
    requested output columns (all when cols is None)."""
    lib = lib or _load()
    m, n, nzc, jc, cp, r, v = _dcsc(A)
    I = _ivec(I)
    J = _ivec(J)
    c, ns = _rows(cols)
    nout = ns if c is not None else len(J)

    def fn(ptr, orow, ov, cap, need):
        return lib.orc_spref_dcsc(m, n, nzc, _ptr(jc), _ptr(cp), _ptr(r), _ptr(v), v.itemsize, _ptr(I), len(I),
                                  _ptr(J), len(J), _ptr(c), ns, _ptr(ptr), _ptr(orow), _ptr(ov), cap,
                                  ctypes.byref(need))
    return _two_call(fn, nout, v.dtype)
