"""Shared helpers for the tests: independent reference computations (dense
brute force, SciPy), tiny random inputs and golden-file parsing."""
from __future__ import annotations

import os

import numpy as np
import scipy.sparse as sp

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rand_csr(rng, m, n, density, vdtype=np.float64, ptr_dtype=np.int64):
    """Tiny random canonical CSR with values in (0, 1] (no zeros)."""
    mask = rng.random((m, n)) < density
    rowptr = np.zeros(m + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(mask.sum(1))
    col = np.nonzero(mask)[1].astype(np.int32)
    val = (rng.integers(1, 2 ** 20, size=col.size) / 2 ** 20).astype(vdtype)
    return (m, n, rowptr.astype(ptr_dtype), col, val)


def dense(A):
    """(values, pattern) dense pair; the pattern keeps stored zeros apart."""
    m, n, rp, c, v = A
    D = np.zeros((m, n), dtype=v.dtype)
    M = np.zeros((m, n), dtype=bool)
    rp = np.asarray(rp, dtype=np.int64)
    for r in range(m):
        for k in range(rp[r], rp[r + 1]):
            D[r, c[k]] = v[k]
            M[r, c[k]] = True
    return D, M


def from_dense(D, M):
    """CSR triple from a dense (values, pattern) pair, columns ascending."""
    m = D.shape[0]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    cols, vals = [], []
    for r in range(m):
        cc = np.nonzero(M[r])[0]
        cols.append(cc)
        vals.append(D[r, cc])
        rowptr[r + 1] = rowptr[r] + len(cc)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals).astype(D.dtype) if vals else np.zeros(0, D.dtype)
    return rowptr, col, val


def to_scipy(A):
    m, n, rp, c, v = A
    return sp.csr_matrix((np.asarray(v), np.asarray(c), np.asarray(rp, dtype=np.int64)), shape=(m, n))


def from_scipy(S):
    S = S.tocsr().copy()
    S.sort_indices()
    return (np.asarray(S.indptr, dtype=np.int64), np.asarray(S.indices, dtype=np.int32),
            np.asarray(S.data))


def selection(idx, ncols, dtype):
    """Boolean selection matrix R with R[i, idx[i]] = 1 (Sec. 2 formulations)."""
    k = len(idx)
    return sp.csr_matrix((np.ones(k, dtype=dtype), np.asarray(idx, dtype=np.int64),
                          np.arange(k + 1, dtype=np.int64)), shape=(k, ncols))


def bits(v):
    v = np.asarray(v)
    return v.view(np.uint64 if v.itemsize == 8 else np.uint32)


def assert_csr_equal(got, exp, what=""):
    grp, gc, gv = got
    erp, ec, ev = exp
    np.testing.assert_array_equal(np.asarray(grp, dtype=np.int64), np.asarray(erp, dtype=np.int64),
                                  err_msg=f"{what}: rowptr")
    np.testing.assert_array_equal(np.asarray(gc), np.asarray(ec), err_msg=f"{what}: col")
    np.testing.assert_array_equal(bits(gv), bits(np.asarray(ev, dtype=np.asarray(gv).dtype)),
                                  err_msg=f"{what}: val bits")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            out[key] = rest
    return out


def ints(xs):
    return np.array([int(x) for x in xs], dtype=np.int64)


def floats(xs, dtype=np.float64):
    return np.array([float(x) for x in xs], dtype=dtype)


def to_dcsc(A, compress=True):
    """(m, n, jc or None, colptr, row, val) of a CSR triple: the CSC from
    SciPy, and with compress the stored non-empty columns only (DCSC)."""
    m, n = A[0], A[1]
    S = to_scipy(A).tocsc()
    S.sort_indices()
    cp = np.asarray(S.indptr, dtype=np.int64)
    if not compress:
        return (m, n, None, cp, np.asarray(S.indices, dtype=np.int32), np.asarray(S.data))
    nz = np.nonzero(np.diff(cp))[0]
    cpz = np.concatenate([[0], np.cumsum(np.diff(cp)[nz])]).astype(np.int64)
    return (m, n, nz.astype(np.int32), cpz, np.asarray(S.indices, dtype=np.int32), np.asarray(S.data))


def csc_of(S):
    """(colptr, row, val) of a SciPy matrix in CSC with sorted row indices."""
    S = S.tocsc().copy()
    S.sort_indices()
    return (np.asarray(S.indptr, dtype=np.int64), np.asarray(S.indices, dtype=np.int32), np.asarray(S.data))
