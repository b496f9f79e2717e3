"""Helpers for GPU parity tests: seeded inputs with controlled row lengths,
GPU/CPU conversions and bit-exact comparison against the oracle."""
from __future__ import annotations

import numpy as np
import torch

import synth


def mixed_csr(seed, m, n, lengths, ptr_dtype=torch.int32, val_dtype=torch.float64, device="cuda"):
    """CSR whose row r has lengths[r % len(lengths)] distinct random columns."""
    rng = np.random.default_rng(seed)
    lens = np.array([min(lengths[r % len(lengths)], n) for r in range(m)], dtype=np.int64)
    rng.shuffle(lens)
    cols = []
    for r in range(m):
        L = int(lens[r])
        if L == 0:
            continue
        if L * 4 > n:
            c = np.sort(rng.choice(n, L, replace=False))
        else:
            c = np.unique(rng.integers(0, n, 2 * L))[:L]
            while len(c) < L:
                c = np.unique(np.concatenate([c, rng.integers(0, n, L)]))[:L]
            c = np.sort(rng.permutation(c)[:L])
        cols.append(c)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(lens)
    val = synth.values(synth.stream_key(seed, "mixed-val"), len(col), val_dtype)
    return synth.CSR(m, n, torch.from_numpy(rowptr).to(ptr_dtype).to(device),
                     torch.from_numpy(col).to(device), val.to(device))


def np_csr(C):
    return (C.rowptr.cpu().numpy().astype(np.int64), C.col.cpu().numpy(), C.val.cpu().numpy())


def bits(v):
    v = np.asarray(v)
    return v.view(np.uint64 if v.itemsize == 8 else np.uint32)


def assert_same(got, exp, what=""):
    grp, gc, gv = got
    erp, ec, ev = exp
    assert np.array_equal(np.asarray(grp, np.int64), np.asarray(erp, np.int64)), f"{what}: rowptr differs"
    assert np.array_equal(gc, ec), f"{what}: col differs"
    assert np.array_equal(bits(gv), bits(ev)), f"{what}: val bits differ"


def rows_of(C, rows):
    """(rowptr, col, val) of the listed rows of a GPU/CPU CSR, as numpy."""
    rp = C.rowptr.cpu().numpy().astype(np.int64)
    col = C.col.cpu().numpy()
    val = C.val.cpu().numpy()
    out_rp = [0]
    cs, vs = [], []
    for r in rows:
        a, b = rp[r], rp[r + 1]
        cs.append(col[a:b])
        vs.append(val[a:b])
        out_rp.append(out_rp[-1] + (b - a))
    return (np.array(out_rp, np.int64),
            np.concatenate(cs) if cs else np.zeros(0, np.int32),
            np.concatenate(vs) if vs else np.zeros(0, val.dtype))


def sample_rows(seed, nrows, k):
    rng = np.random.default_rng(seed)
    k = min(k, nrows)
    pick = rng.choice(nrows, k, replace=False)
    return np.sort(np.concatenate([pick, [0, nrows - 1]]).astype(np.int64))
