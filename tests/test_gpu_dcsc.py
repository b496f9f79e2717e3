"""GPU parity for extraction on column-compressed storage (CSC and DCSC):
C = A(I, J) returned in CSC, bit-exact against the oracle's column walk
(appendix Alg. 5)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import bits, mixed_csr

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _np(C):
    return (C.colptr.cpu().numpy().astype(np.int64), C.row.cpu().numpy(), C.val.cpu().numpy())


def _same(got, exp, what):
    gp, gr, gv = got
    ep, er, ev = exp
    assert np.array_equal(gp, np.asarray(ep, np.int64)), f"{what}: colptr differs"
    assert np.array_equal(gr, er), f"{what}: row differs"
    assert np.array_equal(bits(gv), bits(ev)), f"{what}: val bits differ"


def _compress(A):
    """DCSC of a CSC: keep the non-empty columns."""
    cp = A.colptr.long()
    nz = torch.nonzero(cp[1:] - cp[:-1]).flatten()
    colptr = torch.zeros(nz.numel() + 1, dtype=torch.int64, device=cp.device)
    colptr[1:] = torch.cumsum((cp[1:] - cp[:-1])[nz], 0)
    return synth.DCSC(A.nrows, A.ncols, nz.to(torch.int32), colptr.to(A.colptr.dtype), A.row, A.val)


def _csc_with_column_lengths(seed, m, n, lengths, ptr, vdt):
    """CSC whose column c has lengths[c % len(lengths)] rows (a CSR of the
    transpose read as CSC)."""
    T = mixed_csr(seed, n, m, lengths, ptr, vdt)
    return synth.DCSC(m, n, None, T.rowptr, T.col, T.val)


@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
@pytest.mark.parametrize("compress", [True, False])
def test_hypersparse_small(hp, ptr, vdt, compress):
    _say(f"dcsc: hypersparse 3000 x 20000, compress {compress}, ptr {ptr}, val {vdt}")
    A = synth.dcsc_uniform(3000, 20000, 6000, 1, "t-hyper", ptr, vdt, compress, "cuda")
    I = synth.subset(2, A.nrows, 900, repeat_frac=0.05, device="cuda")
    J = synth.subset(3, A.ncols, 7000, repeat_frac=0.05, device="cuda")
    _same(_np(hp.spref_dcsc(A, I, J)), oracle.spref_dcsc(A, I, J), "hypersparse")
    Is, Js = torch.sort(I).values, torch.sort(J).values
    _same(_np(hp.spref_dcsc(A, Is, Js)), oracle.spref_dcsc(A, Is, Js), "sorted I, J")


@pytest.mark.parametrize("compress", [True, False])
def test_columns_of_every_sort_class(hp, compress):
    """Output columns of every length class (selected rows repeated so that
    some output columns exceed the block-sort limit)."""
    _say(f"dcsc: long columns, compress {compress}")
    A = _csc_with_column_lengths(21, 6000, 400, [0, 1, 3, 17, 0, 70, 300, 2500, 5000, 0], torch.int64,
                                 torch.float64)
    if compress:
        A = _compress(A)
    rng = np.random.default_rng(22)
    I = torch.as_tensor(np.concatenate([rng.permutation(6000), rng.choice(6000, 1500)]).astype(np.int32),
                        device="cuda")
    J = synth.subset(23, A.ncols, 300, repeat_frac=0.1, device="cuda")
    _same(_np(hp.spref_dcsc(A, I, J)), oracle.spref_dcsc(A, I, J), "every class")


def test_edges_and_errors(hp):
    _say("dcsc: empty I and J, unstored columns only, range errors")
    A = synth.dcsc_uniform(200, 5000, 300, 31, "t-edge", torch.int32, torch.float64, True, "cuda")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    J = synth.subset(32, A.ncols, 400, device="cuda")
    I = synth.subset(33, A.nrows, 50, device="cuda")
    _same(_np(hp.spref_dcsc(A, e, J)), oracle.spref_dcsc(A, e, J), "empty I")
    _same(_np(hp.spref_dcsc(A, I, e)), oracle.spref_dcsc(A, I, e), "empty J")
    stored = set(A.jc.cpu().tolist())
    unstored = torch.tensor([c for c in range(A.ncols) if c not in stored][:100], dtype=torch.int32,
                            device="cuda")
    C = hp.spref_dcsc(A, I, unstored)
    assert C.nnz == 0 and int(C.colptr[-1]) == 0
    empty = synth.DCSC(200, 5000, e, torch.zeros(1, dtype=torch.int32, device="cuda"), e,
                       torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert hp.spref_dcsc(empty, I, J).nnz == 0
    with pytest.raises(hp.HPError) as ex:
        hp.spref_dcsc(A, torch.tensor([0, 200], dtype=torch.int32, device="cuda"), J)
    assert ex.value.name == "HP_ERR_INDEX_RANGE"
    with pytest.raises(hp.HPError) as ex:
        hp.spref_dcsc(A, I, torch.tensor([5000], dtype=torch.int32, device="cuda"))
    assert ex.value.name == "HP_ERR_INDEX_RANGE"


def test_hypersparse_full_size(hp):
    """2^26 x 2^26 with 2^24 nonzeros in DCSC, I and J 25% with 1% repeats:
    sampled output columns against the oracle, and the whole result equal to
    the plain CSC of the same matrix."""
    _say("dcsc: 2^26 hypersparse, full size")
    w = synth.workload_hypersparse(scale=26, device="cuda")
    A, I, J = w["A"], w["I"], w["J"]
    C = hp.spref_dcsc(A, I, J)
    torch.cuda.synchronize()
    # the same matrix as plain CSC (every column pointer stored)
    cp = torch.zeros(A.ncols + 1, dtype=torch.int64, device="cuda")
    cnt = A.colptr[1:] - A.colptr[:-1]
    cp.index_add_(0, A.jc.long() + 1, cnt)
    cp = torch.cumsum(cp, 0)
    Ac = synth.DCSC(A.nrows, A.ncols, None, cp, A.row, A.val)
    C2 = hp.spref_dcsc(Ac, I, J)
    assert torch.equal(C.colptr, C2.colptr) and torch.equal(C.row, C2.row)
    assert torch.equal(C.val.view(torch.int64), C2.val.view(torch.int64))
    del C2, Ac
    cols = np.sort(np.random.default_rng(41).choice(J.numel(), 6, replace=False)).astype(np.int64)
    got_cp = C.colptr.cpu().numpy()
    rows = C.row.cpu().numpy()
    vals = C.val.cpu().numpy()
    ep, er, ev = oracle.spref_dcsc(A, I, J, cols=cols)
    for s, j in enumerate(cols):
        a, b = got_cp[j], got_cp[j + 1]
        c, d = ep[s], ep[s + 1]
        assert np.array_equal(rows[a:b], er[c:d]), f"column {j}: rows"
        assert np.array_equal(bits(vals[a:b]), bits(ev[c:d])), f"column {j}: values"


def test_argument_errors(hp):
    """Malformed descriptors are rejected on the host, before any launch."""
    _say("dcsc: argument errors")
    A = synth.dcsc_uniform(100, 400, 200, 61, "t-arg", torch.int32, torch.float64, True, "cuda")
    I = synth.subset(62, A.nrows, 20, device="cuda")
    J = synth.subset(63, A.ncols, 30, device="cuda")
    h = hp.handle(0)
    Ad = hp.to_dcsc_t(A)
    need = hp._SZ(0)
    import ctypes
    h.check(hp.hp_spref_dcsc_workspace(h.h, ctypes.byref(Ad), 20, 30, ctypes.byref(need)))
    bad = hp.to_dcsc_t(A)
    bad.dcsc = 2
    assert hp.hp_spref_dcsc_workspace(h.h, ctypes.byref(bad), 20, 30, ctypes.byref(need)) == 1
    bad = hp.to_dcsc_t(A)
    bad.nzc = A.ncols + 1
    assert hp.hp_spref_dcsc_workspace(h.h, ctypes.byref(bad), 20, 30, ctypes.byref(need)) == 1
    bad = hp.to_dcsc_t(A)
    bad.jc = None
    assert hp.hp_spref_dcsc_workspace(h.h, ctypes.byref(bad), 20, 30, ctypes.byref(need)) == 1
    C, ws, info = h.spref_dcsc_plan(A, I, J)
    Cc = hp.to_dcsc_t(C)
    Cc.dcsc = 1   # the output is CSC
    Ac = hp.to_dcsc_t(A)
    assert hp.hp_spref_dcsc_exec(h.h, ctypes.byref(Ac), hp._idx(I), 20, hp._idx(J), 30, ctypes.byref(Cc),
                                 hp._dptr(ws), ws.numel(), ctypes.byref(info), None, 0) == 1
    h.spref_dcsc_exec(A, I, J, C, ws, info)   # the proper call still works
    assert C.nnz == oracle.spref_dcsc(A, I, J)[0][-1]


@pytest.mark.parametrize("ptr", [torch.int32, torch.int64])
def test_crowded_and_sparse_buckets(hp, ptr):
    """Stored columns packed at the low ids (hundreds per bucket of the
    column index: the searched lookup) and scattered over the rest (a few
    per bucket: the loaded-together lookup), against the oracle."""
    m, n = 3000, 100_000
    dense = mixed_csr(71, 1000, m, [0, 1, 4, 30, 300], ptr, torch.float64)   # columns 0..999 as rows of A^T
    rng = np.random.default_rng(72)
    far = np.sort(rng.choice(np.arange(1000, n), 600, replace=False)).astype(np.int32)
    far_rows = [np.sort(rng.choice(m, int(k), replace=False)).astype(np.int32) for k in rng.integers(1, 6, far.size)]
    dp = dense.rowptr.cpu().numpy().astype(np.int64)
    keep = np.nonzero(np.diff(dp))[0].astype(np.int32)          # stored (non-empty) low columns
    jc = np.concatenate([keep, far])
    cnt = np.concatenate([np.diff(dp)[keep], [len(r) for r in far_rows]]).astype(np.int64)
    colptr = np.zeros(jc.size + 1, dtype=np.int64)
    colptr[1:] = np.cumsum(cnt)
    row = np.concatenate([dense.col.cpu().numpy()] + far_rows).astype(np.int32)
    val = synth.values(synth.stream_key(73, "crowded"), row.size, torch.float64)
    A = synth.DCSC(m, n, torch.as_tensor(jc, device="cuda"), torch.as_tensor(colptr).to(ptr).cuda(),
                   torch.as_tensor(row, device="cuda"), val.cuda())
    I = synth.subset(74, m, 1500, repeat_frac=0.05, device="cuda")
    J = torch.as_tensor(np.concatenate([rng.integers(0, 1000, 3000), rng.choice(far, 400),
                                        rng.integers(1000, n, 3000)]).astype(np.int32), device="cuda")
    _same(_np(hp.spref_dcsc(A, I, J)), oracle.spref_dcsc(A, I, J), "crowded and sparse buckets")
