"""Batched form (stage launches over all requests): every result is
bit-identical to the plain per-call path, and to the oracle where checked;
a failing request is isolated; replaying the captured exec graph rewrites
the same bytes."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, mixed_csr, np_csr

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _plain(hp, r):
    if r["kind"] == "spref":
        return hp.spref(r["A"], r["I"], r["J"])
    return hp.permute(r["A"], r["p"], r.get("q"))


def _oracle(r):
    if r["kind"] == "spref":
        return oracle.spref(r["A"], r["I"], r["J"])
    return oracle.permute(r["A"], r["p"], r.get("q"))


def test_batched_two_requests(hp):
    _say("batched: 2 requests, R-MAT scale 6")
    A = synth.rmat(6, 4, 2, "tiny", symmetric=False, device="cuda")
    p = synth.randperm(1, A.nrows, "cuda")
    I = synth.subset(2, A.nrows, 20, device="cuda")
    reqs = [dict(kind="permute", A=A, p=p), dict(kind="spref", A=A, I=I, J=I)]
    b = hp.Batch(hp.handle(0), reqs)
    assert b.plan() == [0, 0]
    b.exec()
    got = b.results()
    for k, r in enumerate(reqs):
        assert_same(np_csr(got[k]), _oracle(r), f"request {k} ({r['kind']})")


def _reqs(seed, count, pool):
    rng = np.random.default_rng(seed)
    reqs = []
    for t in range(count):
        A = pool[t % len(pool)]
        kind = ["spref", "permute"][t % 2] if t % 7 else "spref"
        if kind == "permute":
            p = synth.randperm(synth.stream_key(seed, "p", t), A.nrows, "cuda")
            sym = t % 5 == 0 and A.nrows == A.ncols
            q = None if sym else synth.randperm(synth.stream_key(seed, "q", t), A.ncols, "cuda")
            reqs.append(dict(kind="permute", A=A, p=p, q=q))
        else:
            fi, fj = rng.uniform(0.05, 0.5, 2)
            rep = 0.02 if t % 3 == 0 else 0.0
            srt = t % 4 == 1
            I = synth.subset(synth.stream_key(seed, "I", t), A.nrows, max(1, int(fi * A.nrows)), sort=srt,
                             repeat_frac=rep, device="cuda")
            J = synth.subset(synth.stream_key(seed, "J", t), A.ncols, max(1, int(fj * A.ncols)), sort=srt,
                             repeat_frac=rep, device="cuda")
            reqs.append(dict(kind="spref", A=A, I=I, J=J))
    return reqs


@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_batched_equals_plain(hp, ptr, vdt):
    _say(f"batched: 40 mixed requests, ptr {ptr}, val {vdt}")
    pool = [synth.rmat(s, ef, 7, f"bp{s}", symmetric=False, ptr_dtype=ptr, val_dtype=vdt, device="cuda")
            for s, ef in [(8, 8), (10, 16), (12, 32), (13, 8)]]
    # rows of every sort class, including rows above the block-sort limit
    pool.append(mixed_csr(51, 500, 6000, [0, 1, 3, 17, 70, 300, 2500, 5000], ptr, vdt))
    reqs = _reqs(3, 40, pool)
    b = hp.Batch(hp.handle(0), reqs)
    st = b.plan()
    assert all(s == 0 for s in st), st
    b.exec()
    got = b.results()
    torch.cuda.synchronize()
    for k, r in enumerate(reqs):
        assert_same(np_csr(got[k]), np_csr(_plain(hp, r)), f"request {k} ({r['kind']})")
    for k in (0, 1, 2, 3, 39):
        assert_same(np_csr(got[k]), _oracle(reqs[k]), f"request {k} vs oracle")
    _say("batched: graph replay")
    first = [np_csr(c) for c in got]
    for c in got:   # clobber the arena so the replay has to rewrite everything
        c.col.fill_(-7)
        c.val.fill_(-1.0)
    b.exec()
    again = b.results()
    for k in range(len(reqs)):
        assert_same(np_csr(again[k]), first[k], f"replay {k}")


def test_batched_edges(hp):
    _say("batched: empty index sets, empty matrix rows, single request")
    A = mixed_csr(9, 300, 400, [0, 0, 5, 40, 300], torch.int32, torch.float32)
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    I = synth.subset(11, A.nrows, 50, device="cuda")
    J = synth.subset(12, A.ncols, 80, repeat_frac=0.1, device="cuda")
    reqs = [dict(kind="spref", A=A, I=e, J=J), dict(kind="spref", A=A, I=I, J=e),
            dict(kind="spref", A=A, I=I, J=J), dict(kind="permute", A=A,
                                                  p=synth.randperm(13, A.nrows, "cuda"),
                                                  q=synth.randperm(14, A.ncols, "cuda"))]
    b = hp.Batch(hp.handle(0), reqs)
    assert b.plan() == [0, 0, 0, 0]
    b.exec()
    got = b.results()
    for k, r in enumerate(reqs):
        assert_same(np_csr(got[k]), _oracle(r), f"request {k}")
    one = hp.Batch(hp.handle(0), reqs[2:3])
    assert one.plan() == [0]
    one.exec()
    assert_same(np_csr(one.results()[0]), _oracle(reqs[2]), "single request")


def test_batched_isolates_failed_request(hp):
    _say("batched: failing requests beside good ones")
    A = synth.rmat(9, 8, 1, "bf", symmetric=False, device="cuda")
    p = synth.randperm(4, A.nrows, "cuda")
    bad = p.clone()
    bad[0] = bad[1]
    I = synth.subset(5, A.nrows, 100, device="cuda")
    out_of_range = torch.tensor([0, A.nrows], dtype=torch.int32, device="cuda")
    reqs = [dict(kind="permute", A=A, p=p), dict(kind="permute", A=A, p=bad),
            dict(kind="spref", A=A, I=I, J=I), dict(kind="spref", A=A, I=out_of_range, J=I)]
    b = hp.Batch(hp.handle(0), reqs)
    st = b.plan()
    assert st == [0, 3, 0, 2], st
    b.exec()
    got = b.results()
    assert got[1] is None and got[3] is None
    assert_same(np_csr(got[0]), np_csr(hp.permute(A, p)), "ok permute")
    assert_same(np_csr(got[2]), np_csr(hp.spref(A, I, I)), "ok spref")


def test_batched_long_rows_wide(hp):
    _say("batched: long rows with more than 2^20 output columns")
    n = 2_500_000
    A = mixed_csr(91, 24, n, [0, 5, 2500, 20000], torch.int32, torch.float32)
    I = synth.subset(92, A.nrows, 30, repeat_frac=0.2, device="cuda")
    J = synth.subset(93, n, 2_200_000, device="cuda")
    reqs = [dict(kind="spref", A=A, I=I, J=J),
            dict(kind="permute", A=A, p=synth.randperm(94, A.nrows, "cuda"), q=synth.randperm(95, n, "cuda")),
            dict(kind="spref", A=A, I=I, J=J[:900_000])]
    b = hp.Batch(hp.handle(0), reqs)
    assert b.plan() == [0, 0, 0]
    b.exec()
    got = b.results()
    for k, r in enumerate(reqs):
        assert_same(np_csr(got[k]), np_csr(_plain(hp, r)), f"request {k} ({r['kind']})")


def test_batched_with_assignment_requests(hp):
    """Assignment requests (all three operators) batched with extractions and
    permutations: every result equals its plain call and the oracle; a
    failing assignment (repeated index) is isolated; the replayed exec graph
    rewrites the same bytes."""
    _say("batched: assignment requests among extractions and permutations")
    pool = [synth.rmat(s, 8, 21, f"ba{s}", symmetric=True, ptr_dtype=torch.int64, val_dtype=torch.float64,
                       device="cuda") for s in (9, 11)]
    pool.append(mixed_csr(22, 700, 900, [0, 1, 4, 30, 300, 2500], torch.int64, torch.float64))
    reqs = []
    for t in range(12):
        A = pool[t % len(pool)]
        nI, nJ = max(1, A.nrows // (5 + t)), max(1, A.ncols // (4 + t))
        I = synth.subset(synth.stream_key(23, "I", t), A.nrows, nI, device="cuda")
        J = synth.subset(synth.stream_key(23, "J", t), A.ncols, nJ, device="cuda")
        if t % 3 == 0:
            B = synth.bernoulli_block(nI, nJ, 0.05, 24, f"bB{t}", ptr_dtype=torch.int64, val_dtype=torch.float64,
                                      device="cuda")
            reqs.append(dict(kind="spasgn", A=A, B=B, I=I, J=J, op=["second", "plus", "replace"][(t // 3) % 3]))
        elif t % 3 == 1:
            reqs.append(dict(kind="spref", A=A, I=I, J=J))
        else:
            reqs.append(dict(kind="permute", A=A, p=synth.randperm(synth.stream_key(23, "p", t), A.nrows, "cuda"),
                             q=synth.randperm(synth.stream_key(23, "q", t), A.ncols, "cuda")))
    A = pool[0]
    bad_I = torch.tensor([1, 1], dtype=torch.int32, device="cuda")
    Bb = synth.bernoulli_block(2, 3, 0.5, 25, "bBad", ptr_dtype=torch.int64, val_dtype=torch.float64, device="cuda")
    reqs.append(dict(kind="spasgn", A=A, B=Bb, I=bad_I, J=torch.arange(3, dtype=torch.int32, device="cuda"),
                     op="second"))
    b = hp.Batch(hp.handle(0), reqs)
    st = b.plan()
    assert st[:-1] == [0] * (len(reqs) - 1) and st[-1] == 4, st          # HP_ERR_DUPLICATE_INDEX
    b.exec()
    got = b.results()
    torch.cuda.synchronize()
    assert got[-1] is None
    for k, r in enumerate(reqs[:-1]):
        if r["kind"] == "spasgn":
            plain = hp.spasgn(r["A"], r["B"], r["I"], r["J"], r["op"])
            exp = oracle.spasgn(r["A"], r["B"], r["I"], r["J"], r["op"])
        elif r["kind"] == "spref":
            plain = hp.spref(r["A"], r["I"], r["J"])
            exp = oracle.spref_map(r["A"], r["I"], r["J"])
        else:
            plain = hp.permute(r["A"], r["p"], r["q"])
            exp = oracle.permute_map(r["A"], r["p"], r["q"])
        assert_same(np_csr(got[k]), np_csr(plain), f"request {k} ({r['kind']}) vs plain")
        assert_same(np_csr(got[k]), exp, f"request {k} ({r['kind']}) vs oracle")
    first = [np_csr(c) if c is not None else None for c in got]
    for c in got:
        if c is not None:
            c.col.fill_(-7)
            c.val.fill_(-1.0)
    b.exec()
    again = b.results()
    for k in range(len(reqs) - 1):
        assert_same(np_csr(again[k]), first[k], f"replay {k}")
