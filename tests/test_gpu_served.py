"""Served form: every request's result is bit-identical alone (plain call)
and inside the concurrent mix; tight budgets make batches wait or split but
never change a result; a request that cannot fit is rejected alone."""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, np_csr

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _pool(ptr):
    out = [synth.rmat(s, 16, 3, f"srv{s}", symmetric=True, ptr_dtype=ptr, val_dtype=torch.float32, device="cuda")
           for s in (9, 11, 12)]
    out.append(synth.erdos_renyi(3000, 2500, 16.0, 4, "srv-er", ptr_dtype=ptr, val_dtype=torch.float32,
                                 device="cuda"))
    return out


def _requests(seed, count, pool):
    """60/20/20 extraction / assignment / permutation over the pool."""
    rng = np.random.default_rng(seed)
    reqs = []
    for t in range(count):
        A = pool[int(rng.integers(len(pool)))]
        u = rng.random()
        if u < 0.6:
            f1, f2 = rng.uniform(0.05, 0.5, 2)
            I = synth.subset(synth.stream_key(seed, "I", t), A.nrows, max(1, int(f1 * A.nrows)),
                             repeat_frac=0.01, device="cuda")
            J = synth.subset(synth.stream_key(seed, "J", t), A.ncols, max(1, int(f2 * A.ncols)),
                             repeat_frac=0.01, device="cuda")
            reqs.append(dict(kind="spref", A=A, I=I, J=J))
        elif u < 0.8:
            f1, f2 = rng.uniform(0.01, 0.1, 2)
            nI, nJ = max(1, int(f1 * A.nrows)), max(1, int(f2 * A.ncols))
            I = synth.subset(synth.stream_key(seed, "aI", t), A.nrows, nI, device="cuda")
            J = synth.subset(synth.stream_key(seed, "aJ", t), A.ncols, nJ, device="cuda")
            dens = min(1.0, 0.01 * A.nnz / (nI * nJ))
            B = synth.bernoulli_block(nI, nJ, dens, seed, f"aB{t}", ptr_dtype=A.rowptr.dtype,
                                      val_dtype=torch.float32, device="cuda")
            op = ["second", "plus", "replace"][t % 3]
            reqs.append(dict(kind="spasgn", A=A, I=I, J=J, B=B, op=op))
        else:
            p = synth.randperm(synth.stream_key(seed, "p", t), A.nrows, "cuda")
            q = synth.randperm(synth.stream_key(seed, "q", t), A.ncols, "cuda")
            reqs.append(dict(kind="permute", A=A, p=p, q=q))
    return reqs


def _alone(hp, r):
    if r["kind"] == "spref":
        return hp.spref(r["A"], r["I"], r["J"])
    if r["kind"] == "permute":
        return hp.permute(r["A"], r["p"], r["q"])
    return hp.spasgn(r["A"], r["B"], r["I"], r["J"], r["op"])


def _submit(srv, r):
    if r["kind"] == "spref":
        return srv.submit("spref", r["A"], I=r["I"], J=r["J"])
    if r["kind"] == "permute":
        return srv.submit("permute", r["A"], p=r["p"], q=r["q"])
    return srv.submit("spasgn", r["A"], I=r["I"], J=r["J"], B=r["B"], op=r["op"])


def _run_mix(hp, srv, reqs, gaps_s):
    ids = {}
    for k, r in enumerate(reqs):
        ids[_submit(srv, r)] = k
        if gaps_s[k] > 0:
            time.sleep(gaps_s[k])
    srv.drain()
    done = {}
    while len(done) < len(reqs):
        for c in srv.poll():
            done[ids[c["id"]]] = c
    return done


@pytest.mark.parametrize("ptr", [torch.int32, torch.int64])
def test_served_alone_equals_mix(hp, ptr):
    _say(f"served: 60 requests, mixed kinds, ptr {ptr}")
    pool = _pool(ptr)
    reqs = _requests(5, 60, pool)
    alone = [np_csr(_alone(hp, r)) for r in reqs]
    torch.cuda.synchronize()
    srv = hp.Server(512 << 20, max_inflight=4, max_batch=64)
    rng = np.random.default_rng(1)
    gaps = np.where(rng.random(len(reqs)) < 0.3, rng.exponential(0.002, len(reqs)), 0.0)
    done = _run_mix(hp, srv, reqs, gaps)
    for k, r in enumerate(reqs):
        c = done[k]
        assert c["status"] == 0, (k, r["kind"], c["status"])
        assert_same(np_csr(c["C"]), alone[k], f"request {k} ({r['kind']})")
        assert c["t_submit_ns"] <= c["t_start_ns"] <= c["t_done_ns"]
    assert max(c["batch_size"] for c in done.values()) > 1, "no request was batched with another"
    for k in (0, 1, 2):
        r = reqs[k]
        if r["kind"] == "spref":
            assert_same(np_csr(done[k]["C"]), oracle.spref(r["A"], r["I"], r["J"]), "vs oracle")
    for c in done.values():
        srv.release(c["id"])
    assert srv.memory()[0] == 0
    srv.close()


def test_served_tight_budget_and_rejection(hp):
    _say("served: tight budget (waits and splits), one request that cannot fit")
    pool = _pool(torch.int32)
    reqs = _requests(9, 30, pool[:2])
    alone = [np_csr(_alone(hp, r)) for r in reqs]
    torch.cuda.synchronize()
    srv = hp.Server(24 << 20, max_inflight=3, max_batch=16)
    big = synth.rmat(17, 16, 6, "srv-big", symmetric=True, device="cuda")   # ~4M nnz: output > budget
    pbig = synth.randperm(7, big.nrows, "cuda")
    ids = {}
    for k, r in enumerate(reqs):
        ids[_submit(srv, r)] = k
    bid = srv.submit("permute", big, p=pbig, q=pbig)
    srv.drain()
    got = {}
    for c in srv.poll():
        got[c["id"]] = c
    assert got[bid]["status"] == 13, got[bid]["status"]          # HP_ERR_REJECTED
    for rid, k in ids.items():
        c = got[rid]
        assert c["status"] == 0, (k, c["status"])
        assert_same(np_csr(c["C"]), alone[k], f"request {k}")
        srv.release(rid)
    assert srv.memory()[0] == 0
    assert srv.memory()[1] <= 24 << 20
    srv.close()


def test_served_rejects_invalid_at_submit(hp):
    A = synth.rmat(8, 8, 1, "srv-inv", device="cuda")
    srv = hp.Server(8 << 20, max_inflight=1)
    I = torch.arange(4, dtype=torch.int32, device="cuda")
    B = synth.bernoulli_block(3, 4, 0.5, 0, "srv-b", ptr_dtype=torch.int32, val_dtype=torch.float32, device="cuda")
    with pytest.raises(hp.HPError):
        srv.submit("spasgn", A, I=I, J=I, B=B)          # B is 3 x 4, I has 4 entries
    bad = torch.zeros(A.nrows, dtype=torch.int32, device="cuda")
    rid = srv.submit("permute", A, p=bad, q=None)          # not a permutation: fails at plan
    srv.drain()
    (c,) = srv.poll()
    assert c["id"] == rid and c["status"] == 3
    srv.close()


def test_served_inputs_written_asynchronously(hp):
    """Inputs still being written on the caller's stream when they are
    submitted: each request carries an event of that stream and the worker
    waits for it, so the results equal the same requests run alone.  No
    global synchronisation between writing the inputs and submitting."""
    _say("served: inputs written by queued work, submitted at once")
    A = synth.rmat(12, 16, 11, "srv-async", symmetric=True, device="cuda")
    busy = torch.randn(4096, 4096, device="cuda")
    srv = hp.Server(256 << 20, max_inflight=4, max_batch=8)
    subs = {}
    torch.cuda.synchronize()
    for t in range(16):
        busy = busy @ busy * 1e-3          # keeps the stream busy before the copies below
        B = synth.CSR(A.nrows, A.ncols, torch.empty_like(A.rowptr).fill_(-1), torch.empty_like(A.col).fill_(-1),
                      torch.empty_like(A.val).fill_(float("nan")))
        B.rowptr.copy_(A.rowptr)
        B.col.copy_(A.col)
        B.val.copy_(A.val)
        perm = torch.randperm(A.nrows, device="cuda").to(torch.int32)
        if t % 2:
            I = perm[: A.nrows // 3]
            subs[srv.submit("spref", B, I=I, J=I)] = ("spref", I)
        else:
            subs[srv.submit("permute", B, p=perm, q=None)] = ("permute", perm)
    srv.drain()
    got = {}
    while len(got) < len(subs):
        for c in srv.poll():
            got[c["id"]] = c
    for rid, c in got.items():
        assert c["status"] == 0, c["status"]
        kind, x = subs[rid]
        alone = hp.spref(A, x, x) if kind == "spref" else hp.permute(A, x)
        assert_same(np_csr(c["C"]), np_csr(alone), f"request {rid} ({kind})")
        srv.release(rid)
    srv.close()
