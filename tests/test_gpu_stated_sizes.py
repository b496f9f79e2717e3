"""Whole-output parity at the workloads' stated sizes.

Every test here compares the complete GPU output, byte for byte, with the
oracle's routines through inverse index tables (their cost is the entries
read, so whole outputs at full size finish in seconds on the host cores),
or, for the served form, with the same request run alone through the plain
calls:
  - R-MAT extraction: scale 22, edge factor 16, symmetrised, int32 CSR,
    fp32; I, J random 25% subsets, unsorted, 1% repeated indices;
  - grid: 4096 x 4096 5-point grid (int64 row pointers, fp64), general
    permutation P A Q^T, the select-second assignment of a Bernoulli(1e-4)
    block into a contiguous 10% range, and the two fused;
  - batched: 512 extraction / permutation requests over 64 R-MAT matrices
    of scale 12-20 and edge factor 8-32, every result against its plain
    call and against the oracle;
  - served: Poisson arrivals at 2,000 requests/s, 60/20/20 extraction /
    assignment / permutation over 32 resident R-MAT and Erdos-Renyi
    matrices of scale 16-24 (int32 and int64 row pointers), every result
    in the mix against the same request alone.
"""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, np_csr

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))   # host threads for the oracle


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _host(A):
    """(m, n, rowptr int64, col, val) numpy tuple of a device CSR."""
    return (A.nrows, A.ncols, A.rowptr.cpu().numpy().astype(np.int64), A.col.cpu().numpy(), A.val.cpu().numpy())


def _bits(t):
    return t.view(torch.int64 if t.element_size() == 8 else torch.int32)


def _equal_dev(X, Y):
    return (X.nrows == Y.nrows and X.ncols == Y.ncols and torch.equal(X.rowptr, Y.rowptr)
            and torch.equal(X.col, Y.col) and torch.equal(_bits(X.val), _bits(Y.val)))


@pytest.mark.timeout(900)
def test_rmat_extract_whole_output(hp):
    _say(f"stated size: R-MAT scale 22 extraction, whole output vs oracle ({NT} threads)")
    w = synth.workload_rmat_extract(device="cuda")
    A, I, J = w["A"], w["I"], w["J"]
    C = hp.spref(A, I, J)
    got = np_csr(C)
    t = time.perf_counter()
    exp = oracle.spref_map(_host(A), I, J, threads=NT)
    _say(f"  oracle {time.perf_counter() - t:.1f}s, {C.nnz} entries")
    assert_same(got, exp, "R-MAT extraction")


@pytest.mark.timeout(900)
def test_grid_permute_whole_output(hp):
    _say(f"stated size: 4096^2 grid permutation, whole output vs oracle ({NT} threads)")
    w = synth.workload_grid(side=4096, with_block=False, device="cuda")
    A, p, q = w["A"], w["p"], w["q"]
    C = hp.permute(A, p, q)
    got = np_csr(C)
    del C
    t = time.perf_counter()
    exp = oracle.permute_map(_host(A), p, q, threads=NT)
    _say(f"  oracle {time.perf_counter() - t:.1f}s")
    assert_same(got, exp, "grid permutation")


@pytest.mark.timeout(900)
def test_grid_assign_and_fused_whole_output(hp):
    _say(f"stated size: 4096^2 grid assignment (select-second) and fused update, whole outputs vs oracle")
    w = synth.workload_grid(side=4096, device="cuda")
    A, B, I, J, p, q = w["A"], w["B"], w["I"], w["J"], w["p"], w["q"]
    Ah, Bh = _host(A), _host(B)
    t = time.perf_counter()
    X = oracle.spasgn(Ah, Bh, I, J, "second", threads=NT)
    _say(f"  oracle assignment {time.perf_counter() - t:.1f}s, {len(X[1])} entries")
    C = hp.spasgn(A, B, I, J, "second")
    assert_same(np_csr(C), X, "grid assignment")
    del C
    torch.cuda.empty_cache()
    t = time.perf_counter()
    exp = oracle.permute_map((A.nrows, A.ncols) + tuple(X), p, q, threads=NT)
    _say(f"  oracle permutation of the assignment {time.perf_counter() - t:.1f}s")
    del X
    F = hp.spasgn_permute(A, B, I, J, p, q, "second")
    assert_same(np_csr(F), exp, "fused assignment and permutation")


def _plain(hp, r):
    if r["kind"] == "spref":
        return hp.spref(r["A"], r["I"], r["J"])
    if r["kind"] == "permute":
        return hp.permute(r["A"], r["p"], r.get("q"))
    return hp.spasgn(r["A"], r["B"], r["I"], r["J"], r["op"])


@pytest.mark.timeout(900)
def test_batched_512_requests_stated_size(hp):
    _say("stated size: batched form, 512 requests over 64 R-MAT (scale 12-20, ef 8-32)")
    pool = synth.batched_pool(device="cuda")
    reqs = synth.batched_requests(pool, device="cuda")
    for r in reqs:
        r["A"] = pool[r["mat"]]
    b = hp.Batch(hp.handle(0), reqs)
    st = b.plan()
    assert all(s == 0 for s in st), st
    b.exec()
    got = b.results()
    torch.cuda.synchronize()
    _say("  every result against its plain call")
    for k, r in enumerate(reqs):
        assert _equal_dev(got[k], _plain(hp, r)), f"request {k} ({r['kind']}) differs from its plain call"
    _say(f"  every result against the oracle ({NT} threads)")
    hosts = {}
    t = time.perf_counter()
    for k, r in enumerate(reqs):
        if r["mat"] not in hosts:
            hosts[r["mat"]] = _host(r["A"])
        Ah = hosts[r["mat"]]
        if r["kind"] == "spref":
            exp = oracle.spref_map(Ah, r["I"], r["J"], threads=NT)
        else:
            exp = oracle.permute_map(Ah, r["p"], r["q"], threads=NT)
        assert_same(np_csr(got[k]), exp, f"request {k} ({r['kind']}) vs oracle")
    _say(f"  oracle over 512 requests {time.perf_counter() - t:.1f}s")


def _submit(srv, r):
    if r["kind"] == "spref":
        return srv.submit("spref", r["A"], I=r["I"], J=r["J"])
    if r["kind"] == "permute":
        return srv.submit("permute", r["A"], p=r["p"], q=r["q"])
    return srv.submit("spasgn", r["A"], I=r["I"], J=r["J"], B=r["B"], op=r["op"])


@pytest.mark.timeout(1200)
def test_served_stated_size_alone_equals_mix(hp):
    _say("stated size: served form, 32 matrices of scale 16-24, Poisson 2000 req/s, 60/20/20")
    t = time.perf_counter()
    pool = synth.served_pool(0, 32, 16, 24, device="cuda")
    var = synth.served_variants(pool, 0, 4, device="cuda")
    torch.cuda.synchronize()
    _say(f"  pool of {len(pool)} ({sum(A.nnz for A in pool)} nnz, scales 16-24, int32/int64 rowptr) "
         f"in {time.perf_counter() - t:.1f}s")
    assert {A.rowptr.dtype for A in pool} == {torch.int32, torch.int64}
    assert max(A.nrows for A in pool) == 1 << 24
    arr, trace = synth.served_trace(var, 2000.0, 0.12, 0)
    arr = arr.numpy()
    kinds = [r["kind"] for r in trace]
    assert {"spref", "spasgn", "permute"} <= set(kinds)
    srv = hp.Server(96 << 30, max_inflight=4, max_batch=16)
    wave = 40
    batched = 0
    for w0 in range(0, len(trace), wave):
        part = list(range(w0, min(len(trace), w0 + wave)))
        _say(f"  requests {part[0]}-{part[-1]} of {len(trace)}: mix")
        ids = {}
        t0 = time.perf_counter()
        for k in part:                           # arrivals at the trace's times
            dt = (arr[k] - arr[part[0]]) - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            ids[_submit(srv, trace[k])] = k
        srv.drain()
        done = {}
        while len(done) < len(part):
            for c in srv.poll():
                done[ids[c["id"]]] = c
        _say(f"  requests {part[0]}-{part[-1]}: alone, compared")
        for k in part:
            c = done[k]
            assert c["status"] == 0, (k, trace[k]["kind"], c["status"])
            batched += c["batch_size"] > 1
            alone = _plain(hp, trace[k])
            assert _equal_dev(c["C"], alone), f"request {k} ({trace[k]['kind']}) differs alone and in the mix"
            del alone
            srv.release(c["id"])
    assert srv.memory()[0] == 0
    srv.close()
    assert batched > 0, "no request ran batched with another"
    _say(f"  {len(trace)} requests, {batched} ran in a batch of more than one")
