"""hp_permute_noalloc, the permutation entry point that allocates nothing,
against the existing hp_permute_plan / hp_permute_exec on the same inputs:
two calls in a row on one device (the second on a smaller matrix with rows
long enough to use the exec part of the scratch array), each bit-identical
to the plain calls and to the oracle; an input beyond the fixed scratch
size is rejected."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, mixed_csr, np_csr

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _bits(t):
    return t.view(torch.int64 if t.element_size() == 8 else torch.int32)


def _same_dev(X, Y, what):
    assert torch.equal(X.rowptr, Y.rowptr), f"{what}: rowptr"
    assert torch.equal(X.col, Y.col), f"{what}: col"
    assert torch.equal(_bits(X.val), _bits(Y.val)), f"{what}: val bits"


def _host(A):
    return (A.nrows, A.ncols, A.rowptr.cpu().numpy().astype(np.int64), A.col.cpu().numpy(), A.val.cpu().numpy())


def test_noalloc_equals_plan_exec_two_calls(hp):
    h = hp.handle(0)
    # first call: a random graph of 2^20 rows (int64 row pointers, fp64)
    m = 1 << 20
    _say(f"no-alloc permute: first call, random graph of {m} rows, general P A Q^T")
    A1 = synth.erdos_renyi(m, m, 6.0, 201, "na1", torch.int64, torch.float64, "cuda")
    p1 = synth.randperm(202, m, "cuda")
    q1 = synth.randperm(203, m, "cuda")
    C1 = h.permute_noalloc(A1, p1, q1)
    R1 = h.permute(A1, p1, q1)
    torch.cuda.synchronize()
    _same_dev(C1, R1, "first call vs plan/exec")
    assert_same(np_csr(C1), oracle.permute_map(_host(A1), p1, q1, threads=NT), "first call vs oracle")
    # second, smaller call: symmetric form, int32 / fp32, rows of every sort
    # class including some above 2048 entries (exec workspace in the scratch)
    _say("no-alloc permute: second call, 30000 rows with rows over 2048 entries, symmetric P A P^T")
    A2 = mixed_csr(204, 30000, 30000, [0, 1, 3, 5, 17, 70, 300, 0, 2, 4] * 30 + [2500, 6000],
                   torch.int32, torch.float32)
    p2 = synth.randperm(205, A2.nrows, "cuda")
    C2 = h.permute_noalloc(A2, p2)
    R2 = h.permute(A2, p2)
    torch.cuda.synchronize()
    _same_dev(C2, R2, "second call vs plan/exec")
    assert_same(np_csr(C2), oracle.permute_map(_host(A2), p2, None, threads=NT), "second call vs oracle")
    # the first result is untouched by the second call
    _same_dev(C1, R1, "first result after the second call")


def test_noalloc_rejects_inputs_beyond_the_scratch(hp):
    h = hp.handle(0)
    m = 1 << 22
    _say(f"no-alloc permute: {m} rows exceed the fixed scratch array")
    A = synth.CSR(m, m, torch.zeros(m + 1, dtype=torch.int32, device="cuda"),
                  torch.zeros(0, dtype=torch.int32, device="cuda"), torch.zeros(0, dtype=torch.float32, device="cuda"))
    p = torch.arange(m, dtype=torch.int32, device="cuda")
    with pytest.raises(hp.HPError) as e:
        h.permute_noalloc(A, p)
    assert e.value.name == "HP_ERR_WORKSPACE"
    # still usable afterwards, on a small input
    A3 = mixed_csr(206, 500, 400, [0, 2, 7, 40], torch.int64, torch.float64)
    p3, q3 = synth.randperm(207, 500, "cuda"), synth.randperm(208, 400, "cuda")
    _same_dev(h.permute_noalloc(A3, p3, q3), h.permute(A3, p3, q3), "small call after a rejection")
