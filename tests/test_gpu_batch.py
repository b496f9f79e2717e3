"""Batched form: every result bit-identical to the plain per-call path (and
to the oracle where checked); a failing request is isolated; re-running
the captured exec graph gives the same bytes."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, mixed_csr, np_csr

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="single-launch persistent batch kernel with device-side dependency counters "
                            "stalled in plan on the GPU twice (2 requests, R-MAT scale 6); that kernel was "
                            "removed and the batched form now runs as stream-ordered stage launches, "
                            "covered by test_gpu_batched.py"),
]


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def test_batch_tiny(hp):
    A = synth.rmat(6, 4, 2, "tiny", symmetric=False, device="cuda")
    p = synth.randperm(1, A.nrows, "cuda")
    I = synth.subset(2, A.nrows, 20, device="cuda")
    reqs = [dict(kind="permute", A=A, p=p), dict(kind="spref", A=A, I=I, J=I)]
    b = hp.Batch(hp.handle(0), reqs)
    assert b.plan() == [0, 0]
    b.exec()
    got = b.results()
    assert_same(np_csr(got[0]), oracle.permute(A, p), "tiny permute")
    assert_same(np_csr(got[1]), oracle.spref(A, I, I), "tiny spref")


def _reqs(seed, count, pool, ptr, vdt):
    rng = np.random.default_rng(seed)
    reqs = []
    for t in range(count):
        A = pool[t % len(pool)]
        kind = ["spref", "permute"][t % 2] if t % 7 else "spref"
        if kind == "permute":
            p = synth.randperm(synth.stream_key(seed, "p", t), A.nrows, "cuda")
            q = None if (t % 5 == 0 and A.nrows == A.ncols) else synth.randperm(synth.stream_key(seed, "q", t), A.ncols, "cuda")
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


def _plain(hp, r):
    if r["kind"] == "spref":
        return hp.spref(r["A"], r["I"], r["J"])
    return hp.permute(r["A"], r["p"], r.get("q"))


@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_batch_equals_plain(hp, ptr, vdt):
    pool = [synth.rmat(s, ef, 7, f"bp{s}", symmetric=False, ptr_dtype=ptr, val_dtype=vdt, device="cuda")
            for s, ef in [(8, 8), (10, 16), (12, 32), (13, 8)]]
    pool.append(mixed_csr(51, 500, 6000, [0, 1, 3, 17, 70, 300, 2500, 5000], ptr, vdt))
    reqs = _reqs(3, 40, pool, ptr, vdt)
    b = hp.Batch(hp.handle(0), reqs)
    st = b.plan()
    assert all(s == 0 for s in st), st
    b.exec()
    got = b.results()
    torch.cuda.synchronize()
    for k, r in enumerate(reqs):
        assert_same(np_csr(got[k]), np_csr(_plain(hp, r)), f"request {k} ({r['kind']})")
    for k in (0, 1, 2, 3):
        r = reqs[k]
        exp = oracle.spref(r["A"], r["I"], r["J"]) if r["kind"] == "spref" else oracle.permute(r["A"], r["p"], r.get("q"))
        assert_same(np_csr(got[k]), exp, f"request {k} vs oracle")
    # replaying the captured exec graph rewrites identical bytes
    first = [np_csr(c) for c in got]
    b.exec()
    again = b.results()
    for k in range(len(reqs)):
        assert_same(np_csr(again[k]), first[k], f"replay {k}")


def test_batch_isolates_failed_request(hp):
    A = synth.rmat(9, 8, 1, "bf", symmetric=False, device="cuda")
    p = synth.randperm(4, A.nrows, "cuda")
    bad = p.clone()
    bad[0] = bad[1]
    I = synth.subset(5, A.nrows, 100, device="cuda")
    reqs = [dict(kind="permute", A=A, p=p), dict(kind="permute", A=A, p=bad),
            dict(kind="spref", A=A, I=I, J=I), dict(kind="spref", A=A, I=torch.tensor([0, A.nrows], dtype=torch.int32, device="cuda"), J=I)]
    b = hp.Batch(hp.handle(0), reqs)
    st = b.plan()
    assert st == [0, 3, 0, 2], st
    b.exec()
    got = b.results()
    assert got[1] is None and got[3] is None
    assert_same(np_csr(got[0]), np_csr(hp.permute(A, p)), "ok permute")
    assert_same(np_csr(got[2]), np_csr(hp.spref(A, I, I)), "ok spref")
