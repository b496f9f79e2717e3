"""Incremental update driver: the fused and separate modes give the same
matrices; after the last step the matrix is A relabelled by the composed
permutations (the oracle's permutation of A), and A itself without
permutations; the block counts behind the load-imbalance metric match a
direct count."""
import sys

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
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm, incremental
    return hipperm, incremental


def _block_counts(A, gr, gc):
    rp, col, _ = np_csr(A)
    rows = np.repeat(np.arange(A.nrows), np.diff(rp))
    bi = rows * gr // A.nrows
    bj = col.astype(np.int64) * gc // A.ncols
    return np.bincount(bi * gc + bj, minlength=gr * gc)


def test_helpers(env):
    hp, _ = env
    _say("incremental: gather_index, invert_perm, block_nnz")
    h = hp.handle(0)
    p = synth.randperm(1, 1000, "cuda")
    pinv = h.invert_perm(p)
    assert torch.equal(p[pinv.long()], torch.arange(1000, dtype=torch.int32, device="cuda"))
    idx = torch.tensor([5, -1, 999, 1000, 0], dtype=torch.int32, device="cuda")
    g = h.gather_index(p, idx)
    pc = p.cpu().numpy()
    assert g.cpu().tolist() == [pc[5], -1, pc[999], -1, pc[0]]
    x = idx.clone()
    h.gather_index(p, x, out=x)     # in place
    assert x.cpu().tolist() == g.cpu().tolist()
    A = synth.rmat(10, 8, 2, "inc-bn", symmetric=False, device="cuda")
    for gr, gc in [(8, 8), (1, 1), (3, 5), (64, 64)]:
        got = h.block_nnz(A, gr, gc).cpu().numpy()
        assert np.array_equal(got, _block_counts(A, gr, gc)), (gr, gc)
    # more grid rows than matrix rows (empty grid rows), and a matrix of
    # several entry chunks per wavefront with empty rows
    from tests._gpu import mixed_csr
    for Am, gr, gc in [(mixed_csr(3, 5, 40, [0, 7, 40]), 8, 3),
                       (mixed_csr(4, 3000, 500, [0, 0, 1, 90, 300], torch.int64), 7, 9)]:
        got = h.block_nnz(Am, gr, gc).cpu().numpy()
        assert np.array_equal(got, _block_counts(Am, gr, gc)), (gr, gc)
    with pytest.raises(hp.HPError):
        h.block_nnz(A, 65, 64)


@pytest.mark.parametrize("sym", [True, False])
def test_modes_small(env, sym):
    hp, inc = env
    _say(f"incremental: R-MAT scale 10, 9 blocks, symmetric {sym}")
    h = hp.handle(0)
    w = synth.workload_incremental(seed=3, scale=10, device="cuda")
    A = w["A"]
    perms = [(p, None if sym else synth.randperm(synth.stream_key(7, "q", k), A.ncols, "cuda"))
             for k, p in enumerate(w["P"])]
    sp = inc.split(h, A, w["I"], w["J"])
    assert sp.large.nnz + sum(b.nnz for b in sp.B) == A.nnz
    fused = inc.run(h, sp, "fused", perms)
    sep = inc.run(h, sp, "separate", perms)
    assert_same(np_csr(fused.C), np_csr(sep.C), "fused vs separate")
    assert fused.nnz == sep.nnz and fused.imbalance == sep.imbalance
    assert fused.nnz[-1] == A.nnz
    q = fused.q_total
    assert_same(np_csr(fused.C), oracle.permute(A, fused.p_total, q), "final vs oracle permutation of A")
    plain = inc.run(h, sp, "assign", perms)
    assert_same(np_csr(plain.C), np_csr(A), "assign only restores A")
    once = inc.run(h, sp, "perm-once", perms)
    p0, q0 = perms[0]
    assert_same(np_csr(once.C), oracle.permute(A, p0, q0), "one permutation then assignments")
    # the metric: direct count of the final matrix
    cnt = _block_counts(fused.C, 8, 8)
    assert abs(fused.imbalance[-1] - cnt.max() / cnt.mean()) < 1e-9


@pytest.mark.timeout(900)
def test_full_size(env):
    """R-MAT scale 22 as in the incremental workload: the blocks split off
    equal the oracle's extractions, and after the nine fused steps the
    matrix equals the oracle's permutation of A by the step permutations
    composed on the host, bit for bit over the whole output."""
    import os
    hp, inc = env
    nt = max(1, min(16, os.cpu_count() or 1))
    _say("incremental: R-MAT scale 22, fused steps, whole output vs oracle")
    h = hp.handle(0)
    w = synth.workload_incremental(scale=22, device="cuda")
    A = w["A"]
    sp = inc.split(h, A, w["I"], w["J"])
    Ah = (A.nrows, A.ncols, A.rowptr.cpu().numpy().astype(np.int64), A.col.cpu().numpy(), A.val.cpu().numpy())
    for k, (Ik, Jk) in enumerate(zip(w["I"], w["J"])):
        assert_same(np_csr(sp.B[k]), oracle.spref_map(Ah, Ik, Jk, threads=nt), f"block {k}")
    assert sp.large.nnz + sum(b.nnz for b in sp.B) == A.nnz
    r = inc.run(h, sp, "fused", [(p, None) for p in w["P"]])
    # row i after step k is row p_1[p_2[...p_k[i]]] of A: compose on the host
    total = np.arange(A.nrows, dtype=np.int64)
    for p in w["P"]:
        total = total[p.cpu().numpy().astype(np.int64)]
    exp = oracle.permute_map(Ah, total, None, threads=nt)
    assert_same(np_csr(r.C), exp, "final matrix vs oracle permutation of A")
    assert np.array_equal(r.p_total.cpu().numpy(), total)
    assert r.imbalance[-1] < 1.5 < r.imbalance[0]


def test_helper_errors(env):
    hp, _ = env
    h = hp.handle(0)
    p = synth.randperm(5, 100, "cuda")
    with pytest.raises(hp.HPError) as ex:   # out overlapping the map
        h.gather_index(p, p[:10].clone(), out=p[50:60])
    assert ex.value.name == "HP_ERR_ALIAS"
    with pytest.raises(hp.HPError) as ex:
        h.invert_perm(p, out=p)
    assert ex.value.name == "HP_ERR_ALIAS"
