"""GPU parity for the fused assign-and-permute C = P (A (+) B') Q^T: bit-equal
to the two separate calls (spasgn, then permute) on the GPU, and to the
oracle's composition of the same two operations."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, mixed_csr, np_csr, rows_of, sample_rows

pytestmark = pytest.mark.gpu
OPS = ["second", "plus", "replace"]


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.int32), device="cuda")


def _oracle(A, B, I, J, p, q, op):
    X = oracle.spasgn(A, B, I, J, op)
    return oracle.permute((A.nrows, A.ncols) + tuple(X), p, q)


def _check(hp, A, B, I, J, p, q, op, what, with_oracle=True):
    C = hp.spasgn_permute(A, B, I, J, p, q, op)
    sep = hp.permute(hp.spasgn(A, B, I, J, op), p, q)
    got = np_csr(C)
    assert_same(got, np_csr(sep), f"{what}: fused vs separate")
    if with_oracle:
        assert_same(got, _oracle(A, B, I, J, p, q, op), f"{what}: vs oracle")
    return C


SHORT = [0, 1, 2, 3, 4, 1, 2, 3, 4, 4, 4, 0, 7, 20]   # rows of <= 4 entries hold most entries


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_short_rows_slots_and_pull_agree(hp, op, ptr, vdt):
    """Rows outside I of at most 4 entries holding most entries: the plan
    asks for row slots (exec_ws_bytes above aux[3]); exec with them, with
    them at an address off the 256-byte grid, and with only aux[3] bytes
    (rows pulled straight from A) all equal the separate calls and the
    oracle; below aux[3] is refused."""
    _say(f"fused: short rows, op {op}, ptr {ptr}, val {vdt}")
    h = hp.Handle(0)
    m, n = 4000, 3000
    A = mixed_csr(31, m, n, SHORT, ptr, vdt)
    rng = np.random.default_rng(32)
    I = _t(rng.choice(m, 400, replace=False))
    J = _t(rng.choice(n, 300, replace=False))
    B = synth.bernoulli_block(400, 300, 0.02, 33, "fsb", ptr, vdt, "cuda")
    p = synth.randperm(34, m, "cuda")
    q = synth.randperm(35, n, "cuda")
    ref = np_csr(h.permute(h.spasgn(A, B, I, J, op), p, q))
    assert_same(ref, _oracle(A, B, I, J, p, q, op), "separate vs oracle")
    C, ws, info = h.spasgn_permute_plan(A, B, I, J, p, q, op)
    assert info.exec_ws_bytes > info.aux[3] >= 0
    assert_same(np_csr(h.spasgn_permute_exec(A, B, I, J, p, q, C, ws, info, op)), ref, "row slots")
    C, ws, info = h.spasgn_permute_plan(A, B, I, J, p, q, op)
    big = torch.empty(info.exec_ws_bytes + 4, dtype=torch.uint8, device="cuda")
    assert_same(np_csr(h.spasgn_permute_exec(A, B, I, J, p, q, C, ws, info, op, xws=big[4:])), ref,
                "row slots, offset workspace")
    C, ws, info = h.spasgn_permute_plan(A, B, I, J, p, q, op)
    small = torch.empty(max(info.aux[3], 1), dtype=torch.uint8, device="cuda")[: info.aux[3]]
    assert_same(np_csr(h.spasgn_permute_exec(A, B, I, J, p, q, C, ws, info, op,
                                             xws=small if info.aux[3] else None)), ref, "pulled from A")
    if info.aux[3] > 0:
        with pytest.raises(hp.HPError) as e:
            h.spasgn_permute_exec(A, B, I, J, p, q, C, ws, info, op, xws=small[:-1])
        assert e.value.name == "HP_ERR_WORKSPACE"
    # symmetric form through the slots
    As = mixed_csr(36, m, m, SHORT, ptr, vdt)
    Js = _t(rng.choice(m, 300, replace=False))
    refs = np_csr(h.permute(h.spasgn(As, B, I, Js, op), p))
    orefs = _oracle(As, B, I, Js, p, None, op)
    assert_same(refs, orefs, "symmetric, separate vs oracle")
    assert_same(np_csr(h.spasgn_permute(As, B, I, Js, p, None, op)), orefs, "symmetric, row slots")
    h.close()


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_rmat_random(hp, op, ptr, vdt):
    _say(f"fused: R-MAT scale 11, op {op}, ptr {ptr}, val {vdt}")
    A = synth.rmat(11, 8, 3, "fz", symmetric=False, ptr_dtype=ptr, val_dtype=vdt, device="cuda")
    rng = np.random.default_rng(4)
    I = _t(rng.choice(A.nrows, 300, replace=False))
    J = _t(rng.choice(A.ncols, 500, replace=False))
    B = synth.bernoulli_block(300, 500, 0.03, 5, "fzb", ptr, vdt, "cuda")
    p = synth.randperm(6, A.nrows, "cuda")
    q = synth.randperm(7, A.ncols, "cuda")
    _check(hp, A, B, I, J, p, q, op, "random I, J")
    _check(hp, A, B, torch.sort(I).values, torch.sort(J).values, p, q, op, "sorted I, J")
    _check(hp, A, B, I, J, p, None, op, "symmetric P A P^T")


@pytest.mark.parametrize("op", OPS)
def test_grid_contiguous_block(hp, op):
    _say(f"fused: 128x128 grid, contiguous I = J, op {op}")
    w = synth.workload_grid(side=128, frac=0.10, density=0.02, device="cuda")
    _check(hp, w["A"], w["B"], w["I"], w["J"], w["p"], w["q"], op, "grid")


@pytest.mark.parametrize("op", OPS)
def test_long_rows(hp, op):
    """Output rows in every sort class, including rows above the block-sort limit."""
    _say(f"fused: long rows, op {op}")
    m, n = 300, 6000
    A = mixed_csr(41, m, n, [0, 1, 3, 17, 100, 250, 700, 5000])
    rng = np.random.default_rng(9)
    I = _t(rng.choice(m, 120, replace=False))
    J = _t(rng.choice(n, 5000, replace=False))
    B = mixed_csr(42, 120, 5000, [0, 10, 200, 300, 4500])
    _check(hp, A, B, I, J, synth.randperm(43, m, "cuda"), synth.randperm(44, n, "cuda"), op, "long rows")


def test_edges_and_errors(hp):
    _say("fused: empty B, empty I and J, identity permutations, error paths")
    A = mixed_csr(51, 40, 40, [0, 2, 6, 30])
    I = _t([3, 7, 9])
    J = _t([1, 4])
    p = synth.randperm(52, 40, "cuda")
    q = synth.randperm(53, 40, "cuda")
    B0 = mixed_csr(54, 3, 2, [0])
    _check(hp, A, B0, I, J, p, q, "second", "empty B")
    e = _t(np.zeros(0))
    _check(hp, A, mixed_csr(55, 0, 0, [0]), e, e, p, q, "plus", "empty I, J")
    ident = _t(np.arange(40))
    B = mixed_csr(56, 3, 2, [1, 2])
    C = hp.spasgn_permute(A, B, I, J, ident, ident, "plus")
    assert_same(np_csr(C), np_csr(hp.spasgn(A, B, I, J, "plus")), "identity permutations")
    bad = p.clone()
    bad[0] = bad[1]
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn_permute(A, B, I, J, bad, q)
    assert ex.value.name == "HP_ERR_NOT_PERMUTATION"
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn_permute(A, B, I, J, p, _t(np.arange(1, 41)))
    assert ex.value.name == "HP_ERR_INDEX_RANGE"
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn_permute(A, B, _t([3, 3, 9]), J, p, q)
    assert ex.value.name == "HP_ERR_DUPLICATE_INDEX"
    R = mixed_csr(57, 30, 40, [2])
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn_permute(R, B, I, J, synth.randperm(58, 30, "cuda"), None)
    assert ex.value.name == "HP_ERR_SHAPE"
    h = hp.handle(0)
    C, ws, info = h.spasgn_permute_plan(A, B, I, J, p, q, "second")
    with pytest.raises(hp.HPError) as ex:     # exec must see q null exactly when plan did
        h.spasgn_permute_exec(A, B, I, J, p, None, C, ws, info, "second")
    assert ex.value.name == "HP_ERR_INVALID_ARG"
    with pytest.raises(hp.HPError) as ex:     # a plain assignment plan is not a fused one
        C2, ws2, info2 = h.spasgn_plan(A, B, I, J, "second")
        h.spasgn_permute_exec(A, B, I, J, p, q, C2, ws, info2, "second")
    assert ex.value.name == "HP_ERR_INVALID_ARG"


def test_grid_full_size(hp):
    """4096^2 grid, int64 rowptr, fp64, contiguous 10% I = J, B density 1e-4,
    random P and Q: bit-equal to the separate calls over the whole output,
    and to the oracle on sampled rows."""
    _say("fused: 4096^2 grid, full size")
    w = synth.workload_grid(side=4096, device="cuda")
    A, B, I, J, p, q = w["A"], w["B"], w["I"], w["J"], w["p"], w["q"]
    C = hp.spasgn_permute(A, B, I, J, p, q, "second")
    sep = hp.permute(hp.spasgn(A, B, I, J, "second"), p, q)
    torch.cuda.synchronize()
    assert torch.equal(C.rowptr, sep.rowptr) and torch.equal(C.col, sep.col)
    assert torch.equal(C.val.view(torch.int64), sep.val.view(torch.int64))
    del sep
    # sampled output rows: X = oracle assignment at rows p[i], then the
    # oracle's column permutation of just those rows
    pc = p.cpu().numpy()
    r0 = int(I[0])
    inI = np.nonzero((pc >= r0) & (pc < r0 + I.numel()))[0][:24]
    rows = np.unique(np.concatenate([sample_rows(61, A.nrows, 24), inI]))
    X = oracle.spasgn(A, B, I, J, "second", rows=pc[rows])
    k = len(rows)
    exp = oracle.permute((k, A.ncols) + tuple(X), np.arange(k, dtype=np.int32), q)
    assert_same(rows_of(C, rows), exp, "sampled rows vs oracle")


def test_rows_outside_I_of_every_copy_path(hp):
    """Fused form over rows outside I of every copy class (see the plain test)."""
    _say("fused: rows of 3 to 70000 entries outside I")
    m, n = 48, 100_000
    A = mixed_csr(71, m, n, [0, 3, 600, 70_000, 2_000, 1, 66_000, 513])
    rng = np.random.default_rng(72)
    I = _t(rng.choice(m, 6, replace=False))
    J = _t(rng.choice(n, 3000, replace=False))
    B = mixed_csr(73, 6, 3000, [0, 40, 700])
    _check(hp, A, B, I, J, synth.randperm(74, m, "cuda"), synth.randperm(75, n, "cuda"), "plus", "copy paths")
