"""GPU parity for spref (C = A(I, J)): bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, mixed_csr, np_csr, rows_of, sample_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.int32), device="cuda")


def test_er_small_sorted_unique(hp):
    w = synth.workload_er_small(device="cuda")
    A, I = w["A"], w["I"]
    C = hp.spref(A, I, I)
    assert_same(np_csr(C), oracle.spref(A, I, I), "A(I, I)")


@pytest.mark.parametrize("scale", [12, 15])
def test_rmat_unsorted_repeated(hp, scale):
    w = synth.workload_rmat_extract(scale=scale, device="cuda")
    A, I, J = w["A"], w["I"], w["J"]
    C = hp.spref(A, I, J)
    assert_same(np_csr(C), oracle.spref(A, I, J), f"rmat scale {scale}")
    C2 = hp.spref(A, I, J)
    assert_same(np_csr(C2), np_csr(C), "repeat run identical")


LENGTHS = [0, 1, 2, 3, 7, 16, 17, 64, 65, 900, 1024, 1025, 3000, 4097, 9000]


@pytest.mark.parametrize("ptr", [torch.int32, torch.int64])
@pytest.mark.parametrize("vdt", [torch.float32, torch.float64])
def test_big_rows_and_duplicates(hp, ptr, vdt):
    m, n = 400, 10000
    A = mixed_csr(21, m, n, LENGTHS, ptr, vdt)
    rng = np.random.default_rng(5)
    I = _t(rng.integers(0, m, 600))                      # rows replicated
    J = _t(np.concatenate([rng.permutation(n), rng.integers(0, n, 2500)])[rng.permutation(n + 2500)])
    C = hp.spref(A, I, J)
    assert_same(np_csr(C), oracle.spref(A, I, J), f"big rows {ptr} {vdt}")


def test_monotone_with_big_rows(hp):
    m, n = 300, 12000
    A = mixed_csr(22, m, n, LENGTHS)
    rng = np.random.default_rng(6)
    I = _t(np.sort(rng.choice(m, 200, replace=False)))
    J = _t(np.sort(rng.choice(n, 9000, replace=False)))
    C = hp.spref(A, I, J)
    assert_same(np_csr(C), oracle.spref(A, I, J), "monotone J")


def test_heavy_column_repeats(hp):
    m, n = 200, 3000
    A = mixed_csr(23, m, n, [5, 50, 500])
    rng = np.random.default_rng(7)
    J = _t(np.concatenate([np.full(700, 11), np.full(300, 1500), rng.integers(0, n, 400)]))
    I = _t(rng.integers(0, m, 150))
    C = hp.spref(A, I, J)
    assert_same(np_csr(C), oracle.spref(A, I, J), "heavy repeats")


def test_empty_sets(hp):
    A = mixed_csr(24, 50, 60, [0, 3, 8])
    I = _t(np.arange(10))
    e = _t(np.zeros(0))
    C = hp.spref(A, I, e)
    assert C.nnz == 0 and C.rowptr.cpu().tolist() == [0] * 11
    C = hp.spref(A, e, I)
    assert C.nnz == 0 and C.rowptr.cpu().tolist() == [0]
    allrows = _t(np.arange(50))
    assert_same(np_csr(hp.spref(A, allrows, _t(np.arange(60)))), np_csr(A), "identity extraction")


@pytest.mark.parametrize("ptr", [torch.int32, torch.int64])
def test_fewer_entries_than_rows(hp, ptr):
    """A matrix with fewer stored entries than rows: the selected rows that
    have entries are listed first and only they are walked (short and big
    rows, repeated and unordered I and J, sorted and unsorted output); the
    same selection on a denser matrix walks every row."""
    lengths = [0] * 500 + [1, 5, 40, 300, 2]
    A = mixed_csr(27, 40000, 3000, lengths, ptr, torch.float64)
    assert A.nnz < A.nrows
    I = synth.subset(28, A.nrows, 30000, repeat_frac=0.05, device="cuda")
    J = synth.subset(29, A.ncols, 2000, repeat_frac=0.05, device="cuda")
    assert_same(np_csr(hp.spref(A, I, J)), oracle.spref(A, I, J), "unsorted I, J")
    Is, Js = torch.sort(I).values, torch.sort(torch.unique(J)).values
    assert_same(np_csr(hp.spref(A, Is, Js)), oracle.spref(A, Is, Js), "sorted I, unique sorted J")
    D = mixed_csr(30, 4000, 3000, [0, 1, 5, 40, 300, 2], ptr, torch.float64)
    assert D.nnz >= D.nrows
    I2 = synth.subset(31, D.nrows, 3000, repeat_frac=0.05, device="cuda")
    assert_same(np_csr(hp.spref(D, I2, J)), oracle.spref(D, I2, J), "denser matrix")


def test_errors_and_overflow(hp):
    A = mixed_csr(25, 20, 30, [4])
    with pytest.raises(hp.HPError) as e:
        hp.spref(A, _t([0, 20]), _t([1, 2]))
    assert e.value.name == "HP_ERR_INDEX_RANGE"
    with pytest.raises(hp.HPError) as e:
        hp.spref(A, _t([0, 1]), _t([-1]))
    assert e.value.name == "HP_ERR_INDEX_RANGE"
    # one dense row selected 45000 times: 2.25e9 outputs cannot use an int32 rowptr
    n = 50000
    dense = synth.CSR(1, n, torch.tensor([0, n], dtype=torch.int32, device="cuda"),
                      torch.arange(n, dtype=torch.int32, device="cuda"),
                      torch.ones(n, dtype=torch.float32, device="cuda"))
    with pytest.raises(hp.HPError) as e:
        hp.spref(dense, torch.zeros(45000, dtype=torch.int32, device="cuda"),
                 torch.arange(n, dtype=torch.int32, device="cuda"))
    assert e.value.name == "HP_ERR_OVERFLOW"


def test_rmat_full_size_sampled(hp):
    """R-MAT scale 22, ef 16, symmetrised; I, J 25% unsorted with 1% repeats."""
    w = synth.workload_rmat_extract(device="cuda")
    A, I, J = w["A"], w["I"], w["J"]
    C = hp.spref(A, I, J)
    torch.cuda.synchronize()
    rows = sample_rows(13, I.numel(), 40)
    assert_same(rows_of(C, rows), oracle.spref(A, I, J, rows=rows), "sampled rows")
    # closed-form nnz: sum over selected rows of the multiplicity of each column in J
    mult = torch.bincount(J.long(), minlength=A.ncols)
    rp = A.rowptr.long()
    lens = rp[I.long() + 1] - rp[I.long()]
    starts = torch.repeat_interleave(rp[I.long()], lens)
    offs = torch.arange(int(lens.sum()), device="cuda") - torch.repeat_interleave(
        torch.cumsum(lens, 0) - lens, lens)
    expect = int(mult[A.col[(starts + offs)].long()].sum())
    assert C.nnz == expect
    # every row strictly increasing
    cr = C.rowptr.long()
    same_row = torch.ones(C.nnz, dtype=torch.bool, device="cuda")
    same_row[cr[:-1][cr[:-1] < C.nnz]] = False
    assert bool(torch.all((C.col[1:] > C.col[:-1]) | ~same_row[1:]))
    C2 = hp.spref(A, I, J)
    assert torch.equal(C2.col, C.col) and torch.equal(C2.val.view(torch.int32), C.val.view(torch.int32))


@pytest.mark.parametrize("ptr", [torch.int32, torch.int64])
def test_long_rows_over_2pow20_columns(hp, ptr):
    """Output rows above 2048 entries with more than 2^20 output columns:
    long rows are split by key range before ranking (3 buckets here)."""
    n = 3_000_000
    A = mixed_csr(77, 40, n, [0, 7, 300, 3000, 12000, 30000], ptr, torch.float32)
    I = synth.subset(78, A.nrows, 50, repeat_frac=0.3, device="cuda")
    J = synth.subset(79, n, 2_500_000, repeat_frac=0.01, device="cuda")
    C = hp.spref(A, I, J)
    torch.cuda.synchronize()
    rows = sample_rows(80, I.numel(), 6)
    assert_same(rows_of(C, rows), oracle.spref(A, I, J, rows=rows), "sampled rows")
    cr = C.rowptr.long()
    same_row = torch.ones(C.nnz, dtype=torch.bool, device="cuda")
    same_row[cr[:-1][cr[:-1] < C.nnz]] = False
    assert bool(torch.all((C.col[1:] > C.col[:-1]) | ~same_row[1:]))


def test_big_row_selected_many_times(hp):
    """A long row selected hundreds of times: more long-row chunks than the
    count pass can record masks for, so the gather looks entries up itself."""
    A = mixed_csr(61, 300, 20000, [0, 2, 9, 6000], torch.int32, torch.float32)
    rp = A.rowptr.cpu().numpy()
    hub = int(np.argmax(np.diff(rp)))
    I = torch.tensor([hub] * 250 + list(range(0, 300, 7)), dtype=torch.int32, device="cuda")
    I = I[torch.randperm(I.numel(), generator=torch.Generator().manual_seed(3)).to("cuda")]
    J = synth.subset(62, A.ncols, 9000, repeat_frac=0.05, device="cuda")
    C = hp.spref(A, I, J)
    torch.cuda.synchronize()
    rows = sample_rows(63, I.numel(), 12)
    assert_same(rows_of(C, rows), oracle.spref(A, I, J, rows=rows), "sampled rows")
