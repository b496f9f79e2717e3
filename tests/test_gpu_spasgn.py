"""GPU parity for spasgn (A(I, J) = B): bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import assert_same, mixed_csr, np_csr, rows_of, sample_rows

pytestmark = pytest.mark.gpu
OPS = ["second", "plus", "replace"]


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_20776_amd import hipperm
    return hipperm


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.int32), device="cuda")


def _block(seed, nI, nJ, density, ptr, vdt):
    return synth.bernoulli_block(nI, nJ, density, seed, "tblk", ptr, vdt, "cuda")


@pytest.mark.parametrize("op", OPS)
def test_grid_contiguous_block(hp, op):
    w = synth.workload_grid(side=128, frac=0.10, density=0.02, device="cuda")
    A, B, I, J = w["A"], w["B"], w["I"], w["J"]
    C = hp.spasgn(A, B, I, J, op)
    assert_same(np_csr(C), oracle.spasgn(A, B, I, J, op), f"grid {op}")


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_rmat_random_index_sets(hp, op, ptr, vdt):
    A = synth.rmat(12, 8, 3, "asg", symmetric=False, ptr_dtype=ptr, val_dtype=vdt, device="cuda")
    rng = np.random.default_rng(4)
    I = _t(rng.choice(A.nrows, 700, replace=False))
    J = _t(rng.choice(A.ncols, 900, replace=False))
    B = _block(5, 700, 900, 0.03, ptr, vdt)
    C = hp.spasgn(A, B, I, J, op)
    assert_same(np_csr(C), oracle.spasgn(A, B, I, J, op), f"rmat {op}")
    # sorted index sets take the merge path
    Is, Js = torch.sort(I).values, torch.sort(J).values
    C2 = hp.spasgn(A, B, Is, Js, op)
    assert_same(np_csr(C2), oracle.spasgn(A, B, Is, Js, op), f"rmat sorted {op}")


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_rows_of_I_out_of_J_order(hp, op, ptr, vdt):
    """J unsorted, so the mapped B columns of a row of I do not increase:
    rows of up to 64 A + B entries are placed by counting, longer ones up to
    256 are written unsorted and ordered by the class sorts, longer still go
    the long-row way; also through the fused form."""
    m, n = 900, 2000
    A = mixed_csr(81, m, n, [0, 3, 12, 16, 40, 90, 150, 230, 400], ptr, vdt)
    rng = np.random.default_rng(82)
    nI, nJ = 300, 1200
    I = _t(rng.choice(m, nI, replace=False))
    J = _t(rng.choice(n, nJ, replace=False))                         # unsorted
    B = mixed_csr(83, nI, nJ, [0, 2, 10, 30, 60, 120, 200, 250], ptr, vdt)
    ref = oracle.spasgn(A, B, I, J, op)
    assert_same(np_csr(hp.spasgn(A, B, I, J, op)), ref, f"J out of order, {op}")
    p = synth.randperm(84, m, "cuda")
    q = synth.randperm(85, n, "cuda")
    Cf = np_csr(hp.spasgn_permute(A, B, I, J, p, q, op))
    assert_same(Cf, oracle.permute((m, n) + tuple(ref), p, q), f"fused, J out of order, {op}")


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("ptr,vdt", [(torch.int32, torch.float32), (torch.int64, torch.float64)])
def test_long_B_rows_one_wavefront_a_row(hp, op, ptr, vdt):
    """B rows averaging over 64 entries take the one-wavefront-a-row merge:
    A rows of up to 64 entries and B rows of up to 256 merged in registers,
    longer ones through the one-wavefront merge in LDS; J sorted (merged in
    place), a contiguous range (no lookup of J), and unsorted; also fused."""
    m, n = 1000, 3000
    A = mixed_csr(91, m, n, [0, 1, 5, 40, 63, 64, 65, 120], ptr, vdt)
    rng = np.random.default_rng(92)
    nI, nJ = 400, 1500
    I = _t(rng.choice(m, nI, replace=False))
    Js = _t(np.sort(rng.choice(n, nJ, replace=False)))
    Jr = _t(np.arange(700, 700 + nJ))
    Ju = _t(rng.choice(n, nJ, replace=False))
    B = mixed_csr(93, nI, nJ, [0, 1, 63, 64, 65, 128, 200, 255, 256, 257], ptr, vdt)
    assert B.nnz > 64 * nI
    p = synth.randperm(94, m, "cuda")
    q = synth.randperm(95, n, "cuda")
    for J, name in ((Js, "sorted J"), (Jr, "J a range"), (Ju, "unsorted J")):
        ref = oracle.spasgn(A, B, I, J, op)
        assert_same(np_csr(hp.spasgn(A, B, I, J, op)), ref, f"{name}, {op}")
        Cf = np_csr(hp.spasgn_permute(A, B, I, J, p, q, op))
        assert_same(Cf, oracle.permute((m, n) + tuple(ref), p, q), f"fused, {name}, {op}")


def test_fused_row_sort_wide_columns(hp):
    """The fused merge's own row sort with mapped columns at or above 2^24
    (the wavefront sort ranks by counting instead of packing key and
    position): more than 2^24 columns, long B rows, whole output against
    the oracle."""
    m, n = 300, (1 << 24) + 5000
    A = mixed_csr(97, m, n, [0, 2, 9, 40], torch.int64, torch.float64)
    rng = np.random.default_rng(98)
    nI, nJ = 120, 30000
    I = _t(rng.choice(m, nI, replace=False))
    J = _t(rng.choice(n, nJ, replace=False))
    B = mixed_csr(99, nI, nJ, [0, 70, 130, 200, 256], torch.int64, torch.float64)
    assert B.nnz > 64 * nI
    p = synth.randperm(100, m, "cuda")
    q = synth.randperm(101, n, "cuda")
    ref = oracle.spasgn(A, B, I, J, "second")
    Cf = np_csr(hp.spasgn_permute(A, B, I, J, p, q, "second"))
    # the O(entries) oracle routine (pinned to the literal one on CPU): the
    # literal one is O(rows x columns), minutes at 2^24 columns
    assert_same(Cf, oracle.permute_map((m, n) + tuple(ref), p, q), "fused, wide columns")


@pytest.mark.parametrize("op", OPS)
def test_huge_rows_whole_grid(hp, op):
    """Rows of I with more than 4096 A + B entries are counted and merged by
    every workgroup together: huge A rows against short B rows and the
    reverse, several huge rows in one call, sorted and unsorted J, plain and
    fused, whole output against the oracle."""
    m, n = 60, 20000
    A = mixed_csr(111, m, n, [0, 5, 6000, 9000, 40], torch.int64, torch.float64)
    rng = np.random.default_rng(112)
    nI, nJ = 30, 15000
    I = _t(rng.choice(m, nI, replace=False))
    p = synth.randperm(113, m, "cuda")
    q = synth.randperm(114, n, "cuda")
    for J, name in ((_t(rng.choice(n, nJ, replace=False)), "unsorted J"),
                    (_t(np.sort(rng.choice(n, nJ, replace=False))), "sorted J")):
        B = mixed_csr(115, nI, nJ, [0, 3, 5000, 8000, 100], torch.int64, torch.float64)
        ref = oracle.spasgn(A, B, I, J, op)
        assert_same(np_csr(hp.spasgn(A, B, I, J, op)), ref, f"{name}, {op}")
        Cf = np_csr(hp.spasgn_permute(A, B, I, J, p, q, op))
        assert_same(Cf, oracle.permute((m, n) + tuple(ref), p, q), f"fused, {name}, {op}")


@pytest.mark.parametrize("op", OPS)
def test_long_rows_fallback(hp, op):
    m, n = 300, 6000
    A = mixed_csr(31, m, n, [0, 3, 100, 250, 700, 5000])
    rng = np.random.default_rng(8)
    I = _t(rng.choice(m, 120, replace=False))
    J = _t(rng.choice(n, 5000, replace=False))
    B = mixed_csr(32, 120, 5000, [0, 10, 200, 300, 4500])
    C = hp.spasgn(A, B, I, J, op)
    assert_same(np_csr(C), oracle.spasgn(A, B, I, J, op), f"long rows {op}")


def test_empty_and_errors(hp):
    A = mixed_csr(33, 40, 50, [0, 2, 6])
    I = _t([3, 7, 9])
    J = _t([1, 4])
    B0 = mixed_csr(34, 3, 2, [0])
    assert_same(np_csr(hp.spasgn(A, B0, I, J)), np_csr(A), "empty B")
    e = _t(np.zeros(0))
    Be = mixed_csr(35, 0, 0, [0])
    assert_same(np_csr(hp.spasgn(A, Be, e, e)), np_csr(A), "empty I, J")
    B = mixed_csr(36, 3, 2, [1, 2])
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn(A, B, _t([3, 3, 9]), J)
    assert ex.value.name == "HP_ERR_DUPLICATE_INDEX"
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn(A, B, I, _t([1, 50]))
    assert ex.value.name == "HP_ERR_INDEX_RANGE"
    with pytest.raises(hp.HPError) as ex:
        hp.spasgn(A, B, _t([3, 7]), J)
    assert ex.value.name == "HP_ERR_SHAPE"


def test_workspace_depends_on_B(hp):
    """The assignment workspaces grow with nnz(B) (the list of rows of I with
    more than 4096 A + B entries) and refuse a NULL B."""
    import ctypes
    from paper_2509_20776_amd import hipperm as H
    h = H.handle(0)
    A = mixed_csr(121, 5000, 60, [0, 3, 9])
    Ac = H.to_csr_t(A)
    sizes = []
    for nnzb in (0, 1 << 24):
        Bc = H.to_csr_t(mixed_csr(122, 5, 6, [0, 1]))
        Bc.nnz = nnzb   # only the count is read
        for fn in (H.hp_spasgn_workspace, H.hp_spasgn_permute_workspace):
            need = ctypes.c_size_t(0)
            assert fn(h.h, ctypes.byref(Ac), ctypes.byref(Bc), ctypes.byref(need)) == 0
            sizes.append(need.value)
    assert sizes[2] > sizes[0] and sizes[3] > sizes[1]
    for fn in (H.hp_spasgn_workspace, H.hp_spasgn_permute_workspace):
        need = ctypes.c_size_t(0)
        assert fn(h.h, ctypes.byref(Ac), None, ctypes.byref(need)) != 0


def test_streaming_round_trip(hp):
    """80% of the edges plus four 5% parts assigned back gives A again."""
    A = synth.rmat(11, 8, 9, "rt", symmetric=False, device="cuda")
    rp, col, val = np_csr(A)
    rows = np.repeat(np.arange(A.nrows), np.diff(rp))
    lab = np.random.default_rng(10).choice(5, size=len(col), p=[0.8, 0.05, 0.05, 0.05, 0.05])

    def sub(mask):
        r, c, v = rows[mask], col[mask], val[mask]
        return r, c, v

    r0, c0, v0 = sub(lab == 0)
    cnt = np.bincount(r0, minlength=A.nrows)
    cur = synth.CSR(A.nrows, A.ncols, torch.from_numpy(np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)).cuda(),
                    torch.from_numpy(c0).cuda(), torch.from_numpy(v0).cuda())
    for part in range(1, 5):
        r, c, v = sub(lab == part)
        I = np.unique(r)
        J = np.unique(c)
        ri = np.searchsorted(I, r)
        cj = np.searchsorted(J, c).astype(np.int32)
        order = np.lexsort((cj, ri))
        bc = np.bincount(ri, minlength=len(I))
        B = synth.CSR(len(I), len(J), torch.from_numpy(np.concatenate([[0], np.cumsum(bc)]).astype(np.int32)).cuda(),
                      torch.from_numpy(cj[order]).cuda(), torch.from_numpy(v[order]).cuda())
        cur = hp.spasgn(cur, B, _t(I), _t(J), "second")
    assert_same(np_csr(cur), np_csr(A), "round trip")


def test_grid_full_size_sampled(hp):
    """4096^2 grid, int64 rowptr, fp64; I = J a contiguous 10% range; B at density 1e-4."""
    w = synth.workload_grid(side=4096, device="cuda")
    A, B, I, J = w["A"], w["B"], w["I"], w["J"]
    C = hp.spasgn(A, B, I, J, "second")
    torch.cuda.synchronize()
    r0, r1 = int(I[0]), int(I[-1]) + 1
    rows = np.unique(np.concatenate([sample_rows(17, A.nrows, 16), np.arange(r0, r0 + 8),
                                     np.arange(r1 - 8, r1 + 8)]))
    assert_same(rows_of(C, rows), oracle.spasgn(A, B, I, J, "second", rows=rows), "sampled rows")
    # rows outside I are A's rows, shifted
    arp, crp = A.rowptr, C.rowptr
    assert torch.equal(C.col[:int(crp[r0])], A.col[:int(arp[r0])])
    assert torch.equal(C.col[int(crp[r1]):], A.col[int(arp[r1]):])
    assert torch.equal(C.val[int(crp[r1]):].view(torch.int64), A.val[int(arp[r1]):].view(torch.int64))
    # block replace then extraction returns B exactly
    R = hp.spasgn(A, B, I, J, "replace")
    X = hp.spref(R, I, J)
    assert torch.equal(X.rowptr, B.rowptr) and torch.equal(X.col, B.col)
    assert torch.equal(X.val.view(torch.int64), B.val.view(torch.int64))


@pytest.mark.parametrize("op", OPS)
def test_rows_outside_I_of_every_copy_path(hp, op):
    """Rows outside I of every length class of the copy: the 64-row wavefront
    copy, a workgroup per row (over 512 entries) and the whole grid per row
    (over 65536 entries), with long rows at neighbouring ids."""
    m, n = 48, 100_000
    A = mixed_csr(71, m, n, [0, 3, 600, 70_000, 2_000, 1, 66_000, 513])
    rng = np.random.default_rng(72)
    I = _t(rng.choice(m, 6, replace=False))
    J = _t(rng.choice(n, 3000, replace=False))
    B = mixed_csr(73, 6, 3000, [0, 40, 700])
    assert_same(np_csr(hp.spasgn(A, B, I, J, op)), oracle.spasgn(A, B, I, J, op), f"copy paths {op}")
