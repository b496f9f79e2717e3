"""Pins for the CPU oracle: it must agree with computations that do not share
its code -- dense brute force, SciPy fancy indexing, the selection-matrix
products of the paper's problem formulation (Sec. 2.1-2.3), hand-worked
examples, closed-form counts and invariants."""
import itertools

import numpy as np
import pytest

import oracle
from tests._util import (assert_csr_equal, csc_of, dense, floats, from_dense, from_scipy, ints,
                         rand_csr, read_golden, selection, to_dcsc, to_scipy)

SHAPES = [(1, 1), (2, 3), (5, 5), (7, 4), (9, 13), (16, 16), (33, 20)]

# Both routine families of each operation face every pin: the literal search
# over all (i, j) pairs and the routine through inverse index tables, the
# latter single-threaded and split over threads.
PERMUTES = {
    "literal": lambda A, p, q=None, rows=None: oracle.permute(A, p, q, rows=rows),
    "map": lambda A, p, q=None, rows=None: oracle.permute_map(A, p, q, rows=rows),
    "map-threads": lambda A, p, q=None, rows=None: oracle.permute_map(A, p, q, rows=rows, threads=3),
}
SPREFS = {
    "literal": lambda A, I, J, rows=None: oracle.spref(A, I, J, rows=rows),
    "map": lambda A, I, J, rows=None: oracle.spref_map(A, I, J, rows=rows),
    "map-threads": lambda A, I, J, rows=None: oracle.spref_map(A, I, J, rows=rows, threads=3),
}
SPASGNS = {
    "serial": lambda A, B, I, J, op="second", rows=None: oracle.spasgn(A, B, I, J, op, rows=rows),
    "threads": lambda A, B, I, J, op="second", rows=None: oracle.spasgn(A, B, I, J, op, rows=rows, threads=3),
}


def _rows_of(full, rows):
    """The listed rows (in list order, repeats kept) of a full result."""
    rp, c, v = full
    out_rp, cs, vs = [0], [], []
    for i in rows:
        a, b = rp[i], rp[i + 1]
        cs.append(c[a:b])
        vs.append(v[a:b])
        out_rp.append(out_rp[-1] + (b - a))
    return (np.array(out_rp, np.int64), np.concatenate(cs) if cs else c[:0], np.concatenate(vs) if vs else v[:0])


def _brute_permute(A, p, q):
    D, M = dense(A)
    return from_dense(D[np.ix_(p, q)], M[np.ix_(p, q)])


def _brute_spref(A, I, J):
    D, M = dense(A)
    return from_dense(D[np.ix_(I, J)], M[np.ix_(I, J)])


def _brute_spasgn(A, B, I, J, op):
    D, M = dense(A)
    m, n = D.shape
    bm, bn, brp, bc, bv = B
    if op == "replace":
        M[np.ix_(I, J)] = False
        D[np.ix_(I, J)] = 0
    for i in range(bm):
        for k in range(brp[i], brp[i + 1]):
            r, c = I[i], J[bc[k]]
            if op == "plus" and M[r, c]:
                D[r, c] = D[r, c] + bv[k]          # numpy: one add in the value dtype
            else:
                D[r, c] = bv[k]
            M[r, c] = True
    return from_dense(D, M)


# ---------------------------------------------------------------- golden ---

@pytest.mark.parametrize("how", sorted(PERMUTES))
def test_golden_permute(how):
    g = read_golden("permute_3x4.txt")
    m, n = ints(g["shape"])
    A = (int(m), int(n), ints(g["rowptr"]), ints(g["col"]).astype(np.int32), floats(g["val"]))
    got = PERMUTES[how](A, ints(g["p"]), ints(g["q"]))
    assert_csr_equal(got, (ints(g["expect_rowptr"]), ints(g["expect_col"]), floats(g["expect_val"])),
                     "golden permute")


@pytest.mark.parametrize("how", sorted(SPREFS))
def test_golden_spref(how):
    g = read_golden("spref_dup_3x4.txt")
    m, n = ints(g["shape"])
    A = (int(m), int(n), ints(g["rowptr"]), ints(g["col"]).astype(np.int32), floats(g["val"]))
    got = SPREFS[how](A, ints(g["I"]), ints(g["J"]))
    assert_csr_equal(got, (ints(g["expect_rowptr"]), ints(g["expect_col"]), floats(g["expect_val"])),
                     "golden spref")


@pytest.mark.parametrize("how", sorted(SPASGNS))
@pytest.mark.parametrize("op", ["second", "plus", "replace"])
def test_golden_spasgn(op, how):
    g = read_golden("spasgn_3x4.txt")
    m, n = ints(g["shape"])
    A = (int(m), int(n), ints(g["rowptr"]), ints(g["col"]).astype(np.int32), floats(g["val"]))
    bm, bn = ints(g["Bshape"])
    B = (int(bm), int(bn), ints(g["Browptr"]), ints(g["Bcol"]).astype(np.int32), floats(g["Bval"]))
    got = SPASGNS[how](A, B, ints(g["I"]), ints(g["J"]), op)
    exp = (ints(g[f"{op}_rowptr"]), ints(g[f"{op}_col"]), floats(g[f"{op}_val"]))
    assert_csr_equal(got, exp, f"golden spasgn {op}")


# --------------------------------------------------------------- permute ---

@pytest.mark.parametrize("how", sorted(PERMUTES))
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("vdtype", [np.float64, np.float32])
def test_permute_brute_scipy_selection(shape, vdtype, how):
    rng = np.random.default_rng(hash(shape) % 1000)
    m, n = shape
    A = rand_csr(rng, m, n, 0.3, vdtype)
    p = rng.permutation(m)
    q = rng.permutation(n)
    got = PERMUTES[how](A, p, q)
    assert_csr_equal(got, _brute_permute(A, p, q), "brute")
    S = to_scipy(A)
    assert_csr_equal(got, from_scipy(S[p][:, q]), "scipy fancy indexing")
    Pm = selection(p, m, vdtype)
    Qm = selection(q, n, vdtype)
    assert_csr_equal(got, from_scipy(Pm @ S @ Qm.T), "P A Q^T")


@pytest.mark.parametrize("how", sorted(PERMUTES))
def test_permute_symmetric_equals_general(how):
    rng = np.random.default_rng(1)
    A = rand_csr(rng, 12, 12, 0.25)
    p = rng.permutation(12)
    perm = PERMUTES[how]
    assert_csr_equal(perm(A, p), perm(A, p, p), "symmetric")
    assert_csr_equal(perm(A, p), _brute_permute(A, p, p), "symmetric brute")


@pytest.mark.parametrize("how", sorted(PERMUTES))
def test_permute_invariants(how):
    rng = np.random.default_rng(2)
    m, n = 40, 30
    A = rand_csr(rng, m, n, 0.2)
    p1, q1 = rng.permutation(m), rng.permutation(n)
    p2, q2 = rng.permutation(m), rng.permutation(n)
    perm = PERMUTES[how]
    A1 = perm(A, p1, q1)
    assert A1[0][-1] == A[2][-1]                       # nnz preserved
    lens = np.diff(A[2])
    assert sorted(np.diff(A1[0])) == sorted(lens)       # row-length multiset preserved
    # inverse permutations restore A byte for byte
    back = perm((m, n) + A1, np.argsort(p1), np.argsort(q1))
    assert_csr_equal(back, A[2:], "inverse")
    # identity
    assert_csr_equal(perm(A, np.arange(m), np.arange(n)), A[2:], "identity")
    # composition: A''[i,j] = A[p1[p2[i]], q1[q2[j]]]
    A2 = perm((m, n) + A1, p2, q2)
    assert_csr_equal(A2, perm(A, p1[p2], q1[q2]), "composition")


@pytest.mark.parametrize("how", sorted(PERMUTES))
def test_permute_sampled_rows_match_full(how):
    rng = np.random.default_rng(3)
    A = rand_csr(rng, 50, 60, 0.1)
    p, q = rng.permutation(50), rng.permutation(60)
    perm = PERMUTES[how]
    full = _brute_permute(A, p, q)
    for rows in (np.array([49, 0, 7, 7, 23]), np.arange(50)[::-1].copy(), np.zeros(0, np.int64)):
        assert_csr_equal(perm(A, p, q, rows=rows), _rows_of(full, rows), f"rows {rows[:5]}")
    with pytest.raises(oracle.OracleError) as e:
        perm(A, p, q, rows=np.array([3, 50]))
    assert e.value.name == "INDEX_RANGE"


# ----------------------------------------------------------------- spref ---

@pytest.mark.parametrize("how", sorted(SPREFS))
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("vdtype", [np.float64, np.float32])
def test_spref_brute_scipy_selection(shape, vdtype, how):
    rng = np.random.default_rng(7 + hash(shape) % 1000)
    m, n = shape
    A = rand_csr(rng, m, n, 0.35, vdtype)
    for trial in range(4):
        nI = int(rng.integers(0, 2 * m + 1))
        nJ = int(rng.integers(0, 2 * n + 1))
        I = rng.integers(0, m, nI)          # duplicates and any order
        J = rng.integers(0, n, nJ)
        got = SPREFS[how](A, I, J)
        assert_csr_equal(got, _brute_spref(A, I, J), "brute")
        if nI and nJ:
            S = to_scipy(A)
            assert_csr_equal(got, from_scipy(S[I][:, J]), "scipy")
            R = selection(I, m, vdtype)
            Q = selection(J, n, vdtype)
            assert_csr_equal(got, from_scipy(R @ S @ Q.T), "R A Q^T")
        # closed-form count: sum over selected rows of the multiplicity of each column in J
        mult = np.bincount(J, minlength=n)
        rp, c = A[2], A[3]
        expect = sum(int(mult[c[k]]) for i in I for k in range(rp[i], rp[i + 1]))
        assert got[0][-1] == expect


@pytest.mark.parametrize("how", sorted(SPREFS))
def test_spref_special_cases(how):
    rng = np.random.default_rng(11)
    m, n = 25, 19
    A = rand_csr(rng, m, n, 0.3)
    spref = SPREFS[how]
    # whole index sets in order reproduce A
    assert_csr_equal(spref(A, np.arange(m), np.arange(n)), A[2:], "identity")
    # full permutations make extraction a permutation (Sec. 2.2)
    p, q = rng.permutation(m), rng.permutation(n)
    assert_csr_equal(spref(A, p, q), _brute_permute(A, p, q), "perm special case")
    # sorted unique subsets keep the original order
    I = np.sort(rng.choice(m, 9, replace=False))
    J = np.sort(rng.choice(n, 7, replace=False))
    got = spref(A, I, J)
    D, M = dense(A)
    assert_csr_equal(got, from_dense(D[I][:, J], M[I][:, J]), "ordered submatrix")
    # empty index sets give an empty, correctly shaped result
    e = spref(A, np.zeros(0, np.int64), J)
    assert e[0].tolist() == [0] and e[1].size == 0
    e = spref(A, I, np.zeros(0, np.int64))
    assert e[0].tolist() == [0] * (len(I) + 1)
    # one column repeated many times: every copy is emitted, in position order
    J = np.array([3, 5, 3, 3, 0, 5])
    assert_csr_equal(spref(A, np.arange(m), J), _brute_spref(A, np.arange(m), J), "repeats")


@pytest.mark.parametrize("how", sorted(SPREFS))
def test_spref_sampled_rows_match_full(how):
    """The sampled-row mode returns exactly the listed rows of the full
    result (in list order, repeats kept)."""
    rng = np.random.default_rng(13)
    A = rand_csr(rng, 40, 30, 0.3)
    I = rng.integers(0, 40, 55)
    J = rng.integers(0, 30, 45)
    full = _brute_spref(A, I, J)
    spref = SPREFS[how]
    for rows in (np.array([54, 0, 9, 9, 31, 2]), np.arange(55)[::-1].copy(), np.zeros(0, np.int64)):
        assert_csr_equal(spref(A, I, J, rows=rows), _rows_of(full, rows), f"rows {rows[:6]}")
    with pytest.raises(oracle.OracleError) as e:
        spref(A, I, J, rows=np.array([0, 55]))
    assert e.value.name == "INDEX_RANGE"


@pytest.mark.parametrize("how", sorted(SPREFS))
def test_spref_exhaustive_tiny(how):
    """Every index vector of length <= 2 over a 3 x 3 matrix, against brute force."""
    rng = np.random.default_rng(5)
    A = rand_csr(rng, 3, 3, 0.5)
    vecs = [()] + [(a,) for a in range(3)] + list(itertools.product(range(3), repeat=2))
    for I in vecs:
        for J in vecs:
            I_ = np.array(I, dtype=np.int64)
            J_ = np.array(J, dtype=np.int64)
            assert_csr_equal(SPREFS[how](A, I_, J_), _brute_spref(A, I_, J_), f"{I} {J}")


# ---------------------------------------------------------------- spasgn ---

def _rand_assign(rng, m, n, vdtype=np.float64):
    A = rand_csr(rng, m, n, 0.3, vdtype)
    nI = int(rng.integers(0, m + 1))
    nJ = int(rng.integers(0, n + 1))
    I = rng.choice(m, nI, replace=False)
    J = rng.choice(n, nJ, replace=False)
    B = rand_csr(rng, nI, nJ, 0.4, vdtype)
    return A, B, I, J


@pytest.mark.parametrize("how", sorted(SPASGNS))
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("vdtype", [np.float64, np.float32])
@pytest.mark.parametrize("op", ["second", "plus", "replace"])
def test_spasgn_brute(shape, vdtype, op, how):
    rng = np.random.default_rng(17 + hash((shape, op)) % 1000)
    for trial in range(3):
        A, B, I, J = _rand_assign(rng, *shape, vdtype)
        got = SPASGNS[how](A, B, I, J, op)
        assert_csr_equal(got, _brute_spasgn(A, B, I, J, op), f"brute {op}")


@pytest.mark.parametrize("vdtype", [np.float64, np.float32])
def test_spasgn_plus_is_selection_product(vdtype):
    """PLUS is A + P B Q^T with the Boolean P, Q of Sec. 2.3."""
    rng = np.random.default_rng(23)
    for trial in range(6):
        m, n = 20 + trial, 15 + 2 * trial
        A, B, I, J = _rand_assign(rng, m, n, vdtype)
        if len(I) == 0 or len(J) == 0:
            continue
        S = to_scipy(A)
        P = selection(I, m, vdtype).T.tocsr()      # m x |I|, P[r,i]=1 iff r = I[i]
        Q = selection(J, n, vdtype).T.tocsr()
        exp = from_scipy(S + P @ to_scipy(B) @ Q.T)
        assert_csr_equal(oracle.spasgn(A, B, I, J, "plus"), exp, "A + P B Q^T")


def test_spasgn_invariants():
    rng = np.random.default_rng(29)
    m, n = 30, 26
    A, B, I, J = _rand_assign(rng, m, n)
    Da, Ma = dense(A)
    inside = np.zeros((m, n), bool)
    inside[np.ix_(I, J)] = True
    for op in ("second", "plus", "replace"):
        got = oracle.spasgn(A, B, I, J, op)
        Dg, Mg = dense((m, n) + got)
        # outside I x J nothing changes
        assert np.array_equal(Mg & ~inside, Ma & ~inside)
        assert np.array_equal(np.where(~inside, Dg, 0), np.where(~inside, Da, 0))
    # block replace then extract gives B back exactly
    rep = oracle.spasgn(A, B, I, J, "replace")
    assert_csr_equal(oracle.spref((m, n) + rep, I, J), B[2:], "extract after replace")
    # select-second: entries outside pattern(B') keep A's value
    sec = oracle.spasgn(A, B, I, J, "second")
    Dg, Mg = dense((m, n) + sec)
    Bp = np.zeros((m, n), bool)
    bm, bn, brp, bc, bv = B
    for i in range(bm):
        for k in range(brp[i], brp[i + 1]):
            Bp[I[i], J[bc[k]]] = True
    assert np.array_equal(Mg, Ma | Bp)
    assert np.array_equal(np.where(~Bp, Dg, 0), np.where(~Bp, Da, 0))


@pytest.mark.parametrize("how", sorted(SPASGNS))
@pytest.mark.parametrize("op", ["second", "plus", "replace"])
def test_spasgn_sampled_rows_match_full(op, how):
    """The sampled-row mode returns exactly the listed rows of the full
    result: rows inside and outside I, repeated and out of order."""
    rng = np.random.default_rng(41)
    A, B, I, J = _rand_assign(rng, 30, 24)
    while len(I) < 3 or len(I) > 27:
        A, B, I, J = _rand_assign(rng, 30, 24)
    full = _brute_spasgn(A, B, I, J, op)
    outside = np.setdiff1d(np.arange(30), I)
    for rows in (np.array([I[0], outside[0], I[-1], I[0], 29, 0]), np.arange(30)[::-1].copy(),
                 np.zeros(0, np.int64)):
        assert_csr_equal(SPASGNS[how](A, B, I, J, op, rows=rows), _rows_of(full, rows), f"rows {rows[:6]}")
    with pytest.raises(oracle.OracleError) as e:
        SPASGNS[how](A, B, I, J, op, rows=np.array([30]))
    assert e.value.name == "INDEX_RANGE"


def test_map_routines_thread_count_independent():
    """The table routines give the same bytes for any thread count on a
    matrix with long and empty rows."""
    rng = np.random.default_rng(43)
    A = rand_csr(rng, 300, 200, 0.05)
    rp = A[2].copy()
    p, q = rng.permutation(300), rng.permutation(200)
    I, J = rng.integers(0, 300, 400), rng.integers(0, 200, 260)
    base_p = oracle.permute_map(A, p, q)
    base_s = oracle.spref_map(A, I, J)
    for t in (2, 5, 16):
        assert_csr_equal(oracle.permute_map(A, p, q, threads=t), base_p, f"permute {t}")
        assert_csr_equal(oracle.spref_map(A, I, J, threads=t), base_s, f"spref {t}")
    assert np.array_equal(rp, A[2])


def test_spasgn_round_trip_streaming():
    """Split A's edges into 80% + 4 x 5%, assign the parts back one by one
    (the streaming-update experiment of the assignment results): A returns."""
    rng = np.random.default_rng(31)
    m, n = 60, 60
    A = rand_csr(rng, m, n, 0.15)
    D, M = dense(A)
    label = rng.choice(5, size=(m, n), p=[0.8, 0.05, 0.05, 0.05, 0.05])
    cur = from_dense(np.where(label == 0, D, 0), M & (label == 0))
    for part in range(1, 5):
        Mp = M & (label == part)
        I = np.nonzero(Mp.any(1))[0]
        J = np.nonzero(Mp.any(0))[0]
        Bd, Bm = D[np.ix_(I, J)], Mp[np.ix_(I, J)]
        B = (len(I), len(J)) + from_dense(np.where(Bm, Bd, 0), Bm)
        cur = oracle.spasgn((m, n) + cur, B, I, J, "second")
    assert_csr_equal(cur, A[2:], "round trip")


# ---------------------------------------------------------------- errors ---

def test_error_statuses():
    rng = np.random.default_rng(37)
    A = rand_csr(rng, 6, 5, 0.4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.permute(A, np.array([0, 1, 2, 3, 4, 4]), np.arange(5))
    assert e.value.name == "NOT_PERMUTATION"
    with pytest.raises(oracle.OracleError) as e:
        oracle.permute(A, np.arange(6), np.array([0, 1, 2, 3, 5]))
    assert e.value.name == "INDEX_RANGE"
    with pytest.raises(oracle.OracleError) as e:
        oracle.permute(A, np.arange(6))                 # symmetric needs square
    assert e.value.name == "SHAPE"
    with pytest.raises(oracle.OracleError) as e:
        oracle.spref(A, np.array([0, 6]), np.arange(5))
    assert e.value.name == "INDEX_RANGE"
    with pytest.raises(oracle.OracleError) as e:
        oracle.permute_map(A, np.array([0, 1, 2, 3, 4, 4]), np.arange(5))
    assert e.value.name == "NOT_PERMUTATION"
    with pytest.raises(oracle.OracleError) as e:
        oracle.permute_map(A, np.arange(6))
    assert e.value.name == "SHAPE"
    with pytest.raises(oracle.OracleError) as e:
        oracle.spref_map(A, np.array([0, 1]), np.array([5]))
    assert e.value.name == "INDEX_RANGE"
    B = rand_csr(rng, 2, 2, 0.5)
    with pytest.raises(oracle.OracleError) as e:
        oracle.spasgn(A, B, np.array([1, 1]), np.array([0, 2]))
    assert e.value.name == "DUPLICATE_INDEX"
    with pytest.raises(oracle.OracleError) as e:
        oracle.spasgn(A, B, np.array([1, 2, 3]), np.array([0, 2]))
    assert e.value.name == "SHAPE"
    assert oracle.check_csr(A) == "OK"
    bad = (6, 5, A[2], A[3][::-1].copy(), A[4])
    assert oracle.check_csr(bad) != "OK"


# ------------------------------------------- extraction on CSC / DCSC -------

def _brute_spref_csc(A, I, J):
    """CSC of C = A(I, J) from the dense matrix (fancy indexing of numpy)."""
    D, M = dense(A)
    Dc, Mc = D[np.ix_(I, J)].T, M[np.ix_(I, J)].T    # CSR of C^T is the CSC of C
    return from_dense(Dc, Mc)


def test_golden_spref_dcsc():
    g = read_golden("spref_dcsc_3x5.txt")
    m, n = ints(g["shape"])
    A = (int(m), int(n), ints(g["jc"]).astype(np.int32), ints(g["colptr"]), ints(g["row"]).astype(np.int32),
         floats(g["val"]))
    got = oracle.spref_dcsc(A, ints(g["I"]), ints(g["J"]))
    assert_csr_equal(got, (ints(g["expect_colptr"]), ints(g["expect_row"]), floats(g["expect_val"])),
                     "golden spref dcsc")


@pytest.mark.parametrize("shape,density", [((1, 1), 1.0), ((5, 7), 0.4), ((9, 13), 0.3), ((33, 20), 0.1),
                                           ((40, 120), 0.01), ((16, 16), 0.0)])
@pytest.mark.parametrize("vdtype", [np.float64, np.float32])
def test_spref_dcsc_brute_scipy_csr_oracle(shape, density, vdtype):
    """Against dense brute force, SciPy fancy indexing and the CSR oracle
    (converted to CSC by SciPy); CSC and DCSC storage give the same C."""
    rng = np.random.default_rng(shape[0] * 131 + shape[1])
    m, n = shape
    A = rand_csr(rng, m, n, density, vdtype)
    I = rng.integers(0, m, 2 * m + 1)
    J = rng.integers(0, n, 2 * n + 1)
    exp = _brute_spref_csc(A, I, J)
    for compress in (True, False):
        got = oracle.spref_dcsc(to_dcsc(A, compress), I, J)
        assert_csr_equal(got, exp, f"dcsc {compress} vs brute")
    assert_csr_equal(got, csc_of(to_scipy(A)[I][:, J]), "vs scipy")
    crow, ccol, cval = oracle.spref(A, I, J)
    C = to_scipy((len(I), len(J), crow, ccol, cval))
    assert_csr_equal(got, csc_of(C), "vs csr oracle")


def test_spref_dcsc_special_cases():
    rng = np.random.default_rng(5)
    A = rand_csr(rng, 10, 50, 0.05)
    Ad = to_dcsc(A)
    assert len(Ad[2]) < 50                       # some columns are not stored
    missing = np.setdiff1d(np.arange(50), Ad[2])[:4]
    # only unstored columns selected: all output columns empty
    cp, r, v = oracle.spref_dcsc(Ad, np.arange(10), missing)
    assert list(cp) == [0] * (len(missing) + 1) and len(r) == 0
    # empty I or J
    cp, r, v = oracle.spref_dcsc(Ad, np.zeros(0, np.int64), np.arange(50))
    assert len(cp) == 51 and cp[-1] == 0
    cp, r, v = oracle.spref_dcsc(Ad, np.arange(10), np.zeros(0, np.int64))
    assert list(cp) == [0]
    # identity selection returns A's own CSC
    assert_csr_equal(oracle.spref_dcsc(Ad, np.arange(10), np.arange(50)), csc_of(to_scipy(A)), "identity")
    # sampled output columns equal the matching columns of the full result
    I = rng.integers(0, 10, 12)
    J = rng.integers(0, 50, 30)
    full = oracle.spref_dcsc(Ad, I, J)
    cols = np.array([0, 7, 29, 3])
    part = oracle.spref_dcsc(Ad, I, J, cols=cols)
    for s, j in enumerate(cols):
        a, b = full[0][j], full[0][j + 1]
        c, d = part[0][s], part[0][s + 1]
        assert np.array_equal(full[1][a:b], part[1][c:d]) and np.array_equal(full[2][a:b], part[2][c:d])
    with pytest.raises(oracle.OracleError) as e:
        oracle.spref_dcsc(Ad, np.array([10]), np.array([0]))
    assert e.value.name == "INDEX_RANGE"
    with pytest.raises(oracle.OracleError) as e:
        oracle.spref_dcsc(Ad, np.array([0]), np.array([50]))
    assert e.value.name == "INDEX_RANGE"
