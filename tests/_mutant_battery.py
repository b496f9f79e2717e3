"""Runs the oracle pins against an oracle library given on the command line.

Exit status 0: every pin held (a planted mistake survived); 1: some pin failed.
Used by test_oracle_mutants.py, always in a child process."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from tests import test_oracle_pins as T  # noqa: E402
from tests._util import assert_csr_equal, rand_csr, to_dcsc  # noqa: E402


def battery(lib):
    rng = np.random.default_rng(99)
    for (m, n) in [(7, 7), (12, 9), (16, 16)]:
        for vd in (np.float64, np.float32):
            A = rand_csr(rng, m, n, 0.35, vd)
            p, q = rng.permutation(m), rng.permutation(n)
            exp = T._brute_permute(A, p, q)
            assert_csr_equal(oracle.permute(A, p, q, lib=lib), exp, "perm")
            for t in (1, 3):
                assert_csr_equal(oracle.permute_map(A, p, q, lib=lib, threads=t), exp, "perm map")
            rows = np.array([m - 1, 0, 2, 2, m // 2])
            assert_csr_equal(oracle.permute(A, p, q, rows=rows, lib=lib), T._rows_of(exp, rows), "perm rows")
            assert_csr_equal(oracle.permute_map(A, p, q, rows=rows, lib=lib), T._rows_of(exp, rows),
                             "perm map rows")
            I = rng.integers(0, m, 2 * m)
            J = rng.integers(0, n, 2 * n)
            exp = T._brute_spref(A, I, J)
            assert_csr_equal(oracle.spref(A, I, J, lib=lib), exp, "spref")
            for t in (1, 3):
                assert_csr_equal(oracle.spref_map(A, I, J, lib=lib, threads=t), exp, "spref map")
            rows = np.array([2 * m - 1, 0, 3, 3, m])
            assert_csr_equal(oracle.spref(A, I, J, rows=rows, lib=lib), T._rows_of(exp, rows), "spref rows")
            assert_csr_equal(oracle.spref_map(A, I, J, rows=rows, lib=lib), T._rows_of(exp, rows),
                             "spref map rows")
            for compress in (True, False):
                assert_csr_equal(oracle.spref_dcsc(to_dcsc(A, compress), I, J, lib=lib),
                                 T._brute_spref_csc(A, I, J), "spref dcsc")
            for op in ("second", "plus", "replace"):
                for trial in range(3):
                    A2, B, I2, J2 = T._rand_assign(rng, m, n, vd)
                    exp = T._brute_spasgn(A2, B, I2, J2, op)
                    assert_csr_equal(oracle.spasgn(A2, B, I2, J2, op, lib=lib, threads=1 + 2 * (trial % 2)),
                                     exp, op)
                    rows = np.array([m - 1, 0, 1, 1] + [int(x) for x in I2[:2]])
                    assert_csr_equal(oracle.spasgn(A2, B, I2, J2, op, rows=rows, lib=lib), T._rows_of(exp, rows),
                                     op + " rows")
    A = rand_csr(rng, 6, 5, 0.4)
    try:
        oracle.permute(A, np.array([0, 1, 2, 3, 4, 4]), np.arange(5), lib=lib)
        raise AssertionError("duplicate p accepted")
    except oracle.OracleError as e:
        assert e.name == "NOT_PERMUTATION"
    B = rand_csr(rng, 2, 2, 0.5)
    try:
        oracle.spasgn(A, B, np.array([1, 1]), np.array([0, 2]), lib=lib)
        raise AssertionError("duplicate I accepted")
    except oracle.OracleError as e:
        assert e.name == "DUPLICATE_INDEX"


if __name__ == "__main__":
    lib = oracle._load(sys.argv[1])
    try:
        battery(lib)
    except AssertionError as e:
        print("pin failed:", str(e).splitlines()[0])
        sys.exit(1)
    sys.exit(0)
