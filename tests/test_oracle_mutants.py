"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of oracle/hp_oracle.c with one plausible mistake (a
dropped term, a wrong index, swapped operands, a wrong operator), compiled on
the CPU and run through the pin battery in a child process.  The real oracle
must pass the same battery."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hp_oracle.c")
BATTERY = os.path.join(ROOT, "tests", "_mutant_battery.py")

MUTANTS = {
    "perm_row_unmapped": ("int64_t src = p[i];", "int64_t src = i;"),
    "perm_col_unmapped": ("find_in_row(rowptr, col, src, q[j])", "find_in_row(rowptr, col, src, (int32_t)j)"),
    "perm_writes_old_col": ("out_col[cnt] = (int32_t)j;\n                copy_val(out_val, cnt, val, k, vsize);\n            }\n            cnt++;\n        }\n        out_ptr[s + 1] = cnt;\n    }\n    *need = cnt;\n    return ORC_OK;\n}\n\n/* ---- extraction",
                            "out_col[cnt] = q[j];\n                copy_val(out_val, cnt, val, k, vsize);\n            }\n            cnt++;\n        }\n        out_ptr[s + 1] = cnt;\n    }\n    *need = cnt;\n    return ORC_OK;\n}\n\n/* ---- extraction"),
    "spref_drops_last_col": ("for (int64_t j = 0; j < nJ; j++) {\n            int64_t k = find_in_row(rowptr, col, I[i], J[j]);",
                             "for (int64_t j = 0; j + 1 < nJ; j++) {\n            int64_t k = find_in_row(rowptr, col, I[i], J[j]);"),
    "spref_swapped_operands": ("find_in_row(rowptr, col, I[i], J[j])", "find_in_row(rowptr, col, J[j] % m, I[i])"),
    "asgn_second_keeps_a": ("else copy_val(out_val, cnt, bval, bp[kb].k, vsize);   /* select-second */",
                            "else copy_val(out_val, cnt, val, ka, vsize);"),
    "asgn_plus_subtracts": ("z = x + y;", "z = x - y;"),
    "asgn_b_cols_unmapped": ("bp[nb].c = J[bcol[k]];", "bp[nb].c = bcol[k];"),
    "asgn_rows_unmapped": ("for (int64_t i = 0; i < nI; i++) rowpos[I[i]] = i;",
                           "for (int64_t i = 0; i < nI; i++) rowpos[i] = i;"),
    "asgn_replace_off_by_one": ("colpos[col[ka]] >= 0", "colpos[col[ka]] > 0"),
    "perm_no_dup_check": ("if (seen[v[i]]) { st = ORC_NOT_PERMUTATION; break; }", ""),
    "asgn_no_dup_check": ("if (seen[v[i]]) { st = ORC_DUPLICATE_INDEX; break; }", ""),
    "dcsc_stored_col_unmapped": ("if (jc[mid] == c) return mid;", "if (jc[mid] == c) return c < nzc ? c : mid;"),
    "dcsc_row_not_position": ("out_row[cnt] = (int32_t)i;", "out_row[cnt] = I[i];"),
    "dcsc_search_skips_last": ("int64_t lo = colptr[k], hi = colptr[k + 1] - 1;",
                               "int64_t lo = colptr[k], hi = colptr[k + 1] - 2;"),
    # the routines through index tables
    "pmap_qinv_not_inverted": ("for (int64_t j = 0; j < n; j++) qinv[q[j]] = (int32_t)j;",
                               "for (int64_t j = 0; j < n; j++) qinv[j] = q[j];"),
    "pmap_row_unmapped": ("const int64_t src = x->p[i];", "const int64_t src = i;"),
    "map_rows_left_unsorted": ("    qsort(e, (size_t)n, sizeof(ent_t), cmp_ent);\n", ""),
    "smap_first_copy_only": ("for (int64_t t = x->lstart[c]; t < x->lstart[c + 1]; t++) {",
                             "for (int64_t t = x->lstart[c]; t < x->lstart[c + 1] && t == x->lstart[c]; t++) {"),
    "smap_positions_unmapped": ("work[cnt].c = x->list[t];", "work[cnt].c = (int32_t)(t - x->lstart[c]);"),
    "smap_row_shifted": ("const int64_t r = x->I[i];", "const int64_t r = x->I[i > 0 ? i - 1 : 0];"),
    # the sampled-row modes
    "spref_rows_first_only": ("int64_t i = rows ? rows[s] : s;\n        if (i < 0 || i >= nI) return ORC_INDEX_RANGE;",
                              "int64_t i = rows ? rows[0] : s;\n        if (i < 0 || i >= nI) return ORC_INDEX_RANGE;"),
    "perm_rows_first_only": ("int64_t i = rows ? rows[s] : s;\n        if (i < 0 || i >= m) return ORC_INDEX_RANGE;",
                             "int64_t i = rows ? rows[0] : s;\n        if (i < 0 || i >= m) return ORC_INDEX_RANGE;"),
    "driver_rows_first_only": ("return rows ? rows[s] : s;", "return rows ? rows[0] : s;"),
    "driver_all_rows_shifted": ("return rows ? rows[s] : s;", "return rows ? rows[s] : (s % 2 ? s - 1 : s);"),
}


def _build(tmp_path, name, src_text):
    c = tmp_path / f"{name}.c"
    c.write_text(src_text)
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", f"-I{os.path.dirname(SRC)}",
                           str(c), "-o", str(so)])
    return str(so)


def _run(so):
    return subprocess.run([sys.executable, BATTERY, so], capture_output=True, text=True, timeout=300)


def test_real_oracle_passes_battery():
    r = _run(oracle.build())
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation site for {name} not found"
    so = _build(tmp_path, name, text.replace(old, new, 1))
    r = _run(so)
    assert r.returncode != 0, f"planted mistake {name} survived every pin"
