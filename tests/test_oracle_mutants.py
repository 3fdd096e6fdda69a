"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutant is a textual edit of oracle.c (a dropped term, a wrong sign or
index, a transposed operand, an off-by-one), compiled on the CPU into a
temporary library. The real oracle is not touched.
"""
import os

import pytest

import oracle
import pins

MUTANTS = {
    "drop_last_term": ("for (i64 k = rowptr[i]; k < rowptr[i + 1]; ++k) {\n        u64 a = canon(val[k], m);\n        u64 xv",
                       "for (i64 k = rowptr[i]; k + 1 < rowptr[i + 1]; ++k) {\n        u64 a = canon(val[k], m);\n        u64 xv"),
    "canon_no_wrap": ("if (r < 0) r += (i64)m;", ""),
    "canon_negated": ("  return (u64)r;\n}", "  return r == 0 ? 0 : (u64)((i64)m - r);\n}"),
    "alpha_beta_swapped": ("(alpha * acc % m + beta * yv % m) % m", "(beta * acc % m + alpha * yv % m) % m"),
    "beta_dropped": ("(alpha * acc % m + beta * yv % m) % m", "(alpha * acc % m) % m"),
    "wrong_x_column": ("X[(i64)col[k] * ldx + b]", "X[(i64)col[k] * ldx + (s - 1 - b)]"),
    "transpose_wrong_row": ("u64 xv = (u64)X[i * ldx + b];", "u64 xv = (u64)X[(nrows - 1 - i) * ldx + b];"),
    "transpose_scatters_to_row": ("acc[j * s + b] = (acc[j * s + b] + a * xv) % m;",
                                  "acc[(i < ncols ? i : j) * s + b] = (acc[(i < ncols ? i : j) * s + b] + a * xv) % m;"),
    "power_off_by_one": ("for (i64 it = 0; it < k; ++it)", "for (i64 it = 0; it <= k; ++it)"),
    "sequence_shifted": ("  for (i64 i = 0; i < L; ++i) {\n    for (i64 a = 0; a < s; ++a)",
                         "  oracle_spmm(n, n, rowptr, col, val, m, s, 1, V, ldv, 0, W, s);\n  for (i64 i = 0; i < L; ++i) {\n    for (i64 a = 0; a < s; ++a)"),
    "projection_transposed": ("S[(i * s + a) * s + b] = (i64)acc;", "S[(i * s + b) * s + a] = (i64)acc;"),
    "projection_drops_last_row": ("for (i64 k = 0; k < n; ++k) acc =", "for (i64 k = 0; k + 1 < n; ++k) acc ="),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    find, repl = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(find) >= 1, "mutation site for %s no longer exists in oracle.c" % name
    mut_src = tmp_path / ("oracle_%s.c" % name)
    mut_src.write_text(src.replace(find, repl, 1))
    lib = oracle.build(force=True, src=str(mut_src), out=str(tmp_path / ("lib_%s.so" % name)))
    orc = oracle.Oracle(lib)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    assert caught, "mutant %s passed every pin" % name
