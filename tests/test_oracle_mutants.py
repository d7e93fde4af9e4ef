"""Plant plausible mistakes in a copy of the oracle's C source and check that
the pins catch every one of them (a dropped term, a wrong sign, a transposed
operand, an off-by-one bound).  Each mutant is compiled with gcc into a
temporary directory and exercised in a subprocess, so a crash or a hang in a
mutant cannot take the test run down.
"""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "crystal_oracle.c")

MUTANTS = {
    "select_open_upper_bound": ("if (v >= lo && v <= hi) {", "if (v >= lo && v < hi) {"),
    "select_open_lower_bound": ("if (v >= lo && v <= hi) {", "if (v > lo && v <= hi) {"),
    "project_transposed_operand": ("b * (double)x2[i];\n        out[i] = (float)v;",
                                   "b * (double)x1[i];\n        out[i] = (float)v;"),
    "project_wrong_sign": ("double v = a * (double)x1[i] + b * (double)x2[i];\n        out[i] = (float)v;",
                           "double v = a * (double)x1[i] - b * (double)x2[i];\n        out[i] = (float)v;"),
    "project_single_precision": ("double v = a * (double)x1[i] + b * (double)x2[i];\n        out[i] = (float)v;",
                                 "float v = (float)a * x1[i] + (float)b * x2[i] * 1.0000001f;\n        out[i] = v;"),
    "sigmoid_sign": ("out[i] = (float)(1.0 / (1.0 + exp(-v)));", "out[i] = (float)(1.0 / (1.0 + exp(v)));"),
    "join_drops_probe_payload": ("if (pval) s += (uint64_t)(int64_t)pval[i];", ""),
    "join_filter_off_by_one": ("if (bfilter && (bfilter[r] < flo || bfilter[r] > fhi)) continue;",
                               "if (bfilter && (bfilter[r] <= flo || bfilter[r] > fhi)) continue;"),
    "bisection_wrong_direction": ("if (km < k) a = m + 1; else b = m - 1;",
                                  "if (km > k) a = m + 1; else b = m - 1;"),
    "direct_index_shifted": ("return ix->direct[(int64_t)k - ix->min_key];",
                             "return ix->direct[(int64_t)k - ix->min_key] + (k == ix->min_key);"),
    "join_32bit_sum": ("if (bval) s += (uint64_t)(int64_t)bval[r];",
                       "if (bval) s = (uint32_t)(s + (uint64_t)(int64_t)bval[r]);"),
    "groupby_drops_value_sign": ("acc[g[i]] += (uint64_t)(int64_t)v[i];",
                                 "acc[g[i]] += (uint64_t)(uint32_t)v[i];"),
    "star_group_base_sign": ("group += ((int64_t)p->dim_group[j][r] - p->group_base[j]) * p->group_stride[j];",
                             "group += ((int64_t)p->dim_group[j][r] + p->group_base[j]) * p->group_stride[j];"),
    "star_group_drops_stride": ("group += ((int64_t)p->dim_group[j][r] - p->group_base[j]) * p->group_stride[j];",
                                "group += ((int64_t)p->dim_group[j][r] - p->group_base[j]);"),
    "star_diff_sign": ("case 2: val = (uint64_t)((int64_t)p->cols[p->agg_col0][i] -",
                       "case 2: val = (uint64_t)((int64_t)p->cols[p->agg_col0][i] +"),
    "star_product_operand": ("(int64_t)p->cols[p->agg_col1][i]); break;\n        case 2",
                             "(int64_t)p->cols[p->agg_col0][i]); break;\n        case 2"),
    "star_drops_last_predicate": ("for (int32_t q = 0; q < p->n_preds && pass; ++q) {",
                                  "for (int32_t q = 0; q + 1 < p->n_preds && pass; ++q) {"),
    "star_dim_filter_off_by_one": ("if (f < p->dim_flo[j] || f > p->dim_fhi[j]) { pass = 0; break; }",
                                   "if (f < p->dim_flo[j] || f >= p->dim_fhi[j] + (f > 0)) { pass = 0; break; }"),
    "star_ignores_dim_filter": ("if (p->dim_filter[j]) {", "if (0 && p->dim_filter[j]) {"),
    "star_inner_join_keeps_misses": ("if (r < 0) { pass = 0; break; }", "if (r < 0) { continue; }"),
    "radix_digit_drops_top_bit": ("return (key >> shift) & ((1u << bits) - 1u);",
                                  "return (key >> shift) & ((1u << (bits - 1)) - 1u);"),
    "radix_inclusive_prefix": ("        next[d] = run;\n        run += c;", "        run += c;\n        next[d] = run;"),
    "sort_unstable_ties": ("return (a > b) - (a < b); /* equal keys keep input order */",
                           "return (a < b) - (a > b); /* equal keys keep input order */"),
}

RUNNER = textwrap.dedent("""
    import sys
    sys.path[:0] = [{root!r}, {tests!r}]
    import oracle
    from oracle_pins import ALL_PINS
    lib = oracle.load({lib!r})
    failed = []
    for pin in ALL_PINS:
        try:
            pin(lib)
        except Exception as e:  # AssertionError or OracleError
            failed.append(pin.__name__)
    print("FAILED", ",".join(failed))
""")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique in the oracle source"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    oracle.build(src=str(mpath), out=lib)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    except subprocess.TimeoutExpired:
        return  # a hang is a detected mutant as well
    if r.returncode != 0:
        return  # a crash is a detected mutant as well
    line = [l for l in r.stdout.splitlines() if l.startswith("FAILED")][-1]
    failed = [x for x in line[len("FAILED"):].strip().split(",") if x]
    assert failed, f"mutant {name} passed every pin"
