"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of oracle.c (a swapped operand, a wrong
sign, a mirrored or transposed index, an off-by-one, a dropped term, a wrong
identity), builds it with gcc into a temporary library, and runs the pin suite
against it in a child process.  The suite must fail for every mutant.  Nothing
here touches the HIP library.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text to replace, replacement, which occurrence (0-based))
MUTANTS = [
    ("axpy_swapped_operands", "*res = p[0] * x + y;", "*res = p[0] * y + x;", 0),
    ("affine_sign", "*res = p[0] * x + p[1];", "*res = p[0] * x - p[1];", 0),
    ("affine_tanh_grouping", "tanh(p[0] * x + p[1])", "tanh(p[0] * (x + p[1]))", 0),
    ("reduce_drops_first_term",
     "for (int64_t i = 0; i < n; ++i) {\n        double v = (double)x[i];",
     "for (int64_t i = 1; i < n; ++i) {\n        double v = (double)x[i];", 0),
    ("abs_sum_without_abs", "acc = acc + fabs((double)x[i]);",
     "acc = acc + (double)x[i];", 0),
    ("mapreduce_mag_without_abs", "mag = mag + fabs(v);", "mag = mag + v;", 0),
    ("overlap1d_mirrored", "border_index(i + k - r, n", "border_index(i - k + r, n", 0),
    ("overlap2d_rows_mirrored", "border_index(i + a - ry, rows",
     "border_index(i - a + ry, rows", 0),
    ("separable_x_factor_mirrored", "return (double)wy[a] * (double)wx[b];",
     "return (double)wy[a] * (double)wx[2 * rx - b];", 0),
    ("clamp_ends_swapped", "*k = j < 0 ? 0 : n - 1;", "*k = j < 0 ? n - 1 : 0;", 0),
    ("cyclic_off_by_one", "*k = m < 0 ? m + n : m;", "*k = m < 0 ? m + n - 1 : m;", 0),
    ("const_pad_ignored", "(double)x[src]\n                                                               : (double)pad;",
     "(double)x[src]\n                                                               : 0.0;", 0),
    ("scan_identity_swapped", "TOUT macc = op == ORC_MIN ? TMAX : TMIN;",
     "TOUT macc = op == ORC_MIN ? TMIN : TMAX;", 0),
    ("scan_inclusive_is_exclusive",
     "            if (!scan_excludes_self(kind))                                     \\\n"
     "                out[i] = op == ORC_SUM ? (TOUT)sacc : macc;",
     "            if (!scan_excludes_self(kind))                                     \\\n"
     "                out[i] = op == ORC_SUM ? (TOUT)(sacc - (UACC)v) : macc;", 0),
    ("scan_f32_mag_without_abs", "m = m + fabs(v);\n        if (!scan_excludes_self(kind)) {",
     "m = m + v;\n        if (!scan_excludes_self(kind)) {", 0),
    ("reverse_exclusive_keeps_self",
     "return kind == ORC_EXCLUSIVE || kind == ORC_REVERSE_EXCLUSIVE;",
     "return kind == ORC_EXCLUSIVE;", 0),
    ("reverse_scan_runs_forward", "return kind >= ORC_REVERSE_INCLUSIVE ? n - 1 - t : t;",
     "return t;", 0),
    ("adjoint1d_mirrored", "if (!border_index(i + k - r, n, edge, &src)) continue;",
     "if (!border_index(i - k + r, n, edge, &src)) continue;", 0),
    ("adjoint2d_cols_mirrored", "if (!border_index(j + b - rx, cols, edge, &sj)) continue;",
     "if (!border_index(j - b + rx, cols, edge, &sj)) continue;", 0),
    ("grad_affine_tanh_drops_scale", "*fx = p[0] * d;", "*fx = d;", 0),
    ("grad_tanh_wrong", "*fx = 1.0 - t * t;", "*fx = 1.0 - t;", 0),
    ("grad_axpy_param", "case ORC_MAP_AXPY: *fx = p[0]; *fy = 1.0; *fp0 = x; break;",
     "case ORC_MAP_AXPY: *fx = p[0]; *fy = 1.0; *fp0 = 1.0; break;", 0),
    ("reduce_i64_wraps_at_32", "for (int64_t i = 0; i < n; ++i) acc = acc + (uint64_t)(int64_t)x[i];",
     "for (int64_t i = 0; i < n; ++i) acc = (uint32_t)(acc + (uint64_t)(int64_t)x[i]);", 0),
    ("min_is_max", "if (op == ORC_MIN) acc = v < acc ? v : acc;",
     "if (op == ORC_MIN) acc = v > acc ? v : acc;", 0),
    ("fsum_drops_low_parts", "if (lo != 0.0) m->p[i++] = lo;", "(void)lo;", 0),
    ("fsum_no_halfway_fix", "if (y == x - hi) hi = x;", "(void)x;", 0),
    ("chain_skips_map", "elem_fn(map_op, params, nparams, (double)x[i], 0.0, &t[i]);",
     "t[i] = (double)x[i];", 0),
    ("chain_rows_mirrored", "int in_r = border_index(i + a - ry, rows, edge, &si);",
     "int in_r = border_index(i - a + ry, rows, edge, &si);", 1),
    ("chain_pad_ignored", "double v = (in_r && in_c) ? tf[si * cols + sj] : (double)pad;",
     "double v = (in_r && in_c) ? tf[si * cols + sj] : 0.0;", 0),
    ("chain_grad_cols_mirrored",
     "if (!border_index(j + b - rx, cols, edge, &sj)) continue;",
     "if (!border_index(j - b + rx, cols, edge, &sj)) continue;", 1),
    ("chain_grad_pad_reads_count",
     "if (!border_index(i + a - ry, rows, edge, &si)) continue;\n"
     "                        if (!border_index(j + b - rx, cols, edge, &sj)) continue;\n"
     "                        double term = weight2d(w2d, wy, wx, rx, a, b) * g1;",
     "if (!border_index(i + a - ry, rows, edge, &si)) si = i;\n"
     "                        if (!border_index(j + b - rx, cols, edge, &sj)) sj = j;\n"
     "                        double term = weight2d(w2d, wy, wx, rx, a, b) * g1;", 0),
    ("chain_grad_ignores_adjoint", "dx[k] = gt[k] * fx;", "dx[k] = g1 * fx;", 0),
    ("chain_grad_param_swapped", "s0 = s0 + gt[k] * fp0;", "s0 = s0 + gt[k] * fp1;", 0),
    ("segments_drop_last", "out[s] = oracle_reduce_f32(op, x + off[s], off[s + 1] - off[s]);",
     "out[s] = oracle_reduce_f32(op, x + off[s], off[s + 1] - off[s] - (off[s + 1] > off[s]));",
     0),
]


def _mutate(text, old, new, which):
    pos = -1
    for _ in range(which + 1):
        pos = text.find(old, pos + 1)
        assert pos >= 0, f"mutation anchor not found: {old!r}"
    return text[:pos] + new + text[pos + len(old):]


@pytest.mark.parametrize("name,old,new,which", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new, which):
    text = open(SRC).read()
    mutated = _mutate(text, old, new, which)
    assert mutated != text
    csrc = tmp_path / "oracle.c"
    csrc.write_text(mutated)
    (tmp_path / "oracle.h").write_text(open(os.path.join(ROOT, "oracle", "oracle.h")).read())
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp",
                    "-fPIC", "-shared", "-o", str(lib), str(csrc), "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, SKEL_ORACLE_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p",
                          "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert res.returncode != 0, f"mutant {name} survived the pins:\n{res.stdout[-2000:]}"
