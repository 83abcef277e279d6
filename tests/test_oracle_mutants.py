"""Planted mistakes: each pin set must reject a broken copy of the oracle.

Every mutant below is the oracle's C source with one plausible mistake (a
dropped term, a wrong sign or index, a swapped operand).  It is compiled to a
temporary library and the pins run against it in a child process (a mutant
that reads out of bounds may crash; that also counts as caught).  A mutant
that passes every pin would mean the pins cannot tell that mistake apart.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "xs_oracle.c")

MUTANTS = [
    ("bisect_strict_compare", "if (grid[mid] <= e)", "if (grid[mid] < e)"),
    ("bisect_no_minus_one", "  int64_t i = lo - 1;", "  int64_t i = lo;"),
    ("count_strict_compare", "if (grid[p] <= e) ++count;",
     "if (grid[p] < e) ++count;"),
    ("count_no_upper_clamp", "  if (i > n - 2) i = n - 2;\n  return i;\n}\n\nint64_t xso_bracket_bisect",
     "  return i;\n}\n\nint64_t xso_bracket_bisect"),
    ("no_low_energy_clamp", "    if (eh < grid[0]) eh = grid[0];\n    if (eh > grid[n - 1])",
     "    if (eh > grid[n - 1])"),
    ("no_high_energy_clamp", "    if (eh > grid[n - 1]) eh = grid[n - 1];\n    const double f",
     "    const double f"),
    ("wrong_denominator", "(grid[i + 1] - grid[i]);\n    const double g",
     "(grid[i + 1] - grid[0]);\n    const double g"),
    ("numerator_unclamped_e", "const double f = (eh - grid[i])",
     "const double f = (e - grid[i])"),
    ("g_sign", "const double g = 1.0 - f;", "const double g = 1.0 + f;"),
    ("swap_weights", "const double a = g * lo[c];", "const double a = f * lo[c];"),
    ("hi_channel_index", "const double b = f * hi[c];", "const double b = f * hi[0];"),
    ("lo_channel_index", "const double a = g * lo[c];", "const double a = g * lo[0];"),
    ("point_stride", "const double* lo = t->xs + (base + i) * XSO_CHANNELS;\n    const double* hi = lo + XSO_CHANNELS;\n    for (int c = 0; c < XSO_CHANNELS; ++c) {\n      const double a",
     "const double* lo = t->xs + (base + i);\n    const double* hi = lo + XSO_CHANNELS;\n    for (int c = 0; c < XSO_CHANNELS; ++c) {\n      const double a"),
    ("hi_is_lo", "const double* hi = lo + XSO_CHANNELS;\n    for (int c = 0; c < XSO_CHANNELS; ++c) {\n      const double a",
     "const double* hi = lo;\n    for (int c = 0; c < XSO_CHANNELS; ++c) {\n      const double a"),
    ("drop_density", "const double term = rho * sigma;", "const double term = sigma;"),
    ("no_accumulation", "sum[c] = sum[c] + term;", "sum[c] = term;"),
    ("first_nuclide_only", "const int32_t k = t->mat_nuclides[j];\n    const double rho = t->mat_density[j];",
     "const int32_t k = t->mat_nuclides[first];\n    const double rho = t->mat_density[j];"),
    ("density_of_first", "const double rho = t->mat_density[j];",
     "const double rho = t->mat_density[first];"),
    ("skip_last_nuclide", "for (int32_t j = first; j < last; ++j) {\n    const int32_t k = t->mat_nuclides[j];\n    const double rho",
     "for (int32_t j = first; j < last - 1; ++j) {\n    const int32_t k = t->mat_nuclides[j];\n    const double rho"),
    ("f32_no_compensation", "const float y = term - comp[c];", "const float y = term;"),
    ("f32_g_in_fp32", "const float g32 = (float)(1.0 - f);",
     "const float g32 = 1.0f - f32;"),
    ("f32_drop_density", "const float term = rho * sigma;", "const float term = sigma;"),
    ("f32_density_in_fp64", "const float rho = (float)t->mat_density[j];",
     "const double rho = t->mat_density[j];"),
    ("f32_x_unrounded_product", "const float b = f32 * (float)hi[c];",
     "const float b = (float)(f32 * hi[c]);"),
    ("f32_interpolate_in_fp64", "const float sigma = a + b;",
     "const float sigma = (float)((double)(1.0 - f) * lo[c] + f * hi[c]);"),
    ("invalid_not_nan", "for (int c = 0; c < XSO_CHANNELS; ++c) out[c] = NAN;",
     "for (int c = 0; c < XSO_CHANNELS; ++c) out[c] = 0.0;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert old in src, f"mutation site for {name} not found in the oracle"
    mutated = src.replace(old, new, 1)
    c_path = tmp_path / "mutant.c"
    c_path.write_text(mutated)
    so_path = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC",
                    "-shared", "-I", os.path.join(ROOT, "oracle"), "-o",
                    str(so_path), str(c_path), "-lm"], check=True)
    code = ("import sys; from tests import pins; "
            f"f = pins.run_all({str(so_path)!r}); print(f); "
            "sys.exit(1 if f else 0)")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} passed every pin"
