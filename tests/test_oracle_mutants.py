"""Each plausible mistake planted in a copy of the oracle's C source (on the
CPU, in a temporary directory) must make at least one oracle pin fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "xy_sign": ("out[1] = -k * offdiag_sum(U, V, W);", "out[1] = k * offdiag_sum(U, V, W);"),
    "xz_wrong_log_axis": ("out[2] = -k * offdiag_sum(U, W, V);", "out[2] = -k * offdiag_sum(U, V, W);"),
    "faces_swapped": ("U[0] = dx + hx; U[1] = dx - hx;", "U[0] = dx - hx; U[1] = dx + hx;"),
    "transposed_block": ("blk[ld + 0] = t6[1];", "blk[ld + 0] = t6[2];"),
    "mixed_log_sign": ("return log((w1 + R1) * (R2 - w2) / rho2);",
                       "return log((w1 + R1) * (R2 + w2) / rho2);"),
    "anis_axis": ("H[3 * a + i] += ka * me * e[i] + Ha[i];", "H[3 * a + i] += ka * me * e[0] + Ha[i];"),
    "exchange_half": ("H[3 * a + i] += coef * (m[3 * b + i] - m[3 * a + i]);",
                      "H[3 * a + i] += 0.5 * coef * (m[3 * b + i] - m[3 * a + i]);"),
    "damping_sign": ("dmdt[3 * a + 0] = -P->c1 * p0 - P->c2 * q0;",
                     "dmdt[3 * a + 0] = -P->c1 * p0 + P->c2 * q0;"),
    "tableau_bstar": ("-92097.0 / 339200", "-92097.0 / 339000"),
    "demag_scale": ("const double k = 1.0 / (4.0 * ORC_PI);", "const double k = 1.0 / (4.0 * 3.14);"),
    "threshold_ties_kept": ("if (fabs((double)(float)*e) <= cut) *e = 0.0;",
                            "if (fabs((double)(float)*e) < cut) *e = 0.0;"),
    "threshold_rank_floor": ("int64_t r = (int64_t)ceil(frac * (double)K);",
                             "int64_t r = (int64_t)floor(frac * (double)K);"),
    "threshold_self_blocks": ("if (row / 3 == col / 3) continue;", "if (row < 0) continue;"),
    "threshold_no_zero_floor": ("if (mag > floor32) v[K++] = mag;", "if (mag > 0.0) v[K++] = mag;"),
    "demag_target_ms": ("acc += row[col] * Ms[col / 3] * m[col];", "acc += row[col] * Ms[r / 3] * m[col];"),
    "rows_target_ms": ("double mx = Ms[b] * m[3 * b], my = Ms[b] * m[3 * b + 1], mz = Ms[b] * m[3 * b + 2];",
                       "double mx = Ms[a] * m[3 * b], my = Ms[a] * m[3 * b + 1], mz = Ms[a] * m[3 * b + 2];"),
    "rows_component_swap": ("h[1] += t6[1] * mx + t6[3] * my + t6[4] * mz;",
                            "h[1] += t6[1] * mx + t6[4] * my + t6[3] * mz;"),
}

PIN_FILES = ["tests/test_oracle_tensor.py", "tests/test_oracle_fields.py",
             "tests/test_oracle_dynamics.py", "tests/test_oracle_threshold.py",
             "tests/test_oracle_rows.py"]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    work = tmp_path / "tree"
    work.mkdir()
    shutil.copytree(os.path.join(ROOT, "oracle"), work / "oracle",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), work / "tests",
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "paper_2107_05364_amd"), work / "paper_2107_05364_amd",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
    src = work / "oracle" / "oracle.c"
    text = src.read_text()
    assert text.count(old) == 1, name
    src.write_text(text.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not slow"] + PIN_FILES, cwd=work, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, "mutant %s survived:\n%s" % (name, r.stdout[-2000:])
