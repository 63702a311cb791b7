"""Mutation check of the oracle's pins: plant one plausible mistake at a time
in a temporary copy of the oracle's C source (a wrong sign, a transposed
operand, a dropped term, a wrong index), build that copy, and require that
the pin suites fail against it.  The real oracle is never modified.  CPU only.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# (file, original text, planted text)
MUTANTS = {
    "trig-apply-sign": ("jacobi.c", "x[k] = c * xk - s * yk;", "x[k] = c * xk + s * yk;"),
    "hyp-apply-sign": ("jacobi.c", "} else {\n            x[k] = c * xk + s * yk;",
                       "} else {\n            x[k] = c * xk - s * yk;"),
    "trig-zeta-swapped": ("jacobi.c", "zeta = (aqq - app) / (2 * apq);",
                          "zeta = (app - aqq) / (2 * apq);"),
    "hyp-tanh-sign": ("jacobi.c", "t = -sg / (az + R_SQRT((az - 1) * (az + 1)));",
                      "t = sg / (az + R_SQRT((az - 1) * (az + 1)));"),
    "gram-transposed-operand": ("jacobi.c", "sxy = sxy + x[k] * y[k];", "sxy = sxy + x[k] * x[k];"),
    "cos-wrong-sign": ("jacobi.c", "c = 1 / R_SQRT(1 + t * t);", "c = 1 / R_SQRT(1 - t * t);"),
    "v-not-accumulated": ("jacobi.c",
                          "    if (W) apply_pair(W + (size_t)p * ldw, W + (size_t)q * ldw, wlen, c, s, same_sign);",
                          ""),
    "lambda-sign-dropped": ("jacobi.c", "lambda[i] = (double)((J && J[i] < 0) ? -nrm2 : nrm2);",
                            "lambda[i] = (double)nrm2;"),
    "threshold-factor-dropped": ("jacobi.c", "if (!(R_FABS(apq) > tol * R_SQRT(app) * R_SQRT(aqq))) return 0;",
                                 "if (!(R_FABS(apq) > tol * R_SQRT(app))) return 0;"),
    "ordering-index-off-by-one": ("ordering.c", "int j = ((k - i - 1) % n + n) % n + 1;",
                                  "int j = ((k - i) % n + n) % n + 1;"),
    "modmod-extra-pair-wrong": ("ordering.c", "int i = k / 2, j = k / 2 + n / 2;",
                                "int i = k / 2, j = k / 2 + n / 2 - 1;"),
    "block-update-transposed": ("jacobi.c",
                                "const real v = VP[(size_t)c * w + k], *in = GP + (size_t)k * m;",
                                "const real v = VP[(size_t)k * w + c], *in = GP + (size_t)k * m;"),
    "block-gram-wrong-column": ("jacobi.c",
                                "acc[2] = acc[2] + x[r] * y0[2 * (size_t)m + r];",
                                "acc[2] = acc[2] + x[r] * y0[(size_t)m + r];"),
    "block-gram-not-mirrored": ("jacobi.c", "                AP[(size_t)k * w + l0 + q] = acc[q];\n",
                                ""),
    "sp-reversal-dropped": ("jacobi.c", "const int src = pp[nn - 1 - c];", "const int src = pp[c];"),
    "sp-pivot-smallest": ("jacobi.c", "if (W[(size_t)i * k + i] > W[(size_t)t * k + t]) t = i;",
                          "if (W[(size_t)i * k + i] < W[(size_t)t * k + t]) t = i;"),
    "sp-schur-sign": ("jacobi.c",
                      "sum = sum - RS[(size_t)(np + r) * w + k] * RS[(size_t)(np + c) * w + k];",
                      "sum = sum + RS[(size_t)(np + r) * w + k] * RS[(size_t)(np + c) * w + k];"),
    "sp-vp-rows-not-permuted": ("jacobi.c",
                                "VP[(size_t)c * w + perm[r]] = VQ[(size_t)c * w + r];",
                                "VP[(size_t)c * w + r] = VQ[(size_t)c * w + r];"),
    "sp-signs-not-moved": ("jacobi.c", "for (int c = 0; c < w; ++c) Jc[colp[c]] = JS[c];", ""),
    "block-cholesky-term-dropped": ("jacobi.c",
                                    "sum = sum - R[(size_t)i * w + k] * R[(size_t)j * w + k];",
                                    "sum = sum - R[(size_t)i * w + k] * R[(size_t)i * w + k];"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    fname, old, new = MUTANTS[name]
    for f in ("ordering.c", "jacobi.c"):
        shutil.copy(os.path.join(ORACLE, f), tmp_path / f)
    src = (tmp_path / fname).read_text()
    assert src.count(old) == 1, "mutation site must be unique"
    (tmp_path / fname).write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    try:
        from oracle import build as B
        lib = B.build(srcdir=str(tmp_path), lib=str(tmp_path / "liboracle.so"))
    finally:
        sys.path.remove(ROOT)
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_ordering.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_signpivot.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "the pins did not notice the planted mistake %r" % name
    assert "failed" in r.stdout
