"""Planted mistakes in copies of the oracle must each be caught by some pin.

Each mutant rewrites one spot of oracle.c (a flipped tie rule, a dropped or
swapped term, a wrong sign, a different boundary, a strict threshold, counts
without multiplicity, flushed denormals, ...), is compiled into a temporary
library, and the pin suite is run against it.  This shows that the pins are
sharp enough to catch the plausible errors; the real oracle passes them all.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

import oracle
import synth

from . import pins  # noqa: F401  (the child process imports it)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "tie_u_ge": [("if (u > best) {", "if (u >= best) {")],
    "tie_l_ge": [("if (l > best) {", "if (l >= best) {")],
    "tie_order_LU": [("      if (u > best) {\n        best = u;\n        c = 'U';\n      }\n      if (l > best) {\n        best = l;\n        c = 'L';\n      }",
                      "      if (l > best) {\n        best = l;\n        c = 'L';\n      }\n      if (u > best) {\n        best = u;\n        c = 'U';\n      }")],
    "boundary_i_times_g": [("H[i * W] = H[(i - 1) * W] + g;", "H[i * W] = (float)i * g;"),
                           ("H[j] = H[j - 1] + g;", "H[j] = (float)j * g;")],
    "u_without_gap": [("float u = H[(i - 1) * W + j] + g;", "float u = H[(i - 1) * W + j];")],
    "drop_w3_term": [("t = w[3] * f3;", "t = 0.0f * f3;")],
    "swap_f1_f2": [("float f1 = ratio(ms, a);\n  float f2 = ratio(mt, b);", "float f1 = ratio(mt, b);\n  float f2 = ratio(ms, a);")],
    "f3_max_over_min": [("float f3 = ratio(lo, hi);", "float f3 = ratio(hi, lo);")],
    "sigmoid_sign": [("exp(-(double)z)", "exp((double)z)")],
    "sigmoid_in_float": [("return (float)(1.0 / (1.0 + exp(-(double)z)));", "return 1.0f / (1.0f + expf(-z) + 1e-6f);")],
    "threshold_strict": [("if (s >= tau) {", "if (s > tau) {")],
    "mt_unique_ids": [("for (int64_t p = tgt_sent_off[j]; p < tgt_sent_off[j + 1]; p++)\n        if (in_sorted(X[i], nX[i], tgt_tok[p])) mt++;",
                       "for (int64_t p = 0; p < nY[j]; p++)\n        if (in_sorted(X[i], nX[i], Y[j][p])) mt++;")],
    "ms_counts_translations": [("          if (in_sorted(Y[j], nY[j], L->tgt[e])) {\n            ms++;\n            break;\n          }",
                                "          if (in_sorted(Y[j], nY[j], L->tgt[e])) {\n            ms++;\n          }")],
    "flush_denormals": [("H[i * W + j] = best;", "H[i * W + j] = (best > -1.17549435e-38f && best < 1.17549435e-38f) ? 0.0f : best;")],
    "traceback_swap_UL": [("    } else if (c == 'U') {\n      i--;\n    } else {\n      j--;\n    }\n  }\n  for",
                           "    } else if (c == 'U') {\n      j--;\n    } else {\n      i--;\n    }\n  }\n  for")],
    "diag_uses_wrong_cell": [("float d = H[(i - 1) * W + (j - 1)] + S[(int64_t)(i - 1) * m + (j - 1)];",
                              "float d = H[(i - 1) * W + (j - 1)] + S[(int64_t)(j - 1 < n ? j - 1 : i - 1) * m + (i - 1 < m ? i - 1 : j - 1)];")],
}


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, workdir):
    synth.build(force=False)
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
        src = src.replace(old, new)
    cpath = os.path.join(workdir, f"{name}.c")
    lpath = os.path.join(workdir, f"lib{name}.so")
    with open(cpath, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", *oracle.CFLAGS, cpath, "-o", lpath, "-lm"])
    # run the pins in a child process: a mutant may also crash (out-of-bounds walk)
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import oracle, synth\n"
        "from tests import pins\n"
        "O = oracle.Oracle(%r)\n"
        "caught = []\n"
        "for check in pins.ALL + [lambda o: pins.check_identity_document(o, synth)]:\n"
        "    try:\n"
        "        check(O)\n"
        "    except AssertionError:\n"
        "        caught.append(getattr(check, '__name__', 'identity'))\n"
        "print('caught by', caught)\n"
        "sys.exit(3 if caught else 0)\n" % (ROOT, lpath))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} passed every pin: {r.stdout} {r.stderr[-2000:]}"
    if r.returncode != 3:  # crashed rather than failing a pin: still detected, say how
        print(f"mutant {name} crashed the pin run (rc={r.returncode})")
