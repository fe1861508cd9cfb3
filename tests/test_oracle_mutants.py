"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign or index, a
transposed operand, a wrong restart choice) in a temporary copy of the
oracle's C source, builds it, and runs the pin suite against that build in a
subprocess: the suite has to fail.  Everything happens on the CPU.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lapeig_oracle.c")

MUTANTS = {
    "spmv_wrong_index": ("s += val[p] * x[col[p]];", "s += val[p] * x[i];"),
    "quadform_dropped_half": ("return 0.5 * s;", "return s;"),
    "quadform_wrong_sign": ("s += (-val[p]) * d * d;", "s += (val[p]) * d * d;"),
    "jacobi_rotation_sign": ("A[k * n + q] = s * akp + c * akq;", "A[k * n + q] = -s * akp + c * akq;"),
    "mgs_wrong_sign": ("axpy(n, -dot(n, qj, v), qj, v);", "axpy(n, dot(n, qj, v), qj, v);"),
    "ic0_forward_sign": ("s -= K->val[e] * z[K->col[e]];", "s += K->val[e] * z[K->col[e]];"),
    "ic0_transposed_solve": ("z[K->col[e]] -= K->val[e] * z[i];", "z[i] -= K->val[e] * z[K->col[e]];"),
    "pcg_shift_sign": ("axpy(n, -theta, tmp, s);", "axpy(n, theta, tmp, s);"),
    "pcg_beta_sign": ("p[i] = z[i] + beta * p[i];", "p[i] = z[i] - beta * p[i];"),
    # (dropping the left projection of the operator product is not in this
    # list: the preconditioner's own projections remove those components, so
    # that change leaves the computed correction unchanged)
    "pcg_unprojected_preconditioner": ("prec_apply(P, n, tmp, z);\n        project_out(n, q, Q, z);\n        double rho_new",
                                       "prec_apply(P, n, tmp, z);\n        double rho_new"),
    "jd_border_sign": ("H[m * m_max + i] = h;", "H[m * m_max + i] = -h;"),
    "jd_restart_keeps_largest": ("basis_times(n, m, V, Y, 0, m_min, V2);",
                                 "basis_times(n, m, V, Y, m - m_min, m_min, V2);"),
    "jd_no_deflation_against_locked": ("double vn = orc_mgs(n, nx, X, v);",
                                       "double vn = orc_mgs(n, 0, X, v);"),
    "splitmix_constant": ("0x94d049bb133111ebULL", "0x94d049bb133111ecULL"),
    "fsai_unscaled_row": ("double sc = 1.0 / sqrt(g[iv]);", "double sc = 1.0 / g[iv];"),
    "fsai_missing_shift": ("if (a == b) e *= 1.0 + tau;", "if (a == b) e *= 1.0;"),
    "fsai_no_transpose": ("for (int e = Z->rowptr[v]; e < Z->rowptr[v + 1]; ++e) z[Z->col[e]] += Z->val[e] * y[v];",
                          "for (int e = Z->rowptr[v]; e < Z->rowptr[v + 1]; ++e) z[v] += Z->val[e] * y[Z->col[e]];"),
    "components_merge": ("if (label[j] < 0) { label[j] = ncomp; queue[tail++] = j; }",
                         "if (label[j] < 0) { label[j] = 0; queue[tail++] = j; }"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor missing for {name}"
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "mutant.c"
    csrc.write_text(mutated)
    lib = oracle.build_from(str(csrc), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, LAPEIG_ORACLE_LIB=lib)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           "--timeout", "30", "-k", "not arpack and not weighted_vs_dense",
           os.path.join(ROOT, "tests", "test_oracle_pins.py")]
    proc = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert proc.returncode != 0, f"planted mistake {name} passed every pin:\n{proc.stdout[-2000:]}"
