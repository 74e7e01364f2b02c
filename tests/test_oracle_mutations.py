"""The oracle pins must catch plausible mistakes: each case plants one mistake
in a copy of the oracle's C source (on the CPU only), rebuilds the copy and
runs the pin suite against it, which has to fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "operator_diagonal": ("out[idx] = (2.0 * dim * centre - nb) * inv_h2;",
                          "out[idx] = (2.0 * dim * centre + nb) * inv_h2;"),
    "operator_h_scale": ("double inv_h2 = 1.0 / (h * h);", "double inv_h2 = 1.0 / h;"),
    "jacobi_damping": ("out[p] = c[p] + omega * r[p] / diag;", "out[p] = c[p] + r[p] / diag;"),
    "restrict_weights": ("const double w[3] = {0.25 * g, 0.5 * g, 0.25 * g};",
                         "const double w[3] = {0.25 * g, 0.25 * g, 0.5 * g};"),
    "restrict_offset": ("int fi = 2 * I + ox, fj = 2 * J + oy", "int fi = 2 * I + ox + 1, fj = 2 * J + oy"),
    "prolong_weight": ("if (d == 1 || d == -1) return 0.5;", "if (d == 1 || d == -1) return 0.25;"),
    "coarse_correction_sign": ("for (long p = 0; p < N; p++) c[p] += tmp[p];",
                               "for (long p = 0; p < N; p++) c[p] -= tmp[p];"),
    "base_solve": ("c[0] = b[0] / ref_diag(dim, n, disc);", "c[0] = b[0] / (2.0 * ref_diag(dim, n, disc));"),
    "fd_diag": ("return 2.0 * dim / (h * h);", "return 2.0 * dim / h;"),
    "q1_element_mass": ("const double m1[2][2] = {{h / 3.0, h / 6.0}, {h / 6.0, h / 3.0}};",
                        "const double m1[2][2] = {{h / 3.0, h / 4.0}, {h / 4.0, h / 3.0}};"),
    "q1_restrict_scale": ("const double g = disc == REF_DISC_Q1 ? 2.0 : 1.0;",
                          "const double g = disc == REF_DISC_Q1 ? 1.0 : 1.0;"),
    "q1_diag": ("* dim * pow(h, dim - 2) / pow(3.0, dim - 1);", "* dim * pow(h, dim - 2) / pow(3.0, dim);"),
    "q1_cell_range": ("for (int cx = 0; cx <= n; cx++)", "for (int cx = 0; cx < n; cx++)"),
    "chain_stops_early": ("while (n > n_base) {", "while (n > n_base + 1) {"),
    "no_post_smoothing": ("for (int s = 0; s < nu2; s++) {             /* post-smooth */",
                          "for (int s = 0; s < 0; s++) {             /* post-smooth */"),
    "scaling_not_compensated": ("u[p] += alpha * c[p];", "u[p] += c[p];"),
    "recursive_residual_sign": ("r[p] -= alpha * ac[p];", "r[p] += alpha * ac[p];"),
    "norm_without_sqrt": ("return sqrt(ref_sumsq(v, N));", "return ref_sumsq(v, N);"),
    "norm_pairwise_drops_entry": ("return ref_sumsq(v, m) + ref_sumsq(v + m, N - m);",
                                  "return ref_sumsq(v, m) + ref_sumsq(v + m, N - m - 1);"),
    "norminf_without_abs": ("double a = fabs(v[p]);", "double a = v[p];"),
    "initial_guess_ignored": ("if (!o->use_initial_guess) memset(u, 0, sizeof(double) * N);",
                              "memset(u, 0, sizeof(double) * N);"),
    "initial_residual_from_b": ("    ref_residual_d(dim, n, disc, b, u, r);\n    int st = REF_OK;",
                                "    memcpy(r, b, sizeof(double) * N);\n    int st = REF_OK;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTATIONS[name]
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = (dst / "mg_ref.c").read_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    (dst / "mg_ref.c").write_text(src.replace(old, new))
    env = dict(os.environ, MGREF_ORACLE_DIR=str(dst))
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                           os.path.join(ROOT, "tests", "test_oracle_q1.py")],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert proc.returncode != 0, f"pins did not catch mutation {name}:\n{proc.stdout[-2000:]}"
