"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins in test_oracle_pins.py catch every one of them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gp_oracle.c")

# (name, original text, mutated text)
MUTATIONS = [
    ("nugget_dropped", "R[(size_t)i * n + i] = (REAL)1 + delta;", "R[(size_t)i * n + i] = (REAL)1;"),
    ("power_ignored", "pow(diff, p)", "(diff * diff)"),
    ("theta_index", "prod *= exp(-theta[k] * pw);", "prod *= exp(-theta[0] * pw);"),
    ("x_index_transposed", "fabs((REAL)X[(size_t)i * d + k] - (REAL)X[(size_t)j * d + k]);\n                REAL pw",
     "fabs((REAL)X[(size_t)k * d + i % d] - (REAL)X[(size_t)j * d + k]);\n                REAL pw"),
    ("chol_sign", "for (int m = 0; m < j; ++m) s -= rj[m] * rj[m];", "for (int m = 0; m < j; ++m) s += rj[m] * rj[m];"),
    ("chol_offdiag_index", "for (int m = 0; m < j; ++m) t -= ri[m] * rj[m];", "for (int m = 0; m < j; ++m) t -= ri[m] * rj[m + 1];"),
    ("chol_no_divide", "ri[j] = t / ljj;", "ri[j] = t;"),
    ("logdet_not_doubled", "logdet *= 2;", "logdet *= 1;"),
    ("fwd_solve_sign", "for (int m = 0; m < i; ++m) t -= ri[m] * z[m];", "for (int m = 0; m < i; ++m) t += ri[m] * z[m];"),
    ("mu_inverted", "REAL mu = ab / aa;", "REAL mu = aa / ab;"),
    ("one_pass_dropped_mu", "REAL r = b[i] - mu * a[i];", "REAL r = b[i] - a[i];"),
    ("sigma_not_over_n", "REAL sigma2 = Q / (REAL)n;", "REAL sigma2 = Q;"),
    ("nll_missing_n", "REAL nll = logdet + (REAL)n * log(sigma2);", "REAL nll = logdet + log(sigma2);"),
    ("grad_sign", "((REAL)n / Q * alpha[i] * alpha[j] - Ri[(size_t)i * n + j]);",
     "((REAL)n / Q * alpha[i] * alpha[j] + Ri[(size_t)i * n + j]);"),
    ("grad_missing_R", "gk += R[(size_t)i * n + j] * D *", "gk += D *"),
    ("back_solve_transposed", "t -= L[(size_t)m * n + i] * w[m];", "t -= L[(size_t)i * n + m] * w[m];"),
    ("pred_mse_term_dropped", "mse[j] = (double)(sigma2 * (1 - rRr + (1 - oRr) * (1 - oRr) / oRo));",
     "mse[j] = (double)(sigma2 * (1 - rRr));"),
    ("pred_mean_without_mu", "REAL m = mu, rRr = 0, oRr = 0;", "REAL m = 0, rRr = 0, oRr = 0;"),
    ("pred_cross_power_ignored", "REAL pw = (diff == 0) ? (REAL)0 : pow(diff, p);\n                prod *= exp(-th[k] * pw);",
     "REAL pw = diff;\n                prod *= exp(-th[k] * pw);"),
    ("pred_ones_forward_only", "back_solve(n, L, z, one_inv);", "memcpy(one_inv, z, sizeof(REAL) * n);"),
]


@pytest.mark.parametrize("name,orig,mut", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, orig, mut):
    src = open(SRC).read()
    assert src.count(orig) >= 1, f"mutation anchor not found: {name}"
    msrc = tmp_path / "gp_oracle.c"
    msrc.write_text(src.replace(orig, mut, 1))
    objs = []
    for real, sfx in (("double", "f64"), ("long double", "f80")):
        obj = str(tmp_path / f"o_{sfx}.o")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-c", str(msrc), "-o", obj,
                               f"-DREAL={real}", f"-DSFX(name)=name##_{sfx}"])
        objs.append(obj)
    lib = str(tmp_path / "liboracle.so")
    subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", lib] + objs + ["-lm"])
    env = dict(os.environ, GP_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} was not caught by any pin"
