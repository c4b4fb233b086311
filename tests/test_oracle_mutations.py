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
    ("theta_index", "prod *= corr_factor(fam, diff, theta[k], p);",
     "prod *= corr_factor(fam, diff, theta[0], p);"),
    ("x_index_transposed",
     "fabs((REAL)X[(size_t)i * d + k] - (REAL)X[(size_t)j * d + k]);\n                prod",
     "fabs((REAL)X[(size_t)k * d + i % d] - (REAL)X[(size_t)j * d + k]);\n                prod"),
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
    ("grad_missing_R", "gk += R[(size_t)i * n + j] * G *", "gk += G *"),
    ("back_solve_transposed", "t -= L[(size_t)m * n + i] * w[m];", "t -= L[(size_t)i * n + m] * w[m];"),
    ("pred_mse_term_dropped", "mse[j] = (double)(sigma2 * (1 - rRr + (1 - oRr) * (1 - oRr) / oRo));",
     "mse[j] = (double)(sigma2 * (1 - rRr));"),
    ("pred_mean_without_mu", "REAL m = mu, rRr = 0, oRr = 0;", "REAL m = 0, rRr = 0, oRr = 0;"),
    ("pred_cross_power_ignored", "prod *= corr_factor(fam, diff, th[k], p);",
     "prod *= corr_factor(fam, diff, th[k], (REAL)1);"),
    ("pred_ones_forward_only", "back_solve(n, L, z, one_inv);", "memcpy(one_inv, z, sizeof(REAL) * n);"),
    ("matern_theta_ignored", "REAL h = th * diff;", "REAL h = diff;"),
    ("matern32_constant", "REAL c = sqrt((REAL)3);\n        return (1 + c * h)",
     "REAL c = sqrt((REAL)2);\n        return (1 + c * h)"),
    ("matern52_square_term_dropped", "return (1 + c * h + c * c * h * h / 3) * exp(-c * h);",
     "return (1 + c * h) * exp(-c * h);"),
    ("matern32_grad_factor", "return diff * c * c * h / (1 + c * h);", "return diff * c * h / (1 + c * h);"),
    ("matern52_grad_factor", "return diff * c * c * h * (1 + c * h) / (3 * (1 + c * h + c * c * h * h / 3));",
     "return diff * c * c * h / (3 * (1 + c * h + c * c * h * h / 3));"),
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
