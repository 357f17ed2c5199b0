"""Planted mistakes in the oracles must fail their pins (CPU only).

Each case copies the oracle package to a temporary folder, changes one
expression of oracle.c (interpolation, alpha_s) or mlp.py (surrogate network)
-- a dropped term, a wrong sign, index or operand, a wrong slope rule, a wrong
tie or branch rule -- and runs that file's pin tests (test_oracle_pins.py,
test_mlp_oracle.py) against the copy in a child process.  The pins must catch
every mistake; the unchanged copy must pass them.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = {"oracle.c": os.path.join(ROOT, "tests", "test_oracle_pins.py"),
        "mlp.py": os.path.join(ROOT, "tests", "test_mlp_oracle.py")}

# name -> (text in oracle.c, replacement)
C_MUTATIONS = {
    "hermite_h10_sign": ("double h10 = u * v2;", "double h10 = -u * v2;"),
    "hermite_h11_sign": ("double h11 = -u2 * v;", "double h11 = u2 * v;"),
    "hermite_h01_term": ("double h01 = u2 * (3 - 2 * u);", "double h01 = u2 * (2 - 2 * u);"),
    "hermite_h00_factor": ("double h00 = v2 * (1 + 2 * u);", "double h00 = v2 * (1 + u);"),
    "hermite_drops_width": ("+ h01 * f[(long)(i + 1) * st] + h11 * D * fd_slope(t, f, st, n, i + 1);",
                            "+ h01 * f[(long)(i + 1) * st] + h11 * fd_slope(t, f, st, n, i + 1);"),
    "interior_slope_one_sided": ("return 0.5 * (secant(t, f, st, j - 1) + secant(t, f, st, j));",
                                 "return secant(t, f, st, j);"),
    "end_slope_zero": ("if (j == n - 1) return secant(t, f, st, n - 2);", "if (j == n - 1) return 0.0;"),
    "secant_linear_coordinate": ("/ log(t[j + 1] / t[j]);", "/ (t[j + 1] - t[j]);"),
    "search_tie_to_lower_cell": ("if (t[j] <= v) i = j;", "if (t[j] < v) i = j;"),
    "parameter_missing_ratio": ("return log(v / t[i]) / log(t[i + 1] / t[i]);",
                                "return log(v / t[i]) / log(t[i + 1]);"),
    "threshold_to_lower_subgrid": ("if (g->qk[j][0] <= q2) k = j;", "if (g->qk[j][0] < q2) k = j;"),
    "values_transposed": ("const double* fr = V + (long)r * P + c;\n"
                          "        G[r] = hermite_cell(xk, fr, (long)nq * P, nx, ix, ux);",
                          "const double* fr = V + (long)r * nx * P + c;\n"
                          "        G[r] = hermite_cell(xk, fr, (long)P, nx, ix, ux);"),
    "lowx_parameter_sign": ("double s = log(x / xk[0]) / log(xk[1] / xk[0]);",
                            "double s = log(xk[0] / x) / log(xk[1] / xk[0]);"),
    "lowx_linear_branch_sign": ("r.v = loglin ? f0.v * pow(f1.v / f0.v, s) : f0.v + s * (f1.v - f0.v);",
                                "r.v = loglin ? f0.v * pow(f1.v / f0.v, s) : f0.v + s * (f0.v - f1.v);"),
    "highq_anchor_at_lower_knot": ("r.v = loglin ? f1.v * pow(f1.v / f0.v, s) : f1.v + s * (f1.v - f0.v);",
                                   "r.v = loglin ? f0.v * pow(f1.v / f0.v, s) : f0.v + s * (f1.v - f0.v);"),
    "highq_parameter_wrong_knot": ("double s = log(q2 / qk[nq - 1]) / log(qk[nq - 1] / qk[nq - 2]);",
                                   "double s = log(q2 / qk[nq - 2]) / log(qk[nq - 1] / qk[nq - 2]);"),
    "lowq_exponent_sign": ("out.v = f0.v * pow(r, gamma * r + 1.0 - r);",
                           "out.v = f0.v * pow(r, gamma * r + 1.0 + r);"),
    "lowq_gamma_inverted": ("double gamma = log(f1.v / f0.v) / L01;", "double gamma = log(f0.v / f1.v) / L01;"),
    "lowq_ignores_high_x_rule": ("&& x <= X_HIGH);", ");"),
    "invalid_x_above_xmax_accepted": ("|| !(q2 > 0.0) || x > xmax) return REG_INVALID;",
                                      "|| !(q2 > 0.0)) return REG_INVALID;"),
    "gluon_alias_dropped": ("if (pid == 0) pid = 21;", ""),
    "scale_sums_stencil": ("if (m > M) M = m;", "M += m;"),
    "scale_drops_continuation_weights": ("return fabs(e0) * f0.s + fabs(e1) * f1.s;", "return f0.s + f1.s;"),
    "alphas_upper_constant_wrong": ("if (v > q2k[nk - 1]) { out[i] = a[nk - 1]; continue; }",
                                    "if (v > q2k[nk - 1]) { out[i] = a[nk - 2]; continue; }"),
    "alphas_threshold_to_lower_segment": ("if (q2k[j] == q2k[j - 1] && q2k[j] <= v) s0 = j;",
                                          "if (q2k[j] == q2k[j - 1] && q2k[j] < v) s0 = j;"),
}

# name -> (text in mlp.py, replacement)
MLP_MUTATIONS = {
    "mlp_tanh_derivative": ("dz = dh * (1.0 - h3 * h3)", "dz = dh * (1.0 - h3)"),
    "mlp_loss_normalisation": ("dy = 2.0 * d / (B * O)", "dy = 2.0 * d / B"),
    "mlp_bias_gradient_mean": ('g["b4"] = dy.sum(0)', 'g["b4"] = dy.mean(0)'),
    "mlp_wrong_layer_input": ('g["W2"] = dzr.T @ a1', 'g["W2"] = dzr.T @ a2'),
    "mlp_transposed_backprop": ('dh = dzr @ hi(W["W3"])', 'dh = dzr @ hi(W["W3"].T)'),
    "split_drops_lo_activation": ("return ah @ Wh.T + al @ Wh.T + ah @ Wl.T", "return ah @ Wh.T + ah @ Wl.T"),
    "split_lo_not_residual": ("return hi, bf16(a - hi)", "return hi, bf16(a)"),
    "mlp_first_layer_bias_missing": ('z1 = x @ W["W1"].T + P["b1"]', 'z1 = x @ W["W1"].T'),
    "bf16_ties_away_from_zero": ("r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16",
                                 "r = ((u + 0x8000) >> 16) << 16"),
    "adam_no_bias_correction": ("m_hat = m / (1.0 - b1 ** t)", "m_hat = m"),
    "adam_eps_inside_sqrt": ("lr * m_hat / (np.sqrt(v_hat) + eps)", "lr * m_hat / np.sqrt(v_hat + eps)"),
    "adam_second_moment_of_abs": ("v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g",
                                  "v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * np.abs(g)"),
    "cosine_schedule_reversed": ("(1.0 + math.cos(math.pi * frac))", "(1.0 - math.cos(math.pi * frac))"),
    "train_schedule_off_by_one": ("cosine_lr(t, lr0, lr_final, total), t + 1)",
                                  "cosine_lr(t + 1, lr0, lr_final, total), t + 1)"),
}

MUTATIONS = {k: ("oracle.c",) + v for k, v in C_MUTATIONS.items()}
MUTATIONS.update({k: ("mlp.py",) + v for k, v in MLP_MUTATIONS.items()})


def planted_copy(tmp_path, mutation):
    dst = tmp_path / "oracle"
    os.makedirs(dst)
    for f in ("__init__.py", "oracle.c", "mlp.py", "fk.py"):
        shutil.copy(os.path.join(ROOT, "oracle", f), dst / f)
    if mutation is not None:
        fname, old, new = MUTATIONS[mutation]
        src = (dst / fname).read_text()
        assert src.count(old) == 1, "mutation text not found once in %s: %r" % (fname, old)
        (dst / fname).write_text(src.replace(old, new))
    # compile here, so a planted change that does not build is an error of this test, not a catch
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                           "-o", str(dst / "liboracle.so"), str(dst / "oracle.c"), "-lm"])
    return tmp_path


def run_pins(folder, pins):
    env = dict(os.environ)
    env["PYTHONPATH"] = os.pathsep.join([str(folder), ROOT])
    p = subprocess.run([sys.executable, "-m", "pytest", pins, "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=str(folder), env=env, capture_output=True, text=True, timeout=600)
    return p.returncode, p.stdout + p.stderr


def test_unchanged_copy_passes_pins(tmp_path):
    folder = planted_copy(tmp_path, None)
    for pins in PINS.values():
        rc, log = run_pins(folder, pins)
        assert rc == 0, log[-3000:]
    assert str(tmp_path) in subprocess.run(
        [sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=str(tmp_path),
        env=dict(os.environ, PYTHONPATH=os.pathsep.join([str(tmp_path), ROOT])),
        capture_output=True, text=True).stdout


@pytest.mark.parametrize("mutation", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path, mutation):
    rc, log = run_pins(planted_copy(tmp_path, mutation), PINS[MUTATIONS[mutation][0]])
    assert rc == 1, "pins did not catch %s (exit %d):\n%s" % (mutation, rc, log[-3000:])
