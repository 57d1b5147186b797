"""The oracle's pins catch plausible mistakes (CPU): each mutant below plants
one mistake in a copy of the C oracle (a wrong sign, index, weight, side
rule, colour order or grid spacing), the copy is compiled and swapped in, and
at least one pin of tests/test_oracle_pins.py must fail on it.  The Python
parts of the oracle get the same treatment: a mistake planted in a copy of
oracle/exact.py (the array-form operator) or oracle/net.py (the network's
emulated roundings) must fail one of the checks of test_oracle_exact.py or
test_oracle_net_rounding.py run on that copy."""
import importlib.util
import os
import shutil
import subprocess
import types

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.dirname(oracle.__file__)


def _pins():
    spec = importlib.util.spec_from_file_location("oracle_pins", os.path.join(HERE, "test_oracle_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


P = _pins()


def _cn_pins():
    spec = importlib.util.spec_from_file_location("oracle_cn_pins", os.path.join(HERE, "test_oracle_cn.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


C = _cn_pins()


def _bc_pins():
    spec = importlib.util.spec_from_file_location("oracle_bc_pins", os.path.join(HERE, "test_oracle_bc.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


B = _bc_pins()


def _projection_pins():
    spec = importlib.util.spec_from_file_location("oracle_projection_pins",
                                                  os.path.join(HERE, "test_oracle_projection.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


J = _projection_pins()


def _bottom_pins():
    spec = importlib.util.spec_from_file_location("oracle_bottom_pins", os.path.join(HERE, "test_oracle_bottom.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


Q = _bottom_pins()


def _load_test_module(name, fname):
    spec = importlib.util.spec_from_file_location(name, os.path.join(HERE, fname))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


X = _load_test_module("oracle_exact_pins", "test_oracle_exact.py")
G = _load_test_module("oracle_fmg_pins", "test_oracle_fmg.py")
R = _load_test_module("oracle_net_rounding_pins", "test_oracle_net_rounding.py")

# name -> (text in mg_oracle.c, replacement); each text occurs exactly once
MUTANTS = {
    "relaxation_sign": ("(f[IDX(n, i, j)] + c * nb) / diag", "(f[IDX(n, i, j)] - c * nb) / diag"),
    "dirichlet_ghost_sign": ("(bc[OG_XLO] == OG_DIRICHLET ? -lo : lo)", "(bc[OG_XLO] == OG_DIRICHLET ? lo : lo)"),
    "neumann_ghost_sign": ("(bc[OG_YHI] == OG_DIRICHLET ? -hi : hi)", "(bc[OG_YHI] == OG_DIRICHLET ? -hi : -hi)"),
    "periodic_wrap_side": ("bc[OG_YHI] == OG_PERIODIC ? lo :", "bc[OG_YHI] == OG_PERIODIC ? hi :"),
    "residual_dropped_term": (" + (phi[IDX(n, i, j - 1)] - p)) * ih2;\n            r[IDX(n, i, j)]",
                              ") * ih2;\n            r[IDX(n, i, j)]"),
    "residual_sign": ("f[IDX(n, i, j)] - (alpha * p - beta * lap)", "f[IDX(n, i, j)] - (alpha * p + beta * lap)"),
    "restriction_weight": ("0.25 * (fine[IDX(n, 2 * I, 2 * J)]", "0.5 * (fine[IDX(n, 2 * I, 2 * J)]"),
    "restriction_index": ("fine[IDX(n, 2 * I + 1, 2 * J + 1)]", "fine[IDX(n, 2 * I + 1, 2 * J)]"),
    "prolongation_slope_sign": ("double dx = a ? 0.25 : -0.25", "double dx = a ? -0.25 : 0.25"),
    "prolongation_slope_axis": ("0.5 * (coarse[IDX(nc, I + 1, J)] - coarse[IDX(nc, I - 1, J)])",
                                "0.5 * (coarse[IDX(nc, I, J + 1)] - coarse[IDX(nc, I, J - 1)])"),
    "coarse_spacing": ("double h = p->h * (double)(1 << lev);", "double h = p->h;"),
    "colour_order": ("relax_colour(n, h, alpha, beta, bc, phi, f, 0); /* red   */",
                     "relax_colour(n, h, alpha, beta, bc, phi, f, 1); /* red   */"),
    "cn_rhs_sign": ("f[IDX(n, i, j)] = p + beta * lap;", "f[IDX(n, i, j)] = p - beta * lap;"),
    "cn_rhs_half_step": ("f[IDX(n, i, j)] = p + beta * lap;", "f[IDX(n, i, j)] = p + 2.0 * beta * lap;"),
    "dirichlet_data_factor": ("if (bc[OG_XLO] == OG_DIRICHLET) a[IDX(n, -1, j)] += 2.0 * vl;",
                              "if (bc[OG_XLO] == OG_DIRICHLET) a[IDX(n, -1, j)] += vl;"),
    "neumann_data_sign": ("if (bc[OG_XLO] == OG_NEUMANN) a[IDX(n, -1, j)] -= h * vl;",
                          "if (bc[OG_XLO] == OG_NEUMANN) a[IDX(n, -1, j)] += h * vl;"),
    "divergence_axis": ("(vv[IDX(n, i, j + 1)] - vv[IDX(n, i, j - 1)]) * i2h;",
                        "(vv[IDX(n, i + 1, j)] - vv[IDX(n, i - 1, j)]) * i2h;"),
    "projection_gradient_sign": ("u[IDX(n, i, j)] -= (phi[IDX(n, i + 1, j)] - phi[IDX(n, i - 1, j)]) * i2h;",
                                 "u[IDX(n, i, j)] += (phi[IDX(n, i + 1, j)] - phi[IDX(n, i - 1, j)]) * i2h;"),
    "direct_dirichlet_side": ("row[k] += c; /* ghost = -cell */", "row[k] -= c; /* ghost = -cell */"),
    "direct_periodic_as_neumann": ("row[((jj + n) % n) * n + (ii + n) % n] -= c;", "row[k] -= c;"),
    "direct_singular_shift_sign": ("for (int q = 0; q < m; ++q) row[q] += c;",
                                   "for (int q = 0; q < m; ++q) row[q] += (q == k ? c : 0.0);"),
    "direct_back_substitution": ("s -= A[(size_t)k * w + q] * A[(size_t)q * w + m];",
                                 "s -= A[(size_t)k * w + q] * A[(size_t)k * w + m];"),
    # FMG: each level starts from zero instead of the prolongated coarse phi
    "fmg_skips_prolongation": ("og_prolong_add(p->n >> (l + 1), p->bc, P[l + 1], P[l]);\n        for (int k",
                               "(void)0;\n        for (int k"),
    # FMG: every level's f restricted from the finest array with the wrong size
    "fmg_restricts_wrong_level": ("og_restrict(p->n >> (l - 1), F[l - 1], F[l]);",
                                  "og_restrict(p->n >> (l - 1), F[0], F[l]);"),
    # FMG: the coarse phi added to the finer level twice
    "fmg_prolongation_doubled": ("og_prolong_add(p->n >> (l + 1), p->bc, P[l + 1], P[l]);\n        for (int k",
                                 "og_prolong_add(p->n >> (l + 1), p->bc, P[l + 1], P[l]);\n"
                                 "        og_prolong_add(p->n >> (l + 1), p->bc, P[l + 1], P[l]);\n        for (int k"),
}
# Not a mutant: dropping the removal of each restricted right-hand side's mean
# (singular problems) changes the iterates only by rounding -- the residual of
# a compatible periodic problem has zero sum and restriction keeps sums, so the
# removal only stops rounding drift (checked: 3e-16 relative at 64^2 and 256^2).

# a compact set of pins (each a call with fixed arguments)
BATTERY = [
    (P.test_mg_converges_to_dense_solution, ("DDDD", (0.0, -1.0), 8)),
    (P.test_mg_converges_to_dense_solution, ("NNNN", (0.0, -1.0), 8)),
    (P.test_mg_converges_to_dense_solution, ("PPPP", (0.0, -1.0), 8)),
    (P.test_mg_converges_to_dense_solution, ("DNPP", (1.0, 0.5 / 64), 8)),
    (P.test_mg_converges_to_dense_solution, ("PPND", (0.0, -1.0), 8)),
    (P.test_smoother_black_residual_zero, ("DNPP",)),
    (P.test_restriction_conserves_and_keeps_constants, ()),
    (P.test_prolongation_constants_and_linears, ()),
    (P.test_residual_matches_assembled_matrix, ()),
    (P.test_vcycle_convergence_factor_h_independent, ("PPPP",)),
    (P.test_vcycle_convergence_factor_h_independent, ("DDDD",)),
    (P.test_mg_matches_transform_solution_n128, ("PPPP",)),
    (C.test_cn_step_multiplies_an_eigenmode_by_the_closed_form_factor, ("NNNN", 2.0)),
    (B.test_side_data_solve_matches_the_extended_dense_system, ("DNND", (0.0, -1.0))),
    (B.test_side_data_solve_matches_the_extended_dense_system, ("NDDN", (1.0, 0.02))),
    (J.test_discrete_curl_is_left_unchanged, ()),
    (J.test_gradient_of_a_mode_in_closed_form, ()),
    (Q.test_direct_bottom_on_the_top_level_is_the_dense_solution, ("DNPP", (1.0, 0.5 / 64), 8)),
    (Q.test_direct_bottom_on_the_top_level_is_the_dense_solution, ("PPPP", (0.0, -1.0), 4)),
    (Q.test_direct_bottom_on_the_top_level_is_the_dense_solution, ("NDDN", (0.0, -1.0), 8)),
    (G.test_fmg_reaches_discretization_accuracy, (64,)),
    (G.test_fmg_with_many_cycles_is_the_discrete_solution, ("NDDN", (0.0, -1.0))),
    (G.test_fmg_is_linear_in_f, ()),
]


def _build(src_text: str, out_dir: str) -> str:
    shutil.copy(os.path.join(ORACLE_DIR, "mg_oracle.h"), out_dir)
    src = os.path.join(out_dir, "mg_oracle.c")
    with open(src, "w") as fh:
        fh.write(src_text)
    lib = os.path.join(out_dir, "libmutant.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", lib,
                    src, "-lm"], check=True, cwd=out_dir, capture_output=True)
    return lib


def _failures(monkeypatch, lib_path):
    monkeypatch.setattr(oracle, "_lib_handle", oracle._load(lib_path))
    failed = []
    for fn, args in BATTERY:
        try:
            with np.errstate(all="ignore"):  # mutants may produce NaN histories
                fn(*args)
        except Exception:  # an assertion, or a solve that stopped with an error
            failed.append(f"{fn.__name__}{args}")
    return failed


def test_unmutated_copy_passes_the_battery(tmp_path, monkeypatch):
    src = open(os.path.join(ORACLE_DIR, "mg_oracle.c")).read()
    assert _failures(monkeypatch, _build(src, str(tmp_path))) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "mg_oracle.c")).read()
    assert src.count(old) == 1, name
    failed = _failures(monkeypatch, _build(src.replace(old, new), str(tmp_path)))
    assert failed, f"no pin caught the mutant {name}"


# ---- mistakes planted in the Python parts of the oracle
# name -> (file under oracle/, text, replacement, checks run on the mutated module)
EXACT_BATTERY = [
    lambda E: X.check_apply_operator_equals_assembled(E, "DNPP", (0.0, -1.0)),
    lambda E: X.check_apply_operator_equals_assembled(E, "PPDN", (1.0, 0.37)),
    lambda E: X.check_relative_residual_equals_assembled(E, "NDDD", (0.0, -1.0)),
    lambda E: X.check_residual_equals_c_oracle(E, "DDNN", (1.0, 0.37)),
    lambda E: X.check_exact_solutions_have_rounding_residual(E),
]
NET_BATTERY = [
    lambda N: R.check_worked_example(N),
    lambda N: R.check_worked_example_unrounded(N),
    lambda N: R.check_bound(N, 0, True),
    lambda N: R.check_bound(N, 1, False),
]
PY_MUTANTS = {
    # the last layer's weight gradient from the activations' hi part only
    "net_backward_drops_pair_lo": ("net.py", "grads[5] = conv_w(g, a[5], DIL[5])",
                                   "grads[5] = conv_w(g, hi[5], DIL[5])", NET_BATTERY),
    # the back-propagated gradient rounded before the adjoint convolution, not after
    "net_backward_rounding_moved": ("net.py", "        g = r(conv_t(g, ws[l], DIL[l]))",
                                    "        g = conv_t(r(g), ws[l], DIL[l])", NET_BATTERY),
    # the output gradient left unrounded
    "net_output_gradient_unrounded": ("net.py", "g = r(2.0 * (y - t) / n)[..., None]",
                                      "g = (2.0 * (y - t) / n)[..., None]", NET_BATTERY),
    # activations between layers carried as one bfloat16 (the lo part dropped)
    "net_forward_drops_activation_lo": ("net.py", "a.append(h + bf16(v - h))", "a.append(h)", NET_BATTERY),
    # Dirichlet ghost with the Neumann sign in the array-form operator
    "exact_operator_dirichlet_sign": ("exact.py", "g[sl_ghost] = -g[sl_in]", "g[sl_ghost] = g[sl_in]",
                                      EXACT_BATTERY),
    # periodic ghost copied from the adjacent cell instead of the opposite side
    "exact_operator_periodic_side": ("exact.py", "g[sl_ghost] = g[sl_opp]", "g[sl_ghost] = g[sl_in]",
                                     EXACT_BATTERY),
}


def _py_mutant(fname, old, new):
    """A copy of oracle/<fname> with `old` replaced by `new`, loaded as a
    module of the oracle package (its relative imports resolve there)."""
    src = open(os.path.join(ORACLE_DIR, fname)).read()
    assert src.count(old) == 1, (fname, old)
    mod = types.ModuleType("oracle._mutant_" + fname[:-3])
    mod.__package__ = "oracle"
    mod.__file__ = os.path.join(ORACLE_DIR, fname)
    exec(compile(src.replace(old, new), mod.__file__, "exec"), mod.__dict__)
    return mod


def _py_failures(mod, battery):
    failed = 0
    for check in battery:
        try:
            with np.errstate(all="ignore"):
                check(mod)
        except Exception:
            failed += 1
    return failed


@pytest.mark.parametrize("fname,battery", [("exact.py", EXACT_BATTERY), ("net.py", NET_BATTERY)])
def test_unmutated_python_copies_pass_their_battery(fname, battery):
    assert _py_failures(_py_mutant(fname, "import numpy as np", "import numpy as np"), battery) == 0


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_pins_catch_python_mutant(name):
    fname, old, new, battery = PY_MUTANTS[name]
    assert _py_failures(_py_mutant(fname, old, new), battery) > 0, f"no pin caught the mutant {name}"
