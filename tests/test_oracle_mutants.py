"""The pins catch plausible mistakes in the oracle.

Each mutant is a copy of `oracle/se2_oracle.c` with one deliberate mistake of the
kind a careful reader could still make (a dropped term, a wrong sign, a swapped
index, a transposed operand, a wrong weight).  The copy is built with gcc into a
temporary directory on the CPU, swapped in for the real oracle build, and the pins
of `pins.py` are run against it: at least one of them must fail.  The real oracle
is restored afterwards and still passes every pin (`test_oracle_pins.py`).
"""
from __future__ import annotations

import contextlib
import inspect
import os
import subprocess

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "se2_oracle.c")

# (name, text in se2_oracle.c, replacement, occurrence to replace (0 = first))
MUTANTS = [
    # Section 4.3, eq. (logcomp): half-angle coordinates
    ("b2_sign", "b[1] = -x * s + y * c;", "b[1] = x * s + y * c;", 0),
    ("full_angle_not_half", "double c = cos(0.5 * t), s = sin(0.5 * t);", "double c = cos(t), s = sin(t);", 0),
    ("no_small_angle_wrap", "double t = wrap_angle(theta);", "double t = theta;", 0),
    # Section 4.3, eq. (rhob): weighted sum of squares
    ("w3_term_dropped", " + (w3 * b[2]) * (w3 * b[2])", "", 0),
    ("w1_w2_swapped", "(w1 * b[0]) * (w1 * b[0]) + (w2 * b[1]) * (w2 * b[1])",
     "(w2 * b[0]) * (w2 * b[0]) + (w1 * b[1]) * (w1 * b[1])", 0),
    # Section 2.3: h^-1 g = (R_{-theta_h}(x_g - x_h), theta_g - theta_h)
    ("rotation_by_plus_theta", "out[0] = c * dx + s * dy;\n    out[1] = -s * dx + c * dy;",
     "out[0] = c * dx - s * dy;\n    out[1] = s * dx + c * dy;", 0),
    ("angle_difference_reversed", "out[2] = tg - th;", "out[2] = th - tg;", 0),
    ("rotation_by_output_angle", "rel_element((double)dx, (double)dy, th_i, th_o, r);",
     "rel_element((double)dx, (double)dy, th_o, th_o, r);", 0),
    # axial grids: the smaller of the two lifts
    ("axial_min_dropped", "if (d2b < d2) d2 = d2b;", "(void)d2b;", 0),
    # Gibbs kernel K = exp(-rho^2/eps)
    ("kernel_half_eps", "if (logk) logk[idx] = -d2 / eps;", "if (logk) logk[idx] = -d2 / (2.0 * eps);", 0),
    # Section 4.2: (K * f)(g) = sum_h K(h^-1 g) f(h) over the window, log form
    ("conv_dx_dy_transposed", "const double *kr = logk + ((((size_t)(dy + R) * W + (dx + R)) * nt + ko) * nt);",
     "const double *kr = logk + ((((size_t)(dx + R) * W + (dy + R)) * nt + ko) * nt);", 0),
    ("conv_offset_sign", "int jy = iy - dy;", "int jy = iy + dy;", 0),
    # (swapping ko and ki in the table alone is no mistake: negating the offset only flips
    #  the signs of b1 and b2, so the table is symmetric in (ko, ki) at every offset)
    ("conv_input_at_output_orientation", "for (int ki = 0; ki < nt; ++ki) t[n++] = kr[ki] + fr[ki];",
     "for (int ki = 0; ki < nt; ++ki) t[n++] = kr[ki] + fr[ko];", 0),
    ("conv_window_misses_last_row", "for (int dy = -R; dy <= R; ++dy) {\n                        int jy = iy - dy;",
     "for (int dy = -R; dy < R; ++dy) {\n                        int jy = iy - dy;", 0),
    ("lse_shift_lost", "return m + log(s);", "return log(s);", 0),
    ("linear_conv_missing_exp", "s += exp(kr[ki]) * fr[ki];", "s += kr[ki] * fr[ki];", 0),
    # Section 4.1: a = mu / K b, b = nu / K^T a
    ("b_update_uses_mu", "scaling_update(n, lognu, c, psi);", "scaling_update(n, logmu, c, psi);", 0),
    ("a_update_reads_old_psi", "oc_conv_log(nx, ny, nt, R, logk, psi, c);\n        scaling_update(n, logmu, c, phi_next);",
     "oc_conv_log(nx, ny, nt, R, logk, phi, c);\n        scaling_update(n, logmu, c, phi_next);", 0),
    ("marginal_gap_unweighted", "e += exp(logmu[i]) * fabs(expm1(p_old[i] - p_new[i]));",
     "e += fabs(expm1(p_old[i] - p_new[i]));", 0),
    # Appendix A: barycenter = prod_i d_i^lambda_i, v_i <- v_i * bar / d_i
    ("ibp_equal_weights", "logbar[i] += lambdas[m] * ld[n * m + i];", "logbar[i] += ld[n * m + i] / nmeas;", 0),
    ("ibp_v_update_sign", "else lv[n * m + i] += logbar[i] - ld[n * m + i];",
     "else lv[n * m + i] += ld[n * m + i] - logbar[i];", 0),
    ("ibp_d_without_v", "ld[n * m + i] = (v == -INFINITY || c[i] == -INFINITY) ? -INFINITY : v + c[i];",
     "ld[n * m + i] = (v == -INFINITY || c[i] == -INFINITY) ? -INFINITY : c[i];", 0),
    # Section 2.2 / 4.1: cost sum pi rho^2 and the plan's marginals
    ("cost_with_log_kernel", "if (cost_tab) rc += p * cost_tab[kb + ki];", "if (cost_tab) rc += p * (-logk[kb + ki]);", 0),
    ("plan_without_psi", "double p = exp(phi[xo] + logk[kb + ki] + psi[yb + ki]);",
     "double p = exp(phi[xo] + logk[kb + ki]);", 0),
    ("cost_without_plan_weight", "if (cost_tab) rc += p * cost_tab[kb + ki];", "if (cost_tab) rc += cost_tab[kb + ki];", 0),
    ("second_marginal_offset_sign", "int iy = jy + dy;", "int iy = jy - dy;", 0),
    # the plan-difference checker: both plans from their own potentials
    ("plan_l1_returns_zero", "    return tot;\n}", "    return 0.0 * tot;\n}", 0),
    ("plan_l1_b_from_phi_a", "double pb = exp(phi_b[xo] + logk[kb + ki] + psi_b[yb + ki]);",
     "double pb = exp(phi_a[xo] + logk[kb + ki] + psi_b[yb + ki]);", 0),
    ("plan_l1_b_from_psi_a", "double pb = exp(phi_b[xo] + logk[kb + ki] + psi_b[yb + ki]);",
     "double pb = exp(phi_b[xo] + logk[kb + ki] + psi_a[yb + ki]);", 0),
    ("plan_l1_b_from_a", "double pb = exp(phi_b[xo] + logk[kb + ki] + psi_b[yb + ki]);",
     "double pb = exp(phi_a[xo] + logk[kb + ki] + psi_a[yb + ki]);", 0),
    ("plan_l1_signed", "tot += fabs(pa - pb);", "tot += pa - pb;", 0),
]


def _mutate(src: str, old: str, new: str, occurrence: int) -> str:
    pos = -1
    for _ in range(occurrence + 1):
        pos = src.find(old, pos + 1)
        assert pos >= 0, f"mutation site not found: {old!r}"
    return src[:pos] + new + src[pos + len(old):]


@contextlib.contextmanager
def _oracle_build(path: str):
    saved = oracle._lib
    oracle._lib = oracle.load_library(path)
    try:
        yield
    finally:
        oracle._lib = saved


def _first_failing_pin():
    for pin in pins.ALL_PINS:
        try:
            pin()
        except Exception:          # an assertion, or a mutant that breaks a run outright
            return pin.__name__
    return None


def test_mutation_sites_are_unique_enough():
    src = open(SRC).read()
    for name, old, _, occ in MUTANTS:
        assert src.count(old) >= occ + 1, name


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new, occ):
    src = open(SRC).read()
    mutated = _mutate(src, old, new, occ)
    assert mutated != src
    csrc = tmp_path / f"mut_{name}.c"
    csrc.write_text(mutated)
    so = tmp_path / f"libmut_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(csrc), "-lm"])
    with _oracle_build(str(so)):
        caught = _first_failing_pin()
    assert caught is not None, f"no pin fails for the mutant {name}"


# Mistakes in the Python half of the oracle (the JKO step, the porous-medium energy, the
# lift and projection, the split of a signed score, eps-scaling): (name, function of
# `oracle`, text in its source, replacement).  The mutated function is compiled in the
# oracle module's namespace and swapped in for the original while the pins run.
PY_MUTANTS = [
    # Section 5.4: the prox condition log q + c q^(m-1) = log p
    ("prox_wrong_power", "porous_prox_log", "c * np.exp((m - 1.0) * mid)", "c * np.exp(m * mid)"),
    ("prox_c_without_m_factor", "porous_c", "(tau / eps) * m / (m - 1.0) * ref ** (1.0 - m)",
     "(tau / eps) * ref ** (1.0 - m)"),
    # b = prox(K^T a) / K^T a, and the next measure is the prox itself
    ("jko_b_is_prox_not_ratio", "jko_step", "psi = np.where(np.isfinite(sv), y - sv, -np.inf)",
     "psi = np.where(np.isfinite(sv), y, -np.inf)"),
    ("jko_next_measure_before_prox", "jko_step", "nu = np.exp(y)", "nu = np.exp(sv)"),
    ("energy_without_reference_cell", "porous_energy", "np.sum((nu / ref) ** m)", "np.sum(nu ** m)"),
    # Section 5.3: bins centred on theta_k, and b_t = P(U+) - P(U-)
    ("lift_bins_not_centred", "lift_field", "take = (rel >= -step / 2) & (rel < step / 2)",
     "take = (rel >= 0) & (rel < step)"),
    ("lift_axial_ignored", "lift_field", "period = PI if axial else 2 * PI", "period = 2 * PI"),
    ("project_argmax_of_last_axis_missed", "project", "np.argmax(u, axis=-1)", "np.argmax(u, axis=0)"),
    ("flow_next_step_not_renormalised", "gradient_flow", "mu = nu / nu.sum()", "mu = nu"),
    ("project_adds_negative_part", "project", "mass = mass - u_minus.sum(axis=-1)",
     "mass = mass + u_minus.sum(axis=-1)"),
    ("split_not_normalised", "split_signed", "return (plus / sp if sp > 0 else plus), (minus / sn if sn > 0 else minus)",
     "return plus, minus"),
    # eps-scaling: the schedule ends at eps; g = eps log b carried over between stages
    ("schedule_without_final_eps", "eps_schedule", "return out + [eps]", "return out"),
    ("stage_potentials_not_rescaled", "sinkhorn_eps_scaling", "init = None if psi is None else psi * (sched[-2] / eps)",
     "init = psi"),
    ("ibp_stage_potentials_not_rescaled", "ibp_eps_scaling", "init = None if lv is None else lv * (sched[-2] / eps)",
     "init = lv"),
]


@pytest.mark.parametrize("name,func,old,new", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_pins_catch_python_mutant(monkeypatch, name, func, old, new):
    src = inspect.getsource(getattr(oracle, func))
    assert src.count(old) == 1, name
    ns = {}
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), vars(oracle), ns)
    monkeypatch.setattr(oracle, func, ns[func])
    assert _first_failing_pin() is not None, f"no pin fails for the mutant {name}"
