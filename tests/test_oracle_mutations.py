"""The oracle's pins must catch plausible mistakes: each case below plants one
(a flipped sign, a dropped term, transposed axes or operands, a wrong
quadrature weight or integrator coefficient, a wrong misfit or start angle) in
a copy of the oracle source, builds it, and expects some pin to fail."""
import os

import pytest

import oracle
from tests import test_oracle_pins as P
from tests import test_oracle_pins3 as P3

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle_rt.c")

MUTATIONS = {
    "rhs_sign": ("k[2] = -(gx - gd * y[2]) / c;", "k[2] = (gx - gd * y[2]) / c;"),
    "rhs_dropped_projection": ("k[3] = -(gy - gd * y[3]) / c;", "k[3] = -(gy) / c;"),
    "gradient_transposed": ("gx[iy * nx + ix] = d;", "gy[iy * nx + ix] = d;"),
    "hat_operands_swapped": ("w[1] = t * (1.0 - s);\n    w[2] = (1.0 - t) * s;",
                             "w[1] = (1.0 - t) * s;\n    w[2] = t * (1.0 - s);"),
    "trapezoid_last_weight": ("if (mi == M - 1) return (ds + dsp) / 2.0;", "if (mi == M - 1) return ds;"),
    "rk4_coefficient": ("i < 4; i++) out[i] = y[i] + ds / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);",
                        "i < 4; i++) out[i] = y[i] + ds / 6.0 * (k1[i] + 2.0 * k2[i] + k3[i] + k4[i]);"),
    "heun_combination": ("i < 4; i++) out[i] = y[i] + ds / 2.0 * (k1[i] + k2[i]);",
                         "i < 4; i++) out[i] = y[i] + ds * k2[i];"),
    "misfit_sign": ("return mod2pi(atan2(qy, qx) - pe) - mod2pi(pr - pe);",
                    "return mod2pi(pr - pe) - mod2pi(atan2(qy, qx) - pe);"),
    "straight_angle_offset": ("return (mod2pi(elem_angle(ring, rcv) - elem_angle(ring, e)) - PI) / 2.0;",
                              "return (mod2pi(elem_angle(ring, rcv) - elem_angle(ring, e)) - PI) / 2.0 + 0.01;"),
    "edge_stencil": ("d = (-3.0 * c[iy * nx + 0] + 4.0 * c[iy * nx + 1] - c[iy * nx + 2]) / 2.0;",
                     "d = c[iy * nx + 1] - c[iy * nx + 0];"),
    "dtdc_kappa": ("kappa = -1.0 / (cc * cc);", "kappa = -1.0 / cc;"),
    "rayborn_sign": ("acc += w * (im * cos(ph) - re * sin(ph));", "acc += w * (im * cos(ph) + re * sin(ph));"),
    "fan_sample_angle_off_by_one": ("TH[j - 1] = straight_angle(ring, e, k);",
                                    "TH[j - 1] = straight_angle(ring, e, (k + 1) % n);"),
    "bspline_gain_dropped": ("for (int k = 0; k < n; k++) v[k * stride] *= 6.0;",
                             "for (int k = 0; k < n; k++) v[k * stride] *= 1.0;"),
    "bspline_anticausal_init": ("v[(n - 1) * stride] = (z / (z * z - 1.0)) * (v[(n - 1) * stride] + z * v[(n - 2) * stride]);",
                                "v[(n - 1) * stride] = (z / (z * z - 1.0)) * v[(n - 1) * stride];"),
    "bspline_weight_term_sign": ("w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;",
                                 "w[2] = (-3.0 * t * t * t - 3.0 * t * t + 3.0 * t + 1.0) / 6.0;"),
    "bspline_derivative_sign": ("dw[0] = -u * u / 2.0;", "dw[0] = u * u / 2.0;"),
    "bspline_half_sample_mirror": ("if (i < 0) return -i;", "if (i < 0) return -i - 1;"),
    "fan_cubic_weight_sign": ("if (k != i) w *= (0.0 - g[k]) / (g[i] - g[k]);",
                              "if (k != i) w *= (0.0 + g[k]) / (g[i] - g[k]);"),
    "fan_cubic_shifted_stencil": ("const double *g = G + a - 1, *t = TH + a - 1;",
                                  "const double *g = G + a - 1, *t = TH + a;"),
    "fan_cubic_bracket_ends": ("double lo = t[1] < t[2] ? t[1] : t[2], hi = t[1] < t[2] ? t[2] : t[1];",
                               "double lo = t[0] < t[3] ? t[0] : t[3], hi = t[0] < t[3] ? t[3] : t[0];"),
    "fan_quintic_weight_sign": ("if (l != i) w *= (0.0 - g[l]) / (g[i] - g[l]);",
                                "if (l != i) w *= (0.0 + g[l]) / (g[i] - g[l]);"),
    "fan_quintic_shifted_stencil": ("const double *g = G + a - 2, *t = TH + a - 2;",
                                    "const double *g = G + a - 2, *t = TH + a - 1;"),
    "fan_quintic_hedge_dropped": ("if (out->n_marches == 0 && have_q && thq != th) c[1] = thq;",
                                  "if (out->n_marches == 0 && have_q && thq != th) c[1] = c[1];"),
    "sart_rowsum_dropped": ("double r = (b[i] - proj) / M[i];", "double r = (b[i] - proj);"),
    "sart_colsum_dropped": ("if (V[j] != 0.0) x[j] += lambda * upd[j] / V[j];",
                            "if (V[j] != 0.0) x[j] += lambda * upd[j];"),
    "sart_sequential_update": ("for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) upd[col[k]] += val[k] * r;",
                               "for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) x[col[k]] += lambda * val[k] * r "
                               "/ V[col[k]];"),
    "paraxial_dKdd_sign": ("+ (gp * d[a] + gd * p[a]) / c;", "- (gp * d[a] + gd * p[a]) / c;"),
    "paraxial_dc_term_dropped": (" + (G[a] - gd * d[a]) * dcq / (c * c)", ""),
    "paraxial_start_perturbation": ("0.0, 0.0, -sin(psi), cos(psi)}, yn[8];", "0.0, 0.0, sin(psi), -cos(psi)}, yn[8];"),
    "paraxial_hit_shift_dropped": ("dqx += dt * ax;", "dqx += 0.0 * ax;"),
    "paraxial_bspline_curvature_weight": ("double ddwx[4] = {1.0 - t, 3.0 * t - 2.0, 1.0 - 3.0 * t, t};",
                                          "double ddwx[4] = {1.0 - t, 3.0 * t - 2.0, 1.0 - 3.0 * t, -t};"),
    "paraxial_bilinear_hessian_operand": ("H[1] += ws[k] * m->gx[n[k]];", "H[1] += wt[k] * m->gx[n[k]];"),
    "fan_target_wrong_receiver": ("G[j - 1] = row[j - 1].st == ST_LINKED ? (row[j - 1].g + Dj) - Dr : NAN;",
                                  "G[j - 1] = row[j - 1].st == ST_LINKED ? row[j - 1].g - Dr : NAN;"),
}

PINS = [
    lambda o: P.test_gradient_exact_on_quadratics(o),
    lambda o: P.test_gradient_is_not_transposed(o),
    lambda o: P.test_bilinear_exact_and_gradient_of_quadratic(o),
    lambda o: P.test_bspline_matches_library_mirror_spline(o),
    lambda o: P.test_bspline_reproduces_cubics_in_the_interior(o),
    lambda o: P.test_homogeneous_straight_rays(o),
    lambda o: P.test_homogeneous_weights_are_hat_line_integrals(o),
    lambda o: P.test_linear_gradient_closed_form(o, (250.0, 300.0), "rk4"),
    lambda o: P.test_linear_gradient_closed_form(o, (400.0, 0.0), "heun"),
    lambda o: P.test_weak_medium_links_in_two_marches(o),
    lambda o: P.test_fisheye_analytic_medium_closed_form(o),
    lambda o: P.test_paper_fisheye_acoustic_length(o, "analytic", "rk4"),
    lambda o: P.test_paper_fisheye_radius_deviation(o, "analytic", "rk4"),
    lambda o: P.test_paper_fisheye_radius_deviation(o, "analytic", "heun"),
    lambda o: P.test_linear_gradient_second_order_in_step(o),
    lambda o: P.test_adjoint_is_transpose_of_weights(o),
    lambda o: P.test_dtdc_adjoint_matches_finite_differences(o),
    lambda o: P.test_rayborn_rho_is_derivative_of_phase_data(o),
    lambda o: P.test_fan_cubic_exact_for_cubic_inverse(o),
    lambda o: P.test_fan_cubic_fourth_order_on_smooth_inverse(o),
    lambda o: P.test_fan_cubic_falls_back(o),
    lambda o: P.test_fan_quintic_exact_for_quintic_inverse(o),
    lambda o: P.test_fan_quintic_sixth_order_on_smooth_inverse(o),
    lambda o: P.test_fan_quintic_falls_back(o),
    lambda o: P.test_fan_first_round_traces_the_quintic(o),
    lambda o: P.test_fan_start_same_roots_fewer_rays(o),
    lambda o: P.test_fan_start_fisheye_reversed_orientation(o),
    lambda o: P.test_paraxial_homogeneous_closed_form(o, "rk4"),
    lambda o: P.test_paraxial_matches_finite_differences(o, "bspline", 1e-7),
    lambda o: P.test_paraxial_matches_finite_differences(o, "bilinear", 2e-5),
    lambda o: P.test_paraxial_fisheye_focus(o),
    lambda o: P.test_sart_one_row_is_exact(o),
    lambda o: P.test_sart_step_is_preconditioned_gradient_step(o),
    lambda o: P.test_sart_consistent_system_converges(o),
    lambda o: P.test_sart_zero_rows_and_columns_take_no_part(o),
]


SRC3 = os.path.join(os.path.dirname(oracle.__file__), "oracle_rt3.c")

MUTATIONS3 = {
    "rhs3_sign": ("k[3 + a] = -(G[a] - gd * y[3 + a]) / c;", "k[3 + a] = (G[a] - gd * y[3 + a]) / c;"),
    "trilinear_axes_swapped": ("(by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);",
                               "(by ? f[2] : 1.0 - f[2]) * (bz ? f[1] : 1.0 - f[1]);"),
    "gradient3_wrong_stride": ("m->g[n + k] = diff1(m->c, idx3(m, ix, 0, iz), (size_t)m->nx, iy, m->ny);",
                               "m->g[n + k] = diff1(m->c, idx3(m, 0, iy, iz), 1, ix, m->nx);"),
    "jacobian3_length_term": ("dq[i] = L * dd[i] - 2.0 * d[i] * ed;", "dq[i] = L * dd[i];"),
    "quadrature3_last_weight": ("acc += (ds + dsp) / 2.0 / c + dsp / 2.0 / cq;", "acc += ds / c + dsp / 2.0 / cq;"),
    "sphere_crossing_root": ("double t = (B >= 0) ? (-2.0 * C) / (B + sqrt(D)) : (-B + sqrt(D)) / (2.0 * A);\n"
                             "            if (t > 1.0) t = 1.0;\n            if (t < 0.0) t = 0.0;\n"
                             "            for (int i = 0; i < 3; i++)",
                             "double t = (B >= 0) ? (-B - sqrt(D)) / (2.0 * A) : (2.0 * C) / (-B + sqrt(D));\n"
                             "            if (t > 1.0) t = 1.0;\n            if (t < 0.0) t = 0.0;\n"
                             "            for (int i = 0; i < 3; i++)"),
    "broyden_update_sign": ("J[0] += r0 * du[0] / uu;\n                J[1] += r0 * du[1] / uu;",
                            "J[0] -= r0 * du[0] / uu;\n                J[1] -= r0 * du[1] / uu;"),
}

PINS3 = [
    lambda o: P3.test3_homogeneous_straight_rays(o),
    lambda o: P3.test3_homogeneous_jacobian_matches_traced_misfit(o),
    lambda o: P3.test3_linear_gradient_closed_form(o, (50.0, -70.0, 80.0)),
    lambda o: P3.test3_fisheye_antipodal_focus(o, "analytic", 0.003),
    lambda o: P3.test3_fisheye_antipodal_focus(o, "grid", 0.05),
    lambda o: P3.test3_fisheye_circles(o, "rk4", 1e-4),
    lambda o: P3.test3_reciprocity_gaussian_volume(o),
    lambda o: P3.test3_broyden_links_and_status_paths(o),
]


@pytest.mark.parametrize("name", sorted(MUTATIONS3))
def test_planted_mistake_3d_is_caught(name, tmp_path, orc):
    old, new = MUTATIONS3[name]
    src = open(SRC3).read()
    assert src.count(old) == 1, name
    mut = tmp_path / "oracle_rt3_mut.c"
    mut.write_text(src.replace(old, new))
    lib = oracle.build(src=SRC, src3=str(mut), out=str(tmp_path / "liboracle_mut3.so"))
    caught = None
    with oracle.use_library(lib):
        for k, pin in enumerate(PINS3):
            try:
                pin(oracle)
            except (AssertionError, ValueError, IndexError, ZeroDivisionError):
                caught = k
                break
    assert caught is not None, f"no 3-D pin fails with the planted mistake {name!r}"


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, orc):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    lib = oracle.build(src=str(mut), out=str(tmp_path / "liboracle_mut.so"))
    caught = None
    with oracle.use_library(lib):
        for k, pin in enumerate(PINS):
            try:
                pin(oracle)
            except (AssertionError, ValueError, IndexError, ZeroDivisionError):
                caught = k
                break
    assert caught is not None, f"no pin fails with the planted mistake {name!r}"
