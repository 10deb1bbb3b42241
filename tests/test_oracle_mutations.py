"""The pins are sharp enough to catch plausible mistakes in the oracle.

Each case copies the oracle's C source, plants one mistake of the kind a
reader of the paper might make (a dropped factor, a swapped operand, a wrong
sign, an off-by-one in a predicate), compiles the copy with gcc into a
temporary library and runs the named pins against it: at least one of them
must fail. The correct oracle passes the same pins (test_oracle_pins.py), so a
pin that fails here is failing because of the planted mistake.

CPU only; the mutants never leave the temporary directory.
"""
import os

import pytest

import oracle
import test_oracle_pins as pins
import workloads as wl

SRC = os.path.join(os.path.dirname(oracle.__file__), "sph_oracle.c")

# name -> (text in the oracle, its replacement, pins that must catch it)
MUTANTS = {
    # eq. 10: the viscosity term
    "eq10_no_h": ("Pi = -p->alpha * h * cbar", "Pi = -p->alpha * cbar",
                  [(pins.test_shear_wave_viscosity, {})]),
    "eq10_eta2_not_scaled": ("double eta2 = p->eta2_h2 * h * h;", "double eta2 = p->eta2_h2;",
                             [(pins.test_shear_wave_viscosity, {})]),
    "eq10_c_a_for_cbar": ("double cbar = 0.5 * (c[a] + c[b]);", "double cbar = c[a];",
                          [(pins.test_momentum_antisymmetry, {})]),
    "eq10_rho_a_for_rhobar": ("double rbar = 0.5 * (rho[a] + rho[b]);", "double rbar = rho[a];",
                              [(pins.test_momentum_antisymmetry, {})]),
    "eq10_switch_inverted": ("if (vdotr < 0.0) {", "if (vdotr > 0.0) {",
                             [(pins.test_viscosity_acts_on_approaching_pairs_only, dict(approach=True)),
                              (pins.test_viscosity_acts_on_approaching_pairs_only, dict(approach=False))]),
    # eq. 9 and 7
    "eq9_pa_twice": ("double coef = mass[b] * (pa + pb + Pi);", "double coef = mass[b] * (pa + pa + Pi);",
                     [(pins.test_momentum_antisymmetry, {})]),
    "eq7_sign": ("d += t;", "d -= t;", [(pins.test_compression_raises_density, {})]),
    # eq. 31 signal term and eq. 30-32
    "eq31_no_h": ("double sig = fabs(h * vdotr / r2);", "double sig = fabs(vdotr / r2);",
                  [(pins.test_signal_term_uniform_compression, dict(wall_fraction=0.0, rho_factor=1.0))]),
    "eq31_over_r": ("double sig = fabs(h * vdotr / r2);", "double sig = fabs(h * vdotr / r);",
                    [(pins.test_signal_term_uniform_compression, dict(wall_fraction=0.0, rho_factor=1.0))]),
    "eq31_c0_for_c_a": ("double v = h / (c[a] + vs[a]);", "double v = h / (p->c0 + vs[a]);",
                        [(pins.test_signal_term_uniform_compression, dict(wall_fraction=0.0, rho_factor=1.01))]),
    # eq. 6: density summation
    "eq6_no_self": ("double sum = mass[a] * W0;", "double sum = 0.0;",
                    [(pins.test_density_summation_lone_particle, dict(kernel=wl.WENDLAND, w0=7.0 / (4.0 * 3.141592653589793)))]),
    "eq6_volume_for_mass": ("sum += mass[b] * orc_kernel_w(K, sqrt(rx * rx + ry * ry), h);",
                            "sum += mass[b] / rho[b] * orc_kernel_w(K, sqrt(rx * rx + ry * ry), h);",
                            [(pins.test_density_summation_lattice_interior, {})]),
    # eq. 29: repulsive-force walls
    "eq29_P_period": ("double P = 0.5 * (1.0 + cos(PI * xi / db));", "double P = 0.5 * (1.0 + cos(2.0 * PI * xi / db));",
                      [(pins.test_wall_force_closed_form, dict(psi_h=0.5, xi_frac=0.3, u_perp=0.0))]),
    "eq29_R_without_sqrt": ("double R = A * (1.0 - q) / sqrt(q);", "double R = A * (1.0 - q) / q;",
                            [(pins.test_wall_force_closed_form, dict(psi_h=0.5, xi_frac=0.0, u_perp=0.0))]),
    "eq29_eps_when_receding": ("double eu = up >= 0.0 ? 0.0", "double eu = up <= 0.0 ? 0.0",
                               [(pins.test_wall_force_closed_form, dict(psi_h=0.5, xi_frac=0.0, u_perp=-0.05))]),
    # eq. 14, 18, 23, 24: colour, normal, curvature, surface force
    "eq14_no_self": ("double sum = mass[a] / rho[a] * W0;", "double sum = 0.0;",
                     [(pins.test_colour_bulk_and_surface, {})]),
    "eq18_C_b_alone": ("nx += vol * (C[b] - C[a]) * gx;\n                ny += vol * (C[b] - C[a]) * gy;",
                       "nx += vol * C[b] * gx;\n                ny += vol * C[b] * gy;",
                       [(pins.test_flat_surface_normal_integral, {})]),
    "eq18_mass_for_volume": ("double vol = mass[b] / rho[b];\n                nx +=",
                             "double vol = mass[b];\n                nx +=",
                             [(pins.test_flat_surface_normal_integral, {})]),
    "eq23_den_no_self": ("double num = 0.0, den = mass[a] / rho[a] * W0, snum = 0.0;",
                         "double num = 0.0, den = 0.0, snum = 0.0;",
                         [(pins.test_circle_curvature, dict(R=16.0))]),
    "eq24_unit_normal": ("sx = f * nv[2 * a];\n                sy = f * nv[2 * a + 1];",
                         "sx = f * nhat[2 * a];\n                sy = f * nhat[2 * a + 1];",
                         [(pins.test_disc_surface_tension_magnitude, dict(kernel=wl.WENDLAND))]),
    "eq24_no_inv_rho": ("double f = -p->sigma / rho[a] * k_a;", "double f = -p->sigma * k_a;",
                        [(pins.test_disc_surface_tension_magnitude, dict(kernel=wl.WENDLAND))]),
    "eq24_sign": ("double f = -p->sigma / rho[a] * k_a;", "double f = p->sigma / rho[a] * k_a;",
                  [(pins.test_disc_surface_tension_magnitude, dict(kernel=wl.WENDLAND))]),
    # kernels (eq. 27-28) and the Tait equation (eq. 26)
    "eq28_printed_constant": ("return 7.0 / (64.0 * PI * h * h);", "return 7.0 / (8.0 * PI * h * h);",
                              [(pins.test_kernel_unit_integral, dict(kernel=wl.WENDLAND, h=1.0))]),
    "eq27_inner_piece": ("if (q <= 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;",
                         "if (q <= 1.0) return 1.0 - 1.5 * q * q + 0.5 * q * q * q;",
                         [(pins.test_kernel_unit_integral, dict(kernel=wl.CUBIC, h=1.0))]),
    "eq26_sound_speed_exponent": ("return p->c0 * pow(rho / p->rho0, 0.5 * (p->gamma - 1.0));",
                                  "return p->c0 * pow(rho / p->rho0, 0.5 * p->gamma);",
                                  [(pins.test_tait_eos, {})]),
    # neighbour predicate (Section 2-7)
    "predicate_not_strict": ("return r2 < R2;", "return r2 <= R2;",
                             [(pins.test_cell_list_matches_brute_force, dict(case="exact_2h"))]),
    # predictor-corrector (Section 2-8)
    "corrector_old_acceleration": ("vel[2 * a] = vx + T * a1[2 * a];\n                    vel[2 * a + 1] = vy + T * a1[2 * a + 1];",
                                   "vel[2 * a] = vx + T * a0[2 * a];\n                    vel[2 * a + 1] = vy + T * a0[2 * a + 1];",
                                   [(pins.test_second_order_in_time, {})]),
    "corrector_drops_half_step_drift": ("pos[2 * a] = pos[2 * a] + T * (vx + 0.5 * T * a1[2 * a]);\n"
                                        "                    pos[2 * a + 1] = pos[2 * a + 1] + T * (vy + 0.5 * T * a1[2 * a + 1]);",
                                        "pos[2 * a] = pos[2 * a] + T * vx;\n"
                                        "                    pos[2 * a + 1] = pos[2 * a + 1] + T * vy;",
                                        [(pins.test_free_fall_is_exact, {})]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, orc, name):
    old, new, checks = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site of {name} not found in the oracle"
    mutant = tmp_path / f"orc_{name}.c"
    mutant.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(mutant), str(tmp_path / f"liborc_{name}.so"))
    caught = []
    with oracle.using(lib):
        for fn, kw in checks:
            try:
                fn(oracle, **kw)
            except AssertionError:
                caught.append(fn.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
