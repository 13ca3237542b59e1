"""The pins are sharp: plant one plausible mistake at a time in the oracle's
C source (on the CPU), rebuild it, and check that at least one pin fails.

Each mutation is a dropped term, a flipped sign, a wrong weight, index or
direction table entry in one part of the coupled step.
"""
import os

import pytest

from oracle import build_oracle
from oracle import oracle as orc
from tests import test_oracle_adjoint as AD
from tests import test_oracle_cde as CD
from tests import test_oracle_pins as P
from tests import test_oracle_pressure as PR
from tests import test_oracle_walls as WL

PINS = [
    (P.test_feq_full_moment_basis, dict(rho=1.03, ux=0.05, uy=-0.02)),
    (P.test_feq_weights_isotropy, {}),
    (P.test_geq_full_moment_basis, dict(w0=1 / 3, C=0.7, ux=0.05, uy=-0.03)),
    (P.test_periodic_conservation_mass_momentum_solute, {}),
    (P.test_source_and_decay_enter_solute_budget, {}),
    (P.test_uniform_equilibrium_is_fixed_point, {}),
    (P.test_tau_f_one_streams_the_equilibrium, {}),
    (P.test_tau_g_one_is_ftcs_scheme, dict(w0=1 / 3)),
    (P.test_compound_lattice_exact_fourier_evolution, {}),
    (P.test_closed_box_conserves_with_bounce_back_and_closed_valves, {}),
    (P.test_inlet_mass_inflow_closed_form, {}),
    (P.test_inlet_concentration_fills_channel, {}),
    (P.test_poiseuille_profile_and_linear_pressure_drop, {}),
    (P.test_advected_gaussian_closed_form_and_second_order, {}),
    (AD.test_adjoint_step_is_transpose_of_forward_step, dict(t_phase=0)),
    (AD.test_adjoint_step_is_transpose_of_forward_step, dict(t_phase=15)),
    (AD.test_adjoint_gradients_match_central_differences, {}),
    (CD.test_cde_step_equals_the_coupled_compound_update, {}),
    (CD.test_cde_uniform_velocity_exact_fourier_evolution, {}),
    (CD.test_cde_closed_box_conserves_solute, {}),
]
# the pins of the paper's walls, tried first for mistakes in their code
WALL_PINS = [
    (WL.test_ghost_density_extrapolated_linearly, dict(valve=False)),
    (WL.test_ghost_density_extrapolated_linearly, dict(valve=True)),
    (WL.test_ghost_momentum_vanishes_at_the_halfway_wall, {}),
    (WL.test_ghost_compound_even_about_the_wall, {}),
    (WL.test_compound_only_step_ghost_rule, {}),
    (WL.test_rest_state_is_fixed_point, {}),
    (WL.test_compound_uniform_across_the_channel_stays_so, {}),
    (WL.test_pressure_driven_flow_no_slip_points, {}),
]
# the pressure boundary's pins, tried first for mistakes in its code
PRESSURE_PINS = [
    (PR.test_density_and_concentration_held_exactly, {}),
    (PR.test_mass_and_compound_accounting, {}),
    (PR.test_uniform_rest_state_is_fixed_point, {}),
    (PR.test_closed_pressure_valves_are_walls, {}),
    (PR.test_cde_step_equals_coupled_compound_with_pressure_boundaries, {}),
    (PR.test_pressure_driven_poiseuille, {}),
]

MUTATIONS = {
    "diagonal weight": ("1.0 / 36.0, 1.0 / 36.0};", "1.0 / 36.0, 1.0 / 35.0};"),
    "feq (e.u)^2 coefficient": ("4.5 * eu * eu - 1.5 * usq", "4.0 * eu * eu - 1.5 * usq"),
    "feq u^2 coefficient": ("4.5 * eu * eu - 1.5 * usq", "4.5 * eu * eu - 1.0 * usq"),
    "feq linear coefficient": ("1.0 + 3.0 * eu", "1.0 + 2.0 * eu"),
    "geq divides by cs2": ("(1.0 + eu / cs2)", "(1.0 + eu * cs2)"),
    "compound axis weight": ("wg5[i] = (1.0 - w0) / 4.0;", "wg5[i] = (1.0 - w0) / 5.0;"),
    "opposite of diagonals": ("{0, 3, 4, 1, 2, 7, 8, 5, 6}", "{0, 3, 4, 1, 2, 8, 7, 6, 5}"),
    "direction table": ("EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1}", "EY[9] = {0, 0, 1, 0, -1, 1, -1, -1, 1}"),
    "f relaxation sign": ("fx[i] - omega_f * (fx[i] - feq[i])", "fx[i] + omega_f * (fx[i] - feq[i])"),
    "g relaxation term": ("gx[i] - omega_g * (gx[i] - geq[i])", "gx[i] - omega_g * (gx[i] + geq[i])"),
    "u_y from j_x": ("double ux = jx / rho, uy = jy / rho;\n  u[0]", "double ux = jx / rho, uy = jx / rho;\n  u[0]"),
    "source weight dropped": ("+ wg[i] * src;", "+ src;"),
    "decay sign": ("- L->k_decay * C;", "+ L->k_decay * C;"),
    "inlet momentum sign": ("in_f = out_f - 6.0 * WF[i]", "in_f = out_f + 6.0 * WF[i]"),
    "inlet momentum factor": ("in_f = out_f - 6.0 * WF[i]", "in_f = out_f - 3.0 * WF[i]"),
    "anti-bounce-back factor": ("2.0 * wg[i] * c_in[code]", "1.0 * wg[i] * c_in[code]"),
    "anti-bounce-back sign": ("in_g = -out_g + 2.0", "in_g = out_g + 2.0"),
    "outlet f sign": ("in_f = -out_f + 2.0 * WF[i]", "in_f = out_f + 2.0 * WF[i]"),
    "outlet g direction": ("if (has_g) in_g = gp[5 * node + i];", "if (has_g) in_g = gp[5 * node + opp];"),
    "periodic wrap": ("x = (x + L->nx) % L->nx;", "x = (x + L->nx + 1) % L->nx;"),
    "inlet profile": ("4.0 * L->seg_umax[seg]", "6.0 * L->seg_umax[seg]"),
    "wall bounce-back loses mass": ("in_f = out_f;\n          in_g = out_g;\n        } else if",
                                    "in_f = 0.999 * out_f;\n          in_g = out_g;\n        } else if"),
    "tau_f": ("double omega_f = 1.0 / L->tau_f;", "double omega_f = 1.0 / (L->tau_f + 0.05);"),
    "tau_g": ("double omega_g = 1.0 / L->tau_g;", "double omega_g = 1.0 / (L->tau_g + 0.05);"),
    "adjoint inlet sign": ("ls[j] -= lx[opp];", "ls[j] += lx[opp];"),
    "adjoint outlet re-emission": ("ls[j] += lx[j]; /* the outlet", "ls[j] += 0.0 * lx[j]; /* the outlet"),
    "adjoint collision": ("lam_out[5 * node + i] = (1.0 - omega) * ls[i] + s;",
                          "lam_out[5 * node + i] = (1.0 - omega) * ls[i] + 0.5 * s;"),
    "adjoint C_in factor": ("ra[code] += 2.0 * wg[opp]", "ra[code] += 1.0 * wg[opp]"),
    "adjoint omega sign": ("dw -= ls[j] * (gx[j] - W[j] * C);", "dw += ls[j] * (gx[j] - W[j] * C);"),
    "adjoint source weight": ("dr += wg[j] * ls[j];", "dr += ls[j];"),
    "compound-only relaxation": ("gx[i] - omega * (gx[i] - geq[i])", "gx[i] - omega * (gx[i] + geq[i])"),
    "compound-only inlet sign": ("in = -out + 2.0 * wg[i] * c_in[code];", "in = out + 2.0 * wg[i] * c_in[code];"),
    "compound-only outlet direction": ("in = gp[5 * node + i];", "in = gp[5 * node + OPP[i]];"),
    "compound-only streaming": ("gn[5 * node + i] = gp[5 * ((size_t)ys * nx + xs) + i];",
                                "gn[5 * node + i] = gp[5 * ((size_t)ys * nx + xs) + OPP[i]];"),
    "compound-only source": ("+ wg[i] * src;\n    }\n\n  memset(gn", "+ src;\n    }\n\n  memset(gn"),
    "compound-only wall": ("        if (kind == ORC_SEG_NONE)\n          in = out;", "        if (kind == ORC_SEG_NONE)\n          in = 0.999 * out;"),
    "pressure do-nothing after collision": ("in_f = f[9 * node + i];", "in_f = fp[9 * node + i];"),
    "pressure rescale inverted": ("double gam = L->seg_rho[m] / rho;", "double gam = rho / L->seg_rho[m];"),
    "pressure compound guard dropped": ("if (C > 0.0) {\n    double gam = c_in[m] / C;",
                                        "if (1) {\n    double gam = c_in[m] / C;"),
    "pressure compound held everywhere": ("if (!L->seg_fixc[m]) return 0.0;", "if (0) return 0.0;"),
    "pressure ignores the valves": ("L->seg_kind[code] == ORC_SEG_PRESSURE && open[code]) return code;",
                                    "L->seg_kind[code] == ORC_SEG_PRESSURE) return code;"),
    "pressure rescale not counted": ("return L->seg_rho[m] - rho;", "return 0.0;"),
    "pressure compound not counted": ("return c_in[m] - C;", "return 0.0;"),
    "compound-only pressure rule": ("in = L->seg_fixc[code] ? g[5 * node + i] : gp[5 * node + i];",
                                    "in = L->seg_fixc[code] ? gp[5 * node + i] : gp[5 * node + i];"),
    "paper wall rule: ghost momentum sign": ("orc_feq(rho_s, -jx / rho_s, -jy / rho_s, feq);",
                                             "orc_feq(rho_s, jx / rho_s, -jy / rho_s, feq);"),
    "paper wall rule: density extrapolation": ("rho_s = 2.0 * rho - rho_a;", "rho_s = rho_a;"),
    "paper wall rule: Guo relaxation": ("gz[i] = gs[i] + (1.0 - omega_g) * (g[5 * node + i] - gz0[i]);\n    }\n  }\n}",
                                        "gz[i] = gs[i] + (g[5 * node + i] - gz0[i]);\n    }\n  }\n}"),
    "paper wall rule: Guo ghost velocity": ("orc_geq(C, -jx / rho_s, -jy / rho_s, L->w0, gs);",
                                            "orc_geq(C, -jx / rho_s, jy / rho_s, L->w0, gs);"),
    "paper wall rule: compound-only ghost": ("orc_geq(C, -ux, -uy, L->w0, gs);", "orc_geq(C, -ux, uy, L->w0, gs);"),
    "paper wall rule: wall link test": ("    if (!(code == 1 || L->seg_kind[code] == ORC_SEG_NONE || !open[code])) continue;\n    double rho_s",
                                        "    if (!(code == 1)) continue;\n    double rho_s"),
    "adjoint wall transpose": ("            ls[j] += lx[opp];\n          } else if (kind == ORC_SEG_INLET) {",
                               "            ls[j] += lx[j];\n          } else if (kind == ORC_SEG_INLET) {"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_some_pin_catches(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(build_oracle.SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    mut = os.path.join(tmp_path, "mut.c")
    with open(mut, "w") as fh:
        fh.write(src.replace(old, new, 1))
    lib_path = build_oracle.build(src=mut, out=os.path.join(tmp_path, "libmut.so"))
    orc.use_library(lib_path)
    caught = []
    if "pressure" in name:
        pins = PRESSURE_PINS + PINS
    elif "wall rule" in name:
        pins = WALL_PINS + PINS
    else:
        pins = PINS + PRESSURE_PINS
    try:
        for fn, kw in pins:
            try:
                fn(**kw)
            except AssertionError:
                caught.append(fn.__name__)
                break
    finally:
        orc.use_library(None)
    assert caught, f"no pin fails when the oracle has: {name}"
