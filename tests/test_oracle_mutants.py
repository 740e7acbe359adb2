"""The pins must be able to fail: each planted mistake in the oracle source
(a dropped or wrong term, a sign, an index, a table entry, a reading of the
paper) is compiled on the CPU and must break at least one pin."""
import os
import shutil
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "maclab_oracle.c")

MUTANTS = {
    "quadratic_coeff": ("4.5 * eu * eu", "4.0 * eu * eu"),
    "isotropic_coeff": ("- 1.5 * uu / e2", "- 1.0 * uu / e2"),
    "linear_scale": ("3.0 * eu / e2", "3.0 * eu / e"),
    "push_not_pull": ("int64_t si = wrap(i - c[a][0], nx);", "int64_t si = wrap(i + c[a][0], nx);"),
    "momentum_component": ("m[cc] += e * (real)c[a][cc] * f;", "m[cc] += e * (real)c[a][(cc + 1) % d] * f;"),
    "force_sign": ("m[cc] / r + dt * p->G[cc] / r", "m[cc] / r - dt * p->G[cc] / r"),
    "old_density": ("m[cc] / r + dt", "m[cc] / rho[i + nx * (j + ny * k)] + dt"),
    "viscosity_map": ("return 6.0 * (real)nu / (real)dx;", "return 3.0 * (real)nu / (real)dx;"),
    "d3q19_weight": ("(real)1 / 18, (real)1 / 36, (real)1 / 36, (real)1 / 36,\n    (real)1 / 36, (real)1 / 36",
                     "(real)1 / 36, (real)1 / 36, (real)1 / 36, (real)1 / 36,\n    (real)1 / 36, (real)1 / 36"),
    "d3q19_velocity": ("{-1, 0, 1}, {1, 0, -1}}", "{1, 0, 1}, {1, 0, -1}}"),
    "d2q9_velocity": ("{1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}}", "{1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}}"),
    "corner_owner": ("for (int f = 0; f < 6; ++f) {\n    if (p->face_kind[f] == ORACLE_PERIODIC) continue;",
                     "for (int f = 5; f >= 0; --f) {\n    if (p->face_kind[f] == ORACLE_PERIODIC) continue;"),
    "neumann_density_not_copied": ("          rho[x] = rho[s];", "          rho[x] = rho[x];"),
    "pressure_velocity_not_copied": ("for (int c = 0; c < d; ++c) u[c * N + x] = u[c * N + s];",
                                     "for (int c = 0; c < d; ++c) u[c * N + x] = u[c * N + x];"),
    "interior_two_nodes_in": ("if (idx[ax] < 1) idx[ax] = 1;", "if (idx[ax] < 2) idx[ax] = 2;"),
    "interior_periodic_clamped": ("    if (p->face_kind[2 * ax] == ORACLE_PERIODIC) continue;\n    if (idx[ax] < 1)",
                                  "    if (idx[ax] < 1)"),
    "derived_faces_not_updated": ("  copy_from_interior(p, rho_new, u_new);\n}", "  (void)rho_new;\n}"),
    "pressure_density_not_held": ("if (p->face_kind[f] != ORACLE_RHO_NEUMANN) rho[x] = p->face_rho[f];",
                                  "if (p->face_kind[f] == ORACLE_FIXED) rho[x] = p->face_rho[f];"),
    "energy_half": ("nsum_add(&E, 0.5 * rho[x] * uu);", "nsum_add(&E, rho[x] * uu);"),
    "adjoint_division_sign": ("rt[x] = rb[x] - dot / r1;", "rt[x] = rb[x] + dot / r1;"),
    "adjoint_downstream_index": ("int64_t xi = wrap(i + c[a][0], nx);", "int64_t xi = wrap(i - c[a][0], nx);"),
    "adjoint_force_dt": ("grad_G[cc] += dt * mb[cc * N + x];", "grad_G[cc] += mb[cc * N + x];"),
    "adjoint_quadratic": ("9.0 * eu * ea / (e * e * e * e)", "4.5 * eu * ea / (e * e * e * e)"),
    "fixed_nodes_updated": ("if (fixed_face(p, i, j, k) >= 0) {\n          /* Recipe step (iv)",
                            "if (fixed_face(p, i, j, k) >= 7) {\n          /* Recipe step (iv)"),
}


def _battery():
    yield pins.test_lattice_tables_match_paper, {}
    for q in (9, 19):
        yield pins.test_feq_moments, {"q": q}
        yield pins.test_shear_wave_exact_factor, {"q": q, "amp": 0.2}
        yield pins.test_conservation_periodic, {"q": q, "n": (12, 10, 1) if q == 9 else (6, 5, 4), "force": True}
    yield pins.test_parameter_map, {}
    yield pins.test_single_step_4x4_closed_form, {}
    for args in ((9, (9, 8, 1), True), (19, (6, 5, 5), True), (9, (12, 10, 1), False), (19, (6, 5, 4), False)):
        yield pins.test_equivalence_with_bgk_tau1, {"q": args[0], "n": args[1], "walls": args[2], "force": True}
    yield pins.test_poiseuille_steady_profile_is_exact, {"nu": 0.001, "u0": 0.1}
    yield pins.test_boundary_precedence, {}
    yield pins.test_diagnostics_match_exact_sums, {}
    yield pins.test_adjoint_matches_central_differences, {"q": 9, "n": (9, 7, 1), "walls": True}
    yield pins.test_adjoint_matches_central_differences, {"q": 19, "n": (5, 4, 4), "walls": False}
    yield pins.test_adjoint_force_closed_form, {}
    for q in (9, 19):
        yield pins.test_derived_faces_copy_the_nearest_interior_node, {"q": q}
        yield pins.test_shear_wave_through_pressure_faces_keeps_the_exact_factor, {"q": q}
    yield pins.test_rho_neumann_plates_keep_the_channel_profiles_exact, {"nu": 0.001, "u0": 0.1, "dpdx": -1e-4}
    yield pins.test_pressure_driven_channel_is_poiseuille, {}


def _caught(lib):
    prev = oracle.use(lib)
    try:
        for fn, kw in _battery():
            try:
                fn(None, **kw)
            except (AssertionError, ValueError):
                return fn.__name__
        return None
    finally:
        oracle.use(prev)


def test_unmutated_battery_passes():
    oracle.build()
    assert _caught(None) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    find, repl = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(find) == 1, f"mutation anchor for {name} not unique"
    msrc = tmp_path / "maclab_oracle.c"
    msrc.write_text(src.replace(find, repl))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared", str(msrc),
                    "-o", lib, "-lm"], check=True)
    assert _caught(lib) is not None, f"no pin catches mutant {name}"
