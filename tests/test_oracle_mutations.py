"""The oracle's pins catch plausible mistakes: each mutation below is a one-line slip in
``oracle/ctoracle.c`` (a flipped sign, a dropped term, a wrong formula or index); the test
builds the oracle with it, runs the pins against that build and requires at least one pin to
fail.  The unmodified source must pass every pin used here (checked first).

Only the oracle is mutated, on the CPU; nothing here touches the HIP engine.
"""
import math
import os
import subprocess

import pytest

import oracle
import test_oracle_geometry_pins as G
import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "ctoracle.c")
EXACT = os.path.join(os.path.dirname(oracle.__file__), "exact_ray.c")

# (id, original text, replacement); each original must occur exactly once
MUTATIONS = [
    ("theta_sign",
     "double Rz[3][3] = {{cos(th), -sin(th), 0}, {sin(th), cos(th), 0}, {0, 0, 1}};",
     "double Rz[3][3] = {{cos(th), sin(th), 0}, {-sin(th), cos(th), 0}, {0, 0, 1}};"),
    ("phi_sign",
     "double Rx[3][3] = {{1, 0, 0}, {0, cos(ph), -sin(ph)}, {0, sin(ph), cos(ph)}};",
     "double Rx[3][3] = {{1, 0, 0}, {0, cos(ph), sin(ph)}, {0, -sin(ph), cos(ph)}};"),
    ("psi_sign",
     "double Ry[3][3] = {{cos(ps), 0, sin(ps)}, {0, 1, 0}, {-sin(ps), 0, cos(ps)}};",
     "double Ry[3][3] = {{cos(ps), 0, -sin(ps)}, {0, 1, 0}, {sin(ps), 0, cos(ps)}};"),
    ("pose_order_phi_first", "matmul3(Rx, Ry, T);\n    matmul3(Rz, T, R);",
     "matmul3(Ry, Rx, T);\n    matmul3(Rz, T, R);"),
    ("x_src_sign", "const double s0[3] = {g->x_src[b],", "const double s0[3] = {-g->x_src[b],"),
    ("z_src_sign", "three_d ? g->z_src[b] : 0.0};", "three_d ? -g->z_src[b] : 0.0};"),
    ("x_ofst_sign", "f->o[0] = g->x_ofst[b];", "f->o[0] = -g->x_ofst[b];"),
    ("y_ofst_sign", "f->o[1] = g->y_ofst[b];", "f->o[1] = -g->y_ofst[b];"),
    ("z_ofst_sign", "f->o[2] = three_d ? g->z_ofst[b] : 0.0;",
     "f->o[2] = three_d ? -g->z_ofst[b] : 0.0;"),
    ("u_ofst_sign", "* g->du - g->u_ofst[b];", "* g->du + g->u_ofst[b];"),
    ("v_ofst_sign", "* g->dv - g->v_ofst[b] : 0.0;", "* g->dv + g->v_ofst[b] : 0.0;"),
    ("curved_v_flat_denominator", "f->sdd * dot3(ps, f->ev) / sqrt(a * a + w * w);",
     "f->sdd * dot3(ps, f->ev) / w;"),
    ("curved_u_tangent", "*u = f->sdd * atan2(a, w);", "*u = f->sdd * a / w;"),
    ("sf_transaxial_at_bottom_face",
     "p[2] = c[2];\n        project(g, f, p, &u, &v);\n        tau[k] = u;",
     "p[2] = c[2] - hz;\n        project(g, f, p, &u, &v);\n        tau[k] = u;"),
    ("sf_bottom_face_at_midplane", "p[2] = c[2] - hz;\n            project(g, f, p, &u, &v);\n            bmin",
     "p[2] = c[2];\n            project(g, f, p, &u, &v);\n            bmin"),
    ("sf_amp_max", "fp->amp = fmin(lx, ly);", "fp->amp = fmax(lx, ly);"),
    ("sf_no_polar_amplitude", "return sqrt(rx * rx + ry * ry + rz * rz) / hypot(rx, ry);",
     "return 1.0;"),
    ("trap_ramp_no_half", "return r1 > eps ? (t - k[0]) * (t - k[0]) / (2.0 * r1) : 0.0;",
     "return r1 > eps ? (t - k[0]) * (t - k[0]) / r1 : 0.0;"),
    ("sf_cell_average_no_du",
     "fp->F1[i] = (trap_cdf(tau, e + g->du, 1e-12 * g->du) - trap_cdf(tau, e, 1e-12 * g->du)) / g->du;",
     "fp->F1[i] = (trap_cdf(tau, e + g->du, 1e-12 * g->du) - trap_cdf(tau, e, 1e-12 * g->du));"),
    ("dd_rows_along_edge_ray",
     "/* axial map along the column-centre ray */\n        det_point(g, f, f->u_first + i * g->du, 0.0, q);",
     "/* axial map along the column-centre ray */\n        det_point(g, f, ue0 + i * g->du, 0.0, q);"),
    ("dd_no_slab_factor", "return dd_y_driven(f) ? g->dy * r / fabs(ry) : g->dx * r / fabs(rx);",
     "return dd_y_driven(f) ? r / fabs(ry) : r / fabs(rx);"),
    ("dd_axial_fraction_of_voxel",
     "fp->Fz[k * g->nv + (j - j_lo)] = oz > 0.0 ? oz / (rhi - rlo) : 0.0;",
     "fp->Fz[k * g->nv + (j - j_lo)] = oz > 0.0 ? oz / g->dz : 0.0;"),
    ("dd_fixed_axis", "return fabs(f->n[1]) >= fabs(f->n[0]);", "return 1;"),
]

# Pins run against each mutated build, cheapest first; a mutation is caught by the first
# one that fails.
CHECKS = [
    ("G1 source offsets (SF)", lambda o: G.test_g1_source_offsets(o, "sf")),
    ("G1 source offsets (DD)", lambda o: G.test_g1_source_offsets(o, "dd")),
    ("G2 object offsets (SF)", lambda o: G.test_g2_object_offsets(o, "sf")),
    ("G2 object offsets (DD)", lambda o: G.test_g2_object_offsets(o, "dd")),
    ("G3 detector offsets (SF)", lambda o: G.test_g3_detector_offsets(o, "sf")),
    ("G3 detector offsets (DD)", lambda o: G.test_g3_detector_offsets(o, "dd")),
    ("G4 psi", G.test_g4_in_plane_tilt_psi),
    ("G4 mid-plane corners", G.test_g4_transaxial_corners_at_mid_plane),
    ("G5 phi", G.test_g5_off_plane_tilt_phi),
    ("G5 pose order", G.test_g5_pose_order),
    ("G6 curved wide fan (SF)", lambda o: G.test_g6_curved_detector_wide_fan(o, "sf")),
    ("G6 curved wide fan (DD)", lambda o: G.test_g6_curved_detector_wide_fan(o, "dd")),
    ("G6 curved 2D", G.test_g6_curved_fan2d),
    ("G8 curved mirror (SF)", lambda o: G.test_g8_curved_mirror(o, "sf")),
    ("G8 curved mirror (DD)", lambda o: G.test_g8_curved_mirror(o, "dd")),
    ("P1 single voxel", P.test_p1_single_voxel_closed_form),
    ("P1b orientation", P.test_p1_direction_conventions),
    ("P2 parallel 2D SF", lambda o: P.test_p2_parallel_2d_sf_exact(o, 30.0)),
    ("P2 parallel 3D SF", lambda o: P.test_p2_parallel_3d_sf_exact(o, 33.0)),
    ("P2 parallel tilted", lambda o: P.test_p2_parallel_tilted_sf_exact(o, 12.0)),
    ("P2 parallel DD", lambda o: P.test_p2_parallel_2d_dd_exact_on_axes(o, 90.0)),
    ("P3 mass (SF)", lambda o: P.test_p3_mass_conservation(o, "sf", 27.0)),
    ("P3 mass (DD)", lambda o: P.test_p3_mass_conservation(o, "dd", 27.0)),
] + [(f"G7 brute force {c[0]}", (lambda c: lambda o: G.test_g7_brute_force_with_offsets(o, *c))(c))
     for c in G.BF_CASES] + [
    ("P7 brute force (flat)", lambda o: P.test_p7_brute_force_cone(o, "flat")),
]


def _build(tmp_path, text, tag):
    src = tmp_path / f"ctoracle_{tag}.c"
    src.write_text(text)
    so = tmp_path / f"libctoracle_{tag}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", "-o", str(so), str(src), EXACT, "-lm"], check=True)
    return str(so)


def _first_failure(path):
    saved = oracle._lib
    oracle._lib = oracle.load(path)
    try:
        for name, fn in CHECKS:
            try:
                fn(oracle)
            except (AssertionError, ValueError, NotImplementedError, FloatingPointError):
                return name
        return None
    finally:
        oracle._lib = saved


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


def test_unmutated_build_passes_every_check(source, tmp_path):
    assert _first_failure(_build(tmp_path, source, "orig")) is None


@pytest.mark.parametrize("mid,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(source, tmp_path, mid, old, new):
    assert source.count(old) == 1, f"mutation {mid}: pattern not found once in ctoracle.c"
    caught = _first_failure(_build(tmp_path, source.replace(old, new), mid))
    print(f"{mid}: caught by {caught}")
    assert caught is not None, f"mutation {mid} passes every pin"
