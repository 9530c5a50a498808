"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the pin suite against the
copy; the suite must fail.  The mistakes are the ones a reader could make
when writing the method down: a dropped term, a wrong sign, a transposed
operand, a cumulative instead of a from-the-original displacement, a wrong
tie-break, a missed winding swap.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "drop_blue_term": ("w[c] = (mr * cam->right[c] + mg * cam->up[c]) + mb * cam->forward[c];",
                       "w[c] = (mr * cam->right[c] + mg * cam->up[c]);"),
    "red_sign": ("float mr = 2.0f * prev[0] - 1.0f;", "float mr = 1.0f - 2.0f * prev[0];"),
    "red_green_swapped": ("float mg = 2.0f * prev[1] - 1.0f;", "float mg = 2.0f * prev[0] - 1.0f;"),
    "row_order_flipped": ("float fy = 1.0f - (float)(2 * y + 1) / (float)H;",
                          "float fy = (float)(2 * y + 1) / (float)H - 1.0f;"),
    "eye_and_dir_both_lambda_dir": ("dp[c] = q[c] + lambda_dir * w[c];",
                                    "dp[c] = q[c] + (lambda_eye + lambda_dir) * w[c];"),
    "edge_function_transposed": ("float V = Ax * Cy - Ay * Cx;", "float V = Ay * Cx - Ax * Cy;"),
    "no_winding_swap": ("if (d[kz] < 0.0f) { int tmp = kx; kx = ky; ky = tmp; }", ""),
    "t_includes_zero": ("if (!(t > 0.0f)) return 0;", "if (t < 0.0f) return 0;"),
    "farthest_hit": ("if (orc_intersect(o, d, tr, tr + 3, tr + 6, &t, &fr) && t < best) {",
                     "if (orc_intersect(o, d, tr, tr + 3, tr + 6, &t, &fr) && (best == INFINITY || t > best)) {"),
    "tie_highest_id": ("if (!found || t < best || (t == best && id < best_id)) {",
                       "if (!found || t < best || (t == best && id > best_id)) {"),
    "front_back_swapped": ("if (!front) for (int c = 0; c < 3; ++c) n[c] = -n[c];",
                           "if (front) for (int c = 0; c < 3; ++c) n[c] = -n[c];"),
    "no_clamp": ("rgb[c] = clamp01(s->rgb[3 * id + c] * shade);", "rgb[c] = s->rgb[3 * id + c] * shade;"),
    "cumulative_displacement": ("const float* prev = k == 0 ? NULL : &out[(size_t)(k - 1) * P * 3];",
                                "const float* prev = k < 2 ? NULL : &out[(size_t)(k - 2) * P * 3];"),
    "aspect_inverted": ("float aspect = (float)W / (float)H;", "float aspect = (float)H / (float)W;"),
    "depth_signed_not_abs": ("float kz = (z < INFINITY) ? fabsf(z - z0) : 0.0f;",
                             "float kz = (z < INFINITY) ? (z - z0) : 0.0f;"),
    "depth_miss_displaced": ("float kz = (z < INFINITY) ? fabsf(z - z0) : 0.0f;",
                             "float kz = (z < INFINITY) ? fabsf(z - z0) : 1.0f;"),
    "cross_product_reversed": ("w[0] = C[1] * N[2] - C[2] * N[1];", "w[0] = C[2] * N[1] - C[1] * N[2];"),
    "view_direction_unnormalised": ("for (int c = 0; c < 3; ++c) C[c] = q[c] / ql;",
                                    "for (int c = 0; c < 3; ++c) C[c] = q[c];"),
    "aux_depth_is_t": ("        aux[0] = ((P[0] - cam->eye[0])", "        aux[0] = t + 0.0f * ((P[0] - cam->eye[0])"),
    "gather_green_down": ("float py = ((float)y + 0.5f) - mg * max_smudge;", "float py = ((float)y + 0.5f) + mg * max_smudge;"),
    "gather_mirror_off_by_one": ("return m < n ? m : p - 1 - m;", "return m < n ? m : p - m;"),
    "gather_wrap_negative": ("{ int m = i % n; return m < 0 ? m + n : m; }", "{ int m = i % n; return m < 0 ? 0 : m; }"),
    "gather_rounds_to_nearest": ("int sx = edge_index((int)floorf(px), W, edge);", "int sx = edge_index((int)roundf(px), W, edge);"),
    # the BVH's boxes are no longer widened beyond the triangles' own bounds:
    # rays along box faces then lose hits the brute-force scan finds
    "bvh_box_widening_dropped": ("const double pad = ldexp(s->radius + omax, -18);", "const double pad = 0.0;"),
}

# Pin files each mutation runs against (default: the pin suite).
PIN_FILES = ["test_oracle_pins.py", "test_oracle_modes.py", "test_oracle_gather.py"]
MUTATION_FILES = {"bvh_box_widening_dropped": ["test_oracle_bvh_fullsize.py"]}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(os.path.join(ROOT, "oracle", "rcp_oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor not found: {name}"
    (tmp_path / "rcp_oracle.c").write_text(src.replace(old, new))
    (tmp_path / "rcp_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "rcp_oracle.h")).read())
    lib = tmp_path / "librcp_oracle_mut.so"
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, "-o", str(lib), str(tmp_path / "rcp_oracle.c"), "-lm"])
    env = dict(os.environ, RCP_ORACLE_LIB=str(lib))
    files = [os.path.join(ROOT, "tests", f) for f in MUTATION_FILES.get(name, PIN_FILES)]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutation {name}:\n{r.stdout[-2000:]}"
