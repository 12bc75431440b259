"""Planted mistakes in the oracle must each fail at least one pin (CPU only).

Each mutant is a copy of ``oracle/bp_oracle.c`` with one plausible mistake
(a dropped term, a wrong sign or index, a transposed operand, a wrong edge
convention), compiled with gcc into a temporary library.  The pins of
``oracle_pins`` run against it; the test passes only if some pin fails.
"""
import os

import pytest

import oracle
import oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "bp_oracle.c")

MUTANTS = {
    # (truncation instead of floor is no mistake here: the tent weights of the taps it would
    # pick wrongly are 0, so the sum is unchanged -- an equivalent mutant, not planted)
    "nearest_not_floor": ("const long c0 = (long)floor(s), r0 = (long)floor(t);",
                          "const long c0 = (long)round(s), r0 = (long)round(t);"),
    "bounds_swapped": ("if (i < 0 || i >= W || j < 0 || j >= H)", "if (i < 0 || i >= H || j < 0 || j >= W)"),
    "weight_1_over_w": ("return val / (w * w);", "return val / w;"),
    "matrix_transposed": ("double u = A[0] * wx + A[1] * wy + A[2] * wz + A[3];",
                          "double u = A[0] * wx + A[3] * wy + A[6] * wz + A[9];"),
    "taps_transposed": ("sum += pixel(img, W, H, i, j) * tent(s - (double)i) * wt;",
                        "sum += pixel(img, W, H, j, i) * tent(s - (double)i) * wt;"),
    "column_weight_from_row": ("sum += pixel(img, W, H, i, j) * tent(s - (double)i) * wt;",
                               "sum += pixel(img, W, H, i, j) * tent(t - (double)i) * wt;"),
    "neighbourhood_to_the_left": ("for (long i = c0; i <= c0 + 1; ++i)", "for (long i = c0 - 1; i <= c0; ++i)"),
    "row_weights_swapped": ("const double wt = tent(t - (double)j);", "const double wt = 1.0 - tent(t - (double)j);"),
    "no_w_test": ("if (!(w > 0.0))\n        return 0.0;", "if (0)\n        return 0.0;"),
    "voxel_corner_not_centre": ("double wx = jb->O[0] + jb->MM * (double)(jb->x0 + ix);",
                                "double wx = jb->O[0] + jb->MM * ((double)(jb->x0 + ix) + 0.5);"),
    "dropped_v_offset": ("double v = A[4] * wx + A[5] * wy + A[6] * wz + A[7];",
                         "double v = A[4] * wx + A[5] * wy + A[6] * wz;"),
    "edge_guard_open": ("if (!(s > -1.0 && s < (double)W && t > -1.0 && t < (double)H))",
                        "if (!(s > 0.0 && s < (double)W && t > -1.0 && t < (double)H))"),
    "skip_first_view": ("                for (int k = 0; k < jb->n_views; ++k) {",
                        "                for (int k = 1; k < jb->n_views; ++k) {"),
    "points_skip_last_view": ("        for (int k = 0; k < jb->n_views; ++k) {\n            const double c",
                              "        for (int k = 0; k < jb->n_views - 1; ++k) {\n            const double c"),
    "overwrite_not_accumulate": ("double sum = *voxel;", "double sum = 0.0;"),
    "magnitude_mode_signed": ("                    sum += jb->absolute ? fabs(c) : c;",
                              "                    sum += c;"),
    "points_magnitude_mode_signed": ("jb->P + 12 * (long)k, wx, wy, wz);\n            sum += jb->absolute ? fabs(c) : c;",
                                     "jb->P + 12 * (long)k, wx, wy, wz);\n            sum += c;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / "bp_mutant.c"
    src.write_text(text.replace(old, new))
    lib = oracle.load_library(oracle.build_library(str(src), str(tmp_path / "bp_mutant.so")))
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError as e:  # the pin caught the mutant
            failed.append(f"{pin.__name__}: {str(e)[:80]}")
    assert failed, f"no pin catches mutant {name}"
