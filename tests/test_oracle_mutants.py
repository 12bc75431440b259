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
    "trunc_not_floor": ("double fx = floor(ix), fy = floor(iy);", "double fx = trunc(ix), fy = trunc(iy);"),
    "bounds_swapped": ("if (i < 0 || i >= W || j < 0 || j >= H)", "if (i < 0 || i >= H || j < 0 || j >= W)"),
    "weight_1_over_w": ("return val / (w * w);", "return val / w;"),
    "matrix_transposed": ("double u = A[0] * wx + A[1] * wy + A[2] * wz + A[3];",
                          "double u = A[0] * wx + A[3] * wy + A[6] * wz + A[9];"),
    "taps_swapped": ("double valtl = pixel(img, W, H, iix, iiy + 1);",
                     "double valtl = pixel(img, W, H, iix + 1, iiy);"),
    "fraction_sign": ("double scalex = ix - fx;", "double scalex = fx - ix;"),
    "weight_rows_swapped": ("return (1.0 - scaley) * valb + scaley * valt;",
                            "return scaley * valb + (1.0 - scaley) * valt;"),
    "no_w_test": ("if (!(w > 0.0))\n        return 0.0;", "if (0)\n        return 0.0;"),
    "voxel_corner_not_centre": ("double wx = jb->O[0] + jb->MM * (double)(jb->x0 + ix);",
                                "double wx = jb->O[0] + jb->MM * ((double)(jb->x0 + ix) + 0.5);"),
    "dropped_v_offset": ("double v = A[4] * wx + A[5] * wy + A[6] * wz + A[7];",
                         "double v = A[4] * wx + A[5] * wy + A[6] * wz;"),
    "edge_guard_open": ("if (!(ix > -1.0 && ix < (double)W && iy > -1.0 && iy < (double)H))",
                        "if (!(ix > 0.0 && ix < (double)W && iy > -1.0 && iy < (double)H))"),
    "skip_first_view": ("                for (int k = 0; k < jb->n_views; ++k)",
                        "                for (int k = 1; k < jb->n_views; ++k)"),
    "points_skip_last_view": ("        for (int k = 0; k < jb->n_views; ++k)\n            sum +=",
                              "        for (int k = 0; k < jb->n_views - 1; ++k)\n            sum +="),
    "overwrite_not_accumulate": ("double sum = *voxel;", "double sum = 0.0;"),
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
