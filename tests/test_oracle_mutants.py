"""Plant plausible mistakes in a copy of the oracle source (on the CPU) and
check that at least one pin catches each of them. This is what makes the
pins worth trusting: a dropped term, a wrong sign, a transposed index, the
wrong rounding rule or a fused multiply-add all fail."""
import os

import numpy as np
import pytest

import oracle
from oracle import build as obuild
import pins
import pins_fit
import pins_demosaic
import pins_demosaic_gradient

SRC = os.path.join(os.path.dirname(obuild.__file__), "oracle.cpp")

MUTANTS = {
    "drop_a2": [("acc = acc + a[2];", "acc = acc + 0.0;")],
    "drop_a3": [("double acc = a[3];", "double acc = 0.0;")],
    "sign_a0": [("acc = acc + a[0];", "acc = acc - a[0];")],
    "swap_a1_a2": [("acc = acc + a[2];", "acc = acc + a[@];"),
                   ("acc = acc + a[1];", "acc = acc + a[2];"),
                   ("acc = acc + a[@];", "acc = acc + a[1];")],
    "floor_plus_half": [("std::round(acc)", "std::floor(acc + 0.5)")],
    "half_to_even": [("std::round(acc)", "std::nearbyint(acc)")],
    "fused_last_step": [("acc = acc * x;\n    acc = acc + a[0];", "acc = std::fma(acc, x, a[0]);")],
    "single_precision": [("double acc = a[3];", "float acc = (float)a[3];")],
    "clamp_top_off_by_one": [("if (r >= top) return (uint16_t)(levels - 1);",
                              "if (r >= top) return (uint16_t)(levels);")],
    "mask_not_min": [("if (v > top) v = top;", "v = (uint16_t)(v & top);")],
    "lut_ignores_band": [("out[pix] = lut[row * (size_t)levels + (size_t)v];",
                          "out[pix] = lut[(size_t)d * (size_t)levels + (size_t)v];")],
    "image_stride_swap": [
        ("const size_t pix = ((size_t)b * (size_t)lines + (size_t)n) * (size_t)detectors\n"
         "                                   + (size_t)d;\n                uint16_t v = dn[pix];",
         "const size_t pix = ((size_t)b * (size_t)detectors + (size_t)d) * (size_t)lines\n"
         "                                   + (size_t)n;\n                uint16_t v = dn[pix];")],
    "lut_transposed": [("lut[row * (size_t)levels + (size_t)v] = oracle_lut_entry",
                        "lut[(size_t)v * (size_t)bands * (size_t)detectors + row] = oracle_lut_entry")],
    "level_off_by_one": [("const double x = (double)v;", "const double x = (double)(v + 1);")],
}


# Plausible mistakes in the least-squares fit (§III.B), two of them the
# paper's own misprints taken literally.
MUTANTS_FIT = {
    "fit_a00_is_one": [("M[j][k] = S[j + k];", "M[j][k] = j + k == 0 ? 1.0 : S[j + k];")],
    "fit_b_without_xj": [("if (k <= m) T[k] = T[k] + p * yi;", "if (k <= m) T[k] = T[k] + yi;")],
    "fit_power_off_by_one": [("M[j][k] = S[j + k];", "M[j][k] = S[j + k < 2 * m ? j + k + 1 : j + k];")],
    "fit_pivot_row_not_scaled": [("for (int k = 0; k < w; ++k) M[c][k] = M[c][k] / piv;", "")],
    "fit_drops_first_point": [("for (int32_t i = 0; i < points; ++i) {\n                const double xi",
                               "for (int32_t i = 1; i < points; ++i) {\n                const double xi")],
    "fit_target_ignores_band": [("const double yi = y[(size_t)b * (size_t)points + (size_t)i];",
                                 "const double yi = y[(size_t)i];")],
    "fit_padding_one": [("a[j] = 0.0;", "a[j] = 1.0;")],
    "fit_x_stride_swap": [("const double xi = x[((size_t)b * (size_t)points + (size_t)i) * (size_t)detectors\n"
                           "                                    + (size_t)d];",
                           "const double xi = x[((size_t)b * (size_t)detectors + (size_t)d) * (size_t)points\n"
                           "                                    + (size_t)i];")],
}


# Plausible mistakes in the bilinear demosaicing (§III.A).
MUTANTS_DEMOSAIC = {
    "dm_truncating_average": [("R = self;\n                    G = (cross + 2) >> 2;",
                               "R = self;\n                    G = cross >> 2;")],
    "dm_green_red_row_swapped": [("G = self;\n                    R = (horiz + 1) >> 1;\n"
                                  "                    B = (vert + 1) >> 1;",
                                  "G = self;\n                    R = (vert + 1) >> 1;\n"
                                  "                    B = (horiz + 1) >> 1;")],
    "dm_edge_repeated": [("if (i < 0) return -i;", "if (i < 0) return -i - 1;"),
                         ("if (i >= n) return 2 * (n - 1) - i;", "if (i >= n) return 2 * n - 1 - i;")],
    "dm_pattern_bggr": [("const bool red_row = (r % 2) == 0;", "const bool red_row = (r % 2) == 1;"),
                        ("const bool red_col = (c % 2) == 0;", "const bool red_col = (c % 2) == 1;")],
    "dm_planes_swapped": [("out[p] = (uint16_t)R;", "out[p] = (uint16_t)B;"),
                          ("out[2 * plane + p] = (uint16_t)B;", "out[2 * plane + p] = (uint16_t)R;")],
    "dm_diag_for_green": [("B = self;\n                    G = (cross + 2) >> 2;",
                           "B = self;\n                    G = (diag + 2) >> 2;")],
}

MUTANTS_GRADIENT = {
    "gr_direction_swapped": [("if (dh < dv) G = (2 * (gl + gr) + lh + 2) >> 2;",
                              "if (dh > dv) G = (2 * (gl + gr) + lh + 2) >> 2;")],
    "gr_no_laplacian": [("if (dh < dv) G = (2 * (gl + gr) + lh + 2) >> 2;",
                         "if (dh < dv) G = (2 * (gl + gr) + 2) >> 2;")],
    "gr_laplacian_sign": [("const int32_t lv = 2 * C - at(r - 2, c) - at(r + 2, c);",
                           "const int32_t lv = at(r - 2, c) + at(r + 2, c) - 2 * C;")],
    "gr_tie_horizontal": [("else G = (2 * (gl + gr + gu + gd) + lh + lv + 4) >> 3;",
                           "else G = (2 * (gl + gr) + lh + 2) >> 2;")],
    "gr_gradient_no_abs": [("std::abs(gl - gr)", "(gl - gr)")],
    "gr_no_clamp": [("G = clamp16(G);", "")],
    "gr_pair_raw_green": [("2 * g0 - g_at(r1, c1)", "2 * g0 - at(r1, c1)")],
    "gr_own_green_raw": [("const int32_t g0 = g_at(r, c);", "const int32_t g0 = at(r, c);")],
    "gr_diagonals_swapped": [("if (dn < dp) v = (n1 + n2 + ln + 1) >> 1;",
                              "if (dn > dp) v = (n1 + n2 + ln + 1) >> 1;")],
    "gr_diag_tie_truncates": [("else v = (n1 + n2 + p1 + p2 + ln + lp + 2) >> 2;",
                               "else v = (n1 + n2 + p1 + p2 + ln + lp) >> 2;")],
    "gr_green_pairs_swapped": [("red = pair(r, c - 1, r, c + 1);\n                    blue = pair(r - 1, c, r + 1, c);",
                                "red = pair(r - 1, c, r + 1, c);\n                    blue = pair(r, c - 1, r, c + 1);")],
}


def _saturation_pin(o):
    L = 1024
    lut = (np.arange(2 * L, dtype=np.int64).reshape(1, 2, L) % 997).astype(np.uint16)
    dn = np.array([[[1023, 1024], [2047, 65535]]], dtype=np.uint16)
    out = o.correct(dn, lut)
    assert out.tolist() == [[[lut[0, 0, 1023], lut[0, 1, 1023]],
                             [lut[0, 0, 1023], lut[0, 1, 1023]]]]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"mutation site not unique for {name}: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "oracle_mutant.cpp"
    path.write_text(src)
    lib = obuild.build(src=str(path), out=str(tmp_path / "liboracle_mutant.so"))
    o = oracle.Oracle(lib)
    caught = []
    for pin in pins.ALL_PINS + [_saturation_pin]:
        try:
            pin(o)
        except AssertionError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} passed every pin"


@pytest.mark.parametrize("name", sorted(MUTANTS_FIT))
def test_fit_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTANTS_FIT[name]:
        assert src.count(old) == 1, f"mutation site not unique for {name}: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "oracle_mutant.cpp"
    path.write_text(src)
    lib = obuild.build(src=str(path), out=str(tmp_path / "liboracle_mutant.so"))
    o = oracle.Oracle(lib)
    caught = []
    for pin in pins_fit.ALL_FIT_PINS:
        try:
            pin(o)
        except AssertionError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} passed every fit pin"


@pytest.mark.parametrize("name", sorted(MUTANTS_DEMOSAIC))
def test_demosaic_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTANTS_DEMOSAIC[name]:
        assert src.count(old) == 1, f"mutation site not unique for {name}: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "oracle_mutant.cpp"
    path.write_text(src)
    lib = obuild.build(src=str(path), out=str(tmp_path / "liboracle_mutant.so"))
    o = oracle.Oracle(lib)
    caught = []
    for pin in pins_demosaic.ALL_DEMOSAIC_PINS:
        try:
            pin(o)
        except AssertionError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} passed every demosaicing pin"


@pytest.mark.parametrize("name", sorted(MUTANTS_GRADIENT))
def test_gradient_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTANTS_GRADIENT[name]:
        assert src.count(old) == 1, f"mutation site not unique for {name}: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / "oracle_mutant.cpp"
    path.write_text(src)
    lib = obuild.build(src=str(path), out=str(tmp_path / "liboracle_mutant.so"))
    o = oracle.Oracle(lib)
    caught = []
    for pin in pins_demosaic_gradient.ALL_GRADIENT_PINS:
        try:
            pin(o)
        except AssertionError:
            caught.append(pin.__name__)
            break
    assert caught, f"mutant {name} passed every gradient demosaicing pin"
