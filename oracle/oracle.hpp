// Reference CPU implementation of look-up-table generation and image correction.
//
// TEST INFRASTRUCTURE ONLY. This code is the oracle that the GPU library is
// checked against. Only the test suite, the smoke check and the benchmark's
// CPU-baseline leg may load it. It shares no source, header, table or helper
// with the GPU library, and the GPU library never calls it.
//
// The paper (Banerjee & Dave, §I) names LUT generation with image correction
// as a typical compute-heavy task but gives no formula for it. The definition
// fixed here, and used by both sides, is:
//
//   LUT build, for every band b, detector d and level v in [0, L):
//     lut[b][d][v] = clamp(round_half_away(P_bd(v)), 0, L-1)
//     P_bd(v) = ((a3*v + a2)*v + a1)*v + a0        (Horner, binary64, no FMA)
//     with a0..a3 = coeffs[b][d][0..3] (ascending degree; quadratics use a3 = 0)
//   Clamp happens in binary64 before the integer conversion:
//     NaN, negatives, -0 and -Inf give 0;  values >= L-1 (and +Inf) give L-1.
//
//   Correction (per pixel gather), band-sequential push-broom image [B][N][D]:
//     out[b][n][d] = lut[b][d][min(dn[b][n][d], L-1)]
//
//   Least-squares calibration fit (§III.B, case study 2), per band b and detector d,
//   over n points (x_i, y_i) = (x[b][i][d], y[b][i]), i < n, polynomial order m <= 3:
//     normal equations  A a = B,  A[j][k] = sum_i x_i^(j+k)  (A[0][0] = n),
//                                 B[j]    = sum_i x_i^j * y_i,   j, k = 0..m
//     solved as a = A^-1 B, A^-1 by Gauss-Jordan elimination with partial pivoting.
//   Powers by repeated multiplication, sums over i in increasing order, binary64,
//   no FMA. coeffs[b][d][0..3] = a_0..a_m, then +0.0 above the order; a singular
//   system (no nonzero pivot) gives NaN in all four.
//
//   Bilinear Bayer demosaicing (§III.A, case study 1): a raw image [H][W] of
//   16-bit samples behind an RGGB colour filter (R at even row and even
//   column, B at odd row and odd column, G elsewhere) becomes three planes
//   rgb[c][H][W]. Each pixel keeps its own sample for its own colour; each
//   missing colour is the average of the neighbours of that colour among its
//   8 direct neighbours, rounded half up in integers:
//     at R: G = (N + S + E + W + 2) >> 2,  B = (NW + NE + SW + SE + 2) >> 2
//     at B: G = (N + S + E + W + 2) >> 2,  R = (NW + NE + SW + SE + 2) >> 2
//     at G in a red row:  R = (E + W + 1) >> 1,  B = (N + S + 1) >> 1
//     at G in a blue row: B = (E + W + 1) >> 1,  R = (N + S + 1) >> 1
//   Outside the image, rows and columns are mirrored about the edge sample
//   (index -1 reads 1, index H reads H-2), which keeps the colour pattern.
//   H and W are even.
//
//   Gradient-based demosaicing (named in the paper's task list, §II, and in §III.A; the method
//   is Hamilton & Adams' adaptive colour plane interpolation, U.S. Patent
//   5,629,734, 1997), same filter, borders and layout, integer arithmetic:
//   stage 1, green at R and B pixels (C = own colour, Cl2/Cr2/Cu2/Cd2 the same
//   colour two pixels away, Gl/Gr/Gu/Gd the green neighbours):
//     dH = |Gl - Gr| + |2C - Cl2 - Cr2|,  dV = |Gu - Gd| + |2C - Cu2 - Cd2|
//     dH < dV:  G = (2 (Gl + Gr) + 2C - Cl2 - Cr2 + 2) >> 2
//     dV < dH:  G = (2 (Gu + Gd) + 2C - Cu2 - Cd2 + 2) >> 2
//     equal:    G = (2 (Gl + Gr + Gu + Gd) + 4C - Cl2 - Cr2 - Cu2 - Cd2 + 4) >> 3
//   stage 2, with the green plane G' of stage 1 (G' = G at green pixels):
//     at a green pixel, each missing colour X from its two neighbours X1, X2
//     (horizontal for the colour of the row, vertical for the other):
//       X = (X1 + X2 + 2 G - G'1 - G'2 + 1) >> 1
//     at a B (R) pixel, R (B) from the diagonal pair with the smaller
//       |X1 - X2| + |2 G' - G'1 - G'2| (both pairs when equal:
//       (sum of 4 X + 4 G' - sum of 4 G' + 2) >> 2), else (X1 + X2 + 2 G' - G'1 - G'2 + 1) >> 1
//   >> is an arithmetic shift (floor); every interpolated value is clamped to
//   [0, 65535]. H and W are even and at least 4.
//
// Parity pins (independent of this file) live in tests/test_oracle_pins.py,
// tests/test_oracle_fit_pins.py, tests/test_oracle_demosaic_pins.py and
// tests/test_oracle_demosaic_gradient_pins.py.
#pragma once
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

// One LUT entry: binary64 Horner over a[0..3] at integer level v, then
// round half away from zero and clamp to [0, levels-1].
uint16_t oracle_lut_entry(const double* a, int32_t v, int32_t levels);

// lut[(b*D + d)*L + v] for all b < bands, d < detectors, v < levels.
// coeffs is [bands][detectors][4] binary64.
void oracle_lut_build(const double* coeffs, int32_t bands, int32_t detectors,
                      int32_t levels, uint16_t* lut);

// out[(b*N + n)*D + d] = lut[(b*D + d)*L + min(dn[(b*N + n)*D + d], L-1)].
void oracle_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                    int32_t detectors, int32_t bands, int32_t levels,
                    uint16_t* out);

// Brute force: the same result as oracle_correct(oracle_lut_build(...)), but
// every pixel evaluates its polynomial directly, without any table.
void oracle_pixel(const double* coeffs, const uint16_t* dn, int64_t lines,
                  int32_t detectors, int32_t bands, int32_t levels,
                  uint16_t* out);

// Least-squares fit (definition above). x is [bands][points][detectors],
// y is [bands][points], coeffs is [bands][detectors][4]; 0 <= order <= 3.
void oracle_fit(const double* x, const double* y, int32_t bands, int32_t points,
                int32_t detectors, int32_t order, double* coeffs);

// Bilinear demosaicing (definition above) of `images` raw images
// [images][height][width] into rgb [images][3][height][width].
void oracle_demosaic(const uint16_t* raw, int32_t images, int32_t height, int32_t width,
                     uint16_t* rgb);

// Gradient-based (adaptive colour plane) demosaicing, definition above.
void oracle_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t height,
                              int32_t width, uint16_t* rgb);

#ifdef __cplusplus
}
#endif
