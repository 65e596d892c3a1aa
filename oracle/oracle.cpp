// Reference CPU implementation of look-up-table generation and image correction.
//
// TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
// benchmark's CPU-baseline leg, never by the GPU library. Plain, single
// threaded, slow on purpose: every loop follows the definition in oracle.hpp
// with no blocking, fusion or reordering.
//
// Built with the host compiler and -O2 -ffp-contract=off -fno-fast-math on
// x86-64 (SSE2 binary64, so every + and * below is one correctly rounded
// IEEE-754 operation and nothing is fused into an FMA).
//
// Paper: Banerjee & Dave, "GPGPU Based Parallelized Client-Server Framework
// for Providing High Performance Computation Support", §I, which names LUT
// generation and image correction as the task; the paper gives no formula,
// so the definition in oracle.hpp is the one this project fixes.
#include "oracle.hpp"

#include <cmath>
#include <cstdlib>
#include <cstddef>

extern "C" {

uint16_t oracle_lut_entry(const double* a, int32_t v, int32_t levels) {
    // The level is an integer below 2^16, so the conversion is exact.
    const double x = (double)v;
    // Horner from the cubic coefficient down; one rounding per operation.
    double acc = a[3];
    acc = acc * x;
    acc = acc + a[2];
    acc = acc * x;
    acc = acc + a[1];
    acc = acc * x;
    acc = acc + a[0];
    // C round(): nearest integer, halfway cases away from zero. Exact.
    const double r = std::round(acc);
    // Clamp in binary64 before converting; NaN fails the first test.
    if (!(r > 0.0)) return 0;
    const double top = (double)(levels - 1);
    if (r >= top) return (uint16_t)(levels - 1);
    return (uint16_t)r;
}

void oracle_lut_build(const double* coeffs, int32_t bands, int32_t detectors,
                      int32_t levels, uint16_t* lut) {
    for (int32_t b = 0; b < bands; ++b) {
        for (int32_t d = 0; d < detectors; ++d) {
            const size_t row = (size_t)b * (size_t)detectors + (size_t)d;
            const double* a = coeffs + row * 4;
            for (int32_t v = 0; v < levels; ++v) {
                lut[row * (size_t)levels + (size_t)v] = oracle_lut_entry(a, v, levels);
            }
        }
    }
}

void oracle_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                    int32_t detectors, int32_t bands, int32_t levels,
                    uint16_t* out) {
    const uint16_t top = (uint16_t)(levels - 1);
    for (int32_t b = 0; b < bands; ++b) {
        for (int64_t n = 0; n < lines; ++n) {
            for (int32_t d = 0; d < detectors; ++d) {
                const size_t pix = ((size_t)b * (size_t)lines + (size_t)n) * (size_t)detectors
                                   + (size_t)d;
                uint16_t v = dn[pix];
                if (v > top) v = top;
                const size_t row = (size_t)b * (size_t)detectors + (size_t)d;
                out[pix] = lut[row * (size_t)levels + (size_t)v];
            }
        }
    }
}

void oracle_pixel(const double* coeffs, const uint16_t* dn, int64_t lines,
                  int32_t detectors, int32_t bands, int32_t levels,
                  uint16_t* out) {
    for (int32_t b = 0; b < bands; ++b) {
        for (int64_t n = 0; n < lines; ++n) {
            for (int32_t d = 0; d < detectors; ++d) {
                const size_t pix = ((size_t)b * (size_t)lines + (size_t)n) * (size_t)detectors
                                   + (size_t)d;
                int32_t v = dn[pix];
                if (v > levels - 1) v = levels - 1;
                const double* a = coeffs + ((size_t)b * (size_t)detectors + (size_t)d) * 4;
                out[pix] = oracle_lut_entry(a, v, levels);
            }
        }
    }
}

// Case study 2 of the paper (§III.B): the least-squares polynomial fit,
// applied per detector to its calibration points. Setting the first
// derivatives of the squared error to zero gives the normal equations
// A a = B with A[j][k] = sum_i x_i^(j+k) and B[j] = sum_i x_i^j y_i (the
// printed derivative lacks the factor -2 x_i^j and the printed A starts with
// 1 where sum_i x_i^0 = n belongs; both are read as the standard equations).
// The paper solves them as a = A^-1 B; A^-1 comes from Gauss-Jordan
// elimination of [A | I] with partial pivoting.
void oracle_fit(const double* x, const double* y, int32_t bands, int32_t points,
                int32_t detectors, int32_t order, double* coeffs) {
    const int m = order;
    const int w = 2 * (m + 1);  // columns of [A | I]
    for (int32_t b = 0; b < bands; ++b) {
        for (int32_t d = 0; d < detectors; ++d) {
            // Power sums S[k] = sum_i x_i^k (k <= 2m) and T[j] = sum_i x_i^j y_i.
            double S[7] = {0, 0, 0, 0, 0, 0, 0};
            double T[4] = {0, 0, 0, 0};
            for (int32_t i = 0; i < points; ++i) {
                const double xi = x[((size_t)b * (size_t)points + (size_t)i) * (size_t)detectors
                                    + (size_t)d];
                const double yi = y[(size_t)b * (size_t)points + (size_t)i];
                double p = 1.0;  // x_i^k
                for (int k = 0; k <= 2 * m; ++k) {
                    S[k] = S[k] + p;
                    if (k <= m) T[k] = T[k] + p * yi;
                    p = p * xi;
                }
            }
            // [A | I]
            double M[4][8];
            for (int j = 0; j <= m; ++j) {
                for (int k = 0; k <= m; ++k) {
                    M[j][k] = S[j + k];
                    M[j][m + 1 + k] = j == k ? 1.0 : 0.0;
                }
            }
            bool singular = false;
            for (int c = 0; c <= m; ++c) {
                // Pivot: the first row (from c down) of largest magnitude in column c.
                int pr = c;
                double best = std::fabs(M[c][c]);
                for (int r = c + 1; r <= m; ++r) {
                    if (std::fabs(M[r][c]) > best) {
                        best = std::fabs(M[r][c]);
                        pr = r;
                    }
                }
                if (!(best > 0.0)) {
                    singular = true;
                    break;
                }
                if (pr != c) {
                    for (int k = 0; k < w; ++k) {
                        const double t = M[c][k];
                        M[c][k] = M[pr][k];
                        M[pr][k] = t;
                    }
                }
                const double piv = M[c][c];
                for (int k = 0; k < w; ++k) M[c][k] = M[c][k] / piv;
                for (int r = 0; r <= m; ++r) {
                    if (r == c) continue;
                    const double f = M[r][c];
                    for (int k = 0; k < w; ++k) M[r][k] = M[r][k] - f * M[c][k];
                }
            }
            double* a = coeffs + ((size_t)b * (size_t)detectors + (size_t)d) * 4;
            for (int j = 0; j < 4; ++j) {
                if (singular) {
                    a[j] = std::nan("");
                } else if (j > m) {
                    a[j] = 0.0;
                } else {
                    // a_j = sum_k (A^-1)[j][k] * B[k]
                    double s = 0.0;
                    for (int k = 0; k <= m; ++k) s = s + M[j][m + 1 + k] * T[k];
                    a[j] = s;
                }
            }
        }
    }
}

// Case study 1 of the paper (§III.A): bilinear demosaicing of a Bayer image.
// The paper describes the four cases (red pixel, blue pixel, green pixel in
// a red row, green pixel in a blue row) and the averaging over the 8 direct
// neighbours; it does not say how averages are rounded or what happens at
// the border. Read here: integer averages rounded half up, and mirrored
// indices outside the image.
static int32_t mirror(int32_t i, int32_t n) {
    if (i < 0) return -i;
    if (i >= n) return 2 * (n - 1) - i;
    return i;
}

void oracle_demosaic(const uint16_t* raw, int32_t images, int32_t height, int32_t width,
                     uint16_t* rgb) {
    const size_t plane = (size_t)height * (size_t)width;
    for (int32_t k = 0; k < images; ++k) {
        const uint16_t* im = raw + (size_t)k * plane;
        uint16_t* out = rgb + (size_t)k * 3 * plane;
        auto at = [&](int32_t r, int32_t c) -> uint32_t {
            return im[(size_t)mirror(r, height) * (size_t)width + (size_t)mirror(c, width)];
        };
        for (int32_t r = 0; r < height; ++r) {
            for (int32_t c = 0; c < width; ++c) {
                const uint32_t self = at(r, c);
                const uint32_t cross = at(r - 1, c) + at(r + 1, c) + at(r, c - 1) + at(r, c + 1);
                const uint32_t diag = at(r - 1, c - 1) + at(r - 1, c + 1) + at(r + 1, c - 1)
                                      + at(r + 1, c + 1);
                const uint32_t horiz = at(r, c - 1) + at(r, c + 1);
                const uint32_t vert = at(r - 1, c) + at(r + 1, c);
                uint32_t R, G, B;
                const bool red_row = (r % 2) == 0;
                const bool red_col = (c % 2) == 0;
                if (red_row && red_col) {          // red pixel
                    R = self;
                    G = (cross + 2) >> 2;
                    B = (diag + 2) >> 2;
                } else if (!red_row && !red_col) {  // blue pixel
                    B = self;
                    G = (cross + 2) >> 2;
                    R = (diag + 2) >> 2;
                } else if (red_row) {               // green pixel in a red row
                    G = self;
                    R = (horiz + 1) >> 1;
                    B = (vert + 1) >> 1;
                } else {                            // green pixel in a blue row
                    G = self;
                    B = (horiz + 1) >> 1;
                    R = (vert + 1) >> 1;
                }
                const size_t p = (size_t)r * (size_t)width + (size_t)c;
                out[p] = (uint16_t)R;
                out[plane + p] = (uint16_t)G;
                out[2 * plane + p] = (uint16_t)B;
            }
        }
    }
}

// Gradient-based demosaicing: the paper lists it beside bilinear demosaicing
// (§II) without describing it; the method followed is Hamilton & Adams'
// adaptive colour plane interpolation (U.S. Patent 5,629,734): interpolate
// green along the direction of the smaller gradient, with a second-order
// correction from the pixel's own colour, then red and blue from colour
// differences with the interpolated green. Integer arithmetic as defined in
// oracle.hpp.
static int32_t clamp16(int32_t v) { return v < 0 ? 0 : (v > 65535 ? 65535 : v); }

void oracle_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t height,
                              int32_t width, uint16_t* rgb) {
    const size_t plane = (size_t)height * (size_t)width;
    for (int32_t k = 0; k < images; ++k) {
        const uint16_t* im = raw + (size_t)k * plane;
        uint16_t* out = rgb + (size_t)k * 3 * plane;
        uint16_t* gp = out + plane;  // the green plane, written by stage 1
        auto at = [&](int32_t r, int32_t c) -> int32_t {
            return im[(size_t)mirror(r, height) * (size_t)width + (size_t)mirror(c, width)];
        };
        auto g_at = [&](int32_t r, int32_t c) -> int32_t {
            return gp[(size_t)mirror(r, height) * (size_t)width + (size_t)mirror(c, width)];
        };
        // Stage 1: green everywhere.
        for (int32_t r = 0; r < height; ++r) {
            for (int32_t c = 0; c < width; ++c) {
                const bool green = ((r + c) % 2) == 1;
                int32_t G;
                if (green) {
                    G = at(r, c);
                } else {
                    const int32_t C = at(r, c);
                    const int32_t gl = at(r, c - 1), gr = at(r, c + 1);
                    const int32_t gu = at(r - 1, c), gd = at(r + 1, c);
                    const int32_t lh = 2 * C - at(r, c - 2) - at(r, c + 2);
                    const int32_t lv = 2 * C - at(r - 2, c) - at(r + 2, c);
                    const int32_t dh = std::abs(gl - gr) + std::abs(lh);
                    const int32_t dv = std::abs(gu - gd) + std::abs(lv);
                    if (dh < dv) G = (2 * (gl + gr) + lh + 2) >> 2;
                    else if (dv < dh) G = (2 * (gu + gd) + lv + 2) >> 2;
                    else G = (2 * (gl + gr + gu + gd) + lh + lv + 4) >> 3;
                    G = clamp16(G);
                }
                gp[(size_t)r * (size_t)width + (size_t)c] = (uint16_t)G;
            }
        }
        // Stage 2: red and blue from colour differences with the green plane.
        for (int32_t r = 0; r < height; ++r) {
            for (int32_t c = 0; c < width; ++c) {
                const size_t p = (size_t)r * (size_t)width + (size_t)c;
                const int32_t self = at(r, c);
                const int32_t g0 = g_at(r, c);
                const bool in_red_row = (r & 1) == 0;
                const bool in_red_col = (c & 1) == 0;
                int32_t red, blue;
                // Colour X at a green pixel from neighbours (r1, c1) and (r2, c2).
                auto pair = [&](int32_t r1, int32_t c1, int32_t r2, int32_t c2) {
                    return clamp16((at(r1, c1) + at(r2, c2) + 2 * g0 - g_at(r1, c1)
                                    - g_at(r2, c2) + 1) >> 1);
                };
                // Colour X at an R or B pixel from its four diagonal neighbours.
                auto diagonal = [&]() {
                    const int32_t n1 = at(r - 1, c - 1), n2 = at(r + 1, c + 1);
                    const int32_t p1 = at(r - 1, c + 1), p2 = at(r + 1, c - 1);
                    const int32_t ln = 2 * g0 - g_at(r - 1, c - 1) - g_at(r + 1, c + 1);
                    const int32_t lp = 2 * g0 - g_at(r - 1, c + 1) - g_at(r + 1, c - 1);
                    const int32_t dn = std::abs(n1 - n2) + std::abs(ln);
                    const int32_t dp = std::abs(p1 - p2) + std::abs(lp);
                    int32_t v;
                    if (dn < dp) v = (n1 + n2 + ln + 1) >> 1;
                    else if (dp < dn) v = (p1 + p2 + lp + 1) >> 1;
                    else v = (n1 + n2 + p1 + p2 + ln + lp + 2) >> 2;
                    return clamp16(v);
                };
                if (in_red_row && in_red_col) {          // red pixel
                    red = self;
                    blue = diagonal();
                } else if (!in_red_row && !in_red_col) {  // blue pixel
                    blue = self;
                    red = diagonal();
                } else if (in_red_row) {               // green pixel in a red row
                    red = pair(r, c - 1, r, c + 1);
                    blue = pair(r - 1, c, r + 1, c);
                } else {                            // green pixel in a blue row
                    blue = pair(r, c - 1, r, c + 1);
                    red = pair(r - 1, c, r + 1, c);
                }
                out[p] = (uint16_t)red;
                out[2 * plane + p] = (uint16_t)blue;
            }
        }
    }
}

}  // extern "C"
