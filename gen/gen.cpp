// Seeded synthetic input generators for the LUT-correction workloads.
//
// This module only draws inputs: calibration coefficients, digital-number
// (DN) images, calibration acquisitions for the least-squares fit, raw
// Bayer images, batch request shapes and serving job traces. It holds none of
// the LUT or correction arithmetic. Both the GPU library's tests and the CPU
// oracle receive the same host buffers produced here.
//
// Random numbers come from SplitMix64 used as a counter-based generator
// (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): draw i of stream `key` is mix64(key + (i + 1) * golden_gamma),
// where mix64 is the published SplitMix64 output finaliser. Any sub-range of
// an image can therefore be regenerated on its own, and the result does not
// depend on the thread count. Normals use the Box-Muller transform.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr double kTwoPi = 6.283185307179586476925286766559;

enum Role : uint64_t {
    kRoleCoef = 1,
    kRoleDn = 2,
    kRoleSat = 3,
    kRoleMix = 4,
    kRolePhase = 5,
    kRoleDims = 6,
    kRoleArrival = 7,
    kRoleCalib = 8,
    kRoleBayer = 9,
};

inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

inline uint64_t stream_key(uint64_t seed, uint64_t cfg, uint64_t req, uint64_t band,
                           uint64_t role) {
    uint64_t k = mix64(seed + kGamma);
    k = mix64(k ^ (cfg + 1) * kGamma);
    k = mix64(k ^ (req + 1) * 0xD1B54A32D192ED03ULL);
    k = mix64(k ^ (band + 1) * 0xAEF17502108EF2D9ULL);
    k = mix64(k ^ (role + 1) * 0x8CB92BA72F3D8DD7ULL);
    return k;
}

// Uniform in [0, 1) with 53 random bits.
inline double unif(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// Uniform integer in [0, n).
inline uint64_t below(uint64_t x, uint64_t n) {
    return (uint64_t)(((unsigned __int128)x * (unsigned __int128)n) >> 64);
}

// Standard normal from draws 2i and 2i+1 of one stream (Box-Muller, cosine branch).
inline double normal(uint64_t key, uint64_t i) {
    const double u1 = 1.0 - unif(draw(key, 2 * i));  // (0, 1]
    const double u2 = unif(draw(key, 2 * i + 1));
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(kTwoPi * u2);
}

int thread_count(int requested) {
    if (requested > 0) return requested;
    const char* env = std::getenv("OMP_NUM_THREADS");
    int t = env ? std::atoi(env) : 0;
    if (t <= 0) t = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(t, 16));
}

template <typename F>
void parallel_rows(int64_t rows, int threads, F&& body) {
    const int t = (int)std::min<int64_t>(thread_count(threads), std::max<int64_t>(rows, 1));
    if (t <= 1) {
        body(0, rows);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t per = (rows + t - 1) / t;
    for (int k = 0; k < t; ++k) {
        const int64_t r0 = k * per;
        const int64_t r1 = std::min(rows, r0 + per);
        if (r0 >= r1) break;
        pool.emplace_back([&body, r0, r1] { body(r0, r1); });
    }
    for (auto& th : pool) th.join();
}

}  // namespace

extern "C" {

// Exposed so tests can check the generator against SplitMix64's published
// reference outputs.
uint64_t gen_splitmix64_next(uint64_t* state) {
    *state += kGamma;
    return mix64(*state);
}

uint64_t gen_stream_key(uint64_t seed, uint64_t cfg, uint64_t req, uint64_t band,
                        uint64_t role) {
    return stream_key(seed, cfg, req, band, role);
}

uint64_t gen_draw(uint64_t key, uint64_t i) { return draw(key, i); }

// Per-band, per-detector calibration coefficients, [bands][detectors][4].
//  kind 0 (10-bit, quadratic): a0 ~ N(0, 8), a1 ~ U(0.9, 1.1), a2 ~ N(0, 1e-5), a3 = 0
//  kind 1 (12-bit, cubic):     a0 ~ N(0, 32), a1 ~ U(0.9, 1.1), a2 ~ N(0, 1e-6),
//                              a3 ~ N(0, 1e-10)
// The second parameter of N is the standard deviation.
void gen_coeffs(uint64_t seed, int32_t cfg, int64_t req, int32_t kind, int32_t bands,
                int32_t detectors, double* out) {
    for (int32_t b = 0; b < bands; ++b) {
        const uint64_t key = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)b,
                                        kRoleCoef);
        for (int32_t d = 0; d < detectors; ++d) {
            double* a = out + ((size_t)b * (size_t)detectors + (size_t)d) * 4;
            const uint64_t base = (uint64_t)d * 4;
            const double u = unif(draw(key, 2 * (base + 1)));
            if (kind == 0) {
                a[0] = 8.0 * normal(key, base + 0);
                a[1] = 0.9 + 0.2 * u;
                a[2] = 1e-5 * normal(key, base + 2);
                a[3] = 0.0;
            } else {
                a[0] = 32.0 * normal(key, base + 0);
                a[1] = 0.9 + 0.2 * u;
                a[2] = 1e-6 * normal(key, base + 2);
                a[3] = 1e-10 * normal(key, base + 3);
            }
        }
    }
}

// DN image rows [n0, n0 + nlines) of a [bands][lines][detectors] uint16 image,
// written as [bands][nlines][detectors].
//  kind 0: uniform U{0..1023}
//  kind 1: per band clamp(llround(N(400, 150)), 0, 1023), then each pixel is
//          set to 1023 (saturated) with probability 0.01
//  kind 2: 12-bit scene: per pixel, with probability 1/2 a uniform U{0..4095},
//          else the smooth field clamp(round(2048 + 1800 sin(2 pi d / 1536 + phi_b)
//          cos(2 pi n / 2304 + psi_b)), 0, 4095), phases drawn per band
//  kind 3: uniform U{0..4095}
void gen_dn(uint64_t seed, int32_t cfg, int64_t req, int32_t kind, int32_t bands,
            int64_t lines, int32_t detectors, int64_t n0, int64_t nlines, uint16_t* out,
            int32_t threads) {
    (void)lines;
    const size_t D = (size_t)detectors;
    for (int32_t b = 0; b < bands; ++b) {
        const uint64_t kdn = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)b, kRoleDn);
        const uint64_t ksat = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)b, kRoleSat);
        const uint64_t kmix = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)b, kRoleMix);
        const uint64_t kph = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)b, kRolePhase);
        uint16_t* ob = out + (size_t)b * (size_t)nlines * D;
        std::vector<double> sin_d;
        double psi = 0.0;
        if (kind == 2) {
            const double phi = kTwoPi * unif(draw(kph, 0));
            psi = kTwoPi * unif(draw(kph, 1));
            sin_d.resize(D);
            for (size_t d = 0; d < D; ++d) sin_d[d] = std::sin(kTwoPi * (double)d / 1536.0 + phi);
        }
        parallel_rows(nlines, threads, [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                const int64_t n = n0 + r;
                uint16_t* row = ob + (size_t)r * D;
                const uint64_t i0 = (uint64_t)n * D;
                if (kind == 0 || kind == 3) {
                    const uint64_t m = kind == 0 ? 1024 : 4096;
                    for (size_t d = 0; d < D; ++d) row[d] = (uint16_t)below(draw(kdn, i0 + d), m);
                } else if (kind == 1) {
                    for (size_t d = 0; d < D; ++d) {
                        const uint64_t i = i0 + d;
                        const double x = 400.0 + 150.0 * normal(kdn, i);
                        long long q = std::llround(x);
                        q = std::min<long long>(std::max<long long>(q, 0), 1023);
                        if (unif(draw(ksat, i)) < 0.01) q = 1023;
                        row[d] = (uint16_t)q;
                    }
                } else {
                    const double cn = std::cos(kTwoPi * (double)n / 2304.0 + psi);
                    for (size_t d = 0; d < D; ++d) {
                        const uint64_t i = i0 + d;
                        if (draw(kmix, i) >> 63) {
                            row[d] = (uint16_t)below(draw(kdn, i), 4096);
                        } else {
                            double s = std::round(2048.0 + 1800.0 * sin_d[d] * cn);
                            s = std::min(std::max(s, 0.0), 4095.0);
                            row[d] = (uint16_t)s;
                        }
                    }
                }
            }
        });
    }
}

// Shapes of n uneven batch requests: lines and detectors uniform integers in
// [512, 8192], bands in {1..4}, bit depth in {10, 12}.
void gen_batch_dims(uint64_t seed, int32_t cfg, int32_t n, int64_t* lines, int32_t* detectors,
                    int32_t* bands, int32_t* depth) {
    for (int32_t r = 0; r < n; ++r) {
        const uint64_t k = stream_key(seed, (uint64_t)cfg, (uint64_t)r, 0, kRoleDims);
        lines[r] = 512 + (int64_t)below(draw(k, 0), 8192 - 512 + 1);
        detectors[r] = 512 + (int32_t)below(draw(k, 1), 8192 - 512 + 1);
        bands[r] = 1 + (int32_t)below(draw(k, 2), 4);
        depth[r] = below(draw(k, 3), 2) ? 12 : 10;
    }
}

// A serving trace of n jobs: Poisson arrivals at `qps` jobs/s (exponential
// gaps), sizes log-uniform in [mpix_lo, mpix_hi] megapixels, bands in {1..4},
// detectors uniform in [1024, 12000], lines = max(1, round(size / (bands *
// detectors))), bit depth in {10, 12}.
void gen_serve_jobs(uint64_t seed, int32_t cfg, int32_t n, double qps, double mpix_lo,
                    double mpix_hi, double* arrival_s, int64_t* lines, int32_t* detectors,
                    int32_t* bands, int32_t* depth) {
    double t = 0.0;
    const uint64_t ka = stream_key(seed, (uint64_t)cfg, 0, 0, kRoleArrival);
    for (int32_t r = 0; r < n; ++r) {
        const uint64_t k = stream_key(seed, (uint64_t)cfg, (uint64_t)r, 0, kRoleDims);
        t += -std::log(1.0 - unif(draw(ka, (uint64_t)r))) / qps;
        arrival_s[r] = t;
        const double lo = std::log(mpix_lo), hi = std::log(mpix_hi);
        const double pix = std::exp(lo + (hi - lo) * unif(draw(k, 0))) * 1e6;
        bands[r] = 1 + (int32_t)below(draw(k, 1), 4);
        detectors[r] = 1024 + (int32_t)below(draw(k, 2), 12000 - 1024 + 1);
        const double nl = std::round(pix / ((double)bands[r] * (double)detectors[r]));
        lines[r] = nl < 1.0 ? 1 : (int64_t)nl;
        depth[r] = below(draw(k, 3), 2) ? 12 : 10;
    }
}

// Calibration acquisitions for the least-squares fit: per band, `points`
// flat-field lines at reference levels y_i = (i + 1) / (points + 1) * (L - 1),
// and each detector's response to them,
//   x[b][i][d] = o + g * y_i + c * y_i^2 + e,
// with per-detector o ~ N(0, L / 128), g ~ U(0.9, 1.1), c ~ N(0, 0.01 / L)
// and per-point noise e ~ N(0, 0.5) (an average over frames). y is
// [bands][points], x is [bands][points][detectors].
void gen_calib(uint64_t seed, int32_t cfg, int64_t req, int32_t bands, int32_t points,
               int32_t detectors, int32_t levels, double* x, double* y) {
    const double top = (double)(levels - 1);
    for (int32_t b = 0; b < bands; ++b) {
        const uint64_t key = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)b,
                                        kRoleCalib);
        for (int32_t i = 0; i < points; ++i)
            y[(size_t)b * (size_t)points + (size_t)i] =
                (double)(i + 1) / (double)(points + 1) * top;
        for (int32_t d = 0; d < detectors; ++d) {
            const uint64_t base = (uint64_t)d * (uint64_t)(points + 4);
            const double o = (double)levels / 128.0 * normal(key, base + 0);
            const double g = 0.9 + 0.2 * unif(draw(key, 2 * (base + 1)));
            const double c = 0.01 / (double)levels * normal(key, base + 2);
            for (int32_t i = 0; i < points; ++i) {
                const double yi = y[(size_t)b * (size_t)points + (size_t)i];
                const double e = 0.5 * normal(key, base + 4 + (uint64_t)i);
                x[((size_t)b * (size_t)points + (size_t)i) * (size_t)detectors + (size_t)d] =
                    o + g * yi + c * yi * yi + e;
            }
        }
    }
}

// Raw 16-bit Bayer images (RGGB) [images][height][width]: a smooth scene per
// colour channel k (0 = R, 1 = G, 2 = B),
//   v = 30000 + 20000 sin(2 pi c / 517 + phi_k) cos(2 pi r / 389 + psi_k) + 500 e,
// e ~ N(0, 1) per pixel, sampled at each pixel for the colour of its filter,
// rounded and clamped to [0, 65535]; phases drawn per image and channel.
void gen_bayer(uint64_t seed, int32_t cfg, int64_t req, int32_t images, int32_t height,
               int32_t width, uint16_t* out, int32_t threads) {
    for (int32_t k = 0; k < images; ++k) {
        const uint64_t key = stream_key(seed, (uint64_t)cfg, (uint64_t)req, (uint64_t)k,
                                        kRoleBayer);
        double phi[3], psi[3];
        for (int ch = 0; ch < 3; ++ch) {
            phi[ch] = kTwoPi * unif(draw(key, (uint64_t)(2 * ch)));
            psi[ch] = kTwoPi * unif(draw(key, (uint64_t)(2 * ch + 1)));
        }
        uint16_t* im = out + (size_t)k * (size_t)height * (size_t)width;
        parallel_rows(height, threads, [&](int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                for (int32_t c = 0; c < width; ++c) {
                    const int ch = (r % 2 == 0 && c % 2 == 0) ? 0 : (r % 2 == 1 && c % 2 == 1) ? 2 : 1;
                    const uint64_t i = 8 + (uint64_t)r * (uint64_t)width + (uint64_t)c;
                    double v = 30000.0 + 20000.0 * std::sin(kTwoPi * (double)c / 517.0 + phi[ch]) *
                                             std::cos(kTwoPi * (double)r / 389.0 + psi[ch]) +
                               500.0 * normal(key, i);
                    v = std::min(std::max(std::round(v), 0.0), 65535.0);
                    im[(size_t)r * (size_t)width + (size_t)c] = (uint16_t)v;
                }
            }
        });
    }
}

}  // extern "C"
