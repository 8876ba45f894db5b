/* Bulk SplitMix64 streams for the seeded workload generators.
 *
 * Same definitions as workloads/rng.py (SplitMix64: Steele, Lea and Flood,
 * OOPSLA 2014; Box-Muller transform for normals), written as one pass over
 * the output so that large operands are produced without temporaries.
 * Output i of a stream with seed s is mix(s + (i + 1) * golden_gamma).
 */
#include <math.h>
#include <stdint.h>

#define WL_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t wl_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline double wl_unit(uint64_t z) {
  return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

void wl_splitmix64(uint64_t seed, int64_t start, int64_t n, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = wl_mix(seed + (uint64_t)(start + i + 1) * WL_GAMMA);
}

/* Complex normals, re and im i.i.d. N(0, 1/2); element j (absolute index
 * start + j) uses stream outputs 2j and 2j+1.  out holds 2n doubles. */
void wl_complex_normal(uint64_t seed, int64_t start, int64_t n, double* out) {
  const double two_pi = 6.283185307179586476925286766559;
  const double rs = 0.70710678118654752440084436210485;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    uint64_t c = (uint64_t)(2 * (start + j));
    double u1 = wl_unit(wl_mix(seed + (c + 1) * WL_GAMMA));
    double u2 = wl_unit(wl_mix(seed + (c + 2) * WL_GAMMA));
    double r = sqrt(-2.0 * log(u1)) * rs;
    double t = two_pi * u2;
    out[2 * j] = r * cos(t);
    out[2 * j + 1] = r * sin(t);
  }
}

/* Complex values with re, im uniform integers in [lo, hi]. */
void wl_gaussian_int(uint64_t seed, int64_t start, int64_t n, int64_t lo, int64_t hi,
                     double* out) {
  uint64_t span = (uint64_t)(hi - lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < 2 * n; ++j) {
    uint64_t c = (uint64_t)(2 * start + j);
    out[j] = (double)((int64_t)(wl_mix(seed + (c + 1) * WL_GAMMA) % span) + lo);
  }
}

/* Complex values whose re and im are odd integers 257..511 with random signs
 * (re and im of element j from stream outputs 2j and 2j+1: magnitude from the
 * low bits, sign from bit 40). */
void wl_wide_odd(uint64_t seed, int64_t start, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < 2 * n; ++j) {
    uint64_t z = wl_mix(seed + (uint64_t)(2 * start + j + 1) * WL_GAMMA);
    double mag = (double)(257 + 2 * (int64_t)(z % 128));
    out[j] = ((z >> 40) & 1) ? -mag : mag;
  }
}

/* Complex values from {0, 1, -1, i, -i}, element j from stream output j. */
void wl_unit_values(uint64_t seed, int64_t start, int64_t n, double* out) {
  static const double re[5] = {0, 1, -1, 0, 0}, im[5] = {0, 0, 0, 1, -1};
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    uint64_t k = wl_mix(seed + (uint64_t)(start + j + 1) * WL_GAMMA) % 5;
    out[2 * j] = re[k];
    out[2 * j + 1] = im[k];
  }
}
