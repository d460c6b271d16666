/* Seeded synthetic input streams (counter-based SplitMix64 output function).
 *
 * Holds no selection arithmetic: it only draws numbers.  Element i of the
 * stream with seed s is mix64(mix64(s) + (i + 1) * 0x9E3779B97F4A7C15), the
 * output function of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), so every
 * element is independent of the others and slices fill in parallel.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t elem(uint64_t base, uint64_t i) { return mix64(base + (i + 1) * GAMMA); }

void synth_u64(uint64_t seed, uint64_t start, uint64_t count, uint64_t* out) {
  const uint64_t b = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)count; ++j) out[j] = elem(b, start + (uint64_t)j);
}

void synth_uniform_u32(uint64_t seed, uint64_t n, uint32_t* out) {
  const uint64_t b = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) out[j] = (uint32_t)(elem(b, (uint64_t)j) >> 32);
}

void synth_mod_u32(uint64_t seed, uint64_t n, uint32_t modulus, uint32_t* out) {
  const uint64_t b = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) out[j] = (uint32_t)(elem(b, (uint64_t)j) % modulus);
}

/* Box-Muller, cosine branch, in double; rounded to nearest float. */
void synth_normal_f32(uint64_t seed, uint64_t n, float* out) {
  const uint64_t b = mix64(seed);
  const double inv53 = 1.0 / 9007199254740992.0;
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) {
    uint64_t x1 = elem(b, 2 * (uint64_t)j), x2 = elem(b, 2 * (uint64_t)j + 1);
    double u1 = ((double)(x1 >> 11) + 1.0) * inv53;
    double u2 = (double)(x2 >> 11) * inv53;
    out[j] = (float)(sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
  }
}

/* The same Box-Muller draw kept in double (64-bit keys). */
void synth_normal_f64(uint64_t seed, uint64_t n, double* out) {
  const uint64_t b = mix64(seed);
  const double inv53 = 1.0 / 9007199254740992.0;
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) {
    uint64_t x1 = elem(b, 2 * (uint64_t)j), x2 = elem(b, 2 * (uint64_t)j + 1);
    double u1 = ((double)(x1 >> 11) + 1.0) * inv53;
    double u2 = (double)(x2 >> 11) * inv53;
    out[j] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  }
}

void synth_mod_u64(uint64_t seed, uint64_t n, uint64_t modulus, uint64_t* out) {
  const uint64_t b = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) out[j] = elem(b, (uint64_t)j) % modulus;
}
