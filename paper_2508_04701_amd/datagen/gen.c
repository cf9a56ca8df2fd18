/* Seeded synthetic column generators for the star-schema and join/group-by
 * workloads. This module holds input plumbing only: it draws numbers and
 * nothing of the relational method itself. Both the oracle tests and the GPU
 * path receive the arrays it produces.
 *
 * Every draw is counter based, so the output does not depend on the thread
 * count: draw i of stream (seed, stream) is output i of a SplitMix64
 * sequence (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) whose start state is derived from (seed, stream).
 * Integers in [0, r) use Lemire's multiply-high mapping ("Fast random integer
 * generation in an interval", 2019) without the rejection step, which
 * biases a range r by at most r / 2^64. Zipf ranks use rejection-inversion
 * (Hoermann and Derflinger, "Rejection-inversion to generate variates from
 * monotone discrete distributions", 1996). */

#include <math.h>
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Output i (0-based) of the SplitMix64 sequence seeded with s. */
uint64_t gen_splitmix64_at(uint64_t s, uint64_t i) { return sm_mix(s + (i + 1) * GAMMA); }

/* Start state of stream `stream` under `seed`. */
static inline uint64_t stream_base(uint64_t seed, uint64_t stream) {
  return sm_mix(sm_mix(seed + GAMMA) + (stream + 1) * GAMMA);
}

static inline uint64_t draw(uint64_t base, uint64_t i) { return sm_mix(base + (i + 1) * GAMMA); }

static inline uint64_t below(uint64_t x, uint64_t r) {
  return (uint64_t)(((unsigned __int128)x * r) >> 64);
}

static inline double unit_double(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Raw 64-bit draws. */
void gen_u64(uint64_t seed, uint64_t stream, int64_t n, uint64_t* out) {
  uint64_t base = stream_base(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = draw(base, (uint64_t)i);
}

/* Uniform integers in [lo, hi) written as int8 / int32 / int64 (width 1/4/8). */
void gen_uniform(uint64_t seed, uint64_t stream, int64_t lo, int64_t hi, int64_t n, void* out,
                 int width) {
  uint64_t base = stream_base(seed, stream);
  uint64_t r = (uint64_t)(hi - lo);
  if (width == 1) {
    int8_t* o = (int8_t*)out;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) o[i] = (int8_t)(lo + (int64_t)below(draw(base, (uint64_t)i), r));
  } else if (width == 4) {
    int32_t* o = (int32_t*)out;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) o[i] = (int32_t)(lo + (int64_t)below(draw(base, (uint64_t)i), r));
  } else {
    int64_t* o = (int64_t*)out;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) o[i] = lo + (int64_t)below(draw(base, (uint64_t)i), r);
  }
}

/* A seeded permutation of 0..n-1 (Fisher-Yates, sequential). */
void gen_permutation_i32(uint64_t seed, uint64_t stream, int64_t n, int32_t* out) {
  uint64_t base = stream_base(seed, stream);
  for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)below(draw(base, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

/* out[i] = mix(base + first + i): distinct 64-bit values because the
 * SplitMix64 finaliser is a bijection on 64-bit words. */
void gen_unique_i64(uint64_t seed, uint64_t stream, int64_t first, int64_t n, int64_t* out) {
  uint64_t base = stream_base(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = (int64_t)sm_mix(base + (uint64_t)(first + i));
}

/* Maps each value v of `in` to mix(base + (v - 1) mod m): used to turn Zipf
 * ranks into keys (m = population) or into a coarser derived attribute. */
void gen_map_ranks_i64(uint64_t seed, uint64_t stream, int64_t m, int64_t n, const int64_t* in,
                       int64_t* out) {
  uint64_t base = stream_base(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = (int64_t)sm_mix(base + (uint64_t)((in[i] - 1) % m));
}

/* Zipf(theta) ranks in [1, N] by rejection-inversion. The hat function is
 * h(x) = x^-theta with antiderivative H. Attempt a of row i uses the word
 * mix(draw(i) ^ a * GAMMA), so rows stay independent of the thread count. */
static double zipf_H(double x, double theta) {
  double e = 1.0 - theta;
  return fabs(e) < 1e-12 ? log(x) : (pow(x, e) - 1.0) / e;
}
static double zipf_Hinv(double y, double theta) {
  double e = 1.0 - theta;
  return fabs(e) < 1e-12 ? exp(y) : pow(1.0 + y * e, 1.0 / e);
}

void gen_zipf(uint64_t seed, uint64_t stream, int64_t N, double theta, int64_t n, int64_t* out) {
  uint64_t base = stream_base(seed, stream);
  double h_x1 = zipf_H(1.5, theta) - 1.0; /* H(1.5) - h(1) */
  double h_n = zipf_H((double)N + 0.5, theta);
  double s = 2.0 - zipf_Hinv(zipf_H(2.5, theta) - pow(2.0, -theta), theta);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = 1;
    for (uint64_t a = 0;; ++a) {
      double u = h_n + unit_double(sm_mix(draw(base, (uint64_t)i) ^ (a * GAMMA))) * (h_x1 - h_n);
      double x = zipf_Hinv(u, theta);
      k = (int64_t)(x + 0.5);
      if (k < 1) k = 1;
      if (k > N) k = N;
      if ((double)k - x <= s || u >= zipf_H((double)k + 0.5, theta) - pow((double)k, -theta)) break;
    }
    out[i] = k;
  }
}
