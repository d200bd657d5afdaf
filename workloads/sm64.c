/* SplitMix64 stream fill (Steele, Lea and Flood, OOPSLA 2014), multithreaded.
 *
 * Input generation only: output i of the stream seeded with s is
 * mix(s + (i + 1) * GAMMA).  Produces exactly the values of the numpy
 * implementation in gen.py (tests/test_inputs_cpu.py compares the two, and
 * the stream with the published generator's first outputs); it exists
 * because the batched workload needs ~10^9 values and numpy's 64-bit
 * multiply is slow.
 */
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void sm64_fill_u64(uint64_t seed, int64_t start, int64_t count, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i)
    out[i] = mix(seed + (uint64_t)(start + i + 1) * GAMMA);
}

void sm64_fill_pm1_f64(uint64_t seed, int64_t start, int64_t count, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    uint64_t z = mix(seed + (uint64_t)(start + i + 1) * GAMMA);
    out[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
  }
}

void sm64_fill_pm1_f32(uint64_t seed, int64_t start, int64_t count, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    uint64_t z = mix(seed + (uint64_t)(start + i + 1) * GAMMA);
    out[i] = (float)((double)(z >> 11) * 0x1p-52 - 1.0);
  }
}

/* Random-rows structure: entry e = row*k + j draws z = SM64(seed, e); it is
 * global iff (z >> 40) < thr24, with column z & (nrows-1), else
 * blk*(row/blk) + (z & (blk-1)).  nrows and blk are powers of two. */
void gen_random_rows_cols(uint64_t seed, int64_t nrows, int64_t k, int64_t blk,
                          uint64_t thr24, int32_t* cols) {
  const int64_t nnz = nrows * k;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nnz; ++e) {
    uint64_t z = mix(seed + (uint64_t)(e + 1) * GAMMA);
    int64_t row = e / k;
    int64_t c = ((z >> 40) < thr24) ? (int64_t)(z & (uint64_t)(nrows - 1))
                                    : (row / blk) * blk + (int64_t)(z & (uint64_t)(blk - 1));
    cols[e] = (int32_t)c;
  }
}
