/* Plain multithreaded CPU versions of the exchange's data movement, used as
 * the all-cores CPU baseline.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only the test suite and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with
 * the HIP library and includes none of its headers.
 *
 * Each routine is the plain definition written as a loop over its output
 * (OpenMP splits the loop; every output element is computed by one thread,
 * so the results do not depend on the thread count):
 *   - pack (Start; Listing 4 and Sec. 2.4 of MPI Advance): send[k] = x[idx[k]];
 *   - redistribution pack and unpack (Wait; Sec. 2.2 last paragraph):
 *     out[k] = src[idx[k]], or the identity copy when idx is NULL;
 *   - backward of the pack: gx[i] = g[perm[ptr[i]]] + g[perm[ptr[i]+1]] + ...,
 *     sequential additions in the gradient's type starting from the first
 *     term (a lone -0.0 stays -0.0), +0.0 for an empty row.
 * Rows are ncols values of 4 (float) or 8 (double) bytes; a row is the unit
 * every index addresses.
 * Pinned by tests/test_cpu_oracle.py: brute force against the numpy oracle's
 * definitions, index-encoded values, signed zeros and integer-valued sums.
 */
#include <omp.h>
#include <stdint.h>
#include <string.h>

int oc_threads(void) { return omp_get_max_threads(); }

/* out[k, :] = src[idx ? idx[k] : k, :] for k < n (rows of row_bytes). */
void oc_gather(const void* src, const int32_t* idx, int64_t n, int64_t row_bytes, void* out) {
  const char* s = (const char*)src;
  char* o = (char*)out;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    const int64_t from = idx ? (int64_t)idx[k] : k;
    memcpy(o + k * row_bytes, s + from * row_bytes, (size_t)row_bytes);
  }
}

/* gx[i, c] = sum over e in [ptr[i], ptr[i+1]) in order of g[perm[e], c]. */
void oc_transpose_sum_f64(const double* g, const int32_t* ptr, const int32_t* perm, int64_t n, int64_t ncols,
                          double* gx) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double* o = gx + i * ncols;
    const int32_t a = ptr[i], b = ptr[i + 1];
    for (int64_t c = 0; c < ncols; ++c) o[c] = 0.0;
    if (a == b) continue;
    for (int64_t c = 0; c < ncols; ++c) o[c] = g[(int64_t)perm[a] * ncols + c];
    for (int32_t e = a + 1; e < b; ++e) {
      const double* t = g + (int64_t)perm[e] * ncols;
      for (int64_t c = 0; c < ncols; ++c) o[c] = o[c] + t[c];
    }
  }
}

void oc_transpose_sum_f32(const float* g, const int32_t* ptr, const int32_t* perm, int64_t n, int64_t ncols,
                          float* gx) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    float* o = gx + i * ncols;
    const int32_t a = ptr[i], b = ptr[i + 1];
    for (int64_t c = 0; c < ncols; ++c) o[c] = 0.0f;
    if (a == b) continue;
    for (int64_t c = 0; c < ncols; ++c) o[c] = g[(int64_t)perm[a] * ncols + c];
    for (int32_t e = a + 1; e < b; ++e) {
      const float* t = g + (int64_t)perm[e] * ncols;
      for (int64_t c = 0; c < ncols; ++c) o[c] = o[c] + t[c];
    }
  }
}
