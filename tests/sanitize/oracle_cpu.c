/* The multithreaded C oracle loops under AddressSanitizer and
 * UndefinedBehaviorSanitizer: gathers with and without an index list,
 * empty lists, empty rows and tails of every length.  Values are checked
 * against their definitions; any mismatch or sanitizer report ends the
 * program with a non-zero status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oc_gather(const void* src, const int32_t* idx, int64_t n, int64_t row_bytes, void* out);
void oc_transpose_sum_f64(const double* g, const int32_t* ptr, const int32_t* perm, int64_t n, int64_t ncols,
                          double* gx);
void oc_transpose_sum_f32(const float* g, const int32_t* ptr, const int32_t* perm, int64_t n, int64_t ncols,
                          float* gx);

int main(void) {
  int bad = 0;
  for (int64_t n = 0; n < 70; ++n) {
    const int64_t rows = 37, nc = 3;
    double* src = malloc(sizeof(double) * rows * nc);
    double* out = malloc(sizeof(double) * (n ? n : 1) * nc);
    int32_t* idx = malloc(sizeof(int32_t) * (n ? n : 1));
    for (int64_t i = 0; i < rows * nc; ++i) src[i] = (double)i;
    for (int64_t k = 0; k < n; ++k) idx[k] = (int32_t)((k * 7 + 3) % rows);
    oc_gather(src, idx, n, nc * 8, out);
    for (int64_t k = 0; k < n; ++k)
      for (int64_t c = 0; c < nc; ++c) bad += out[k * nc + c] != src[idx[k] * nc + c];
    const int64_t m = n < rows ? n : rows;
    oc_gather(src, NULL, m, nc * 8, out);
    for (int64_t k = 0; k < m * nc; ++k) bad += out[k] != src[k];
    /* transpose sums: row i of n gets the slots e with e % (n + 1) == i (rows past e's range empty) */
    const int64_t E = 2 * n + 5;
    int32_t* ptr = malloc(sizeof(int32_t) * (n + 1));
    int32_t* perm = malloc(sizeof(int32_t) * E);
    double* g = malloc(sizeof(double) * E * nc);
    float* gf = malloc(sizeof(float) * E * nc);
    double* gx = malloc(sizeof(double) * (n ? n : 1) * nc);
    float* gxf = malloc(sizeof(float) * (n ? n : 1) * nc);
    int64_t at = 0;
    for (int64_t i = 0; i < n; ++i) {
      ptr[i] = (int32_t)at;
      for (int64_t e = 0; e < E; ++e)
        if (e % (n + 1) == i) perm[at++] = (int32_t)e;
    }
    ptr[n] = (int32_t)at;
    for (int64_t i = 0; i < E * nc; ++i) { g[i] = (double)(i % 11); gf[i] = (float)(i % 5); }
    oc_transpose_sum_f64(g, ptr, perm, n, nc, gx);
    oc_transpose_sum_f32(gf, ptr, perm, n, nc, gxf);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t c = 0; c < nc; ++c) {
        double s = 0.0;
        float sf = 0.0f;
        for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) { s += g[perm[e] * nc + c]; sf += gf[perm[e] * nc + c]; }
        bad += gx[i * nc + c] != s;
        bad += gxf[i * nc + c] != sf;
      }
    free(src); free(out); free(idx); free(ptr); free(perm); free(g); free(gf); free(gx); free(gxf);
  }
  printf("%d mismatch(es)\n", bad);
  return bad ? 1 : 0;
}
