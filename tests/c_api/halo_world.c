/* A C program that uses the library through its C ABI alone (no Python, no
 * torch): a 5-point Laplacian on a 64 x 64 grid in 8 row-strip ranks, 4 per
 * node, locality-aware (2-step) plan built on the GPU from the CSR, one
 * persistent request per rank, the requests batched, and each stage's
 * messages moved by this program between the requests' arenas (the
 * transport the library leaves to its caller).  Checks, with plain loops:
 * every halo equals the vector at the halo's global columns; the backward
 * of every rank's pack equals the sum, per row, of the gradients of the send
 * slots packed from it.  Block and cyclic rank placement.  Exit status 0
 * when every check passes; each failure is printed. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hx.h"

#define NX 64
#define R 8
#define CHECK_HX(call)                                                                  \
  do {                                                                                  \
    int rc_ = (call);                                                                   \
    if (rc_ != HX_SUCCESS) {                                                            \
      fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #call, rc_,         \
              hx_last_error_message());                                                 \
      exit(2);                                                                          \
    }                                                                                   \
  } while (0)
#define CHECK_HIP(call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      fprintf(stderr, "%s:%d: %s -> %s\n", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
      exit(2);                                                                          \
    }                                                                                   \
  } while (0)

static int32_t* field(const hx_plan* p, int r, hx_field f, int64_t* n) {
  CHECK_HX(hx_plan_field_size(p, r, f, n));
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)(*n > 0 ? *n : 1));
  CHECK_HX(hx_plan_field_copy(p, r, f, a));
  return a;
}

/* messages of one stage: copy each message of every sender into its
 * receiver's arena (sender slots [sd, sd + c) -> receiver slots [rd, rd + c)) */
static void transfer(const hx_plan* p, hx_req** req, int stage) {
  const hx_field SP = stage == 1 ? HX_F_S1_PROCS : HX_F_S2_PROCS, SC = stage == 1 ? HX_F_S1_COUNTS : HX_F_S2_COUNTS,
                 SD = stage == 1 ? HX_F_S1_DISPLS : HX_F_S2_DISPLS, RP = stage == 1 ? HX_F_R1_PROCS : HX_F_R2_PROCS,
                 RD = stage == 1 ? HX_F_R1_DISPLS : HX_F_R2_DISPLS;
  for (int q = 0; q < R; ++q) {
    int64_t ns, nn, nd, e1;
    int32_t* sp = field(p, q, SP, &ns);
    int32_t* sc = field(p, q, SC, &nn);
    int32_t* sd = field(p, q, SD, &nd);
    CHECK_HX(hx_plan_field_size(p, q, HX_F_S1_IDX, &e1));
    void* send;
    int64_t send_rows;
    CHECK_HX(hx_req_arena(req[q], HX_ARENA_SEND, &send, &send_rows));
    for (int64_t i = 0; i < ns; ++i) {
      const int d = sp[i];
      int64_t nr, nrd, r1;
      int32_t* rp = field(p, d, RP, &nr);
      int32_t* rd = field(p, d, RD, &nrd);
      int64_t r1c;
      int32_t* r1counts = field(p, d, HX_F_R1_COUNTS, &r1c);
      r1 = 0;
      for (int64_t k = 0; k < r1c; ++k) r1 += r1counts[k];
      int64_t k = 0;
      while (k < nr && rp[k] != q) ++k;
      if (k == nr) {
        fprintf(stderr, "stage %d: rank %d sends to %d, which lists no message from it\n", stage, q, d);
        exit(1);
      }
      void* recv;
      int64_t recv_rows;
      CHECK_HX(hx_req_arena(req[d], HX_ARENA_RECV, &recv, &recv_rows));
      const int64_t src_row = (stage == 1 ? 0 : e1) + sd[i];
      const int64_t dst_row = (stage == 1 ? 0 : r1) + rd[k];
      CHECK_HIP(hipMemcpy((char*)recv + dst_row * 8, (const char*)send + src_row * 8, (size_t)sc[i] * 8,
                          hipMemcpyDeviceToDevice));
      free(rp);
      free(rd);
      free(r1counts);
    }
    free(sp);
    free(sc);
    free(sd);
  }
}

static int run(int node_map) {
  const int64_t n = (int64_t)NX * NX;
  int64_t row_starts[R + 1];
  for (int r = 0; r <= R; ++r) row_starts[r] = n * r / R;
  /* 5-point CSR: row y*NX + x references itself and its 4 neighbours */
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t* cols = (int32_t*)malloc(sizeof(int32_t) * (size_t)(5 * n));
  int64_t nnz = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t y = i / NX, x = i % NX;
    rp[i] = nnz;
    if (y > 0) cols[nnz++] = (int32_t)(i - NX);
    if (x > 0) cols[nnz++] = (int32_t)(i - 1);
    cols[nnz++] = (int32_t)i;
    if (x < NX - 1) cols[nnz++] = (int32_t)(i + 1);
    if (y < NX - 1) cols[nnz++] = (int32_t)(i + NX);
  }
  rp[n] = nnz;
  int64_t* rp_d;
  int32_t* cols_d;
  CHECK_HIP(hipMalloc((void**)&rp_d, sizeof(int64_t) * (size_t)(n + 1)));
  CHECK_HIP(hipMalloc((void**)&cols_d, sizeof(int32_t) * (size_t)nnz));
  CHECK_HIP(hipMemcpy(rp_d, rp, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(cols_d, cols, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
  hx_info info = {HX_LOCALITY_2STEP, 4, node_map};
  hx_plan* plan = NULL;
  CHECK_HX(hx_plan_from_csr(R, row_starts, &info, rp_d, cols_d, NULL, &plan));

  /* the vector: x[g] = 0.5 g + 1 (exact in FP64); one request per rank */
  hx_req* req[R];
  double* xd[R];
  double* hd[R];
  double* gs[R];
  double* gx[R];
  int64_t H[R], E1[R];
  for (int r = 0; r < R; ++r) {
    const int64_t nl = row_starts[r + 1] - row_starts[r];
    double* xh = (double*)malloc(sizeof(double) * (size_t)nl);
    for (int64_t i = 0; i < nl; ++i) xh[i] = 0.5 * (double)(row_starts[r] + i) + 1.0;
    CHECK_HX(hx_plan_field_size(plan, r, HX_F_HALO, &H[r]));
    CHECK_HX(hx_plan_field_size(plan, r, HX_F_S1_IDX, &E1[r]));
    CHECK_HIP(hipMalloc((void**)&xd[r], sizeof(double) * (size_t)nl));
    CHECK_HIP(hipMalloc((void**)&hd[r], sizeof(double) * (size_t)(H[r] > 0 ? H[r] : 1)));
    CHECK_HIP(hipMemcpy(xd[r], xh, sizeof(double) * (size_t)nl, hipMemcpyHostToDevice));
    CHECK_HX(hx_req_from_plan(plan, r, xd[r], hd[r], HX_F64, 1, &req[r]));
    /* gradients of the send slots: slot k of rank r carries 1000 r + k */
    double* gh = (double*)malloc(sizeof(double) * (size_t)(E1[r] > 0 ? E1[r] : 1));
    for (int64_t k = 0; k < E1[r]; ++k) gh[k] = 1000.0 * r + (double)k;
    CHECK_HIP(hipMalloc((void**)&gs[r], sizeof(double) * (size_t)(E1[r] > 0 ? E1[r] : 1)));
    CHECK_HIP(hipMalloc((void**)&gx[r], sizeof(double) * (size_t)nl));
    CHECK_HIP(hipMemcpy(gs[r], gh, sizeof(double) * (size_t)E1[r], hipMemcpyHostToDevice));
    CHECK_HX(hx_req_bind_grad(req[r], gs[r], gx[r]));
    free(xh);
    free(gh);
  }
  hx_batch* b = NULL;
  CHECK_HX(hx_batch_init(req, R, NULL, &b));
  /* Start's pack, stage-1 messages, Wait's redistribution, stage-2 messages, unpack */
  CHECK_HX(hx_batch_launch_phase(b, 0, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  transfer(plan, req, 1);
  CHECK_HX(hx_batch_launch_phase(b, 1, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  transfer(plan, req, 2);
  CHECK_HX(hx_batch_launch_phase(b, 2, NULL));
  CHECK_HX(hx_batch_backward(b, NULL));
  CHECK_HIP(hipDeviceSynchronize());

  int bad = 0;
  for (int r = 0; r < R; ++r) {
    int64_t nh;
    int32_t* halo_cols = field(plan, r, HX_F_HALO, &nh);
    double* got = (double*)malloc(sizeof(double) * (size_t)(nh > 0 ? nh : 1));
    CHECK_HIP(hipMemcpy(got, hd[r], sizeof(double) * (size_t)nh, hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < nh; ++j)
      if (got[j] != 0.5 * (double)halo_cols[j] + 1.0) {
        if (bad++ < 10) fprintf(stderr, "map %d rank %d halo[%lld]: %g, want x[%d]\n", node_map, r, (long long)j,
                                got[j], halo_cols[j]);
      }
    /* backward of the pack: per local row, the sum of its slots' gradients */
    const int64_t nl = row_starts[r + 1] - row_starts[r];
    int64_t ne;
    int32_t* idx = field(plan, r, HX_F_S1_IDX, &ne);
    double* want = (double*)calloc((size_t)(nl > 0 ? nl : 1), sizeof(double));
    for (int64_t k = 0; k < ne; ++k) want[idx[k]] += 1000.0 * r + (double)k;
    double* g = (double*)malloc(sizeof(double) * (size_t)(nl > 0 ? nl : 1));
    CHECK_HIP(hipMemcpy(g, gx[r], sizeof(double) * (size_t)nl, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nl; ++i)
      if (g[i] != want[i]) {
        if (bad++ < 10) fprintf(stderr, "map %d rank %d g_x[%lld]: %g, want %g\n", node_map, r, (long long)i, g[i],
                                want[i]);
      }
    free(halo_cols);
    free(got);
    free(idx);
    free(want);
    free(g);
  }
  printf("node map %d: %d mismatch(es), halo rows %lld..%lld per rank\n", node_map, bad, (long long)H[0],
         (long long)H[R - 1]);
  CHECK_HX(hx_batch_free(&b));
  for (int r = 0; r < R; ++r) {
    CHECK_HX(hx_req_free(&req[r]));
    CHECK_HIP(hipFree(xd[r]));
    CHECK_HIP(hipFree(hd[r]));
    CHECK_HIP(hipFree(gs[r]));
    CHECK_HIP(hipFree(gx[r]));
  }
  CHECK_HX(hx_plan_free(&plan));
  CHECK_HIP(hipFree(rp_d));
  CHECK_HIP(hipFree(cols_d));
  free(rp);
  free(cols);
  return bad;
}

int main(void) {
  int bad = run(HX_NODES_BLOCK) + run(HX_NODES_CYCLIC);
  printf("%s\n", bad ? "FAILED" : "ok");
  return bad ? 1 : 0;
}
