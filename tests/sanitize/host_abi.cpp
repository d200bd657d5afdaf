// Host paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer:
// argument validation, topology handles, the allocator hook and its
// out-of-memory path, plan describe/free on null handles, the collective
// per-rank init's joins, checks and free orders.  None of these
// calls reach the GPU, so the program runs on a machine without one.  Each
// check prints what it tested; any failed expectation or sanitizer report
// ends the program with a non-zero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hx.h"

static int failures = 0;
#define EXPECT(cond, what)                                        \
  do {                                                            \
    if (!(cond)) {                                                \
      std::fprintf(stderr, "FAILED: %s (%s)\n", what, #cond);     \
      ++failures;                                                 \
    } else {                                                      \
      std::printf("ok: %s\n", what);                              \
    }                                                             \
  } while (0)

static int n_alloc = 0, n_free = 0;
static void* refuse(size_t, void*, void*) { ++n_alloc; return nullptr; }
static void count_free(void*, void*) { ++n_free; }

int main() {
  EXPECT(hx_version() != nullptr, "version string");
  EXPECT(hx_error_string(HX_ERR_RANGE) != nullptr && hx_error_string(12345) != nullptr, "error strings");

  // topology: valid, then every rejected form
  hx_topo* t = nullptr;
  const int rp[2] = {0, 2}, sp[2] = {0, 2}, dup[2] = {2, 2}, self[1] = {1}, far[1] = {9};
  EXPECT(hx_topo_create(1, 4, 2, rp, nullptr, 2, sp, nullptr, 0, &t) == HX_SUCCESS && t, "topology created");
  hx_topo* bad = nullptr;
  EXPECT(hx_topo_create(1, 4, 2, rp, nullptr, 2, sp, nullptr, 1, &bad) == HX_ERR_UNSUPPORTED, "reorder refused");
  EXPECT(hx_topo_create(1, 4, 2, dup, nullptr, 2, sp, nullptr, 0, &bad) == HX_ERR_RANGE, "duplicate neighbor");
  EXPECT(hx_topo_create(1, 4, 1, self, nullptr, 2, sp, nullptr, 0, &bad) == HX_ERR_RANGE, "self neighbor");
  EXPECT(hx_topo_create(1, 4, 1, far, nullptr, 2, sp, nullptr, 0, &bad) == HX_ERR_RANGE, "neighbor out of range");
  EXPECT(hx_topo_create(1, 4, 2, rp, nullptr, 2, sp, nullptr, 0, nullptr) == HX_ERR_ARG, "null out");

  // init: inconsistent displacements, index out of range, negative counts
  // (device pointers are never touched before these checks)
  void* x = reinterpret_cast<void*>(0x1000);
  void* h = reinterpret_cast<void*>(0x2000);
  const int sc[2] = {2, 3}, sd_bad[2] = {0, 3}, idx[5] = {0, 1, 2, 3, 4}, idx_far[5] = {0, 1, 2, 3, 10};
  const int rc[2] = {2, 3}, rc_neg[2] = {-1, 6};
  hx_req* r = nullptr;
  EXPECT(hx_neighbor_alltoallv_init(x, 10, sc, sd_bad, idx, h, rc, nullptr, HX_F64, 1, t, &r) == HX_ERR_ARG,
         "send displacements not the prefix sum");
  EXPECT(hx_neighbor_alltoallv_init(x, 10, sc, nullptr, idx_far, h, rc, nullptr, HX_F64, 1, t, &r) == HX_ERR_RANGE,
         "send index out of range");
  EXPECT(hx_neighbor_alltoallv_init(x, 10, sc, nullptr, idx, h, rc_neg, nullptr, HX_F64, 1, t, &r) == HX_ERR_ARG,
         "negative receive count");
  EXPECT(r == nullptr, "no request on error");

  // the allocator hook: a refusing allocator gives HX_ERR_NOMEM, frees nothing
  EXPECT(hx_set_allocator(refuse, count_free, nullptr) == HX_SUCCESS, "allocator installed");
  EXPECT(hx_neighbor_alltoallv_init(x, 10, sc, nullptr, idx, h, rc, nullptr, HX_F64, 1, t, &r) == HX_ERR_NOMEM,
         "allocation failure is HX_ERR_NOMEM");
  EXPECT(n_alloc == 1 && n_free == 0 && r == nullptr, "one refused allocation, nothing freed");
  EXPECT(hx_set_allocator(refuse, nullptr, nullptr) == HX_ERR_ARG, "half an allocator refused");
  EXPECT(hx_set_allocator(nullptr, nullptr, nullptr) == HX_SUCCESS, "default allocator restored");

  // plans: validation before any device work
  hx_plan* p = nullptr;
  const int64_t rs_bad[3] = {0, 3, 2}, rs[3] = {0, 2, 4}, hp[3] = {0, 0, 0};
  hx_info info{HX_PLAIN, 1, HX_NODES_BLOCK};
  EXPECT(hx_plan_from_halos(2, rs_bad, &info, hp, nullptr, nullptr, &p) == HX_ERR_ARG, "decreasing row starts");
  EXPECT(hx_plan_from_halos(2, rs, nullptr, hp, nullptr, nullptr, &p) == HX_ERR_ARG, "null info");
  info.ppn = 0;
  info.variant = HX_LOCALITY_2STEP;
  EXPECT(hx_plan_from_halos(2, rs, &info, hp, nullptr, nullptr, &p) == HX_ERR_ARG, "ppn 0");
  info.ppn = 1;
  info.node_map = 7;
  EXPECT(hx_plan_from_halos(2, rs, &info, hp, nullptr, nullptr, &p) == HX_ERR_ARG, "unknown node map");
  info.node_map = HX_NODES_BLOCK;
  info.variant = 9;
  EXPECT(hx_plan_from_halos(2, rs, &info, hp, nullptr, nullptr, &p) == HX_ERR_ARG, "unknown variant");
  info.node_map = HX_NODES_CYCLIC;
  info.variant = HX_LOCALITY_3STEP;
  EXPECT(hx_plan_from_halos(2, rs, &info, hp, nullptr, nullptr, &p) == HX_ERR_UNSUPPORTED, "3-step with cyclic map");
  std::vector<int64_t> many(HX_PLAN_MAX_RANKS + 2);
  for (size_t i = 0; i < many.size(); ++i) many[i] = (int64_t)i;
  info = hx_info{HX_PLAIN, 1, HX_NODES_BLOCK};
  EXPECT(hx_plan_from_halos(HX_PLAN_MAX_RANKS + 1, many.data(), &info, many.data(), nullptr, nullptr, &p) ==
             HX_ERR_UNSUPPORTED,
         "more ranks than the dense tables allow");
  EXPECT(p == nullptr, "no plan on error");
  EXPECT(hx_plan_describe(nullptr, nullptr, nullptr, nullptr, nullptr) == HX_ERR_ARG, "describe a null plan");

  // the collective per-rank init: joins and their host checks, a set whose
  // lists disagree (it fails before any device work), both orders of
  // freeing a pending request and its communicator
  {
    const int64_t crs[3] = {0, 3, 6};
    hx_info ci{HX_LOCALITY_2STEP, 1, HX_NODES_BLOCK};
    hx_comm* c = nullptr;
    EXPECT(hx_comm_create(2, crs, &ci, nullptr, &c) == HX_SUCCESS && c, "communicator created");
    hx_topo *t0 = nullptr, *t1 = nullptr;
    const int to1[1] = {1}, to0[1] = {0};
    EXPECT(hx_topo_create(0, 2, 1, to1, nullptr, 1, to1, nullptr, 0, &t0) == HX_SUCCESS &&
               hx_topo_create(1, 2, 1, to0, nullptr, 1, to0, nullptr, 0, &t1) == HX_SUCCESS,
           "topologies of two ranks");
    const int one[1] = {1}, two[1] = {2};
    const int64_t s0[1] = {1}, r0[2] = {3, 4}, s1[2] = {3, 4}, r1[1] = {0};
    hx_req *q0 = nullptr, *q1 = nullptr, *again = nullptr;
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 3, one, nullptr, s0, h, two, nullptr, r0, HX_F64, 1, t0, c, &q0) ==
                   HX_SUCCESS && q0,
           "rank 0 joins, pending");
    EXPECT(hx_start(q0, nullptr) == HX_ERR_STATE, "a pending request refuses Start");
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 3, one, nullptr, s0, h, two, nullptr, r0, HX_F64, 1, t0, c,
                                               &again) == HX_ERR_STATE && !again,
           "a rank joins once");
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 3, two, nullptr, s1, h, one, nullptr, r1, HX_F64, 1, t1, c, &q1) ==
                   HX_ERR_ARG && !q1,
           "lists that disagree fail before device work");
    EXPECT(hx_req_free(&q0) == HX_SUCCESS && !q0, "pending request freed before its communicator");
    EXPECT(hx_comm_free(&c) == HX_SUCCESS && !c, "communicator freed");
    EXPECT(hx_comm_create(2, crs, &ci, nullptr, &c) == HX_SUCCESS, "second communicator");
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 3, one, nullptr, s0, h, two, nullptr, r0, HX_F64, 1, t0, c, &q0) ==
               HX_SUCCESS,
           "rank 0 joins the second");
    EXPECT(hx_comm_free(&c) == HX_SUCCESS, "communicator freed with a request still pending");
    EXPECT(hx_start(q0, nullptr) == HX_ERR_STATE && hx_req_free(&q0) == HX_SUCCESS, "the orphan stays pending, then frees");
    // 3-step: a rank's request packs from its node's rows (both ranks on one node: 6 rows)
    ci = hx_info{HX_LOCALITY_3STEP, 2, HX_NODES_BLOCK};
    EXPECT(hx_comm_create(2, crs, &ci, nullptr, &c) == HX_SUCCESS, "3-step communicator");
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 3, one, nullptr, s0, h, two, nullptr, r0, HX_F64, 1, t0, c, &q0) ==
               HX_ERR_ARG,
           "3-step: the rank's own row count refused");
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 6, one, nullptr, s0, h, two, nullptr, r0, HX_F64, 1, t0, c, &q0) ==
               HX_SUCCESS,
           "3-step: the node's row count");
    EXPECT(hx_req_free(&q0) == HX_SUCCESS && hx_comm_free(&c) == HX_SUCCESS, "3-step request and communicator freed");
    // more ranks per node than ranks: one node of every rank (no int overflow on the way)
    ci = hx_info{HX_LOCALITY_3STEP, 2147483647, HX_NODES_BLOCK};
    EXPECT(hx_comm_create(2, crs, &ci, nullptr, &c) == HX_SUCCESS, "3-step communicator, ppn INT_MAX");
    EXPECT(hx_neighbor_locality_alltoallv_init(x, 6, one, nullptr, s0, h, two, nullptr, r0, HX_F64, 1, t0, c, &q0) ==
               HX_SUCCESS,
           "ppn INT_MAX: the node's rows are every row");
    EXPECT(hx_req_free(&q0) == HX_SUCCESS && hx_comm_free(&c) == HX_SUCCESS, "freed");
    ci.node_map = HX_NODES_CYCLIC;
    EXPECT(hx_comm_create(2, crs, &ci, nullptr, &c) == HX_ERR_UNSUPPORTED && !c, "3-step with a cyclic map refused");
    EXPECT(hx_topo_free(&t0) == HX_SUCCESS && hx_topo_free(&t1) == HX_SUCCESS, "topologies freed");
  }

  // freeing null handles is allowed
  EXPECT(hx_plan_free(&p) == HX_SUCCESS && hx_req_free(&r) == HX_SUCCESS, "free null handles");
  EXPECT(hx_topo_free(&t) == HX_SUCCESS && t == nullptr, "topology freed");
  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
