// The per-rank form of the locality-aware init (MPI Advance Sec. 2.2, last
// paragraph: the extension takes, beside the usual neighbor lists, the
// global indices of every value a rank sends and receives).  Its
// deduplication over a node needs what every rank of the node receives, so
// the init is collective: here one process plays every rank of a simulated
// communicator (hx_comm).  Each rank's call checks and records its own
// lists and returns a pending request; the call that completes the set
// checks the ranks' lists against each other (what q sends to s is, element
// for element, what s receives from q), builds the plan on the GPU from the
// receive indices, fills every pending request from it and maps the unpack
// onto each caller's own receive order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <new>
#include <vector>

#include "common.h"
#include "internal.h"

using namespace hx;

namespace {

// counts >= 0; displs NULL or their exclusive prefix sum (the library packs
// arenas and the halo densely in neighbor order)
int dense_layout(int n, const int* counts, const int* displs, int64_t* total, const char* what) {
  if (n > 0 && !counts) return fail(HX_ERR_ARG, "%s: null counts", what);
  int64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    if (counts[i] < 0) return fail(HX_ERR_ARG, "%s: negative count %d at %d", what, counts[i], i);
    if (displs && displs[i] != acc)
      return fail(HX_ERR_ARG, "%s: displacement %d at %d is not the prefix sum %lld", what, displs[i], i,
                  (long long)acc);
    acc += counts[i];
  }
  if (acc >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "%s: more than 2^31 rows", what);
  *total = acc;
  return HX_SUCCESS;
}

// Every rank has joined: cross-check, build the plan, fill the requests.
int complete(hx_comm* c) {
  const int R = c->R;
  const std::vector<int64_t>& rs = c->row_starts;
  // what q sends to s, element for element, is what s receives from q; a
  // receive message without a matching send (or the reverse) is an error
  std::vector<std::vector<int64_t>> roff(R), soff(R);
  for (int r = 0; r < R; ++r) {
    const auto& sl = c->slot[r];
    roff[r].assign(sl.rcounts.size() + 1, 0);
    for (size_t i = 0; i < sl.rcounts.size(); ++i) roff[r][i + 1] = roff[r][i] + sl.rcounts[i];
    soff[r].assign(sl.scounts.size() + 1, 0);
    for (size_t i = 0; i < sl.scounts.size(); ++i) soff[r][i + 1] = soff[r][i] + sl.scounts[i];
  }
  int64_t matched = 0, nonempty_recv = 0;
  for (int s = 0; s < R; ++s)
    for (size_t i = 0; i < c->slot[s].rcounts.size(); ++i) nonempty_recv += c->slot[s].rcounts[i] > 0;
  for (int q = 0; q < R; ++q) {
    const auto& sq = c->slot[q];
    for (size_t i = 0; i < sq.sprocs.size(); ++i) {
      const int s = sq.sprocs[i];
      const auto& ss = c->slot[s];
      const auto it = std::find(ss.rprocs.begin(), ss.rprocs.end(), q);
      const int64_t n = sq.scounts[i];
      if (it == ss.rprocs.end()) {
        if (n > 0) return fail(HX_ERR_ARG, "rank %d sends %lld values to rank %d, which receives none from it", q,
                               (long long)n, s);
        continue;
      }
      const size_t k = (size_t)(it - ss.rprocs.begin());
      if (ss.rcounts[k] != n)
        return fail(HX_ERR_ARG, "rank %d sends %lld values to rank %d, which expects %d", q, (long long)n, s,
                    ss.rcounts[k]);
      if (!std::equal(sq.sind.begin() + soff[q][i], sq.sind.begin() + soff[q][i + 1],
                      ss.rind.begin() + roff[s][k]))
        return fail(HX_ERR_ARG, "the global indices rank %d sends to rank %d differ from those it receives", q, s);
      matched += n > 0;
    }
  }
  if (matched != nonempty_recv) return fail(HX_ERR_ARG, "a rank receives values its source does not send");
  // halos: every rank's receive indices, ascending and distinct
  std::vector<int64_t> hp(1, 0);
  std::vector<int32_t> cols;
  std::vector<std::vector<int64_t>> sorted(R);
  for (int r = 0; r < R; ++r) {
    sorted[r] = c->slot[r].rind;
    std::sort(sorted[r].begin(), sorted[r].end());
    if (std::adjacent_find(sorted[r].begin(), sorted[r].end()) != sorted[r].end())
      return fail(HX_ERR_ARG, "rank %d receives a global index twice", r);
    for (int64_t g : sorted[r]) cols.push_back((int32_t)g);
    hp.push_back((int64_t)cols.size());
  }
  if ((int64_t)cols.size() >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "total halo beyond 2^31 entries");
  DevMem cols_d;
  HX_TRY(upload_vec(cols_d, cols));
  hx_plan* plan = nullptr;
  HX_TRY(hx_plan_from_halos(R, rs.data(), &c->info, hp.data(), cols_d.as<int32_t>(), c->stream, &plan));
  struct PlanGuard {
    hx_plan* p;
    ~PlanGuard() { hx_plan_free(&p); }
  } guard{plan};
  for (int r = 0; r < R; ++r) {
    hx_req* q = c->slot[r].req;
    if (!q) continue;  // freed by its owner before the set completed
    HX_TRY(req_fill_from_plan(plan, r, q->x, q->halo, q->dtype, q->ncols, q));
    // the caller's receive order: position u holds global index rind[u],
    // which the plan's halo (ascending) holds at sigma(u)
    const auto& rind = c->slot[r].rind;
    std::vector<int32_t> sigma(rind.size());
    bool ident = true;
    for (size_t u = 0; u < rind.size(); ++u) {
      sigma[u] = (int32_t)(std::lower_bound(sorted[r].begin(), sorted[r].end(), rind[u]) - sorted[r].begin());
      ident = ident && sigma[u] == (int32_t)u;
    }
    if (!ident) {
      std::vector<int32_t> base(rind.size());
      if (q->unpack_identity) {
        for (size_t j = 0; j < base.size(); ++j) base[j] = (int32_t)j;
      } else if (!base.empty()) {
        HX_HIP(hipMemcpy(base.data(), q->unpack_src.p, base.size() * 4, hipMemcpyDeviceToHost));
      }
      std::vector<int32_t> mine(rind.size());
      for (size_t u = 0; u < rind.size(); ++u) mine[u] = base[sigma[u]];
      HX_TRY(upload_vec(q->unpack_src, mine));
      q->unpack_identity = false;
      req_compute_bytes(q);
    }
  }
  // the requests are complete and independent of the communicator, which
  // stops tracking them (they may be freed before it)
  for (int r = 0; r < R; ++r)
    if (hx_req* q = c->slot[r].req) {
      q->pending = false;
      q->comm = nullptr;
      c->slot[r].req = nullptr;
    }
  return HX_SUCCESS;
}

}  // namespace

extern "C" int hx_comm_create(int nranks, const int64_t* row_starts, const hx_info* info, void* stream,
                              hx_comm** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (nranks <= 0 || !row_starts || !info) return fail(HX_ERR_ARG, "bad nranks, row_starts or info");
  if (row_starts[0] != 0) return fail(HX_ERR_ARG, "row_starts[0] must be 0");
  for (int r = 0; r < nranks; ++r)
    if (row_starts[r + 1] < row_starts[r]) return fail(HX_ERR_ARG, "row_starts must be non-decreasing");
  if (info->variant != HX_PLAIN && info->variant != HX_LOCALITY_2STEP && info->variant != HX_LOCALITY_3STEP)
    return fail(HX_ERR_ARG, "bad variant %d", info->variant);
  if (info->ppn < 1) return fail(HX_ERR_ARG, "ppn must be >= 1");
  if (info->node_map != HX_NODES_BLOCK && info->node_map != HX_NODES_CYCLIC) return fail(HX_ERR_ARG, "bad node map");
  if (info->variant == HX_LOCALITY_3STEP && info->node_map != HX_NODES_BLOCK)
    return fail(HX_ERR_UNSUPPORTED, "the 3-step variant needs block placement");
  auto* c = new (std::nothrow) hx_comm;
  if (!c) return fail(HX_ERR_NOMEM, "out of host memory");
  c->R = nranks;
  c->row_starts.assign(row_starts, row_starts + nranks + 1);
  c->info = *info;
  c->info.ppn = std::min(info->ppn, nranks);  // (as a plan does: one node of every rank)
  c->stream = (hipStream_t)stream;
  c->slot.resize(nranks);
  *out = c;
  return HX_SUCCESS;
}

extern "C" int hx_comm_free(hx_comm** c) {
  if (!c || !*c) return HX_SUCCESS;
  for (auto& sl : (*c)->slot)
    if (sl.req) sl.req->comm = nullptr;  // stays pending: its set can no longer complete
  delete *c;
  *c = nullptr;
  return HX_SUCCESS;
}

extern "C" int hx_neighbor_locality_alltoallv_init(const void* x_local, int64_t n_local, const int* sendcounts,
                                                   const int* sdispls, const int64_t* global_sindices, void* halo,
                                                   const int* recvcounts, const int* rdispls,
                                                   const int64_t* global_rindices, hx_dtype dtype, int ncols,
                                                   const hx_topo* topo, hx_comm* comm, hx_req** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (!topo || !comm) return fail(HX_ERR_ARG, "null topology or communicator");
  if (comm->state != 0) return fail(HX_ERR_STATE, "the communicator's collective init is over");
  if (topo->nranks != comm->R) return fail(HX_ERR_ARG, "topology of %d ranks, communicator of %d", topo->nranks,
                                           comm->R);
  const int r = topo->rank;
  if (comm->slot[r].joined) return fail(HX_ERR_STATE, "rank %d has already joined", r);
  if (dtype != HX_F32 && dtype != HX_F64) return fail(HX_ERR_ARG, "bad dtype");
  if (ncols <= 0) return fail(HX_ERR_ARG, "ncols must be positive");
  const std::vector<int64_t>& rs = comm->row_starts;
  // the vector a request packs from: the rank's rows, or (3-step, where an
  // aggregator packs its node-mates' rows) its node's rows
  int64_t want = rs[r + 1] - rs[r];
  if (comm->info.variant == HX_LOCALITY_3STEP) {
    const int first = r / comm->info.ppn * comm->info.ppn;
    const int last = (int)std::min<int64_t>(comm->R, (int64_t)first + comm->info.ppn);
    want = rs[last] - rs[first];
  }
  if (n_local != want)
    return fail(HX_ERR_ARG, "rank %d: n_local %lld, but its request packs from %lld rows", r, (long long)n_local,
                (long long)want);
  int64_t E = 0, H = 0;
  const int ns = (int)topo->send_procs.size(), nr = (int)topo->recv_procs.size();
  HX_TRY(dense_layout(ns, sendcounts, sdispls, &E, "send"));
  HX_TRY(dense_layout(nr, recvcounts, rdispls, &H, "recv"));
  if ((E > 0 && !global_sindices) || (H > 0 && !global_rindices)) return fail(HX_ERR_ARG, "null global indices");
  if (E > 0 && !x_local) return fail(HX_ERR_ARG, "null x_local");
  if (H > 0 && !halo) return fail(HX_ERR_ARG, "null halo");
  for (int64_t k = 0; k < E; ++k)
    if (global_sindices[k] < rs[r] || global_sindices[k] >= rs[r + 1])
      return fail(HX_ERR_RANGE, "rank %d sends global index %lld, which it does not own", r,
                  (long long)global_sindices[k]);
  int64_t at = 0;
  for (int i = 0; i < nr; ++i) {
    const int q = topo->recv_procs[i];
    for (int k = 0; k < recvcounts[i]; ++k, ++at)
      if (global_rindices[at] < rs[q] || global_rindices[at] >= rs[q + 1])
        return fail(HX_ERR_RANGE, "rank %d receives global index %lld from rank %d, which does not own it", r,
                    (long long)global_rindices[at], q);
  }
  std::unique_ptr<hx_req> q(new (std::nothrow) hx_req);
  if (!q) return fail(HX_ERR_NOMEM, "out of host memory");
  q->dtype = dtype;
  q->ncols = ncols;
  q->row_bytes = (size_t)ncols * dtype_bytes(dtype);
  q->rank = r;
  q->n_local = n_local;
  q->x = static_cast<const char*>(x_local);
  q->halo = static_cast<char*>(halo);
  q->pending = true;
  q->comm = comm;
  auto& sl = comm->slot[r];
  sl.rprocs = topo->recv_procs;
  sl.sprocs = topo->send_procs;
  sl.rcounts.assign(recvcounts, recvcounts + nr);
  sl.scounts.assign(sendcounts, sendcounts + ns);
  sl.rind.assign(global_rindices, global_rindices + H);
  sl.sind.assign(global_sindices, global_sindices + E);
  sl.joined = true;
  sl.req = q.get();
  ++comm->joined;
  if (comm->joined < comm->R) {
    *out = q.release();
    return HX_SUCCESS;
  }
  const int rc = complete(comm);
  if (rc != HX_SUCCESS) {
    comm->state = rc;
    sl.req = nullptr;  // the completing call's own request is not returned; the others stay pending
    return rc;
  }
  comm->state = 1;
  *out = q.release();
  return HX_SUCCESS;
}
