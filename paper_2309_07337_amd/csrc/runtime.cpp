// Host runtime of the C ABI: errors, device memory, topology handles,
// persistent requests (init / Start / Wait / backward), batches captured in
// hipGraphs, the plain one-launch-per-member form, and the schedule tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"

namespace hx {

namespace {
thread_local std::string g_msg;
thread_local int g_hip = 0;
}  // namespace

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_msg = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  g_hip = (int)e;
  char buf[1024];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  g_msg = buf;
  return e == hipErrorOutOfMemory ? HX_ERR_NOMEM : HX_ERR_HIP;
}

// Installed allocator (none: hipMalloc / hipFree).
namespace {
std::mutex g_alloc_mu;
hx_alloc_fn g_alloc_fn = nullptr;
hx_free_fn g_free_fn = nullptr;
void* g_alloc_ctx = nullptr;
}  // namespace

void DevMem::release() {
  if (p && owned) {
    if (free_fn) {
      // the caller's allocator may hand the block out again at once: wait
      // until no kernel still uses it, as hipFree does
      (void)hipDeviceSynchronize();
      free_fn(p, free_ctx);
    } else {
      (void)hipFree(p);
    }
  }
  p = nullptr;
  bytes = 0;
  free_fn = nullptr;
  free_ctx = nullptr;
  owned = true;
}

int DevMem::alloc(size_t nbytes, hipStream_t stream) {
  release();
  if (nbytes == 0) return HX_SUCCESS;
  hx_alloc_fn af;
  hx_free_fn ff;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    af = g_alloc_fn;
    ff = g_free_fn;
    ctx = g_alloc_ctx;
  }
  if (af) {
    void* q = af(nbytes, (void*)stream, ctx);
    if (!q) return fail(HX_ERR_NOMEM, "the installed allocator failed to provide %zu bytes", nbytes);
    if (((uintptr_t)q & 15) != 0) {
      ff(q, ctx);
      return fail(HX_ERR_ARG, "the installed allocator returned a pointer that is not 16-byte aligned");
    }
    p = q;
    bytes = nbytes;
    free_fn = ff;
    free_ctx = ctx;
    return HX_SUCCESS;
  }
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    g_hip = (int)e;
    return fail(HX_ERR_NOMEM, "hipMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
  }
  bytes = nbytes;
  return HX_SUCCESS;
}

int upload(DevMem& dst, const void* host, size_t bytes) {
  HX_TRY(dst.alloc(bytes));
  if (bytes) HX_HIP(hipMemcpy(dst.p, host, bytes, hipMemcpyHostToDevice));
  return HX_SUCCESS;
}

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

int device_lds_per_block() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 65536;
    cached[dev] = v;
  }
  return cached[dev];
}

Sched default_sched(int kind, int row_bytes) {
  Sched s;
  s.block_threads = 256;
  s.blocks_per_cu = 8;
  s.nontemporal = 0;
  s.per_neighbor = 0;
  // about 32 KiB of output per tile
  int rows = std::max(64, (32 << 10) / std::max(row_bytes, 1));
  rows = std::min(rows, 8192);
  // segmented sum: the largest tile whose row pointers are staged in LDS
  if (kind == KIND_SEGSUM) rows = std::min(kStageRows, std::max(64, (64 << 10) / std::max(row_bytes, 1)));
  s.tile_rows = rows;
  // rows in flight per lane: 4, except for rows of 16 bytes or less, whose
  // gathers measure best with 1 (more lanes, not more rows per lane)
  s.unroll = row_bytes <= 16 && kind == KIND_GATHER ? 1 : 4;
  // segmented sums: 512 lanes, 1024 for rows of 64 B and more (more terms in
  // flight per chunk; such rows read no term windows by default)
  if (kind == KIND_SEGSUM) s.block_threads = row_bytes >= 64 ? 1024 : 512;
  // rows of 64 B and more: push by default (on gfx950 scattered full-line
  // writes run as fast as scattered reads, and the push form reads each
  // source row once instead of once per slot); short rows: pull
  s.push_pack = kind == KIND_GATHER && row_bytes >= 64 ? 1 : 0;
  // short rows: gathers and segmented sums read their jobs' windows from LDS
  s.lds_window = row_bytes <= 16 ? 1 : 0;
  // gathers without windows: one workgroup per tile (a window would be
  // staged again by every workgroup); segmented sums of rows of 64 B and
  // more: the same, two terms per lane in flight
  if (kind == KIND_GATHER && !s.lds_window) s.blocks_per_cu = kOneShotBpc;
  if (kind == KIND_SEGSUM && row_bytes >= 64) {
    s.blocks_per_cu = kOneShotBpc;
    s.unroll = 2;
  }
  // gathers of 4- and 8-byte rows: 16-byte row groups per lane, one
  // workgroup of 512 lanes per (up to) 16384-row tile, the job's window (if
  // it has one) staged once per tile while the tile's indices are in flight
  if (kind == KIND_GATHER && (row_bytes == 4 || row_bytes == 8)) {
    s.pair_rows = 1;
    s.tile_rows = 16384;
    s.block_threads = 512;
    s.blocks_per_cu = kOneShotBpc;
    s.unroll = 4;
  }
  return s;
}

Sched resolve_sched(const hx_sched* p, int kind, int row_bytes) {
  Sched s = default_sched(kind, row_bytes);
  if (!p) return s;
  if (p->tile_rows > 0) s.tile_rows = p->tile_rows;
  if (p->block_threads > 0) s.block_threads = p->block_threads;
  if (p->blocks_per_cu > 0) s.blocks_per_cu = p->blocks_per_cu;
  s.nontemporal = p->nontemporal <= 0 ? 0 : (p->nontemporal >= 2 ? 2 : 1);
  s.per_neighbor = p->per_neighbor ? 1 : 0;
  if (p->unroll > 0) s.unroll = p->unroll <= 1 ? 1 : (p->unroll == 2 ? 2 : 4);
  if (p->push_pack == 1) s.push_pack = 1;
  else if (p->push_pack == 2) s.push_pack = 0;
  if (p->lds_window == 1) s.lds_window = 1;
  else if (p->lds_window == 2) s.lds_window = 0;
  if (p->pair_rows == 1) s.pair_rows = 1;
  else if (p->pair_rows == 2) s.pair_rows = 0;
  return s;
}

hx_sched to_public(const Sched& s) {
  hx_sched o;
  o.tile_rows = s.tile_rows;
  o.block_threads = s.block_threads;
  o.blocks_per_cu = s.blocks_per_cu;
  o.nontemporal = s.nontemporal;
  o.per_neighbor = s.per_neighbor;
  o.unroll = s.unroll;
  o.push_pack = s.push_pack ? 1 : 2;
  o.lds_window = s.lds_window ? 1 : 2;
  o.pair_rows = s.pair_rows ? 1 : 2;
  return o;
}

}  // namespace hx

using namespace hx;

// ===========================================================================
// Topology
// ===========================================================================
static int check_procs(int rank, int nranks, int n, const int* procs, const char* what) {
  if (n < 0) return fail(HX_ERR_ARG, "%s: negative neighbor count", what);
  if (n > 0 && !procs) return fail(HX_ERR_ARG, "%s: null neighbor list", what);
  std::vector<int> v(procs, procs + n);
  for (int p : v)
    if (p < 0 || p >= nranks || p == rank)
      return fail(HX_ERR_RANGE, "%s: neighbor %d out of range or self", what, p);
  std::sort(v.begin(), v.end());
  if (std::adjacent_find(v.begin(), v.end()) != v.end())
    return fail(HX_ERR_RANGE, "%s: duplicate neighbor", what);
  return HX_SUCCESS;
}

extern "C" int hx_topo_create(int rank, int nranks, int n_recvs, const int* recv_procs,
                              const int* recv_weights, int n_sends, const int* send_procs,
                              const int* send_weights, int reorder, hx_topo** out) {
  (void)recv_weights;
  (void)send_weights;
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (nranks <= 0 || rank < 0 || rank >= nranks) return fail(HX_ERR_ARG, "bad rank/nranks");
  if (reorder != 0) return fail(HX_ERR_UNSUPPORTED, "reorder is not supported (ranks are fixed)");
  HX_TRY(check_procs(rank, nranks, n_recvs, recv_procs, "recv_procs"));
  HX_TRY(check_procs(rank, nranks, n_sends, send_procs, "send_procs"));
  auto* t = new (std::nothrow) hx_topo;
  if (!t) return fail(HX_ERR_NOMEM, "out of host memory");
  t->rank = rank;
  t->nranks = nranks;
  t->recv_procs.assign(recv_procs, recv_procs + n_recvs);
  t->send_procs.assign(send_procs, send_procs + n_sends);
  *out = t;
  return HX_SUCCESS;
}

extern "C" int hx_topo_free(hx_topo** t) {
  if (!t) return HX_SUCCESS;
  delete *t;
  *t = nullptr;
  return HX_SUCCESS;
}

// ===========================================================================
// Requests
// ===========================================================================
static int req_phase_jobs(const hx_req* r, int phase, const Sched& sc, std::vector<GatherJob>* g,
                          std::vector<SegSumJob>* s);

// Launch table of one phase from its jobs: the backward is a segmented sum;
// the pack is a push (scatter) or a pull (gather) by the schedule; the other
// phases are gathers.
int hx::build_phase_table(int phase, const Sched& sc, int dtype, int row_bytes, const std::vector<GatherJob>& g,
                          const std::vector<SegSumJob>& s, LaunchTable* t) {
  if (phase == PH_BWD) return build_segsum_table(s, dtype, row_bytes, sc, t);
  // (a request with completion counters packs in the pull form whatever the schedule)
  if (phase == PH_PACK && sc.push_pack && g.empty()) return build_scatter_table(s, dtype, row_bytes, sc, t);
  if (phase == PH_PACK && !g.empty() && !s.empty())
    return fail(HX_ERR_STATE, "pack jobs of both forms in one launch");
  return build_gather_table(g, dtype, row_bytes, sc, t, phase);
}

static int build_req_tables(hx_req* r) {
  if (r->tables_built) return HX_SUCCESS;
  for (int ph = 0; ph < 4; ++ph) {
    std::vector<GatherJob> g;
    std::vector<SegSumJob> s;
    const int kind = ph == PH_BWD ? KIND_SEGSUM : KIND_GATHER;
    const Sched sc = default_sched(kind, (int)r->row_bytes);
    HX_TRY(req_phase_jobs(r, ph, sc, &g, &s));
    HX_TRY(build_phase_table(ph, sc, r->dtype, (int)r->row_bytes, g, s, &r->lt[ph]));
  }
  r->tables_built = true;
  return HX_SUCCESS;
}

static int req_phase_jobs(const hx_req* r, int phase, const Sched& sc, std::vector<GatherJob>* g,
                          std::vector<SegSumJob>* s) {
  const size_t rb = r->row_bytes;
  const bool per_nbr = sc.per_neighbor != 0;
  switch (phase) {
    case PH_PACK: {
      if (r->ready.p) {
        // partition-ready pack: pull form, one job per message, each with its
        // message's completion counter
        auto* cnt = r->ready.as<unsigned long long>();
        int64_t off = 0;
        for (size_t m = 0; m < r->s1_counts.size(); ++m) {
          const int64_t c = r->s1_counts[m];
          if (c > 0) {
            GatherJob j{r->x, r->send.as<char>() + off * (int64_t)rb, r->s1_idx.as<int32_t>() + off, c, 0, r->n_local};
            j.ready = cnt + m;
            g->push_back(j);
          }
          off += c;
        }
        break;
      }
      if (sc.push_pack) {
        if (r->E1 > 0)
          s->push_back(SegSumJob{r->x, r->send.as<char>(), r->bt_ptr.as<int32_t>(), r->bt_perm.as<int32_t>(),
                                 r->n_local});
        break;
      }
      GatherJob j{r->x, r->send.as<char>(), r->s1_idx.as<int32_t>(), r->E1, 0, r->n_local};
      if (per_nbr) split_gather_by_counts(j, r->s1_counts, rb, g);
      else g->push_back(j);
      break;
    }
    case PH_REDIST: {
      GatherJob j{r->recv.as<char>(), r->send.as<char>() + r->E1 * (int64_t)rb, r->s2_src.as<int32_t>(),
                  r->E2, 0, r->R1};
      if (per_nbr) split_gather_by_counts(j, r->s2_counts, rb, g);
      else g->push_back(j);
      break;
    }
    case PH_UNPACK: {
      GatherJob j{r->recv.as<char>(), r->halo, r->unpack_identity ? nullptr : r->unpack_src.as<int32_t>(),
                  r->H, 0, r->R1 + r->R2};
      if (per_nbr && r->unpack_identity) split_gather_by_counts(j, r->r1_counts, rb, g);
      else g->push_back(j);
      break;
    }
    case PH_BWD: {
      if (r->g_x && (r->g_send || r->E1 == 0)) {
        SegSumJob jb{r->g_send, r->g_x, r->bt_ptr.as<int32_t>(), r->bt_perm.as<int32_t>(), r->n_local};
        jb.win_rows = r->E1;  // the terms are the request's own send-slot gradients
        s->push_back(jb);
      }
      break;
    }
    default:
      return fail(HX_ERR_ARG, "bad phase");
  }
  return HX_SUCCESS;
}

int hx::req_jobs(const hx_req* r, int phase, const Sched& sc, std::vector<GatherJob>* g,
                 std::vector<SegSumJob>* s) {
  return req_phase_jobs(r, phase, sc, g, s);
}

static int64_t count_distinct_host(const std::vector<int32_t>& idx, int64_t domain) {
  if (idx.empty() || domain <= 0) return 0;
  std::vector<uint8_t> seen((size_t)domain, 0);
  int64_t u = 0;
  for (int32_t v : idx)
    if (v >= 0 && v < domain && !seen[v]) { seen[v] = 1; ++u; }
  return u;
}

void hx::req_compute_bytes(hx_req* r) {
  const int64_t rb = (int64_t)r->row_bytes;
  r->bytes[PH_PACK] = (r->E1 + r->U_pack) * rb + 4 * r->E1;
  r->bytes[PH_REDIST] = (r->E2 + r->U_redist) * rb + 4 * r->E2;
  r->bytes[PH_UNPACK] = 2 * r->H * rb + (r->unpack_identity ? 0 : 4 * r->H);
  r->bytes[PH_BWD] = (r->E1 + r->n_local) * rb + 4 * (r->E1 + r->n_local + 1);
}

// Builds the transpose of the pack map (rows -> send slots, ascending slot)
// on the host for list-initialised requests.
static void host_transpose(const std::vector<int32_t>& idx, int64_t n_local, std::vector<int32_t>* ptr,
                           std::vector<int32_t>* perm) {
  ptr->assign((size_t)n_local + 1, 0);
  for (int32_t v : idx) (*ptr)[(size_t)v + 1]++;
  for (int64_t i = 0; i < n_local; ++i) (*ptr)[(size_t)i + 1] += (*ptr)[(size_t)i];
  std::vector<int32_t> fill(ptr->begin(), ptr->end() - 1);
  perm->assign(idx.size(), 0);
  for (size_t k = 0; k < idx.size(); ++k) (*perm)[(size_t)fill[(size_t)idx[k]]++] = (int32_t)k;
}

static int check_layout(int n, const int* counts, const int* displs, int64_t* total, const char* what) {
  if (n > 0 && !counts) return fail(HX_ERR_ARG, "%s: null counts", what);
  int64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    if (counts[i] < 0) return fail(HX_ERR_ARG, "%s: negative count", what);
    if (displs && displs[i] != acc)
      return fail(HX_ERR_ARG, "%s: displacement %d of neighbor %d is not the packed prefix %lld", what,
                  displs[i], i, (long long)acc);
    acc += counts[i];
  }
  if (acc >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "%s: more than 2^31 rows", what);
  *total = acc;
  return HX_SUCCESS;
}

extern "C" int hx_neighbor_alltoallv_init(const void* x_local, int64_t n_local, const int* sendcounts,
                                          const int* sdispls, const int* send_idx, void* halo,
                                          const int* recvcounts, const int* rdispls, hx_dtype dtype,
                                          int ncols, const hx_topo* topo, hx_req** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (!topo) return fail(HX_ERR_ARG, "null topology");
  if (dtype != HX_F32 && dtype != HX_F64) return fail(HX_ERR_ARG, "bad dtype");
  if (ncols <= 0) return fail(HX_ERR_ARG, "ncols must be positive");
  if (n_local < 0) return fail(HX_ERR_ARG, "negative n_local");
  if (n_local >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "n_local beyond 2^31 rows");
  int64_t E = 0, H = 0;
  HX_TRY(check_layout((int)topo->send_procs.size(), sendcounts, sdispls, &E, "send"));
  HX_TRY(check_layout((int)topo->recv_procs.size(), recvcounts, rdispls, &H, "recv"));
  if (E > 0 && !send_idx) return fail(HX_ERR_ARG, "null send_idx");
  if (E > 0 && !x_local) return fail(HX_ERR_ARG, "null x_local");
  if (H > 0 && !halo) return fail(HX_ERR_ARG, "null halo");
  for (int64_t k = 0; k < E; ++k)
    if (send_idx[k] < 0 || send_idx[k] >= n_local)
      return fail(HX_ERR_RANGE, "send_idx[%lld] = %d outside [0, %lld)", (long long)k, send_idx[k],
                  (long long)n_local);
  std::unique_ptr<hx_req> r(new (std::nothrow) hx_req);
  if (!r) return fail(HX_ERR_NOMEM, "out of host memory");
  r->dtype = dtype;
  r->ncols = ncols;
  r->row_bytes = (size_t)ncols * dtype_bytes(dtype);
  r->variant = HX_PLAIN;
  r->rank = topo->rank;
  r->n_local = n_local;
  r->E1 = E;
  r->E2 = 0;
  r->R1 = H;
  r->R2 = 0;
  r->H = H;
  r->x = static_cast<const char*>(x_local);
  r->halo = static_cast<char*>(halo);
  r->unpack_identity = true;
  std::vector<int32_t> idx(send_idx, send_idx + E);
  r->s1_counts.assign(sendcounts, sendcounts + topo->send_procs.size());
  r->r1_counts.assign(recvcounts, recvcounts + topo->recv_procs.size());
  std::vector<int32_t> ptr, perm;
  host_transpose(idx, n_local, &ptr, &perm);
  HX_TRY(upload_vec(r->s1_idx, idx));
  HX_TRY(upload_vec(r->bt_ptr, ptr));
  HX_TRY(upload_vec(r->bt_perm, perm));
  HX_TRY(r->send.alloc((size_t)E * r->row_bytes));
  HX_TRY(r->recv.alloc((size_t)H * r->row_bytes));
  r->U_pack = count_distinct_host(idx, n_local);
  r->U_redist = 0;
  req_compute_bytes(r.get());
  *out = r.release();
  return HX_SUCCESS;
}

int hx::req_usable(const hx_req* r) {
  if (r->pending) return fail(HX_ERR_STATE, "the collective init this request joined has not completed");
  return HX_SUCCESS;
}

extern "C" int hx_start(hx_req* r, void* stream) {
  if (!r) return fail(HX_ERR_ARG, "null request");
  HX_TRY(req_usable(r));
  if (r->active) return fail(HX_ERR_STATE, "request already active");
  HX_TRY(build_req_tables(r));
  HX_TRY(launch_table(r->lt[PH_PACK], (hipStream_t)stream));
  r->active = true;
  return HX_SUCCESS;
}

extern "C" int hx_wait(hx_req* r, void* stream) {
  if (!r) return fail(HX_ERR_ARG, "null request");
  HX_TRY(req_usable(r));
  if (!r->active) return HX_SUCCESS;
  HX_TRY(build_req_tables(r));
  HX_TRY(launch_table(r->lt[PH_REDIST], (hipStream_t)stream));
  HX_TRY(launch_table(r->lt[PH_UNPACK], (hipStream_t)stream));
  r->active = false;
  return HX_SUCCESS;
}

extern "C" int hx_req_arena(hx_req* r, int which, void** dev_ptr, int64_t* rows) {
  if (!r || !dev_ptr || !rows) return fail(HX_ERR_ARG, "null argument");
  HX_TRY(req_usable(r));
  if (which == HX_ARENA_SEND) {
    *dev_ptr = r->send.p;
    *rows = r->E1 + r->E2;
  } else if (which == HX_ARENA_RECV) {
    *dev_ptr = r->recv.p;
    *rows = r->R1 + r->R2;
  } else {
    return fail(HX_ERR_ARG, "bad arena id");
  }
  return HX_SUCCESS;
}

extern "C" int hx_req_enable_ready(hx_req* r, unsigned long long** dev_counters) {
  if (!r || !dev_counters) return fail(HX_ERR_ARG, "null argument");
  HX_TRY(req_usable(r));
  if (r->active) return fail(HX_ERR_STATE, "request active");
  if (!r->ready.p) {
    const size_t n = std::max<size_t>(r->s1_counts.size(), 1);
    HX_TRY(r->ready.alloc(n * sizeof(unsigned long long)));
    HX_HIP(hipMemset(r->ready.p, 0, n * sizeof(unsigned long long)));
    r->tables_built = false;  // the pack is rebuilt per message
  }
  *dev_counters = r->ready.as<unsigned long long>();
  return HX_SUCCESS;
}

extern "C" int hx_req_bind_grad(hx_req* r, const void* g_send, void* g_x) {
  if (!r) return fail(HX_ERR_ARG, "null request");
  HX_TRY(req_usable(r));
  if ((r->E1 > 0 && !g_send) || (r->n_local > 0 && !g_x)) return fail(HX_ERR_ARG, "null gradient buffer");
  r->g_send = static_cast<const char*>(g_send);
  r->g_x = static_cast<char*>(g_x);
  static std::atomic<uint64_t> bind_counter{0};
  r->grad_gen = ++bind_counter;  // batches holding this member rebuild their backward
  r->lt[PH_BWD] = LaunchTable();
  std::vector<GatherJob> g;
  std::vector<SegSumJob> s;
  const Sched sc = default_sched(KIND_SEGSUM, (int)r->row_bytes);
  HX_TRY(req_phase_jobs(r, PH_BWD, sc, &g, &s));
  HX_TRY(build_segsum_table(s, r->dtype, (int)r->row_bytes, sc, &r->lt[PH_BWD]));
  return HX_SUCCESS;
}

extern "C" int hx_backward(hx_req* r, void* stream) {
  if (!r) return fail(HX_ERR_ARG, "null request");
  HX_TRY(req_usable(r));
  if (!r->g_x && r->n_local > 0) return fail(HX_ERR_STATE, "no gradient buffers bound");
  return launch_table(r->lt[PH_BWD], (hipStream_t)stream);
}

extern "C" int hx_req_free(hx_req** r) {
  if (!r || !*r) return HX_SUCCESS;
  if ((*r)->active) return fail(HX_ERR_STATE, "request active: wait before freeing it");
  if ((*r)->batch_refs > 0) return fail(HX_ERR_STATE, "request is a member of %d batch(es): free them first",
                                        (*r)->batch_refs);
  if ((*r)->comm) (*r)->comm->slot[(*r)->rank].req = nullptr;  // the collective forgets it
  delete *r;
  *r = nullptr;
  return HX_SUCCESS;
}

// ===========================================================================
// Batches
// ===========================================================================
namespace {

int capture_graph(hipStream_t cap, const std::function<int(hipStream_t)>& body, hipGraphExec_t* exec,
                  bool* has) {
  *has = false;
  HX_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int rc = body(cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cap, &g);
  if (rc != HX_SUCCESS) {
    if (e == hipSuccess && g) (void)hipGraphDestroy(g);
    return rc;
  }
  HX_HIP(e);
  size_t nn = 0;
  (void)hipGraphGetNodes(g, nullptr, &nn);
  if (nn == 0) {
    (void)hipGraphDestroy(g);
    return HX_SUCCESS;
  }
  hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HX_HIP(ie);
  *has = true;
  return HX_SUCCESS;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string s = p.gcnArchName;
  auto c = s.find(':');
  return c == std::string::npos ? s : s.substr(0, c);
}

int ilog2(int64_t v) {
  int l = 0;
  while (v > 1) { v >>= 1; ++l; }
  return l;
}

std::mutex g_cache_mu;

}  // namespace

void hx::batch_destroy_graphs(hx_batch* b) {
  for (int i = 0; i < 3; ++i) {
    if (b->has_graph[i]) (void)hipGraphExecDestroy(b->graph[i]);
    b->has_graph[i] = false;
  }
}

hx_batch::~hx_batch() {
  batch_destroy_graphs(this);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

int hx::batch_phase_jobs(const hx_batch* b, int phase, const Sched& sc, bool merged,
                         std::vector<std::vector<GatherJob>>* g, std::vector<std::vector<SegSumJob>>* s) {
  g->clear();
  s->clear();
  if (b->world) return world_phase_jobs(b, phase, sc, merged, g, s);
  for (hx_req* r : b->members) {
    std::vector<GatherJob> gj;
    std::vector<SegSumJob> sj;
    HX_TRY(req_phase_jobs(r, phase, sc, &gj, &sj));
    if (b->tuning)  // candidate launches of the tuner leave completion counters alone
      for (auto& j : gj) j.ready = nullptr;
    g->push_back(gj);
    s->push_back(sj);
  }
  return HX_SUCCESS;
}

// Batched launch table of a phase under a schedule (all members' jobs).
int hx::batch_build_table(const hx_batch* b, int phase, const Sched& sc, LaunchTable* t) {
  std::vector<std::vector<GatherJob>> g;
  std::vector<std::vector<SegSumJob>> s;
  HX_TRY(batch_phase_jobs(b, phase, sc, true, &g, &s));
  *t = LaunchTable();
  std::vector<GatherJob> ga;
  std::vector<SegSumJob> sa;
  for (auto& v : g) ga.insert(ga.end(), v.begin(), v.end());
  for (auto& v : s) sa.insert(sa.end(), v.begin(), v.end());
  return build_phase_table(phase, sc, b->dtype, (int)b->row_bytes, ga, sa, t);
}

// One launch per member: the plain form, with the library's default schedule.
int hx::batch_build_plain(hx_batch* b, int phase) {
  b->plain[phase].clear();
  std::vector<std::vector<GatherJob>> g;
  std::vector<std::vector<SegSumJob>> s;
  const int kind = phase == PH_BWD ? KIND_SEGSUM : KIND_GATHER;
  const Sched sc = default_sched(kind, (int)b->row_bytes);
  HX_TRY(batch_phase_jobs(b, phase, sc, false, &g, &s));
  const size_t nm = std::max(g.size(), s.size());
  b->plain[phase].resize(nm);
  for (size_t m = 0; m < nm; ++m) {
    static const std::vector<GatherJob> no_g;
    static const std::vector<SegSumJob> no_s;
    HX_TRY(build_phase_table(phase, sc, b->dtype, (int)b->row_bytes, m < g.size() ? g[m] : no_g,
                             m < s.size() ? s[m] : no_s, &b->plain[phase][m]));
  }
  b->plain_built[phase] = true;
  return HX_SUCCESS;
}

// (Re)builds the batched tables for the current schedules and captures the
// start / wait / backward graphs.
// Forwarder sums of a staged locality world (bound gradients), one job per
// forwarder: its terms are its own halo's rows and, mostly, its own stage-2
// slots (the window).  Runs on the backward phase's schedule.
static int build_fwd_sum_table(const hx_batch* b, const Sched& sc, LaunchTable* t) {
  *t = LaunchTable();
  if (!b->staged_bwd || !b->g_out) return HX_SUCCESS;
  std::vector<SegSumJob> fjs;
  for (int q = 0; q < b->R; ++q) {
    const int64_t k0 = b->r1_off[q];
    SegSumJob fj{b->g_in, b->g_r1.as<char>() + k0 * (int64_t)b->row_bytes, b->fwd_ptr.as<int32_t>() + k0,
                 b->fwd_idx.as<int32_t>(), b->r1_off[q + 1] - k0};
    fj.in2 = b->g_s2.as<char>();
    fj.split = (int32_t)b->H_tot;
    fj.win_lo = b->H_tot + b->s2_off[q];
    fj.win_rows = b->s2_off[q + 1] - b->s2_off[q];
    fjs.push_back(fj);
  }
  return build_segsum_table(fjs, b->dtype, (int)b->row_bytes, sc, t, TAG_FWD_SUM);
}

// Gradient bindings of a member batch's requests (the backward tables and
// graph hold their g_send / g_x pointers).
static std::vector<uint64_t> member_grad_gens(const hx_batch* b) {
  std::vector<uint64_t> v;
  v.reserve(b->members.size());
  for (const hx_req* r : b->members) v.push_back(r->grad_gen);
  return v;
}

int hx::batch_prepare(hx_batch* b) {
  batch_destroy_graphs(b);
  if (!b->world) b->bwd_gens_captured = member_grad_gens(b);
  for (int ph = 0; ph < 4; ++ph) HX_TRY(batch_build_table(b, ph, b->sched[ph], &b->lt[ph]));
  HX_TRY(build_fwd_sum_table(b, b->sched[PH_BWD], &b->lt_fwd_sum));
  if (!b->cap_stream) HX_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HX_TRY(capture_graph(b->cap_stream, [&](hipStream_t s) { return batch_run_start(b, s); }, &b->graph[0],
                       &b->has_graph[0]));
  HX_TRY(capture_graph(b->cap_stream, [&](hipStream_t s) { return batch_run_wait(b, s); }, &b->graph[1],
                       &b->has_graph[1]));
  HX_TRY(capture_graph(b->cap_stream, [&](hipStream_t s) { return batch_run_backward(b, s); },
                       &b->graph[2], &b->has_graph[2]));
  return HX_SUCCESS;
}

int hx::batch_run_start(hx_batch* b, hipStream_t s) {
  HX_TRY(launch_table(b->lt[PH_PACK], s));
  if (b->world && (b->flags & HX_WORLD_SIM_TRANSFER)) HX_TRY(launch_table(b->lt_xfer[0], s));
  return HX_SUCCESS;
}

int hx::batch_run_wait(hx_batch* b, hipStream_t s) {
  HX_TRY(launch_table(b->lt[PH_REDIST], s));
  if (b->world && (b->flags & HX_WORLD_SIM_TRANSFER)) HX_TRY(launch_table(b->lt_xfer[1], s));
  HX_TRY(launch_table(b->lt[PH_UNPACK], s));
  return HX_SUCCESS;
}

static std::string cache_key(const hx_batch* b, int phase) {
  std::ostringstream k;
  int64_t rows = 0;
  int njobs = 0;
  std::vector<std::vector<GatherJob>> g;
  std::vector<std::vector<SegSumJob>> s;
  Sched neutral;  // the shape key counts rows of the pull form, whatever the schedule
  if (batch_phase_jobs(b, phase, neutral, true, &g, &s) == HX_SUCCESS) {
    for (auto& v : g) for (auto& j : v) { rows += j.nrows; ++njobs; }
    for (auto& v : s) for (auto& j : v) { rows += j.nrows; ++njobs; }
  }
  k << arch_name() << "|p" << phase << "|t" << b->dtype << "|rb" << b->row_bytes << "|r" << ilog2(rows + 1)
    << "|j" << ilog2(njobs + 1) << "|w" << (b->world ? 1 : 0);
  if (b->world) k << "|v" << b->variant;  // 2-step and 3-step worlds differ in shape
  if (phase == PH_BWD && b->staged_bwd) k << "|staged";  // forwarder + owner sums, not the closed form
  return k.str();
}

static const char* cache_path() { return std::getenv("HX_TUNE_CACHE"); }

static bool cache_lookup(const std::string& key, Sched* out) {
  const char* path = cache_path();
  if (!path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k;
    Sched s;
    if (!(ls >> k >> s.tile_rows >> s.block_threads >> s.blocks_per_cu >> s.nontemporal >> s.per_neighbor >>
          s.unroll >> s.push_pack))
      continue;
    if (!(ls >> s.lds_window)) s.lds_window = 0;  // lines written before the field existed
    if (!(ls >> s.pair_rows)) s.pair_rows = 0;
    if (k == key) { *out = s; found = true; }
  }
  return found;
}

static void cache_store(const std::string& key, const Sched& s) {
  const char* path = cache_path();
  if (!path) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << s.tile_rows << ' ' << s.block_threads << ' ' << s.blocks_per_cu << ' ' << s.nontemporal
    << ' ' << s.per_neighbor << ' ' << s.unroll << ' ' << s.push_pack << ' ' << s.lds_window << ' ' << s.pair_rows
    << '\n';
}

// Members with pack completion counters need the pull form of the pack.
static bool batch_has_ready(const hx_batch* b) {
  for (const hx_req* r : b->members)
    if (r->ready.p) return true;
  return false;
}

int hx::batch_init_scheds(hx_batch* b, const hx_sched* sched) {
  for (int ph = 0; ph < 4; ++ph) {
    b->sched_from_cache[ph] = sched == nullptr;
    const int kind = ph == PH_BWD ? KIND_SEGSUM : KIND_GATHER;
    if (sched) {
      b->sched[ph] = resolve_sched(sched, kind, (int)b->row_bytes);
    } else {
      Sched s;
      b->sched[ph] = cache_lookup(cache_key(b, ph), &s) ? s : default_sched(kind, (int)b->row_bytes);
    }
  }
  if (batch_has_ready(b)) b->sched[PH_PACK].push_pack = 0;
  return HX_SUCCESS;
}

extern "C" int hx_batch_init(hx_req* const* reqs, int n, const hx_sched* sched, hx_batch** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (n <= 0 || !reqs) return fail(HX_ERR_ARG, "empty batch");
  for (int i = 0; i < n; ++i) {
    if (!reqs[i]) return fail(HX_ERR_ARG, "null member %d", i);
    HX_TRY(req_usable(reqs[i]));
    if (reqs[i]->dtype != reqs[0]->dtype || reqs[i]->ncols != reqs[0]->ncols)
      return fail(HX_ERR_ARG, "members differ in dtype or ncols");
  }
  std::unique_ptr<hx_batch> b(new (std::nothrow) hx_batch);
  if (!b) return fail(HX_ERR_NOMEM, "out of host memory");
  b->world = false;
  b->dtype = reqs[0]->dtype;
  b->ncols = reqs[0]->ncols;
  b->row_bytes = reqs[0]->row_bytes;
  b->members.assign(reqs, reqs + n);
  for (int ph = 0; ph < 4; ++ph) {
    b->bytes[ph] = 0;
    for (hx_req* r : b->members) b->bytes[ph] += r->bytes[ph];
  }
  HX_TRY(batch_init_scheds(b.get(), sched));
  HX_TRY(batch_prepare(b.get()));
  for (hx_req* r : b->members) ++r->batch_refs;  // released by hx_batch_free
  *out = b.release();
  return HX_SUCCESS;
}

// Replays start (0), wait (1) or backward (2): the captured graph, or the
// same launch tables directly.
static int launch_graph(hx_batch* b, int which, hipStream_t s) {
  if (b->replay_direct) {
    if (which == 0) return batch_run_start(b, s);
    if (which == 1) return batch_run_wait(b, s);
    return batch_run_backward(b, s);
  }
  if (!b->has_graph[which]) return HX_SUCCESS;
  HX_HIP(hipGraphLaunch(b->graph[which], s));
  return HX_SUCCESS;
}

extern "C" int hx_batch_set_sched(hx_batch* b, int phase, const hx_sched* sched) {
  if (!b || !sched) return fail(HX_ERR_ARG, "null argument");
  if (phase < 0 || phase > 3) return fail(HX_ERR_ARG, "bad phase %d", phase);
  if (b->active) return fail(HX_ERR_STATE, "batch is active");
  const int kind = phase == PH_BWD ? KIND_SEGSUM : KIND_GATHER;
  const Sched old = b->sched[phase];
  b->sched[phase] = resolve_sched(sched, kind, (int)b->row_bytes);
  b->sched_from_cache[phase] = false;
  if (phase == PH_PACK && batch_has_ready(b)) b->sched[PH_PACK].push_pack = 0;
  const int rc = batch_prepare(b);
  if (rc != HX_SUCCESS) {
    b->sched[phase] = old;  // keep the batch usable with its previous schedule
    (void)batch_prepare(b);
  }
  return rc;
}

extern "C" int hx_batch_set_replay(hx_batch* b, int mode) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (mode != HX_REPLAY_GRAPH && mode != HX_REPLAY_DIRECT) return fail(HX_ERR_ARG, "bad replay mode %d", mode);
  b->replay_direct = mode == HX_REPLAY_DIRECT;
  return HX_SUCCESS;
}

extern "C" int hx_batch_get_replay(const hx_batch* b, int* mode) {
  if (!b || !mode) return fail(HX_ERR_ARG, "null argument");
  *mode = b->replay_direct ? HX_REPLAY_DIRECT : HX_REPLAY_GRAPH;
  return HX_SUCCESS;
}

// Average time of `reps` start + wait steps in one replay mode (after one
// warm-up step); the batch keeps that mode.
static int time_replay(hx_batch* b, hipStream_t s, bool direct, int reps, float* ms) {
  b->replay_direct = direct;
  hipEvent_t e0, e1;
  HX_HIP(hipEventCreate(&e0));
  HX_HIP(hipEventCreate(&e1));
  int rc = launch_graph(b, 0, s);
  if (rc == HX_SUCCESS) rc = launch_graph(b, 1, s);
  if (rc == HX_SUCCESS && hipEventRecord(e0, s) != hipSuccess) rc = fail(HX_ERR_HIP, "event record");
  for (int i = 0; i < reps && rc == HX_SUCCESS; ++i) {
    rc = launch_graph(b, 0, s);
    if (rc == HX_SUCCESS) rc = launch_graph(b, 1, s);
  }
  if (rc == HX_SUCCESS && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    rc = fail(HX_ERR_HIP, "event timing");
  if (rc == HX_SUCCESS) *ms /= (float)reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

extern "C" int hx_batch_start(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (b->active) return fail(HX_ERR_STATE, "batch already active");
  HX_TRY(launch_graph(b, 0, (hipStream_t)stream));
  b->active = true;
  return HX_SUCCESS;
}

extern "C" int hx_batch_wait(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (!b->active) return HX_SUCCESS;
  HX_TRY(launch_graph(b, 1, (hipStream_t)stream));
  b->active = false;
  return HX_SUCCESS;
}

extern "C" int hx_batch_start_plain(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (b->active) return fail(HX_ERR_STATE, "batch already active");
  hipStream_t s = (hipStream_t)stream;
  if (!b->plain_built[PH_PACK]) HX_TRY(batch_build_plain(b, PH_PACK));
  for (auto& t : b->plain[PH_PACK]) HX_TRY(launch_table(t, s));
  if (b->world && (b->flags & HX_WORLD_SIM_TRANSFER)) HX_TRY(launch_table(b->lt_xfer[0], s));
  b->active = true;
  return HX_SUCCESS;
}

extern "C" int hx_batch_wait_plain(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (!b->active) return HX_SUCCESS;
  hipStream_t s = (hipStream_t)stream;
  if (!b->plain_built[PH_REDIST]) HX_TRY(batch_build_plain(b, PH_REDIST));
  if (!b->plain_built[PH_UNPACK]) HX_TRY(batch_build_plain(b, PH_UNPACK));
  for (auto& t : b->plain[PH_REDIST]) HX_TRY(launch_table(t, s));
  if (b->world && (b->flags & HX_WORLD_SIM_TRANSFER)) HX_TRY(launch_table(b->lt_xfer[1], s));
  for (auto& t : b->plain[PH_UNPACK]) HX_TRY(launch_table(t, s));
  b->active = false;
  return HX_SUCCESS;
}

extern "C" int hx_batch_bind_grad(hx_batch* b, const void* g_in, void* g_out) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (!b->world) return fail(HX_ERR_ARG, "member batches use each member's hx_req_bind_grad");
  // (empty buffers may be null: a decomposition without halo entries, or without rows)
  if ((!g_in && b->H_tot > 0) || (!g_out && b->n > 0)) return fail(HX_ERR_ARG, "null gradient buffer");
  b->g_in = static_cast<const char*>(g_in);
  b->g_out = static_cast<char*>(g_out);
  b->plain_built[PH_BWD] = false;
  const int rbi = (int)b->row_bytes;
  const Sched gsc = default_sched(KIND_GATHER, rbi);
  if (b->unpack_identity) {
    // plain world: halo gradients travel back to the senders' slots (the
    // simulated reverse transfer), then each rank sums its own slots
    HX_TRY(b->g_send_all.alloc((size_t)b->E1_tot * b->row_bytes));
    std::vector<GatherJob> xb{GatherJob{b->g_in, b->g_send_all.as<char>(), b->gidx_back.as<int32_t>(), b->E1_tot}};
    HX_TRY(build_gather_table(xb, b->dtype, rbi, gsc, &b->lt_xfer[2]));
  } else if (b->staged_bwd) {
    // locality world, staged: forwarder sums read the halo gradients (own
    // terms) and the stage-2 send-slot gradients (split = H)
    HX_TRY(b->g_s2.alloc((size_t)b->E2_tot * b->row_bytes));
    HX_TRY(b->g_r1.alloc((size_t)b->R1_tot * b->row_bytes));
    HX_TRY(b->g_send_all.alloc((size_t)b->E1_tot * b->row_bytes));
    std::vector<GatherJob> x2{GatherJob{b->g_in, b->g_s2.as<char>(), b->gidx_back2.as<int32_t>(), b->E2_tot}};
    HX_TRY(build_gather_table(x2, b->dtype, rbi, gsc, &b->lt_xfer[3]));
    std::vector<GatherJob> x1{GatherJob{b->g_r1.as<char>(), b->g_send_all.as<char>(), b->gidx_back.as<int32_t>(),
                                        b->E1_tot}};
    HX_TRY(build_gather_table(x1, b->dtype, rbi, gsc, &b->lt_xfer[2]));
  }
  // the backward's shape (and so its tuning-cache key) exists only now
  Sched cached;
  if (b->sched_from_cache[PH_BWD] && cache_lookup(cache_key(b, PH_BWD), &cached)) b->sched[PH_BWD] = cached;
  return batch_prepare(b);
}

// Backward of a batch.  Plain worlds: with the simulated transport the
// reverse stage-1 transfer first, then the owner sums.  Staged locality
// worlds: [reverse stage-2 transfer], forwarder sums, [reverse stage-1
// transfer], owner sums.  Others: the fixed-order sums.
static int run_backward(hx_batch* b, hipStream_t s, bool plain_form) {
  const bool sim = b->world && (b->flags & HX_WORLD_SIM_TRANSFER);
  if (b->world && b->staged_bwd) {
    if (sim) HX_TRY(launch_table(b->lt_xfer[3], s));
    HX_TRY(launch_table(b->lt_fwd_sum, s));
    if (sim) HX_TRY(launch_table(b->lt_xfer[2], s));
  } else if (b->world && b->unpack_identity && sim) {
    HX_TRY(launch_table(b->lt_xfer[2], s));
  }
  if (!plain_form) return launch_table(b->lt[PH_BWD], s);
  for (auto& t : b->plain[PH_BWD]) HX_TRY(launch_table(t, s));
  return HX_SUCCESS;
}

// Member gradients bound (or rebound to other buffers) since the backward
// tables were built: rebuild the tables (batched and plain) and recapture
// the graphs.
static int refresh_member_grads(hx_batch* b) {
  if (b->world || member_grad_gens(b) == b->bwd_gens_captured) return HX_SUCCESS;
  b->plain_built[PH_BWD] = false;
  Sched cached;  // gradients bound after the batch was made: the backward's cache key changes
  if (b->sched_from_cache[PH_BWD] && cache_lookup(cache_key(b, PH_BWD), &cached)) b->sched[PH_BWD] = cached;
  return batch_prepare(b);
}

extern "C" int hx_batch_backward(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (b->world && !b->g_out) return fail(HX_ERR_STATE, "no gradient buffers bound");
  HX_TRY(refresh_member_grads(b));
  return launch_graph(b, 2, (hipStream_t)stream);
}

extern "C" int hx_batch_backward_plain(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (b->world && !b->g_out) return fail(HX_ERR_STATE, "no gradient buffers bound");
  HX_TRY(refresh_member_grads(b));
  if (!b->plain_built[PH_BWD]) HX_TRY(batch_build_plain(b, PH_BWD));
  return run_backward(b, (hipStream_t)stream, true);
}

int hx::batch_run_backward(hx_batch* b, hipStream_t s) { return run_backward(b, s, false); }

// One phase's kernel on its own, launched directly from the same
// launch table the graphs replay (for per-kernel timing).
extern "C" int hx_batch_launch_phase(hx_batch* b, int phase, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (phase < 0 || phase > 3) return fail(HX_ERR_ARG, "bad phase %d", phase);
  if (b->active) return fail(HX_ERR_STATE, "batch active: call hx_batch_wait first");
  if (phase == PH_BWD) {
    if (b->world && !b->g_out) return fail(HX_ERR_STATE, "no gradient buffers bound");
    if (!b->world && member_grad_gens(b) != b->bwd_gens_captured)
      return fail(HX_ERR_STATE, "gradients bound after the last backward: call hx_batch_backward once first");
  }
  if (phase == PH_BWD && b->world && b->staged_bwd)  // the staged backward's forwarder sums first
    HX_TRY(launch_table(b->lt_fwd_sum, (hipStream_t)stream));
  return launch_table(b->lt[phase], (hipStream_t)stream);
}

extern "C" int hx_batch_get_sched(const hx_batch* b, int phase, hx_sched* out) {
  if (!b || !out || phase < 0 || phase > 3) return fail(HX_ERR_ARG, "bad argument");
  *out = to_public(b->sched[phase]);
  return HX_SUCCESS;
}

extern "C" int hx_batch_bytes(const hx_batch* b, int phase, int64_t* bytes) {
  if (!b || !bytes || phase < 0 || phase > 3) return fail(HX_ERR_ARG, "bad argument");
  *bytes = b->bytes[phase];
  return HX_SUCCESS;
}

// ---------------------------------------------------------------------------
// Tuner: times candidate schedules for each phase on the batch's buffers.
// ---------------------------------------------------------------------------
// Average launch time of a table: `reps` back-to-back launches between two
// events (queued faster than they run, so host launch cost stays hidden),
// best of two trials after a warm-up launch.
static int time_table(const LaunchTable& t, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, float* best) {
  HX_TRY(launch_table(t, s));  // warm-up
  *best = 1e30f;
  for (int trial = 0; trial < 2; ++trial) {
    HX_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) HX_TRY(launch_table(t, s));
    HX_HIP(hipEventRecord(e1, s));
    HX_HIP(hipEventSynchronize(e1));
    float ms = 0;
    HX_HIP(hipEventElapsedTime(&ms, e0, e1));
    *best = std::min(*best, ms / reps);
    // short kernels: enough launches for about a millisecond per trial (at
    // most 50), so that clock noise stays below the 2 % a candidate must win by
    if (trial == 0 && *best * reps < 1.0f) reps = std::min(50, std::max(reps, (int)std::ceil(1.0f / *best)));
  }
  return HX_SUCCESS;
}

extern "C" int hx_batch_tune(hx_batch* b, void* stream) {
  if (!b) return fail(HX_ERR_ARG, "null batch");
  if (b->active) return fail(HX_ERR_STATE, "batch is active");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HX_HIP(hipEventCreate(&e0));
  HX_HIP(hipEventCreate(&e1));
  const bool log = std::getenv("HX_TUNE_LOG") != nullptr;  // every candidate's time on stderr
  struct TuningFlag {
    hx_batch* b;
    ~TuningFlag() { b->tuning = false; }
  } tuning_flag{b};
  b->tuning = true;
  int rc = HX_SUCCESS;
  for (int ph = 0; ph < 4 && rc == HX_SUCCESS; ++ph) {
    if (b->lt[ph].empty()) continue;
    const int kind = ph == PH_BWD ? KIND_SEGSUM : KIND_GATHER;
    const int rb = (int)b->row_bytes;
    const int base = default_sched(kind, rb).tile_rows;
    Sched best = b->sched[ph];
    float best_ms = 1e30f;
    auto consider = [&](const Sched& c) {
      if (rc != HX_SUCCESS) return;
      LaunchTable t;
      rc = batch_build_table(b, ph, c, &t);
      if (rc != HX_SUCCESS) return;
      float ms = 0;
      rc = time_table(t, s, e0, e1, 3, &ms);
      if (rc == HX_SUCCESS && ph == PH_BWD && b->staged_bwd) {  // forwarder sums share the schedule
        LaunchTable tf;
        float msf = 0;
        rc = build_fwd_sum_table(b, c, &tf);
        if (rc == HX_SUCCESS) rc = time_table(tf, s, e0, e1, 3, &msf);
        ms += msf;
      }
      if (log)
        std::fprintf(stderr, "hx tune phase %d: tile %d bt %d bpc %d nt %d unroll %d push %d win %d pair %d: %.4f ms\n",
                     ph, c.tile_rows, c.block_threads, c.blocks_per_cu, c.nontemporal, c.unroll, c.push_pack,
                     c.lds_window, c.pair_rows, ms);
      if (rc == HX_SUCCESS && ms < best_ms * 0.98f) {
        best_ms = ms;
        best = c;
      }
    };
    consider(best);
    // seeds for gathers of 4- and 8-byte rows: 16-byte row groups per lane,
    // one-shot grids, with whole-job LDS windows (sources in a known window)
    // and without (measured best on the random-matrix exchange); the
    // stage-by-stage search below refines from the fastest
    if (ph != PH_BWD && (rb == 4 || rb == 8) && !(ph == PH_PACK && best.push_pack)) {
      for (int win : {1, 0})
        for (int bt : {256, 512})
          for (int nt : {0, 1}) {
            Sched c = best;
            c.pair_rows = 1;
            c.lds_window = win;
            c.tile_rows = win ? 16384 : 4096;
            c.block_threads = bt;
            c.blocks_per_cu = kOneShotBpc;
            c.unroll = 4;
            c.nontemporal = nt;
            c.per_neighbor = 0;
            c.push_pack = 0;
            consider(c);
          }
    }
    // seeds for segmented sums of rows of one value: one row per lane,
    // per-job LDS term windows or none, one-shot grids
    if (ph == PH_BWD && (rb == 4 || rb == 8) && (size_t)rb == dtype_bytes(b->dtype)) {
      for (int win : {1, 0})
        for (int bt : {256, 512})
          for (int u : {2, 4}) {
            Sched c = best;
            c.pair_rows = 1;
            c.lds_window = win;
            c.tile_rows = 16384;
            c.block_threads = bt;
            c.blocks_per_cu = kOneShotBpc;
            c.unroll = u;
            c.nontemporal = 0;
            c.per_neighbor = 0;
            consider(c);
          }
    }
    // stage 1: work per tile, rows in flight, pull vs push (pack), LDS
    // source windows and two rows per lane (gathers); stage 2: launch shape
    // (persistent or one-shot grid, workgroup size) and streaming hints;
    // stage 3: stage 1 again around the new launch shape; stage 4: rows in
    // flight x launch shape
    auto tile_stage = [&]() {
      const Sched s0 = best;
      for (int tf : {1, 2, 4, 8, 16, 32})
        for (int u : {1, 2, 4})
          for (int push : {0, 1})
            for (int win : {0, 1})
              for (int pair : {0, 1}) {
                if (push && (ph != PH_PACK || batch_has_ready(b))) continue;
                if (win && push) continue;
                // 16-byte row groups per lane: pull gathers of 4- or 8-byte rows;
                // segmented sums of rows of one value: one row per lane
                if (pair && ((b->row_bytes != 8 && b->row_bytes != 4) || push ||
                             (ph == PH_BWD && b->row_bytes != dtype_bytes(b->dtype))))
                  continue;
                Sched c = s0;
                c.tile_rows = std::max(16, base * tf / 8);
                c.unroll = u;
                c.push_pack = ph == PH_PACK ? push : s0.push_pack;
                c.lds_window = win;
                c.pair_rows = pair;
                c.per_neighbor = 0;
                consider(c);
              }
    };
    tile_stage();
    {
      const Sched s1 = best;
      for (int bpc : {2, 4, 8, kOneShotBpc})
        for (int bt : {256, 512, 1024})
          for (int nt : {0, 1})
            for (int flip : {0, 1}) {
              // (gathers: LDS windows again with each launch shape, where the
              // occupancy they allow depends on the workgroup size)
              if (bt == 1024 && ph == PH_PACK && s1.push_pack) continue;  // push pack: at most 512 lanes
              if (flip && (ph == PH_BWD || (ph == PH_PACK && s1.push_pack))) continue;
              Sched c = s1;
              c.lds_window = flip ? !s1.lds_window : s1.lds_window;
              c.blocks_per_cu = bpc;
              c.block_threads = bt;
              c.nontemporal = nt;
              consider(c);
            }
    }
    tile_stage();
    // stage 4: rows in flight and launch shape together around the chosen
    // tile (the stage-by-stage search can stop at a near tie between them)
    {
      const Sched s3 = best;
      for (int u : {1, 2, 4})
        for (int bpc : {2, 4, 8, kOneShotBpc})
          for (int bt : {256, 512, 1024}) {
            if (bt == 1024 && ph == PH_PACK && s3.push_pack) continue;  // push pack: at most 512 lanes
            Sched c = s3;
            c.unroll = u;
            c.blocks_per_cu = bpc;
            c.block_threads = bt;
            consider(c);
          }
    }
    // stage 5: one job per message (member batches, pull forms)
    if (!b->world && !(ph == PH_PACK && best.push_pack) && ph != PH_BWD) {
      Sched c = best;
      c.per_neighbor = 1;
      consider(c);
    }
    // stage 6: streaming loads for the LDS window staging of 4- and 8-byte
    // row gathers (a window is read once; it pays where the arena was not
    // just left in the caches by the previous phase)
    if (ph != PH_BWD && (rb == 4 || rb == 8) && best.pair_rows && best.lds_window && !(ph == PH_PACK && best.push_pack)) {
      Sched c = best;
      c.nontemporal = 2;
      consider(c);
    }
    if (rc == HX_SUCCESS) {
      b->sched[ph] = best;
      b->sched_from_cache[ph] = false;  // tuned here: kept when gradients are bound again
      cache_store(cache_key(b, ph), best);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HX_TRY(rc);
  // replay: the captured graphs, or the same tables launched directly where
  // that measures faster (a graph launch has a fixed cost).  The trial runs
  // on tables built while tuning, which signal no completion counters.
  HX_TRY(batch_prepare(b));
  float ms_graph = 0, ms_direct = 0;
  int rr = time_replay(b, s, false, 20, &ms_graph);
  if (rr == HX_SUCCESS) rr = time_replay(b, s, true, 20, &ms_direct);
  const bool direct = rr == HX_SUCCESS && ms_direct < ms_graph * 0.98f;
  if (log && rr == HX_SUCCESS)
    std::fprintf(stderr, "hx tune replay: graph %.4f ms, direct %.4f ms per start + wait -> %s\n", ms_graph,
                 ms_direct, direct ? "direct" : "graph");
  b->tuning = false;  // the tables kept for Start/Wait signal their counters again
  HX_TRY(batch_prepare(b));
  b->replay_direct = direct;
  return rr;
}

extern "C" int hx_batch_free(hx_batch** b) {
  if (!b || !*b) return HX_SUCCESS;
  for (hx_req* r : (*b)->members) --r->batch_refs;
  delete *b;
  *b = nullptr;
  return HX_SUCCESS;
}

// ===========================================================================
// Errors / version
// ===========================================================================
extern "C" const char* hx_error_string(int code) {
  switch (code) {
    case HX_SUCCESS: return "success";
    case HX_ERR_ARG: return "invalid argument";
    case HX_ERR_RANGE: return "index out of range";
    case HX_ERR_STATE: return "invalid request state";
    case HX_ERR_NOMEM: return "out of memory";
    case HX_ERR_UNSUPPORTED: return "unsupported";
    case HX_ERR_HIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

extern "C" int hx_set_allocator(hx_alloc_fn alloc_fn, hx_free_fn free_fn, void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(HX_ERR_ARG, "hx_set_allocator: give both functions or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc_fn = alloc_fn;
  g_free_fn = free_fn;
  g_alloc_ctx = alloc_fn ? ctx : nullptr;
  return HX_SUCCESS;
}

extern "C" int hx_last_hip_error(void) { return g_hip; }
extern "C" const char* hx_last_error_message(void) { return g_msg.c_str(); }
extern "C" const char* hx_version(void) { return "hx 0.1 gfx950"; }
