// Requests and whole-decomposition batches ("worlds") built from a plan.
//
// A world keeps every rank's arenas in one flat allocation each:
//   send_all = [stage-1 send of rank 0, 1, ... | stage-2 send of rank 0, 1, ...]
//   recv_all = [stage-1 recv of rank 0, 1, ... | stage-2 recv of rank 0, 1, ...]
// and turns each phase into one gather over global row indices, so a phase
// of all ranks is a single launch (one job per rank where the job's LDS
// window is its own rank's rows or arena).  The simulated transfer of a stage
// is one more gather, from each sender's message segment into the receiver's
// slots.  The backward is the closed-form adjoint over halo_all rows, or, for
// a locality plan with HX_WORLD_STAGED_BACKWARD, the forward's stages in
// reverse (forwarder sums, then owner sums).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "common.h"
#include "internal.h"

namespace hx {
namespace {

constexpr int TB = 256;

unsigned blocks_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TB - 1) / TB, 1 << 16));
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ int upper_rank(const int64_t* __restrict__ starts, int R, int64_t v) {
  int lo = 0, hi = R - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Largest l in [a, b) with v[l] <= x (v ascending).
__device__ __forceinline__ int64_t upper_in(const int32_t* __restrict__ v, int64_t a, int64_t b, int64_t x) {
  int64_t lo = a, hi = b - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// out[k] = base[rank(k)] + in[k], rank(k) from the entry offsets.
__global__ void k_add_rank_base(const int32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ off, int R,
                                const int64_t* __restrict__ base, int32_t* out) {
  GRID_STRIDE(k, n) {
    const int r = upper_rank(off, R, k);
    out[k] = (int32_t)(base[r] + in[k]);
  }
}

// Transpose of the pack map in world coordinates: global row -> rows of
// send_all, from the per-rank transposes (local rows, local slots).
__global__ void k_world_pack_ptr(const int32_t* __restrict__ bt_ptr, const int64_t* __restrict__ bt_off,
                                 const int64_t* __restrict__ rs, const int64_t* __restrict__ s1_off, int R, int64_t n,
                                 int64_t E1_tot, int32_t* out) {
  GRID_STRIDE(g, n + 1) {
    if (g == n) {
      out[g] = (int32_t)E1_tot;
      continue;
    }
    const int q = upper_rank(rs, R, g);
    out[g] = (int32_t)(bt_ptr[bt_off[q] + (g - rs[q])] + s1_off[q]);
  }
}

__global__ void k_fill_neg(int32_t* p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = -1;
}

__global__ void k_fill_zero(int32_t* p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = 0;
}

// inv[map[i]] = i for a permutation map (out-of-range targets are skipped and
// leave -1, which the range check then reports).
__global__ void k_invert(const int32_t* __restrict__ map, int64_t n, int32_t* inv) {
  GRID_STRIDE(i, n) {
    const int32_t t = map[i];
    if (t >= 0 && t < n) inv[t] = (int32_t)i;
  }
}

// inv[map[i] - lo] = i for the n entries of an injective map (targets
// outside [lo, lo + range) are skipped; untouched entries keep their fill).
__global__ void k_invert_range(const int32_t* __restrict__ map, int64_t n, int64_t lo, int64_t range, int32_t* inv) {
  GRID_STRIDE(i, n) {
    const int64_t t = (int64_t)map[i] - lo;
    if (t >= 0 && t < range) inv[t] = (int32_t)i;
  }
}

// out[e] = b[off + a[e]] (composition of two maps).
__global__ void k_compose(const int32_t* __restrict__ a, int64_t n, const int32_t* __restrict__ b, int64_t off,
                          int32_t* out) {
  GRID_STRIDE(e, n) out[e] = b[off + a[e]];
}

// Number of terms of every forwarder sum: the own-halo term when the slot's
// own rank reads it (own[k] >= 0), plus its redistribution entries.
__global__ void k_forward_lens(const int32_t* __restrict__ own, const int32_t* __restrict__ gp, int64_t n,
                               int32_t* out) {
  GRID_STRIDE(k, n) out[k] = (own[k] >= 0 ? 1 : 0) + gp[k + 1] - gp[k];
}

// Forwarder-sum CSR (staged backward): the terms of stage-1 receive slot k
// are its own halo's gradient row own[k] (when read), then the stage-2 send
// slots e that forward it, in ascending e, as rows split + e.
__global__ void k_forward_terms(const int32_t* __restrict__ own, const int32_t* __restrict__ gp,
                                const int32_t* __restrict__ gperm, const int32_t* __restrict__ fptr, int64_t R1_tot,
                                int64_t split, int32_t* fidx) {
  GRID_STRIDE(k, R1_tot) {
    int32_t pos = fptr[k];
    if (own[k] >= 0) fidx[pos++] = own[k];
    for (int32_t j = gp[k]; j < gp[k + 1]; ++j) fidx[pos++] = (int32_t)(split + gperm[j]);
  }
}

// Unpack map in world coordinates: slot u of rank r's [stage-1 | stage-2]
// receive arena -> row of recv_all.
__global__ void k_world_unpack(const int32_t* __restrict__ u, int64_t n, const int64_t* __restrict__ hoff, int R,
                               const int64_t* __restrict__ r1_off, const int64_t* __restrict__ r2_off,
                               int64_t R1_tot, int32_t* out) {
  GRID_STRIDE(e, n) {
    const int r = upper_rank(hoff, R, e);
    const int64_t R1r = r1_off[r + 1] - r1_off[r];
    const int64_t v = u[e];
    out[e] = (int32_t)(v < R1r ? r1_off[r] + v : R1_tot + r2_off[r] + (v - R1r));
  }
}

// Simulated transfer of one stage: for every receive slot, the row of the
// sender's send arena holding it.  Receive lists (procs, displs, entry
// offsets) of each rank and send lists of each rank, all ascending.
__global__ void k_transfer_map(int64_t nslots, int R, const int64_t* __restrict__ roff,
                               const int64_t* __restrict__ rp_off, const int32_t* __restrict__ r_procs,
                               const int32_t* __restrict__ r_counts, const int32_t* __restrict__ r_displs,
                               const int64_t* __restrict__ soff, const int64_t* __restrict__ sp_off,
                               const int32_t* __restrict__ s_procs, const int32_t* __restrict__ s_counts,
                               const int32_t* __restrict__ s_displs, int64_t send_base, int32_t* out,
                               int* err) {
  GRID_STRIDE(i, nslots) {
    const int r = upper_rank(roff, R, i);
    const int64_t il = i - roff[r];
    if (rp_off[r + 1] <= rp_off[r]) {
      atomicOr(err, 1);
      out[i] = 0;
      continue;
    }
    const int64_t l = upper_in(r_displs, rp_off[r], rp_off[r + 1], il);
    const int q = r_procs[l];
    const int64_t a = sp_off[q], b = sp_off[q + 1];
    const int64_t pos = upper_in(s_procs, a, b, r);
    if (b <= a || s_procs[pos] != r || s_counts[pos] != r_counts[l]) {
      atomicOr(err, 1);
      out[i] = 0;
      continue;
    }
    out[i] = (int32_t)(send_base + soff[q] + s_displs[pos] + (il - r_displs[l]));
  }
}

int check_err(const DevMem& err, const char* what) {
  int h = 0;
  HX_HIP(hipMemcpy(&h, err.p, sizeof h, hipMemcpyDeviceToHost));
  if (h) return fail(HX_ERR_ARG, "%s: send and receive lists do not match", what);
  return HX_SUCCESS;
}

}  // namespace

int world_phase_jobs(const hx_batch* b, int phase, const Sched& sc, bool merged,
                     std::vector<std::vector<GatherJob>>* g, std::vector<std::vector<SegSumJob>>* s) {
  const int64_t rb = (int64_t)b->row_bytes;
  const char* sa = b->send_all.as<char>();
  const char* ra = b->recv_all.as<char>();
  switch (phase) {
    case PH_PACK:
      if (sc.push_pack) {
        if (b->E1_tot == 0) break;
        if (merged) {
          s->push_back({SegSumJob{b->x_global, (char*)sa, b->wp_ptr.as<int32_t>(), b->wp_idx.as<int32_t>(), b->n}});
        } else {
          for (int r = 0; r < b->R; ++r) {
            const int64_t r0 = b->row_starts[r];
            s->push_back({SegSumJob{b->x_global + r0 * rb, (char*)sa, b->wp_ptr.as<int32_t>() + r0,
                                    b->wp_idx.as<int32_t>(), b->row_starts[r + 1] - r0}});
          }
        }
      } else if (merged && !sc.lds_window) {
        g->push_back({GatherJob{b->x_global, (char*)sa, b->gidx_pack.as<int32_t>(), b->E1_tot}});
      } else {
        // one job per rank: its indices stay inside its own rows (the window)
        std::vector<GatherJob> v;
        for (int r = 0; r < b->R; ++r)
          v.push_back(GatherJob{b->x_global, (char*)sa + b->s1_off[r] * rb, b->gidx_pack.as<int32_t>() + b->s1_off[r],
                                b->s1_off[r + 1] - b->s1_off[r], b->row_starts[r],
                                b->row_starts[r + 1] - b->row_starts[r]});
        if (merged) g->push_back(v);
        else for (auto& x : v) g->push_back({x});
      }
      break;
    case PH_REDIST:
      if (merged && !sc.lds_window) {
        g->push_back({GatherJob{ra, (char*)sa + b->E1_tot * rb, b->gidx_redist.as<int32_t>(), b->E2_tot}});
      } else {
        // one job per rank: it forwards values from its own stage-1 receive arena
        std::vector<GatherJob> v;
        for (int r = 0; r < b->R; ++r)
          v.push_back(GatherJob{ra, (char*)sa + (b->E1_tot + b->s2_off[r]) * rb,
                                b->gidx_redist.as<int32_t>() + b->s2_off[r], b->s2_off[r + 1] - b->s2_off[r],
                                b->r1_off[r], b->r1_off[r + 1] - b->r1_off[r]});
        if (merged) g->push_back(v);
        else for (auto& x : v) g->push_back({x});
      }
      break;
    case PH_UNPACK:
      if (merged && (b->unpack_identity || !sc.lds_window)) {
        g->push_back({GatherJob{ra, b->halo_all, b->unpack_identity ? nullptr : b->gidx_unpack.as<int32_t>(),
                                b->H_tot}});
      } else if (!b->unpack_identity) {
        // one job per rank; its window is its stage-2 receive arena, where
        // nearly all of its halo comes from (entries from the stage-1 arena
        // read global memory)
        std::vector<GatherJob> v;
        for (int r = 0; r < b->R; ++r) {
          const int64_t h0 = b->halo_off[r], h = b->halo_off[r + 1] - h0;
          v.push_back(GatherJob{ra, b->halo_all + h0 * rb, b->gidx_unpack.as<int32_t>() + h0, h,
                                b->R1_tot + b->r2_off[r], b->r2_off[r + 1] - b->r2_off[r]});
        }
        if (merged) g->push_back(v);
        else for (auto& x : v) g->push_back({x});
      } else {
        for (int r = 0; r < b->R; ++r) {  // plain world, one launch per rank
          const int64_t h0 = b->halo_off[r], h = b->halo_off[r + 1] - h0;
          g->push_back({GatherJob{ra + h0 * rb, b->halo_all + h0 * rb, nullptr, h}});
        }
      }
      break;
    case PH_BWD: {
      if (!b->g_out) break;
      // plain and staged locality worlds: each rank sums the gradients of its
      // own send slots (the reverse transfer delivered them into
      // g_send_all); otherwise the closed-form adjoint over halo_all rows
      const bool local = b->unpack_identity || b->staged_bwd;
      const char* in = local ? b->g_send_all.as<char>() : b->g_in;
      const int32_t* ptr = local ? b->wp_ptr.as<int32_t>() : b->wb_ptr.as<int32_t>();
      const int32_t* idx = local ? b->wp_idx.as<int32_t>() : b->wb_idx.as<int32_t>();
      if (merged && !(local && sc.lds_window)) {
        s->push_back({SegSumJob{in, b->g_out, ptr, idx, b->n}});
      } else {
        // one job per rank; its terms are its own send slots (the window)
        std::vector<SegSumJob> v;
        for (int r = 0; r < b->R; ++r) {
          const int64_t r0 = b->row_starts[r];
          SegSumJob jb{in, b->g_out + r0 * rb, ptr + r0, idx, b->row_starts[r + 1] - r0};
          if (local) {
            jb.win_lo = b->s1_off[r];
            jb.win_rows = b->s1_off[r + 1] - b->s1_off[r];
          }
          v.push_back(jb);
        }
        if (merged) s->push_back(v);
        else for (auto& x : v) s->push_back({x});
      }
      break;
    }
    default:
      return fail(HX_ERR_ARG, "bad phase");
  }
  return HX_SUCCESS;
}

}  // namespace hx

using namespace hx;

// ===========================================================================
// Per-rank request from a plan
// ===========================================================================
static int copy_slice(const hx_plan* p, int f, int rank, DevMem* dst) {
  const int64_t c = p->size(f, rank);
  HX_TRY(dst->alloc((size_t)c * 4));
  if (c) HX_HIP(hipMemcpy(dst->p, p->d[f].as<int32_t>() + p->off[f][rank], (size_t)c * 4, hipMemcpyDeviceToDevice));
  return HX_SUCCESS;
}

static int host_slice(const hx_plan* p, int f, int rank, std::vector<int32_t>* out) {
  out->resize((size_t)p->size(f, rank));
  if (!out->empty())
    HX_HIP(hipMemcpy(out->data(), p->d[f].as<int32_t>() + p->off[f][rank], out->size() * 4, hipMemcpyDeviceToHost));
  return HX_SUCCESS;
}

static int64_t distinct_count(const std::vector<int32_t>& v, int64_t domain) {
  if (v.empty() || domain <= 0) return 0;
  std::vector<uint8_t> seen((size_t)domain, 0);
  int64_t u = 0;
  for (int32_t x : v)
    if (x >= 0 && x < domain && !seen[(size_t)x]) { seen[(size_t)x] = 1; ++u; }
  return u;
}

int hx::req_fill_from_plan(const hx_plan* p, int rank, const void* x_local, void* halo, int dtype, int ncols,
                           hx_req* r) {
  if (!p) return fail(HX_ERR_ARG, "null plan");
  if (rank < 0 || rank >= p->R) return fail(HX_ERR_RANGE, "rank out of range");
  if (dtype != HX_F32 && dtype != HX_F64) return fail(HX_ERR_ARG, "bad dtype");
  if (ncols <= 0) return fail(HX_ERR_ARG, "ncols must be positive");
  r->dtype = dtype;
  r->ncols = ncols;
  r->row_bytes = (size_t)ncols * dtype_bytes(dtype);
  r->variant = p->variant;
  r->rank = rank;
  if (p->variant == HX_LOCALITY_3STEP) {
    if (p->node_map != HX_NODES_BLOCK) return fail(HX_ERR_UNSUPPORTED, "3-step plans need block placement");
    // an aggregator packs its node-mates' rows: the request reads the rows of
    // its whole node (block placement: ranks nd*ppn .. own them contiguously)
    const int first = rank / p->ppn * p->ppn;
    const int last = (int)std::min<int64_t>(p->R, (int64_t)first + p->ppn);
    r->n_local = p->row_starts[last] - p->row_starts[first];
  } else {
    r->n_local = p->row_starts[rank + 1] - p->row_starts[rank];
  }
  r->H = p->size(HX_F_HALO, rank);
  r->E1 = p->size(HX_F_S1_IDX, rank);
  r->E2 = p->size(HX_F_S2_SRC, rank);
  r->R1 = p->r1_off[rank + 1] - p->r1_off[rank];
  r->R2 = p->r2_off[rank + 1] - p->r2_off[rank];
  if ((r->E1 > 0 && !x_local) || (r->H > 0 && !halo)) return fail(HX_ERR_ARG, "null vector or halo");
  r->x = static_cast<const char*>(x_local);
  r->halo = static_cast<char*>(halo);
  r->unpack_identity = p->variant == HX_PLAIN;
  HX_TRY(copy_slice(p, HX_F_S1_IDX, rank, &r->s1_idx));
  HX_TRY(copy_slice(p, HX_F_S2_SRC, rank, &r->s2_src));
  if (!r->unpack_identity) HX_TRY(copy_slice(p, HX_F_UNPACK_SRC, rank, &r->unpack_src));
  HX_TRY(copy_slice(p, HX_F_BT_PTR, rank, &r->bt_ptr));
  HX_TRY(copy_slice(p, HX_F_BT_PERM, rank, &r->bt_perm));
  HX_TRY(host_slice(p, HX_F_S1_COUNTS, rank, &r->s1_counts));
  HX_TRY(host_slice(p, HX_F_S2_COUNTS, rank, &r->s2_counts));
  HX_TRY(host_slice(p, HX_F_R1_COUNTS, rank, &r->r1_counts));
  std::vector<int32_t> s1, s2;
  HX_TRY(host_slice(p, HX_F_S1_IDX, rank, &s1));
  HX_TRY(host_slice(p, HX_F_S2_SRC, rank, &s2));
  for (int32_t v : s1)
    if (v < 0 || v >= r->n_local) return fail(HX_ERR_RANGE, "plan: pack index outside the rank's rows");
  for (int32_t v : s2)
    if (v < 0 || v >= r->R1) return fail(HX_ERR_RANGE, "plan: redistribution index outside stage-1 arena");
  if (!r->unpack_identity) {
    std::vector<int32_t> u;
    HX_TRY(host_slice(p, HX_F_UNPACK_SRC, rank, &u));
    for (int32_t v : u)
      if (v < 0 || v >= r->R1 + r->R2) return fail(HX_ERR_RANGE, "plan: unpack index outside the arena");
  } else if (r->R1 != r->H || r->R2 != 0) {
    return fail(HX_ERR_ARG, "plain plan with a receive arena that is not the halo");
  }
  {
    std::vector<int32_t> bp, bq;
    HX_TRY(host_slice(p, HX_F_BT_PTR, rank, &bp));
    HX_TRY(host_slice(p, HX_F_BT_PERM, rank, &bq));
    if ((int64_t)bp.size() != r->n_local + 1 || bp.front() != 0 || bp.back() != r->E1)
      return fail(HX_ERR_RANGE, "plan: transpose pointer array inconsistent");
    for (size_t i = 1; i < bp.size(); ++i)
      if (bp[i] < bp[i - 1]) return fail(HX_ERR_RANGE, "plan: transpose pointer array decreasing");
    for (int32_t v : bq)
      if (v < 0 || v >= r->E1) return fail(HX_ERR_RANGE, "plan: transpose entry outside the send arena");
  }
  r->U_pack = distinct_count(s1, r->n_local);
  r->U_redist = distinct_count(s2, r->R1);
  HX_TRY(r->send.alloc((size_t)(r->E1 + r->E2) * r->row_bytes));
  HX_TRY(r->recv.alloc((size_t)(r->R1 + r->R2) * r->row_bytes));
  req_compute_bytes(r);
  return HX_SUCCESS;
}

extern "C" int hx_req_from_plan(const hx_plan* p, int rank, const void* x_local, void* halo, hx_dtype dtype,
                                int ncols, hx_req** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  std::unique_ptr<hx_req> r(new (std::nothrow) hx_req);
  if (!r) return fail(HX_ERR_NOMEM, "out of host memory");
  HX_TRY(req_fill_from_plan(p, rank, x_local, halo, dtype, ncols, r.get()));
  *out = r.release();
  return HX_SUCCESS;
}

// ===========================================================================
// World batch
// ===========================================================================
extern "C" int hx_batch_from_plan(const hx_plan* p, const void* x_global, void* halo_all, hx_dtype dtype, int ncols,
                                  int flags, const hx_sched* sched, hx_batch** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (!p) return fail(HX_ERR_ARG, "null plan");
  if (dtype != HX_F32 && dtype != HX_F64) return fail(HX_ERR_ARG, "bad dtype");
  if (ncols <= 0) return fail(HX_ERR_ARG, "ncols must be positive");
  const int R = p->R;
  std::unique_ptr<hx_batch> b(new (std::nothrow) hx_batch);
  if (!b) return fail(HX_ERR_NOMEM, "out of host memory");
  b->world = true;
  b->variant = p->variant;
  b->dtype = dtype;
  b->ncols = ncols;
  b->row_bytes = (size_t)ncols * dtype_bytes(dtype);
  b->flags = flags;
  b->R = R;
  b->n = p->n;
  b->row_starts = p->row_starts;
  b->s1_off = p->off[HX_F_S1_IDX];
  b->s2_off = p->off[HX_F_S2_SRC];
  b->r1_off = p->r1_off;
  b->r2_off = p->r2_off;
  b->halo_off = p->off[HX_F_HALO];
  b->E1_tot = b->s1_off.back();
  b->E2_tot = b->s2_off.back();
  b->R1_tot = b->r1_off.back();
  b->R2_tot = b->r2_off.back();
  b->H_tot = b->halo_off.back();
  b->unpack_identity = p->variant == HX_PLAIN;
  if ((b->E1_tot > 0 && !x_global) || (b->H_tot > 0 && !halo_all)) return fail(HX_ERR_ARG, "null vector or halo");
  if (b->E1_tot + b->E2_tot >= INT32_MAX || b->R1_tot + b->R2_tot >= INT32_MAX)
    return fail(HX_ERR_UNSUPPORTED, "world arenas beyond 2^31 rows");
  b->x_global = static_cast<const char*>(x_global);
  b->halo_all = static_cast<char*>(halo_all);
  const size_t rb = b->row_bytes;
  hipStream_t s = nullptr;
  HX_TRY(b->send_all.alloc((size_t)(b->E1_tot + b->E2_tot) * rb));
  HX_TRY(b->recv_all.alloc((size_t)(b->R1_tot + b->R2_tot) * rb));

  DevMem rs_d, s1o, s2o, r1o, r2o, ho, err;
  HX_TRY(upload_vec(rs_d, b->row_starts));
  HX_TRY(upload_vec(s1o, b->s1_off));
  HX_TRY(upload_vec(s2o, b->s2_off));
  HX_TRY(upload_vec(r1o, b->r1_off));
  HX_TRY(upload_vec(r2o, b->r2_off));
  HX_TRY(upload_vec(ho, b->halo_off));
  HX_TRY(err.alloc(4));
  HX_HIP(hipMemset(err.p, 0, 4));

  // pack: x_global rows (pack indices count from the rank's first row, or
  // from its node's first row for the 3-step plan)
  const bool v3 = p->variant == HX_LOCALITY_3STEP;
  std::vector<int64_t> pbase((size_t)R + 1, 0);
  for (int r = 0; r <= R; ++r) pbase[r] = v3 && r < R ? b->row_starts[(r / p->ppn) * p->ppn] : b->row_starts[r];
  DevMem pbase_d;
  HX_TRY(upload_vec(pbase_d, pbase));
  HX_TRY(b->gidx_pack.alloc((size_t)b->E1_tot * 4));
  if (b->E1_tot)
    hipLaunchKernelGGL(k_add_rank_base, dim3(blocks_for(b->E1_tot)), dim3(TB), 0, s, p->d[HX_F_S1_IDX].as<int32_t>(),
                       b->E1_tot, s1o.as<int64_t>(), R, pbase_d.as<int64_t>(), b->gidx_pack.as<int32_t>());
  HX_HIP(hipGetLastError());
  // push form of the pack: global row -> send_all rows (ascending)
  if (v3) {
    // senders other than the owner: group the global pack map directly
    HX_TRY(dev_check_range(b->gidx_pack.as<int32_t>(), b->E1_tot, b->n, "pack map", s));
    HX_TRY(b->wp_ptr.alloc((size_t)(b->n + 1) * 4));
    HX_TRY(b->wp_idx.alloc((size_t)std::max<int64_t>(b->E1_tot, 1) * 4));
    HX_TRY(dev_group_by_key(b->gidx_pack.as<int32_t>(), b->E1_tot, b->n, b->wp_ptr.as<int32_t>(),
                            b->wp_idx.as<int32_t>(), s));
  } else {
    DevMem bto;
    HX_TRY(upload_vec(bto, p->off[HX_F_BT_PTR]));
    HX_TRY(b->wp_ptr.alloc((size_t)(b->n + 1) * 4));
    HX_TRY(b->wp_idx.alloc((size_t)b->E1_tot * 4));
    hipLaunchKernelGGL(k_world_pack_ptr, dim3(blocks_for(b->n + 1)), dim3(TB), 0, s, p->d[HX_F_BT_PTR].as<int32_t>(),
                       bto.as<int64_t>(), rs_d.as<int64_t>(), s1o.as<int64_t>(), R, b->n, b->E1_tot,
                       b->wp_ptr.as<int32_t>());
    if (b->E1_tot)
      hipLaunchKernelGGL(k_add_rank_base, dim3(blocks_for(b->E1_tot)), dim3(TB), 0, s,
                         p->d[HX_F_BT_PERM].as<int32_t>(), b->E1_tot, s1o.as<int64_t>(), R, s1o.as<int64_t>(),
                         b->wp_idx.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_HIP(hipDeviceSynchronize());
  }
  // redistribution: rows of recv_all (stage-1 part of the forwarder)
  HX_TRY(b->gidx_redist.alloc((size_t)b->E2_tot * 4));
  if (b->E2_tot)
    hipLaunchKernelGGL(k_add_rank_base, dim3(blocks_for(b->E2_tot)), dim3(TB), 0, s, p->d[HX_F_S2_SRC].as<int32_t>(),
                       b->E2_tot, s2o.as<int64_t>(), R, r1o.as<int64_t>(), b->gidx_redist.as<int32_t>());
  // unpack
  if (!b->unpack_identity) {
    HX_TRY(b->gidx_unpack.alloc((size_t)b->H_tot * 4));
    if (b->H_tot)
      hipLaunchKernelGGL(k_world_unpack, dim3(blocks_for(b->H_tot)), dim3(TB), 0, s,
                         p->d[HX_F_UNPACK_SRC].as<int32_t>(), b->H_tot, ho.as<int64_t>(), R, r1o.as<int64_t>(),
                         r2o.as<int64_t>(), b->R1_tot, b->gidx_unpack.as<int32_t>());
  }
  HX_HIP(hipGetLastError());
  // simulated transfers
  {
    DevMem rp1, sp1, rp2, sp2;
    HX_TRY(upload_vec(rp1, p->off[HX_F_R1_PROCS]));
    HX_TRY(upload_vec(sp1, p->off[HX_F_S1_PROCS]));
    HX_TRY(upload_vec(rp2, p->off[HX_F_R2_PROCS]));
    HX_TRY(upload_vec(sp2, p->off[HX_F_S2_PROCS]));
    HX_TRY(b->gidx_x1.alloc((size_t)b->R1_tot * 4));
    HX_TRY(b->gidx_x2.alloc((size_t)b->R2_tot * 4));
    if (b->R1_tot)
      hipLaunchKernelGGL(k_transfer_map, dim3(blocks_for(b->R1_tot)), dim3(TB), 0, s, b->R1_tot, R, r1o.as<int64_t>(),
                         rp1.as<int64_t>(), p->d[HX_F_R1_PROCS].as<int32_t>(), p->d[HX_F_R1_COUNTS].as<int32_t>(),
                         p->d[HX_F_R1_DISPLS].as<int32_t>(), s1o.as<int64_t>(), sp1.as<int64_t>(),
                         p->d[HX_F_S1_PROCS].as<int32_t>(), p->d[HX_F_S1_COUNTS].as<int32_t>(),
                         p->d[HX_F_S1_DISPLS].as<int32_t>(), (int64_t)0, b->gidx_x1.as<int32_t>(),
                         err.as<int>());
    if (b->R2_tot)
      hipLaunchKernelGGL(k_transfer_map, dim3(blocks_for(b->R2_tot)), dim3(TB), 0, s, b->R2_tot, R, r2o.as<int64_t>(),
                         rp2.as<int64_t>(), p->d[HX_F_R2_PROCS].as<int32_t>(), p->d[HX_F_R2_COUNTS].as<int32_t>(),
                         p->d[HX_F_R2_DISPLS].as<int32_t>(), s2o.as<int64_t>(), sp2.as<int64_t>(),
                         p->d[HX_F_S2_PROCS].as<int32_t>(), p->d[HX_F_S2_COUNTS].as<int32_t>(),
                         p->d[HX_F_S2_DISPLS].as<int32_t>(), b->E1_tot, b->gidx_x2.as<int32_t>(),
                         err.as<int>());
    HX_HIP(hipGetLastError());
    HX_HIP(hipDeviceSynchronize());
    HX_TRY(check_err(err, "world transfer"));
  }
  // every index a kernel will follow stays inside its source
  HX_TRY(dev_check_range(b->gidx_pack.as<int32_t>(), b->E1_tot, b->n, "pack map", s));
  HX_TRY(dev_check_range(b->wp_idx.as<int32_t>(), b->E1_tot, b->E1_tot, "pack transpose", s));
  HX_TRY(dev_check_range(b->wp_ptr.as<int32_t>(), b->n + 1, b->E1_tot + 1, "pack transpose pointers", s));
  HX_TRY(dev_check_range(b->gidx_redist.as<int32_t>(), b->E2_tot, b->R1_tot, "redistribution map", s));
  if (!b->unpack_identity)
    HX_TRY(dev_check_range(b->gidx_unpack.as<int32_t>(), b->H_tot, b->R1_tot + b->R2_tot, "unpack map", s));
  else if (b->R1_tot != b->H_tot || b->R2_tot != 0)
    return fail(HX_ERR_ARG, "plain plan with a receive arena that is not the halo");
  HX_TRY(dev_check_range(b->gidx_x1.as<int32_t>(), b->R1_tot, b->E1_tot, "stage-1 transfer", s));
  HX_TRY(dev_check_range(b->gidx_x2.as<int32_t>(), b->R2_tot, b->E1_tot + b->E2_tot, "stage-2 transfer", s));
  // adjoint CSR: global column -> rows of halo_all, ascending (= ascending rank)
  HX_TRY(b->wb_ptr.alloc((size_t)(b->n + 1) * 4));
  HX_TRY(b->wb_idx.alloc((size_t)b->H_tot * 4));
  HX_TRY(dev_group_by_key(p->d[HX_F_HALO].as<int32_t>(), b->H_tot, b->n, b->wb_ptr.as<int32_t>(),
                          b->wb_idx.as<int32_t>(), s));
  // transfer launch tables
  {
    const Sched sc = default_sched(KIND_GATHER, (int)rb);
    std::vector<GatherJob> x1{GatherJob{b->send_all.as<char>(), b->recv_all.as<char>(), b->gidx_x1.as<int32_t>(),
                                        b->R1_tot}};
    std::vector<GatherJob> x2{GatherJob{b->send_all.as<char>(), b->recv_all.as<char>() + b->R1_tot * (int64_t)rb,
                                        b->gidx_x2.as<int32_t>(), b->R2_tot}};
    HX_TRY(build_gather_table(x1, dtype, (int)rb, sc, &b->lt_xfer[0]));
    HX_TRY(build_gather_table(x2, dtype, (int)rb, sc, &b->lt_xfer[1]));
  }
  // plain worlds: the reverse of the stage-1 transfer (send slot -> the halo
  // row that received it), used to deliver halo gradients back to the senders
  if (b->unpack_identity && b->E1_tot > 0) {
    if (b->E1_tot != b->R1_tot) return fail(HX_ERR_ARG, "plain plan: sends and receives differ in size");
    HX_TRY(b->gidx_back.alloc((size_t)b->E1_tot * 4));
    hipLaunchKernelGGL(k_fill_neg, dim3(blocks_for(b->E1_tot)), dim3(TB), 0, s, b->gidx_back.as<int32_t>(), b->E1_tot);
    hipLaunchKernelGGL(k_invert, dim3(blocks_for(b->R1_tot)), dim3(TB), 0, s, b->gidx_x1.as<int32_t>(), b->R1_tot,
                       b->gidx_back.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(dev_check_range(b->gidx_back.as<int32_t>(), b->E1_tot, b->H_tot, "reverse transfer", s));
  }
  // staged backward of a locality plan (the forward's stages reversed):
  //   reverse unpack   a relabelling: the gradient of receive slot k is the
  //                    halo gradient row that read it (inv_unpack[k])
  //   reverse stage 2  g_s2[e] = g_halo[inv_unpack[R1 + inv2[e]]]   (transport)
  //   forwarder sums   g_r1[k] = g_halo[own row of k] (when read), then
  //                    g_s2[e] for the entries e forwarding k, ascending
  //   reverse stage 1  g_send[e] = g_r1[inv1[e]]                     (transport)
  //   owner sums       g_x = pack transpose over g_send (as the plain world)
  if ((flags & HX_WORLD_STAGED_BACKWARD) && !b->unpack_identity) {
    b->staged_bwd = true;
    const int64_t S = b->R1_tot + b->R2_tot;
    if (b->E1_tot != b->R1_tot || b->E2_tot != b->R2_tot)
      return fail(HX_ERR_ARG, "plan: sends and receives of a stage differ in size");
    if (b->H_tot + b->E2_tot >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "halo + stage-2 rows beyond 2^31");
    DevMem inv_unpack, inv2, gp, gperm, lens;
    HX_TRY(inv_unpack.alloc((size_t)std::max<int64_t>(S, 1) * 4));
    HX_TRY(inv2.alloc((size_t)std::max<int64_t>(b->E2_tot, 1) * 4));
    HX_TRY(b->gidx_back.alloc((size_t)b->E1_tot * 4));
    HX_TRY(b->gidx_back2.alloc((size_t)b->E2_tot * 4));
    hipLaunchKernelGGL(k_fill_neg, dim3(blocks_for(S + 1)), dim3(TB), 0, s, inv_unpack.as<int32_t>(), S);
    if (b->H_tot)
      hipLaunchKernelGGL(k_invert_range, dim3(blocks_for(b->H_tot)), dim3(TB), 0, s, b->gidx_unpack.as<int32_t>(),
                         b->H_tot, (int64_t)0, S, inv_unpack.as<int32_t>());
    if (b->E1_tot) {
      hipLaunchKernelGGL(k_fill_neg, dim3(blocks_for(b->E1_tot)), dim3(TB), 0, s, b->gidx_back.as<int32_t>(), b->E1_tot);
      hipLaunchKernelGGL(k_invert_range, dim3(blocks_for(b->R1_tot)), dim3(TB), 0, s, b->gidx_x1.as<int32_t>(),
                         b->R1_tot, (int64_t)0, b->E1_tot, b->gidx_back.as<int32_t>());
    }
    if (b->E2_tot) {
      hipLaunchKernelGGL(k_fill_neg, dim3(blocks_for(b->E2_tot)), dim3(TB), 0, s, inv2.as<int32_t>(), b->E2_tot);
      hipLaunchKernelGGL(k_invert_range, dim3(blocks_for(b->R2_tot)), dim3(TB), 0, s, b->gidx_x2.as<int32_t>(),
                         b->R2_tot, b->E1_tot, b->E2_tot, inv2.as<int32_t>());
    }
    HX_HIP(hipGetLastError());
    HX_TRY(dev_check_range(inv2.as<int32_t>(), b->E2_tot, b->R2_tot, "reverse stage-2 transfer", s));
    if (b->E2_tot)
      hipLaunchKernelGGL(k_compose, dim3(blocks_for(b->E2_tot)), dim3(TB), 0, s, inv2.as<int32_t>(), b->E2_tot,
                         inv_unpack.as<int32_t>(), b->R1_tot, b->gidx_back2.as<int32_t>());
    HX_HIP(hipGetLastError());
    // forwarder-sum CSR; own rows are inv_unpack over the stage-1 slots
    HX_TRY(gp.alloc((size_t)(b->R1_tot + 1) * 4));
    HX_TRY(gperm.alloc((size_t)std::max<int64_t>(b->E2_tot, 1) * 4));
    HX_TRY(lens.alloc((size_t)(b->R1_tot + 1) * 4));
    HX_TRY(b->fwd_ptr.alloc((size_t)(b->R1_tot + 1) * 4));
    HX_TRY(dev_group_by_key(b->gidx_redist.as<int32_t>(), b->E2_tot, b->R1_tot, gp.as<int32_t>(), gperm.as<int32_t>(),
                            s));
    if (b->R1_tot)
      hipLaunchKernelGGL(k_forward_lens, dim3(blocks_for(b->R1_tot)), dim3(TB), 0, s, inv_unpack.as<int32_t>(),
                         gp.as<int32_t>(), b->R1_tot, lens.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(dev_exclusive_scan_i32(lens.as<int32_t>(), b->fwd_ptr.as<int32_t>(), b->R1_tot, s));
    int32_t nterms = 0;
    HX_HIP(hipMemcpy(&nterms, b->fwd_ptr.as<int32_t>() + b->R1_tot, 4, hipMemcpyDeviceToHost));
    b->fwd_terms = nterms;
    HX_TRY(b->fwd_idx.alloc((size_t)std::max<int32_t>(nterms, 1) * 4));
    if (b->R1_tot)
      hipLaunchKernelGGL(k_forward_terms, dim3(blocks_for(b->R1_tot)), dim3(TB), 0, s, inv_unpack.as<int32_t>(),
                         gp.as<int32_t>(), gperm.as<int32_t>(), b->fwd_ptr.as<int32_t>(), b->R1_tot, b->H_tot,
                         b->fwd_idx.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_HIP(hipDeviceSynchronize());
    HX_TRY(dev_check_range(b->gidx_back.as<int32_t>(), b->E1_tot, b->R1_tot, "reverse stage-1 transfer", s));
    HX_TRY(dev_check_range(b->gidx_back2.as<int32_t>(), b->E2_tot, b->H_tot, "reverse stage-2 transfer", s));
    HX_TRY(dev_check_range(b->fwd_idx.as<int32_t>(), nterms, b->H_tot + b->E2_tot, "forwarder sums", s));
  }
  // algorithmic bytes per phase
  {
    int64_t U1 = 0, U2 = 0;
    HX_TRY(dev_count_nonzero_flags(b->gidx_pack.as<int32_t>(), b->E1_tot, b->n, &U1, s));
    HX_TRY(dev_count_nonzero_flags(b->gidx_redist.as<int32_t>(), b->E2_tot, b->R1_tot + b->R2_tot, &U2, s));
    const int64_t rbi = (int64_t)rb;
    b->bytes[PH_PACK] = (b->E1_tot + U1) * rbi + 4 * b->E1_tot;
    b->bytes[PH_REDIST] = (b->E2_tot + U2) * rbi + 4 * b->E2_tot;
    b->bytes[PH_UNPACK] = 2 * b->H_tot * rbi + (b->unpack_identity ? 0 : 4 * b->H_tot);
    b->bytes[PH_BWD] = (b->H_tot + b->n) * rbi + 4 * (b->H_tot + b->n + 1);
    if (b->staged_bwd)  // forwarder sums + owner sums
      b->bytes[PH_BWD] = ((b->fwd_terms + b->R1_tot) * rbi + 4 * (b->fwd_terms + b->R1_tot + 1)) +
                         ((b->E1_tot + b->n) * rbi + 4 * (b->E1_tot + b->n + 1));
  }
  HX_TRY(batch_init_scheds(b.get(), sched));
  HX_TRY(batch_prepare(b.get()));
  *out = b.release();
  return HX_SUCCESS;
}

extern "C" int hx_batch_arena(hx_batch* b, int which, void** dev_ptr, int64_t* rows) {
  if (!b || !dev_ptr || !rows) return fail(HX_ERR_ARG, "null argument");
  if (!b->world) return fail(HX_ERR_ARG, "not a world batch");
  if (which == HX_ARENA_SEND) {
    *dev_ptr = b->send_all.p;
    *rows = b->E1_tot + b->E2_tot;
  } else if (which == HX_ARENA_RECV) {
    *dev_ptr = b->recv_all.p;
    *rows = b->R1_tot + b->R2_tot;
  } else if (which == HX_ARENA_GRAD_SEND) {
    if (!b->unpack_identity && !b->staged_bwd)
      return fail(HX_ERR_ARG, "locality worlds without the staged backward have no gradient send arena");
    if (!b->g_out) return fail(HX_ERR_STATE, "no gradient buffers bound");
    *dev_ptr = b->g_send_all.p;
    *rows = b->E1_tot;
  } else {
    return fail(HX_ERR_ARG, "bad arena id");
  }
  return HX_SUCCESS;
}

// Row offset of a rank's stage-1 part; its stage-2 part starts at
// (total stage-1 rows + the offset returned for which | 2).
extern "C" int hx_batch_arena_offset(hx_batch* b, int which, int rank, int64_t* row_offset) {
  if (!b || !row_offset) return fail(HX_ERR_ARG, "null argument");
  if (!b->world) return fail(HX_ERR_ARG, "not a world batch");
  if (rank < 0 || rank > b->R) return fail(HX_ERR_RANGE, "rank out of range");
  switch (which) {
    case HX_ARENA_SEND: *row_offset = b->s1_off[rank]; break;
    case HX_ARENA_RECV: *row_offset = b->r1_off[rank]; break;
    case HX_ARENA_SEND | 2: *row_offset = b->E1_tot + b->s2_off[rank]; break;
    case HX_ARENA_RECV | 2: *row_offset = b->R1_tot + b->r2_off[rank]; break;
    default: return fail(HX_ERR_ARG, "bad arena id");
  }
  return HX_SUCCESS;
}
