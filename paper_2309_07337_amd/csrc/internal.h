// Definitions of the opaque handles and internal entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.h"

namespace hx {
enum Phase { PH_PACK = 0, PH_REDIST = 1, PH_UNPACK = 2, PH_BWD = 3 };
}
struct hx_comm;

// A rank's neighbor topology (host copies of its lists).
struct hx_topo {
  int rank = 0, nranks = 0;
  std::vector<int> recv_procs, send_procs;
};

// One rank's persistent request (rank-local arrays on the device).
struct hx_req {
  int dtype = HX_F64;
  int ncols = 1;
  size_t row_bytes = 8;
  int variant = HX_PLAIN;
  int rank = 0;
  int64_t n_local = 0, H = 0, E1 = 0, E2 = 0, R1 = 0, R2 = 0;
  const char* x = nullptr;
  char* halo = nullptr;
  bool unpack_identity = true;
  std::vector<int32_t> s1_counts, s2_counts, r1_counts;  // message sizes (per-neighbor schedules)
  hx::DevMem s1_idx, s2_src, unpack_src, bt_ptr, bt_perm;
  hx::DevMem send, recv;  // [E1 | E2] and [R1 | R2] rows
  int64_t U_pack = 0, U_redist = 0;  // distinct source rows of the pack / redistribution
  int64_t bytes[4] = {0, 0, 0, 0};
  const char* g_send = nullptr;
  char* g_x = nullptr;
  uint64_t grad_gen = 0;  // changes at every hx_req_bind_grad (unique across requests)
  bool active = false;
  bool tables_built = false;
  hx::LaunchTable lt[4];
  hx::DevMem ready;  // per stage-1 message completion counters (uint64), when enabled
  // joined a collective locality-aware init that has not completed yet: the
  // request has no arrays and every call but free refuses it
  bool pending = false;
  hx_comm* comm = nullptr;  // the communicator it joined (while pending)
  int batch_refs = 0;       // batches holding it as a member (it may not be freed before them)
};

// A simulated communicator for the collective locality-aware init: every
// rank's lists are collected, and the call that completes the set builds
// the plan and fills every joined request.
struct hx_comm {
  int R = 0;
  std::vector<int64_t> row_starts;  // host [R+1]
  hx_info info{};
  hipStream_t stream = nullptr;
  struct Slot {
    bool joined = false;
    hx_req* req = nullptr;  // while pending; nullptr once freed by its owner or completed
    std::vector<int> rprocs, rcounts, sprocs, scounts;
    std::vector<int64_t> rind, sind;  // global indices in the caller's order
  };
  std::vector<Slot> slot;
  int joined = 0;
  int state = 0;  // 0 collecting, 1 complete, < 0 failed with that code
};

// Plan of a whole decomposition: per-rank arrays stored flat on the device,
// with host copies of the per-rank offsets of every field.
struct hx_plan {
  int R = 0;
  int ppn = 1;
  int node_map = HX_NODES_BLOCK;
  int variant = HX_PLAIN;
  int64_t n = 0;
  std::vector<int64_t> row_starts;               // host [R+1]
  std::vector<int64_t> off[HX_F_COUNT];          // host [R+1] per field
  hx::DevMem d[HX_F_COUNT];                      // device int32 flat arrays
  hx::DevMem row_starts_d;                       // device int64 [R+1]
  std::vector<int64_t> r1_off, r2_off;           // host [R+1]: receive-arena row offsets
  // totals
  int64_t tot(int f) const { return off[f].empty() ? 0 : off[f].back(); }
  int64_t size(int f, int r) const { return off[f][r + 1] - off[f][r]; }
};

struct hx_batch {
  bool world = false;
  int variant = HX_PLAIN;  // worlds: the plan's variant (part of the tuning-cache key)
  int dtype = HX_F64;
  int ncols = 1;
  size_t row_bytes = 8;
  int flags = 0;
  std::vector<hx_req*> members;
  hx::Sched sched[4];
  bool sched_from_cache[4] = {true, true, true, true};  // no schedule given: the phase takes the tuning cache's
  hx::LaunchTable lt[4];
  std::vector<hx::LaunchTable> plain[4];
  bool plain_built[4] = {false, false, false, false};
  hx::LaunchTable lt_xfer[4];               // simulated transfers: stage 1, stage 2, reverse of stage 1, of stage 2
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  bool has_graph[3] = {false, false, false};
  bool replay_direct = false;  // start / wait / backward launch the tables directly instead of the graphs
  bool active = false;
  bool tuning = false;                      // hx_batch_tune running: candidates skip completion counters
  int64_t bytes[4] = {0, 0, 0, 0};
  std::vector<uint64_t> bwd_gens_captured;  // members' grad_gen when the backward tables were built
  // world (all ranks of a plan over flat arrays)
  int R = 0;
  int64_t n = 0;
  const char* x_global = nullptr;
  char* halo_all = nullptr;
  const char* g_in = nullptr;
  char* g_out = nullptr;
  std::vector<int64_t> row_starts, s1_off, s2_off, r1_off, r2_off, halo_off;
  int64_t E1_tot = 0, E2_tot = 0, R1_tot = 0, R2_tot = 0, H_tot = 0;
  bool unpack_identity = true;
  hx::DevMem send_all, recv_all;             // [S1 | S2], [RECV1 | RECV2] of all ranks
  hx::DevMem gidx_pack, gidx_redist, gidx_unpack, gidx_x1, gidx_x2, gidx_back;
  hx::DevMem g_send_all;                     // plain worlds: gradients of every rank's send slots
  hx::DevMem wb_ptr, wb_idx;                 // adjoint CSR: global column -> halo_all rows
  hx::DevMem wp_ptr, wp_idx;                 // transpose of the pack map: global row -> send_all rows
  // staged backward of a locality world (forwarder sums, owner sums)
  bool staged_bwd = false;
  hx::DevMem gidx_back2;                     // stage-2 send slot -> halo row whose gradient it carries back
  hx::DevMem fwd_ptr, fwd_idx;               // forwarder-sum CSR over stage-1 receive slots
  int64_t fwd_terms = 0;
  hx::DevMem g_s2;                           // gradients of every stage-2 send slot
  hx::DevMem g_r1;                           // forwarder sums (stage-1 receive slot gradients)
  hx::LaunchTable lt_fwd_sum;                // forwarder sums
  ~hx_batch();
};

namespace hx {
int req_jobs(const hx_req* r, int phase, const Sched& sc, std::vector<GatherJob>* g,
             std::vector<SegSumJob>* s);
int build_phase_table(int phase, const Sched& sc, int dtype, int row_bytes, const std::vector<GatherJob>& g,
                      const std::vector<SegSumJob>& s, LaunchTable* t);
void req_compute_bytes(hx_req* r);
// Fills r (fresh, or pending) with rank `rank`'s arrays of plan p.
int req_fill_from_plan(const hx_plan* p, int rank, const void* x_local, void* halo, int dtype, int ncols,
                       hx_req* r);
// HX_ERR_STATE for a request whose collective init has not completed.
int req_usable(const hx_req* r);
void batch_destroy_graphs(hx_batch* b);
int batch_phase_jobs(const hx_batch* b, int phase, const Sched& sc, bool merged,
                     std::vector<std::vector<GatherJob>>* g, std::vector<std::vector<SegSumJob>>* s);
int batch_build_table(const hx_batch* b, int phase, const Sched& sc, LaunchTable* t);
int batch_build_plain(hx_batch* b, int phase);
int batch_prepare(hx_batch* b);
int batch_run_start(hx_batch* b, hipStream_t s);
int batch_run_wait(hx_batch* b, hipStream_t s);
int batch_run_backward(hx_batch* b, hipStream_t s);
int batch_init_scheds(hx_batch* b, const hx_sched* sched);
int world_phase_jobs(const hx_batch* b, int phase, const Sched& sc, bool merged,
                     std::vector<std::vector<GatherJob>>* g, std::vector<std::vector<SegSumJob>>* s);

// Device helpers implemented in plan.hip.
int dev_exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);  // out[n] = total
// HX_ERR_RANGE unless every idx[i] is in [0, hi).
int dev_check_range(const int32_t* idx, int64_t n, int64_t hi, const char* what, hipStream_t s);
int dev_count_nonzero_flags(const int32_t* idx, int64_t n, int64_t domain, int64_t* distinct,
                            hipStream_t s);
// Stable grouping of entries by key: for each key k in [0, nkeys), the
// entries e with keys[e] == k in ascending e.  ptr [nkeys+1], perm [n].
int dev_group_by_key(const int32_t* keys, int64_t n, int64_t nkeys, int32_t* ptr, int32_t* perm,
                     hipStream_t s);
}  // namespace hx
