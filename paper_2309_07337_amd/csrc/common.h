// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "hx.h"

namespace hx {

// ---------------------------------------------------------------------------
// Errors: thread-local last message / last HIP error.
// ---------------------------------------------------------------------------
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define HX_HIP(call)                                                  \
  do {                                                                \
    hipError_t hx_e_ = (call);                                        \
    if (hx_e_ != hipSuccess) return ::hx::hip_fail(hx_e_, #call, __FILE__, __LINE__); \
  } while (0)

#define HX_TRY(call)                 \
  do {                               \
    int hx_rc_ = (call);             \
    if (hx_rc_ != HX_SUCCESS) return hx_rc_; \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory owned by library objects.  Every allocation goes through the
// allocator installed with hx_set_allocator (hipMalloc / hipFree when none
// is); a block remembers the free function of the allocator that made it,
// so installing another allocator later never mismatches a free.
// ---------------------------------------------------------------------------
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  hx_free_fn free_fn = nullptr;  // nullptr: hipFree
  void* free_ctx = nullptr;
  bool owned = true;             // false: a view of memory owned elsewhere (never freed here)
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept { take(o); }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) { release(); take(o); }
    return *this;
  }
  ~DevMem() { release(); }
  void release();
  // frees previous contents; zero bytes -> nullptr.  stream: the stream the
  // memory will first be used on (passed to an installed allocator).
  int alloc(size_t nbytes, hipStream_t stream = nullptr);
  // views nbytes at q (memory this object does not own and never frees)
  void borrow(void* q, size_t nbytes) {
    release();
    p = q;
    bytes = nbytes;
    owned = false;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }

 private:
  void take(DevMem& o) {
    p = o.p; bytes = o.bytes; free_fn = o.free_fn; free_ctx = o.free_ctx; owned = o.owned;
    o.p = nullptr; o.bytes = 0; o.free_fn = nullptr; o.free_ctx = nullptr; o.owned = true;
  }
};

int upload(DevMem& dst, const void* host, size_t bytes);
template <class T>
int upload_vec(DevMem& dst, const std::vector<T>& v) {
  return upload(dst, v.data(), v.size() * sizeof(T));
}

int device_cus();  // number of compute units of the current device
int device_lds_per_block();  // LDS bytes one workgroup may use on the current device

// ---------------------------------------------------------------------------
// Kernels' work descriptions.
// ---------------------------------------------------------------------------
// dst[r, :] = src[idx ? idx[r] : r, :] for r < nrows (rows of row_bytes).
// A job may name a source window: every idx[r] lies in [win_lo, win_lo +
// win_rows) (win_rows = 0: no window), which lets the kernel stage it in LDS.
struct GatherJob {
  const char* src;
  char* dst;
  const int32_t* idx;
  int64_t nrows;
  int64_t win_lo = 0;
  int64_t win_rows = 0;
  // when set: after each tile, the rows it wrote are added to *ready once
  // they are visible device-wide (a message's completion counter)
  unsigned long long* ready = nullptr;
  // set by the table builder: every index of the job lies in its window
  int32_t win_all = 0;
};
// out[i, :] = in[idx[ptr[i]], :] + in[idx[ptr[i]+1], :] + ... (ascending,
// first term first; empty -> +0) for i < nrows.  Terms t >= split come from
// the second input instead: in2[t - split, :] (segmented sums only).
struct SegSumJob {
  const char* in;
  char* out;
  const int32_t* ptr;
  const int32_t* idx;
  int64_t nrows;
  const char* in2 = nullptr;
  int32_t split = INT32_MAX;
  // segmented sums: terms [win_lo, win_lo + win_rows) (all in one input) may
  // be staged in LDS (win_rows = 0: none)
  int64_t win_lo = 0;
  int64_t win_rows = 0;
};

// Gather: pull rows through an index (GatherJob).  Segsum: fixed-order sum
// over the segments of a CSR (SegSumJob).  Scatter: push each row of a CSR's
// rows to its slots (SegSumJob: in = rows, out = slots).
enum JobKind { KIND_GATHER = 0, KIND_SEGSUM = 1, KIND_SCATTER = 2 };
// Which step a table serves (selects the kernel symbol only, so profiles
// separate the steps): gathers PACK / REDIST / UNPACK / TRANSFER, the push
// pack (PACK), segmented sums OWNER_SUM / FWD_SUM (the staged backward's
// forwarder sums).
enum GatherTag { TAG_PACK = 0, TAG_REDIST = 1, TAG_UNPACK = 2, TAG_TRANSFER = 3, TAG_OWNER_SUM = 4,
                 TAG_FWD_SUM = 5 };

struct Sched {
  int tile_rows = 0;
  int block_threads = 0;
  int blocks_per_cu = 0;
  int nontemporal = 0;
  int per_neighbor = 0;
  int unroll = 0;     // rows (or 16-byte row groups) per lane in flight: 1, 2, 4
  int push_pack = 0;  // pack in push form (read each source row once)
  int lds_window = 0; // gathers stage each job's source window in LDS
  int pair_rows = 0;  // gathers of 4- or 8-byte rows: 16 bytes of rows per lane (2 or 4 rows)
};
Sched default_sched(int kind, int row_bytes);

// LDS staging in the CSR-driven kernels (push pack, segmented sum): tiles of
// at most kStageRows rows stage their row pointers, and their entry indices
// when there are at most kStageEntries; the segmented sum gathers the terms
// of consecutive rows into at most kSegValueBytes of LDS before adding them.
constexpr int kStageRows = 512;
constexpr int kStageEntries = 2048;
constexpr int kSegValueBytes = 65536;
// blocks_per_cu of a one-shot grid: the grid never exceeds the tile count
// (rounded up to 8), so this gives one workgroup per tile, dispatched by the
// hardware in tile order.  On gfx950 that keeps the rows in flight in a
// compact moving window of memory and balances uneven tiles, which measures
// 5-15 % faster than a persistent grid walking per-workgroup tile ranges
// for streaming gathers, scatters and copies of 64 B rows and more.
constexpr int kOneShotBpc = 1 << 20;
// Largest source window a gather stages in LDS (larger ones read global
// memory): two such workgroups fit in the 160 KiB of a gfx950 CU.
constexpr int kWinBytes = 80 << 10;
// Same for a segmented sum's term window (its workgroups also hold about
// 6.5 KiB of staged pointers and indices).
constexpr int kSegWinBytes = 72 << 10;
Sched resolve_sched(const hx_sched* s, int kind, int row_bytes);
hx_sched to_public(const Sched& s);

// A prepared launch: jobs and their tile prefix in device memory, plus the
// launch shape.  Launch reads the tables at run time, so a captured graph
// stays valid as long as the table lives.
struct LaunchTable {
  int kind = KIND_GATHER;
  int tag = TAG_TRANSFER;
  int dtype = HX_F64;
  int row_bytes = 0;
  int vec_bytes = 0;  // 16, 8 or 4: divides row_bytes and all base pointers
  int win_bytes = 0;  // dynamic LDS of a gather table whose jobs use windows
  int val_bytes = 0;  // segmented sums: dynamic LDS term buffer (whole rows)
  int vec16 = 0;      // gathers of 4- or 8-byte rows in 16-byte groups per lane (alignment allows it);
                      // segmented sums of rows of one value: one row per lane
  int vec_depth = 4;  // one-value segmented sums: terms per row loaded together (4 or 16)
  int partial_win = 0;  // row-group gathers: some job's window misses some of its indices
  Sched sched;
  int njobs = 0;
  int64_t ntiles = 0;
  int grid = 0;
  DevMem jobs;        // GatherJob[] or SegSumJob[]
  DevMem tile_start;  // int64_t[njobs + 1]
  DevMem tile_terms;  // segmented sums, push pack: int2[ntiles], entry range {ptr[r0], ptr[r1]} of each tile
  bool empty() const { return ntiles == 0; }
};

int build_gather_table(const std::vector<GatherJob>& jobs, int dtype, int row_bytes,
                       const Sched& s, LaunchTable* t, int tag = TAG_TRANSFER);
int build_segsum_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes,
                       const Sched& s, LaunchTable* t, int tag = TAG_OWNER_SUM);
// The same table for one job, written by a kernel on stream into caller-
// provided device memory `area` of area_bytes (job descriptor, tile prefix,
// tile entry ranges; nothing is allocated), then launched on stream.  The
// area must stay untouched until the launch has run.  HX_ERR_UNSUPPORTED when
// the tile entry ranges do not fit (limit: segsum_area_max_tiles).
int launch_segsum_in_area(const SegSumJob& job, int dtype, int row_bytes, const Sched& s, void* area,
                          size_t area_bytes, hipStream_t stream, int tag = TAG_OWNER_SUM);
constexpr size_t kAreaHeadBytes = 512;  // job descriptor and tile prefix ahead of the entry ranges
inline int64_t segsum_area_max_tiles(size_t area_bytes) {
  return area_bytes <= kAreaHeadBytes ? 0 : (int64_t)((area_bytes - kAreaHeadBytes) / sizeof(int2));
}
int build_scatter_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes,
                        const Sched& s, LaunchTable* t, int tag = TAG_PACK);
int launch_table(const LaunchTable& t, hipStream_t stream);

// Split a gather job per message (per neighbor) using the message counts.
void split_gather_by_counts(const GatherJob& j, const std::vector<int32_t>& counts,
                            size_t row_bytes, std::vector<GatherJob>* out);

inline size_t dtype_bytes(int dtype) { return dtype == HX_F32 ? 4 : 8; }

}  // namespace hx
