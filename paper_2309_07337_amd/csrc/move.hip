// Launch tables of the data-movement kernels: the job table and tile prefix
// in device memory, the launch shape, and the dispatch to the kernel
// translation units (move_gather / move_scatter / move_segsum).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "move_kernels.h"

namespace hx {
namespace {

// outside[j] = how many of job j's indices lie outside its source window
// (rows outside a window are read from global memory, so a window that
// holds few of them only costs its staging).
__global__ void __launch_bounds__(256) k_check_windows(const GatherJob* __restrict__ jobs, int njobs,
                                                       int64_t* __restrict__ outside) {
  __shared__ unsigned long long s_out;
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    const GatherJob g = jobs[j];
    if (threadIdx.x == 0) s_out = 0;
    __syncthreads();
    unsigned long long out = 0;
    if (g.win_rows > 0 && g.idx != nullptr) {
      for (int64_t e = threadIdx.x; e < g.nrows; e += blockDim.x) {
        const int64_t v = g.idx[e];
        out += (v < g.win_lo || v >= g.win_lo + g.win_rows) ? 1 : 0;
      }
    }
    if (out) atomicAdd(&s_out, out);  // LDS atomic
    __syncthreads();
    if (threadIdx.x == 0) outside[j] = (int64_t)s_out;
    __syncthreads();  // s_out is reset for the next job
  }
}

// te[t] = {ptr[r0], ptr[r1]} of tile t of a segmented-sum or push table
// (its rows [r0, r1) of job j), so a workgroup can load its tile's row
// pointers and entry indices together instead of one after the other.
__global__ void __launch_bounds__(256) k_tile_terms(const SegSumJob* __restrict__ jobs,
                                                    const int64_t* __restrict__ ts, int njobs, int64_t ntiles,
                                                    int tile_rows, int2* __restrict__ te) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles;
       t += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = njobs - 1;  // largest j with ts[j] <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ts[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int64_t r0 = (t - ts[lo]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, jobs[lo].nrows);
    te[t] = make_int2(jobs[lo].ptr[r0], jobs[lo].ptr[r1]);
  }
}

// Total terms of a segmented sum's jobs: the sum of ptr[nrows] - ptr[0].
__global__ void __launch_bounds__(256) k_term_count(const SegSumJob* __restrict__ jobs, int njobs,
                                                    unsigned long long* __restrict__ total) {
  unsigned long long acc = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < njobs; j += gridDim.x * blockDim.x)
    acc += (unsigned long long)(jobs[j].ptr[jobs[j].nrows] - jobs[j].ptr[0]);
  if (acc) atomicAdd(total, acc);
}

// The launch table of a single segmented-sum job written in place: the job
// descriptor, the tile prefix {0, ntiles} and every tile's entry range (as
// k_tile_terms), all from the kernel's arguments and the job's row pointers.
__global__ void __launch_bounds__(256) k_area_table(SegSumJob job, int64_t ntiles, int tile_rows,
                                                    SegSumJob* __restrict__ jobs, int64_t* __restrict__ ts,
                                                    int2* __restrict__ te) {
  const int64_t first = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (first == 0) {
    jobs[0] = job;
    ts[0] = 0;
    ts[1] = ntiles;
  }
  for (int64_t t = first; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r0 = t * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, job.nrows);
    te[t] = make_int2(job.ptr[r0], job.ptr[r1]);
  }
}

// Clears the windows of jobs that hold less than half of their indices
// and marks the jobs whose window holds all of them (device-side count).
int drop_bad_windows(std::vector<GatherJob>* w) {
  std::vector<int> at;
  for (size_t i = 0; i < w->size(); ++i) {
    (*w)[i].win_all = 0;
    if ((*w)[i].win_rows > 0 && (*w)[i].nrows > 0) at.push_back((int)i);
  }
  if (at.empty()) return HX_SUCCESS;
  std::vector<GatherJob> sub;
  for (int i : at) sub.push_back((*w)[i]);
  DevMem d_jobs, d_out;
  HX_TRY(upload_vec(d_jobs, sub));
  HX_TRY(d_out.alloc(sub.size() * sizeof(int64_t)));
  const int grid = (int)std::min<size_t>(sub.size(), 4096);
  hipLaunchKernelGGL(k_check_windows, dim3(grid), dim3(256), 0, 0, d_jobs.as<GatherJob>(), (int)sub.size(),
                     d_out.as<int64_t>());
  HX_HIP(hipGetLastError());
  std::vector<int64_t> outside(sub.size(), 0);
  HX_HIP(hipMemcpy(outside.data(), d_out.p, outside.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  for (size_t k = 0; k < at.size(); ++k) {
    GatherJob& g = (*w)[at[k]];
    if (g.idx == nullptr || 2 * outside[k] > g.nrows) {
      g.win_lo = 0;
      g.win_rows = 0;
    } else {
      g.win_all = outside[k] == 0 ? 1 : 0;
    }
  }
  return HX_SUCCESS;
}

// Vector width usable for a table: divides row_bytes and every base pointer.
int pick_vec(int row_bytes, uintptr_t align_or) {
  for (int vb : {16, 8, 4}) {
    if (row_bytes % vb == 0 && (align_or % vb) == 0) return vb;
  }
  return 0;
}

// Launch shape of a table (schedule checks, the jobs with rows and their tile
// prefix, vector width, grid); allocates nothing.
template <class J>
int shape_table(const std::vector<J>& jobs, int kind, int dtype, int row_bytes, const Sched& s0, LaunchTable* t,
                uintptr_t align_or, std::vector<J>* kept_out, std::vector<int64_t>* ts_out) {
  t->kind = kind;
  t->dtype = dtype;
  t->row_bytes = row_bytes;
  t->sched = s0;
  t->vec16 = 0;
  if (t->sched.tile_rows <= 0 || t->sched.block_threads <= 0 || t->sched.blocks_per_cu <= 0)
    return fail(HX_ERR_ARG, "invalid schedule (tile_rows %d, block_threads %d, blocks_per_cu %d)",
                t->sched.tile_rows, t->sched.block_threads, t->sched.blocks_per_cu);
  if (t->sched.block_threads != 256 && t->sched.block_threads != 512 &&
      !(kind != KIND_SCATTER && t->sched.block_threads == 1024))
    return fail(HX_ERR_ARG, "block_threads must be 256, 512 or 1024");
  // keep only jobs with rows; tile prefix
  std::vector<J>& kept = *kept_out;
  std::vector<int64_t>& ts = *ts_out;
  kept.clear();
  ts.assign(1, 0);
  for (const J& j : jobs) {
    if (j.nrows <= 0) continue;
    kept.push_back(j);
    ts.push_back(ts.back() + (j.nrows + t->sched.tile_rows - 1) / t->sched.tile_rows);
  }
  t->njobs = (int)kept.size();
  t->ntiles = ts.back();
  if (t->ntiles == 0) {
    t->grid = 0;
    t->jobs.release();
    t->tile_start.release();
    t->tile_terms.release();
    return HX_SUCCESS;
  }
  t->vec_bytes = pick_vec(row_bytes, align_or);
  if (t->vec_bytes == 0) return fail(HX_ERR_ARG, "rows of %d bytes / buffers not 4-byte aligned", row_bytes);
  if (kind == KIND_SEGSUM && (size_t)t->vec_bytes < dtype_bytes(dtype))
    return fail(HX_ERR_ARG, "FP64 buffers must be 8-byte aligned");
  int64_t want = (int64_t)t->sched.blocks_per_cu * device_cus();
  want = std::min<int64_t>(want, (t->ntiles + 7) / 8 * 8);
  want = std::min<int64_t>(want, int64_t(1) << 30);  // a launchable grid; larger tables take tile ranges
  want = std::max<int64_t>(8, (want + 7) / 8 * 8);
  t->grid = (int)want;
  return HX_SUCCESS;
}

template <class J>
int build_table(const std::vector<J>& jobs, int kind, int dtype, int row_bytes, const Sched& s0, LaunchTable* t,
                uintptr_t align_or) {
  std::vector<J> kept;
  std::vector<int64_t> ts;
  HX_TRY(shape_table(jobs, kind, dtype, row_bytes, s0, t, align_or, &kept, &ts));
  if (t->ntiles == 0) return HX_SUCCESS;
  HX_TRY(upload_vec(t->jobs, kept));
  HX_TRY(upload_vec(t->tile_start, ts));
  return HX_SUCCESS;
}

// Entry range of every tile of a CSR-driven table (segmented sum, push
// pack), read by their staged forms.
int fill_tile_terms(LaunchTable* t) {
  if (t->ntiles == 0) return HX_SUCCESS;
  HX_TRY(t->tile_terms.alloc((size_t)t->ntiles * sizeof(int2)));
  const int grid = (int)std::min<int64_t>((t->ntiles + 255) / 256, 4096);
  hipLaunchKernelGGL(k_tile_terms, dim3(grid), dim3(256), 0, 0, t->jobs.as<SegSumJob>(), t->tile_start.as<int64_t>(),
                     t->njobs, t->ntiles, t->sched.tile_rows, t->tile_terms.as<int2>());
  HX_HIP(hipGetLastError());
  HX_HIP(hipStreamSynchronize(0));
  return HX_SUCCESS;
}

uintptr_t align_of(const std::vector<SegSumJob>& jobs, int row_bytes) {
  uintptr_t a = (uintptr_t)row_bytes;
  for (const auto& j : jobs) {
    if (j.nrows <= 0) continue;
    a |= (uintptr_t)j.in | (uintptr_t)j.out;
    if (j.in2) a |= (uintptr_t)j.in2;
  }
  return a;
}

}  // namespace

int build_gather_table(const std::vector<GatherJob>& jobs, int dtype, int row_bytes, const Sched& s, LaunchTable* t,
                       int tag) {
  t->tag = tag;
  uintptr_t a = (uintptr_t)row_bytes;
  for (const auto& j : jobs) {
    if (j.nrows <= 0) continue;
    a |= (uintptr_t)j.src | (uintptr_t)j.dst;
  }
  // short rows in 16-byte groups per lane: rows of 4 or 8 bytes whose
  // buffers are aligned to the row size, and every index list congruent
  // with its destination (the first row whose destination is 16-byte
  // aligned also aligns the V-wide index loads, V = 16 / row_bytes)
  bool vec = s.pair_rows && (row_bytes == 8 || row_bytes == 4) && (a % (uintptr_t)row_bytes) == 0;
  if (vec) {
    const uintptr_t V = 16 / (uintptr_t)row_bytes;
    for (const auto& j : jobs) {
      if (j.nrows <= 0 || j.idx == nullptr) continue;
      if (((uintptr_t)j.idx % 4) != 0 || ((uintptr_t)j.idx / 4) % V != ((uintptr_t)j.dst / row_bytes) % V)
        vec = false;
    }
  }
  // source windows: kept where the schedule asks for them and they fit (the
  // 16-byte group form stages from the window's 16-byte aligned start)
  std::vector<GatherJob> w(jobs);
  const int64_t win_cap = std::min<int64_t>(kWinBytes, device_lds_per_block());
  auto win_span = [&](const GatherJob& j) -> int64_t {
    const int64_t bytes = j.win_rows * (int64_t)row_bytes;
    return vec ? bytes + (int64_t)(((uintptr_t)j.src + (uintptr_t)(j.win_lo * row_bytes)) & 15) : bytes;
  };
  for (auto& j : w) {
    if (!s.lds_window || j.idx == nullptr || j.win_rows <= 0 || win_span(j) > win_cap || j.win_lo < 0) {
      j.win_lo = 0;
      j.win_rows = 0;
    }
  }
  HX_TRY(drop_bad_windows(&w));
  int64_t win_bytes = 0;
  for (const auto& j : w) {
    if (j.win_rows <= 0) continue;
    if (!vec) a |= (uintptr_t)(j.src + j.win_lo * (int64_t)row_bytes);
    win_bytes = std::max(win_bytes, win_span(j));
  }
  HX_TRY(build_table(w, KIND_GATHER, dtype, row_bytes, s, t, a));
  // (the runtime-row-size kernel form ignores windows and reads global memory)
  t->win_bytes = t->ntiles > 0 ? (int)((win_bytes + 15) / 16 * 16) : 0;
  t->vec16 = t->ntiles > 0 && vec ? 1 : 0;
  t->partial_win = 0;
  for (const auto& j : w)
    if (j.nrows > 0 && j.win_rows > 0 && !j.win_all) t->partial_win = 1;
  return HX_SUCCESS;
}

// Shape of a segmented-sum table: term windows, launch shape, term buffer
// (no device memory).
// Shape of a segmented sum of rows of one value, one row per lane: each
// job keeps its term window where it fits (80 KiB with the staging's
// alignment) and lies in one input; no term buffer.
int shape_segsum_vec_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes, const Sched& s,
                           LaunchTable* t, int tag, std::vector<SegSumJob>* kept, std::vector<int64_t>* ts) {
  t->tag = tag;
  std::vector<SegSumJob> w(jobs);
  const int64_t cap = std::min<int64_t>(kWinBytes, device_lds_per_block());
  int64_t win_bytes = 0;
  for (auto& j : w) {
    const int64_t hi = j.win_lo + j.win_rows;
    const bool one_input = hi <= j.split || j.win_lo >= j.split;
    int64_t span = 0;
    if (j.win_rows > 0 && j.win_lo >= 0 && one_input) {
      const char* a = j.win_lo < j.split ? j.in + j.win_lo * (int64_t)row_bytes
                                         : j.in2 + (j.win_lo - j.split) * (int64_t)row_bytes;
      span = j.win_rows * (int64_t)row_bytes + (int64_t)((uintptr_t)a & 15);
    }
    if (!s.lds_window || j.nrows <= 0 || span <= 0 || span > cap) {
      j.win_lo = j.win_rows = 0;
    } else {
      win_bytes = std::max(win_bytes, span);
    }
  }
  HX_TRY(shape_table(w, KIND_SEGSUM, dtype, row_bytes, s, t, align_of(w, row_bytes), kept, ts));
  t->win_bytes = t->ntiles > 0 ? (int)((win_bytes + 15) / 16 * 16) : 0;
  t->val_bytes = 0;
  t->vec16 = t->ntiles > 0 ? 1 : 0;
  t->vec_depth = 4;  // (set from the jobs' term counts when the table is uploaded)
  return HX_SUCCESS;
}

int shape_segsum_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes, const Sched& s,
                       LaunchTable* t, int tag, std::vector<SegSumJob>* kept, std::vector<int64_t>* ts) {
  if (s.pair_rows && (row_bytes == 4 || row_bytes == 8) && (size_t)row_bytes == dtype_bytes(dtype))
    return shape_segsum_vec_table(jobs, dtype, row_bytes, s, t, tag, kept, ts);
  t->tag = tag;
  // term windows: kept where the schedule asks for them, they fit, and they
  // lie inside one of the two inputs
  // (all jobs or none: a job without a window would run the windowed form's
  // row-parallel loop from global memory, slower than the plain form)
  std::vector<SegSumJob> w(jobs);
  const int64_t cap = std::min<int64_t>(kSegWinBytes, device_lds_per_block() - (8 << 10));
  int64_t win_bytes = 0;
  // (the windowed kernel is bounded to 512 lanes)
  bool all = s.lds_window != 0 && s.block_threads <= 512;
  for (const auto& j : w) {
    if (j.nrows <= 0) continue;
    const int64_t bytes = j.win_rows * (int64_t)row_bytes;
    const int64_t hi = j.win_lo + j.win_rows;
    const bool one_input = hi <= j.split || j.win_lo >= j.split;
    if (j.win_rows <= 0 || j.win_lo < 0 || bytes > cap || !one_input) all = false;
    else win_bytes = std::max(win_bytes, bytes);
  }
  if (!all) {
    win_bytes = 0;
    for (auto& j : w) j.win_lo = j.win_rows = 0;
  }
  uintptr_t a = align_of(w, row_bytes);
  for (const auto& j : w)
    if (j.win_rows > 0 && j.nrows > 0)
      a |= (uintptr_t)(j.win_lo < j.split ? j.in + j.win_lo * (int64_t)row_bytes
                                           : j.in2 + (j.win_lo - j.split) * (int64_t)row_bytes);
  HX_TRY(shape_table(w, KIND_SEGSUM, dtype, row_bytes, s, t, a, kept, ts));
  t->win_bytes = t->ntiles > 0 ? (int)win_bytes : 0;
  // term buffer: about two terms per tile row, at least 4 KiB and at most
  // kSegValueBytes, whole rows (small tiles leave LDS for more workgroups)
  int64_t vb = std::min<int64_t>(kSegValueBytes, std::max<int64_t>(4096, 2 * (int64_t)s.tile_rows * row_bytes));
  t->val_bytes = t->ntiles > 0 && row_bytes > 0 ? (int)(vb / row_bytes * row_bytes) : 0;
  return HX_SUCCESS;
}

int build_segsum_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes, const Sched& s,
                       LaunchTable* t, int tag) {
  std::vector<SegSumJob> kept;
  std::vector<int64_t> ts;
  HX_TRY(shape_segsum_table(jobs, dtype, row_bytes, s, t, tag, &kept, &ts));
  if (t->ntiles == 0) return HX_SUCCESS;
  HX_TRY(upload_vec(t->jobs, kept));
  HX_TRY(upload_vec(t->tile_start, ts));
  if (t->vec16) {
    // one-value sums: 16 terms per row loaded together (one row per lane)
    // where rows average more than three terms (the owner sums of high
    // fan-out packs), else 4
    int64_t rows = 0;
    for (const auto& j : kept) rows += j.nrows;
    DevMem d_terms;
    HX_TRY(d_terms.alloc(sizeof(unsigned long long)));
    HX_HIP(hipMemset(d_terms.p, 0, sizeof(unsigned long long)));
    const int grid = (int)std::min<size_t>((kept.size() + 255) / 256, 1024);
    hipLaunchKernelGGL(k_term_count, dim3(grid), dim3(256), 0, 0, t->jobs.as<SegSumJob>(), t->njobs,
                       d_terms.as<unsigned long long>());
    HX_HIP(hipGetLastError());
    unsigned long long terms = 0;
    HX_HIP(hipMemcpy(&terms, d_terms.p, sizeof(terms), hipMemcpyDeviceToHost));
    t->vec_depth = (int64_t)terms > 3 * rows ? 16 : 4;
  }
  return fill_tile_terms(t);
}

int launch_segsum_in_area(const SegSumJob& job, int dtype, int row_bytes, const Sched& s, void* area,
                          size_t area_bytes, hipStream_t stream, int tag) {
  LaunchTable t;
  std::vector<SegSumJob> kept;
  std::vector<int64_t> ts;
  HX_TRY(shape_segsum_table(std::vector<SegSumJob>(1, job), dtype, row_bytes, s, &t, tag, &kept, &ts));
  if (t.ntiles == 0) return HX_SUCCESS;
  if (t.ntiles > segsum_area_max_tiles(area_bytes))
    return fail(HX_ERR_UNSUPPORTED, "%lld tiles of %d rows exceed the %lld a %zu-byte area holds",
                (long long)t.ntiles, t.sched.tile_rows, (long long)segsum_area_max_tiles(area_bytes), area_bytes);
  if (area == nullptr || ((uintptr_t)area % 256) != 0) return fail(HX_ERR_ARG, "area must be 256-byte aligned");
  static_assert(sizeof(SegSumJob) + 2 * sizeof(int64_t) <= kAreaHeadBytes, "area head");
  char* base = static_cast<char*>(area);
  t.jobs.borrow(base, sizeof(SegSumJob));
  t.tile_start.borrow(base + 256, 2 * sizeof(int64_t));
  t.tile_terms.borrow(base + kAreaHeadBytes, (size_t)t.ntiles * sizeof(int2));
  const int grid = (int)std::min<int64_t>((t.ntiles + 255) / 256, 4096);
  hipLaunchKernelGGL(k_area_table, dim3(grid), dim3(256), 0, stream, kept[0], t.ntiles, t.sched.tile_rows,
                     t.jobs.as<SegSumJob>(), t.tile_start.as<int64_t>(), t.tile_terms.as<int2>());
  HX_HIP(hipGetLastError());
  return launch_table(t, stream);
}

int build_scatter_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes, const Sched& s,
                        LaunchTable* t, int tag) {
  t->tag = tag;
  Sched sc = s;
  sc.block_threads = std::min(sc.block_threads, 512);  // the push pack runs at most 512 lanes
  HX_TRY(build_table(jobs, KIND_SCATTER, dtype, row_bytes, sc, t, align_of(jobs, row_bytes)));
  return fill_tile_terms(t);
}

int launch_table(const LaunchTable& t, hipStream_t s) {
  if (t.ntiles == 0) return HX_SUCCESS;
  if (t.kind == KIND_GATHER) launch_gather_kernels(t, s);
  else if (t.kind == KIND_SCATTER) launch_scatter_kernels(t, s);
  else launch_segsum_kernels(t, s);
  HX_HIP(hipGetLastError());
  return HX_SUCCESS;
}

void split_gather_by_counts(const GatherJob& j, const std::vector<int32_t>& counts, size_t row_bytes,
                            std::vector<GatherJob>* out) {
  int64_t off = 0;
  for (int32_t c : counts) {
    if (c > 0) {
      GatherJob g = j;
      g.dst = j.dst + off * (int64_t)row_bytes;
      g.idx = j.idx ? j.idx + off : nullptr;
      g.src = j.idx ? j.src : j.src + off * (int64_t)row_bytes;
      g.nrows = c;
      out->push_back(g);
    }
    off += c;
  }
  if (off < j.nrows) {  // rows beyond the listed messages (none for valid plans)
    GatherJob g = j;
    g.dst = j.dst + off * (int64_t)row_bytes;
    g.idx = j.idx ? j.idx + off : nullptr;
    g.src = j.idx ? j.src : j.src + off * (int64_t)row_bytes;
    g.nrows = j.nrows - off;
    out->push_back(g);
  }
}

}  // namespace hx
