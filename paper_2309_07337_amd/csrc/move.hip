// Data-movement kernels of the exchange: the indexed row gather behind the
// pack (Start), the redistribution pack and the unpack (Wait), and the
// fixed-order segmented sum behind the backward of the pack.
//
// Both kernels are persistent and multi-job: a launch walks a table of jobs
// (one per request, phase or message), cut into tiles of `tile_rows` rows.
// Workgroup b runs on XCD b % 8 (round-robin dispatch), so logical workgroup
// ids are regrouped per XCD and each logical workgroup takes a contiguous
// range of tiles: consecutive tiles -- and the rows they re-read -- stay in
// one XCD's L2.  Rows are moved as 16/8/4-byte vectors with LPR lanes per
// row; U rows per lane are loaded before any is stored, to keep enough bytes
// in flight for HBM.  The work is pure data movement (plus adds in the
// backward): no matrix cores are involved.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace hx {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <int VB> struct RawVec;
template <> struct RawVec<16> { using type = u32x4; };
template <> struct RawVec<8> { using type = u32x2; };
template <> struct RawVec<4> { using type = unsigned int; };

template <class T, int VB> struct NumVec;
template <> struct NumVec<float, 16> { using type = f32x4; };
template <> struct NumVec<float, 8> { using type = f32x2; };
template <> struct NumVec<float, 4> { using type = float; };
template <> struct NumVec<double, 16> { using type = f64x2; };
template <> struct NumVec<double, 8> { using type = double; };

template <class T, bool NT>
__device__ __forceinline__ T ldv(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <class T, bool NT>
__device__ __forceinline__ void stv(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Contiguous tile range of this workgroup; workgroups of one XCD get
// neighbouring ranges.  gridDim.x is a multiple of 8.
__device__ __forceinline__ void tile_range(int64_t ntiles, int64_t* t0, int64_t* t1) {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int per = nb >> 3;
  const int L = (b & 7) * per + (b >> 3);
  *t0 = (int64_t)L * ntiles / nb;
  *t1 = (int64_t)(L + 1) * ntiles / nb;
}

// Largest j with ts[j] <= t (jobs with no tiles are skipped).
__device__ __forceinline__ int find_job(const int64_t* __restrict__ ts, int njobs, int64_t t) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ts[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Indexed row gather.  NV vectors of VB bytes per row (NV = 0: runtime nv),
// LPR lanes per row, U rows per lane in flight.
// ---------------------------------------------------------------------------
template <int VB, int NV, int LPR, int U, bool NT>
__device__ __forceinline__ void gather_body(const GatherJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                            int njobs, int64_t ntiles, int tile_rows, int nv_rt) {
  using V = typename RawVec<VB>::type;
  const int nv = NV > 0 ? NV : nv_rt;
  constexpr int NVPL = NV > 0 ? (NV + LPR - 1) / LPR : 1;
  const int lane_v = threadIdx.x % LPR;
  const int rsub = threadIdx.x / LPR;
  const int rows_per_pass = blockDim.x / LPR;
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const char* __restrict__ src = jobs[j].src;
    char* __restrict__ dst = jobs[j].dst;
    const int32_t* __restrict__ idx = jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const size_t rb = (size_t)nv * VB;
    if constexpr (NV > 0) {
      for (int64_t base = r0 + rsub; base < r1; base += (int64_t)rows_per_pass * U) {
        V v[U][NVPL];
        int64_t srow[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t r = base + (int64_t)u * rows_per_pass;
          srow[u] = (r < r1) ? (idx ? (int64_t)ldv<int32_t, NT>(idx + r) : r) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (srow[u] >= 0) {
            const V* sp = reinterpret_cast<const V*>(src + srow[u] * rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) v[u][k] = sp[vi];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t r = base + (int64_t)u * rows_per_pass;
          if (srow[u] >= 0) {
            V* dp = reinterpret_cast<V*>(dst + r * rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) stv<V, NT>(dp + vi, v[u][k]);
            }
          }
        }
      }
    } else {
      for (int64_t r = r0 + rsub; r < r1; r += rows_per_pass) {
        const int64_t s = idx ? (int64_t)ldv<int32_t, NT>(idx + r) : r;
        const V* sp = reinterpret_cast<const V*>(src + s * rb);
        V* dp = reinterpret_cast<V*>(dst + r * rb);
        for (int vi = lane_v; vi < nv; vi += LPR) stv<V, NT>(dp + vi, sp[vi]);
      }
    }
  }
}

// One kernel symbol per phase (same body), so profiles attribute time to the
// pack (Start), the redistribution pack and the unpack (Wait), and the
// simulated transfer separately.
#define HX_GATHER_KERNEL(NAME)                                                                       \
  template <int VB, int NV, int LPR, int U, bool NT>                                                 \
  __global__ void __launch_bounds__(512)                                                             \
      NAME(const GatherJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,            \
           int64_t ntiles, int tile_rows, int nv_rt) {                                               \
    gather_body<VB, NV, LPR, U, NT>(jobs, ts, njobs, ntiles, tile_rows, nv_rt);                      \
  }
HX_GATHER_KERNEL(k_pack)
HX_GATHER_KERNEL(k_redist)
HX_GATHER_KERNEL(k_unpack)
HX_GATHER_KERNEL(k_transfer)
#undef HX_GATHER_KERNEL

// ---------------------------------------------------------------------------
// Fixed-order segmented sum: out[i] = in[idx[ptr[i]]] + in[idx[ptr[i]+1]] + ...
// Additions in T, strictly in ascending e, the accumulator starting from the
// first term; an empty segment stores +0.
// ---------------------------------------------------------------------------
template <class T, int VB, int NV, int LPR, bool NT>
__global__ void __launch_bounds__(512)
k_segsum(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,
         int64_t ntiles, int tile_rows, int nv_rt) {
  using V = typename NumVec<T, VB>::type;
  const int nv = NV > 0 ? NV : nv_rt;
  const int lane_v = threadIdx.x % LPR;
  const int rsub = threadIdx.x / LPR;
  const int rows_per_pass = blockDim.x / LPR;
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const char* __restrict__ in = jobs[j].in;
    char* __restrict__ out = jobs[j].out;
    const int32_t* __restrict__ ptr = jobs[j].ptr;
    const int32_t* __restrict__ idx = jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const size_t rb = (size_t)nv * VB;
    for (int64_t r = r0 + rsub; r < r1; r += rows_per_pass) {
      const int32_t p0 = ptr[r];
      const int32_t p1 = ptr[r + 1];
      V* dp = reinterpret_cast<V*>(out + r * rb);
      for (int vi = lane_v; vi < nv; vi += LPR) {
        V acc = (V)(T)0;
        // Terms are loaded K at a time (independent loads in flight) and then
        // added strictly in ascending e: the order of additions is fixed.
        constexpr int K = 4;
        for (int32_t e0 = p0; e0 < p1; e0 += K) {
          V v[K];
#pragma unroll
          for (int k = 0; k < K; ++k)
            if (e0 + k < p1)
              v[k] = reinterpret_cast<const V*>(in + (int64_t)ldv<int32_t, NT>(idx + e0 + k) * rb)[vi];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (e0 + k < p1) acc = (e0 + k == p0) ? v[k] : acc + v[k];
          }
        }
        stv<V, NT>(dp + vi, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side dispatch.
// ---------------------------------------------------------------------------
template <int VB, int NV, int LPR, int U, bool NT>
void go_gather_nt(const LaunchTable& t, hipStream_t s, int nv) {
  const dim3 g(t.grid), b(t.sched.block_threads);
  const GatherJob* jobs = t.jobs.as<GatherJob>();
  const int64_t* ts = t.tile_start.as<int64_t>();
  switch (t.tag) {
    case TAG_PACK:
      hipLaunchKernelGGL((k_pack<VB, NV, LPR, U, NT>), g, b, 0, s, jobs, ts, t.njobs, t.ntiles, t.sched.tile_rows, nv);
      break;
    case TAG_REDIST:
      hipLaunchKernelGGL((k_redist<VB, NV, LPR, U, NT>), g, b, 0, s, jobs, ts, t.njobs, t.ntiles, t.sched.tile_rows,
                         nv);
      break;
    case TAG_UNPACK:
      hipLaunchKernelGGL((k_unpack<VB, NV, LPR, U, NT>), g, b, 0, s, jobs, ts, t.njobs, t.ntiles, t.sched.tile_rows,
                         nv);
      break;
    default:
      hipLaunchKernelGGL((k_transfer<VB, NV, LPR, U, NT>), g, b, 0, s, jobs, ts, t.njobs, t.ntiles,
                         t.sched.tile_rows, nv);
      break;
  }
}

template <int VB, int NV, int LPR, int U>
void go_gather(const LaunchTable& t, hipStream_t s, int nv) {
  if (t.sched.nontemporal) go_gather_nt<VB, NV, LPR, U, true>(t, s, nv);
  else go_gather_nt<VB, NV, LPR, U, false>(t, s, nv);
}

template <class T, int VB, int NV, int LPR>
void go_segsum(const LaunchTable& t, hipStream_t s, int nv) {
  const dim3 g(t.grid), b(t.sched.block_threads);
  if (t.sched.nontemporal)
    hipLaunchKernelGGL((k_segsum<T, VB, NV, LPR, true>), g, b, 0, s, t.jobs.as<SegSumJob>(),
                       t.tile_start.as<int64_t>(), t.njobs, t.ntiles, t.sched.tile_rows, nv);
  else
    hipLaunchKernelGGL((k_segsum<T, VB, NV, LPR, false>), g, b, 0, s, t.jobs.as<SegSumJob>(),
                       t.tile_start.as<int64_t>(), t.njobs, t.ntiles, t.sched.tile_rows, nv);
}

// Vector width usable for a table: divides row_bytes and every base pointer.
int pick_vec(int row_bytes, uintptr_t align_or) {
  for (int vb : {16, 8, 4}) {
    if (row_bytes % vb == 0 && (align_or % vb) == 0) return vb;
  }
  return 0;
}

template <int VB>
void dispatch_gather(const LaunchTable& t, hipStream_t s) {
  const int nv = t.row_bytes / VB;
  if constexpr (VB == 16) {
    switch (nv) {
      case 1: return go_gather<16, 1, 1, 4>(t, s, nv);
      case 2: return go_gather<16, 2, 2, 4>(t, s, nv);
      case 4: return go_gather<16, 4, 4, 4>(t, s, nv);
      case 8: return go_gather<16, 8, 8, 4>(t, s, nv);
      case 16: return go_gather<16, 16, 16, 4>(t, s, nv);
      case 32: return go_gather<16, 32, 32, 2>(t, s, nv);
      case 64: return go_gather<16, 64, 64, 2>(t, s, nv);
      default: break;
    }
  } else if constexpr (VB == 8) {
    if (nv == 1) return go_gather<8, 1, 1, 8>(t, s, nv);
    if (nv == 3) return go_gather<8, 3, 1, 4>(t, s, nv);
  } else {
    if (nv == 1) return go_gather<4, 1, 1, 8>(t, s, nv);
  }
  if (nv >= 64) return go_gather<VB, 0, 64, 1>(t, s, nv);
  if (nv >= 16) return go_gather<VB, 0, 16, 1>(t, s, nv);
  if (nv >= 4) return go_gather<VB, 0, 4, 1>(t, s, nv);
  return go_gather<VB, 0, 1, 1>(t, s, nv);
}

template <class T, int VB>
void dispatch_segsum(const LaunchTable& t, hipStream_t s) {
  const int nv = t.row_bytes / VB;
  if constexpr (VB == 16) {
    switch (nv) {
      case 1: return go_segsum<T, 16, 1, 1>(t, s, nv);
      case 8: return go_segsum<T, 16, 8, 8>(t, s, nv);
      case 16: return go_segsum<T, 16, 16, 16>(t, s, nv);
      default: break;
    }
  } else if constexpr (VB == 8) {
    if (nv == 1) return go_segsum<T, 8, 1, 1>(t, s, nv);
  } else {
    if (nv == 1) return go_segsum<T, 4, 1, 1>(t, s, nv);
  }
  if (nv >= 64) return go_segsum<T, VB, 0, 64>(t, s, nv);
  if (nv >= 16) return go_segsum<T, VB, 0, 16>(t, s, nv);
  if (nv >= 4) return go_segsum<T, VB, 0, 4>(t, s, nv);
  return go_segsum<T, VB, 0, 1>(t, s, nv);
}

template <class J>
int build_table(const std::vector<J>& jobs, int kind, int dtype, int row_bytes, const Sched& s0,
                LaunchTable* t, uintptr_t align_or) {
  t->kind = kind;
  t->dtype = dtype;
  t->row_bytes = row_bytes;
  t->sched = s0;
  if (t->sched.tile_rows <= 0 || t->sched.block_threads <= 0 || t->sched.blocks_per_cu <= 0)
    return fail(HX_ERR_ARG, "invalid schedule (tile_rows %d, block_threads %d, blocks_per_cu %d)",
                t->sched.tile_rows, t->sched.block_threads, t->sched.blocks_per_cu);
  if (t->sched.block_threads != 256 && t->sched.block_threads != 512)
    return fail(HX_ERR_ARG, "block_threads must be 256 or 512");
  // keep only jobs with rows; tile prefix
  std::vector<J> kept;
  std::vector<int64_t> ts(1, 0);
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
    return HX_SUCCESS;
  }
  t->vec_bytes = pick_vec(row_bytes, align_or);
  if (t->vec_bytes == 0)
    return fail(HX_ERR_ARG, "rows of %d bytes / buffers not 4-byte aligned", row_bytes);
  if (kind == KIND_SEGSUM && (size_t)t->vec_bytes < dtype_bytes(dtype))
    return fail(HX_ERR_ARG, "FP64 buffers must be 8-byte aligned");
  HX_TRY(upload_vec(t->jobs, kept));
  HX_TRY(upload_vec(t->tile_start, ts));
  int64_t want = (int64_t)t->sched.blocks_per_cu * device_cus();
  want = std::min<int64_t>(want, (t->ntiles + 7) / 8 * 8);
  want = std::max<int64_t>(8, (want + 7) / 8 * 8);
  t->grid = (int)want;
  return HX_SUCCESS;
}

}  // namespace

int build_gather_table(const std::vector<GatherJob>& jobs, int dtype, int row_bytes,
                       const Sched& s, LaunchTable* t, int tag) {
  t->tag = tag;
  uintptr_t a = (uintptr_t)row_bytes;
  for (const auto& j : jobs) {
    if (j.nrows <= 0) continue;
    a |= (uintptr_t)j.src | (uintptr_t)j.dst;
  }
  return build_table(jobs, KIND_GATHER, dtype, row_bytes, s, t, a);
}

int build_segsum_table(const std::vector<SegSumJob>& jobs, int dtype, int row_bytes,
                       const Sched& s, LaunchTable* t) {
  uintptr_t a = (uintptr_t)row_bytes;
  for (const auto& j : jobs) {
    if (j.nrows <= 0) continue;
    a |= (uintptr_t)j.in | (uintptr_t)j.out;
  }
  return build_table(jobs, KIND_SEGSUM, dtype, row_bytes, s, t, a);
}

int launch_table(const LaunchTable& t, hipStream_t s) {
  if (t.ntiles == 0) return HX_SUCCESS;
  const int vb = t.vec_bytes;  // divides row_bytes and every base pointer
  if (t.kind == KIND_GATHER) {
    if (vb == 16) dispatch_gather<16>(t, s);
    else if (vb == 8) dispatch_gather<8>(t, s);
    else dispatch_gather<4>(t, s);
  } else {
    if (t.dtype == HX_F32) {
      if (vb == 16) dispatch_segsum<float, 16>(t, s);
      else if (vb == 8) dispatch_segsum<float, 8>(t, s);
      else dispatch_segsum<float, 4>(t, s);
    } else {
      if (vb == 16) dispatch_segsum<double, 16>(t, s);
      else dispatch_segsum<double, 8>(t, s);
    }
  }
  HX_HIP(hipGetLastError());
  return HX_SUCCESS;
}

void split_gather_by_counts(const GatherJob& j, const std::vector<int32_t>& counts,
                            size_t row_bytes, std::vector<GatherJob>* out) {
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
