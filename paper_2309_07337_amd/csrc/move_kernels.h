// Device bodies of the data-movement kernels (included by the move_*.hip
// translation units, which instantiate and launch them).
//
// All kernels are multi-job: a launch walks a table of jobs cut into tiles
// of `tile_rows` rows.  Workgroup b runs on XCD b % 8 (round-robin
// dispatch), so logical workgroup ids are regrouped per XCD and each logical
// workgroup takes a contiguous range of tiles: consecutive tiles -- and the
// rows they share -- stay in one XCD's L2.  With a grid as large as the tile
// count (one-shot) each workgroup takes one tile and the hardware hands them
// out in order; with a smaller grid (persistent) each walks its range, which
// lets a job's LDS window be staged once.  Rows move as 16/8/4-byte vectors with LPR
// lanes per row; U rows per lane are loaded before any is stored, to keep
// enough bytes in flight for HBM.  LDS carries the rest: CSR-driven kernels
// stage each tile's row pointers and entry indices (the push pack then runs
// entry-parallel; the segmented sum gathers a chunk's terms entry-parallel
// and adds them per row from LDS), and short-row gathers and sums can stage
// a job's whole source window.  Pure data movement (plus adds in the
// segmented sums): no matrix cores are involved.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace hx {
namespace kern {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
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

// Every buffer a job names is device (global) memory.  Pointers read from a
// job table carry no address space, so the compiler would access them with
// FLAT instructions (address-space checks, both wait counters, and LDS-window
// reads merged into the same FLAT access); the bodies below cast them to the
// global address space (HX_G), which gives global loads and stores with a
// scalar base and 32-bit lane offsets, and keeps LDS reads as LDS reads.
#define HX_G __attribute__((address_space(1)))
#define HX_L __attribute__((address_space(3)))

template <class T, bool NT, class P>
__device__ __forceinline__ T ldv(P p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <class T, bool NT, class P>
__device__ __forceinline__ void stv(P p, T v) {
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

// Completion counter of a message (partition-ready pack): once every lane's
// stores of the tile are done (workgroup barrier), one lane makes them
// visible device-wide (release fence) and adds the tile's rows.  A reader
// that sees the counter reach its target (acquire) sees the rows.
__device__ __forceinline__ void signal_tile(unsigned long long* ready, int64_t rows) {
  if (ready == nullptr) return;  // uniform: the whole tile belongs to one job
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(ready, (unsigned long long)rows);
  }
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
// Pull: dst[r] = src[idx ? idx[r] : r].  NV vectors of VB bytes per row
// (NV = 0: runtime nv, then U must be 1), LPR lanes per row.
// ---------------------------------------------------------------------------
// Source windows (use_win != 0, fixed shapes only): a job with win_rows > 0
// reads mostly source rows [win_lo, win_lo + win_rows) (the table builder
// counts them on the device and drops windows that hold less than half of
// a job's indices), and the table's dynamic LDS holds that many rows.  The
// workgroup copies the window into LDS with coalesced loads when it reaches
// a new such job and then gathers rows inside it from LDS, the others from
// global memory: one wide read of the window instead of one L2 request per
// (usually short, scattered) row.
template <int VB, int NV, int LPR, int U, bool NT>
__device__ __forceinline__ void gather_body(const GatherJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                            int njobs, int64_t ntiles, int tile_rows, int nv_rt, int use_win) {
  using V = typename RawVec<VB>::type;
  const int nv = NV > 0 ? NV : nv_rt;
  constexpr int NVPL = NV > 0 ? (NV + LPR - 1) / LPR : 1;
  const int lane_v = threadIdx.x % LPR;
  const int rsub = threadIdx.x / LPR;
  const int rows_per_pass = blockDim.x / LPR;
  extern __shared__ __align__(16) unsigned char s_dyn[];
  V* __restrict__ s_win = reinterpret_cast<V*>(s_dyn);
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  int staged = -1;
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const HX_G char* __restrict__ src = (const HX_G char*)jobs[j].src;
    HX_G char* __restrict__ dst = (HX_G char*)jobs[j].dst;
    const HX_G int32_t* __restrict__ idx = (const HX_G int32_t*)jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const size_t rb = (size_t)nv * VB;
    int64_t win_lo = 0, win_rows = 0;
    if constexpr (NV > 0) {
      if (use_win && idx != nullptr && jobs[j].win_rows > 0) {
        win_lo = jobs[j].win_lo;
        win_rows = jobs[j].win_rows;
        if (staged != j) {
          __syncthreads();  // every lane is done with the previous window
          const HX_G V* __restrict__ wp = reinterpret_cast<const HX_G V*>(src + win_lo * (int64_t)rb);
          const int nvec = (int)win_rows * NV;
          constexpr int UW = 8;  // loads in flight per lane while staging
          for (int i0 = threadIdx.x; i0 < nvec; i0 += blockDim.x * UW) {
            V w[UW];
#pragma unroll
            for (int u = 0; u < UW; ++u) {
              const int i = i0 + u * blockDim.x;
              if (i < nvec) w[u] = wp[i];
            }
#pragma unroll
            for (int u = 0; u < UW; ++u) {
              const int i = i0 + u * blockDim.x;
              if (i < nvec) s_win[i] = w[u];
            }
          }
          __syncthreads();
          staged = j;
        }
      }
    }
    if constexpr (NV > 0 && VB == 16) {
      if (idx == nullptr) {
        // identity job: the tile is one contiguous byte range; copy it as a
        // flat stream of 16-byte vectors, 8 in flight per lane
        constexpr int UC = 8;
        const HX_G V* __restrict__ sp = reinterpret_cast<const HX_G V*>(src + r0 * rb);
        HX_G V* __restrict__ dp = reinterpret_cast<HX_G V*>(dst + r0 * rb);
        const int64_t nvec = (r1 - r0) * NV;
        for (int64_t i = threadIdx.x; i < nvec; i += (int64_t)blockDim.x * UC) {
          V c[UC];
#pragma unroll
          for (int u = 0; u < UC; ++u) {
            const int64_t k = i + (int64_t)u * blockDim.x;
            if (k < nvec) c[u] = ldv<V, NT>(sp + k);
          }
#pragma unroll
          for (int u = 0; u < UC; ++u) {
            const int64_t k = i + (int64_t)u * blockDim.x;
            if (k < nvec) stv<V, NT>(dp + k, c[u]);
          }
        }
        signal_tile(jobs[j].ready, r1 - r0);
        continue;
      }
    }
    if constexpr (NV > 0) {
      // Lanes past the tile's end re-read its last row, so every index and
      // row load is valid and the U loads of a lane go out together (no
      // branch between them); only the stores are predicated.
      const bool in_lds = win_rows > 0;
      for (int64_t base = r0 + rsub; base < r1; base += (int64_t)rows_per_pass * U) {
        V v[U][NVPL];
        int64_t srow[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t r = min(base + (int64_t)u * rows_per_pass, r1 - 1);
          srow[u] = idx ? (int64_t)ldv<int32_t, NT>(idx + r) : r;
        }
        if (in_lds) {
          // rows inside the window from LDS, the others from global memory
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t wr = srow[u] - win_lo;
            const bool inw = (uint64_t)wr < (uint64_t)win_rows;
            const HX_G V* sp = reinterpret_cast<const HX_G V*>(src + srow[u] * rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) {
                if (inw) v[u][k] = s_win[wr * NV + vi];
                else v[u][k] = sp[vi];
              }
            }
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const HX_G V* sp = reinterpret_cast<const HX_G V*>(src + srow[u] * rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) v[u][k] = idx ? sp[vi] : ldv<V, NT>(sp + vi);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t r = base + (int64_t)u * rows_per_pass;
          if (r < r1) {
            HX_G V* dp = reinterpret_cast<HX_G V*>(dst + r * rb);
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
        const HX_G V* sp = reinterpret_cast<const HX_G V*>(src + s * rb);
        HX_G V* dp = reinterpret_cast<HX_G V*>(dst + r * rb);
        for (int vi = lane_v; vi < nv; vi += LPR) stv<V, NT>(dp + vi, sp[vi]);
      }
    }
    signal_tile(jobs[j].ready, r1 - r0);
  }
}

// ---------------------------------------------------------------------------
// Pull of short rows (RB = 4 or 8 bytes), 16 bytes of rows per lane: a group
// of V = 16 / RB consecutive rows takes one V-wide load of its indices, V
// row reads and one 16-byte store, so a wavefront's index loads and stores
// are single coalesced streams (short rows are bound by memory requests and
// by the latency of the index stream, not by bytes).  Each lane handles U
// groups per pass, their index loads issued together; a job with an LDS
// source window (win_rows > 0) has it staged by the workgroup once (16-byte
// loads of its aligned interior, 4-byte loads of its ragged ends) while the
// first pass's indices are in flight, and rows inside it are read from LDS,
// the others from global memory.  Groups start at the first row whose
// destination is 16-byte aligned; the table builder enables this form only
// where every job's index list is congruent with its destination (the same
// first row aligns the index vector loads), so the rows before that first
// group and after the last one (fewer than V each) go one per lane.
// ---------------------------------------------------------------------------
template <int RB> struct IdxVec;
template <> struct IdxVec<8> { using type = i32x2; };
template <> struct IdxVec<4> { using type = int __attribute__((ext_vector_type(4))); };

template <int RB>
__device__ __forceinline__ u32x4 pack16(const typename RawVec<RB>::type (&v)[16 / RB]) {
  if constexpr (RB == 8) return u32x4{v[0].x, v[0].y, v[1].x, v[1].y};
  else return u32x4{v[0], v[1], v[2], v[3]};
}

// A job's pointer as global memory (GAS) or without an address space.
template <bool GAS, class T>
__device__ __forceinline__ auto gas_ptr(T* p) {
  if constexpr (GAS) return (HX_G T*)p;
  else return p;
}

// GAS: the jobs' buffers are accessed as global memory (tables whose jobs
// have no window, or whose indices all lie in it); otherwise without an
// address space (FLAT), so that a row inside or outside the window is one
// load of either address: measured faster on gfx950, for tables whose
// windows miss some indices, than an LDS read plus a sparse global load.
template <int RB, int U, bool NT, bool GAS>
__device__ __forceinline__ void gather_vec_body(const GatherJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                                int njobs, int64_t ntiles, int tile_rows, int stream_win) {
  constexpr int V = 16 / RB;
  using R = typename RawVec<RB>::type;
  using IV = typename IdxVec<RB>::type;
  using RP = decltype(gas_ptr<GAS>((R*)nullptr));
  using CRP = decltype(gas_ptr<GAS>((const R*)nullptr));
  using CIVP = decltype(gas_ptr<GAS>((const IV*)nullptr));
  using VP = decltype(gas_ptr<GAS>((u32x4*)nullptr));
  extern __shared__ __align__(16) unsigned char s_dyn[];
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  int staged = -1;
  uint32_t lds_a = 0;  // LDS byte of the staged window's first row (0..15)
  const int bd = blockDim.x, tid = threadIdx.x;
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const auto src = gas_ptr<GAS>(jobs[j].src);
    const auto dst = gas_ptr<GAS>(jobs[j].dst);
    const auto idx = gas_ptr<GAS>(jobs[j].idx);
    const int64_t nrows = jobs[j].nrows;
    const int32_t win_lo = (int32_t)jobs[j].win_lo;
    const uint32_t win_rows = (uint32_t)jobs[j].win_rows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    // first row of the tile whose destination is 16-byte aligned
    const int64_t head = (int64_t)(((16 - ((uintptr_t)(dst + r0 * RB) & 15)) & 15) / RB);
    const int64_t a = min(r0 + head, r1);
    const int64_t ng = (r1 - a) / V;  // groups of the tile
    const int64_t tail0 = a + ng * V;
    const int nh = (int)(a - r0), ne = nh + (int)(r1 - tail0);  // rows outside the groups: < V before, < V after
    const bool use_win = win_rows > 0 && idx != nullptr;
    // this lane's row outside the groups (if any): its index is loaded first
    const bool has_edge = tid < ne;
    const int64_t er = tid < nh ? r0 + tid : tail0 + (tid - nh);
    int32_t esr = 0;
    if (has_edge) esr = idx ? idx[er] : (int32_t)er;
    // a row's value: from the staged window when it lies there, else global memory
    auto read_row = [&](int32_t sr) -> R {
      const uint32_t w = (uint32_t)(sr - win_lo);
      if constexpr (GAS) {
        if (use_win && w < win_rows) return *(const HX_L R*)(s_dyn + lds_a + w * (uint32_t)RB);
      } else {
        if (use_win && w < win_rows) return *reinterpret_cast<const R*>(s_dyn + lds_a + w * (uint32_t)RB);
      }
      return *reinterpret_cast<CRP>(src + (int64_t)sr * RB);
    };
    // the U index vectors of a lane for the pass starting at group g0
    // (lanes past the last group reload it: valid loads; stores are predicated)
    auto load_idx = [&](IV (&iv)[U], int64_t g0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = min(g0 + tid + (int64_t)u * bd, max(ng - 1, (int64_t)0));
        if (idx) {
          iv[u] = ldv<IV, NT>(reinterpret_cast<CIVP>(idx + a) + g);
        } else {
#pragma unroll
          for (int k = 0; k < V; ++k) iv[u][k] = (int)(a + g * V + k);
        }
      }
    };
    IV iv[U];
    if (ng > 0) load_idx(iv, 0);
    if (use_win) {
      if (staged != j) {
        if (staged >= 0) __syncthreads();  // every lane is done with the previous window
        const uintptr_t A = (uintptr_t)(src + (int64_t)win_lo * RB), B = A + (uintptr_t)win_rows * RB;
        const uintptr_t base = A & ~(uintptr_t)15;
        const uintptr_t A16 = (A + 15) & ~(uintptr_t)15, B16 = B & ~(uintptr_t)15;
        const int nv = B16 > A16 ? (int)((B16 - A16) >> 4) : 0;
        const auto gp = gas_ptr<GAS>(reinterpret_cast<const u32x4*>(A16));
        u32x4* sp = reinterpret_cast<u32x4*>(s_dyn + (A16 - base));
        // all of a lane's staging loads in flight together (an 80 KiB window
        // is at most 10 per lane with 512 lanes); streaming loads when the
        // schedule asks (a window is read once)
        constexpr int UW = 10;
        for (int i0 = tid; i0 < nv; i0 += bd * UW) {
          u32x4 w[UW];
          if (stream_win) {
#pragma unroll
            for (int u = 0; u < UW; ++u)
              if (i0 + u * bd < nv) w[u] = ldv<u32x4, true>(gp + i0 + u * bd);
          } else {
#pragma unroll
            for (int u = 0; u < UW; ++u)
              if (i0 + u * bd < nv) w[u] = gp[i0 + u * bd];
          }
#pragma unroll
          for (int u = 0; u < UW; ++u)
            if (i0 + u * bd < nv) sp[i0 + u * bd] = w[u];
        }
        // ragged ends: 4-byte words in [A, min(A16, B)) and [max(B16, A16), B)
        if (tid < 8) {
          const uintptr_t w = tid < 4 ? A + 4 * (uintptr_t)tid : max(B16, A16) + 4 * (uintptr_t)(tid - 4);
          const bool ok = tid < 4 ? (w < A16 && w < B) : (w < B);
          if (ok)
            *reinterpret_cast<unsigned int*>(s_dyn + (w - base)) =
                *gas_ptr<GAS>(reinterpret_cast<const unsigned int*>(w));
        }
        lds_a = (uint32_t)(A - base);
        staged = j;
      }
      __syncthreads();  // the window is visible to every lane
    }
    if (ng == 0 && has_edge) stv<R, NT>(reinterpret_cast<RP>(dst + er * RB), read_row(esr));
    // passes of U groups per lane (a tile is usually one pass); the next
    // pass's indices are loaded while this pass's rows are read and stored,
    // and the lane's row outside the groups goes with the first pass
    for (int64_t g0 = 0; g0 < ng; g0 += (int64_t)bd * U) {
      R v[U][V];
      R ev;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < V; ++k) v[u][k] = read_row(iv[u][k]);
      if (g0 == 0 && has_edge) ev = read_row(esr);
      const int64_t gn = g0 + (int64_t)bd * U;
      if (gn < ng) load_idx(iv, gn);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = g0 + tid + (int64_t)u * bd;
        if (g < ng) stv<u32x4, NT>(reinterpret_cast<VP>(dst + a * RB) + g, pack16<RB>(v[u]));
      }
      if (g0 == 0 && has_edge) stv<R, NT>(reinterpret_cast<RP>(dst + er * RB), ev);
    }
    signal_tile(jobs[j].ready, r1 - r0);
  }
}

// ---------------------------------------------------------------------------
// Push: for every source row r with slots idx[ptr[r] .. ptr[r+1]), read the
// row once and write it to each of its slots (the transpose form of the
// pull, so a row sent to several destinations is read from HBM once).
// Staged tiles run entry-parallel (LPR lanes per slot, U slots per lane);
// other tiles row-parallel.  Job fields: in = source rows, out = slots.
// ---------------------------------------------------------------------------
// LDS staging limits (kStageRows, kStageEntries) are declared with the
// schedules in common.h, where the default tile sizes use them.
constexpr int STAGE_ROWS = kStageRows;
constexpr int STAGE_ENTRIES = kStageEntries;

template <int VB, int NV, int LPR, int U, bool NT>
__device__ __forceinline__ void scatter_body(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                             const int2* __restrict__ te, int njobs, int64_t ntiles,
                                             int tile_rows, int nv_rt) {
  using V = typename RawVec<VB>::type;
  const int nv = NV > 0 ? NV : nv_rt;
  constexpr int NVPL = NV > 0 ? (NV + LPR - 1) / LPR : 1;
  const int lane_v = threadIdx.x % LPR;
  const int rsub = threadIdx.x / LPR;
  const int rows_per_pass = blockDim.x / LPR;
  __shared__ int32_t s_ptr[STAGE_ROWS + 1];
  __shared__ int32_t s_idx[STAGE_ENTRIES];
  __shared__ int16_t s_row[STAGE_ENTRIES];
  const bool stage_ptr = NV > 0 && tile_rows <= STAGE_ROWS;
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const HX_G char* __restrict__ in = (const HX_G char*)jobs[j].in;
    HX_G char* __restrict__ out = (HX_G char*)jobs[j].out;
    const HX_G int32_t* __restrict__ ptr = (const HX_G int32_t*)jobs[j].ptr;
    const HX_G int32_t* __restrict__ idx = (const HX_G int32_t*)jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const size_t rb = (size_t)nv * VB;
    if constexpr (NV > 0) {
      int32_t P0 = 0, ne = 0;
      bool stage_idx = false;
      if (stage_ptr) {
        // pointers and entry indices loaded together (the tile's entry
        // range is known)
        const int nt = (int)(r1 - r0);
        const int2 er = te[t];
        P0 = er.x;
        ne = er.y - P0;
        stage_idx = ne <= STAGE_ENTRIES;
        const int nl = max(nt + 1, stage_idx ? ne : 0);
        for (int i = threadIdx.x; i < nl; i += blockDim.x) {
          int32_t pv = 0, iv = 0;
          if (i <= nt) pv = ptr[r0 + i];
          if (stage_idx && i < ne) iv = ldv<int32_t, NT>(idx + P0 + i);
          if (i <= nt) s_ptr[i] = pv;
          if (stage_idx && i < ne) s_idx[i] = iv;
        }
        __syncthreads();
        if (stage_idx) {
          // the tile row of every entry, so the entries can be spread over
          // the lanes evenly whatever the rows' slot counts
          for (int i = threadIdx.x; i < nt; i += blockDim.x)
            for (int32_t e = s_ptr[i]; e < s_ptr[i + 1]; ++e) s_row[e - P0] = (int16_t)i;
          __syncthreads();
        }
      }
      if (stage_idx) {
        // entry-parallel: LPR lanes per entry, U entries per lane; entries of
        // one row sit next to each other, so its reads coalesce or hit L2
        for (int base = rsub; base < ne; base += rows_per_pass * U) {
          // lanes past the last entry re-read it (valid loads, no branch
          // between a lane's U loads); only the stores are predicated
          V v[U][NVPL];
          int32_t dsl[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = min(base + u * rows_per_pass, ne - 1);
            dsl[u] = s_idx[e];
            // (streaming loads under NT: the row's entries sit together, so
            // its reads coalesce in one pass rather than hit the cache later)
            const HX_G V* sp = reinterpret_cast<const HX_G V*>(in + (r0 + s_row[e]) * (int64_t)rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) v[u][k] = ldv<V, NT>(sp + vi);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (base + u * rows_per_pass < ne) {
              HX_G V* dp = reinterpret_cast<HX_G V*>(out + (int64_t)dsl[u] * rb);
#pragma unroll
              for (int k = 0; k < NVPL; ++k) {
                const int vi = lane_v + k * LPR;
                if (NV % LPR == 0 || vi < NV) stv<V, NT>(dp + vi, v[u][k]);
              }
            }
          }
        }
        __syncthreads();  // the next tile overwrites the staged indices
        continue;
      }
      for (int64_t base = r0 + rsub; base < r1; base += (int64_t)rows_per_pass * U) {
        int32_t a[U], len[U];
        int maxlen = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t r = base + (int64_t)u * rows_per_pass;
          a[u] = 0;
          len[u] = 0;
          if (r < r1) {
            if (stage_ptr) {
              a[u] = s_ptr[r - r0];
              len[u] = s_ptr[r - r0 + 1] - a[u];
            } else {
              a[u] = ptr[r];
              len[u] = ptr[r + 1] - a[u];
            }
          }
          maxlen = max(maxlen, len[u]);
        }
        V v[U][NVPL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (len[u] > 0) {
            const HX_G V* sp = reinterpret_cast<const HX_G V*>(in + (base + (int64_t)u * rows_per_pass) * rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) v[u][k] = ldv<V, NT>(sp + vi);
            }
          }
        }
        for (int d = 0; d < maxlen; ++d) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (d < len[u]) {
              const int32_t dst = ldv<int32_t, NT>(idx + a[u] + d);
              HX_G V* dp = reinterpret_cast<HX_G V*>(out + (int64_t)dst * rb);
#pragma unroll
              for (int k = 0; k < NVPL; ++k) {
                const int vi = lane_v + k * LPR;
                if (NV % LPR == 0 || vi < NV) stv<V, NT>(dp + vi, v[u][k]);
              }
            }
          }
        }
      }
      if (stage_ptr) __syncthreads();  // the next tile overwrites the staged pointers
    } else {
      for (int64_t r = r0 + rsub; r < r1; r += rows_per_pass) {
        const int32_t p0 = ptr[r], p1 = ptr[r + 1];
        const HX_G V* sp = reinterpret_cast<const HX_G V*>(in + r * rb);
        for (int vi = lane_v; vi < nv; vi += LPR) {
          if (p0 >= p1) break;
          const V v = sp[vi];
          for (int32_t e = p0; e < p1; ++e)
            stv<V, NT>(reinterpret_cast<HX_G V*>(out + (int64_t)idx[e] * rb) + vi, v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order segmented sum: out[r] = in[idx[ptr[r]]] + in[idx[ptr[r]+1]] + ...
// Additions in T, strictly in ascending position, the accumulator starting
// from the first term (a lone -0 stays -0); an empty segment stores +0.
// Staged tiles go chunk by chunk: the terms of a run of consecutive rows are
// gathered into LDS entry-parallel (U terms per lane in flight, however the
// segment lengths vary), then each row adds its own terms from LDS in order.
// Other tiles run row-parallel, term by term.
// ---------------------------------------------------------------------------
// Index staging (here and in the push form above): the tile's row pointers
// and, when they fit, its entry indices are loaded once into LDS with
// coalesced loads, so each row then costs one dependent global access (its
// terms) instead of three.

// Address of term t of a segmented sum: row t of the first input, or row
// t - split of the second one.
template <class CP>
__device__ __forceinline__ CP term_row(CP in, CP in2, int32_t split, int32_t t, size_t rb) {
  return t < split ? in + (int64_t)t * (int64_t)rb : in2 + (int64_t)(t - split) * (int64_t)rb;
}

template <class T, int VB, int NV, int LPR, int U, bool NT>
__device__ __forceinline__ void segsum_body(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                            const int2* __restrict__ te, int njobs, int64_t ntiles,
                                            int tile_rows, int nv_rt, int cap_terms) {
  using V = typename NumVec<T, VB>::type;
  const int nv = NV > 0 ? NV : nv_rt;
  constexpr int NVPL = NV > 0 ? (NV + LPR - 1) / LPR : 1;
  const int lane_v = threadIdx.x % LPR;
  const int rsub = threadIdx.x / LPR;
  const int rows_per_pass = blockDim.x / LPR;
  __shared__ int32_t s_ptr[STAGE_ROWS + 1];
  __shared__ int32_t s_idx[STAGE_ENTRIES];
  // term buffer: dynamic LDS of cap_terms rows (sized per launch table, so
  // small tiles leave room for more workgroups per CU)
  extern __shared__ __align__(16) unsigned char s_dyn[];
  V* const s_val = reinterpret_cast<V*>(s_dyn);
  // without a term buffer the tile runs row-parallel straight from global
  // memory (no staging, no barriers)
  const bool stage_ptr = NV > 0 && tile_rows <= STAGE_ROWS && cap_terms > 0;
  // (job pointers are accessed without an address space here: FLAT loads
  // measured faster than global ones for this body on gfx950)
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const char* __restrict__ in = jobs[j].in;
    // terms t >= split are rows t - split of the second input
    const int32_t split = jobs[j].split;
    const char* __restrict__ in2 = jobs[j].in2;
    char* __restrict__ out = jobs[j].out;
    const int32_t* __restrict__ ptr = jobs[j].ptr;
    const int32_t* __restrict__ idx = jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const size_t rb = (size_t)nv * VB;
    if constexpr (NV > 0) {
      // prologue: stage the tile's pointers and, when they fit, its entry
      // indices, both loaded together (the tile's entry range is known)
      int32_t P0 = 0;
      bool stage_idx = false;
      const int nt = (int)(r1 - r0);
      if (stage_ptr) {
        const int2 er = te[t];
        P0 = er.x;
        const int32_t ne = er.y - P0;
        stage_idx = ne <= STAGE_ENTRIES;
        const int nl = max(nt + 1, stage_idx ? ne : 0);
        for (int i = threadIdx.x; i < nl; i += blockDim.x) {
          int32_t pv = 0, iv = 0;
          if (i <= nt) pv = ptr[r0 + i];
          if (stage_idx && i < ne) iv = ldv<int32_t, NT>(idx + P0 + i);
          if (i <= nt) s_ptr[i] = pv;
          if (stage_idx && i < ne) s_idx[i] = iv;
        }
        __syncthreads();
      }
      if (stage_idx && cap_terms > 0) {
        // Chunks of consecutive rows whose terms fit in s_val: the terms are
        // loaded entry-parallel (U per lane, all in flight together, whatever
        // the segment lengths), then every row adds its own terms from LDS in
        // entry order and stores the sum.
        const int CAP = cap_terms;  // terms per chunk
        int ra = 0;
        while (ra < nt) {
          int lo = ra, hi = nt;  // last row boundary whose terms still fit
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_ptr[mid] - s_ptr[ra] <= CAP) lo = mid; else hi = mid - 1;
          }
          if (lo == ra) {
            // one row with more terms than fit: its first lane group sums it
            // straight from global memory, in order
            if (rsub == 0) {
              const int32_t a = s_ptr[ra] - P0, len = s_ptr[ra + 1] - s_ptr[ra];
              V* dp = reinterpret_cast<V*>(out + (r0 + ra) * (int64_t)rb);
#pragma unroll
              for (int k = 0; k < NVPL; ++k) {
                const int vi = lane_v + k * LPR;
                if (NV % LPR == 0 || vi < NV) {
                  V acc = reinterpret_cast<const V*>(term_row(in, in2, split, s_idx[a], rb))[vi];
                  for (int32_t d = 1; d < len; ++d)
                    acc = acc + reinterpret_cast<const V*>(term_row(in, in2, split, s_idx[a + d], rb))[vi];
                  stv<V, NT>(dp + vi, acc);
                }
              }
            }
            __syncthreads();
            ++ra;
            continue;
          }
          const int rq = lo;
          const int ea = s_ptr[ra] - P0, eb = s_ptr[rq] - P0;
          for (int base = ea + rsub; base < eb; base += rows_per_pass * U) {
            V v[U][NVPL];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int e = min(base + u * rows_per_pass, eb - 1);  // valid load, no branch
              // (streaming loads under NT: a term is read once)
              const V* sp = reinterpret_cast<const V*>(term_row(in, in2, split, s_idx[e], rb));
#pragma unroll
              for (int k = 0; k < NVPL; ++k) {
                const int vi = lane_v + k * LPR;
                if (NV % LPR == 0 || vi < NV) v[u][k] = ldv<V, NT>(sp + vi);
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int e = base + u * rows_per_pass;
              if (e < eb) {
#pragma unroll
                for (int k = 0; k < NVPL; ++k) {
                  const int vi = lane_v + k * LPR;
                  if (NV % LPR == 0 || vi < NV) s_val[(e - ea) * NV + vi] = v[u][k];
                }
              }
            }
          }
          __syncthreads();
          for (int r = ra + rsub; r < rq; r += rows_per_pass) {
            const int a = s_ptr[r] - P0 - ea, len = s_ptr[r + 1] - s_ptr[r];
            V* dp = reinterpret_cast<V*>(out + (r0 + r) * (int64_t)rb);
#pragma unroll
            for (int k = 0; k < NVPL; ++k) {
              const int vi = lane_v + k * LPR;
              if (NV % LPR == 0 || vi < NV) {
                V acc = (V)(T)0;
                if (len > 0) acc = s_val[a * NV + vi];
                for (int d = 1; d < len; ++d) acc = acc + s_val[(a + d) * NV + vi];
                stv<V, NT>(dp + vi, acc);
              }
            }
          }
          __syncthreads();  // s_val, s_ptr and s_idx are reused next
          ra = rq;
        }
        continue;
      }
      // row-parallel (no term buffer, or tiles whose entries were not
      // staged): one row per lane group, up to U of its terms in flight,
      // added in order
      for (int64_t r = r0 + rsub; r < r1; r += rows_per_pass) {
        int32_t a, len;
        if (stage_ptr) {
          a = s_ptr[r - r0];
          len = s_ptr[r - r0 + 1] - a;
        } else {
          a = ptr[r];
          len = ptr[r + 1] - a;
        }
        V acc[NVPL];
#pragma unroll
        for (int k = 0; k < NVPL; ++k) acc[k] = (V)(T)0;
        for (int32_t d0 = 0; d0 < len; d0 += U) {
          V v[U][NVPL];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (d0 + u < len) {
              const int32_t e = a + d0 + u;
              const int32_t src = stage_idx ? s_idx[e - P0] : ldv<int32_t, NT>(idx + e);
              const V* sp = reinterpret_cast<const V*>(term_row(in, in2, split, src, rb));
#pragma unroll
              for (int k = 0; k < NVPL; ++k) {
                const int vi = lane_v + k * LPR;
                if (NV % LPR == 0 || vi < NV) v[u][k] = sp[vi];
              }
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (d0 + u < len) {
#pragma unroll
              for (int k = 0; k < NVPL; ++k) acc[k] = (d0 + u == 0) ? v[u][k] : acc[k] + v[u][k];
            }
          }
        }
        V* dp = reinterpret_cast<V*>(out + r * (int64_t)rb);
#pragma unroll
        for (int k = 0; k < NVPL; ++k) {
          const int vi = lane_v + k * LPR;
          if (NV % LPR == 0 || vi < NV) stv<V, NT>(dp + vi, acc[k]);
        }
      }
      if (stage_ptr) __syncthreads();  // the next tile overwrites the staged indices
    } else {
      for (int64_t r = r0 + rsub; r < r1; r += rows_per_pass) {
        const int32_t p0 = ptr[r];
        const int32_t p1 = ptr[r + 1];
        V* dp = reinterpret_cast<V*>(out + r * rb);
        for (int vi = lane_v; vi < nv; vi += LPR) {
          V acc = (V)(T)0;
          for (int32_t e = p0; e < p1; ++e) {
            const V v = reinterpret_cast<const V*>(term_row(in, in2, split, ldv<int32_t, NT>(idx + e), rb))[vi];
            acc = (e == p0) ? v : acc + v;
          }
          stv<V, NT>(dp + vi, acc);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Segmented sum over a term window (short rows): a job whose terms mostly lie
// in [win_lo, win_lo + win_rows) of its term space (a rank's own send or
// forwarding slots, all inside one of the two inputs) copies those rows into
// dynamic LDS once per job; each row then adds its terms in order, reading
// in-window terms from LDS and the others (own-halo terms of a forwarder)
// from global memory.  Pointers and entry indices are staged per tile (tiles
// of at most 128 rows and 1536 entries; others read them from global
// memory).  No term staging buffer, so two such workgroups fit per CU.
// ---------------------------------------------------------------------------
template <class T, int VB, int NV, int LPR, int U, bool NT>
__device__ __forceinline__ void segsum_win_body(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                                int njobs, int64_t ntiles, int tile_rows, int nv_rt) {
  using V = typename NumVec<T, VB>::type;
  static_assert(NV > 0, "windowed segmented sums use fixed row shapes");
  constexpr int NVPL = (NV + LPR - 1) / LPR;
  (void)nv_rt;
  const int lane_v = threadIdx.x % LPR;
  const int rsub = threadIdx.x / LPR;
  const int rows_per_pass = blockDim.x / LPR;
  constexpr int WROWS = 128, WENTRIES = 1536;  // smaller staging: the window takes the LDS
  __shared__ int32_t s_ptr[WROWS + 1];
  __shared__ int32_t s_idx[WENTRIES];
  extern __shared__ __align__(16) unsigned char s_dyn[];
  V* __restrict__ s_win = reinterpret_cast<V*>(s_dyn);
  const bool stage_ptr = tile_rows <= WROWS;
  constexpr size_t rb = (size_t)NV * VB;
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  int staged = -1;
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const HX_G char* __restrict__ in = (const HX_G char*)jobs[j].in;
    const int32_t split = jobs[j].split;
    const HX_G char* __restrict__ in2 = (const HX_G char*)jobs[j].in2;
    HX_G char* __restrict__ out = (HX_G char*)jobs[j].out;
    const HX_G int32_t* __restrict__ ptr = (const HX_G int32_t*)jobs[j].ptr;
    const HX_G int32_t* __restrict__ idx = (const HX_G int32_t*)jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const int32_t win_lo = (int32_t)jobs[j].win_lo;
    const int32_t win_rows = (int32_t)jobs[j].win_rows;
    if (win_rows > 0 && staged != j) {
      __syncthreads();  // every lane is done with the previous window
      const HX_G V* __restrict__ wp = reinterpret_cast<const HX_G V*>(term_row(in, in2, split, win_lo, rb));
      const int nvec = win_rows * NV;
      constexpr int UW = 8;
      for (int i0 = threadIdx.x; i0 < nvec; i0 += blockDim.x * UW) {
        V w[UW];
#pragma unroll
        for (int u = 0; u < UW; ++u) {
          const int i = i0 + u * blockDim.x;
          if (i < nvec) w[u] = wp[i];
        }
#pragma unroll
        for (int u = 0; u < UW; ++u) {
          const int i = i0 + u * blockDim.x;
          if (i < nvec) s_win[i] = w[u];
        }
      }
      staged = j;
    }
    int32_t P0 = 0;
    bool stage_idx = false;
    const int nt = (int)(r1 - r0);
    if (stage_ptr) {
      for (int i = threadIdx.x; i <= nt; i += blockDim.x) s_ptr[i] = ptr[r0 + i];
      __syncthreads();
      P0 = s_ptr[0];
      const int32_t ne = s_ptr[nt] - P0;
      stage_idx = ne <= WENTRIES;
      if (stage_idx)
        for (int i = threadIdx.x; i < ne; i += blockDim.x) s_idx[i] = ldv<int32_t, NT>(idx + P0 + i);
    }
    __syncthreads();  // staged window, pointers and indices visible to all lanes
    for (int64_t base = r0 + rsub; base < r1; base += (int64_t)rows_per_pass * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = base + (int64_t)u * rows_per_pass;
        if (r >= r1) break;
        const int32_t a = stage_ptr ? s_ptr[r - r0] : ptr[r];
        const int32_t len = (stage_ptr ? s_ptr[r - r0 + 1] : ptr[r + 1]) - a;
        V acc[NVPL];
#pragma unroll
        for (int k = 0; k < NVPL; ++k) acc[k] = (V)(T)0;
        for (int32_t d = 0; d < len; ++d) {
          const int32_t tm = stage_idx ? s_idx[a + d - P0] : ldv<int32_t, NT>(idx + a + d);
          const uint32_t wr = (uint32_t)(tm - win_lo);
#pragma unroll
          for (int k = 0; k < NVPL; ++k) {
            const int vi = lane_v + k * LPR;
            if (NV % LPR == 0 || vi < NV) {
              V v;
              if (wr < (uint32_t)win_rows) v = s_win[(int64_t)wr * NV + vi];
              else v = reinterpret_cast<const HX_G V*>(term_row(in, in2, split, tm, rb))[vi];
              acc[k] = d == 0 ? v : acc[k] + v;
            }
          }
        }
        HX_G V* dp = reinterpret_cast<HX_G V*>(out + r * (int64_t)rb);
#pragma unroll
        for (int k = 0; k < NVPL; ++k) {
          const int vi = lane_v + k * LPR;
          if (NV % LPR == 0 || vi < NV) stv<V, NT>(dp + vi, acc[k]);
        }
      }
    }
    __syncthreads();  // the next tile overwrites the staged pointers and indices
  }
}

// ---------------------------------------------------------------------------
// Fixed-order segmented sum of short rows (one FP32 or FP64 value per row),
// one row per lane: a pass gives each lane U rows, lane-strided, so that the
// rows' pointer loads, their entries' loads and the stores are coalesced
// across the wavefront.  The passes are pipelined: row pointers two passes
// ahead, the entries of every row's first D terms one pass ahead (all
// together; deeper terms one after another), this pass's values issued before
// those prefetches; a term inside the job's LDS window
// (terms [win_lo, win_lo + win_rows), all in one input, staged once per job
// with every load in flight at once) is read from LDS, any other from global
// memory.  Per row the adds run in entry order from the first term (a lone
// -0 stays -0); an empty row stores +0.
// ---------------------------------------------------------------------------
template <class T, int U, int D, bool NT>
__device__ __forceinline__ void segsum_vec_body(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts,
                                                int njobs, int64_t ntiles, int tile_rows) {
  constexpr int RB = (int)sizeof(T);
  extern __shared__ __align__(16) unsigned char s_dyn[];
  int64_t t0, t1;
  tile_range(ntiles, &t0, &t1);
  if (t0 >= t1) return;
  int j = find_job(ts, njobs, t0);
  int staged = -1;
  uint32_t lds_a = 0;  // LDS byte of the staged window's first term (0..15)
  const int bd = blockDim.x, tid = threadIdx.x;
  const int64_t step = (int64_t)bd * U;  // rows per pass
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= ts[j + 1]) ++j;
    const HX_G char* __restrict__ in = (const HX_G char*)jobs[j].in;
    const HX_G char* __restrict__ in2 = (const HX_G char*)jobs[j].in2;
    const int32_t split = jobs[j].split;
    HX_G char* __restrict__ out = (HX_G char*)jobs[j].out;
    const HX_G int32_t* __restrict__ ptr = (const HX_G int32_t*)jobs[j].ptr;
    const HX_G int32_t* __restrict__ idx = (const HX_G int32_t*)jobs[j].idx;
    const int64_t nrows = jobs[j].nrows;
    const int32_t win_lo = (int32_t)jobs[j].win_lo;
    const uint32_t win_rows = (uint32_t)jobs[j].win_rows;
    const int64_t r0 = (t - ts[j]) * (int64_t)tile_rows;
    const int64_t r1 = min(r0 + (int64_t)tile_rows, nrows);
    const bool use_win = win_rows > 0;
    auto term = [&](int32_t tm) -> T {
      const uint32_t w = (uint32_t)(tm - win_lo);
      if (use_win && w < win_rows) return *(const HX_L T*)(s_dyn + lds_a + w * (uint32_t)RB);
      return *reinterpret_cast<const HX_G T*>(term_row(in, in2, split, tm, RB));
    };
    // row pointers of a lane's U rows of the pass starting at row base
    // (lanes past the tile's end reload its last row: valid loads)
    auto load_ptr = [&](int64_t base, int32_t (&xa)[U], int32_t (&xl)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = min(base + tid + (int64_t)u * bd, r1 - 1);
        xa[u] = ptr[r];
        xl[u] = ptr[r + 1];
      }
    };
    // entries of the first D terms of those rows (xl: row lengths)
    auto load_idx = [&](const int32_t (&xa)[U], const int32_t (&xl)[U], int32_t (&xe)[U][D]) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int d = 0; d < D; ++d) xe[u][d] = xl[u] > d ? ldv<int32_t, NT>(idx + xa[u] + d) : 0;
    };
    auto lengths = [&](int32_t (&xa)[U], int32_t (&xl)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) xl[u] -= xa[u];
    };
    // pipeline: pointers two passes ahead, entries one pass ahead
    int32_t a[U], len[U], an[U], ln[U];
    int32_t e[U][D];
    load_ptr(r0, a, len);
    if (r0 + step < r1) load_ptr(r0 + step, an, ln);
    if (use_win) {
      if (staged != j) {
        if (staged >= 0) __syncthreads();  // every lane is done with the previous window
        const uintptr_t A = (uintptr_t)term_row(in, in2, split, win_lo, RB), B = A + (uintptr_t)win_rows * RB;
        const uintptr_t base = A & ~(uintptr_t)15;
        const uintptr_t A16 = (A + 15) & ~(uintptr_t)15, B16 = B & ~(uintptr_t)15;
        const int nv = B16 > A16 ? (int)((B16 - A16) >> 4) : 0;
        const HX_G u32x4* __restrict__ gp = reinterpret_cast<const HX_G u32x4*>(A16);
        u32x4* sp = reinterpret_cast<u32x4*>(s_dyn + (A16 - base));
        constexpr int UW = 10;  // all of a lane's staging loads in flight together (80 KiB, 512 lanes)
        for (int i0 = tid; i0 < nv; i0 += bd * UW) {
          u32x4 w[UW];
#pragma unroll
          for (int u = 0; u < UW; ++u)
            if (i0 + u * bd < nv) w[u] = gp[i0 + u * bd];
#pragma unroll
          for (int u = 0; u < UW; ++u)
            if (i0 + u * bd < nv) sp[i0 + u * bd] = w[u];
        }
        // ragged ends: 4-byte words in [A, min(A16, B)) and [max(B16, A16), B)
        if (tid < 8) {
          const uintptr_t w = tid < 4 ? A + 4 * (uintptr_t)tid : max(B16, A16) + 4 * (uintptr_t)(tid - 4);
          const bool ok = tid < 4 ? (w < A16 && w < B) : (w < B);
          if (ok) *reinterpret_cast<unsigned int*>(s_dyn + (w - base)) = *reinterpret_cast<const HX_G unsigned int*>(w);
        }
        lds_a = (uint32_t)(A - base);
        staged = j;
      }
      __syncthreads();  // the window is visible to every lane
    }
    lengths(a, len);
    load_idx(a, len, e);
    for (int64_t base = r0; base < r1; base += step) {
      // this pass's values first, then the next passes' prefetches (so that
      // waiting for the values never waits for the prefetches)
      T v[U][D];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int d = 0; d < D; ++d) v[u][d] = len[u] > d ? term(e[u][d]) : (T)0;
      __builtin_amdgcn_sched_barrier(0);
      const bool more = base + step < r1;
      int32_t a1[U], l1[U], e1[U][D];
      if (more) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a1[u] = an[u];
          l1[u] = ln[u] - an[u];
        }
        load_idx(a1, l1, e1);
        if (base + 2 * step < r1) load_ptr(base + 2 * step, an, ln);
      }
      __builtin_amdgcn_sched_barrier(0);
      T acc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc[u] = v[u][0];
#pragma unroll
        for (int d = 1; d < D; ++d)
          if (len[u] > d) acc[u] = acc[u] + v[u][d];
        for (int32_t d = D; d < len[u]; ++d) acc[u] = acc[u] + term(ldv<int32_t, NT>(idx + a[u] + d));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = base + tid + (int64_t)u * bd;
        if (r < r1) stv<T, NT>(reinterpret_cast<HX_G T*>(out + r * RB), acc[u]);
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a[u] = a1[u];
          len[u] = l1[u];
#pragma unroll
          for (int d = 0; d < D; ++d) e[u][d] = e1[u][d];
        }
      }
    }
  }
}

}  // namespace kern

// Launchers implemented in the move_*.hip translation units.
void launch_gather_kernels(const LaunchTable& t, hipStream_t s);
void launch_scatter_kernels(const LaunchTable& t, hipStream_t s);
void launch_segsum_kernels(const LaunchTable& t, hipStream_t s);

}  // namespace hx
