// Pull-form row gathers: pack (Start), redistribution pack and unpack (Wait),
// and the simulated transfer; short rows also in 16-byte groups per lane
// (the *_vec symbols).  One kernel symbol per phase (same body), so
// profiles attribute time to each phase separately.
#include "move_launch.h"

namespace hx {
namespace kern {
namespace {

#define HX_GATHER_KERNEL(NAME)                                                                 \
  template <int VB, int NV, int LPR, int U, bool NT>                                           \
  __global__ void __launch_bounds__(1024)                                                      \
      NAME(const GatherJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,      \
           int64_t ntiles, int tile_rows, int nv_rt, int use_win) {                            \
    gather_body<VB, NV, LPR, U, NT>(jobs, ts, njobs, ntiles, tile_rows, nv_rt, use_win);       \
  }                                                                                            \
  template <int RB, int U, bool NT, bool GAS>                                                  \
  __global__ void __launch_bounds__(1024)                                                      \
      NAME##_vec(const GatherJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs, \
                 int64_t ntiles, int tile_rows, int stream_win) {                              \
    gather_vec_body<RB, U, NT, GAS>(jobs, ts, njobs, ntiles, tile_rows, stream_win);           \
  }                                                                                            \
  struct NAME##_vgo {                                                                          \
    template <int RB, int U, bool NT>                                                          \
    static void go(const LaunchTable& t, hipStream_t s) {                                      \
      const int sw = t.sched.nontemporal >= 2 ? 1 : 0; /* streaming window staging */          \
      if (t.partial_win)                                                                       \
        hipLaunchKernelGGL((NAME##_vec<RB, U, NT, false>), dim3(t.grid), dim3(t.sched.block_threads), \
                           (unsigned)t.win_bytes, s, t.jobs.as<GatherJob>(),                   \
                           t.tile_start.as<int64_t>(), t.njobs, t.ntiles, t.sched.tile_rows, sw); \
      else                                                                                     \
        hipLaunchKernelGGL((NAME##_vec<RB, U, NT, true>), dim3(t.grid), dim3(t.sched.block_threads), \
                           (unsigned)t.win_bytes, s, t.jobs.as<GatherJob>(),                   \
                           t.tile_start.as<int64_t>(), t.njobs, t.ntiles, t.sched.tile_rows, sw); \
    }                                                                                          \
  };                                                                                           \
  struct NAME##_go {                                                                           \
    template <int VB, int NV, int LPR, int U, bool NT>                                         \
    static void go(const LaunchTable& t, hipStream_t s, int nv) {                              \
      hipLaunchKernelGGL((NAME<VB, NV, LPR, U, NT>), dim3(t.grid), dim3(t.sched.block_threads), \
                         (unsigned)t.win_bytes, s, t.jobs.as<GatherJob>(),                     \
                         t.tile_start.as<int64_t>(), t.njobs, t.ntiles, t.sched.tile_rows, nv, \
                         t.win_bytes > 0 ? 1 : 0);                                             \
    }                                                                                          \
  };
HX_GATHER_KERNEL(k_pack)
HX_GATHER_KERNEL(k_redist)
HX_GATHER_KERNEL(k_unpack)
HX_GATHER_KERNEL(k_transfer)
#undef HX_GATHER_KERNEL

// The simulated transfer is not tuned: one fixed variant per shape.
struct transfer_fixed {
  template <int VB, int NV, int LPR, int U, bool NT>
  static void go(const LaunchTable& t, hipStream_t s, int nv) {
    k_transfer_go::go<VB, NV, LPR, (NV > 0 ? 4 : 1), false>(t, s, nv);
  }
};

template <int VB>
void transfer_shape(const LaunchTable& t, hipStream_t s) {
  const int nv = t.row_bytes / VB;
  if constexpr (VB == 16) {
    if (nv == 8) return transfer_fixed::go<16, 8, 8, 4, false>(t, s, nv);
    if (nv == 16) return transfer_fixed::go<16, 16, 16, 4, false>(t, s, nv);
    if (nv == 1) return transfer_fixed::go<16, 1, 1, 4, false>(t, s, nv);
  } else if constexpr (VB == 8) {
    if (nv == 1) return transfer_fixed::go<8, 1, 1, 4, false>(t, s, nv);
  } else {
    if (nv == 1) return transfer_fixed::go<4, 1, 1, 4, false>(t, s, nv);
  }
  if (nv >= 16) return transfer_fixed::go<VB, 0, 16, 1, false>(t, s, nv);
  return transfer_fixed::go<VB, 0, 1, 1, false>(t, s, nv);
}

// Short rows, 16 bytes per lane (the table builder set t.vec16): rows of 4
// or 8 bytes, U groups per lane in {1, 2, 4} (more would spill registers).
template <class F, int RB>
void vec_by_unroll(const LaunchTable& t, hipStream_t s) {
  const bool nt = t.sched.nontemporal != 0;
  switch (unroll_bucket(t.sched.unroll)) {
    case 1: nt ? F::template go<RB, 1, true>(t, s) : F::template go<RB, 1, false>(t, s); break;
    case 2: nt ? F::template go<RB, 2, true>(t, s) : F::template go<RB, 2, false>(t, s); break;
    default: nt ? F::template go<RB, 4, true>(t, s) : F::template go<RB, 4, false>(t, s); break;
  }
}

template <class F>
void vec_launch(const LaunchTable& t, hipStream_t s) {
  if (t.row_bytes == 8) vec_by_unroll<F, 8>(t, s);
  else vec_by_unroll<F, 4>(t, s);
}

}  // namespace
}  // namespace kern

void launch_gather_kernels(const LaunchTable& t, hipStream_t s) {
  using namespace kern;
  if (t.vec16) {
    switch (t.tag) {
      case TAG_PACK: vec_launch<k_pack_vgo>(t, s); return;
      case TAG_REDIST: vec_launch<k_redist_vgo>(t, s); return;
      case TAG_UNPACK: vec_launch<k_unpack_vgo>(t, s); return;
      default: break;  // the simulated transfer keeps its fixed variants
    }
  }
  switch (t.tag) {
    case TAG_PACK: by_vec<k_pack_go>(t, s); break;
    case TAG_REDIST: by_vec<k_redist_go>(t, s); break;
    case TAG_UNPACK: by_vec<k_unpack_go>(t, s); break;
    default:
      if (t.vec_bytes == 16) transfer_shape<16>(t, s);
      else if (t.vec_bytes == 8) transfer_shape<8>(t, s);
      else transfer_shape<4>(t, s);
      break;
  }
}

}  // namespace hx
