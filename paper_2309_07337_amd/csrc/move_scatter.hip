// Push-form pack: each source row is read once and written to every send
// slot it feeds (walks the transpose of the pack map).
#include "move_launch.h"

namespace hx {
namespace kern {
namespace {

#define HX_SCATTER_KERNEL(NAME)                                                                    \
  template <int VB, int NV, int LPR, int U, bool NT>                                               \
  __global__ void __launch_bounds__(512)                                                           \
      NAME(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,          \
           const int2* __restrict__ te, int64_t ntiles, int tile_rows, int nv_rt) {                \
    scatter_body<VB, NV, LPR, U, NT>(jobs, ts, te, njobs, ntiles, tile_rows, nv_rt);               \
  }                                                                                                \
  struct NAME##_go {                                                                               \
    template <int VB, int NV, int LPR, int U, bool NT>                                             \
    static void go(const LaunchTable& t, hipStream_t s, int nv) {                                  \
      hipLaunchKernelGGL((NAME<VB, NV, LPR, U, NT>), dim3(t.grid), dim3(t.sched.block_threads), 0, \
                         s, t.jobs.as<SegSumJob>(), t.tile_start.as<int64_t>(), t.njobs,           \
                         t.tile_terms.as<int2>(), t.ntiles, t.sched.tile_rows, nv);                \
    }                                                                                              \
  };
HX_SCATTER_KERNEL(k_pack_push)
#undef HX_SCATTER_KERNEL

}  // namespace
}  // namespace kern

void launch_scatter_kernels(const LaunchTable& t, hipStream_t s) { kern::by_vec<kern::k_pack_push_go>(t, s); }

}  // namespace hx
