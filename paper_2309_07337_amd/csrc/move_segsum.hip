// Fixed-order segmented sum (the backward of the pack and of the whole
// exchange), instantiated for FP32 and FP64 rows.
#include "move_launch.h"

namespace hx {
namespace kern {
namespace {

template <class T, int VB, int NV, int LPR, int U, bool NT>
__global__ void __launch_bounds__(512)
    k_segsum(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs, int64_t ntiles,
             int tile_rows, int nv_rt) {
  segsum_body<T, VB, NV, LPR, U, NT>(jobs, ts, njobs, ntiles, tile_rows, nv_rt);
}

template <class T>
struct segsum_go {
  template <int VB, int NV, int LPR, int U, bool NT>
  static void go(const LaunchTable& t, hipStream_t s, int nv) {
    if constexpr ((size_t)VB < sizeof(T)) {
      (void)t; (void)s; (void)nv;  // excluded when the table is built
    } else {
      hipLaunchKernelGGL((k_segsum<T, VB, NV, LPR, U, NT>), dim3(t.grid), dim3(t.sched.block_threads), 0, s,
                         t.jobs.as<SegSumJob>(), t.tile_start.as<int64_t>(), t.njobs, t.ntiles, t.sched.tile_rows,
                         nv);
    }
  }
};

}  // namespace
}  // namespace kern

void launch_segsum_kernels(const LaunchTable& t, hipStream_t s) {
  if (t.dtype == HX_F32) kern::by_vec<kern::segsum_go<float>>(t, s);
  else kern::by_vec<kern::segsum_go<double>>(t, s);
}

}  // namespace hx
