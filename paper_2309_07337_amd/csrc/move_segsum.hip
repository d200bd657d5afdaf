// Fixed-order segmented sums, instantiated for FP32 and FP64 rows: the owner
// sums (the backward of the pack and of the exchange) and the staged
// backward's forwarder sums.  One symbol per step (and a *_win form with an
// LDS term window, a *_vec form for rows of one value), same bodies.
#include "move_launch.h"

namespace hx {
namespace kern {
namespace {

#define HX_SEGSUM_KERNEL(NAME)                                                                       \
  template <class T, int VB, int NV, int LPR, int U, bool NT>                                        \
  __global__ void __launch_bounds__(1024)                                                            \
      NAME(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,            \
           const int2* __restrict__ te, int64_t ntiles, int tile_rows, int nv_rt, int cap_terms) {   \
    segsum_body<T, VB, NV, LPR, U, NT>(jobs, ts, te, njobs, ntiles, tile_rows, nv_rt, cap_terms);    \
  }                                                                                                  \
  template <class T, int VB, int NV, int LPR, int U, bool NT>                                        \
  __global__ void __launch_bounds__(512)                                                             \
      NAME##_win(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,      \
                 int64_t ntiles, int tile_rows, int nv_rt) {                                         \
    segsum_win_body<T, VB, NV, LPR, U, NT>(jobs, ts, njobs, ntiles, tile_rows, nv_rt);               \
  }                                                                                                  \
  template <class T, int U, int D, bool NT>                                                          \
  __global__ void __launch_bounds__(1024)                                                            \
      NAME##_vec(const SegSumJob* __restrict__ jobs, const int64_t* __restrict__ ts, int njobs,      \
                 int64_t ntiles, int tile_rows) {                                                    \
    segsum_vec_body<T, U, D, NT>(jobs, ts, njobs, ntiles, tile_rows);                                \
  }                                                                                                  \
  struct NAME##_vgo {                                                                                \
    template <class T, int U, int D, bool NT>                                                        \
    static void go(const LaunchTable& t, hipStream_t s) {                                            \
      hipLaunchKernelGGL((NAME##_vec<T, U, D, NT>), dim3(t.grid), dim3(t.sched.block_threads),       \
                         (unsigned)t.win_bytes, s, t.jobs.as<SegSumJob>(), t.tile_start.as<int64_t>(), \
                         t.njobs, t.ntiles, t.sched.tile_rows);                                      \
    }                                                                                                \
  };                                                                                                 \
  template <class T>                                                                                 \
  struct NAME##_go {                                                                                 \
    template <int VB, int NV, int LPR, int U, bool NT>                                               \
    static void go(const LaunchTable& t, hipStream_t s, int nv) {                                    \
      if constexpr ((size_t)VB < sizeof(T)) {                                                        \
        (void)t; (void)s; (void)nv; /* excluded when the table is built */                           \
      } else {                                                                                       \
        if constexpr (NV > 0 && NV * VB <= 64) { /* term windows pay off for short rows only */    \
          if (t.win_bytes > 0) {                                                                     \
            hipLaunchKernelGGL((NAME##_win<T, VB, NV, LPR, U, NT>), dim3(t.grid),                    \
                               dim3(t.sched.block_threads), (unsigned)t.win_bytes, s,                \
                               t.jobs.as<SegSumJob>(), t.tile_start.as<int64_t>(), t.njobs,          \
                               t.ntiles, t.sched.tile_rows, nv);                                     \
            return;                                                                                  \
          }                                                                                          \
        }                                                                                            \
        const int vb = NV > 0 ? t.val_bytes : 0; /* term buffer (fixed shapes only) */               \
        hipLaunchKernelGGL((NAME<T, VB, NV, LPR, U, NT>), dim3(t.grid), dim3(t.sched.block_threads), \
                           (unsigned)vb, s, t.jobs.as<SegSumJob>(), t.tile_start.as<int64_t>(),      \
                           t.njobs, t.tile_terms.as<int2>(), t.ntiles, t.sched.tile_rows, nv,        \
                           vb / (NV > 0 ? NV * VB : 1));                                             \
      }                                                                                              \
    }                                                                                                \
  };
HX_SEGSUM_KERNEL(k_segsum)
HX_SEGSUM_KERNEL(k_segsum_fwd)
#undef HX_SEGSUM_KERNEL

// One value per row (t.vec16): rows per lane 1, or 2 for unroll >= 2 (more
// would spill registers); terms loaded together per row: 4, or 16 (one row
// per lane) for tables whose rows average more than three terms (t.vec_depth).
template <class F, class T, bool NT>
void vec_launch_nt(const LaunchTable& t, hipStream_t s) {
  if (t.vec_depth > 4) return F::template go<T, 1, 16, NT>(t, s);
  if (unroll_bucket(t.sched.unroll) == 1) F::template go<T, 1, 4, NT>(t, s);
  else F::template go<T, 2, 4, NT>(t, s);
}

template <class F, class T>
void vec_launch(const LaunchTable& t, hipStream_t s) {
  if (t.sched.nontemporal) vec_launch_nt<F, T, true>(t, s);
  else vec_launch_nt<F, T, false>(t, s);
}

}  // namespace
}  // namespace kern

void launch_segsum_kernels(const LaunchTable& t, hipStream_t s) {
  using namespace kern;
  const bool fwd = t.tag == TAG_FWD_SUM;
  if (t.vec16) {
    if (t.dtype == HX_F32) {
      if (fwd) vec_launch<k_segsum_fwd_vgo, float>(t, s);
      else vec_launch<k_segsum_vgo, float>(t, s);
    } else {
      if (fwd) vec_launch<k_segsum_fwd_vgo, double>(t, s);
      else vec_launch<k_segsum_vgo, double>(t, s);
    }
    return;
  }
  if (t.dtype == HX_F32) {
    if (fwd) by_vec<k_segsum_fwd_go<float>>(t, s);
    else by_vec<k_segsum_go<float>>(t, s);
  } else {
    if (fwd) by_vec<k_segsum_fwd_go<double>>(t, s);
    else by_vec<k_segsum_go<double>>(t, s);
  }
}

}  // namespace hx
