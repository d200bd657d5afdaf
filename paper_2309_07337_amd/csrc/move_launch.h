// Shape / unroll / hint dispatch shared by the move_*.hip launch units.
#pragma once

#include "move_kernels.h"

namespace hx {
namespace kern {

// Rows per lane in flight: 1, 2 or 4 (0 = 4).  Measured on gfx950: more
// independent random row loads per lane than 4 only lengthen memory queues.
inline int unroll_bucket(int u) {
  if (u <= 0) return 4;
  if (u == 1) return 1;
  if (u == 2) return 2;
  return 4;
}

// Calls F::template go<VB, NV, LPR, U, NT>(t, s, nv) for the table's shape.
// Fixed shapes (one 16/8/4-byte vector per lane, LPR lanes per row) take
// U in {1, 2, 4}; other row sizes use the runtime-size loop with U = 1.
template <class F, int VB, int NV, int LPR>
void by_unroll(const LaunchTable& t, hipStream_t s, int nv) {
  const bool nt = t.sched.nontemporal != 0;
  switch (unroll_bucket(t.sched.unroll)) {
    case 1:
      if (nt) F::template go<VB, NV, LPR, 1, true>(t, s, nv);
      else F::template go<VB, NV, LPR, 1, false>(t, s, nv);
      break;
    case 2:
      if (nt) F::template go<VB, NV, LPR, 2, true>(t, s, nv);
      else F::template go<VB, NV, LPR, 2, false>(t, s, nv);
      break;
    default:
      if (nt) F::template go<VB, NV, LPR, 4, true>(t, s, nv);
      else F::template go<VB, NV, LPR, 4, false>(t, s, nv);
      break;
  }
}

template <class F, int VB, int LPR>
void generic(const LaunchTable& t, hipStream_t s, int nv) {
  if (t.sched.nontemporal) F::template go<VB, 0, LPR, 1, true>(t, s, nv);
  else F::template go<VB, 0, LPR, 1, false>(t, s, nv);
}

template <class F, int VB>
void by_shape(const LaunchTable& t, hipStream_t s) {
  const int nv = t.row_bytes / VB;
  if constexpr (VB == 16) {
    switch (nv) {
      case 1: return by_unroll<F, 16, 1, 1>(t, s, nv);
      case 2: return by_unroll<F, 16, 2, 2>(t, s, nv);
      case 4: return by_unroll<F, 16, 4, 4>(t, s, nv);
      case 8: return by_unroll<F, 16, 8, 8>(t, s, nv);
      case 16: return by_unroll<F, 16, 16, 16>(t, s, nv);
      case 32: return by_unroll<F, 16, 32, 32>(t, s, nv);
      case 64: return by_unroll<F, 16, 64, 64>(t, s, nv);
      default: break;
    }
  } else if constexpr (VB == 8) {
    if (nv == 1) return by_unroll<F, 8, 1, 1>(t, s, nv);
    if (nv == 3) return by_unroll<F, 8, 3, 1>(t, s, nv);
  } else {
    if (nv == 1) return by_unroll<F, 4, 1, 1>(t, s, nv);
  }
  if (nv >= 64) return generic<F, VB, 64>(t, s, nv);
  if (nv >= 16) return generic<F, VB, 16>(t, s, nv);
  return generic<F, VB, 1>(t, s, nv);
}

template <class F>
void by_vec(const LaunchTable& t, hipStream_t s) {
  if (t.vec_bytes == 16) by_shape<F, 16>(t, s);
  else if (t.vec_bytes == 8) by_shape<F, 8>(t, s);
  else by_shape<F, 4>(t, s);
}

}  // namespace kern
}  // namespace hx
