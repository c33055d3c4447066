// Expansions at a run-time order q <= P, for interaction lists whose entries
// carry their own order (error-bound acceptance). The moments of a cell are
// stored to order P in slot order (by total order first), so the moments of
// order <= q are a prefix of them.
#pragma once
#include "common.h"
#include "generated/expansions.h"

namespace hot {

#define HOT_Q_CASES(CALL) \
  CALL(0) CALL(1) CALL(2) CALL(3) CALL(4) CALL(5) CALL(6) CALL(7) CALL(8)

template <int P, typename T, bool POT, bool K1 = false>
__device__ __forceinline__ void expansion_fwd_q(int q, T X, T Y, T Z, T e2,
                                                const T* __restrict__ M, T& ax, T& ay, T& az,
                                                T& ph) {
  switch (q) {
#define HOT_CASE(Q)                                                     \
  case Q:                                                               \
    if constexpr (Q <= P) expansion_fwd<Q, T, POT, K1>(X, Y, Z, e2, M, ax, ay, az, ph); \
    break;
    HOT_Q_CASES(HOT_CASE)
#undef HOT_CASE
    default:
      break;
  }
}

template <int P, typename T, bool K1 = false>
__device__ __forceinline__ void expansion_sink_adj_q(int q, T X, T Y, T Z, T e2,
                                                     const T* __restrict__ M, T bx, T by, T bz,
                                                     T& gx, T& gy, T& gz) {
  switch (q) {
#define HOT_CASE(Q)                                                                   \
  case Q:                                                                             \
    if constexpr (Q <= P) expansion_sink_adj<Q, T, K1>(X, Y, Z, e2, M, bx, by, bz, gx, gy, gz); \
    break;
    HOT_Q_CASES(HOT_CASE)
#undef HOT_CASE
    default:
      break;
  }
}

#undef HOT_Q_CASES

}  // namespace hot
