// Device helpers shared by the force and adjoint kernels.
#pragma once
#include "common.h"

namespace hot {

// Multi-index (a, b, c) of every moment slot up to order 8 and the expansion
// weight (-1)^|alpha| / alpha! of each.
struct AlphaTable {
  int8_t a[nm(kMaxP)], b[nm(kMaxP)], c[nm(kMaxP)];
  double w[nm(kMaxP)];
};

constexpr AlphaTable make_alpha_table() {
  AlphaTable t{};
  int s = 0;
  for (int n = 0; n <= kMaxP; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        const int c = n - a - b;
        double f = 1.0;
        for (int k = 2; k <= a; ++k) f *= k;
        for (int k = 2; k <= b; ++k) f *= k;
        for (int k = 2; k <= c; ++k) f *= k;
        t.a[s] = (int8_t)a;
        t.b[s] = (int8_t)b;
        t.c[s] = (int8_t)c;
        t.w[s] = ((n & 1) ? -1.0 : 1.0) / f;
        ++s;
      }
  return t;
}

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
};
template <>
struct Vec4<double> {
  using type = double4;
};
template <typename T>
using V4 = typename Vec4<T>::type;

// Dehnen's K1 kernel inside its radius eps (Force Smoothing section), as
// polynomials in v = 1 - r^2 / eps^2 with positive coefficients (no
// cancellation near the edge, v -> 0, where they meet the Newtonian values):
// the pair force is m r eps^-3 k1_force(v), the potential -m eps^-1 k1_pot(v),
// and the Hessian's r r^T coefficient -eps^-5 k1_hess(v).
template <typename T>
__device__ __forceinline__ T k1_force(T v) {
  return hot_fma(v, hot_fma(v, hot_fma(v, T(12.03125), T(1.875)), T(1.5)), T(1));
}
template <typename T>
__device__ __forceinline__ T k1_pot(T v) {
  return hot_fma(v, hot_fma(v, hot_fma(v, hot_fma(v, T(1.50390625), T(0.3125)), T(0.375)),
                            T(0.5)),
                 T(1));
}
template <typename T>
__device__ __forceinline__ T k1_hess(T v) {
  return hot_fma(v, hot_fma(v, T(72.1875), T(7.5)), T(3));
}

template <typename T>
__device__ __forceinline__ void kahan_add(T& s, T& c, T x) {
  const T y = x - c;
  const T t = s + y;
  c = (t - s) - y;
  s = t;
}

// Offsets of every particle (sorted order) from its group's centre, and mass.
// mdiff (nullable, cleared before the launch): set when a mass differs from
// that of the first particle in sorted order.
template <typename T>
__global__ void k_offsets(const double* __restrict__ pos, const double* __restrict__ mass,
                          const uint32_t* __restrict__ perm, const int32_t* __restrict__ group_of,
                          const int32_t* __restrict__ g_cell, const double* __restrict__ c_centre,
                          int64_t n, V4<T>* __restrict__ off, unsigned* __restrict__ flags,
                          unsigned* __restrict__ mdiff = nullptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  const int gc = g_cell[group_of[i]];
  const double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2], m = mass[j];
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) atomicOr(flags, FLAG_NONFINITE_POS);
  if (!(isfinite(m) && m >= 0.0)) atomicOr(flags, FLAG_BAD_MASS);
  if (mdiff && m != mass[perm[0]]) atomicOr(mdiff, 1u);
  V4<T> o;
  o.x = (T)(x - c_centre[3 * gc]);
  o.y = (T)(y - c_centre[3 * gc + 1]);
  o.z = (T)(z - c_centre[3 * gc + 2]);
  o.w = (T)m;
  off[i] = o;
}

// Expansion coefficients of one cell, for a wavefront. Up to ~400 bytes they
// are read straight from global memory at wavefront-uniform addresses (scalar
// loads into SGPRs); larger sets do not fit the SGPR budget, so the wavefront
// stages them in its own LDS slot (16 bytes per lane) and every lane reads
// them back as broadcasts. The next entry's coefficients are fetched into
// registers (prefetch) while the current one is evaluated, and written to the
// slot (commit) at the top of the next iteration. Only wavefront-level
// ordering is needed: the LDS operations of one wavefront execute in order.
template <int P, typename T>
struct MomentStage {
  static constexpr int kStride = nm_pad(P);
  static constexpr bool kLds = nm(P) * (int)sizeof(T) > 400;
  static constexpr int kChunks = kStride * (int)sizeof(T) / 16;
  static constexpr int kPre = kLds ? (kChunks + 63) / 64 : 1;
  struct Regs {
    uint4 v[kPre];
  };
  __device__ static __forceinline__ void prefetch(Regs& r, const T* __restrict__ momw, int64_t c,
                                                  int lane) {
    if constexpr (kLds) {
      const uint4* src = reinterpret_cast<const uint4*>(momw + c * kStride);
#pragma unroll
      for (int k = 0; k < kPre; ++k)
        if (lane + 64 * k < kChunks) r.v[k] = src[lane + 64 * k];
    }
  }
  __device__ static __forceinline__ const T* commit(const Regs& r, const T* __restrict__ momw,
                                                    int64_t c, T* slot, int lane) {
    if constexpr (!kLds) {
      return momw + c * kStride;
    } else {
      uint4* dst = reinterpret_cast<uint4*>(slot);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int k = 0; k < kPre; ++k)
        if (lane + 64 * k < kChunks) dst[lane + 64 * k] = r.v[k];
      __builtin_amdgcn_wave_barrier();
      return slot;
    }
  }
};

}  // namespace hot
