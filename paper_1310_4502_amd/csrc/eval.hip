// Force evaluation over the interaction lists.
//
// Pair kernel: the softened Newtonian pair force (eq. "eom" at a = 1, G = 1,
// with the Plummer smoothing of the Force Smoothing section). Expansion
// kernel: the cell-body Cartesian multipole expansion with Delta = 0 of the
// Multipole Error Bounds section, with the softened Green's function.
//
// m x n blocking (Improving instruction-level parallelism section): one
// wavefront serves up to 64 sinks of one group (one sink per lane) and runs
// over the group's list; every source particle or source cell is
// wavefront-uniform, so its data arrives through scalar loads shared by all
// 64 sinks. The interaction vector of a sink is written back once per
// kernel (the paper's multi-stage write-back), with compensated (Kahan)
// accumulation in mixed precision: one compensated add per expansion entry
// and per block of at least kSumRun pair-summed sources.
//
// Mixed precision: every position enters as an FP32 offset from its own
// group's FP64 centre; the FP64 difference of two centres is formed once per
// (group, entry) and rounded to FP32. Expansions run on coordinates scaled by
// the source cell side s (a power of two): R/s, eps/s and the weighted moments
// M_alpha / s^|alpha| are all O(1), and the result is rescaled by s^-2.
#include "common.h"
#include "eval_common.h"
#include "expansion_q.h"
#include "generated/expansions.h"

namespace hot {
namespace {

constexpr int kB = 256;
constexpr int kWavesPerBlock = kB / 64;

// State per sorted particle: s_x s_y s_z s_phi c_x c_y c_z c_phi.

// The plain FP32 pair kernel fits 64 VGPRs without spilling and runs eight
// waves per SIMD (4 % faster than at five); the FP64 and K1 forms need more
// registers and keep the default.
template <typename T, bool K1>
constexpr int p2p_waves_per_simd() { return (sizeof(T) == 4 && !K1) ? 8 : 1; }

// The group's list comes as its pair segments (sources [first, end) of one
// source group in one image, the centre difference precomputed in FP64 when
// the lists were built), so the kernel follows no list entry, cell or group
// record of its own.
template <typename T, bool POT, bool EPS0, bool K1>
__global__ __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(p2p_waves_per_simd<T, K1>())))
void k_p2p(
    const int2* __restrict__ items, int64_t n_items, const int64_t* __restrict__ pseg_off,
    const PairSeg* __restrict__ pseg, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const V4<T>* __restrict__ off, T eps2, T ie,
    const unsigned* __restrict__ mdiff, T* __restrict__ state, int64_t n) {
  __shared__ V4<T> stage[kWavesPerBlock][64];
  // K1: eps2 is the squared kernel radius, ie its inverse radius
  const T ie2 = ie * ie, ie3 = ie * ie2;
  // every particle of the same mass (k_offsets found none that differs): the
  // pair loop leaves the mass out and the summed blocks are scaled once
  const bool uni = *mdiff == 0u;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V4<T>* slot = stage[w];
  const int64_t it = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int gend = g_first[g] + g_count[g];
  // m x n blocking with n = 2: lane l holds the two sinks item.y + (l & 31)
  // (A) and item.y + 32 + (l & 31) (B); the half h = l / 32 of the wavefront
  // takes the sources of odd (h = 1) or even (h = 0) index, so every source
  // read from LDS serves two pairs. The halves' sums are added at each
  // compensated add; lane l keeps the compensated sums of sink item.y + l.
  const int h = lane >> 5, sub = lane & 31;
  const int iA = item.y + sub, iB = iA + 32;
  const int i = item.y + lane;
  const bool active = i < gend;
  V4<T> mA, mB;
  mA.x = mA.y = mA.z = mA.w = T(0);
  mB = mA;
  if (iA < gend) mA = off[iA];
  if (iB < gend) mB = off[iB];
  T sx = 0, sy = 0, sz = 0, sp = 0, cx = 0, cy = 0, cz = 0, cp = 0;
  // Plain FP32 sums in two alternating accumulators per sink (the halves'
  // sources) over consecutive segments, each segment's sources taken relative
  // to the sink group's centre, until at least kSumRun sources are summed; then
  // the halves are added (lane l < 32 completes sink A = item.y + l, lane
  // l >= 32 sink B = item.y + l) and go into the compensated sums with one
  // compensated add (fewer than kSumRun + n_group terms per plain sum).
  T aAx = 0, aAy = 0, aAz = 0, aAp = 0;
  T aBx = 0, aBy = 0, aBz = 0, aBp = 0;
  T mseg = T(1);
  int n_acc = 0;
#define HOT_FLUSH                                                                    \
  {                                                                                  \
    const T kx = h ? aBx : aAx, ky = h ? aBy : aAy, kz = h ? aBz : aAz;              \
    const T ox = __shfl_xor(h ? aAx : aBx, 32), oy = __shfl_xor(h ? aAy : aBy, 32),  \
            oz = __shfl_xor(h ? aAz : aBz, 32);                                      \
    kahan_add(sx, cx, (kx + ox) * mseg);                                             \
    kahan_add(sy, cy, (ky + oy) * mseg);                                             \
    kahan_add(sz, cz, (kz + oz) * mseg);                                             \
    if (POT) {                                                                       \
      const T kp = h ? aBp : aAp;                                                    \
      const T op = __shfl_xor(h ? aAp : aBp, 32);                                    \
      kahan_add(sp, cp, (kp + op) * mseg);                                           \
    }                                                                                \
    aAx = aAy = aAz = aAp = T(0);                                                    \
    aBx = aBy = aBz = aBp = T(0);                                                    \
    n_acc = 0;                                                                       \
  }
  const int64_t q1 = pseg_off[g + 1];
  for (int64_t q = pseg_off[g]; q < q1; ++q) {
    {
      // a segment: the sources [j, jend) of one source group
      const PairSeg sgm = pseg[q];
      const int j = uniform_i32(sgm.first);
      const int jend = uniform_i32(sgm.end);
      const bool self = uniform_i32(sgm.self) != 0;
      const T dx = (T)sgm.dx, dy = (T)sgm.dy, dz = (T)sgm.dz;
      const T tAx = dx - mA.x, tAy = dy - mA.y, tAz = dz - mA.z;
      const T tBx = dx - mB.x, tBy = dy - mB.y, tBz = dz - mB.z;
      // one pair of a sink (T*) with source s, into accumulators A*
#define HOT_PAIR1(SELF, UM, VALID, SINK_I, TX, TY, TZ, AX, AY, AZ, AP)               \
  {                                                                                  \
    const T rx = s.x + TX, ry = s.y + TY, rz = s.z + TZ;                             \
    if constexpr (!K1) {                                                             \
      const T r2 = hot_fma(rx, rx, hot_fma(ry, ry, hot_fma(rz, rz, eps2)));          \
      T inv = (EPS0 && !(r2 > T(0))) ? T(0) : hot_rsq(r2);                           \
      if (!(VALID) || (SELF && jb + k == (SINK_I))) inv = T(0);                      \
      const T mi = UM ? inv : s.w * inv;                                             \
      const T f3 = mi * (inv * inv);                                                 \
      AX = hot_fma(f3, rx, AX);                                                      \
      AY = hot_fma(f3, ry, AY);                                                      \
      AZ = hot_fma(f3, rz, AZ);                                                      \
      if (POT) AP -= mi;                                                             \
    } else {                                                                         \
      const T r2 = hot_fma(rx, rx, hot_fma(ry, ry, rz * rz));                        \
      const T inv = hot_rsq(r2);                                                     \
      T f3 = inv * (inv * inv);                                                      \
      T mi = inv;                                                                    \
      if (r2 < eps2) {                                                               \
        const T v = (eps2 - r2) * ie2;                                               \
        f3 = ie3 * k1_force(v);                                                      \
        if (POT) mi = ie * k1_pot(v);                                                \
      }                                                                              \
      if (!UM) {                                                                     \
        f3 *= s.w;                                                                   \
        mi *= s.w;                                                                   \
      }                                                                              \
      if (!(VALID) || (SELF && jb + k == (SINK_I))) {                                \
        f3 = T(0);                                                                   \
        mi = T(0);                                                                   \
      }                                                                              \
      AX = hot_fma(f3, rx, AX);                                                      \
      AY = hot_fma(f3, ry, AY);                                                      \
      AZ = hot_fma(f3, rz, AZ);                                                      \
      if (POT) AP -= mi;                                                             \
    }                                                                                \
  }
      // sources k2 + h for k2 = 0, 2, 4, ...: full pairs of sources first, then
      // the odd last one (half 0 only)
#define HOT_BATCH(UM, SELF)                                                          \
  {                                                                                  \
    int k2 = 0;                                                                      \
    _Pragma("unroll 4") for (; k2 + 1 < nbt; k2 += 2) {                              \
      const int k = k2 + h;                                                          \
      const V4<T> s = slot[k];                                                       \
      HOT_PAIR1(SELF, UM, true, iA, tAx, tAy, tAz, aAx, aAy, aAz, aAp)               \
      HOT_PAIR1(SELF, UM, true, iB, tBx, tBy, tBz, aBx, aBy, aBz, aBp)               \
    }                                                                                \
    if (k2 < nbt) {                                                                  \
      const int k = k2 + h;                                                          \
      const V4<T> s = slot[k2];                                                      \
      HOT_PAIR1(SELF, UM, h == 0, iA, tAx, tAy, tAz, aAx, aAy, aAz, aAp)             \
      HOT_PAIR1(SELF, UM, h == 0, iB, tBx, tBy, tBz, aBx, aBy, aBz, aBp)             \
    }                                                                                \
  }
      for (int jb = j; jb < jend; jb += 64) {
        const int nbt = jend - jb < 64 ? jend - jb : 64;
        V4<T> v;
        v.x = v.y = v.z = v.w = T(0);
        if (lane < nbt) v = off[jb + lane];
        __builtin_amdgcn_wave_barrier();
        slot[lane] = v;
        __builtin_amdgcn_wave_barrier();
        if (uni) {
          if (self)
            HOT_BATCH(true, true)
          else
            HOT_BATCH(true, false)
          mseg = slot[0].w;
        } else {
          if (self)
            HOT_BATCH(false, true)
          else
            HOT_BATCH(false, false)
        }
      }
#undef HOT_BATCH
#undef HOT_PAIR1
      n_acc += jend - j;
      if (n_acc >= kSumRun) HOT_FLUSH
    }
  }
  if (n_acc > 0) HOT_FLUSH
#undef HOT_FLUSH
  if (active) {
    T* st = state + (int64_t)i * 8;
    st[0] = sx;
    st[1] = sy;
    st[2] = sz;
    st[3] = sp;
    st[4] = cx;
    st[5] = cy;
    st[6] = cz;
    st[7] = cp;
  }
}

// The FP32 kernels of the two highest orders are held to 128 VGPRs (four
// waves per SIMD instead of three; the cost is a few spilled FP64 centre words).
template <int P, typename T>
constexpr int m2p_waves_per_simd() { return (sizeof(T) == 4 && P >= 7) ? 4 : 1; }

// MIXQ: every entry carries its own order q <= P (m2p_q), error-bound lists.
// PER: every entry carries the image of its cell (periodic lists).
// BG: background subtraction; an entry flagged in m2p_sub takes its cell's
// moments minus those of its uniform cube (momsub) instead of momw.
template <int P, typename T, bool POT, bool MIXQ, bool PER, bool BG, bool K1>
__global__ __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(m2p_waves_per_simd<P, T>())))
void k_m2p(
    const int2* __restrict__ items, int64_t n_items, const int64_t* __restrict__ m2p_off,
    const int32_t* __restrict__ m2p, const int8_t* __restrict__ m2p_q,
    const int8_t* __restrict__ m2p_img, double side, const int8_t* __restrict__ m2p_sub,
    const T* __restrict__ momsub,
    const int8_t* __restrict__ c_level,
    const int32_t* __restrict__ g_first, const int32_t* __restrict__ g_count,
    const int32_t* __restrict__ g_cell, const double* __restrict__ c_centre,
    const V4<T>* __restrict__ off, const T* __restrict__ momw, double inv_side, double eps,
    T* __restrict__ state) {
  using Stage = MomentStage<P, T>;
  __shared__ T smom[Stage::kLds ? kWavesPerBlock * Stage::kStride : 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int gend = g_first[g] + g_count[g];
  const int i = item.y + lane;
  const bool active = i < gend;
  const int gc = g_cell[g];
  const double cgx = c_centre[3 * gc], cgy = c_centre[3 * gc + 1], cgz = c_centre[3 * gc + 2];
  V4<T> me;
  me.x = me.y = me.z = me.w = T(0);
  if (active) me = off[i];
  T sx = 0, sy = 0, sz = 0, sp = 0, cx = 0, cy = 0, cz = 0, cp = 0;
  if (active) {
    const T* st = state + (int64_t)i * 8;
    sx = st[0];
    sy = st[1];
    sz = st[2];
    sp = st[3];
    cx = st[4];
    cy = st[5];
    cz = st[6];
    cp = st[7];
  }
  const int64_t e0 = m2p_off[g], e1 = m2p_off[g + 1];
  T* slot = smom + (Stage::kLds ? w * Stage::kStride : 0);
  typename Stage::Regs pre;
  int cn = 0, ln = 0, qn = P, sn = 0;
  double nx = 0, ny = 0, nz = 0;
  if (e0 < e1) {
    cn = uniform_i32(m2p[e0]);
    if (MIXQ) qn = uniform_i32(m2p_q[e0]);
    if (BG) sn = uniform_i32(m2p_sub[e0]);
    Stage::prefetch(pre, (BG && sn) ? momsub : momw, cn, lane);
    ln = c_level[cn];
    nx = c_centre[3 * cn];
    ny = c_centre[3 * cn + 1];
    nz = c_centre[3 * cn + 2];
    if (PER) {
      double sx, sy, sz;
      image_shift(uniform_i32(m2p_img[e0]), side, sx, sy, sz);
      nx += sx;
      ny += sy;
      nz += sz;
    }
  }
  for (int64_t e = e0; e < e1; ++e) {
    const int c = cn;
    const int q = qn;
    const double inv_s = ldexp(inv_side, ln);
    const T X = (T)((cgx - nx) * inv_s) + me.x * (T)inv_s;
    const T Y = (T)((cgy - ny) * inv_s) + me.y * (T)inv_s;
    const T Z = (T)((cgz - nz) * inv_s) + me.z * (T)inv_s;
    const T* M = Stage::commit(pre, (BG && sn) ? momsub : momw, c, slot, lane);
    if (e + 1 < e1) {
      cn = uniform_i32(m2p[e + 1]);
      if (MIXQ) qn = uniform_i32(m2p_q[e + 1]);
      if (BG) sn = uniform_i32(m2p_sub[e + 1]);
      Stage::prefetch(pre, (BG && sn) ? momsub : momw, cn, lane);
      ln = c_level[cn];
      nx = c_centre[3 * cn];
      ny = c_centre[3 * cn + 1];
      nz = c_centre[3 * cn + 2];
      if (PER) {
        double sx, sy, sz;
        image_shift(uniform_i32(m2p_img[e + 1]), side, sx, sy, sz);
        nx += sx;
        ny += sy;
        nz += sz;
      }
    }
    const double es = eps * inv_s;
    const T e2 = (T)(es * es);
    T ax = 0, ay = 0, az = 0, ph = 0;
    if (MIXQ)
      expansion_fwd_q<P, T, POT, K1>(q, X, Y, Z, e2, M, ax, ay, az, ph);
    else
      expansion_fwd<P, T, POT, K1>(X, Y, Z, e2, M, ax, ay, az, ph);
    const T sa = (T)(-(inv_s * inv_s));
    kahan_add(sx, cx, ax * sa);
    kahan_add(sy, cy, ay * sa);
    kahan_add(sz, cz, az * sa);
    if (POT) kahan_add(sp, cp, ph * (T)inv_s);
  }
  if (active) {
    T* st = state + (int64_t)i * 8;
    st[0] = sx;
    st[1] = sy;
    st[2] = sz;
    st[3] = sp;
    st[4] = cx;
    st[5] = cy;
    st[6] = cz;
    st[7] = cp;
  }
}

// Expansion terms for an item of at most 32 sinks (theta lists without
// background subtraction): the wavefront splits into S = 64 / W slices of
// W = max(8, 2^ceil(log2 n_sinks)) lanes. In each round slice s evaluates
// entry e0 + round S + s for the item's sinks; the round's S cells have their
// coefficients staged together in the wavefront's LDS, so the lanes that an
// item of few sinks leaves idle in k_m2p do useful work. The slices'
// compensated sums are added at the end. Every cross-lane read is executed by
// all lanes (never inside a lane-dependent branch or operand).
template <int P, typename T, bool POT, bool PER, bool K1>
__global__ __launch_bounds__(64) void k_m2p_sl(
    const int2* __restrict__ items, int64_t n_items, const int64_t* __restrict__ m2p_off,
    const int32_t* __restrict__ m2p, const int8_t* __restrict__ m2p_img, double side,
    const int8_t* __restrict__ c_level, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const int32_t* __restrict__ g_cell,
    const double* __restrict__ c_centre, const V4<T>* __restrict__ off,
    const T* __restrict__ momw, double inv_side, double eps, T* __restrict__ state) {
  constexpr int kStride = nm_pad(P);
  constexpr int kChunks = kStride * (int)sizeof(T) / 16;
  constexpr int kMaxS = 8;
  constexpr int kRounds = (kMaxS * kChunks + 63) / 64;
  __shared__ uint4 smom[kMaxS * kChunks];
  const int lane = threadIdx.x;
  const int64_t it = blockIdx.x;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int gend = uniform_i32(g_first[g] + g_count[g]);
  const int ns = gend - item.y < 64 ? gend - item.y : 64;  // <= 32 for these items
  const int lw = ns <= 8 ? 3 : 32 - __clz(ns - 1);
  const int S = 64 >> lw;
  const int p = lane & ((1 << lw) - 1), sl = lane >> lw;
  const int i = item.y + p;
  const bool active = p < ns;
  const int gc = g_cell[g];
  const double cgx = c_centre[3 * gc], cgy = c_centre[3 * gc + 1], cgz = c_centre[3 * gc + 2];
  V4<T> me;
  me.x = me.y = me.z = me.w = T(0);
  if (active) me = off[i];
  T sx = 0, sy = 0, sz = 0, sp = 0, cx = 0, cy = 0, cz = 0, cp = 0;
  if (active && sl == 0) {
    const T* st = state + (int64_t)i * 8;
    sx = st[0];
    sy = st[1];
    sz = st[2];
    sp = st[3];
    cx = st[4];
    cy = st[5];
    cz = st[6];
    cp = st[7];
  }
  const int64_t e0 = m2p_off[g], e1 = m2p_off[g + 1];
  for (int64_t eb = e0; eb < e1; eb += S) {
    // the round's cells (and images), one per lane
    int cl = -1, il = kCentreImage;
    if (lane < S && eb + lane < e1) {
      cl = m2p[eb + lane];
      if (PER) il = m2p_img[eb + lane];
    }
    // stage their coefficients: chunk k of slice s at smom[s kChunks + k]
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const int ch = lane + 64 * r;
      const int s2 = ch / kChunks;
      const int cs = __shfl(cl, s2 < kMaxS ? s2 : 0);
      if (s2 < S && cs >= 0)
        smom[ch] = reinterpret_cast<const uint4*>(momw + (int64_t)cs * kStride)[ch - s2 * kChunks];
    }
    __builtin_amdgcn_wave_barrier();
    // slices without an entry this round evaluate slice 0's and add nothing
    const int cme = __shfl(cl, sl);
    const int c0 = __shfl(cl, 0);  // valid in every round
    const bool ok = cme >= 0;
    const int sme = ok ? sl : 0;
    const int c = ok ? cme : c0;
    double nx = c_centre[3 * c], ny = c_centre[3 * c + 1], nz = c_centre[3 * c + 2];
    if (PER) {
      const int ime = __shfl(il, sl), i0m = __shfl(il, 0);
      double shx, shy, shz;
      image_shift(ok ? ime : i0m, side, shx, shy, shz);
      nx += shx;
      ny += shy;
      nz += shz;
    }
    const double inv_s = ldexp(inv_side, (int)c_level[c]);
    const T X = (T)((cgx - nx) * inv_s) + me.x * (T)inv_s;
    const T Y = (T)((cgy - ny) * inv_s) + me.y * (T)inv_s;
    const T Z = (T)((cgz - nz) * inv_s) + me.z * (T)inv_s;
    const T* M = reinterpret_cast<const T*>(smom) + sme * kStride;
    const double es = eps * inv_s;
    const T e2 = (T)(es * es);
    T ax = 0, ay = 0, az = 0, ph = 0;
    expansion_fwd<P, T, POT, K1>(X, Y, Z, e2, M, ax, ay, az, ph);
    const T sa = ok ? (T)(-(inv_s * inv_s)) : T(0);
    kahan_add(sx, cx, ax * sa);
    kahan_add(sy, cy, ay * sa);
    kahan_add(sz, cz, az * sa);
    if (POT) kahan_add(sp, cp, ph * (ok ? (T)inv_s : T(0)));
  }
  // add the slices' compensated sums (true value s - c) across lanes
  for (int m = 32; m >= (1 << lw); m >>= 1) {
    T o = __shfl_xor(sx, m), oc = __shfl_xor(cx, m);
    kahan_add(sx, cx, o);
    cx += oc;
    o = __shfl_xor(sy, m);
    oc = __shfl_xor(cy, m);
    kahan_add(sy, cy, o);
    cy += oc;
    o = __shfl_xor(sz, m);
    oc = __shfl_xor(cz, m);
    kahan_add(sz, cz, o);
    cz += oc;
    if (POT) {
      o = __shfl_xor(sp, m);
      oc = __shfl_xor(cp, m);
      kahan_add(sp, cp, o);
      cp += oc;
    }
  }
  if (active && sl == 0) {
    T* st = state + (int64_t)i * 8;
    st[0] = sx;
    st[1] = sy;
    st[2] = sz;
    st[3] = sp;
    st[4] = cx;
    st[5] = cy;
    st[6] = cz;
    st[7] = cp;
  }
}

// split of the work items by sink count (at most 32, or more)
__global__ void k_item_flags(const int2* __restrict__ items, int64_t n_items,
                             const int32_t* __restrict__ g_first,
                             const int32_t* __restrict__ g_count, uint32_t* __restrict__ small) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_items) return;
  const int2 it = items[k];
  small[k] = g_first[it.x] + g_count[it.x] - it.y <= 32 ? 1u : 0u;
}

__global__ void k_item_split(const int2* __restrict__ items, int64_t n_items,
                             const uint32_t* __restrict__ small, const uint32_t* __restrict__ pos,
                             int2* __restrict__ out_small, int2* __restrict__ out_big) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_items) return;
  if (small[k])
    out_small[pos[k]] = items[k];
  else
    out_big[k - (int64_t)pos[k]] = items[k];
}

template <typename T>
__global__ void k_finalize(const T* __restrict__ state, const uint32_t* __restrict__ perm,
                           int64_t n, double* __restrict__ acc, double* __restrict__ pot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T* st = state + i * 8;
  const int64_t j = perm[i];
  acc[3 * j] = (double)st[0] - (double)st[4];
  acc[3 * j + 1] = (double)st[1] - (double)st[5];
  acc[3 * j + 2] = (double)st[2] - (double)st[6];
  if (pot) pot[j] = (double)st[3] - (double)st[7];
}

template <typename T, bool POT>
void launch_p2p(hot_ctx* ctx, hot_tree* t, const V4<T>* off, double eps, bool k1, T* state) {
  const unsigned* mdiff = ctx->d_flags + kFlagMass;
  const unsigned grid = grid_for(t->n_items, kWavesPerBlock);
  const T e2 = (T)(eps * eps);
  const T ie = k1 ? (T)(1.0 / eps) : T(0);
  auto go = [&](auto kern) {
    kern<<<grid, kB, 0, ctx->stream>>>(t->items.as<int2>(), t->n_items,
                                       t->pseg_off.as<int64_t>(), t->pseg.as<PairSeg>(),
                                       t->g_first.as<int32_t>(), t->g_count.as<int32_t>(), off,
                                       e2, ie, mdiff, state, t->n);
    HOT_CHECK_LAUNCH();
  };
  if (k1)
    go(k_p2p<T, POT, false, true>);
  else if (e2 > T(0))
    go(k_p2p<T, POT, false, false>);
  else
    go(k_p2p<T, POT, true, false>);
}

template <int P, typename T, bool POT, bool K1>
void launch_m2p_p(hot_ctx* ctx, hot_tree* t, const V4<T>* off, const T* momw, const T* momsub,
                  double eps, T* state) {
  const unsigned grid = grid_for(t->n_items, kWavesPerBlock);
  auto go = [&](auto kern) {
    kern<<<grid, kB, 0, ctx->stream>>>(
        t->items.as<int2>(), t->n_items, t->m2p_off.as<int64_t>(), t->m2p.as<int32_t>(),
        t->m2p_q.as<int8_t>(), t->m2p_img.as<int8_t>(), t->side, t->m2p_sub.as<int8_t>(), momsub,
        t->c_level.as<int8_t>(), t->g_first.as<int32_t>(), t->g_count.as<int32_t>(),
        t->g_cell.as<int32_t>(), t->c_centre.as<double>(), off, momw, 1.0 / t->side, eps, state);
    HOT_CHECK_LAUNCH();
  };
  if (t->list_p >= 0) {
    if (t->periodic)
      go(k_m2p<P, T, POT, true, true, false, K1>);
    else
      go(k_m2p<P, T, POT, true, false, false, K1>);
  } else if (!t->bg && t->n_items_small * 10 >= t->n_items) {
    // theta lists with many part-empty items: those of at most 32 sinks by
    // slices of one wavefront, the others as usual
    if (t->n_items_big > 0) {
      auto kb = t->periodic ? k_m2p<P, T, POT, false, true, false, K1>
                            : k_m2p<P, T, POT, false, false, false, K1>;
      kb<<<grid_for(t->n_items_big, kWavesPerBlock), kB, 0, ctx->stream>>>(
          t->items_big.as<int2>(), t->n_items_big, t->m2p_off.as<int64_t>(), t->m2p.as<int32_t>(),
          t->m2p_q.as<int8_t>(), t->m2p_img.as<int8_t>(), t->side, t->m2p_sub.as<int8_t>(),
          momsub, t->c_level.as<int8_t>(), t->g_first.as<int32_t>(), t->g_count.as<int32_t>(),
          t->g_cell.as<int32_t>(), t->c_centre.as<double>(), off, momw, 1.0 / t->side, eps, state);
      HOT_CHECK_LAUNCH();
    }
    if (t->n_items_small > 0) {
      auto ks = t->periodic ? k_m2p_sl<P, T, POT, true, K1> : k_m2p_sl<P, T, POT, false, K1>;
      ks<<<(unsigned)t->n_items_small, 64, 0, ctx->stream>>>(
          t->items_small.as<int2>(), t->n_items_small, t->m2p_off.as<int64_t>(),
          t->m2p.as<int32_t>(), t->m2p_img.as<int8_t>(), t->side, t->c_level.as<int8_t>(),
          t->g_first.as<int32_t>(), t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(),
          t->c_centre.as<double>(), off, momw, 1.0 / t->side, eps, state);
      HOT_CHECK_LAUNCH();
    }
  } else if (t->periodic) {
    // potentials are refused with background subtraction: no variant for them
    if constexpr (!POT) {
      if (t->bg) {
        go(k_m2p<P, T, POT, false, true, true, K1>);
        return;
      }
    }
    go(k_m2p<P, T, POT, false, true, false, K1>);
  } else {
    go(k_m2p<P, T, POT, false, false, false, K1>);
  }
}

}  // namespace

// Items of at most 32 sinks and the others, listed apart (built with the tree)
void split_items(hot_ctx* ctx, hot_tree* t) {
  hipStream_t st = ctx->stream;
  const int64_t NI = t->n_items;
  DBuf flag, pos;
  flag.alloc(ctx, std::max<int64_t>(1, NI) * sizeof(uint32_t));
  pos.alloc(ctx, (NI + 1) * sizeof(uint32_t));
  k_item_flags<<<grid_for(NI, kB), kB, 0, st>>>(t->items.as<int2>(), NI, t->g_first.as<int32_t>(),
                                               t->g_count.as<int32_t>(), flag.as<uint32_t>());
  HOT_CHECK_LAUNCH();
  // exclusive offsets of the small items, their number in the last slot
  uint32_t* pp = pos.as<uint32_t>();
  scan_u32(ctx, flag.as<uint32_t>(), pp, NI, pp + NI);
  uint32_t ns = 0;
  HOT_HIP(hipMemcpyAsync(&ns, pp + NI, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipStreamSynchronize(st));
  t->items_small.alloc(ctx, std::max<int64_t>(1, (int64_t)ns) * sizeof(int2));
  t->items_big.alloc(ctx, std::max<int64_t>(1, NI - (int64_t)ns) * sizeof(int2));
  k_item_split<<<grid_for(NI, kB), kB, 0, st>>>(t->items.as<int2>(), NI, flag.as<uint32_t>(), pp,
                                               t->items_small.as<int2>(), t->items_big.as<int2>());
  HOT_CHECK_LAUNCH();
  t->n_items_small = ns;
  t->n_items_big = NI - (int64_t)ns;
}

namespace {

template <typename T, bool POT, bool K1>
void launch_m2p_k(hot_ctx* ctx, hot_tree* t, const V4<T>* off, const T* momw, const T* momsub,
                  double eps, T* state) {
  switch (t->p) {
    case 0: launch_m2p_p<0, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 1: launch_m2p_p<1, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 2: launch_m2p_p<2, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 3: launch_m2p_p<3, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 4: launch_m2p_p<4, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 5: launch_m2p_p<5, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 6: launch_m2p_p<6, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 7: launch_m2p_p<7, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    case 8: launch_m2p_p<8, T, POT, K1>(ctx, t, off, momw, momsub, eps, state); break;
    default: invalid("p out of range");
  }
}

template <typename T, bool POT>
void launch_m2p(hot_ctx* ctx, hot_tree* t, const V4<T>* off, const T* momw, const T* momsub,
                double eps, bool k1, T* state) {
  if (k1)
    launch_m2p_k<T, POT, true>(ctx, t, off, momw, momsub, eps, state);
  else
    launch_m2p_k<T, POT, false>(ctx, t, off, momw, momsub, eps, state);
}

template <typename T>
void forces_t(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
              bool k1, double* acc, double* pot, hot_stats* stats, const EvalMem* mem) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  // caller memory where given (every element is written below before it is
  // read: the offsets by k_offsets, the sums by the pair kernel, which
  // covers every sink), else the context allocator
  DBuf off_buf, state_buf;
  V4<T>* off = mem ? static_cast<V4<T>*>(mem->off) : nullptr;
  T* state = mem ? static_cast<T*>(mem->state) : nullptr;
  if (!off) {
    off_buf.alloc(ctx, n * sizeof(V4<T>));
    off = off_buf.as<V4<T>>();
  }
  if (!state) {
    state_buf.alloc(ctx, n * 8 * sizeof(T));
    state = state_buf.as<T>();
  }
  zero_flag_word(ctx, kFlagMass);
  k_offsets<T><<<grid_for(n, kB), kB, 0, st>>>(pos, mass, t->perm.as<uint32_t>(),
                                               t->group_of.as<int32_t>(), t->g_cell.as<int32_t>(),
                                               t->c_centre.as<double>(), n, off, ctx->d_flags,
                                               ctx->d_flags + kFlagMass);
  HOT_CHECK_LAUNCH();
  const T* momw = nullptr;
  if constexpr (sizeof(T) == 4) {
    momw = t->mom32.as<T>();
  } else {
    weighted_fp64(ctx, t);
    momw = t->momw64.as<T>();
  }
  const T* momsub = nullptr;
  if (t->bg) {
    weighted_sub(ctx, t, sizeof(T) == 8);
    momsub = t->momsub.as<T>();
  }
  if (t->n_items_small < 0) ::hot::state("tree without its item split");
  if (stats) HOT_HIP(hipEventRecord(ctx->ev[0], st));
  {
    Phase ph(ctx, HOT_T_EVAL_P2P);
    if (pot)
      launch_p2p<T, true>(ctx, t, off, eps, k1, state);
    else
      launch_p2p<T, false>(ctx, t, off, eps, k1, state);
  }
  if (stats) HOT_HIP(hipEventRecord(ctx->ev[1], st));
  {
    Phase ph(ctx, HOT_T_EVAL_M2P);
    if (pot)
      launch_m2p<T, true>(ctx, t, off, momw, momsub, eps, k1, state);
    else
      launch_m2p<T, false>(ctx, t, off, momw, momsub, eps, k1, state);
  }
  if (stats) HOT_HIP(hipEventRecord(ctx->ev[2], st));
  k_finalize<T><<<grid_for(n, kB), kB, 0, st>>>(state, t->perm.as<uint32_t>(), n, acc, pot);
  HOT_CHECK_LAUNCH();
  if (stats) {
    HOT_HIP(hipEventRecord(ctx->ev[3], st));
    HOT_HIP(hipEventSynchronize(ctx->ev[3]));
    float a = 0, b = 0, c = 0;
    HOT_HIP(hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
    HOT_HIP(hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
    HOT_HIP(hipEventElapsedTime(&c, ctx->ev[0], ctx->ev[3]));
    stats->ms_p2p = a;
    stats->ms_m2p = b;
    stats->ms_total = c;
    stats->p2p_pairs = t->p2p_pairs;
    stats->m2p_pairs = t->m2p_pairs;
  }
}

template <typename T>
__global__ void k_zero_t(T* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// The expansion kernel on the background-subtracted lists with zero matter
// moments and the negated unit-density cube moments: the derivative of the
// forces with respect to the mean density through the flagged entries.
template <typename T>
void cube_field_t(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
                  bool k1, double* out) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  const int64_t nmom = t->n_cells * nm_pad(t->p);
  DBuf off, state, zero, cube;
  off.alloc(ctx, n * sizeof(V4<T>));
  state.alloc(ctx, n * 8 * sizeof(T));
  zero.alloc(ctx, nmom * sizeof(T));
  cube.alloc(ctx, nmom * sizeof(T));
  k_offsets<T><<<grid_for(n, kB), kB, 0, st>>>(pos, mass, t->perm.as<uint32_t>(),
                                               t->group_of.as<int32_t>(), t->g_cell.as<int32_t>(),
                                               t->c_centre.as<double>(), n, off.as<V4<T>>(),
                                               ctx->d_flags);
  HOT_CHECK_LAUNCH();
  k_zero_t<T><<<grid_for(n * 8, kB), kB, 0, st>>>(state.as<T>(), n * 8);
  HOT_CHECK_LAUNCH();
  k_zero_t<T><<<grid_for(nmom, kB), kB, 0, st>>>(zero.as<T>(), nmom);
  HOT_CHECK_LAUNCH();
  weighted_cube(ctx, t, sizeof(T) == 8, cube.p);
  launch_m2p<T, false>(ctx, t, off.as<V4<T>>(), zero.as<T>(), cube.as<T>(), eps, k1,
                       state.as<T>());
  k_finalize<T><<<grid_for(n, kB), kB, 0, st>>>(state.as<T>(), t->perm.as<uint32_t>(), n, out,
                                                nullptr);
  HOT_CHECK_LAUNCH();
}

}  // namespace

void cube_field(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
                int precision, double* out) {
  if (!t->bg) state("cube field without background-subtracted lists");
  const bool k1 = use_k1(precision, eps);
  if (fp64_mode(precision))
    cube_field_t<double>(ctx, t, pos, mass, eps, k1, out);
  else
    cube_field_t<float>(ctx, t, pos, mass, eps, k1, out);
}

void forces(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
            int precision, double* acc, double* pot, hot_stats* stats, const EvalMem* mem) {
  const bool k1 = use_k1(precision, eps);
  if (fp64_mode(precision))
    forces_t<double>(ctx, t, pos, mass, eps, k1, acc, pot, stats, mem);
  else
    forces_t<float>(ctx, t, pos, mass, eps, k1, acc, pot, stats, mem);
}


}  // namespace hot
