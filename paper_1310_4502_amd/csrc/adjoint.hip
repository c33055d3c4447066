// Reverse derivative of the force evaluation: the vector-Jacobian product
// xbar = d(sum_i abar_i . a_i)/dx (and mbar = d/dm) with the tree topology
// (membership, centres, b_max, lists) held fixed. The paper has no adjoint;
// this differentiates exactly the map eval_forces computes.
//
//  pair terms    a_i += m_j K(x_j - x_i), K(r) = r (|r|^2+eps^2)^(-3/2),
//                dK/dr = H(r) = s^(-3/2) I - 3 r r^T s^(-5/2):
//                  sink   xbar_i -= m_j H(r_ij) abar_i      (group-major, like the forward)
//                  source xbar_j += m_j H(r_ij) abar_i      (source-major over transposed lists,
//                                 in work units whose sums are added in a fixed order)
//                                 mbar_j += abar_i . r_ij s^(-3/2)
//  expansion     a_i = -sum_alpha w_alpha M_alpha d^(alpha+e_k) G(x_i - c):
//                  sink   xbar_i += -sum_k abar_ik sum_alpha w M d^(alpha+e_k+e_l) G
//                  cell   Mbar_alpha += -w_alpha sum_i sum_k abar_ik d^(alpha+e_k) G
//                  Mbar flows down the tree through the transpose of the
//                  re-centring (M2M^T) and into the particles of each leaf
//                  through the transpose of the moment definition (P2M^T).
// Variants of the lists: per-entry orders (error-bound lists: the records of
// a cell are split by order, one cell-side launch per order), images
// (periodic lists: sources shifted by n L, the far replicas differentiated
// through the sink positions and the root's moments), cube-subtracted
// moments (background subtraction: the box fields and the mean density are
// differentiated separately).
// Every reduction is a gather in a fixed order: no floating-point atomics.
#include "common.h"
#include "eval_common.h"
#include "expansion_q.h"
#include "generated/expansions.h"

namespace hot {

namespace {

static __constant__ AlphaTable kAlpha = make_alpha_table();

constexpr int kB = 256;
constexpr int kWPB = kB / 64;
constexpr int kCellItemGroups = 48;  // groups per work item of the cell-side kernel
// Records per work unit of the source-side pair kernel: the largest of 1024,
// 512, 256 and 128 that still gives at least kSrcUnitsWanted units (eight per
// wavefront slot of the chip), so that large problems make few partial sums
// and small ones still fill the GPU (at 2^20 Plummer particles 128-record
// units take the kernel from 3.8 to 2.3 ms; at 2^24 1024 saves 3 %).
constexpr int64_t kSrcUnitsWanted = 1 << 16;
inline uint32_t src_chunk(int64_t nrec) {
  uint32_t c = 1024;
  while (c > 128 && nrec / c < kSrcUnitsWanted) c >>= 1;
  return c;
}


int bits_for(int64_t v) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) <= v) ++b;
  return b;
}

// ---------------------------------------------------------------- transposes
// One wavefront per sink group; its lanes stride over the group's list (the
// loads of consecutive entries coalesce), so records come out in entry order.
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// exclusive prefix sum over the lanes of a wavefront; *total gets the sum
__device__ __forceinline__ int wave_excl_scan(int v, int lane, int* total) {
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  *total = __shfl(x, 63);
  return x - v;
}

// records of one P2P entry: the source items its particle range touches
__device__ __forceinline__ void srec_range(const int32_t* __restrict__ p2p,
                                           const int32_t* __restrict__ c_first,
                                           const int32_t* __restrict__ c_count,
                                           const int32_t* __restrict__ item_of, int64_t e,
                                           int& q0, int& q1) {
  const int c = p2p[e];
  const int f = c_first[c];
  q0 = item_of[f];
  q1 = item_of[f + c_count[c] - 1];
}

__global__ __launch_bounds__(kB) void k_srec_count(
    const int64_t* __restrict__ p2p_off, const int32_t* __restrict__ p2p, int64_t G,
    const int32_t* __restrict__ c_first, const int32_t* __restrict__ c_count,
    const int32_t* __restrict__ item_of, int64_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWPB + (threadIdx.x >> 6);
  if (g >= G) return;
  const int64_t e1 = p2p_off[g + 1];
  int64_t k = 0;
  for (int64_t e = p2p_off[g] + lane; e < e1; e += 64) {
    int q0, q1;
    srec_range(p2p, c_first, c_count, item_of, e, q0, q1);
    k += q1 - q0 + 1;
  }
  k = wave_sum_i64(k);
  if (lane == 0) cnt[g] = k;
}

__global__ __launch_bounds__(kB) void k_srec_fill(
    const int64_t* __restrict__ p2p_off, const int32_t* __restrict__ p2p, int64_t G,
    const int32_t* __restrict__ c_first, const int32_t* __restrict__ c_count,
    const int32_t* __restrict__ item_of, const int64_t* __restrict__ rec_off, int gbits,
    uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWPB + (threadIdx.x >> 6);
  if (g >= G) return;
  int64_t o = rec_off[g];
  const int64_t e0 = p2p_off[g], e1 = p2p_off[g + 1];
  for (int64_t b = e0; b < e1; b += 64) {
    const int64_t e = b + lane;
    int q0 = 0, q1 = -1;
    if (e < e1) srec_range(p2p, c_first, c_count, item_of, e, q0, q1);
    int total;
    const int64_t at = o + wave_excl_scan(q1 - q0 + 1, lane, &total);
    for (int q = q0; q <= q1; ++q) {
      key[at + (q - q0)] = ((uint64_t)q << gbits) | (uint64_t)g;
      val[at + (q - q0)] = (uint32_t)e;
    }
    o += total;
  }
}

// work units of the source-side pair kernel: each item's records cut into runs
// of at most chunk (an item without records still gets one unit)
__global__ void k_sunit_count(const uint32_t* __restrict__ soff, int64_t n_items, uint32_t chunk,
                              uint32_t* __restrict__ cnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_items) return;
  const uint32_t n = soff[q + 1] - soff[q];
  cnt[q] = n == 0 ? 1u : (n + chunk - 1) / chunk;
}

__global__ void k_sunit_fill(const uint32_t* __restrict__ soff, int64_t n_items, uint32_t chunk,
                             const uint32_t* __restrict__ uoff, int4* __restrict__ units) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_items) return;
  const uint32_t b = soff[q], e = soff[q + 1];
  const uint32_t u0 = uoff[q], nu = uoff[q + 1] - u0;
  for (uint32_t k = 0; k < nu; ++k) {
    const uint32_t rb = b + k * chunk;
    const uint32_t re = rb + chunk < e ? rb + chunk : e;
    units[u0 + k] = make_int4((int)q, (int)rb, (int)re, nu == 1 ? 1 : 0);
  }
}

// key: the cell, followed by the entry's order in 4 low bits when the lists
// carry orders (m2p_q not null), or by its image in 7 low bits when they
// carry images (m2p_img not null)
__global__ __launch_bounds__(kB) void k_mrec_fill(const int64_t* __restrict__ m2p_off,
                                                  const int32_t* __restrict__ m2p,
                                                  const int8_t* __restrict__ m2p_q,
                                                  const int8_t* __restrict__ m2p_img, int64_t G,
                                                  uint64_t* __restrict__ key,
                                                  uint32_t* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWPB + (threadIdx.x >> 6);
  if (g >= G) return;
  const int64_t e1 = m2p_off[g + 1];
  for (int64_t e = m2p_off[g] + lane; e < e1; e += 64) {
    uint64_t k = (uint64_t)m2p[e];
    if (m2p_q) k = (k << 4) | (uint64_t)m2p_q[e];
    if (m2p_img) k = (k << 7) | (uint64_t)m2p_img[e];
    key[e] = k;
    val[e] = (uint32_t)g;
  }
}

// out[t] = first index of sorted keys with key >= (t << shift), t in [0, T].
__global__ void k_lower_bound(const uint64_t* __restrict__ keys, int64_t n, int shift, int64_t T,
                              uint32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > T) return;
  const uint64_t k = (uint64_t)t << shift;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  out[t] = (uint32_t)lo;
}

// number of items of each cell from its record range
__global__ void k_items_from_off(const uint32_t* __restrict__ rec_off, int64_t C,
                                 uint32_t* __restrict__ nit) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) nit[c] = (rec_off[c + 1] - rec_off[c] + kCellItemGroups - 1) / kCellItemGroups;
}

// cell owning entry k of a CSR with offsets off[0 .. C]: the largest c with
// off[c] <= k (cells without entries are skipped by taking the largest)
__device__ __forceinline__ int64_t owner_of(const uint32_t* __restrict__ off, int64_t C,
                                            uint32_t k) {
  int64_t lo = 0, hi = C;  // off[lo] <= k < off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// one thread per item (a cell may own very many items under periodic lists)
__global__ void k_cell_items(const uint32_t* __restrict__ rec_off, const uint32_t* __restrict__ it_off,
                             int64_t C, int64_t n_items, uint32_t* __restrict__ citem_rec,
                             int32_t* __restrict__ citem_cell) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_items) return;
  const int64_t c = owner_of(it_off, C, (uint32_t)k);
  citem_rec[k] = rec_off[c] + ((uint32_t)k - it_off[c]) * kCellItemGroups;
  citem_cell[k] = (int32_t)c;
}

// Reduction of the item partials of each cell in rounds: per cell, chunks of
// at most kSegChunk consecutive values; one thread per (chunk, slot).
constexpr int kSegChunk = 64;

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

__global__ void k_seg_count(const uint32_t* __restrict__ off, int64_t C,
                            uint32_t* __restrict__ cnt, unsigned* __restrict__ maxlen) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const uint32_t len = off[c + 1] - off[c];
  cnt[c] = (len + kSegChunk - 1) / kSegChunk;
  if (maxlen) atomicMax(maxlen, len);
}

template <typename Tin>
__global__ void k_seg_chunk_sum(const Tin* __restrict__ in, int in_stride,
                                const uint32_t* __restrict__ off_in,
                                const uint32_t* __restrict__ off_out, int64_t C, int64_t n_out,
                                int nmv, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t j;
  int a;
  row_col(t, nmv, j, a);
  if (j >= n_out) return;
  const int64_t c = owner_of(off_out, C, (uint32_t)j);
  const uint32_t k0 = off_in[c] + ((uint32_t)j - off_out[c]) * kSegChunk;
  const uint32_t k1 = min(off_in[c + 1], k0 + kSegChunk);
  double s = 0.0;
  for (uint32_t k = k0; k < k1; ++k) s += (double)in[(int64_t)k * in_stride + a];
  out[j * nmv + a] = s;
}

// Lists with per-entry orders: the records of a cell are sorted by order
// (key = cell << 4 | q); items are runs of at most kCellItemGroups records of
// one order. Per cell, the end of the order-q records is the first key above
// (cell << 4 | q), found by binary search within the cell's range.
__device__ __forceinline__ uint32_t order_end(const uint64_t* __restrict__ key, uint32_t lo,
                                              uint32_t hi, uint64_t k) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// (ish: image bits below the order when the lists are periodic). Also keeps
// the record boundaries of the cell's order runs: bnd[c][0] = first record,
// bnd[c][q + 1] = one past its order-q records.
constexpr int kBnd = kMaxP + 2;
__global__ void k_cq_count(const uint64_t* __restrict__ key, const uint32_t* __restrict__ rec_off,
                           int64_t C, int ish, uint32_t* __restrict__ nit,
                           uint32_t* __restrict__ bnd) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const uint32_t hi = rec_off[c + 1];
  uint32_t b = rec_off[c], n = 0;
  bnd[c * kBnd] = b;
  for (int q = 0; q <= kMaxP; ++q) {
    const uint32_t e = order_end(key, b, hi, (((uint64_t)c << 4) | (uint64_t)(q + 1)) << ish);
    n += (e - b + kCellItemGroups - 1) / kCellItemGroups;
    bnd[c * kBnd + q + 1] = e;
    b = e;
  }
  nit[c] = n;
}

// one thread per item: its cell, its order run and its records
__global__ void k_cq_items(const uint32_t* __restrict__ bnd, const uint32_t* __restrict__ it_off,
                           int64_t C, int64_t n_items, uint32_t* __restrict__ citem_rec,
                           uint32_t* __restrict__ citem_end, int32_t* __restrict__ citem_cell,
                           uint64_t* __restrict__ qkey, uint32_t* __restrict__ qval) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_items) return;
  const int64_t c = owner_of(it_off, C, (uint32_t)k);
  const uint32_t* bc = bnd + c * kBnd;
  uint32_t local = (uint32_t)k - it_off[c];
  for (int q = 0; q <= kMaxP; ++q) {
    const uint32_t b = bc[q], e = bc[q + 1];
    const uint32_t n = (e - b + kCellItemGroups - 1) / kCellItemGroups;
    if (local < n) {
      const uint32_t r = b + local * kCellItemGroups;
      citem_rec[k] = r;
      citem_end[k] = r + kCellItemGroups < e ? r + kCellItemGroups : e;
      citem_cell[k] = (int32_t)c;
      qkey[k] = (uint64_t)q;
      qval[k] = (uint32_t)k;
      return;
    }
    local -= n;
  }
}

// ------------------------------------------------------------------- gathers
template <typename T>
// sorted cotangents, and three times them for the source-side pair kernel
__global__ void k_abar(const double* __restrict__ abar, const uint32_t* __restrict__ perm,
                       int64_t n, V4<T>* __restrict__ ab, V4<T>* __restrict__ ab3) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  V4<T> v;
  v.x = (T)abar[3 * j];
  v.y = (T)abar[3 * j + 1];
  v.z = (T)abar[3 * j + 2];
  v.w = T(0);
  ab[i] = v;
  v.x = T(3) * v.x;
  v.y = T(3) * v.y;
  v.z = T(3) * v.z;
  ab3[i] = v;
}

// ------------------------------------------------------- pair terms, sink side
// state per sorted particle: s_x s_y s_z - c_x c_y c_z -
// The group's list comes as its pair segments, as in the forward pair kernel.
template <typename T, bool EPS0, bool K1>
__global__ __launch_bounds__(kB) void k_p2p_sink_adj(
    const int2* __restrict__ items, int64_t n_items, const int64_t* __restrict__ pseg_off,
    const PairSeg* __restrict__ pseg, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const V4<T>* __restrict__ off,
    const V4<T>* __restrict__ ab4, T eps2, T ie, const unsigned* __restrict__ mdiff,
    T* __restrict__ state) {
  __shared__ V4<T> stage[kWPB][64];
  // K1: eps2 is the squared kernel radius, ie its inverse radius
  const T ie2 = ie * ie, ie3 = ie * ie2, ie5t = (ie3 * ie2) * (T(1) / T(3));
  // every particle of the same mass: the pair loop leaves the mass out and
  // the segment's sums are scaled once
  const bool uni = *mdiff == 0u;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V4<T>* slot = stage[w];
  const int64_t it = (int64_t)blockIdx.x * kWPB + w;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int gend = g_first[g] + g_count[g];
  // m x n blocking with n = 2 as in the forward pair kernel: lane l holds
  // sinks item.y + (l & 31) (A) and item.y + 32 + (l & 31) (B), half h = l / 32
  // takes the sources of index parity h; lane l keeps the compensated sums
  // of sink item.y + l
  const int h = lane >> 5, sub = lane & 31;
  const int iA = item.y + sub, iB = iA + 32;
  const int i = item.y + lane;
  const bool active = i < gend;
  V4<T> mA, mB, bA, bB;
  mA.x = mA.y = mA.z = mA.w = T(0);
  mB = bA = bB = mA;
  if (iA < gend) {
    mA = off[iA];
    bA = ab4[iA];
  }
  if (iB < gend) {
    mB = off[iB];
    bB = ab4[iB];
  }
  const T a3Ax = T(3) * bA.x, a3Ay = T(3) * bA.y, a3Az = T(3) * bA.z;
  const T a3Bx = T(3) * bB.x, a3By = T(3) * bB.y, a3Bz = T(3) * bB.z;
  T sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0;
  // per sink: sum m inv3 ; sum 3 m (r.ab) inv5 r, in plain FP32 over
  // consecutive segments until at least kSumRun sources are summed, then the
  // halves are added (lane l < 32 completes sink A, lane l >= 32 sink B) and
  // xbar_i -= m_j H ab = -(sum m inv3) ab + sum 3 m rd inv5 r goes into the
  // compensated sums with one compensated add
  T pA = 0, qAx = 0, qAy = 0, qAz = 0;
  T pB = 0, qBx = 0, qBy = 0, qBz = 0;
  T mseg = T(1);
  int n_acc = 0;
#define HOT_SINK_FLUSH                                                               \
  {                                                                                  \
    const T kp = (h ? pB : pA) + __shfl_xor(h ? pA : pB, 32);                        \
    const T kx = (h ? qBx : qAx) + __shfl_xor(h ? qAx : qBx, 32);                    \
    const T ky = (h ? qBy : qAy) + __shfl_xor(h ? qAy : qBy, 32);                    \
    const T kz = (h ? qBz : qAz) + __shfl_xor(h ? qAz : qBz, 32);                    \
    const V4<T> ab = h ? bB : bA;                                                    \
    kahan_add(sx, cx, hot_fma(-kp, ab.x, kx) * mseg);                                \
    kahan_add(sy, cy, hot_fma(-kp, ab.y, ky) * mseg);                                \
    kahan_add(sz, cz, hot_fma(-kp, ab.z, kz) * mseg);                                \
    pA = qAx = qAy = qAz = T(0);                                                     \
    pB = qBx = qBy = qBz = T(0);                                                     \
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
      // sources in batches of 64 staged through the wavefront's LDS slot
      // (one coalesced load per lane, read back two sources a read)
#define HOT_SINK_PAIR(SELF, UM, VALID, SINK_I, TX, TY, TZ, A3X, A3Y, A3Z, A, Bx, By, Bz) \
  {                                                                                  \
    const T rx = s.x + TX, ry = s.y + TY, rz = s.z + TZ;                             \
    if constexpr (!K1) {                                                             \
      const T r2 = hot_fma(rx, rx, hot_fma(ry, ry, hot_fma(rz, rz, eps2)));          \
      T inv = (EPS0 && !(r2 > T(0))) ? T(0) : hot_rsq(r2);                           \
      if (!(VALID) || (SELF && jb + k == (SINK_I))) inv = T(0);                      \
      const T inv2 = inv * inv;                                                      \
      const T m3 = UM ? inv * inv2 : s.w * (inv * inv2);                             \
      const T rd3 = hot_fma(rx, A3X, hot_fma(ry, A3Y, rz * A3Z));                    \
      const T q = m3 * (rd3 * inv2);                                                 \
      A += m3;                                                                       \
      Bx = hot_fma(q, rx, Bx);                                                       \
      By = hot_fma(q, ry, By);                                                       \
      Bz = hot_fma(q, rz, Bz);                                                       \
    } else {                                                                         \
      /* K I + B r r^T with kq = K and bb = -B / 3 */                                \
      const T r2 = hot_fma(rx, rx, hot_fma(ry, ry, rz * rz));                        \
      const T inv = hot_rsq(r2);                                                     \
      const T inv2 = inv * inv;                                                      \
      T kq = inv * inv2;                                                             \
      T bb = kq * inv2;                                                              \
      if (r2 < eps2) {                                                               \
        const T v = (eps2 - r2) * ie2;                                               \
        kq = ie3 * k1_force(v);                                                      \
        bb = ie5t * k1_hess(v);                                                      \
      }                                                                              \
      if (!UM) {                                                                     \
        kq *= s.w;                                                                   \
        bb *= s.w;                                                                   \
      }                                                                              \
      if (!(VALID) || (SELF && jb + k == (SINK_I))) {                                \
        kq = T(0);                                                                   \
        bb = T(0);                                                                   \
      }                                                                              \
      const T rd3 = hot_fma(rx, A3X, hot_fma(ry, A3Y, rz * A3Z));                    \
      const T q = bb * rd3;                                                          \
      A += kq;                                                                       \
      Bx = hot_fma(q, rx, Bx);                                                       \
      By = hot_fma(q, ry, By);                                                       \
      Bz = hot_fma(q, rz, Bz);                                                       \
    }                                                                                \
  }
#define HOT_SINK_BATCH(UM, SELF)                                                     \
  {                                                                                  \
    int k2 = 0;                                                                      \
    _Pragma("unroll 2") for (; k2 + 1 < nbt; k2 += 2) {                              \
      const int k = k2 + h;                                                          \
      const V4<T> s = slot[k];                                                       \
      HOT_SINK_PAIR(SELF, UM, true, iA, tAx, tAy, tAz, a3Ax, a3Ay, a3Az, pA, qAx, qAy, qAz) \
      HOT_SINK_PAIR(SELF, UM, true, iB, tBx, tBy, tBz, a3Bx, a3By, a3Bz, pB, qBx, qBy, qBz) \
    }                                                                                \
    if (k2 < nbt) {                                                                  \
      const int k = k2 + h;                                                          \
      const V4<T> s = slot[k2];                                                      \
      HOT_SINK_PAIR(SELF, UM, h == 0, iA, tAx, tAy, tAz, a3Ax, a3Ay, a3Az, pA, qAx, qAy, qAz) \
      HOT_SINK_PAIR(SELF, UM, h == 0, iB, tBx, tBy, tBz, a3Bx, a3By, a3Bz, pB, qBx, qBy, qBz) \
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
            HOT_SINK_BATCH(true, true)
          else
            HOT_SINK_BATCH(true, false)
          mseg = slot[0].w;
        } else {
          if (self)
            HOT_SINK_BATCH(false, true)
          else
            HOT_SINK_BATCH(false, false)
        }
      }
#undef HOT_SINK_BATCH
#undef HOT_SINK_PAIR
      n_acc += jend - j;
      if (n_acc >= kSumRun) HOT_SINK_FLUSH
    }
  }
  if (n_acc > 0) HOT_SINK_FLUSH
#undef HOT_SINK_FLUSH
  if (active) {
    T* st = state + (int64_t)i * 8;
    st[0] = sx;
    st[1] = sy;
    st[2] = sz;
    st[4] = cx;
    st[5] = cy;
    st[6] = cz;
  }
}

// ------------------------------------------------- expansion terms, sink side
// MIXQ: per-entry orders (error-bound lists); PER: per-entry images (periodic)
// The FP32 order-8 kernel is held to three waves per SIMD (168 VGPRs): the
// periodic variants otherwise take a few registers more and drop to two.
template <int P, typename T>
constexpr int sink_adj_waves_per_simd() { return (sizeof(T) == 4 && P == 8) ? 3 : 1; }

// BG: background subtraction; an entry flagged in m2p_sub takes its cell's
// cube-subtracted moments (momsub) instead of momw.
template <int P, typename T, bool MIXQ, bool PER, bool BG, bool K1>
__global__ __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(sink_adj_waves_per_simd<P, T>())))
void k_m2p_sink_adj(
    const int2* __restrict__ items, int64_t n_items, const int64_t* __restrict__ m2p_off,
    const int32_t* __restrict__ m2p, const int8_t* __restrict__ m2p_q,
    const int8_t* __restrict__ m2p_img, double side,
    const int8_t* __restrict__ c_level,
    const int32_t* __restrict__ g_first, const int32_t* __restrict__ g_count,
    const int32_t* __restrict__ g_cell, const double* __restrict__ c_centre,
    const V4<T>* __restrict__ off, const V4<T>* __restrict__ ab4, const T* __restrict__ momw,
    double inv_side, double eps, T* __restrict__ state, const int8_t* __restrict__ m2p_sub,
    const T* __restrict__ momsub) {
  using Stage = MomentStage<P, T>;
  __shared__ T smom[Stage::kLds ? kWPB * Stage::kStride : 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * kWPB + w;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int gend = g_first[g] + g_count[g];
  const int i = item.y + lane;
  const bool active = i < gend;
  const int gc = g_cell[g];
  const double cgx = c_centre[3 * gc], cgy = c_centre[3 * gc + 1], cgz = c_centre[3 * gc + 2];
  V4<T> me, ab;
  me.x = me.y = me.z = me.w = T(0);
  ab = me;
  T sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0;
  if (active) {
    me = off[i];
    ab = ab4[i];
    const T* st = state + (int64_t)i * 8;
    sx = st[0];
    sy = st[1];
    sz = st[2];
    cx = st[4];
    cy = st[5];
    cz = st[6];
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
    T gx = 0, gy = 0, gz = 0;
    if (MIXQ)
      expansion_sink_adj_q<P, T, K1>(q, X, Y, Z, (T)(es * es), M, ab.x, ab.y, ab.z, gx, gy, gz);
    else
      expansion_sink_adj<P, T, K1>(X, Y, Z, (T)(es * es), M, ab.x, ab.y, ab.z, gx, gy, gz);
    const T sc = (T)(-(inv_s * inv_s * inv_s));
    kahan_add(sx, cx, gx * sc);
    kahan_add(sy, cy, gy * sc);
    kahan_add(sz, cz, gz * sc);
  }
  if (active) {
    T* st = state + (int64_t)i * 8;
    st[0] = sx;
    st[1] = sy;
    st[2] = sz;
    st[4] = cx;
    st[5] = cy;
    st[6] = cz;
  }
}

// Sink-side expansion terms for an item of at most 32 sinks (theta lists
// without background subtraction), split like the forward's k_m2p_sl: slices
// of W = max(8, 2^ceil(log2 n_sinks)) lanes take interleaved list entries, the
// round's cells' coefficients staged together in LDS, and the slices'
// compensated sums are added at the end. Every cross-lane read is executed by
// all lanes.
template <int P, typename T, bool PER, bool K1>
__global__ __launch_bounds__(64) void k_m2p_sink_adj_sl(
    const int2* __restrict__ items, int64_t n_items, const int64_t* __restrict__ m2p_off,
    const int32_t* __restrict__ m2p, const int8_t* __restrict__ m2p_img, double side,
    const int8_t* __restrict__ c_level, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const int32_t* __restrict__ g_cell,
    const double* __restrict__ c_centre, const V4<T>* __restrict__ off,
    const V4<T>* __restrict__ ab4, const T* __restrict__ momw, double inv_side, double eps,
    T* __restrict__ state) {
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
  V4<T> me, ab;
  me.x = me.y = me.z = me.w = T(0);
  ab = me;
  if (active) {
    me = off[i];
    ab = ab4[i];
  }
  T sx = 0, sy = 0, sz = 0, cx = 0, cy = 0, cz = 0;
  if (active && sl == 0) {
    const T* st = state + (int64_t)i * 8;
    sx = st[0];
    sy = st[1];
    sz = st[2];
    cx = st[4];
    cy = st[5];
    cz = st[6];
  }
  const int64_t e0 = m2p_off[g], e1 = m2p_off[g + 1];
  for (int64_t eb = e0; eb < e1; eb += S) {
    int cl = -1, il = kCentreImage;
    if (lane < S && eb + lane < e1) {
      cl = m2p[eb + lane];
      if (PER) il = m2p_img[eb + lane];
    }
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
    T gx = 0, gy = 0, gz = 0;
    expansion_sink_adj<P, T, K1>(X, Y, Z, (T)(es * es), M, ab.x, ab.y, ab.z, gx, gy, gz);
    const T sc = ok ? (T)(-(inv_s * inv_s * inv_s)) : T(0);
    kahan_add(sx, cx, gx * sc);
    kahan_add(sy, cy, gy * sc);
    kahan_add(sz, cz, gz * sc);
  }
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
  }
  if (active && sl == 0) {
    T* st = state + (int64_t)i * 8;
    st[0] = sx;
    st[1] = sy;
    st[2] = sz;
    st[4] = cx;
    st[5] = cy;
    st[6] = cz;
  }
}

// ----------------------------------------------------- pair terms, source side
// One wavefront per source item (at most 64 particles of one group). The
// records of the item are sorted by sink group; runs of one group are merged
// into a lane mask (the lanes whose particles lie in one of that group's P2P
// cells). With more than 32 such lanes, lanes are the item's particles and the
// group's sinks are swept uniformly. With k <= 32 of them, the k particles are
// packed into the first W = 2^ceil(log2 k) lanes and the wavefront splits into
// 64 / W slices that sweep interleaved subsets of the sinks, so a group that
// pair-sums only a leaf or two of the item costs n_sinks W / 64 iterations
// instead of n_sinks; the slices' sums are then added across lanes and handed
// back to the particles' own lanes.
// out per sorted particle: s_x s_y s_z s_m c_x c_y c_z c_m
template <typename T, bool EPS0, bool PER, bool K1>
__global__ __launch_bounds__(kB) void k_p2p_src_adj(
    const int4* __restrict__ units, int64_t n_units, const int2* __restrict__ items,
    const uint64_t* __restrict__ skey, const uint32_t* __restrict__ sval, uint64_t gmask,
    const int32_t* __restrict__ p2p, const int8_t* __restrict__ p2p_img, double side,
    const int32_t* __restrict__ c_first,
    const int32_t* __restrict__ c_count, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const int32_t* __restrict__ g_cell,
    const double* __restrict__ c_centre, const V4<T>* __restrict__ off,
    const V4<T>* __restrict__ ab3, T eps2, T ie, T* __restrict__ out, T* __restrict__ part) {
  __shared__ V4<T> stage[kWPB][128];
  // K1: eps2 is the squared kernel radius, ie its inverse radius
  const T ie2 = ie * ie, ie3 = ie * ie2, ie5 = ie3 * ie2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V4<T>* slot = stage[w];
  const int64_t wu = (int64_t)blockIdx.x * kWPB + w;
  if (wu >= n_units) return;
  const int4 unit = units[wu];
  const int2 item = items[uniform_i32(unit.x)];
  const uint32_t r0 = (uint32_t)uniform_i32(unit.y), r1 = (uint32_t)uniform_i32(unit.z);
  const int gs = uniform_i32(item.x);
  const int j = item.y + lane;
  const bool active = j < g_first[gs] + g_count[gs];
  const int gsc = g_cell[gs];
  const double csx = c_centre[3 * gsc], csy = c_centre[3 * gsc + 1], csz = c_centre[3 * gsc + 2];
  V4<T> me;
  me.x = me.y = me.z = me.w = T(0);
  if (active) me = off[j];
  T sx = 0, sy = 0, sz = 0, sm = 0, cx = 0, cy = 0, cz = 0, cm = 0;
  // three times the pair sums: with b = 3 abar_i and d = r . b,
  // 3 H abar = s^-3/2 (b - 3 d r s^-1) and 3 abar . r s^-3/2 = d s^-3/2
#define HOT_SRC_PAIR(SI, B, TX, TY, TZ, ZERO)                                        \
  {                                                                                  \
    const T rx = (TX) - (SI).x, ry = (TY) - (SI).y, rz = (TZ) - (SI).z;              \
    if constexpr (!K1) {                                                             \
      const T r2 = hot_fma(rx, rx, hot_fma(ry, ry, hot_fma(rz, rz, eps2)));          \
      T inv = (EPS0 && !(r2 > T(0))) ? T(0) : hot_rsq(r2);                           \
      if (ZERO) inv = T(0);                                                          \
      const T inv2 = inv * inv;                                                      \
      const T inv3 = inv * inv2;                                                     \
      const T d = hot_fma(rx, (B).x, hot_fma(ry, (B).y, rz * (B).z));                \
      const T dd = (T(3) * d) * inv2;                                                \
      gx = hot_fma(inv3, hot_fma(-dd, rx, (B).x), gx);                               \
      gy = hot_fma(inv3, hot_fma(-dd, ry, (B).y), gy);                               \
      gz = hot_fma(inv3, hot_fma(-dd, rz, (B).z), gz);                               \
      gm = hot_fma(d, inv3, gm);                                                     \
    } else {                                                                         \
      /* 3 H abar = K b + B d r with kq = K, bn = -B */                              \
      const T r2 = hot_fma(rx, rx, hot_fma(ry, ry, rz * rz));                        \
      const T inv = hot_rsq(r2);                                                     \
      const T inv2 = inv * inv;                                                      \
      T kq = inv * inv2;                                                             \
      T bn = T(3) * (kq * inv2);                                                     \
      if (r2 < eps2) {                                                               \
        const T v = (eps2 - r2) * ie2;                                               \
        kq = ie3 * k1_force(v);                                                      \
        bn = ie5 * k1_hess(v);                                                       \
      }                                                                              \
      if (ZERO) {                                                                    \
        kq = T(0);                                                                   \
        bn = T(0);                                                                   \
      }                                                                              \
      const T d = hot_fma(rx, (B).x, hot_fma(ry, (B).y, rz * (B).z));                \
      const T bd = bn * d;                                                           \
      gx = hot_fma(kq, (B).x, hot_fma(-bd, rx, gx));                                 \
      gy = hot_fma(kq, (B).y, hot_fma(-bd, ry, gy));                                 \
      gz = hot_fma(kq, (B).z, hot_fma(-bd, rz, gz));                                 \
      gm = hot_fma(d, kq, gm);                                                       \
    }                                                                                \
  }
  // Records are read in batches of 64, one per lane, so that their loads
  // overlap; position r1 is an end marker that closes the last run. A run is
  // the records of one sink group (and image); mine marks the lanes whose
  // particle lies in one of the run's cells.
  int g = -1, im0 = -1;
  bool mine = false;
  for (uint32_t base = r0; base <= r1; base += 64) {
    const uint32_t rl = base + lane;
    int lg = -1, lim = -1, lf = 0, lc = 0;
    if (rl < r1) {
      const uint32_t e = sval[rl];
      const int c = p2p[e];
      lg = (int)(skey[rl] & gmask);
      lf = c_first[c];
      lc = c_count[c];
      lim = PER ? (int)p2p_img[e] : kCentreImage;
    }
    const int nb = (int)(r1 + 1 - base < 64u ? r1 + 1 - base : 64u);
    for (int bq = 0; bq < nb; ++bq) {
      const int gb = __builtin_amdgcn_readlane(lg, bq);
      const int imb = __builtin_amdgcn_readlane(lim, bq);
      if (gb != g || imb != im0) {
        mine = mine && active;
        const uint64_t mask = __ballot(mine);
        const int k = __popcll(mask);
        if (g >= 0 && k > 0) {
          // sweep the finished run's sink group
          const int gc = uniform_i32(g_cell[g]);
          T dx, dy, dz;  // source group centre minus sink group centre
          if (PER) {
            double shx, shy, shz;
            image_shift(im0, side, shx, shy, shz);
            dx = (T)((csx + shx) - c_centre[3 * gc]);
            dy = (T)((csy + shy) - c_centre[3 * gc + 1]);
            dz = (T)((csz + shz) - c_centre[3 * gc + 2]);
          } else {
            dx = (T)(csx - c_centre[3 * gc]);
            dy = (T)(csy - c_centre[3 * gc + 1]);
            dz = (T)(csz - c_centre[3 * gc + 2]);
          }
          const int i0 = uniform_i32(g_first[g]);
          const int i1 = i0 + uniform_i32(g_count[g]);
          const bool self = g == gs && im0 == kCentreImage;
          T gx = 0, gy = 0, gz = 0, gm = 0;
          if (k > 32) {
            // lanes are the item's particles, sinks wavefront-uniform:
            // r_ij = x_j - x_i = t - off_i; the sinks (offsets and scaled
            // cotangents) staged through LDS in batches of 64
            const T tx = dx + me.x, ty = dy + me.y, tz = dz + me.z;
            for (int ib = i0; ib < i1; ib += 64) {
              const int nbt = i1 - ib < 64 ? i1 - ib : 64;
              V4<T> v, bv;
              v.x = v.y = v.z = v.w = T(0);
              bv = v;
              if (lane < nbt) {
                v = off[ib + lane];
                bv = ab3[ib + lane];
              }
              __builtin_amdgcn_wave_barrier();
              slot[lane] = v;
              slot[64 + lane] = bv;
              __builtin_amdgcn_wave_barrier();
              if (self) {
                for (int kk = 0; kk < nbt; ++kk) {
                  const V4<T> si = slot[kk];
                  const V4<T> b = slot[64 + kk];
                  HOT_SRC_PAIR(si, b, tx, ty, tz, ib + kk == j)
                }
              } else {
#pragma unroll 4
                for (int kk = 0; kk < nbt; ++kk) {
                  const V4<T> si = slot[kk];
                  const V4<T> b = slot[64 + kk];
                  HOT_SRC_PAIR(si, b, tx, ty, tz, false)
                }
              }
            }
          } else {
            // rank of each marked lane among the marked lanes below it; a
            // stable partition (marked lanes first) tells packed lane p its
            // source lane
            const int below = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            const int dest = mine ? below : k + (lane - below);
            const int src_of = __builtin_amdgcn_ds_permute(dest << 2, lane);
            const int lw = k <= 1 ? 0 : 32 - __clz(k - 1);
            const int p = lane & ((1 << lw) - 1);
            const int sl = lane >> lw;  // slice
            const int S = 64 >> lw;
            const int sp = __shfl(src_of, p);
            const bool pact = p < k;
            const int jp = item.y + sp;
            const T tx = dx + __shfl(me.x, sp), ty = dy + __shfl(me.y, sp),
                    tz = dz + __shfl(me.z, sp);
            for (int ib = i0; ib < i1; ib += 64) {
              const int nbt = i1 - ib < 64 ? i1 - ib : 64;
              V4<T> v, bv;
              v.x = v.y = v.z = v.w = T(0);
              bv = v;
              if (lane < nbt) {
                v = off[ib + lane];
                bv = ab3[ib + lane];
              }
              __builtin_amdgcn_wave_barrier();
              slot[lane] = v;
              slot[64 + lane] = bv;
              __builtin_amdgcn_wave_barrier();
#pragma unroll 2
              for (int kb = 0; kb < nbt; kb += S) {
                const int kk = kb + sl;
                const bool ok = pact && kk < nbt;
                const int kc = ok ? kk : 0;
                const V4<T> si = slot[kc];
                const V4<T> b = slot[64 + kc];
                HOT_SRC_PAIR(si, b, tx, ty, tz, !ok || (self && ib + kk == jp))
              }
            }
            // sum over the slices; packed lane 'below' of slice 0 then holds
            // the marked lane's totals
#pragma unroll
            for (int m = 32; m > 0; m >>= 1) {
              if (m < (1 << lw)) break;
              gx += __shfl_xor(gx, m);
              gy += __shfl_xor(gy, m);
              gz += __shfl_xor(gz, m);
              gm += __shfl_xor(gm, m);
            }
            gx = __shfl(gx, below);
            gy = __shfl(gy, below);
            gz = __shfl(gz, below);
            gm = __shfl(gm, below);
          }
          if (mine) {
            const T third = T(1) / T(3);
            const T mw = me.w * third;
            kahan_add(sx, cx, mw * gx);
            kahan_add(sy, cy, mw * gy);
            kahan_add(sz, cz, mw * gz);
            kahan_add(sm, cm, gm * third);
          }
        }
        g = gb;
        im0 = imb;
        mine = false;
      }
      if (gb >= 0) {
        const int f = __builtin_amdgcn_readlane(lf, bq);
        mine = mine || ((j >= f) && (j < f + __builtin_amdgcn_readlane(lc, bq)));
      }
    }
  }
#undef HOT_SRC_PAIR
  T* o = nullptr;
  if (unit.w) {
    if (active) o = out + (int64_t)j * 8;  // the item's only unit
  } else {
    o = part + (wu * 64 + lane) * 8;  // summed over the item's units later
  }
  if (o) {
    o[0] = sx;
    o[1] = sy;
    o[2] = sz;
    o[3] = sm;
    o[4] = cx;
    o[5] = cy;
    o[6] = cz;
    o[7] = cm;
  }
}

// Items with several units: per particle, the units' (sum, compensation) pairs
// added in FP64 in unit order, written back as one pair.
template <typename T>
__global__ void k_src_unit_sum(const int2* __restrict__ items, int64_t n_items,
                               const uint32_t* __restrict__ unit_off,
                               const int32_t* __restrict__ g_first,
                               const int32_t* __restrict__ g_count, const T* __restrict__ part,
                               T* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = t >> 6;
  const int l = (int)(t & 63);
  if (q >= n_items) return;
  const uint32_t u0 = unit_off[q], u1 = unit_off[q + 1];
  if (u1 - u0 <= 1) return;
  const int2 it = items[q];
  const int j = it.y + l;
  if (j >= g_first[it.x] + g_count[it.x]) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t v = u0; v < u1; ++v) {
    const T* a = part + ((int64_t)v * 64 + l) * 8;
    for (int k = 0; k < 4; ++k) acc[k] += (double)a[k] - (double)a[4 + k];
  }
  T* o = out + (int64_t)j * 8;
  for (int k = 0; k < 4; ++k) {
    const T hi = (T)acc[k];
    o[k] = hi;
    o[4 + k] = (T)((double)hi - acc[k]);
  }
}

// ---------------------------------------- expansion terms, moment cotangents
// One wavefront per cell item (a run of at most kCellItemGroups groups whose
// M2P lists hold the cell); lanes are the item's sinks, its groups
// concatenated, 64 at a time. Each
// lane accumulates sum_k abar_k d^(alpha+e_k) G for all alpha in registers; the
// item's partial sums are reduced across lanes with a fixed butterfly.
// P: the expansion order of the item's records. MIXQ (lists with per-entry
// orders): the block's item is qitems[qbase + block], its records end at
// citem_end, and the row is written with stride out_stride, zero-filled from
// nm(P) up to out_nm (the cell's full moment count).
template <int P, typename T, bool MIXQ, bool PER, bool K1>
__global__ __launch_bounds__(64) void k_m2p_cell_adj(
    int64_t n_citems, const uint32_t* __restrict__ citem_rec, const int32_t* __restrict__ citem_cell,
    const uint32_t* __restrict__ crec_off, const uint32_t* __restrict__ qitems, int64_t qbase,
    const uint32_t* __restrict__ citem_end, int out_stride, int out_nm,
    const uint64_t* __restrict__ mkey, double side, const uint32_t* __restrict__ mval,
    const int8_t* __restrict__ c_level, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const int32_t* __restrict__ g_cell,
    const double* __restrict__ c_centre, const V4<T>* __restrict__ off,
    const V4<T>* __restrict__ ab4, double inv_side, double eps, T* __restrict__ part) {
  constexpr int NM = nm(P);
  const int lane = threadIdx.x;
  if ((int64_t)blockIdx.x >= n_citems) return;
  const int64_t it = MIXQ ? (int64_t)qitems[qbase + blockIdx.x] : (int64_t)blockIdx.x;
  const int c = citem_cell[it];
  const uint32_t r0 = citem_rec[it];
  uint32_t r1;
  if (MIXQ) {
    r1 = citem_end[it];
  } else {
    const uint32_t rc = crec_off[c + 1];
    r1 = r0 + kCellItemGroups < rc ? r0 + kCellItemGroups : rc;
  }
  const double inv_s = ldexp(inv_side, (int)c_level[c]);
  const double es = eps * inv_s;
  const T e2 = (T)(es * es);
  const double ccx = c_centre[3 * c], ccy = c_centre[3 * c + 1], ccz = c_centre[3 * c + 2];
  T row[NM];
#pragma unroll
  for (int a = 0; a < NM; ++a) row[a] = T(0);
  // The item's sinks, all its records' groups concatenated, in chunks of 64
  // lanes (groups of few sinks then fill the wavefront together: every sink
  // sees the same cell). Per record, staged in LDS by one lane each: the
  // running sink count, the group's first sink and the scaled difference of
  // the group centre from the (image of the) cell centre.
  __shared__ int s_cum[kCellItemGroups + 1];
  __shared__ int s_first[kCellItemGroups];
  __shared__ T s_d[3][kCellItemGroups];
  const int nr = (int)(r1 - r0);  // at most kCellItemGroups < 64
  int cnt = 0;
  if (lane < nr) {
    const uint32_t r = r0 + (uint32_t)lane;
    const int g = (int)mval[r];
    const int gc = g_cell[g];
    double shx = 0.0, shy = 0.0, shz = 0.0;
    // the record's image of the cell sits at its centre + n L
    if (PER) image_shift((int)(mkey[r] & 127u), side, shx, shy, shz);
    s_d[0][lane] = (T)((c_centre[3 * gc] - (ccx + shx)) * inv_s);
    s_d[1][lane] = (T)((c_centre[3 * gc + 1] - (ccy + shy)) * inv_s);
    s_d[2][lane] = (T)((c_centre[3 * gc + 2] - (ccz + shz)) * inv_s);
    s_first[lane] = g_first[g];
    cnt = g_count[g];
  }
  int inc = cnt;  // inclusive running count over the lanes
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane < nr) s_cum[lane + 1] = inc;
  if (lane == 0) s_cum[0] = 0;
  const int total = nr > 0 ? __shfl(inc, nr - 1) : 0;
  __syncthreads();
  // sink t of the concatenation: record k with s_cum[k] <= t < s_cum[k + 1]
  // (the same number of halvings on every lane), its offset and cotangent
  auto fetch = [&](int t, T& X, T& Y, T& Z, T& bx, T& by, T& bz) {
    X = T(1);
    Y = Z = bx = by = bz = T(0);
    if (t < total) {
      int lo = 0, hi = nr;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_cum[mid] <= t)
          lo = mid;
        else
          hi = mid;
      }
      const int si = s_first[lo] + (t - s_cum[lo]);
      const V4<T> me = off[si];
      const V4<T> ab = ab4[si];
      X = s_d[0][lo] + me.x * (T)inv_s;
      Y = s_d[1][lo] + me.y * (T)inv_s;
      Z = s_d[2][lo] + me.z * (T)inv_s;
      bx = ab.x;
      by = ab.y;
      bz = ab.z;
    }
  };
  // one loop over the chunks with the next chunk's data fetched ahead; a
  // single back edge keeps the row registers in place across iterations
  T X, Y, Z, bx, by, bz;
  fetch(lane, X, Y, Z, bx, by, bz);
  for (int t0 = 0; t0 < total; t0 += 64) {
    const T cX = X, cY = Y, cZ = Z, cbx = bx, cby = by, cbz = bz;
    if (t0 + 64 < total) fetch(t0 + 64 + lane, X, Y, Z, bx, by, bz);
    expansion_cell_adj<P, T, K1>(cX, cY, cZ, e2, cbx, cby, cbz, row);
  }
  T* o = part + it * (int64_t)(MIXQ ? out_stride : nm_pad(P));
  // Sum the rows over the 64 lanes as a reduce-scatter: the row vector, padded
  // with zeros to 64 KR entries, is halved six times; at each step a lane keeps
  // one half (selected by its lane bit), receives the partner's copy of it and
  // adds. Lane l ends with the sums of rows KR l .. KR l + KR - 1, after
  // 32 KR + 16 KR + ... + KR exchanges instead of 6 per row.
  constexpr int KR = (NM + 63) / 64;
  T v[64 * KR];
#pragma unroll
  for (int a = 0; a < 64 * KR; ++a) v[a] = a < NM ? row[a] : T(0);
#pragma unroll
  for (int m = 32, h = 32 * KR; m > 0; m >>= 1, h >>= 1) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const T lo = v[i], hi = v[i + h];
      const T send = up ? lo : hi;
      const T keep = up ? hi : lo;
      v[i] = keep + __shfl_xor(send, m);
    }
  }
#pragma unroll
  for (int i = 0; i < KR; ++i)
    if (KR * lane + i < NM) o[KR * lane + i] = v[i];
  if (MIXQ)
    for (int a = NM + lane; a < out_nm; a += 64) o[a] = T(0);
}

// Mbar_alpha(c) = -w_alpha s^(-2-|alpha|) * sum over the cell's items (in order).
template <typename T>
__global__ void k_mbar_final(const T* __restrict__ part, int stride,
                             const uint32_t* __restrict__ it_off, int64_t C,
                             const int8_t* __restrict__ c_level, double inv_side, int p,
                             double* __restrict__ mbar) {
  const int nmv = nm(p);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c;
  int a;
  row_col(t, nmv, c, a);
  if (c >= C) return;
  double s = 0.0;
  for (uint32_t k = it_off[c]; k < it_off[c + 1]; ++k) s += (double)part[(int64_t)k * stride + a];
  const int order = kAlpha.a[a] + kAlpha.b[a] + kAlpha.c[a];
  const double sc = pow2_pow(ldexp(inv_side, (int)c_level[c]), order + 2);
  mbar[c * nmv + a] = -kAlpha.w[a] * sc * s;
}

// M2M transpose for one level: child Mbar += shift^T of the parent's Mbar.
#define HOT_M2MT_CASE(P, N)                                                \
  case N: {                                                                \
    double acc[((N) + 1) * ((N) + 2) / 2];                                 \
    _Pragma("unroll") for (int k = 0; k < ((N) + 1) * ((N) + 2) / 2; ++k) acc[k] = 0.0; \
    m2mT_p##P##_order##N(Mb, dx, dy, dz, acc);                             \
    double* out = mbar + c * NMV + (N) * ((N) + 1) * ((N) + 2) / 6;        \
    _Pragma("unroll") for (int k = 0; k < ((N) + 1) * ((N) + 2) / 2; ++k) out[k] += acc[k]; \
  } break;

template <int P>
__global__ __launch_bounds__(kB) void k_m2mT(int64_t c0, int64_t c1,
                                             const int32_t* __restrict__ parent,
                                             const double* __restrict__ c_centre,
                                             double* __restrict__ mbar) {
  constexpr int NMV = nm(P);
  int64_t run;
  int N;
  order_block(P, run, N);
  const int64_t c = c0 + run * kB + threadIdx.x;
  if (c >= c1) return;
  const int pa = parent[c];
  const double dx = c_centre[3 * c] - c_centre[3 * pa];
  const double dy = c_centre[3 * c + 1] - c_centre[3 * pa + 1];
  const double dz = c_centre[3 * c + 2] - c_centre[3 * pa + 2];
  const double* Mb = mbar + (int64_t)pa * NMV;
  if constexpr (P == 0) {
    switch (N) { HOT_M2MT_CASE(0, 0) }
  } else if constexpr (P == 1) {
    switch (N) { HOT_M2MT_CASE(1, 0) HOT_M2MT_CASE(1, 1) }
  } else if constexpr (P == 2) {
    switch (N) { HOT_M2MT_CASE(2, 0) HOT_M2MT_CASE(2, 1) HOT_M2MT_CASE(2, 2) }
  } else if constexpr (P == 3) {
    switch (N) { HOT_M2MT_CASE(3, 0) HOT_M2MT_CASE(3, 1) HOT_M2MT_CASE(3, 2) HOT_M2MT_CASE(3, 3) }
  } else if constexpr (P == 4) {
    switch (N) {
      HOT_M2MT_CASE(4, 0) HOT_M2MT_CASE(4, 1) HOT_M2MT_CASE(4, 2) HOT_M2MT_CASE(4, 3)
      HOT_M2MT_CASE(4, 4)
    }
  } else if constexpr (P == 5) {
    switch (N) {
      HOT_M2MT_CASE(5, 0) HOT_M2MT_CASE(5, 1) HOT_M2MT_CASE(5, 2) HOT_M2MT_CASE(5, 3)
      HOT_M2MT_CASE(5, 4) HOT_M2MT_CASE(5, 5)
    }
  } else if constexpr (P == 6) {
    switch (N) {
      HOT_M2MT_CASE(6, 0) HOT_M2MT_CASE(6, 1) HOT_M2MT_CASE(6, 2) HOT_M2MT_CASE(6, 3)
      HOT_M2MT_CASE(6, 4) HOT_M2MT_CASE(6, 5) HOT_M2MT_CASE(6, 6)
    }
  } else if constexpr (P == 7) {
    switch (N) {
      HOT_M2MT_CASE(7, 0) HOT_M2MT_CASE(7, 1) HOT_M2MT_CASE(7, 2) HOT_M2MT_CASE(7, 3)
      HOT_M2MT_CASE(7, 4) HOT_M2MT_CASE(7, 5) HOT_M2MT_CASE(7, 6) HOT_M2MT_CASE(7, 7)
    }
  } else {
    switch (N) {
      HOT_M2MT_CASE(8, 0) HOT_M2MT_CASE(8, 1) HOT_M2MT_CASE(8, 2) HOT_M2MT_CASE(8, 3)
      HOT_M2MT_CASE(8, 4) HOT_M2MT_CASE(8, 5) HOT_M2MT_CASE(8, 6) HOT_M2MT_CASE(8, 7)
      HOT_M2MT_CASE(8, 8)
    }
  }
}

// P2M transpose at the leaves: xbar_j += m_j sum_alpha Mbar alpha_k d^(alpha-e_k),
// mbar_j += sum_alpha Mbar d^alpha, d = x_j - leaf centre (FP64).
template <int P>
__global__ __launch_bounds__(kB) void k_p2mT(const double* __restrict__ spos,
                                             const double* __restrict__ smass, int64_t n,
                                             const int32_t* __restrict__ leaf_of,
                                             const double* __restrict__ c_centre,
                                             const double* __restrict__ mbar,
                                             double* __restrict__ xb, double* __restrict__ mb) {
  constexpr int NMV = nm(P);
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (j >= n) return;
  const int lf = leaf_of[j];
  const double dx = spos[j] - c_centre[3 * lf], dy = spos[n + j] - c_centre[3 * lf + 1],
               dz = spos[2 * n + j] - c_centre[3 * lf + 2];
  double gx = 0, gy = 0, gz = 0, gm = 0;
  const double* Mb = mbar + (int64_t)lf * NMV;
  if constexpr (P == 0) p2mT_p0(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 1) p2mT_p1(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 2) p2mT_p2(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 3) p2mT_p3(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 4) p2mT_p4(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 5) p2mT_p5(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 6) p2mT_p6(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 7) p2mT_p7(Mb, dx, dy, dz, gx, gy, gz, gm);
  if constexpr (P == 8) p2mT_p8(Mb, dx, dy, dz, gx, gy, gz, gm);
  const double m = smass[j];
  xb[3 * j] = m * gx;
  xb[3 * j + 1] = m * gy;
  xb[3 * j + 2] = m * gz;
  mb[j] = gm;
}

template <typename T>
__global__ void k_adj_finalize(const T* __restrict__ sink, const T* __restrict__ src,
                               const double* __restrict__ xb, const double* __restrict__ mb,
                               const uint32_t* __restrict__ perm, int64_t n,
                               double* __restrict__ xbar, double* __restrict__ mbar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T* a = sink + i * 8;
  const T* b = src + i * 8;
  const int64_t j = perm[i];
  for (int d = 0; d < 3; ++d)
    xbar[3 * j + d] = (((double)a[d] - (double)a[4 + d]) + ((double)b[d] - (double)b[4 + d])) +
                      xb[3 * i + d];
  if (mbar) mbar[j] = ((double)b[3] - (double)b[7]) + mb[i];
}

// ------------------------------------------------------------- host drivers
void build_transpose(hot_ctx* ctx, hot_tree* t) {
  hipStream_t st = ctx->stream;
  const int64_t G = t->n_groups, C = t->n_cells, NI = t->n_items;
  // ---- pair records by source item
  {
    DBuf cnt, tot;
    cnt.alloc(ctx, (G + 1) * sizeof(int64_t));
    tot.alloc(ctx, sizeof(int64_t));
    k_srec_count<<<grid_for(G, kWPB), kB, 0, st>>>(t->p2p_off.as<int64_t>(), t->p2p.as<int32_t>(), G,
                                                 t->c_first.as<int32_t>(), t->c_count.as<int32_t>(),
                                                 t->item_of.as<int32_t>(), cnt.as<int64_t>());
    HOT_CHECK_LAUNCH();
    scan_i64(ctx, cnt.as<int64_t>(), cnt.as<int64_t>(), G, tot.as<int64_t>());
    int64_t nrec = 0;
    HOT_HIP(hipMemcpyAsync(&nrec, tot.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HOT_HIP(hipStreamSynchronize(st));
    if (nrec >= (int64_t)INT32_MAX - 128) throw Error{HOT_E_CAPACITY, "too many P2P records"};
    t->n_srec = nrec;
    const int gbits = bits_for(G);
    const int qbits = bits_for(NI);
    if (gbits + qbits > 63) throw Error{HOT_E_CAPACITY, "P2P record key too wide"};
    t->srec_key.alloc(ctx, std::max<int64_t>(1, nrec) * sizeof(uint64_t));
    t->srec_val.alloc(ctx, std::max<int64_t>(1, nrec) * sizeof(uint32_t));
    t->srec_off.alloc(ctx, (NI + 1) * sizeof(uint32_t));
    k_srec_fill<<<grid_for(G, kWPB), kB, 0, st>>>(
        t->p2p_off.as<int64_t>(), t->p2p.as<int32_t>(), G, t->c_first.as<int32_t>(),
        t->c_count.as<int32_t>(), t->item_of.as<int32_t>(), cnt.as<int64_t>(), gbits,
        t->srec_key.as<uint64_t>(), t->srec_val.as<uint32_t>());
    HOT_CHECK_LAUNCH();
    // the records are written group by group in increasing group order, so a
    // stable sort on the item bits alone orders them by (item, group)
    radix_sort(ctx, t->srec_key, t->srec_val, nrec, gbits + qbits, gbits);
    k_lower_bound<<<grid_for(NI + 1, kB), kB, 0, st>>>(t->srec_key.as<uint64_t>(), nrec, gbits, NI,
                                                       t->srec_off.as<uint32_t>());
    HOT_CHECK_LAUNCH();
    t->srec_gbits = gbits;
    // work units of the source-side kernel
    t->schunk_off.alloc(ctx, (NI + 1) * sizeof(uint32_t));
    DBuf ucnt;
    ucnt.alloc(ctx, (NI + 1) * sizeof(uint32_t));
    const uint32_t chunk = src_chunk(nrec);
    k_sunit_count<<<grid_for(NI, kB), kB, 0, st>>>(t->srec_off.as<uint32_t>(), NI, chunk,
                                                   ucnt.as<uint32_t>());
    HOT_CHECK_LAUNCH();
    // exclusive offsets of the NI items, the total in the last slot
    uint32_t* uoff = t->schunk_off.as<uint32_t>();
    scan_u32(ctx, ucnt.as<uint32_t>(), uoff, NI, uoff + NI);
    uint32_t nu = 0;
    HOT_HIP(hipMemcpyAsync(&nu, uoff + NI, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HOT_HIP(hipStreamSynchronize(st));
    t->n_schunk = nu;
    t->schunk.alloc(ctx, std::max<int64_t>(1, (int64_t)nu) * sizeof(int4));
    k_sunit_fill<<<grid_for(NI, kB), kB, 0, st>>>(t->srec_off.as<uint32_t>(), NI, chunk,
                                                  t->schunk_off.as<uint32_t>(),
                                                  t->schunk.as<int4>());
    HOT_CHECK_LAUNCH();
  }
  // ---- expansion records by source cell, split into items
  {
    const int64_t E = t->n_m2p;
    t->n_mrec = E;
    t->mrec_key.alloc(ctx, std::max<int64_t>(1, E) * sizeof(uint64_t));
    t->mrec_val.alloc(ctx, std::max<int64_t>(1, E) * sizeof(uint32_t));
    t->mcell_rec.alloc(ctx, (C + 1) * sizeof(uint32_t));
    t->mcell_item.alloc(ctx, (C + 1) * sizeof(uint32_t));
    const int qsh = t->list_p >= 0 ? 4 : 0;  // order bits below the cell id
    const int ish = t->periodic ? 7 : 0;       // image bits below the cell id
    k_mrec_fill<<<grid_for(G, kWPB), kB, 0, st>>>(
        t->m2p_off.as<int64_t>(), t->m2p.as<int32_t>(),
        t->list_p >= 0 ? t->m2p_q.as<int8_t>() : nullptr,
        t->periodic ? t->m2p_img.as<int8_t>() : nullptr, G, t->mrec_key.as<uint64_t>(),
        t->mrec_val.as<uint32_t>());
    HOT_CHECK_LAUNCH();
    radix_sort(ctx, t->mrec_key, t->mrec_val, E,
               bits_for(C) + qsh + ish);
    k_lower_bound<<<grid_for(C + 1, kB), kB, 0, st>>>(t->mrec_key.as<uint64_t>(), E, qsh + ish, C,
                                                      t->mcell_rec.as<uint32_t>());
    HOT_CHECK_LAUNCH();
    DBuf bnd;
    if (qsh) {
      bnd.alloc(ctx, (size_t)C * kBnd * sizeof(uint32_t));
      k_cq_count<<<grid_for(C, kB), kB, 0, st>>>(t->mrec_key.as<uint64_t>(),
                                                 t->mcell_rec.as<uint32_t>(), C, ish,
                                                 t->mcell_item.as<uint32_t>(), bnd.as<uint32_t>());
    } else {
      k_items_from_off<<<grid_for(C, kB), kB, 0, st>>>(t->mcell_rec.as<uint32_t>(), C,
                                                       t->mcell_item.as<uint32_t>());
    }
    HOT_CHECK_LAUNCH();
    scan_u32(ctx, t->mcell_item.as<uint32_t>(), t->mcell_item.as<uint32_t>(), C,
             t->mcell_item.as<uint32_t>() + C);
    uint32_t nci = 0;
    HOT_HIP(hipMemcpyAsync(&nci, t->mcell_item.as<uint32_t>() + C, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, st));
    HOT_HIP(hipStreamSynchronize(st));
    t->n_citems = nci;
    t->citem_rec.alloc(ctx, std::max<int64_t>(1, nci) * sizeof(uint32_t));
    t->citem_cell.alloc(ctx, std::max<int64_t>(1, nci) * sizeof(int32_t));
    if (qsh) {
      // items of one order each, then their ids sorted by order
      t->citem_end.alloc(ctx, std::max<int64_t>(1, nci) * sizeof(uint32_t));
      t->qitems.alloc(ctx, std::max<int64_t>(1, nci) * sizeof(uint32_t));
      DBuf qkey, qoff;
      qkey.alloc(ctx, std::max<int64_t>(1, nci) * sizeof(uint64_t));
      qoff.alloc(ctx, (kMaxP + 2) * sizeof(uint32_t));
      if (nci > 0) {
        k_cq_items<<<grid_for(nci, kB), kB, 0, st>>>(
            bnd.as<uint32_t>(), t->mcell_item.as<uint32_t>(), C, nci, t->citem_rec.as<uint32_t>(),
            t->citem_end.as<uint32_t>(), t->citem_cell.as<int32_t>(), qkey.as<uint64_t>(),
            t->qitems.as<uint32_t>());
        HOT_CHECK_LAUNCH();
      }
      radix_sort(ctx, qkey, t->qitems, nci, 4);
      k_lower_bound<<<1, kB, 0, st>>>(qkey.as<uint64_t>(), nci, 0, kMaxP + 1, qoff.as<uint32_t>());
      HOT_CHECK_LAUNCH();
      uint32_t h[kMaxP + 2];
      HOT_HIP(hipMemcpyAsync(h, qoff.p, sizeof(h), hipMemcpyDeviceToHost, st));
      HOT_HIP(hipStreamSynchronize(st));
      for (int q = 0; q <= kMaxP + 1; ++q) t->qitem_off[q] = h[q];
    } else {
      t->citem_end.release();
      t->qitems.release();
      if (nci > 0) {
        k_cell_items<<<grid_for(nci, kB), kB, 0, st>>>(t->mcell_rec.as<uint32_t>(),
                                                       t->mcell_item.as<uint32_t>(), C, nci,
                                                       t->citem_rec.as<uint32_t>(),
                                                       t->citem_cell.as<int32_t>());
        HOT_CHECK_LAUNCH();
      }
    }
    // rounds of the cells' partial sums: while some cell has more than
    // kSegChunk values, chunk offsets for the next round
    t->mred_levels = 0;
    const uint32_t* off = t->mcell_item.as<uint32_t>();
    DBuf dmax;
    dmax.alloc(ctx, sizeof(unsigned));
    for (int lev = 0; lev < 3; ++lev) {
      k_zero_u32<<<1, 1, 0, st>>>(dmax.as<unsigned>());
      HOT_CHECK_LAUNCH();
      t->mred_off[lev].alloc(ctx, (C + 1) * sizeof(uint32_t));
      k_seg_count<<<grid_for(C, kB), kB, 0, st>>>(off, C, t->mred_off[lev].as<uint32_t>(),
                                                  dmax.as<unsigned>());
      HOT_CHECK_LAUNCH();
      unsigned mx = 0;
      HOT_HIP(hipMemcpyAsync(&mx, dmax.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
      HOT_HIP(hipStreamSynchronize(st));
      if (mx <= (unsigned)kSegChunk) break;
      scan_u32(ctx, t->mred_off[lev].as<uint32_t>(), t->mred_off[lev].as<uint32_t>(), C,
               t->mred_off[lev].as<uint32_t>() + C);
      uint32_t n_out = 0;
      HOT_HIP(hipMemcpyAsync(&n_out, t->mred_off[lev].as<uint32_t>() + C, sizeof(uint32_t),
                             hipMemcpyDeviceToHost, st));
      HOT_HIP(hipStreamSynchronize(st));
      t->mred_n[lev] = n_out;
      t->mred_levels = lev + 1;
      off = t->mred_off[lev].as<uint32_t>();
    }
  }
  t->has_transpose = true;
}

// expansion terms, sink side (needs no transposed lists)
template <int P, typename T, bool K1>
void launch_expansion_sink_adj(hot_ctx* ctx, hot_tree* t, const V4<T>* off, const V4<T>* ab,
                               const T* momw, const T* momsub, double eps, T* sink_state) {
  hipStream_t st = ctx->stream;
  const double inv_side = 1.0 / t->side;
  const bool mixq = t->list_p >= 0;
  tmark(ctx, HOT_T_ADJ_M2P_SINK, false);
  auto sink = [&](auto kern) {
    kern<<<grid_for(t->n_items, kWPB), kB, 0, st>>>(
        t->items.as<int2>(), t->n_items, t->m2p_off.as<int64_t>(), t->m2p.as<int32_t>(),
        t->m2p_q.as<int8_t>(), t->m2p_img.as<int8_t>(), t->side, t->c_level.as<int8_t>(),
        t->g_first.as<int32_t>(), t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(),
        t->c_centre.as<double>(), off, ab, momw, inv_side, eps, sink_state,
        t->m2p_sub.as<int8_t>(), momsub);
    HOT_CHECK_LAUNCH();
  };
  if (!t->bg && !mixq && t->n_items_small >= 0 && t->n_items_small * 10 >= t->n_items) {
    // many part-empty items (split by the forward evaluation): those of at
    // most 32 sinks by slices of one wavefront, the others as usual
    if (t->n_items_big > 0) {
      auto kb = t->periodic ? k_m2p_sink_adj<P, T, false, true, false, K1> : k_m2p_sink_adj<P, T, false, false, false, K1>;
      kb<<<grid_for(t->n_items_big, kWPB), kB, 0, st>>>(
          t->items_big.as<int2>(), t->n_items_big, t->m2p_off.as<int64_t>(), t->m2p.as<int32_t>(),
          t->m2p_q.as<int8_t>(), t->m2p_img.as<int8_t>(), t->side, t->c_level.as<int8_t>(),
          t->g_first.as<int32_t>(), t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(),
          t->c_centre.as<double>(), off, ab, momw, inv_side, eps, sink_state,
          t->m2p_sub.as<int8_t>(), momsub);
      HOT_CHECK_LAUNCH();
    }
    if (t->n_items_small > 0) {
      auto ks = t->periodic ? k_m2p_sink_adj_sl<P, T, true, K1> : k_m2p_sink_adj_sl<P, T, false, K1>;
      ks<<<(unsigned)t->n_items_small, 64, 0, st>>>(
          t->items_small.as<int2>(), t->n_items_small, t->m2p_off.as<int64_t>(),
          t->m2p.as<int32_t>(), t->m2p_img.as<int8_t>(), t->side, t->c_level.as<int8_t>(),
          t->g_first.as<int32_t>(), t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(),
          t->c_centre.as<double>(), off, ab, momw, inv_side, eps, sink_state);
      HOT_CHECK_LAUNCH();
    }
  } else if (t->bg)
    sink(k_m2p_sink_adj<P, T, false, true, true, K1>);
  else if (mixq && t->periodic)
    sink(k_m2p_sink_adj<P, T, true, true, false, K1>);
  else if (mixq)
    sink(k_m2p_sink_adj<P, T, true, false, false, K1>);
  else if (t->periodic)
    sink(k_m2p_sink_adj<P, T, false, true, false, K1>);
  else
    sink(k_m2p_sink_adj<P, T, false, false, false, K1>);
  tmark(ctx, HOT_T_ADJ_M2P_SINK, true);
}

// expansion terms, the moment cotangents (cell side, on the transposed
// lists), then down the tree
template <int P, typename T, bool K1>
void launch_expansion_cell_adj(hot_ctx* ctx, hot_tree* t, const V4<T>* off, const V4<T>* ab,
                               double eps, double* mbar64, const double* pos,
                               const double* abar) {
  hipStream_t st = ctx->stream;
  const double inv_side = 1.0 / t->side;
  const bool mixq = t->list_p >= 0;
  const int64_t C = t->n_cells;
  DBuf part;
  part.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_citems) * nm_pad(P) * sizeof(T));
  tmark(ctx, HOT_T_ADJ_M2P_CELL, false);
  if (t->n_citems > 0) {
    auto cell = [&](auto kern, int64_t n, int64_t base) {
      if (n <= 0) return;
      kern<<<(unsigned)n, 64, 0, st>>>(
          n, t->citem_rec.as<uint32_t>(), t->citem_cell.as<int32_t>(), t->mcell_rec.as<uint32_t>(),
          t->qitems.as<uint32_t>(), base, t->citem_end.as<uint32_t>(), nm_pad(P), nm(P),
          t->mrec_key.as<uint64_t>(), t->side, t->mrec_val.as<uint32_t>(), t->c_level.as<int8_t>(), t->g_first.as<int32_t>(),
          t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(), t->c_centre.as<double>(), off, ab,
          inv_side, eps, part.as<T>());
      HOT_CHECK_LAUNCH();
    };
    if (mixq) {
      // one launch per order present: each kernel holds only its order's row
      const int64_t* qo = t->qitem_off;
#define HOT_CELL_Q(Q) \
  if constexpr (Q <= P) {                                                       \
    if (t->periodic)                                                            \
      cell(k_m2p_cell_adj<Q, T, true, true, K1>, qo[Q + 1] - qo[Q], qo[Q]);         \
    else                                                                        \
      cell(k_m2p_cell_adj<Q, T, true, false, K1>, qo[Q + 1] - qo[Q], qo[Q]);        \
  }
      HOT_CELL_Q(0) HOT_CELL_Q(1) HOT_CELL_Q(2) HOT_CELL_Q(3) HOT_CELL_Q(4) HOT_CELL_Q(5)
      HOT_CELL_Q(6) HOT_CELL_Q(7) HOT_CELL_Q(8)
#undef HOT_CELL_Q
    } else {
      if (t->periodic)
        cell(k_m2p_cell_adj<P, T, false, true, K1>, t->n_citems, 0);
      else
        cell(k_m2p_cell_adj<P, T, false, false, K1>, t->n_citems, 0);
    }
  }
  const int64_t tot = C * nm(P);
  if (t->mred_levels == 0) {
    k_mbar_final<T><<<grid_for(tot, kB), kB, 0, st>>>(part.as<T>(), nm_pad(P),
                                                      t->mcell_item.as<uint32_t>(), C,
                                                      t->c_level.as<int8_t>(), inv_side, P, mbar64);
    HOT_CHECK_LAUNCH();
  } else {
    // cells with many items: chunked rounds, then the final sum per cell
    DBuf red[2];
    const uint32_t* off_in = t->mcell_item.as<uint32_t>();
    const double* in64 = nullptr;
    for (int lev = 0; lev < t->mred_levels; ++lev) {
      const int64_t n_out = t->mred_n[lev];
      DBuf& out = red[lev & 1];
      out.alloc(ctx, (size_t)std::max<int64_t>(1, n_out) * nm(P) * sizeof(double));
      const unsigned grid = grid_for(n_out * nm(P), kB);
      if (lev == 0)
        k_seg_chunk_sum<T><<<grid, kB, 0, st>>>(part.as<T>(), nm_pad(P), off_in,
                                                t->mred_off[lev].as<uint32_t>(), C, n_out, nm(P),
                                                out.as<double>());
      else
        k_seg_chunk_sum<double><<<grid, kB, 0, st>>>(in64, nm(P), off_in,
                                                     t->mred_off[lev].as<uint32_t>(), C, n_out,
                                                     nm(P), out.as<double>());
      HOT_CHECK_LAUNCH();
      off_in = t->mred_off[lev].as<uint32_t>();
      in64 = out.as<double>();
    }
    k_mbar_final<double><<<grid_for(tot, kB), kB, 0, st>>>(in64, nm(P), off_in, C,
                                                           t->c_level.as<int8_t>(), inv_side, P,
                                                           mbar64);
    HOT_CHECK_LAUNCH();
  }
  tmark(ctx, HOT_T_ADJ_M2P_CELL, true);
  tmark(ctx, HOT_T_ADJ_DOWNWARD, false);
  // far periodic replicas: their cotangent of the root's moments (cell 0)
  if (t->periodic) far_replicas_mbar(ctx, t, pos, abar, mbar64);
  // down the tree: level L+1 cells take their parents' cotangents
  for (int L = 1; L <= t->max_level; ++L) {
    const int64_t c0 = t->level_off[L], c1 = t->level_off[L + 1];
    if (c1 <= c0) continue;
    k_m2mT<P><<<order_grid(grid_for(c1 - c0, kB), P), kB, 0, st>>>(c0, c1, t->c_parent.as<int32_t>(), t->c_centre.as<double>(),
                                   mbar64);
    HOT_CHECK_LAUNCH();
  }
}

template <int P>
void launch_p2mT(hot_ctx* ctx, hot_tree* t, const double* spos, const double* smass,
                 const double* mbar64, double* xb, double* mb) {
  k_p2mT<P><<<grid_for(t->n, kB), kB, 0, ctx->stream>>>(spos, smass, t->n, t->leaf_of.as<int32_t>(),
                                                        t->c_centre.as<double>(), mbar64, xb, mb);
  HOT_CHECK_LAUNCH();
}

template <typename T, bool K1>
void launch_expansion_sink_adj_k(hot_ctx* ctx, hot_tree* t, const V4<T>* o4, const V4<T>* a4,
                                 const T* momw, const T* momsub, double eps, T* S) {
  switch (t->p) {
#define HOT_EXP_ADJ(Q) \
  case Q: launch_expansion_sink_adj<Q, T, K1>(ctx, t, o4, a4, momw, momsub, eps, S); break;
    HOT_EXP_ADJ(0) HOT_EXP_ADJ(1) HOT_EXP_ADJ(2) HOT_EXP_ADJ(3) HOT_EXP_ADJ(4) HOT_EXP_ADJ(5)
    HOT_EXP_ADJ(6) HOT_EXP_ADJ(7) HOT_EXP_ADJ(8)
#undef HOT_EXP_ADJ
    default: invalid("p out of range");
  }
}

template <typename T, bool K1>
void launch_expansion_cell_adj_k(hot_ctx* ctx, hot_tree* t, const V4<T>* o4, const V4<T>* a4,
                                 double eps, double* M, const double* pos, const double* abar) {
  switch (t->p) {
#define HOT_EXP_ADJ(Q) \
  case Q: launch_expansion_cell_adj<Q, T, K1>(ctx, t, o4, a4, eps, M, pos, abar); break;
    HOT_EXP_ADJ(0) HOT_EXP_ADJ(1) HOT_EXP_ADJ(2) HOT_EXP_ADJ(3) HOT_EXP_ADJ(4) HOT_EXP_ADJ(5)
    HOT_EXP_ADJ(6) HOT_EXP_ADJ(7) HOT_EXP_ADJ(8)
#undef HOT_EXP_ADJ
    default: invalid("p out of range");
  }
}

// The transposed lists on the context's second stream: it starts after all
// work queued on the main stream so far (the lists), the sink-side kernels
// queued on the main stream next run meanwhile, and join() makes the main
// stream wait for it before anything that reads the transposed lists. The
// transposes allocate, run and free on the second stream (the context's
// stream is switched for the duration); on an error the second stream is
// drained before the error propagates.
struct TransposeAside {
  hot_ctx* ctx;
  hipStream_t main;
  bool active = false;
  TransposeAside(hot_ctx* c, bool need) : ctx(c), main(c->stream) {
    if (!need) return;
    if (!ctx->aux) {
      HOT_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
      for (auto& e : ctx->xev) HOT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    HOT_HIP(hipEventRecord(ctx->xev[0], main));
    HOT_HIP(hipStreamWaitEvent(ctx->aux, ctx->xev[0], 0));
    active = true;
  }
  // build the transposed lists on the second stream (the main stream keeps
  // running what was queued on it)
  void build(hot_tree* t) {
    if (!active) return;
    ctx->stream = ctx->aux;
    try {
      Phase ph(ctx, HOT_T_ADJ_TRANSPOSE);
      build_transpose(ctx, t);
    } catch (...) {
      ctx->stream = main;
      (void)hipStreamSynchronize(ctx->aux);
      active = false;
      throw;
    }
    ctx->stream = main;
  }
  void join() {
    if (!active) return;
    HOT_HIP(hipEventRecord(ctx->xev[1], ctx->aux));
    HOT_HIP(hipStreamWaitEvent(main, ctx->xev[1], 0));
    active = false;
  }
  ~TransposeAside() {
    if (active) {
      // an error between build and join: nothing may outlive the call
      ctx->stream = main;
      (void)hipStreamSynchronize(ctx->aux);
    }
  }
};

template <typename T>
void adjoint_t(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
               int precision, const double* abar, double* xbar, double* mbar) {
  const bool k1 = use_k1(precision, eps);
  hipStream_t st = ctx->stream;
  const int64_t n = t->n, C = t->n_cells;
  const int p = t->p;
  // the transposed lists (source side) are built beside the sink-side work
  TransposeAside aside(ctx, !t->has_transpose);
  DBuf off, ab, ab3, sink, src, mbar64, spos, smass, xb, mb;
  off.alloc(ctx, n * sizeof(V4<T>));
  ab.alloc(ctx, n * sizeof(V4<T>));
  ab3.alloc(ctx, n * sizeof(V4<T>));
  sink.alloc(ctx, n * 8 * sizeof(T));
  src.alloc(ctx, n * 8 * sizeof(T));
  mbar64.alloc(ctx, (size_t)C * nm(p) * sizeof(double));
  spos.alloc(ctx, 3 * n * sizeof(double));
  smass.alloc(ctx, n * sizeof(double));
  xb.alloc(ctx, 3 * n * sizeof(double));
  mb.alloc(ctx, n * sizeof(double));
  zero_flag_word(ctx, kFlagMass);
  k_offsets<T><<<grid_for(n, kB), kB, 0, st>>>(pos, mass, t->perm.as<uint32_t>(),
                                               t->group_of.as<int32_t>(), t->g_cell.as<int32_t>(),
                                               t->c_centre.as<double>(), n, off.as<V4<T>>(),
                                               ctx->d_flags, ctx->d_flags + kFlagMass);
  HOT_CHECK_LAUNCH();
  k_abar<T><<<grid_for(n, kB), kB, 0, st>>>(abar, t->perm.as<uint32_t>(), n, ab.as<V4<T>>(),
                                            ab3.as<V4<T>>());
  HOT_CHECK_LAUNCH();
  gather_sorted(ctx, t, pos, mass, spos.as<double>(), smass.as<double>(), 0);
  const T e2 = (T)(eps * eps);
  const T ie = k1 ? (T)(1.0 / eps) : T(0);
  const unsigned gi = grid_for(t->n_items, kWPB);
  // pair terms
  auto sink_k = k1 ? k_p2p_sink_adj<T, false, true>
                    : (e2 > T(0) ? k_p2p_sink_adj<T, false, false> : k_p2p_sink_adj<T, true, false>);
  tmark(ctx, HOT_T_ADJ_P2P_SINK, false);
  sink_k<<<gi, kB, 0, st>>>(t->items.as<int2>(), t->n_items, t->pseg_off.as<int64_t>(),
                            t->pseg.as<PairSeg>(), t->g_first.as<int32_t>(),
                            t->g_count.as<int32_t>(), off.as<V4<T>>(), ab.as<V4<T>>(), e2, ie,
                            ctx->d_flags + kFlagMass, sink.as<T>());
  HOT_CHECK_LAUNCH();
  tmark(ctx, HOT_T_ADJ_P2P_SINK, true);
  // expansion terms
  const T* momw = nullptr;
  const T* momsub = nullptr;
  if (t->bg) {
    weighted_sub(ctx, t, sizeof(T) == 8);
    momsub = t->momsub.as<T>();
  }
  if constexpr (sizeof(T) == 4) {
    momw = t->mom32.as<T>();
  } else {
    weighted_fp64(ctx, t);
    momw = t->momw64.as<T>();
  }
  V4<T>* o4 = off.as<V4<T>>();
  V4<T>* a4 = ab.as<V4<T>>();
  double* M = mbar64.as<double>();
  T* S = sink.as<T>();
  if (k1)
    launch_expansion_sink_adj_k<T, true>(ctx, t, o4, a4, momw, momsub, eps, S);
  else
    launch_expansion_sink_adj_k<T, false>(ctx, t, o4, a4, momw, momsub, eps, S);
  // the source side reads the transposed lists
  aside.build(t);
  aside.join();
  auto src_k = k1 ? (t->periodic ? k_p2p_src_adj<T, false, true, true>
                                 : k_p2p_src_adj<T, false, false, true>)
             : t->periodic ? (e2 > T(0) ? k_p2p_src_adj<T, false, true, false>
                                        : k_p2p_src_adj<T, true, true, false>)
                           : (e2 > T(0) ? k_p2p_src_adj<T, false, false, false>
                                        : k_p2p_src_adj<T, true, false, false>);
  const int64_t NU = t->n_schunk;
  DBuf upart;
  if (NU > t->n_items) upart.alloc(ctx, (size_t)NU * 64 * 8 * sizeof(T));
  tmark(ctx, HOT_T_ADJ_P2P_SOURCE, false);
  src_k<<<grid_for(NU, kWPB), kB, 0, st>>>(
      t->schunk.as<int4>(), NU, t->items.as<int2>(), t->srec_key.as<uint64_t>(),
      t->srec_val.as<uint32_t>(), (1ull << t->srec_gbits) - 1ull, t->p2p.as<int32_t>(),
      t->p2p_img.as<int8_t>(), t->side, t->c_first.as<int32_t>(), t->c_count.as<int32_t>(),
      t->g_first.as<int32_t>(), t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(),
      t->c_centre.as<double>(), off.as<V4<T>>(), ab3.as<V4<T>>(), e2, ie, src.as<T>(),
      upart.as<T>());
  HOT_CHECK_LAUNCH();
  if (NU > t->n_items) {
    k_src_unit_sum<T><<<grid_for(t->n_items * 64, kB), kB, 0, st>>>(
        t->items.as<int2>(), t->n_items, t->schunk_off.as<uint32_t>(), t->g_first.as<int32_t>(),
        t->g_count.as<int32_t>(), upart.as<T>(), src.as<T>());
    HOT_CHECK_LAUNCH();
  }
  tmark(ctx, HOT_T_ADJ_P2P_SOURCE, true);
  if (k1)
    launch_expansion_cell_adj_k<T, true>(ctx, t, o4, a4, eps, M, pos, abar);
  else
    launch_expansion_cell_adj_k<T, false>(ctx, t, o4, a4, eps, M, pos, abar);
  const double* sp = spos.as<double>();
  const double* sm = smass.as<double>();
  switch (p) {
    case 0: launch_p2mT<0>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 1: launch_p2mT<1>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 2: launch_p2mT<2>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 3: launch_p2mT<3>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 4: launch_p2mT<4>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 5: launch_p2mT<5>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 6: launch_p2mT<6>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 7: launch_p2mT<7>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
    case 8: launch_p2mT<8>(ctx, t, sp, sm, M, xb.as<double>(), mb.as<double>()); break;
  }
  k_adj_finalize<T><<<grid_for(n, kB), kB, 0, st>>>(sink.as<T>(), src.as<T>(), xb.as<double>(),
                                                    mb.as<double>(), t->perm.as<uint32_t>(), n,
                                                    xbar, mbar);
  HOT_CHECK_LAUNCH();
  // far periodic replicas: their direct dependence on the sink position
  if (t->periodic) far_replicas_xbar(ctx, t, pos, abar, xbar);
  // background subtraction: the exact box fields and the mean density
  if (t->bg) background_adjoint(ctx, t, pos, mass, eps, precision, abar, xbar, mbar);
  tmark(ctx, HOT_T_ADJ_DOWNWARD, true);
}

}  // namespace

void adjoint(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
             int precision, const double* abar, double* xbar, double* mbar) {
  if (fp64_mode(precision))
    adjoint_t<double>(ctx, t, pos, mass, eps, precision, abar, xbar, mbar);
  else
    adjoint_t<float>(ctx, t, pos, mass, eps, precision, abar, xbar, mbar);
}

}  // namespace hot
