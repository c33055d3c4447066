// Tree build: root cube, Morton keys, sort, hashed oct-tree cells, b_max and
// sink groups.
//
// Domain Decomposition section: coordinates map to integer keys and the keys
// are sorted. Tree Construction and Traversal section: cells are labelled by
// their keys and found through a hash table ("hcells"). The paper points to a
// sort-and-scan construction for GPUs; this is one: every particle i knows,
// from its sorted neighbours alone, at which levels it starts a cell, so all
// cells of all levels are produced by one counting pass, one scan and one
// scatter, already in (level, key) order.
#include "common.h"

namespace hot {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

// Number of leading octal digits two keys share (0..21).
__device__ __forceinline__ int lcp_level(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0) return kMaxLevel;
  const int h = 63 - __clzll((long long)x);
  return 20 - h / 3;
}

// floor((x - lo) * 2^21 / side), clamped to [0, 2^21 - 1]. The scale is a
// power of two, so only the subtraction rounds.
__device__ __forceinline__ uint32_t quantise(double x, double lo, double scale) {
  double t = floor((x - lo) * scale);
  if (t > 2097151.0) t = 2097151.0;
  if (!(t >= 0.0)) t = 0.0;
  return (uint32_t)t;
}

__device__ __forceinline__ void cell_centre(uint64_t prefix, int level, const double* root,
                                            double c[3]) {
  const uint64_t digits = level ? (prefix & ((1ull << (3 * level)) - 1)) : 0ull;
  const uint32_t ix = compact3(digits >> 2), iy = compact3(digits >> 1), iz = compact3(digits);
  const double h = ldexp(root[3], -(level + 1));
  c[0] = root[0] + (double)(2u * ix + 1u) * h;
  c[1] = root[1] + (double)(2u * iy + 1u) * h;
  c[2] = root[2] + (double)(2u * iz + 1u) * h;
}

__global__ __launch_bounds__(kB) void k_bbox_partial(const double* __restrict__ pos, int64_t n,
                                                     double* __restrict__ part,
                                                     unsigned* __restrict__ flags) {
  __shared__ double sh[6][kB];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = pos[3 * i + d];
      bad |= !isfinite(x);
      mn[d] = fmin(mn[d], x);
      mx[d] = fmax(mx[d], x);
    }
  }
  if (bad) atomicOr(flags, FLAG_NONFINITE_POS);
  for (int d = 0; d < 3; ++d) {
    sh[d][threadIdx.x] = mn[d];
    sh[3 + d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int off = kB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + off]);
        sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + off]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// Root cube: lo = per-axis minimum; side = the power of two at or above the
// largest extent (1 if all points coincide). root = lo[3], side, 2^21/side.
__global__ void k_bbox_final(const double* __restrict__ part, int nparts, double* __restrict__ root) {
  if (threadIdx.x != 0) return;
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = 0; b < nparts; ++b)
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], part[6 * b + d]);
      mx[d] = fmax(mx[d], part[6 * b + 3 + d]);
    }
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) ext = fmax(ext, mx[d] - mn[d]);
  double side = 1.0;
  if (ext > 0.0) {
    int e;
    const double m = frexp(ext, &e);
    side = (m == 0.5) ? ext : ldexp(1.0, e);
  }
  root[0] = mn[0];
  root[1] = mn[1];
  root[2] = mn[2];
  root[3] = side;
  root[4] = 2097152.0 / side;
}

__global__ void k_box_check(const double* __restrict__ pos, int64_t n,
                            const double* __restrict__ root, unsigned* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool bad = false, out = false;
  for (int d = 0; d < 3; ++d) {
    const double x = pos[3 * i + d];
    bad |= !isfinite(x);
    out |= !(x >= root[d] && x <= root[d] + root[3]);
  }
  if (bad) atomicOr(flags, FLAG_NONFINITE_POS);
  if (out) atomicOr(flags, FLAG_OUTSIDE_BOX);
}

__global__ void k_keys(const double* __restrict__ pos, int64_t n, const double* __restrict__ root,
                       uint64_t* __restrict__ key, uint32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double scale = root[4];
  const uint32_t qx = quantise(pos[3 * i], root[0], scale);
  const uint32_t qy = quantise(pos[3 * i + 1], root[1], scale);
  const uint32_t qz = quantise(pos[3 * i + 2], root[2], scale);
  key[i] = (1ull << 63) | (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
  idx[i] = (uint32_t)i;
}

__global__ void k_gather_pos(const double* __restrict__ pos, const uint32_t* __restrict__ perm,
                             int64_t n, double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  s[i] = pos[3 * j];
  s[n + i] = pos[3 * j + 1];
  s[2 * n + i] = pos[3 * j + 2];
}

// w[i] = digits shared by keys i and i + n_leaf (a run of n_leaf + 1 keys).
__global__ void k_window(const uint64_t* __restrict__ key, int64_t n, int n_leaf,
                         int8_t* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  w[i] = (int8_t)((i + n_leaf < n) ? lcp_level(key[i], key[i + n_leaf]) : -1);
}

// For sorted particle j: the deepest level lambda_j of a cell containing it
// (a level-L group splits iff it holds more than n_leaf particles, i.e. iff
// some run of n_leaf + 1 keys containing j shares L digits), and the levels
// at which j is the first particle of a cell: d_j < L <= lambda_j, with d_j
// the digits shared with key j - 1. Also per-block counts per level.
__global__ __launch_bounds__(kB) void k_masks(const uint64_t* __restrict__ key,
                                              const int8_t* __restrict__ w, int64_t n, int n_leaf,
                                              uint32_t* __restrict__ mask,
                                              uint8_t* __restrict__ lam,
                                              int64_t* __restrict__ counts, int64_t nblocks) {
  __shared__ uint32_t wc[kB / 64][kMaxLevel + 1];
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t m = 0;
  if (j < n) {
    int sigma = -1;
    const int64_t i0 = j - n_leaf > 0 ? j - n_leaf : 0;
    for (int64_t i = i0; i <= j; ++i) sigma = max(sigma, (int)w[i]);
    const int lmb = sigma < 0 ? 0 : min(kMaxLevel, sigma + 1);
    const int d = j == 0 ? -1 : lcp_level(key[j - 1], key[j]);
    if (d < 0)
      m = (2u << lmb) - 1u;
    else if (d < lmb)
      m = ((2u << lmb) - 1u) & ~((2u << d) - 1u);
    mask[j] = m;
    lam[j] = (uint8_t)lmb;
  }
  for (int L = 0; L <= kMaxLevel; ++L) {
    const uint64_t b = __ballot((m >> L) & 1u);
    if (lane == 0) wc[wv][L] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x <= kMaxLevel) {
    uint32_t s = 0;
    for (int q = 0; q < kB / 64; ++q) s += wc[q][threadIdx.x];
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s;
  }
}

__global__ void k_level_totals(const int64_t* __restrict__ offs, int64_t nblocks,
                               const int64_t* __restrict__ total, int64_t* __restrict__ out) {
  const int L = threadIdx.x;
  if (L <= kMaxLevel) out[L] = offs[(int64_t)L * nblocks];
  if (L == kMaxLevel + 1) out[L] = *total;
}

__global__ __launch_bounds__(kB) void k_cell_scatter(const uint32_t* __restrict__ mask, int64_t n,
                                                     const int64_t* __restrict__ offs,
                                                     int64_t nblocks,
                                                     int32_t* __restrict__ c_first,
                                                     int8_t* __restrict__ c_level) {
  __shared__ uint32_t wc[kB / 64][kMaxLevel + 1];
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t m = j < n ? mask[j] : 0u;
  for (int L = 0; L <= kMaxLevel; ++L) {
    const uint64_t b = __ballot((m >> L) & 1u);
    if (lane == 0) wc[wv][L] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  for (int L = 0; L <= kMaxLevel; ++L) {
    const uint64_t b = __ballot((m >> L) & 1u);
    if ((m >> L) & 1u) {
      uint32_t pre = 0;
      for (int q = 0; q < wv; ++q) pre += wc[q][L];
      const int64_t idx = offs[(int64_t)L * nblocks + blockIdx.x] + pre + __popcll(b & lt);
      c_first[idx] = (int32_t)j;
      c_level[idx] = (int8_t)L;
    }
  }
}

__global__ void k_cell_fill(const uint64_t* __restrict__ key, int64_t n,
                            const int32_t* __restrict__ c_first, const int8_t* __restrict__ c_level,
                            int64_t C, const double* __restrict__ root, int n_leaf,
                            uint64_t* __restrict__ c_key, int32_t* __restrict__ c_count,
                            uint8_t* __restrict__ c_leaf, double* __restrict__ c_centre) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int64_t s = c_first[c];
  const int L = c_level[c];
  const int sh = 3 * (kMaxLevel - L);
  const uint64_t P = key[s] >> sh;
  const uint64_t maxk = (P << sh) | ((1ull << sh) - 1ull);
  int64_t lo = s + 1, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] <= maxk)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int64_t cnt = lo - s;
  c_key[c] = P;
  c_count[c] = (int32_t)cnt;
  c_leaf[c] = (uint8_t)!(cnt > n_leaf && L < kMaxLevel);
  double cc[3];
  cell_centre(P, L, root, cc);
  c_centre[3 * c] = cc[0];
  c_centre[3 * c + 1] = cc[1];
  c_centre[3 * c + 2] = cc[2];
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_hash_insert(const uint64_t* __restrict__ c_key, int64_t C,
                              unsigned long long* __restrict__ hk, int32_t* __restrict__ hv,
                              uint64_t mask, unsigned* __restrict__ flags) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const uint64_t key = c_key[c];
  uint64_t s = mix64(key) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(&hk[s], (unsigned long long)kEmptyKey,
                                              (unsigned long long)key);
    if (prev == kEmptyKey) {
      hv[s] = (int32_t)c;
      return;
    }
    s = (s + 1) & mask;
  }
  atomicOr(flags, FLAG_HASH_FULL);
}

// Parent and children found by key through the hash table.
__global__ void k_links(const uint64_t* __restrict__ c_key, const int8_t* __restrict__ c_level,
                        const uint8_t* __restrict__ c_leaf, int64_t C,
                        const uint64_t* __restrict__ hk, const int32_t* __restrict__ hv,
                        uint64_t mask, int32_t* __restrict__ parent,
                        int32_t* __restrict__ child, int32_t* __restrict__ nchild) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const uint64_t P = c_key[c];
  parent[c] = c_level[c] == 0 ? -1 : hash_find(hk, hv, mask, P >> 3);
  int first = -1, nc = 0;
  if (!c_leaf[c]) {
    for (int o = 0; o < 8; ++o) {
      const int q = hash_find(hk, hv, mask, (P << 3) | (uint64_t)o);
      if (q >= 0) {
        if (first < 0) first = q;
        ++nc;
      }
    }
  }
  child[c] = first;
  nchild[c] = nc;
}

// Squared b_max of every cell: for each level, the particles of a wave that
// share a level-L cell reduce their squared distance to its centre with a
// segmented max, and the last lane of each run does one max (on the bits of a
// non-negative double, which order like unsigned integers). Each block takes
// a contiguous chunk of particles; the cells of the top kBmaxTop levels (at
// most 585, where every wave of the chunk would hit the same few addresses)
// are reduced in LDS slots indexed by their key bits and written with one
// global atomic per block and cell; deeper cells take a global atomic per run.
constexpr int kBmaxTop = 4;
constexpr int kBmaxSlots = (1 + 8 + 64 + 512);
__device__ __forceinline__ int bmax_slot(uint64_t P, int L) {
  // (8^L - 1) / 7 slots for the levels above, then the L x 3 key bits
  return (int)(((1u << (3 * L)) - 1u) / 7u) + (int)(P & ((1ull << (3 * L)) - 1ull));
}
__global__ __launch_bounds__(kB) void k_bmax(const uint64_t* __restrict__ key,
                                             const uint8_t* __restrict__ lam,
                                             const double* __restrict__ spos, int64_t n,
                                             int64_t chunk, const double* __restrict__ root,
                                             const uint64_t* __restrict__ hk,
                                             const int32_t* __restrict__ hv, uint64_t mask,
                                             unsigned long long* __restrict__ bmax2) {
  __shared__ unsigned long long top[kBmaxSlots];
  for (int q = threadIdx.x; q < kBmaxSlots; q += kB) top[q] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
  for (int64_t jb = j0; jb < j1; jb += kB) {
    const int64_t j = jb + threadIdx.x;
    const bool valid = j < j1;
    const uint64_t k = valid ? key[j] : 0ull;
    const int lmb = valid ? (int)lam[j] : -1;
    double x = 0, y = 0, z = 0;
    if (valid) {
      x = spos[j];
      y = spos[n + j];
      z = spos[2 * n + j];
    }
    // the particle's integer coordinates at the deepest level, decoded once:
    // its level-L cell has the top L bits of each (the digits cell_centre
    // takes from the key prefix), so the centres below are the same numbers
    const uint64_t dig = k & ((1ull << (3 * kMaxLevel)) - 1ull);
    const uint32_t IX = compact3(dig >> 2), IY = compact3(dig >> 1), IZ = compact3(dig);
    for (int L = 0; L <= kMaxLevel; ++L) {
      const bool has = L <= lmb;
      if (!__any(has)) break;
      const unsigned long long P = has ? (k >> (3 * (kMaxLevel - L))) : 0ull;
      unsigned long long v = 0;
      if (has) {
        const int sh = kMaxLevel - L;
        const double h = ldexp(root[3], -(L + 1));
        const double c[3] = {root[0] + (double)(2u * (IX >> sh) + 1u) * h,
                             root[1] + (double)(2u * (IY >> sh) + 1u) * h,
                             root[2] + (double)(2u * (IZ >> sh) + 1u) * h};
        const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        v = (unsigned long long)__double_as_longlong(d2);
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long Pn = __shfl_up(P, off);
        const unsigned long long vn = __shfl_up(v, off);
        if (lane >= off && Pn == P && vn > v) v = vn;
      }
      const unsigned long long Pnext = __shfl_down(P, 1);
      const bool last = (lane == 63) || (Pnext != P) || (j + 1 >= j1);
      if (has && last) {
        if (L < kBmaxTop) {
          atomicMax(&top[bmax_slot(P, L)], v);
        } else {
          const int32_t c = hash_find(hk, hv, mask, P);
          if (c >= 0) atomicMax(&bmax2[c], v);
        }
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kBmaxSlots; q += kB) {
    const unsigned long long v = top[q];
    if (v == 0ull) continue;
    int L = 0;
    while (L + 1 < kBmaxTop && q >= (int)(((1u << (3 * (L + 1))) - 1u) / 7u)) ++L;
    const uint64_t P = (1ull << (3 * L)) | (uint64_t)(q - (int)(((1u << (3 * L)) - 1u) / 7u));
    const int32_t c = hash_find(hk, hv, mask, P);
    if (c >= 0) atomicMax(&bmax2[c], v);
  }
}

__global__ void k_bmax_final(const unsigned long long* __restrict__ b2, int64_t C,
                             double* __restrict__ b) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C) b[c] = sqrt(__longlong_as_double((long long)b2[c]));
}

// Sink groups: the topmost cells with at most n_group particles, or leaves
// that still hold more. gstart[first particle] = cell id.
__global__ void k_group_mark(const int32_t* __restrict__ c_first, const int32_t* __restrict__ c_count,
                             const int32_t* __restrict__ parent, const uint8_t* __restrict__ c_leaf,
                             int64_t C, int n_group, int32_t* __restrict__ gstart) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int cnt = c_count[c];
  const int par = parent[c];
  const bool top_small = cnt <= n_group && (par < 0 || c_count[par] > n_group);
  const bool big_leaf = c_leaf[c] && cnt > n_group;
  if (top_small || big_leaf) gstart[c_first[c]] = (int32_t)c;
}

__global__ void k_flag_ge0(const int32_t* __restrict__ a, int64_t n, uint32_t* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = a[i] >= 0 ? 1u : 0u;
}

__global__ void k_group_compact(const int32_t* __restrict__ gstart, const uint32_t* __restrict__ rank,
                                int64_t n, const int32_t* __restrict__ c_count,
                                int32_t* __restrict__ g_cell, int32_t* __restrict__ g_first,
                                int32_t* __restrict__ g_count, int32_t* __restrict__ group_of) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int32_t c = gstart[j];
  const uint32_t r = rank[j];
  if (c >= 0) {
    g_cell[r] = c;
    g_first[r] = (int32_t)j;
    g_count[r] = c_count[c];
  }
  group_of[j] = (int32_t)(c >= 0 ? r : r - 1);
}

__global__ void k_chunks(const int32_t* __restrict__ g_count, int64_t G, uint32_t* __restrict__ nch) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) nch[g] = (uint32_t)((g_count[g] + kWave - 1) / kWave);
}

__global__ void k_items(const int32_t* __restrict__ g_first, const int32_t* __restrict__ g_count,
                        const uint32_t* __restrict__ off, int64_t G, int2* __restrict__ items) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int f = g_first[g], cnt = g_count[g];
  uint32_t o = off[g];
  for (int s = 0; s < cnt; s += kWave) items[o++] = make_int2((int)g, f + s);
}

__global__ void k_leaf_fill(const int32_t* __restrict__ c_first, const int32_t* __restrict__ c_count,
                            const uint8_t* __restrict__ c_leaf, int64_t C,
                            int32_t* __restrict__ leaf_of) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C || !c_leaf[c]) return;
  const int f = c_first[c], e = f + c_count[c];
  for (int j = f; j < e; ++j) leaf_of[j] = (int32_t)c;
}

// Leaves in particle (Morton) order: leaf_of changes value exactly where a
// leaf starts, so the leaves' ranks are an exclusive scan of those starts;
// consecutive entries of the list hold consecutive particle ranges.
__device__ __forceinline__ bool leaf_starts(const int32_t* __restrict__ leaf_of, int64_t j) {
  return j == 0 || leaf_of[j] != leaf_of[j - 1];
}

__global__ void k_leaf_flags(const int32_t* __restrict__ leaf_of, int64_t n,
                             uint32_t* __restrict__ f) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) f[j] = leaf_starts(leaf_of, j) ? 1u : 0u;
}

__global__ void k_leaf_compact(const int32_t* __restrict__ leaf_of, const uint32_t* __restrict__ rank,
                               int64_t n, int32_t* __restrict__ leaf_list) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && leaf_starts(leaf_of, j)) leaf_list[rank[j]] = leaf_of[j];
}

// item_of[j]: the eval work item (group chunk of at most 64 particles) of j.
__global__ void k_item_of(const int2* __restrict__ items, int64_t n_items,
                          const int32_t* __restrict__ g_first, const int32_t* __restrict__ g_count,
                          int32_t* __restrict__ item_of) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_items) return;
  const int2 it = items[q];
  const int gend = g_first[it.x] + g_count[it.x];
  const int e = it.y + kWave < gend ? it.y + kWave : gend;
  for (int j = it.y; j < e; ++j) item_of[j] = (int32_t)q;
}

__global__ void k_hash_lookup(const uint64_t* __restrict__ q, int64_t nq,
                              const uint64_t* __restrict__ hk, const int32_t* __restrict__ hv,
                              uint64_t mask, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nq) out[i] = q[i] == kEmptyKey ? -1 : hash_find(hk, hv, mask, q[i]);
}

}  // namespace

void build_tree(hot_ctx* ctx, hot_tree* t, const double* pos, const double* box) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  const unsigned gb = grid_for(n, kB);
  unsigned* lflags = ctx->d_flags + kFlagLocal;
  zero_flag_word(ctx, kFlagLocal);
  // ---- root cube
  t->root.alloc(ctx, 8 * sizeof(double));
  if (box) {
    double r[8] = {box[0], box[1], box[2], box[3], 2097152.0 / box[3], 0, 0, 0};
    HOT_HIP(hipMemcpyAsync(t->root.p, r, sizeof(r), hipMemcpyHostToDevice, st));
    k_box_check<<<gb, kB, 0, st>>>(pos, n, t->root.as<double>(), lflags);
    HOT_CHECK_LAUNCH();
  } else {
    const int nparts = (int)std::min<int64_t>(1024, (n + kB - 1) / kB);
    DBuf part;
    part.alloc(ctx, (size_t)nparts * 6 * sizeof(double));
    k_bbox_partial<<<nparts, kB, 0, st>>>(pos, n, part.as<double>(), lflags);
    HOT_CHECK_LAUNCH();
    k_bbox_final<<<1, 64, 0, st>>>(part.as<double>(), nparts, t->root.as<double>());
    HOT_CHECK_LAUNCH();
  }
  // ---- keys and sort
  t->key.alloc(ctx, n * sizeof(uint64_t));
  t->perm.alloc(ctx, n * sizeof(uint32_t));
  k_keys<<<gb, kB, 0, st>>>(pos, n, t->root.as<double>(), t->key.as<uint64_t>(),
                           t->perm.as<uint32_t>());
  HOT_CHECK_LAUNCH();
  radix_sort(ctx, t->key, t->perm, n, 63);
  t->spos.alloc(ctx, 3 * n * sizeof(double));
  k_gather_pos<<<gb, kB, 0, st>>>(pos, t->perm.as<uint32_t>(), n, t->spos.as<double>());
  HOT_CHECK_LAUNCH();
  // ---- cells: levels per particle, counts, scan
  const int64_t nblocks = gb;
  DBuf w, mask, counts, tot;
  w.alloc(ctx, n);
  mask.alloc(ctx, n * sizeof(uint32_t));
  t->lambda.alloc(ctx, n);
  counts.alloc(ctx, (size_t)(kMaxLevel + 1) * nblocks * sizeof(int64_t));
  tot.alloc(ctx, 32 * sizeof(int64_t));
  k_window<<<gb, kB, 0, st>>>(t->key.as<uint64_t>(), n, t->n_leaf, w.as<int8_t>());
  HOT_CHECK_LAUNCH();
  k_masks<<<gb, kB, 0, st>>>(t->key.as<uint64_t>(), w.as<int8_t>(), n, t->n_leaf,
                            mask.as<uint32_t>(), t->lambda.as<uint8_t>(), counts.as<int64_t>(),
                            nblocks);
  HOT_CHECK_LAUNCH();
  scan_i64(ctx, counts.as<int64_t>(), counts.as<int64_t>(), (kMaxLevel + 1) * nblocks,
           tot.as<int64_t>() + 24);
  k_level_totals<<<1, 64, 0, st>>>(counts.as<int64_t>(), nblocks, tot.as<int64_t>() + 24,
                                  tot.as<int64_t>());
  HOT_CHECK_LAUNCH();
  int64_t lv[kMaxLevel + 2];
  double rootv[8];
  unsigned fw[2] = {0u, 0u};
  HOT_HIP(hipMemcpyAsync(lv, tot.p, sizeof(lv), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(rootv, t->root.p, sizeof(rootv), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(fw, ctx->d_flags, sizeof(fw), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipStreamSynchronize(st));
  raise_deferred(ctx, fw[kFlagDeferred]);
  unsigned flags = fw[kFlagLocal];
  if (flags & FLAG_NONFINITE_POS) invalid("non-finite position");
  if (flags & FLAG_OUTSIDE_BOX) invalid("point outside the given box");
  for (int d = 0; d < 3; ++d) t->lo[d] = rootv[d];
  t->side = rootv[3];
  if (!(t->side >= 0x1p-60 && t->side <= 0x1p60))
    invalid("root cube side outside [2^-60, 2^60]");
  const int64_t C = lv[kMaxLevel + 1];
  t->n_cells = C;
  t->level_off.assign(kMaxLevel + 2, C);
  for (int L = 0; L <= kMaxLevel; ++L) t->level_off[L] = lv[L];
  t->level_off[kMaxLevel + 1] = C;
  t->max_level = 0;
  for (int L = 0; L <= kMaxLevel; ++L)
    if (t->level_off[L + 1] > t->level_off[L]) t->max_level = L;
  if (C >= INT32_MAX) throw Error{HOT_E_CAPACITY, "too many cells"};
  // ---- cell arrays
  t->c_first.alloc(ctx, C * sizeof(int32_t));
  t->c_level.alloc(ctx, C);
  t->c_key.alloc(ctx, C * sizeof(uint64_t));
  t->c_count.alloc(ctx, C * sizeof(int32_t));
  t->c_leaf.alloc(ctx, C);
  t->c_centre.alloc(ctx, 3 * C * sizeof(double));
  t->c_parent.alloc(ctx, C * sizeof(int32_t));
  t->c_child.alloc(ctx, C * sizeof(int32_t));
  t->c_nchild.alloc(ctx, C * sizeof(int32_t));
  t->c_bmax2.alloc(ctx, C * sizeof(uint64_t));
  t->c_bmax.alloc(ctx, C * sizeof(double));
  k_cell_scatter<<<gb, kB, 0, st>>>(mask.as<uint32_t>(), n, counts.as<int64_t>(), nblocks,
                                   t->c_first.as<int32_t>(), t->c_level.as<int8_t>());
  HOT_CHECK_LAUNCH();
  const unsigned gc = grid_for(C, kB);
  k_cell_fill<<<gc, kB, 0, st>>>(t->key.as<uint64_t>(), n, t->c_first.as<int32_t>(),
                                t->c_level.as<int8_t>(), C, t->root.as<double>(), t->n_leaf,
                                t->c_key.as<uint64_t>(), t->c_count.as<int32_t>(),
                                t->c_leaf.as<uint8_t>(), t->c_centre.as<double>());
  HOT_CHECK_LAUNCH();
  // ---- hash table of cell keys
  uint64_t slots = 64;
  while (slots < 2 * (uint64_t)C) slots <<= 1;
  t->hash_slots = slots;
  t->h_keys.alloc(ctx, slots * sizeof(uint64_t));
  t->h_vals.alloc(ctx, slots * sizeof(int32_t));
  k_fill<uint64_t><<<grid_for(slots, kB), kB, 0, st>>>(t->h_keys.as<uint64_t>(), slots, kEmptyKey);
  HOT_CHECK_LAUNCH();
  k_hash_insert<<<gc, kB, 0, st>>>(t->c_key.as<uint64_t>(), C,
                                  t->h_keys.as<unsigned long long>(), t->h_vals.as<int32_t>(),
                                  slots - 1, lflags);
  HOT_CHECK_LAUNCH();
  k_links<<<gc, kB, 0, st>>>(t->c_key.as<uint64_t>(), t->c_level.as<int8_t>(),
                            t->c_leaf.as<uint8_t>(), C, t->h_keys.as<uint64_t>(),
                            t->h_vals.as<int32_t>(), slots - 1, t->c_parent.as<int32_t>(),
                            t->c_child.as<int32_t>(), t->c_nchild.as<int32_t>());
  HOT_CHECK_LAUNCH();
  // ---- b_max
  k_fill<uint64_t><<<gc, kB, 0, st>>>(t->c_bmax2.as<uint64_t>(), C, 0ull);
  HOT_CHECK_LAUNCH();
  {
    // chunks of at least 4096 particles, at most 2048 blocks
    const int64_t nblk = std::max<int64_t>(1, std::min<int64_t>(2048, (n + 4095) / 4096));
    const int64_t chunk = ((n + nblk - 1) / nblk + kB - 1) / kB * kB;
    k_bmax<<<(unsigned)nblk, kB, 0, st>>>(t->key.as<uint64_t>(), t->lambda.as<uint8_t>(),
                                          t->spos.as<double>(), n, chunk, t->root.as<double>(),
                                          t->h_keys.as<uint64_t>(), t->h_vals.as<int32_t>(),
                                          slots - 1, t->c_bmax2.as<unsigned long long>());
  }
  HOT_CHECK_LAUNCH();
  k_bmax_final<<<gc, kB, 0, st>>>(t->c_bmax2.as<unsigned long long>(), C, t->c_bmax.as<double>());
  HOT_CHECK_LAUNCH();
  // ---- groups
  DBuf gstart, gflag, gtot;
  gstart.alloc(ctx, n * sizeof(int32_t));
  gflag.alloc(ctx, n * sizeof(uint32_t));
  gtot.alloc(ctx, 2 * sizeof(uint32_t));
  k_fill<int32_t><<<gb, kB, 0, st>>>(gstart.as<int32_t>(), n, -1);
  HOT_CHECK_LAUNCH();
  k_group_mark<<<gc, kB, 0, st>>>(t->c_first.as<int32_t>(), t->c_count.as<int32_t>(),
                                 t->c_parent.as<int32_t>(), t->c_leaf.as<uint8_t>(), C,
                                 t->n_group, gstart.as<int32_t>());
  HOT_CHECK_LAUNCH();
  k_flag_ge0<<<gb, kB, 0, st>>>(gstart.as<int32_t>(), n, gflag.as<uint32_t>());
  HOT_CHECK_LAUNCH();
  scan_u32(ctx, gflag.as<uint32_t>(), gflag.as<uint32_t>(), n, gtot.as<uint32_t>());
  uint32_t G32 = 0;
  HOT_HIP(hipMemcpyAsync(&G32, gtot.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(&flags, lflags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipStreamSynchronize(st));
  if (flags & FLAG_HASH_FULL) throw Error{HOT_E_CAPACITY, "cell hash table full"};
  const int64_t G = G32;
  t->n_groups = G;
  t->g_cell.alloc(ctx, G * sizeof(int32_t));
  t->g_first.alloc(ctx, G * sizeof(int32_t));
  t->g_count.alloc(ctx, G * sizeof(int32_t));
  t->group_of.alloc(ctx, n * sizeof(int32_t));
  k_group_compact<<<gb, kB, 0, st>>>(gstart.as<int32_t>(), gflag.as<uint32_t>(), n,
                                    t->c_count.as<int32_t>(), t->g_cell.as<int32_t>(),
                                    t->g_first.as<int32_t>(), t->g_count.as<int32_t>(),
                                    t->group_of.as<int32_t>());
  HOT_CHECK_LAUNCH();
  // ---- eval work items: one per 64 sinks of a group
  DBuf nch, ntot;
  nch.alloc(ctx, G * sizeof(uint32_t));
  ntot.alloc(ctx, sizeof(uint32_t));
  k_chunks<<<grid_for(G, kB), kB, 0, st>>>(t->g_count.as<int32_t>(), G, nch.as<uint32_t>());
  HOT_CHECK_LAUNCH();
  scan_u32(ctx, nch.as<uint32_t>(), nch.as<uint32_t>(), G, ntot.as<uint32_t>());
  // ---- leaves: owner of every particle, and the list in particle order
  t->leaf_of.alloc(ctx, n * sizeof(int32_t));
  k_leaf_fill<<<gc, kB, 0, st>>>(t->c_first.as<int32_t>(), t->c_count.as<int32_t>(),
                                t->c_leaf.as<uint8_t>(), C, t->leaf_of.as<int32_t>());
  HOT_CHECK_LAUNCH();
  k_leaf_flags<<<gb, kB, 0, st>>>(t->leaf_of.as<int32_t>(), n, gflag.as<uint32_t>());
  HOT_CHECK_LAUNCH();
  scan_u32(ctx, gflag.as<uint32_t>(), gflag.as<uint32_t>(), n, gtot.as<uint32_t>() + 1);
  t->leaf_list.alloc(ctx, C * sizeof(int32_t));
  k_leaf_compact<<<gb, kB, 0, st>>>(t->leaf_of.as<int32_t>(), gflag.as<uint32_t>(), n,
                                    t->leaf_list.as<int32_t>());
  HOT_CHECK_LAUNCH();
  uint32_t NI = 0, NL = 0;
  HOT_HIP(hipMemcpyAsync(&NI, ntot.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(&NL, gtot.as<uint32_t>() + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipStreamSynchronize(st));
  t->n_items = NI;
  t->n_leaves = NL;
  t->items.alloc(ctx, (size_t)NI * sizeof(int2));
  k_items<<<grid_for(G, kB), kB, 0, st>>>(t->g_first.as<int32_t>(), t->g_count.as<int32_t>(),
                                         nch.as<uint32_t>(), G, t->items.as<int2>());
  HOT_CHECK_LAUNCH();
  t->item_of.alloc(ctx, n * sizeof(int32_t));
  k_item_of<<<grid_for(NI, kB), kB, 0, st>>>(t->items.as<int2>(), NI, t->g_first.as<int32_t>(),
                                            t->g_count.as<int32_t>(), t->item_of.as<int32_t>());
  HOT_CHECK_LAUNCH();
  t->c_bmax2.release();
  split_items(ctx, t);
}

void hash_lookup(hot_ctx* ctx, const hot_tree* t, const uint64_t* keys, int32_t* out, int64_t nq) {
  if (nq <= 0) return;
  k_hash_lookup<<<grid_for(nq, kB), kB, 0, ctx->stream>>>(keys, nq, t->h_keys.as<uint64_t>(),
                                                         t->h_vals.as<int32_t>(),
                                                         t->hash_slots - 1, out);
  HOT_CHECK_LAUNCH();
}

}  // namespace hot
