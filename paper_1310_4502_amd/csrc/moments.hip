// Upward pass: raw Cartesian moments about geometric cell centres
// (Multipole Error Bounds section: M^(n)(z) = integral (y - z)^(n) rho(y) dy;
// expansions about cell centres as the Background Subtraction section
// prescribes). Leaves take their particles directly (P2M); every other cell
// re-centres its children's moments (the shift identity of the same section:
// M about a shifted centre written as powers of the shift). FP64.
// A scaled FP32 (or FP64) copy with the expansion weights folded in feeds the
// expansion kernels:  Mw_alpha = (-1)^|alpha| / alpha! * M_alpha / s^|alpha|,
// s = cell side (an exact power of two).
#include "common.h"
#include "eval_common.h"
#include "generated/expansions.h"

namespace hot {

static __constant__ AlphaTable kAlpha = make_alpha_table();

namespace {

constexpr int kB = 256;

__global__ void k_gather_pm(const double* __restrict__ pos, const double* __restrict__ mass,
                            const uint32_t* __restrict__ perm, int64_t n,
                            double* __restrict__ spos, double* __restrict__ smass,
                            unsigned* __restrict__ flags, int check_mass) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  const double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
  spos[i] = x;
  spos[n + i] = y;
  spos[2 * n + i] = z;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) atomicOr(flags, FLAG_NONFINITE_POS);
  if (smass) {
    const double m = mass[j];
    smass[i] = m;
    if (check_mass && !(isfinite(m) && m >= 0.0)) atomicOr(flags, FLAG_BAD_MASS);
  }
}

template <int N>
__device__ __forceinline__ void m2m_order(const double* __restrict__ mom, int nmv, int cf, int nc,
                                          const double* __restrict__ centre, const double* cp,
                                          double* __restrict__ out) {
  constexpr int K = (N + 1) * (N + 2) / 2;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int q = cf; q < cf + nc; ++q) {
    const double* M = mom + (int64_t)q * nmv;
    const double dx = centre[3 * q] - cp[0], dy = centre[3 * q + 1] - cp[1],
                 dz = centre[3 * q + 2] - cp[2];
    if constexpr (N == 0) m2m_order0(M, dx, dy, dz, acc);
    if constexpr (N == 1) m2m_order1(M, dx, dy, dz, acc);
    if constexpr (N == 2) m2m_order2(M, dx, dy, dz, acc);
    if constexpr (N == 3) m2m_order3(M, dx, dy, dz, acc);
    if constexpr (N == 4) m2m_order4(M, dx, dy, dz, acc);
    if constexpr (N == 5) m2m_order5(M, dx, dy, dz, acc);
    if constexpr (N == 6) m2m_order6(M, dx, dy, dz, acc);
    if constexpr (N == 7) m2m_order7(M, dx, dy, dz, acc);
    if constexpr (N == 8) m2m_order8(M, dx, dy, dz, acc);
  }
  const int off = N * (N + 1) * (N + 2) / 6;
#pragma unroll
  for (int k = 0; k < K; ++k) out[off + k] = acc[k];
}

// Leaves only (P2M). One wavefront per 64 consecutive entries of the leaf list
// (leaves in particle order) and one order, the block's: the 64 leaves'
// particles form one contiguous range, staged through LDS in chunks by
// coalesced loads, and lane l sums its own leaf's particles in order. The
// moments leave through LDS in slices of kP2mSlice values per leaf, so that
// neighbouring lanes store neighbouring addresses of a leaf's row.
constexpr int kP2mChunk = 256;
constexpr int kP2mSlice = 16;

template <int N>
__device__ __forceinline__ void p2m_run(int64_t run, const int32_t* __restrict__ leaf_list,
                                        int64_t n_leaves, const int32_t* __restrict__ c_first,
                                        const int32_t* __restrict__ c_count,
                                        const double* __restrict__ c_centre,
                                        const double* __restrict__ spos,
                                        const double* __restrict__ smass, int64_t n, int nmv,
                                        double* __restrict__ mom, double* lds, int* s_cell) {
  constexpr int K = (N + 1) * (N + 2) / 2;
  constexpr int OFF = N * (N + 1) * (N + 2) / 6;
  constexpr int NS = (K + kP2mSlice - 1) / kP2mSlice;
  constexpr int TS = kP2mSlice + 1;  // tile row stride (odd: spreads the banks)
  const int lane = threadIdx.x;
  const int nv = (int)(n_leaves - run * 64 < 64 ? n_leaves - run * 64 : 64);
  int c = 0, f = 0, e = 0;
  double cx = 0.0, cy = 0.0, cz = 0.0;
  if (lane < nv) {
    c = leaf_list[run * 64 + lane];
    f = c_first[c];
    e = f + c_count[c];
    cx = c_centre[3 * c];
    cy = c_centre[3 * c + 1];
    cz = c_centre[3 * c + 2];
  }
  s_cell[lane] = c;  // read after the barriers below
  const int start = __shfl(f, 0), end = __shfl(e, nv - 1);
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  double* X = lds;
  double* Y = lds + kP2mChunk;
  double* Z = lds + 2 * kP2mChunk;
  double* M = lds + 3 * kP2mChunk;
  for (int s = start; s < end; s += kP2mChunk) {
    const int w = end - s < kP2mChunk ? end - s : kP2mChunk;
    __syncthreads();  // the previous chunk has been read
    for (int i = lane; i < w; i += 64) {
      X[i] = spos[s + i];
      Y[i] = spos[n + s + i];
      Z[i] = spos[2 * n + s + i];
      M[i] = smass[s + i];
    }
    __syncthreads();
    const int j0 = f > s ? f : s, j1 = e < s + w ? e : s + w;
    for (int j = j0; j < j1; ++j) {
      const int q = j - s;
      const double dx = X[q] - cx, dy = Y[q] - cy, dz = Z[q] - cz;
      if constexpr (N == 0) p2m_order0(dx, dy, dz, M[q], acc);
      if constexpr (N == 1) p2m_order1(dx, dy, dz, M[q], acc);
      if constexpr (N == 2) p2m_order2(dx, dy, dz, M[q], acc);
      if constexpr (N == 3) p2m_order3(dx, dy, dz, M[q], acc);
      if constexpr (N == 4) p2m_order4(dx, dy, dz, M[q], acc);
      if constexpr (N == 5) p2m_order5(dx, dy, dz, M[q], acc);
      if constexpr (N == 6) p2m_order6(dx, dy, dz, M[q], acc);
      if constexpr (N == 7) p2m_order7(dx, dy, dz, M[q], acc);
      if constexpr (N == 8) p2m_order8(dx, dy, dz, M[q], acc);
    }
  }
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    __syncthreads();  // the staging area (or the previous slice) is free
#pragma unroll
    for (int k = 0; k < kP2mSlice; ++k)
      if (r * kP2mSlice + k < K) lds[lane * TS + k] = acc[r * kP2mSlice + k < K ? r * kP2mSlice + k : 0];
    __syncthreads();
    const int W = K - r * kP2mSlice < kP2mSlice ? K - r * kP2mSlice : kP2mSlice;
    for (int i = lane; i < nv * W; i += 64) {
      const int l = i / W, k = i - l * W;
      mom[(int64_t)s_cell[l] * nmv + OFF + r * kP2mSlice + k] = lds[l * TS + k];
    }
  }
}

__global__ __launch_bounds__(64) void k_p2m(int64_t n_leaves, const int32_t* __restrict__ leaf_list,
                                            const int32_t* __restrict__ c_first,
                                            const int32_t* __restrict__ c_count,
                                            const double* __restrict__ c_centre,
                                            const double* __restrict__ spos,
                                            const double* __restrict__ smass, int64_t n, int p,
                                            double* __restrict__ mom) {
  // the staging chunk (four arrays) and, after it, the output slices
  constexpr int kLds = 4 * kP2mChunk > 64 * (kP2mSlice + 1) ? 4 * kP2mChunk : 64 * (kP2mSlice + 1);
  __shared__ double lds[kLds];
  __shared__ int s_cell[64];
  int64_t run;
  int ord;
  order_block(p, run, ord);
  if (run * 64 >= n_leaves) return;
  const int nmv = nm(p);
#define HOT_P2M_RUN(Q)                                                                         \
  case Q:                                                                                      \
    p2m_run<Q>(run, leaf_list, n_leaves, c_first, c_count, c_centre, spos, smass, n, nmv, mom, \
               lds, s_cell);                                                                           \
    break;
  switch (ord) {
    HOT_P2M_RUN(0) HOT_P2M_RUN(1) HOT_P2M_RUN(2) HOT_P2M_RUN(3) HOT_P2M_RUN(4)
    HOT_P2M_RUN(5) HOT_P2M_RUN(6) HOT_P2M_RUN(7) HOT_P2M_RUN(8)
  }
#undef HOT_P2M_RUN
}

// one level of internal cells [c0, c1)
__global__ __launch_bounds__(kB) void k_m2m(int64_t c0, int64_t c1, const int32_t* __restrict__ c_child,
                                            const int32_t* __restrict__ c_nchild,
                                            const uint8_t* __restrict__ c_leaf,
                                            const double* __restrict__ c_centre, int p,
                                            double* __restrict__ mom) {
  int64_t run;
  int ord;
  order_block(p, run, ord);
  const int64_t c = c0 + run * kB + threadIdx.x;
  if (c >= c1 || c_leaf[c]) return;
  const int nmv = nm(p);
  double* out = mom + c * nmv;
  const double cp[3] = {c_centre[3 * c], c_centre[3 * c + 1], c_centre[3 * c + 2]};
  const int cf = c_child[c], nc = c_nchild[c];
  switch (ord) {
    case 0: m2m_order<0>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 1: m2m_order<1>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 2: m2m_order<2>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 3: m2m_order<3>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 4: m2m_order<4>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 5: m2m_order<5>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 6: m2m_order<6>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 7: m2m_order<7>(mom, nmv, cf, nc, c_centre, cp, out); break;
    case 8: m2m_order<8>(mom, nmv, cf, nc, c_centre, cp, out); break;
  }
}

template <typename T>
__global__ void k_weighted(const double* __restrict__ mom, int64_t C,
                           const int8_t* __restrict__ c_level, double inv_side, int p,
                           T* __restrict__ out) {
  const int nmv = nm(p), stride = nm_pad(p);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c;
  int s;
  row_col(t, stride, c, s);
  if (c >= C) return;
  if (s >= nmv) {
    out[c * stride + s] = T(0);
    return;
  }
  const int order = kAlpha.a[s] + kAlpha.b[s] + kAlpha.c[s];
  const double sc = pow2_pow(ldexp(inv_side, (int)c_level[c]), order);
  out[c * stride + s] = (T)(kAlpha.w[s] * (mom[c * nmv + s] * sc));
}

// The same weighted scaled moments with each cell's uniform cube of the mean
// density taken off (background subtraction). Scaled by the cell side s, the
// raw moments of a cube of mass m_c are m_c prod_d 2^(-alpha_d) / (alpha_d + 1)
// for all alpha_d even (zero otherwise), and m_c = M_total 2^(-3 level): the
// mean density M_total / L^3 (M_total the root's monopole) times s^3.
template <typename T>
__global__ void k_weighted_sub(const double* __restrict__ mom, int64_t C,
                               const int8_t* __restrict__ c_level, double inv_side, int p,
                               T* __restrict__ out) {
  const int nmv = nm(p), stride = nm_pad(p);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c;
  int s;
  row_col(t, stride, c, s);
  if (c >= C) return;
  if (s >= nmv) {
    out[c * stride + s] = T(0);
    return;
  }
  const int a = kAlpha.a[s], b = kAlpha.b[s], cc = kAlpha.c[s];
  const int order = a + b + cc;
  const int lev = (int)c_level[c];
  const double sc = pow2_pow(ldexp(inv_side, lev), order);
  double v = mom[c * nmv + s] * sc;
  if (!((a | b | cc) & 1)) {
    const double cube = ldexp(mom[0], -3 * lev - order) /
                        ((double)(a + 1) * (double)(b + 1) * (double)(cc + 1));
    v -= cube;
  }
  out[c * stride + s] = (T)(kAlpha.w[s] * v);
}

// Weighted scaled moments of each cell's uniform cube per unit density, with
// the minus sign they are subtracted with: -w_alpha L^3 2^(-3 level - |alpha|)
// prod_d 1 / (alpha_d + 1) for all alpha_d even, else 0.
template <typename T>
__global__ void k_weighted_cube(int64_t C, const int8_t* __restrict__ c_level, double vol, int p,
                                T* __restrict__ out) {
  const int nmv = nm(p), stride = nm_pad(p);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c;
  int s;
  row_col(t, stride, c, s);
  if (c >= C) return;
  double v = 0.0;
  if (s < nmv) {
    const int a = kAlpha.a[s], b = kAlpha.b[s], cc = kAlpha.c[s];
    if (!((a | b | cc) & 1))
      v = -kAlpha.w[s] * ldexp(vol, -3 * (int)c_level[c] - (a + b + cc)) /
          ((double)(a + 1) * (double)(b + 1) * (double)(cc + 1));
  }
  out[c * stride + s] = (T)v;
}

}  // namespace

void weighted_cube(hot_ctx* ctx, hot_tree* t, bool fp64, void* out) {
  const int64_t tot = t->n_cells * nm_pad(t->p);
  const double vol = (t->side * t->side) * t->side;
  if (fp64)
    k_weighted_cube<double><<<grid_for(tot, kB), kB, 0, ctx->stream>>>(
        t->n_cells, t->c_level.as<int8_t>(), vol, t->p, static_cast<double*>(out));
  else
    k_weighted_cube<float><<<grid_for(tot, kB), kB, 0, ctx->stream>>>(
        t->n_cells, t->c_level.as<int8_t>(), vol, t->p, static_cast<float*>(out));
  HOT_CHECK_LAUNCH();
}

void weighted_sub(hot_ctx* ctx, hot_tree* t, bool fp64) {
  const int64_t C = t->n_cells;
  const int p = t->p;
  const int64_t tot = C * nm_pad(p);
  t->momsub.alloc(ctx, (size_t)tot * (fp64 ? sizeof(double) : sizeof(float)));
  if (fp64)
    k_weighted_sub<double><<<grid_for(tot, kB), kB, 0, ctx->stream>>>(
        t->mom64.as<double>(), C, t->c_level.as<int8_t>(), 1.0 / t->side, p,
        t->momsub.as<double>());
  else
    k_weighted_sub<float><<<grid_for(tot, kB), kB, 0, ctx->stream>>>(
        t->mom64.as<double>(), C, t->c_level.as<int8_t>(), 1.0 / t->side, p,
        t->momsub.as<float>());
  HOT_CHECK_LAUNCH();
}

void gather_sorted(hot_ctx* ctx, const hot_tree* t, const double* pos, const double* mass,
                   double* spos, double* smass, int check_mass) {
  const int64_t n = t->n;
  k_gather_pm<<<grid_for(n, kB), kB, 0, ctx->stream>>>(pos, mass, t->perm.as<uint32_t>(), n, spos,
                                                       smass, ctx->d_flags, check_mass);
  HOT_CHECK_LAUNCH();
}

void build_moments(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, int p) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n, C = t->n_cells;
  DBuf spos, smass;
  spos.alloc(ctx, 3 * n * sizeof(double));
  smass.alloc(ctx, n * sizeof(double));
  gather_sorted(ctx, t, pos, mass, spos.as<double>(), smass.as<double>(), 1);
  t->mom64.alloc(ctx, (size_t)C * nm(p) * sizeof(double));
  t->p = -1;
  {
    const int64_t NL = t->n_leaves;
    k_p2m<<<order_grid((NL + 63) / 64, p), 64, 0, st>>>(
        NL, t->leaf_list.as<int32_t>(), t->c_first.as<int32_t>(), t->c_count.as<int32_t>(),
        t->c_centre.as<double>(), spos.as<double>(), smass.as<double>(), n, p,
        t->mom64.as<double>());
    HOT_CHECK_LAUNCH();
  }
  for (int L = t->max_level - 1; L >= 0; --L) {
    const int64_t c0 = t->level_off[L], c1 = t->level_off[L + 1];
    if (c1 <= c0) continue;
    k_m2m<<<order_grid(grid_for(c1 - c0, kB), p), kB, 0, st>>>(c0, c1, t->c_child.as<int32_t>(), t->c_nchild.as<int32_t>(),
                               t->c_leaf.as<uint8_t>(), t->c_centre.as<double>(), p,
                               t->mom64.as<double>());
    HOT_CHECK_LAUNCH();
  }
  // scaled, weighted FP32 copy for the mixed-precision expansion kernels
  t->mom32.alloc(ctx, (size_t)C * nm_pad(p) * sizeof(float));
  const int64_t tot = C * nm_pad(p);
  k_weighted<float><<<grid_for(tot, kB), kB, 0, st>>>(t->mom64.as<double>(), C,
                                                      t->c_level.as<int8_t>(), 1.0 / t->side, p,
                                                      t->mom32.as<float>());
  HOT_CHECK_LAUNCH();
  t->momw64_valid = false;
  t->p = p;
}

void weighted_fp64(hot_ctx* ctx, hot_tree* t) {
  if (t->momw64_valid) return;
  const int64_t C = t->n_cells;
  const int p = t->p;
  t->momw64.alloc(ctx, (size_t)C * nm_pad(p) * sizeof(double));
  const int64_t tot = C * nm_pad(p);
  k_weighted<double><<<grid_for(tot, kB), kB, 0, ctx->stream>>>(
      t->mom64.as<double>(), C, t->c_level.as<int8_t>(), 1.0 / t->side, p,
      t->momw64.as<double>());
  HOT_CHECK_LAUNCH();
  t->momw64_valid = true;
}

}  // namespace hot
