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
__device__ __forceinline__ void p2m_order(const double* __restrict__ spos,
                                          const double* __restrict__ smass, int64_t n, int first,
                                          int count, const double* c, double* __restrict__ out) {
  constexpr int K = (N + 1) * (N + 2) / 2;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int j = first; j < first + count; ++j) {
    const double dx = spos[j] - c[0], dy = spos[n + j] - c[1], dz = spos[2 * n + j] - c[2];
    const double m = smass[j];
    if constexpr (N == 0) p2m_order0(dx, dy, dz, m, acc);
    if constexpr (N == 1) p2m_order1(dx, dy, dz, m, acc);
    if constexpr (N == 2) p2m_order2(dx, dy, dz, m, acc);
    if constexpr (N == 3) p2m_order3(dx, dy, dz, m, acc);
    if constexpr (N == 4) p2m_order4(dx, dy, dz, m, acc);
    if constexpr (N == 5) p2m_order5(dx, dy, dz, m, acc);
    if constexpr (N == 6) p2m_order6(dx, dy, dz, m, acc);
    if constexpr (N == 7) p2m_order7(dx, dy, dz, m, acc);
    if constexpr (N == 8) p2m_order8(dx, dy, dz, m, acc);
  }
  const int off = N * (N + 1) * (N + 2) / 6;
#pragma unroll
  for (int k = 0; k < K; ++k) out[off + k] = acc[k];
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

// leaves only (P2M)
__global__ __launch_bounds__(kB) void k_p2m(int64_t C, const int32_t* __restrict__ c_first,
                                            const int32_t* __restrict__ c_count,
                                            const uint8_t* __restrict__ c_leaf,
                                            const double* __restrict__ c_centre,
                                            const double* __restrict__ spos,
                                            const double* __restrict__ smass, int64_t n, int p,
                                            double* __restrict__ mom) {
  int64_t run;
  int ord;
  order_block(p, run, ord);
  const int64_t c = run * kB + threadIdx.x;
  if (c >= C || !c_leaf[c]) return;
  const int nmv = nm(p);
  double* out = mom + c * nmv;
  const double cc[3] = {c_centre[3 * c], c_centre[3 * c + 1], c_centre[3 * c + 2]};
  const int f = c_first[c], cnt = c_count[c];
  switch (ord) {
    case 0: p2m_order<0>(spos, smass, n, f, cnt, cc, out); break;
    case 1: p2m_order<1>(spos, smass, n, f, cnt, cc, out); break;
    case 2: p2m_order<2>(spos, smass, n, f, cnt, cc, out); break;
    case 3: p2m_order<3>(spos, smass, n, f, cnt, cc, out); break;
    case 4: p2m_order<4>(spos, smass, n, f, cnt, cc, out); break;
    case 5: p2m_order<5>(spos, smass, n, f, cnt, cc, out); break;
    case 6: p2m_order<6>(spos, smass, n, f, cnt, cc, out); break;
    case 7: p2m_order<7>(spos, smass, n, f, cnt, cc, out); break;
    case 8: p2m_order<8>(spos, smass, n, f, cnt, cc, out); break;
  }
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
    k_p2m<<<order_grid(grid_for(C, kB), p), kB, 0, st>>>(C, t->c_first.as<int32_t>(), t->c_count.as<int32_t>(),
                               t->c_leaf.as<uint8_t>(), t->c_centre.as<double>(),
                               spos.as<double>(), smass.as<double>(), n, p,
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
