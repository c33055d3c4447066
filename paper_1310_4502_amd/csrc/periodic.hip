// Periodic boundaries: the far replicas of the root cube (Boundary
// Conditions section). The near replicas -- the cube and its 124 neighbours,
// max|n_d| <= 2 -- are ordinary list entries carrying an image index; the
// rest of the infinite lattice, with a uniform neutralising background
// (Ewald's split; no surface term), is the smooth function
//   F(r) = psi(r) - sum_{max|n_d| <= 2} 1/|r + nL|,
// expanded about the cube centre c with the lattice sums T_gamma = d^gamma F(0)
// of Nijboer and De Wette. Per evaluation:
//   L_beta = sum_{|alpha| <= p} (-1)^|alpha|/alpha! M_alpha(root) T_{alpha+beta}   (|beta| <= p+1)
//   a_k(x) += sum_{|beta| <= p} (x - c)^beta/beta! L_{beta+e_k}.
// T is a constant of the cube side, computed once on the host in FP64.
// Adjoint: x_bar += sum_k abar_k sum_{|beta| <= p-1} u^beta/beta! L_{beta+e_k+e_l},
// and the root's moment cotangent w_alpha sum_gamma T_{alpha+gamma} D_gamma
// with D_gamma = sum_i sum_k abar_ik u_i^(gamma-e_k)/(gamma-e_k)!.
#include <cmath>
#include <vector>

#include "common.h"

namespace hot {
namespace {

constexpr int kTK = 2 * kMaxP + 1;  // highest derivative order needed
constexpr double kSplit = 2.0;      // Ewald split a = kSplit / L
constexpr double kRootPi = 1.7724538509055160273;

constexpr int tri(int n) { return n * (n + 1) * (n + 2) / 6; }
__host__ __device__ inline int slot3(int a, int b, int c) {
  const int n = a + b + c, bc = b + c;
  return n * (n + 1) * (n + 2) / 6 + bc * (bc + 1) / 2 + c;
}

// All derivatives d^(t,u,v) of a radial function h(|x|) at the point x, for
// t + u + v <= K, by the Hermite recursion of McMurchie and Davidson:
// R^(n)_000 = G_n (G_n = 2^n d^n h / ds^n, s = |x|^2),
// R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + x R^(n+1)_{t,u,v} (likewise u, v).
// out[slot3(t,u,v)] = R^(0)_{t,u,v}.
void hermite_all(const double x[3], const double* G, int K, double* out, std::vector<double>& R) {
  // R[n][t][u][v] with t + u + v + n <= K, stored densely (every entry read
  // is written first)
  const int D = K + 1;
  R.resize((size_t)D * D * D * D);
  auto at = [&](int n, int t, int u, int v) -> double& {
    return R[(((size_t)n * D + t) * D + u) * D + v];
  };
  for (int n = 0; n <= K; ++n) at(n, 0, 0, 0) = G[n];
  for (int s = 1; s <= K; ++s)  // total order of (t, u, v)
    for (int n = 0; n + s <= K; ++n)
      for (int t = s; t >= 0; --t)
        for (int u = s - t; u >= 0; --u) {
          const int v = s - t - u;
          double r;
          if (t > 0)
            r = (t > 1 ? (t - 1) * at(n + 1, t - 2, u, v) : 0.0) + x[0] * at(n + 1, t - 1, u, v);
          else if (u > 0)
            r = (u > 1 ? (u - 1) * at(n + 1, t, u - 2, v) : 0.0) + x[1] * at(n + 1, t, u - 1, v);
          else
            r = (v > 1 ? (v - 1) * at(n + 1, t, u, v - 2) : 0.0) + x[2] * at(n + 1, t, u, v - 1);
          at(n, t, u, v) = r;
        }
  for (int s = 0; s <= K; ++s)
    for (int t = s; t >= 0; --t)
      for (int u = s - t; u >= 0; --u) out[slot3(t, u, s - t - u)] = at(0, t, u, s - t - u);
}

// G_n for h = erfc(a r)/r (r > 0): (-1)^n B_n with B_0 = erfc(a r)/r and
// B_n = ((2n - 1) B_{n-1} + (2 a^2)^n e^(-a^2 r^2) / (a sqrt(pi))) / r^2.
void g_erfc(double r, double a, int K, double* G) {
  const double e = std::exp(-a * a * r * r) / (a * kRootPi);
  double B = std::erfc(a * r) / r, q = 1.0;
  G[0] = B;
  for (int n = 1; n <= K; ++n) {
    q *= 2.0 * a * a;
    B = ((2.0 * n - 1.0) * B + q * e) / (r * r);
    G[n] = (n & 1) ? -B : B;
  }
}

// G_n for h = erf(a r)/r: 1/r minus the erfc family, or the Taylor
// coefficients (2a/sqrt(pi)) (-2a^2)^n / (2n + 1) at r = 0.
void g_erf(double r, double a, int K, double* G) {
  if (r == 0.0) {
    double c = 2.0 * a / kRootPi;
    for (int n = 0; n <= K; ++n, c *= -2.0 * a * a) G[n] = c / (2.0 * n + 1.0);
    return;
  }
  g_erfc(r, a, K, G);
  double w = 1.0 / r;
  for (int n = 0; n <= K; ++n) {
    G[n] = w - G[n];  // 2^n d^n/ds^n s^(-1/2) = (-1)^n (2n-1)!! r^-(2n+1)
    w *= -(2.0 * n + 1.0) / (r * r);
  }
}

std::vector<double> lattice_sums(double L) {
  const int K = kTK;
  const double a = kSplit / L;
  std::vector<double> T(tri(K + 1), 0.0), d(tri(K + 1)), work;
  double G[kTK + 1];
  // real space: -erf terms over the near replicas, +erfc terms beyond
  for (int i = -6; i <= 6; ++i)
    for (int j = -6; j <= 6; ++j)
      for (int k = -6; k <= 6; ++k) {
        const int m = std::max(std::abs(i), std::max(std::abs(j), std::abs(k)));
        const double x[3] = {i * L, j * L, k * L};
        const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double sg = m <= 2 ? -1.0 : 1.0;
        if (m <= 2)
          g_erf(r, a, K, G);
        else
          g_erfc(r, a, K, G);
        hermite_all(x, G, K, d.data(), work);
        for (size_t s = 0; s < T.size(); ++s) T[s] += sg * d[s];
      }
  // reciprocal space: (4 pi/L^3) sum_{k != 0} e^(-k^2/4a^2)/k^2 Re(i^n) k^gamma
  const double tp = 2.0 * M_PI / L;
  for (int i = -10; i <= 10; ++i)
    for (int j = -10; j <= 10; ++j)
      for (int k = -10; k <= 10; ++k) {
        if (!i && !j && !k) continue;
        const double kv[3] = {tp * i, tp * j, tp * k};
        const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
        const double w = 4.0 * M_PI / (L * L * L) * std::exp(-k2 / (4.0 * a * a)) / k2;
        double pw[3][kTK + 1];
        for (int c = 0; c < 3; ++c) {
          pw[c][0] = 1.0;
          for (int e = 1; e <= K; ++e) pw[c][e] = pw[c][e - 1] * kv[c];
        }
        for (int s = 0; s <= K; s += 2) {
          const double sg = (s / 2) & 1 ? -1.0 : 1.0;
          for (int t = s; t >= 0; --t)
            for (int u = s - t; u >= 0; --u) {
              const int v = s - t - u;
              T[slot3(t, u, v)] += sg * w * (pw[0][t] * pw[1][u] * pw[2][v]);
            }
        }
      }
  // the neutralising background's constant (the k = 0 term of the split):
  // makes T_0 independent of the split; potentials only
  T[0] -= M_PI / (a * a * L * L * L);
  // F is even in every coordinate: entries with an odd exponent are zero
  for (int s = 0; s <= K; ++s)
    for (int t = s; t >= 0; --t)
      for (int u = s - t; u >= 0; --u)
        if ((t | u | (s - t - u)) & 1) T[slot3(t, u, s - t - u)] = 0.0;
  return T;
}

// one thread per beta: L_beta from the root's moments (slot order, nm(p))
__global__ void k_far_local(const double* __restrict__ M, int p, const double* __restrict__ T,
                            double* __restrict__ Lc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = tri(p + 2);
  if (b >= nb) return;
  // multi-index of slot b
  int n = 0;
  while (tri(n + 1) <= b) ++n;
  int r = b - tri(n), bx = n, by = 0;
  for (int a = n; a >= 0; --a) {
    if (r <= n - a) {
      bx = a;
      by = n - a - r;
      break;
    }
    r -= n - a + 1;
  }
  const int bz = n - bx - by;
  double acc = 0.0;
  for (int s = 0; s <= p; ++s)
    for (int a0 = s; a0 >= 0; --a0)
      for (int a1 = s - a0; a1 >= 0; --a1) {
        const int a2 = s - a0 - a1;
        double f = 1.0;
        for (int q = 2; q <= a0; ++q) f *= q;
        for (int q = 2; q <= a1; ++q) f *= q;
        for (int q = 2; q <= a2; ++q) f *= q;
        const double w = ((s & 1) ? -1.0 : 1.0) / f;
        acc += w * M[slot3(a0, a1, a2)] * T[slot3(a0 + bx, a1 + by, a2 + bz)];
      }
  Lc[b] = acc;
}

// a_k(x_i) += sum_{|beta| <= p} u^beta / beta! L_{beta + e_k}, u = x_i - c
// (pot, if not null: phi -= sum_{|beta| <= p} u^beta/beta! L_beta)
__global__ void k_far_l2p(const double* __restrict__ pos, int64_t n, const double* __restrict__ c,
                          int p, const double* __restrict__ Lc, double* __restrict__ acc,
                          double* __restrict__ pot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double u0 = pos[3 * i] - c[0], u1 = pos[3 * i + 1] - c[1], u2 = pos[3 * i + 2] - c[2];
  double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
  double px = 1.0;  // u0^a / a!
  for (int a = 0; a <= p; ++a) {
    double py = 1.0;
    for (int b = 0; a + b <= p; ++b) {
      double pz = 1.0;
      for (int d = 0; a + b + d <= p; ++d) {
        const double m = (px * py) * pz;
        ax += m * Lc[slot3(a + 1, b, d)];
        ay += m * Lc[slot3(a, b + 1, d)];
        az += m * Lc[slot3(a, b, d + 1)];
        ph -= m * Lc[slot3(a, b, d)];
        pz *= u2 / (d + 1);
      }
      py *= u1 / (b + 1);
    }
    px *= u0 / (a + 1);
  }
  acc[3 * i] += ax;
  acc[3 * i + 1] += ay;
  acc[3 * i + 2] += az;
  if (pot) pot[i] += ph;
}

// Adjoint of the far replicas (u = x_i - c, b_i the acceleration cotangent):
//   xbar_{i,l} += sum_k b_ik sum_{|beta| <= p-1} u^beta/beta! L_{beta+e_k+e_l},
//   Mbar_alpha(root) += w_alpha sum_{|gamma| <= p+1} T_{alpha+gamma} D_gamma,
//   D_gamma = sum_i sum_k b_ik u^(gamma-e_k)/(gamma-e_k)!   (gamma_k >= 1).
__global__ void k_far_l2p_adj(const double* __restrict__ pos, const double* __restrict__ abar,
                              int64_t n, const double* __restrict__ c, int p,
                              const double* __restrict__ Lc, double* __restrict__ xbar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double u0 = pos[3 * i] - c[0], u1 = pos[3 * i + 1] - c[1], u2 = pos[3 * i + 2] - c[2];
  const double b0 = abar[3 * i], b1 = abar[3 * i + 1], b2 = abar[3 * i + 2];
  double gx = 0.0, gy = 0.0, gz = 0.0;
  double px = 1.0;
  for (int a = 0; a < p; ++a) {
    double py = 1.0;
    for (int b = 0; a + b < p; ++b) {
      double pz = 1.0;
      for (int d = 0; a + b + d < p; ++d) {
        const double m = (px * py) * pz;
        // sum_k b_k L_{beta+e_k+e_l} for l = x, y, z
        const double hx = b0 * Lc[slot3(a + 2, b, d)] + b1 * Lc[slot3(a + 1, b + 1, d)] +
                          b2 * Lc[slot3(a + 1, b, d + 1)];
        const double hy = b0 * Lc[slot3(a + 1, b + 1, d)] + b1 * Lc[slot3(a, b + 2, d)] +
                          b2 * Lc[slot3(a, b + 1, d + 1)];
        const double hz = b0 * Lc[slot3(a + 1, b, d + 1)] + b1 * Lc[slot3(a, b + 1, d + 1)] +
                          b2 * Lc[slot3(a, b, d + 2)];
        gx += m * hx;
        gy += m * hy;
        gz += m * hz;
        pz *= u2 / (d + 1);
      }
      py *= u1 / (b + 1);
    }
    px *= u0 / (a + 1);
  }
  xbar[3 * i] += gx;
  xbar[3 * i + 1] += gy;
  xbar[3 * i + 2] += gz;
}

constexpr int kDTile = 128;  // particles staged per round
constexpr int kDBlocks = 1024;

// Per-block partial sums of D_gamma for every gamma of order <= p + 1 (one
// thread each, slot order; at most nm(kMaxP + 1) = 220 <= 256). A round
// stages a tile of particles in LDS as the scaled powers u_d^e / e! (e <= p)
// and their cotangents; thread gamma then adds, particle by particle,
// sum_k abar_k u^(gamma - e_k) / (gamma - e_k)!. Grid-stride over the tiles,
// fixed order: deterministic.
__global__ __launch_bounds__(256) void k_far_dpart(const double* __restrict__ pos,
                                                   const double* __restrict__ abar, int64_t n,
                                                   const double* __restrict__ c, int p, int ng,
                                                   double* __restrict__ part) {
  __shared__ double pw[kDTile][3][kMaxP + 1];
  __shared__ double bb[kDTile][3];
  const bool valid = (int)threadIdx.x < ng;
  int gx = 0, gy = 0, gz = 0;
  if (valid) {
    const int b = threadIdx.x;
    int nn = 0;
    while (tri(nn + 1) <= b) ++nn;
    int r = b - tri(nn), ex = nn, ey = 0;
    for (int a = nn; a >= 0; --a) {
      if (r <= nn - a) {
        ex = a;
        ey = nn - a - r;
        break;
      }
      r -= nn - a + 1;
    }
    gx = ex;
    gy = ey;
    gz = nn - ex - ey;
  }
  const double c0 = c[0], c1 = c[1], c2 = c[2];
  double acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * kDTile; base < n;
       base += (int64_t)gridDim.x * kDTile) {
    __syncthreads();
    if (threadIdx.x < kDTile) {
      const int j = threadIdx.x;
      const int64_t i = base + j;
      const bool in = i < n;
      const double u[3] = {in ? pos[3 * i] - c0 : 0.0, in ? pos[3 * i + 1] - c1 : 0.0,
                           in ? pos[3 * i + 2] - c2 : 0.0};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        bb[j][d] = in ? abar[3 * i + d] : 0.0;
        double v = 1.0;
        pw[j][d][0] = 1.0;
        for (int e = 1; e <= p; ++e) {
          v = v * u[d] / (double)e;
          pw[j][d][e] = v;
        }
      }
    }
    __syncthreads();
    if (valid) {
      for (int j = 0; j < kDTile; ++j) {
        double v = 0.0;
        if (gx > 0) v += bb[j][0] * ((pw[j][0][gx - 1] * pw[j][1][gy]) * pw[j][2][gz]);
        if (gy > 0) v += bb[j][1] * ((pw[j][0][gx] * pw[j][1][gy - 1]) * pw[j][2][gz]);
        if (gz > 0) v += bb[j][2] * ((pw[j][0][gx] * pw[j][1][gy]) * pw[j][2][gz - 1]);
        acc += v;
      }
    }
  }
  if (valid) part[(int64_t)blockIdx.x * ng + threadIdx.x] = acc;
}

// Mbar(root)_alpha += w_alpha sum_gamma T_{alpha+gamma} D_gamma, D from the partials
__global__ void k_far_mbar(const double* __restrict__ part, int nblocks, int ng, int p,
                           const double* __restrict__ T, double* __restrict__ mbar_root) {
  extern __shared__ double D[];
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * ng + g];
    D[g] = s;
  }
  __syncthreads();
  const int na = tri(p + 1);
  for (int al = threadIdx.x; al < na; al += blockDim.x) {
    int nn = 0;
    while (tri(nn + 1) <= al) ++nn;
    int r = al - tri(nn), ax = nn, ay = 0;
    for (int a = nn; a >= 0; --a) {
      if (r <= nn - a) {
        ax = a;
        ay = nn - a - r;
        break;
      }
      r -= nn - a + 1;
    }
    const int az = nn - ax - ay;
    double f = 1.0;
    for (int q = 2; q <= ax; ++q) f *= q;
    for (int q = 2; q <= ay; ++q) f *= q;
    for (int q = 2; q <= az; ++q) f *= q;
    const double w = ((nn & 1) ? -1.0 : 1.0) / f;
    double acc = 0.0;
    for (int s2 = 0; s2 <= p + 1; ++s2)
      for (int g0 = s2; g0 >= 0; --g0)
        for (int g1 = s2 - g0; g1 >= 0; --g1) {
          const int g2 = s2 - g0 - g1;
          acc += T[slot3(ax + g0, ay + g1, az + g2)] * D[slot3(g0, g1, g2)];
        }
    mbar_root[al] += w * acc;
  }
}

}  // namespace

void far_replicas_mbar(hot_ctx* ctx, hot_tree* t, const double* pos, const double* abar,
                       double* mbar_root) {
  hipStream_t st = ctx->stream;
  const int p = t->p, ng = tri(p + 2);
  DBuf part;
  part.alloc(ctx, (size_t)kDBlocks * ng * sizeof(double));
  k_far_dpart<<<kDBlocks, 256, 0, st>>>(pos, abar, t->n, t->c_centre.as<double>(), p, ng,
                                        part.as<double>());
  HOT_CHECK_LAUNCH();
  k_far_mbar<<<1, 256, ng * sizeof(double), st>>>(part.as<double>(), kDBlocks, ng, p,
                                                  t->lattice.as<double>(), mbar_root);
  HOT_CHECK_LAUNCH();
}

void far_replicas_xbar(hot_ctx* ctx, hot_tree* t, const double* pos, const double* abar,
                       double* xbar) {
  hipStream_t st = ctx->stream;
  const int p = t->p;
  DBuf Lc;
  Lc.alloc(ctx, tri(p + 2) * sizeof(double));
  k_far_local<<<grid_for(tri(p + 2), 256), 256, 0, st>>>(t->mom64.as<double>(), p,
                                                         t->lattice.as<double>(), Lc.as<double>());
  HOT_CHECK_LAUNCH();
  if (p >= 1) {
    k_far_l2p_adj<<<grid_for(t->n, 256), 256, 0, st>>>(pos, abar, t->n, t->c_centre.as<double>(),
                                                       p, Lc.as<double>(), xbar);
    HOT_CHECK_LAUNCH();
  }
}

void lattice_tensor(hot_ctx* ctx, hot_tree* t) {
  if (ctx->lattice_side != t->side) {
    ctx->lattice = lattice_sums(t->side);
    ctx->lattice_side = t->side;
  }
  const std::vector<double>& T = ctx->lattice;
  t->lattice.alloc(ctx, T.size() * sizeof(double));
  HOT_HIP(hipMemcpyAsync(t->lattice.p, T.data(), T.size() * sizeof(double),
                         hipMemcpyHostToDevice, ctx->stream));
  HOT_HIP(hipStreamSynchronize(ctx->stream));
}

void far_replicas(hot_ctx* ctx, hot_tree* t, const double* pos, double* acc, double* pot,
                  double* lc_mem) {
  hipStream_t st = ctx->stream;
  const int p = t->p;
  DBuf Lbuf;
  double* Lc = lc_mem;
  if (!Lc) {
    Lbuf.alloc(ctx, tri(p + 2) * sizeof(double));
    Lc = Lbuf.as<double>();
  }
  // every coefficient is written before k_far_l2p reads it
  k_far_local<<<grid_for(tri(p + 2), 256), 256, 0, st>>>(t->mom64.as<double>(), p,
                                                         t->lattice.as<double>(), Lc);
  HOT_CHECK_LAUNCH();
  k_far_l2p<<<grid_for(t->n, 256), 256, 0, st>>>(pos, t->n, t->c_centre.as<double>(), p, Lc, acc,
                                                 pot);
  HOT_CHECK_LAUNCH();
}

}  // namespace hot
