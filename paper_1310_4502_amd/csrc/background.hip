// Background subtraction, the exact part (Background Subtraction section:
// the uniform background inside the region around a sink group is removed
// through the analytic field of a uniform cube), and its adjoint.
//
// For periodic lists built with background subtraction, every sink gets
//   rho * ( sum over its group's listed boxes of sign * F_box(x)
//           - F_N(g)(x) + F_near-zone(x) ),
// rho = M_total / L^3 the mean density, N(g) the cube of `width` group sides
// about the group's centre and the near zone the 5L cube covered by the 125
// images. F_box is the unsoftened field of unit density filling a box:
//   F(x) = integral over the box of (y - x) / |y - x|^3 dy.
// Along z the w-integral of w / R^3 is -1/R at its ends and the remaining
// double integral of 1/R is a double difference of
//   Phi(a, b, c) = a ln(b + R) + b ln(a + R) - c atan(a b / (c R)),
// whose mixed derivative d^2 Phi / da db is 1/R; so
//   F_z = - sum over the 8 corners of s_u s_v s_w Phi(u, v, w),
// u, v, w the corner's offsets from x, s = +1 at the upper and -1 at the
// lower face, and F_x, F_y by symmetry. The three logarithms and the three
// arctangents of a corner are shared by the components. FP64 throughout.
#include "common.h"

namespace hot {
namespace {

constexpr int kB = 256;
constexpr int kWavesPerBlock = kB / 64;

// ln(b + R) for R = sqrt(b^2 + o2), o2 = sum of the other two squares > 0;
// for b < 0 as ln(o2 / (R - b)), which does not cancel.
__device__ __forceinline__ double ln_b_plus_r(double b, double o2, double R) {
  return b >= 0.0 ? log(b + R) : log(o2 / (R - b));
}

// adds the field of unit density on [lo, hi] at x into f
__device__ __forceinline__ void box_field(const double* __restrict__ lo,
                                          const double* __restrict__ hi, double x, double y,
                                          double z, double& fx, double& fy, double& fz) {
  const double u2[2] = {lo[0] - x, hi[0] - x};
  const double v2[2] = {lo[1] - y, hi[1] - y};
  const double w2[2] = {lo[2] - z, hi[2] - z};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double u = u2[i], v = v2[j], w = w2[k];
        const double uu = u * u, vv = v * v, ww = w * w;
        const double R = sqrt((uu + vv) + ww);
        // a log is needed only where a factor multiplying it is non-zero
        const double Lu = (v != 0.0 || w != 0.0) ? ln_b_plus_r(u, vv + ww, R) : 0.0;
        const double Lv = (u != 0.0 || w != 0.0) ? ln_b_plus_r(v, uu + ww, R) : 0.0;
        const double Lw = (u != 0.0 || v != 0.0) ? ln_b_plus_r(w, uu + vv, R) : 0.0;
        const double Ax = u != 0.0 ? u * atan((v * w) / (u * R)) : 0.0;
        const double Ay = v != 0.0 ? v * atan((u * w) / (v * R)) : 0.0;
        const double Az = w != 0.0 ? w * atan((u * v) / (w * R)) : 0.0;
        const double s = ((i ^ j ^ k) & 1) ? 1.0 : -1.0;
        fx -= s * ((v * Lw + w * Lv) - Ax);
        fy -= s * ((u * Lw + w * Lu) - Ay);
        fz -= s * ((u * Lv + v * Lu) - Az);
      }
}

// one wave per eval item (64 sinks of one group); adds into acc (caller order)
__global__ __launch_bounds__(kB) void k_bg_boxes(
    const int2* __restrict__ items, int64_t n_items, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const int32_t* __restrict__ g_cell,
    const double* __restrict__ c_centre, const int8_t* __restrict__ c_level,
    const int64_t* __restrict__ box_off, const double* __restrict__ boxes,
    const int8_t* __restrict__ box_sign, const uint32_t* __restrict__ perm,
    const double* __restrict__ pos, const double* __restrict__ mom64, double side, int width,
    double lo0, double lo1, double lo2, double* __restrict__ acc) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int i = item.y + lane;
  if (i >= g_first[g] + g_count[g]) return;
  const uint32_t ci = perm[i];
  const double x = pos[3 * ci], y = pos[3 * ci + 1], z = pos[3 * ci + 2];
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const int64_t b0 = box_off[g], b1 = box_off[g + 1];
  for (int64_t b = b0; b < b1; ++b) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    box_field(boxes + 6 * b, boxes + 6 * b + 3, x, y, z, gx, gy, gz);
    const double sg = (double)box_sign[b];
    fx += sg * gx;
    fy += sg * gy;
    fz += sg * gz;
  }
  {
    // minus N(g)
    const int gc = g_cell[g];
    const double h3 = (double)width * ldexp(side, -((int)c_level[gc] + 1));
    const double nlo[3] = {c_centre[3 * gc] - h3, c_centre[3 * gc + 1] - h3,
                           c_centre[3 * gc + 2] - h3};
    const double nhi[3] = {c_centre[3 * gc] + h3, c_centre[3 * gc + 1] + h3,
                           c_centre[3 * gc + 2] + h3};
    double gx = 0.0, gy = 0.0, gz = 0.0;
    box_field(nlo, nhi, x, y, z, gx, gy, gz);
    fx -= gx;
    fy -= gy;
    fz -= gz;
  }
  {
    // plus the near zone, the cube [lo - 2L, lo + 3L]
    const double zlo[3] = {lo0 - 2.0 * side, lo1 - 2.0 * side, lo2 - 2.0 * side};
    const double zhi[3] = {lo0 + 3.0 * side, lo1 + 3.0 * side, lo2 + 3.0 * side};
    box_field(zlo, zhi, x, y, z, fx, fy, fz);
  }
  const double rho = mom64[0] / ((side * side) * side);
  acc[3 * ci] += rho * fx;
  acc[3 * ci + 1] += rho * fy;
  acc[3 * ci + 2] += rho * fz;
}

// ---------------------------------------------------------------- adjoint
// Gradient of the box field, T_kl = d F_k / d x_l (symmetric). The mixed
// derivatives of Phi are ln(b + R) and -atan(a b / (c R)) up to terms that
// are constant in one of the two summed corner coordinates and cancel, so
//   T_xx = -sum s atan(v w / (u R)),  T_xy = sum s ln(w + R),
// and the others by symmetry. On the plane of a face the diagonal term takes
// its limit from the positive side; on the line of an edge the logarithm of
// the edge distance is dropped (it cancels between the edge's two corners
// wherever the gradient is finite).
__device__ __forceinline__ double log_edge(double b, double rho2, double R) {
  if (b >= 0.0) return R > 0.0 ? log(b + R) : 0.0;
  return rho2 > 0.0 ? log(rho2 / (R - b)) : -log(R - b);
}

__device__ __forceinline__ double atan_face(double num, double c, double R) {
  if (c != 0.0) return atan(num / (c * R));
  if (num == 0.0) return 0.0;
  return num > 0.0 ? 1.5707963267948966 : -1.5707963267948966;
}

// adds the field and the gradient of unit density on [lo, hi] at x, scaled by sg
__device__ __forceinline__ void box_field_grad(const double* __restrict__ lo,
                                               const double* __restrict__ hi, double x, double y,
                                               double z, double sg, double f[3], double T[6]) {
  const double u2[2] = {lo[0] - x, hi[0] - x};
  const double v2[2] = {lo[1] - y, hi[1] - y};
  const double w2[2] = {lo[2] - z, hi[2] - z};
  double fx = 0.0, fy = 0.0, fz = 0.0;
  double txx = 0.0, tyy = 0.0, tzz = 0.0, txy = 0.0, txz = 0.0, tyz = 0.0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double u = u2[i], v = v2[j], w = w2[k];
        const double uu = u * u, vv = v * v, ww = w * w;
        const double R = sqrt((uu + vv) + ww);
        const double s = ((i ^ j ^ k) & 1) ? 1.0 : -1.0;
        const double Lu = (v != 0.0 || w != 0.0) ? ln_b_plus_r(u, vv + ww, R) : 0.0;
        const double Lv = (u != 0.0 || w != 0.0) ? ln_b_plus_r(v, uu + ww, R) : 0.0;
        const double Lw = (u != 0.0 || v != 0.0) ? ln_b_plus_r(w, uu + vv, R) : 0.0;
        const double Au = atan_face(v * w, u, R);
        const double Av = atan_face(u * w, v, R);
        const double Aw = atan_face(u * v, w, R);
        fx -= s * ((v * Lw + w * Lv) - u * Au);
        fy -= s * ((u * Lw + w * Lu) - v * Av);
        fz -= s * ((u * Lv + v * Lu) - w * Aw);
        txx -= s * Au;
        tyy -= s * Av;
        tzz -= s * Aw;
        txy += s * log_edge(w, uu + vv, R);
        txz += s * log_edge(v, uu + ww, R);
        tyz += s * log_edge(u, vv + ww, R);
      }
  f[0] += sg * fx;
  f[1] += sg * fy;
  f[2] += sg * fz;
  T[0] += sg * txx;
  T[1] += sg * tyy;
  T[2] += sg * tzz;
  T[3] += sg * txy;
  T[4] += sg * txz;
  T[5] += sg * tyz;
}

// per sink: xbar += rho T^T abar (caller order) and, where the mass cotangent
// is wanted (dpsi non-null), dpsi[i] = abar . (B + cf) with B the unit-density
// box fields and cf the cube field of the expansions
__global__ __launch_bounds__(kB) void k_bg_boxes_adj(
    const int2* __restrict__ items, int64_t n_items, const int32_t* __restrict__ g_first,
    const int32_t* __restrict__ g_count, const int32_t* __restrict__ g_cell,
    const double* __restrict__ c_centre, const int8_t* __restrict__ c_level,
    const int64_t* __restrict__ box_off, const double* __restrict__ boxes,
    const int8_t* __restrict__ box_sign, const uint32_t* __restrict__ perm,
    const double* __restrict__ pos, const double* __restrict__ abar,
    const double* __restrict__ cf, const double* __restrict__ mom64, double side, int width,
    double lo0, double lo1, double lo2, double* __restrict__ xbar, double* __restrict__ dpsi) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (it >= n_items) return;
  const int2 item = items[it];
  const int g = uniform_i32(item.x);
  const int i = item.y + lane;
  if (i >= g_first[g] + g_count[g]) return;
  const uint32_t ci = perm[i];
  const double x = pos[3 * ci], y = pos[3 * ci + 1], z = pos[3 * ci + 2];
  double f[3] = {0.0, 0.0, 0.0}, T[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = box_off[g]; b < box_off[g + 1]; ++b)
    box_field_grad(boxes + 6 * b, boxes + 6 * b + 3, x, y, z, (double)box_sign[b], f, T);
  {
    const int gc = g_cell[g];
    const double h3 = (double)width * ldexp(side, -((int)c_level[gc] + 1));
    const double nlo[3] = {c_centre[3 * gc] - h3, c_centre[3 * gc + 1] - h3,
                           c_centre[3 * gc + 2] - h3};
    const double nhi[3] = {c_centre[3 * gc] + h3, c_centre[3 * gc + 1] + h3,
                           c_centre[3 * gc + 2] + h3};
    box_field_grad(nlo, nhi, x, y, z, -1.0, f, T);
  }
  {
    const double zlo[3] = {lo0 - 2.0 * side, lo1 - 2.0 * side, lo2 - 2.0 * side};
    const double zhi[3] = {lo0 + 3.0 * side, lo1 + 3.0 * side, lo2 + 3.0 * side};
    box_field_grad(zlo, zhi, x, y, z, 1.0, f, T);
  }
  const double rho = mom64[0] / ((side * side) * side);
  const double ax = abar[3 * ci], ay = abar[3 * ci + 1], az = abar[3 * ci + 2];
  xbar[3 * ci] += rho * ((T[0] * ax + T[3] * ay) + T[4] * az);
  xbar[3 * ci + 1] += rho * ((T[3] * ax + T[1] * ay) + T[5] * az);
  xbar[3 * ci + 2] += rho * ((T[4] * ax + T[5] * ay) + T[2] * az);
  if (dpsi)
    dpsi[ci] = ((ax * (f[0] + cf[3 * ci]) + ay * (f[1] + cf[3 * ci + 1])) +
                az * (f[2] + cf[3 * ci + 2]));
}

// deterministic sum: per block a fixed tree over a fixed grid-stride, then
// one block over the partials
constexpr int kRedBlocks = 512;
__global__ __launch_bounds__(256) void k_sum_partial(const double* __restrict__ v, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// mbar[j] += (sum of the partials) / L^3: the mean density is M_total / L^3
__global__ __launch_bounds__(256) void k_add_drho(const double* __restrict__ part, int np,
                                                   double inv_vol, int64_t n,
                                                   double* __restrict__ mbar) {
  __shared__ double tot;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < np; ++b) s += part[b];
    tot = s * inv_vol;
  }
  __syncthreads();
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    mbar[j] += tot;
}

}  // namespace

void background_adjoint(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass,
                        double eps, int precision, const double* abar, double* xbar,
                        double* mbar) {
  hipStream_t st = ctx->stream;
  const int64_t n = t->n;
  DBuf cf, dpsi;
  if (mbar) {
    // the mean density's cotangent: the expansions' cubes scale with it too,
    // so their field (an expansion pass over the flagged entries) is needed
    // only when the mass cotangent is asked for
    cf.alloc(ctx, n * 3 * sizeof(double));
    dpsi.alloc(ctx, n * sizeof(double));
    cube_field(ctx, t, pos, mass, eps, precision, cf.as<double>());
  }
  k_bg_boxes_adj<<<grid_for(t->n_items, kWavesPerBlock), kB, 0, st>>>(
      t->items.as<int2>(), t->n_items, t->g_first.as<int32_t>(), t->g_count.as<int32_t>(),
      t->g_cell.as<int32_t>(), t->c_centre.as<double>(), t->c_level.as<int8_t>(),
      t->box_off.as<int64_t>(), t->boxes.as<double>(), t->box_sign.as<int8_t>(),
      t->perm.as<uint32_t>(), pos, abar, cf.as<double>(), t->mom64.as<double>(), t->side,
      t->bg_width, t->lo[0], t->lo[1], t->lo[2], xbar, dpsi.as<double>());
  HOT_CHECK_LAUNCH();
  if (mbar) {
    DBuf part;
    part.alloc(ctx, kRedBlocks * sizeof(double));
    k_sum_partial<<<kRedBlocks, 256, 0, st>>>(dpsi.as<double>(), n, part.as<double>());
    HOT_CHECK_LAUNCH();
    k_add_drho<<<grid_for(n, 256), 256, 0, st>>>(part.as<double>(), kRedBlocks,
                                                 1.0 / ((t->side * t->side) * t->side), n, mbar);
    HOT_CHECK_LAUNCH();
  }
}

void background_boxes(hot_ctx* ctx, hot_tree* t, const double* pos, double* acc) {
  k_bg_boxes<<<grid_for(t->n_items, kWavesPerBlock), kB, 0, ctx->stream>>>(
      t->items.as<int2>(), t->n_items, t->g_first.as<int32_t>(), t->g_count.as<int32_t>(),
      t->g_cell.as<int32_t>(), t->c_centre.as<double>(), t->c_level.as<int8_t>(),
      t->box_off.as<int64_t>(), t->boxes.as<double>(), t->box_sign.as<int8_t>(),
      t->perm.as<uint32_t>(), pos, t->mom64.as<double>(), t->side, t->bg_width, t->lo[0],
      t->lo[1], t->lo[2], acc);
  HOT_CHECK_LAUNCH();
}

}  // namespace hot
