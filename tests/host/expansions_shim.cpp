// Host build of the generated expansion code (test harness only): the device
// qualifiers become plain inline functions and T = double.
#include <cmath>
#define __device__
#define __forceinline__ inline
#define HOT_ROW_BARRIER()
namespace hot {
inline double hot_fma(double a, double b, double c) { return std::fma(a, b, c); }
inline double hot_rsq(double x) { return 1.0 / std::sqrt(x); }
}  // namespace hot
#include "expansions.h"

template <int P>
static void fwd(int k1, const double* M, const double* R, double e2, double* out) {
  double ax = 0, ay = 0, az = 0, ph = 0;
  if (k1)
    hot::expansion_fwd<P, double, true, true>(R[0], R[1], R[2], e2, M, ax, ay, az, ph);
  else
    hot::expansion_fwd<P, double, true>(R[0], R[1], R[2], e2, M, ax, ay, az, ph);
  out[0] = ax, out[1] = ay, out[2] = az, out[3] = ph;
}
template <int P>
static void sink(int k1, const double* M, const double* R, double e2, const double* b, double* g) {
  double gx = 0, gy = 0, gz = 0;
  if (k1)
    hot::expansion_sink_adj<P, double, true>(R[0], R[1], R[2], e2, M, b[0], b[1], b[2], gx, gy,
                                             gz);
  else
    hot::expansion_sink_adj<P, double>(R[0], R[1], R[2], e2, M, b[0], b[1], b[2], gx, gy, gz);
  g[0] = gx, g[1] = gy, g[2] = gz;
}
template <int P>
static void cell(int k1, const double* R, double e2, const double* b, double* row) {
  if (k1)
    hot::expansion_cell_adj<P, double, true>(R[0], R[1], R[2], e2, b[0], b[1], b[2], row);
  else
    hot::expansion_cell_adj<P, double>(R[0], R[1], R[2], e2, b[0], b[1], b[2], row);
}

#define DISPATCH(F, ...)                 \
  switch (p) {                           \
    case 0: F<0>(__VA_ARGS__); break;    \
    case 1: F<1>(__VA_ARGS__); break;    \
    case 2: F<2>(__VA_ARGS__); break;    \
    case 3: F<3>(__VA_ARGS__); break;    \
    case 4: F<4>(__VA_ARGS__); break;    \
    case 5: F<5>(__VA_ARGS__); break;    \
    case 6: F<6>(__VA_ARGS__); break;    \
    case 7: F<7>(__VA_ARGS__); break;    \
    case 8: F<8>(__VA_ARGS__); break;    \
  }

extern "C" {
// k1: Dehnen's K1 softening with kernel radius sqrt(e2); else Plummer
void shim_fwd(int p, int k1, const double* M, const double* R, double e2, double* out) {
  DISPATCH(fwd, k1, M, R, e2, out);
}
void shim_sink(int p, int k1, const double* M, const double* R, double e2, const double* b,
               double* g) {
  DISPATCH(sink, k1, M, R, e2, b, g);
}
void shim_cell(int p, int k1, const double* R, double e2, const double* b, double* row) {
  DISPATCH(cell, k1, R, e2, b, row);
}
void shim_p2m(int N, double dx, double dy, double dz, double m, double* acc) {
  switch (N) {
    case 0: hot::p2m_order0(dx, dy, dz, m, acc); break;
    case 1: hot::p2m_order1(dx, dy, dz, m, acc); break;
    case 2: hot::p2m_order2(dx, dy, dz, m, acc); break;
    case 3: hot::p2m_order3(dx, dy, dz, m, acc); break;
    case 4: hot::p2m_order4(dx, dy, dz, m, acc); break;
    case 5: hot::p2m_order5(dx, dy, dz, m, acc); break;
    case 6: hot::p2m_order6(dx, dy, dz, m, acc); break;
    case 7: hot::p2m_order7(dx, dy, dz, m, acc); break;
    case 8: hot::p2m_order8(dx, dy, dz, m, acc); break;
  }
}
void shim_m2m(int N, const double* M, double dx, double dy, double dz, double* acc) {
  switch (N) {
    case 0: hot::m2m_order0(M, dx, dy, dz, acc); break;
    case 1: hot::m2m_order1(M, dx, dy, dz, acc); break;
    case 2: hot::m2m_order2(M, dx, dy, dz, acc); break;
    case 3: hot::m2m_order3(M, dx, dy, dz, acc); break;
    case 4: hot::m2m_order4(M, dx, dy, dz, acc); break;
    case 5: hot::m2m_order5(M, dx, dy, dz, acc); break;
    case 6: hot::m2m_order6(M, dx, dy, dz, acc); break;
    case 7: hot::m2m_order7(M, dx, dy, dz, acc); break;
    case 8: hot::m2m_order8(M, dx, dy, dz, acc); break;
  }
}
// transpose of the re-centring for a parent of order p, output order N
void shim_m2mT(int p, int N, const double* Mb, double dx, double dy, double dz, double* acc) {
  if (p == 0 && N == 0) hot::m2mT_p0_order0(Mb, dx, dy, dz, acc);
  if (p == 1 && N == 0) hot::m2mT_p1_order0(Mb, dx, dy, dz, acc);
  if (p == 1 && N == 1) hot::m2mT_p1_order1(Mb, dx, dy, dz, acc);
  if (p == 2 && N == 0) hot::m2mT_p2_order0(Mb, dx, dy, dz, acc);
  if (p == 2 && N == 1) hot::m2mT_p2_order1(Mb, dx, dy, dz, acc);
  if (p == 2 && N == 2) hot::m2mT_p2_order2(Mb, dx, dy, dz, acc);
  if (p == 3 && N == 0) hot::m2mT_p3_order0(Mb, dx, dy, dz, acc);
  if (p == 3 && N == 1) hot::m2mT_p3_order1(Mb, dx, dy, dz, acc);
  if (p == 3 && N == 2) hot::m2mT_p3_order2(Mb, dx, dy, dz, acc);
  if (p == 3 && N == 3) hot::m2mT_p3_order3(Mb, dx, dy, dz, acc);
  if (p == 4 && N == 0) hot::m2mT_p4_order0(Mb, dx, dy, dz, acc);
  if (p == 4 && N == 1) hot::m2mT_p4_order1(Mb, dx, dy, dz, acc);
  if (p == 4 && N == 2) hot::m2mT_p4_order2(Mb, dx, dy, dz, acc);
  if (p == 4 && N == 3) hot::m2mT_p4_order3(Mb, dx, dy, dz, acc);
  if (p == 4 && N == 4) hot::m2mT_p4_order4(Mb, dx, dy, dz, acc);
  if (p == 5 && N == 0) hot::m2mT_p5_order0(Mb, dx, dy, dz, acc);
  if (p == 5 && N == 1) hot::m2mT_p5_order1(Mb, dx, dy, dz, acc);
  if (p == 5 && N == 2) hot::m2mT_p5_order2(Mb, dx, dy, dz, acc);
  if (p == 5 && N == 3) hot::m2mT_p5_order3(Mb, dx, dy, dz, acc);
  if (p == 5 && N == 4) hot::m2mT_p5_order4(Mb, dx, dy, dz, acc);
  if (p == 5 && N == 5) hot::m2mT_p5_order5(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 0) hot::m2mT_p6_order0(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 1) hot::m2mT_p6_order1(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 2) hot::m2mT_p6_order2(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 3) hot::m2mT_p6_order3(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 4) hot::m2mT_p6_order4(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 5) hot::m2mT_p6_order5(Mb, dx, dy, dz, acc);
  if (p == 6 && N == 6) hot::m2mT_p6_order6(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 0) hot::m2mT_p7_order0(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 1) hot::m2mT_p7_order1(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 2) hot::m2mT_p7_order2(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 3) hot::m2mT_p7_order3(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 4) hot::m2mT_p7_order4(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 5) hot::m2mT_p7_order5(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 6) hot::m2mT_p7_order6(Mb, dx, dy, dz, acc);
  if (p == 7 && N == 7) hot::m2mT_p7_order7(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 0) hot::m2mT_p8_order0(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 1) hot::m2mT_p8_order1(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 2) hot::m2mT_p8_order2(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 3) hot::m2mT_p8_order3(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 4) hot::m2mT_p8_order4(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 5) hot::m2mT_p8_order5(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 6) hot::m2mT_p8_order6(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 7) hot::m2mT_p8_order7(Mb, dx, dy, dz, acc);
  if (p == 8 && N == 8) hot::m2mT_p8_order8(Mb, dx, dy, dz, acc);
}
// moment cotangents to one unit-mass particle at offset d: g[0..2] the
// position cotangent, g[3] the mass cotangent (accumulated into g)
void shim_p2mT(int p, const double* Mb, double dx, double dy, double dz, double* g) {
  if (p == 0) hot::p2mT_p0(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 1) hot::p2mT_p1(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 2) hot::p2mT_p2(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 3) hot::p2mT_p3(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 4) hot::p2mT_p4(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 5) hot::p2mT_p5(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 6) hot::p2mT_p6(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 7) hot::p2mT_p7(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
  if (p == 8) hot::p2mT_p8(Mb, dx, dy, dz, g[0], g[1], g[2], g[3]);
}
}
