// CPU oracle for the hashed oct-tree gravitational force evaluation.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and
// the CPU-baseline leg of the benchmark may load or call this library. It
// shares no code, header, table or helper with the GPU library, and neither
// one includes or links the other.
//
// Everything here is plain FP64 and follows the definitions directly:
//   * O-D: direct summation of the softened Newtonian force (eq. "eom" of
//     the Mathematical Approach section at a = 1, G = 1, with the Plummer
//     smoothing of the "Force Smoothing" section), compensated sums.
//   * O-T: a scalar treecode taking the method's steps in order -- integer
//     Morton keys (Domain Decomposition section), a sort, an oct-tree of key
//     prefixes (Tree Construction section), moments about geometric cell
//     centres (Background Subtraction and Multipole Methods sections: the
//     moment tensor definition), a multipole acceptance walk over the source
//     tree for each sink cell (dual-tree traversal, m x n blocking of the
//     Improving instruction-level parallelism section) and the Cartesian
//     cell-body multipole expansion with Delta = 0 (Multipole Error Bounds
//     section), evaluated with the softened Green's function.
//   * Variants of the lists: an absolute-error acceptance test choosing the
//     order per interaction (Multipole Error Bounds section), periodic
//     boundaries with far replicas by lattice sums (Boundary Conditions
//     section), and on top of the periodic lists background subtraction
//     (Background Subtraction section: density contrasts, cube moments
//     subtracted to the matter's order, exact uniform-box fields).
//   * The VJP (reverse derivative) of O-D and of O-T with the tree topology
//     held fixed.
//
// Build flags: -O2 -ffp-contract=off, never fast-math, so that every FP64
// expression below is evaluated exactly as written (IEEE, correctly rounded,
// no fused multiply-add).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

thread_local std::string g_err;

int fail(const char* msg) {
  g_err = msg;
  return -1;
}

constexpr int kBits = 21;  // bits per axis in a key; 63 key bits + placeholder

// ---------------------------------------------------------------------------
// Keys (Domain Decomposition section: coordinates are mapped to integer keys;
// the format itself is deferred by the paper to its 1993 predecessor). Reading
// used here: 21 bits per axis, octant digit 4x + 2y + z, most significant
// digit first, a leading placeholder bit so that a level-L cell key is the
// particle key shifted right by 3 (21 - L).
// ---------------------------------------------------------------------------
uint64_t interleave(uint32_t qx, uint32_t qy, uint32_t qz) {
  uint64_t k = 0;
  for (int b = kBits - 1; b >= 0; --b) {
    uint64_t digit = (uint64_t)(((qx >> b) & 1u) * 4u + ((qy >> b) & 1u) * 2u + ((qz >> b) & 1u));
    k = k * 8u + digit;
  }
  return k;
}

void deinterleave(uint64_t k, int ndigits, uint32_t* ix, uint32_t* iy, uint32_t* iz) {
  uint32_t x = 0, y = 0, z = 0;
  for (int d = ndigits - 1; d >= 0; --d) {
    uint64_t digit = (k >> (3 * d)) & 7u;
    x = x * 2u + (uint32_t)((digit >> 2) & 1u);
    y = y * 2u + (uint32_t)((digit >> 1) & 1u);
    z = z * 2u + (uint32_t)(digit & 1u);
  }
  *ix = x;
  *iy = y;
  *iz = z;
}

bool is_pow2(double s) {
  if (!(s > 0) || !std::isfinite(s)) return false;
  int e;
  double m = std::frexp(s, &e);
  return m == 0.5;
}

// Root cube: lo = per-axis minimum, side = the power of two at or above the
// largest extent (1 if every point coincides).
void root_cube(int64_t n, const double* pos, double lo[3], double* side) {
  for (int d = 0; d < 3; ++d) {
    double m = pos[d];
    for (int64_t i = 1; i < n; ++i) m = std::min(m, pos[3 * i + d]);
    lo[d] = m;
  }
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) {
    double mx = pos[d];
    for (int64_t i = 1; i < n; ++i) mx = std::max(mx, pos[3 * i + d]);
    ext = std::max(ext, mx - lo[d]);
  }
  if (ext == 0.0) {
    *side = 1.0;
    return;
  }
  int e;
  double m = std::frexp(ext, &e);  // ext = m 2^e, m in [0.5, 1)
  *side = (m == 0.5) ? ext : std::ldexp(1.0, e);
}

uint32_t quantise(double x, double lo, double scale) {
  double t = std::floor((x - lo) * scale);
  const double qmax = (double)((1u << kBits) - 1u);
  if (t > qmax) t = qmax;
  if (t < 0) t = 0;
  return (uint32_t)t;
}

// ---------------------------------------------------------------------------
// Tree
// ---------------------------------------------------------------------------
struct Cell {
  int level;
  uint64_t key;  // prefix with placeholder bit
  int64_t first, count;
  int64_t parent;
  int64_t child_first;
  int n_child;
  int is_leaf;
  double centre[3];
  double bmax;
};

struct Tree {
  int64_t n = 0;
  int n_leaf = 16, n_group = 64;
  double lo[3] = {0, 0, 0};
  double side = 1.0;
  std::vector<uint64_t> key;   // sorted keys
  std::vector<int64_t> perm;   // sorted position -> caller index
  std::vector<Cell> cells;     // canonical order: (level, key)
  std::vector<int64_t> groups; // cell ids, ordered by first particle
  std::vector<int64_t> group_of;  // sorted position -> group ordinal
  std::vector<int64_t> leaf_of;   // sorted position -> leaf cell id
  int max_level = 0;
  // interaction lists, CSR over groups
  bool has_lists = false;
  double theta = 0;
  int direct_max = 0;
  std::vector<int64_t> p2p_off, m2p_off;
  std::vector<int32_t> p2p, m2p;
  std::vector<char> list_sel;  // empty: every group has its lists
  // error-bound lists: expansion order of every M2P entry (empty for theta lists)
  std::vector<int8_t> m2p_q;
  int list_p = -1;  // highest order an entry may use (error-bound lists)
  // periodic lists: the image (0 .. 124) of every entry; empty otherwise
  std::vector<int8_t> p2p_img, m2p_img;
  bool periodic = false;
  // background subtraction (periodic lists only): M2P entries whose cell lies
  // outside the group's neighbourhood (1: the cell's uniform cube is taken
  // off its moments), and per group the boxes whose uniform field is added
  // exactly, with sign +1 or -1 (CSR, 6 doubles lo[3], hi[3] per box)
  bool bg = false;
  int bg_width = 3;  // side of N(g) in group sides (odd)
  std::vector<int8_t> m2p_sub;
  std::vector<int64_t> box_off;
  std::vector<double> boxes;
  std::vector<int8_t> box_sign;
  // moments
  int p = -1;
  std::vector<double> mom;        // n_cells x nm(p)
  std::vector<char> mom_valid;
};

int nm(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Multi-index (a, b, c) <-> storage slot: by order n = a+b+c, then a
// descending, then b descending.
int mindex(int a, int b, int c) {
  int n = a + b + c;
  return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

std::vector<int> g_alpha;  // 3 entries per slot, filled up to order 12
void ensure_alpha() {
  if (!g_alpha.empty()) return;
  const int pmax = 12;
  g_alpha.resize(3 * nm(pmax));
  for (int n = 0; n <= pmax; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        int c = n - a - b;
        int s = mindex(a, b, c);
        g_alpha[3 * s] = a;
        g_alpha[3 * s + 1] = b;
        g_alpha[3 * s + 2] = c;
      }
}

double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

double factorial(int k) {
  double r = 1.0;
  for (int i = 2; i <= k; ++i) r *= i;
  return r;
}

void cell_centre(const Tree& t, int level, uint64_t key, double c[3]) {
  uint32_t ix, iy, iz;
  deinterleave(key, level, &ix, &iy, &iz);  // the placeholder bit lies above the digits
  double h = std::ldexp(t.side, -(level + 1));
  uint32_t ic[3] = {ix, iy, iz};
  for (int d = 0; d < 3; ++d) c[d] = t.lo[d] + (double)(2u * ic[d] + 1u) * h;
}

// b_max: largest distance from the geometric centre to a particle of the cell
// (the source radius of the Multipole Error Bounds section's figure).
double cell_bmax(const double* spos, const Cell& c) {
  double m = 0.0;
  for (int64_t j = c.first; j < c.first + c.count; ++j) {
    double dx = spos[3 * j] - c.centre[0];
    double dy = spos[3 * j + 1] - c.centre[1];
    double dz = spos[3 * j + 2] - c.centre[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    if (d2 > m) m = d2;
  }
  return std::sqrt(m);
}

int build_tree(Tree& t, int64_t n, const double* pos, const double* box) {
  t.n = n;
  if (box) {
    for (int d = 0; d < 3; ++d) t.lo[d] = box[d];
    t.side = box[3];
  } else {
    root_cube(n, pos, t.lo, &t.side);
  }
  int e;
  std::frexp(t.side, &e);  // side = 2^(e-1)
  double scale = std::ldexp(1.0, kBits - (e - 1));
  std::vector<uint64_t> k0(n);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) q[d] = quantise(pos[3 * i + d], t.lo[d], scale);
    k0[i] = (1ull << 63) | interleave(q[0], q[1], q[2]);
  }
  // Stable sort by key: equal keys keep caller order.
  t.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) t.perm[i] = i;
  std::stable_sort(t.perm.begin(), t.perm.end(),
                   [&](int64_t a, int64_t b) { return k0[a] < k0[b]; });
  t.key.resize(n);
  for (int64_t i = 0; i < n; ++i) t.key[i] = k0[t.perm[i]];
  std::vector<double> spos(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) spos[3 * i + d] = pos[3 * t.perm[i] + d];

  // Cells level by level, children in octant order: a cell splits when it
  // holds more than n_leaf particles and is above the deepest level.
  t.cells.clear();
  Cell root{};
  root.level = 0;
  root.key = 1;
  root.first = 0;
  root.count = n;
  root.parent = -1;
  t.cells.push_back(root);
  size_t level_begin = 0;
  for (int L = 0; L <= kBits; ++L) {
    size_t level_end = t.cells.size();
    for (size_t ci = level_begin; ci < level_end; ++ci) {
      Cell& c = t.cells[ci];
      c.child_first = -1;
      c.n_child = 0;
      c.is_leaf = !(c.count > t.n_leaf && L < kBits);
      if (c.is_leaf) continue;
      int shift = 3 * (kBits - (L + 1));
      int64_t j = c.first, end = c.first + c.count;
      int64_t cf = (int64_t)t.cells.size();
      int nc = 0;
      while (j < end) {
        uint64_t pre = t.key[j] >> shift;
        int64_t k = j;
        while (k < end && (t.key[k] >> shift) == pre) ++k;
        Cell ch{};
        ch.level = L + 1;
        ch.key = pre;
        ch.first = j;
        ch.count = k - j;
        ch.parent = (int64_t)ci;
        t.cells.push_back(ch);
        ++nc;
        j = k;
      }
      t.cells[ci].child_first = cf;
      t.cells[ci].n_child = nc;
    }
    level_begin = level_end;
    if (level_begin == t.cells.size()) break;
  }
  t.max_level = 0;
  t.leaf_of.assign(n, -1);
  for (size_t ci = 0; ci < t.cells.size(); ++ci) {
    Cell& c = t.cells[ci];
    cell_centre(t, c.level, c.key, c.centre);
    c.bmax = cell_bmax(spos.data(), c);
    t.max_level = std::max(t.max_level, c.level);
    if (c.is_leaf)
      for (int64_t j = c.first; j < c.first + c.count; ++j) t.leaf_of[j] = (int64_t)ci;
  }
  // Sink groups: the topmost cells holding at most n_group particles, or a
  // leaf that still holds more.
  t.groups.clear();
  for (size_t ci = 0; ci < t.cells.size(); ++ci) {
    const Cell& c = t.cells[ci];
    bool top_small = c.count <= t.n_group &&
                     (c.parent < 0 || t.cells[c.parent].count > t.n_group);
    bool big_leaf = c.is_leaf && c.count > t.n_group;
    if (top_small || big_leaf) t.groups.push_back((int64_t)ci);
  }
  std::sort(t.groups.begin(), t.groups.end(),
            [&](int64_t a, int64_t b) { return t.cells[a].first < t.cells[b].first; });
  t.group_of.assign(n, -1);
  for (size_t g = 0; g < t.groups.size(); ++g) {
    const Cell& c = t.cells[t.groups[g]];
    for (int64_t j = c.first; j < c.first + c.count; ++j) t.group_of[j] = (int64_t)g;
  }
  for (int64_t j = 0; j < n; ++j)
    if (t.group_of[j] < 0) return fail("internal: particle without a group");
  t.has_lists = false;
  t.p = -1;
  t.mom.clear();
  t.mom_valid.clear();
  return 0;
}

// ---------------------------------------------------------------------------
// Multipole acceptance (Multipole Error Bounds section, figure of the source
// cell V of radius b_max and sink cell W): reading used here is the group
// form of the b_max / theta criterion -- accept iff the centre distance
// exceeds b_source / theta + b_sink, compared in squares, strict.
// ---------------------------------------------------------------------------
bool accept(const Cell& g, const Cell& c, double theta) {
  double dx = g.centre[0] - c.centre[0];
  double dy = g.centre[1] - c.centre[1];
  double dz = g.centre[2] - c.centre[2];
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double r = c.bmax / theta + g.bmax;
  return d2 > r * r;
}

void walk(const Tree& t, const Cell& g, int64_t ci, double theta, int direct_max,
          std::vector<int32_t>& p2p, std::vector<int32_t>& m2p) {
  const Cell& c = t.cells[ci];
  if (accept(g, c, theta)) {
    if (c.count <= direct_max)
      p2p.push_back((int32_t)ci);
    else
      m2p.push_back((int32_t)ci);
    return;
  }
  if (c.is_leaf) {
    p2p.push_back((int32_t)ci);
    return;
  }
  for (int k = 0; k < c.n_child; ++k) walk(t, g, c.child_first + k, theta, direct_max, p2p, m2p);
}

// ---------------------------------------------------------------------------
// Error-bound acceptance with the order chosen per interaction (Multipole
// Error Bounds section: an absolute-error MAC that picks, per interaction,
// the cheapest expansion order meeting the accuracy). The paper's own bounds
// are in a reference that is not at hand; the reading used here is the
// classical bound on the field of a truncated cell-body expansion of 1/r:
// sources of total mass M within radius b of the expansion centre, field
// point at distance d > b from it, expansion to order q:
//   |a - a_q| <= M / (d - b)^2 * ((q + 2) - (q + 1) t) * t^(q + 1),  t = b / d,
// the sum over n > q of (n + 1) b^n / d^(n + 2) (each degree-n term of the
// Taylor series is a Legendre term bounded by b^n / d^(n + 1), its gradient
// by (n + 1) b^n / d^(n + 2)). A sink of group g lies within b_max(g) of its
// centre, so d = |centre_g - centre_c| - b_max(g); M is bounded by the
// cell's particle count times the largest particle mass (exact arithmetic on
// both sides of the parity tests). The smallest q in [0, p_max] whose bound is
// at most tol is taken; if there is none (or d <= b), the cell is opened.
// FP64, no FMA, this exact order of operations.
// ---------------------------------------------------------------------------
int accept_order_d(double dx, double dy, double dz, const Cell& g, const Cell& c, double tol,
                   double mmax, int pmax) {
  double d = std::sqrt((dx * dx + dy * dy) + dz * dz) - g.bmax;
  double b = c.bmax;
  if (!(d > b)) return -1;
  double t = b / d;
  double h = d - b;
  double A = ((double)c.count * mmax) / (h * h);
  double tp = t;
  for (int q = 0; q <= pmax; ++q) {
    double E = (A * ((double)(q + 2) - (double)(q + 1) * t)) * tp;
    if (E <= tol) return q;
    tp = tp * t;
  }
  return -1;
}

int accept_order(const Cell& g, const Cell& c, double tol, double mmax, int pmax) {
  double dx = g.centre[0] - c.centre[0];
  double dy = g.centre[1] - c.centre[1];
  double dz = g.centre[2] - c.centre[2];
  return accept_order_d(dx, dy, dz, g, c, tol, mmax, pmax);
}

void walk_err(const Tree& t, const Cell& g, int64_t ci, double tol, double mmax, int pmax,
              int direct_max, std::vector<int32_t>& p2p, std::vector<int32_t>& m2p,
              std::vector<int8_t>& m2p_q) {
  const Cell& c = t.cells[ci];
  const int q = accept_order(g, c, tol, mmax, pmax);
  if (q >= 0) {
    if (c.count <= direct_max) {
      p2p.push_back((int32_t)ci);
    } else {
      m2p.push_back((int32_t)ci);
      m2p_q.push_back((int8_t)q);
    }
    return;
  }
  if (c.is_leaf) {
    p2p.push_back((int32_t)ci);
    return;
  }
  for (int k = 0; k < c.n_child; ++k)
    walk_err(t, g, c.child_first + k, tol, mmax, pmax, direct_max, p2p, m2p, m2p_q);
}

// theta >= 0: theta lists; theta < 0: error-bound lists with (tol, mmax, pmax)
int build_lists(Tree& t, double theta, int direct_max, const std::vector<char>& want,
                double tol = 0, double mmax = 0, int pmax = -1) {
  const int64_t G = (int64_t)t.groups.size();
  const bool err = theta < 0;
  std::vector<std::vector<int32_t>> lp(G), lm(G);
  std::vector<std::vector<int8_t>> lq(G);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < G; ++g) {
    if (!(want.empty() || want[g])) continue;
    if (err)
      walk_err(t, t.cells[t.groups[g]], 0, tol, mmax, pmax, direct_max, lp[g], lm[g], lq[g]);
    else
      walk(t, t.cells[t.groups[g]], 0, theta, direct_max, lp[g], lm[g]);
  }
  t.p2p_off.assign(G + 1, 0);
  t.m2p_off.assign(G + 1, 0);
  for (int64_t g = 0; g < G; ++g) {
    t.p2p_off[g + 1] = t.p2p_off[g] + (int64_t)lp[g].size();
    t.m2p_off[g + 1] = t.m2p_off[g] + (int64_t)lm[g].size();
  }
  t.p2p.resize(t.p2p_off[G]);
  t.m2p.resize(t.m2p_off[G]);
  for (int64_t g = 0; g < G; ++g) {
    std::copy(lp[g].begin(), lp[g].end(), t.p2p.begin() + t.p2p_off[g]);
    std::copy(lm[g].begin(), lm[g].end(), t.m2p.begin() + t.m2p_off[g]);
  }
  t.m2p_q.clear();
  t.p2p_img.clear();
  t.m2p_img.clear();
  t.periodic = false;
  t.bg = false;
  t.m2p_sub.clear();
  t.box_off.clear();
  t.boxes.clear();
  t.box_sign.clear();
  if (err) {
    t.m2p_q.resize(t.m2p_off[G]);
    for (int64_t g = 0; g < G; ++g) std::copy(lq[g].begin(), lq[g].end(), t.m2p_q.begin() + t.m2p_off[g]);
  }
  t.list_p = err ? pmax : -1;
  t.has_lists = true;
  t.theta = theta;
  t.direct_max = direct_max;
  return 0;
}

// ---------------------------------------------------------------------------
// Moments (Multipole Error Bounds section, the moment tensor about a centre z):
// M_alpha(z) = sum_j m_j (y_j - z)^alpha, raw (not traceless) multi-index
// moments, |alpha| <= p, about the geometric cell centre.
// ---------------------------------------------------------------------------
// The sum over the cell's particles is Neumaier-compensated, so that its
// rounding does not grow with the particle count: the result is the
// definition's value up to the rounding of the individual terms.
void p2m_direct(const double* spos, const double* smass, const Cell& c, int p, double* out) {
  const int K = nm(p);
  std::vector<double> comp(K, 0.0);
  for (int s = 0; s < K; ++s) out[s] = 0.0;
  for (int64_t j = c.first; j < c.first + c.count; ++j) {
    double d[3] = {spos[3 * j] - c.centre[0], spos[3 * j + 1] - c.centre[1],
                   spos[3 * j + 2] - c.centre[2]};
    for (int s = 0; s < K; ++s) {
      const int* al = &g_alpha[3 * s];
      const double x = smass[j] * (ipow(d[0], al[0]) * ipow(d[1], al[1]) * ipow(d[2], al[2]));
      const double t = out[s] + x;
      comp[s] += std::fabs(out[s]) >= std::fabs(x) ? (out[s] - t) + x : (x - t) + out[s];
      out[s] = t;
    }
  }
  for (int s = 0; s < K; ++s) out[s] += comp[s];
}

// ---------------------------------------------------------------------------
// Softening kernels (Force Smoothing section). Two kernels are provided:
//   * Plummer: the potential of a unit mass is -(r^2 + eps^2)^(-1/2);
//   * K1, Dehnen's compensating kernel with compact support (the section
//     names it as the one used for production runs; its defining reference
//     is not at hand, so the reading used here builds it from the properties
//     the section and that reference state): the unit mass is spread with the
//     density
//       rho(r) = 1575 / (128 pi eps^3) (1 - x^2)^2 (1 - 11 x^2 / 5),  x = r / eps < 1,
//     and nothing beyond eps. (1 - x^2)^2 makes the density vanish with its
//     slope at the edge; the second factor is the lowest-degree one giving
//     unit mass and a zero second moment, int r^2 rho d^3r = 0, the
//     compensation that cancels the leading-order force bias (the density is
//     negative for x > sqrt(5/11), and the force exceeds the Newtonian one
//     over part of the kernel). Enclosed mass mu(x) and potential follow by
//     integration:
//       mu(x)  = x^3 (525 - 1323 x^2 + 1215 x^4 - 385 x^6) / 32,
//       psi(r) = (945 - 2100 x^2 + 2646 x^4 - 1620 x^6 + 385 x^8) / (256 eps)
//     (phi = -m psi); for r >= eps, mu = 1 and psi = 1/r exactly.
// A pair term is written as acceleration m r K(r^2) with r = x_j - x_i and
// Hessian d(r K)/dr = K I + B r r^T; the expansion needs f(s) with
// G(R) = f(|R|^2 + eps^2) (Plummer) or f(|R|^2) (K1).
// ---------------------------------------------------------------------------
enum { kPlummer = 0, kK1 = 1 };

struct Soft {
  int kind;
  double eps;
};

int check_soft(int kind, double eps) {
  if (!(eps >= 0) || !std::isfinite(eps)) return fail("eps must be finite and >= 0");
  if (kind != kPlummer && kind != kK1) return fail("unknown softening kernel");
  return 0;
}

struct PairTerms {
  double K;    // acceleration per unit mass and unit offset
  double psi;  // minus the potential per unit mass
  double B;    // coefficient of r r^T in the Hessian
};

// r2 = |r|^2. Returns false for a pair that contributes nothing (zero
// separation with nothing to soften it).
bool pair_terms(const Soft& sf, double r2, PairTerms* o) {
  if (sf.kind == kK1 && r2 < sf.eps * sf.eps) {
    const double e = sf.eps;
    const double u = r2 / (e * e);
    const double e3 = e * e * e;
    o->K = (525.0 + u * (-1323.0 + u * (1215.0 - 385.0 * u))) / (32.0 * e3);
    o->psi = (945.0 + u * (-2100.0 + u * (2646.0 + u * (-1620.0 + 385.0 * u)))) / (256.0 * e);
    o->B = (-1323.0 + u * (2430.0 - 1155.0 * u)) / (16.0 * e3 * e * e);
    return true;
  }
  const double s = sf.kind == kK1 ? r2 : r2 + sf.eps * sf.eps;
  if (s == 0.0) return false;
  const double inv = 1.0 / std::sqrt(s);
  const double inv3 = inv * inv * inv;
  o->K = inv3;
  o->psi = inv;
  o->B = -3.0 * inv3 * inv * inv;
  return true;
}

// ---------------------------------------------------------------------------
// Derivatives of the softened Green's function G(R) = -(|R|^2 + eps^2)^(-1/2)
// (Force Smoothing section: Plummer smoothing; the expansion of the Multipole
// Error Bounds section is written for an arbitrary G). For any f(s) with
// s = |R|^2 + eps^2, the chain rule gives, per axis,
//   d^a/dx^a f = sum_j a! / (j! (a-2j)!) (2x)^(a-2j) f^(a-j)(s),
// and the three axes compose. With f(s) = -s^(-1/2),
//   2^n f^(n)(s) = (-1)^(n+1) (2n-1)!! s^(-n-1/2).
// ---------------------------------------------------------------------------
struct Radial {
  double F[24];  // F[n] = 2^n f^(n)(s)
};

Radial radial(double s, int nmax) {
  Radial r;
  double is = 1.0 / s;
  double v = 1.0 / std::sqrt(s);  // s^(-1/2)
  double dfact = 1.0;             // (2n-1)!!, with (-1)!! = 1
  for (int n = 0; n <= nmax; ++n) {
    double sign = (n % 2 == 0) ? -1.0 : 1.0;  // (-1)^(n+1)
    r.F[n] = sign * dfact * v;
    dfact *= (double)(2 * n + 1);
    v *= is;
  }
  return r;
}

// F[n] = 2^n f^(n) for the kernel: Plummer takes s = r2 + eps^2 in the form
// above; K1 takes s = r2, the form above outside eps and inside
// f(s) = -P(s / eps^2) / (256 eps), P(u) = 945 - 2100 u + 2646 u^2 - 1620 u^3
// + 385 u^4, so f^(n)(s) = -P^(n)(u) / (256 eps^(2n+1)) (zero for n > 4).
Radial radial_soft(const Soft& sf, double r2, int nmax) {
  if (sf.kind == kPlummer) return radial(r2 + sf.eps * sf.eps, nmax);
  if (!(r2 < sf.eps * sf.eps)) return radial(r2, nmax);
  Radial r;
  const double e = sf.eps;
  const double u = r2 / (e * e);
  // coefficients of P and of its successive derivatives, lowest power first
  double c[5] = {945.0, -2100.0, 2646.0, -1620.0, 385.0};
  int deg = 4;
  double scale = -1.0 / (256.0 * e);  // 2^n / (256 eps^(2n+1)), negated
  for (int n = 0; n <= nmax; ++n) {
    double v = 0.0;
    for (int k = deg; k >= 0; --k) v = v * u + c[k];
    r.F[n] = deg >= 0 ? scale * v : 0.0;
    // differentiate P once
    for (int k = 0; k < deg; ++k) c[k] = c[k + 1] * (double)(k + 1);
    if (deg >= 0) c[deg] = 0.0;
    --deg;
    scale *= 2.0 / (e * e);
  }
  return r;
}

// d^alpha G at R, from the closed-form sum above.
double dG(int a, int b, int c, const double R[3], const Radial& rad) {
  const int al[3] = {a, b, c};
  double total = 0.0;
  for (int gx = 0; 2 * gx <= a; ++gx)
    for (int gy = 0; 2 * gy <= b; ++gy)
      for (int gz = 0; 2 * gz <= c; ++gz) {
        const int g[3] = {gx, gy, gz};
        double term = 1.0;
        for (int d = 0; d < 3; ++d) {
          int e = al[d] - 2 * g[d];
          term *= factorial(al[d]) / (factorial(g[d]) * factorial(e)) * ipow(2.0 * R[d], e);
        }
        int order = a + b + c - (gx + gy + gz);
        // (2R)^e f^(order) = R^e 2^(sum e) f^(order) and sum e = 2 order - |alpha|,
        // so term * f^(order) = term * F[order] / 2^order.
        total += term * rad.F[order] * std::ldexp(1.0, -order);
      }
  return total;
}

// Cell-body expansion (Delta = 0): the potential at R = x - centre is
//   phi = sum_{|alpha|<=p} (-1)^|alpha| / alpha! M_alpha d^alpha G(R)
// and the acceleration a_k = -d phi / d x_k.
void m2p_one(const double* M, int p, const double R[3], const Soft& sf, double acc[3],
             double* phi) {
  const double r2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
  Radial rad = radial_soft(sf, r2, p + 1);
  double a[3] = {0, 0, 0}, ph = 0.0;
  for (int sl = 0; sl < nm(p); ++sl) {
    const int* al = &g_alpha[3 * sl];
    int n = al[0] + al[1] + al[2];
    double w = ((n % 2) ? -1.0 : 1.0) / (factorial(al[0]) * factorial(al[1]) * factorial(al[2]));
    double wm = w * M[sl];
    ph += wm * dG(al[0], al[1], al[2], R, rad);
    a[0] -= wm * dG(al[0] + 1, al[1], al[2], R, rad);
    a[1] -= wm * dG(al[0], al[1] + 1, al[2], R, rad);
    a[2] -= wm * dG(al[0], al[1], al[2] + 1, R, rad);
  }
  acc[0] = a[0];
  acc[1] = a[1];
  acc[2] = a[2];
  if (phi) *phi = ph;
}

// Softened pair kernel: contribution of source j (mass m, offset r = x_j - x_i).
inline void p2p_pair(double m, const double r[3], const Soft& sf, double acc[3], double* phi) {
  PairTerms pt;
  if (!pair_terms(sf, (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2], &pt)) return;
  for (int d = 0; d < 3; ++d) acc[d] += m * r[d] * pt.K;
  if (phi) *phi -= m * pt.psi;
}

// Neumaier-compensated accumulator.
struct NSum {
  double s = 0, c = 0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// ---------------------------------------------------------------------------
// Periodic boundaries (Boundary Conditions section: the periodic replicas of
// the root cube, of side L, with the far replicas summed by the lattice sums
// of Nijboer and De Wette). Reading: the potential of a unit mass, all its
// replicas and a uniform neutralising background (the cosmological
// convention, no surface term), in Ewald's split with parameter a,
//   psi(r) = sum_n erfc(a|r+nL|)/|r+nL|
//          + (4 pi/L^3) sum_{k != 0} exp(-k^2/(4a^2))/k^2 cos(k.r) - pi/(a^2 L^3),
// k = 2 pi m / L; psi does not depend on a. The replicas with max|n_d| <= 2
// (the cube and its 124 neighbours) form the near zone, summed pair by pair
// with the softened kernel like the isolated force; the remainder
//   F(r) = psi(r) - sum_{max|n_d|<=2} 1/|r+nL|
// is smooth inside the cube and enters unsoftened:
//   a_i = sum_j m_j [ sum_near (x_j + nL - x_i)(|x_j + nL - x_i|^2 + eps^2)^(-3/2)
//                     + grad F(x_i - x_j) ]   (the (i, n = 0) self pair skipped).
// The treecode expands F about the cube centre c (u = x_i - c, v = x_j - c):
//   sum_j m_j F(u - v_j) = sum_beta u^beta/beta! L_beta,
//   L_beta = sum_{|alpha| <= p} (-1)^|alpha|/alpha! M_alpha(root) T_{alpha+beta},
//   T_gamma = d^gamma F(0), a_k(far) = sum_{|beta| <= p} u^beta/beta! L_{beta+e_k}.
// ---------------------------------------------------------------------------
constexpr int kWs = 2;               // near zone: max|n_d| <= kWs
constexpr int kImages = 125;         // (2 kWs + 1)^3
constexpr double kSplit = 2.0;       // a = kSplit / L
constexpr double kSqrtPi = 1.7724538509055160273;

void image_shift(int img, double L, double sh[3]) {
  sh[0] = (double)(img / 25 - kWs) * L;
  sh[1] = (double)((img / 5) % 5 - kWs) * L;
  sh[2] = (double)(img % 5 - kWs) * L;
}

// 2^n f^(n)(s) for f(s) = erfc(a sqrt s)/sqrt s at s = r^2 > 0: with
// B_0 = erfc(a r)/r, B_n = ((2n-1) B_{n-1} + (2a^2)^n exp(-a^2 r^2)/(a sqrt pi))/r^2,
// the n-th value is (-1)^n B_n.
void erfc_radial(double r, double a, int nmax, double* F) {
  const double e = std::exp(-a * a * r * r) / (a * kSqrtPi);
  double B = std::erfc(a * r) / r, p2 = 1.0;
  F[0] = B;
  for (int n = 1; n <= nmax; ++n) {
    p2 *= 2.0 * a * a;
    B = ((double)(2 * n - 1) * B + p2 * e) / (r * r);
    F[n] = (n % 2) ? -B : B;
  }
}

// the same for f(s) = erf(a sqrt s)/sqrt s = s^(-1/2) - erfc(...): at r > 0
// the difference of the two families; at r = 0 from the Taylor series
// f(s) = (2a/sqrt pi) sum_k (-a^2 s)^k / (k! (2k+1)).
void erf_radial(double r, double a, int nmax, double* F) {
  if (r == 0.0) {
    double c = 2.0 * a / kSqrtPi;
    for (int n = 0; n <= nmax; ++n) {
      F[n] = c / (double)(2 * n + 1);
      c *= -2.0 * a * a;
    }
    return;
  }
  erfc_radial(r, a, nmax, F);
  double v = 1.0 / r, df = 1.0;
  for (int n = 0; n <= nmax; ++n) {
    const double inv = ((n % 2) ? -df : df) * v;  // 2^n d^n/ds^n s^(-1/2)
    F[n] = inv - F[n];
    df *= (double)(2 * n + 1);
    v /= r * r;
  }
}

// slot of a multi-index of any order (the same order as multi_upto)
size_t slot_of(const std::array<int, 3>& m) {
  const int n = m[0] + m[1] + m[2];
  const int bc = m[1] + m[2];
  return (size_t)(n * (n + 1) * (n + 2) / 6 + bc * (bc + 1) / 2 + m[2]);
}

// multi-indices of total order <= K in slot order (order, then a, b descending)
std::vector<std::array<int, 3>> multi_upto(int K) {
  std::vector<std::array<int, 3>> out;
  for (int n = 0; n <= K; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) out.push_back({a, b, n - a - b});
  return out;
}

// T_gamma = d^gamma F(0) for |gamma| <= K:
//   - sum_{near n} d^gamma [erf(a rho)/rho](nL)
//   + sum_{far n, max|n_d| <= 6} d^gamma [erfc(a rho)/rho](nL)
//   + (4 pi/L^3) sum_{k != 0, max|m_d| <= 10} exp(-k^2/4a^2)/k^2 Re(i^|gamma|) k^gamma.
std::vector<double> lattice_tensor(double L, int K, double split) {
  const double a = split / L;
  const auto mi = multi_upto(K);
  std::vector<double> T(mi.size(), 0.0);
  Radial rad;
  for (int nx = -6; nx <= 6; ++nx)
    for (int ny = -6; ny <= 6; ++ny)
      for (int nz = -6; nz <= 6; ++nz) {
        const int m = std::max(std::abs(nx), std::max(std::abs(ny), std::abs(nz)));
        const double R[3] = {nx * L, ny * L, nz * L};
        const double r = std::sqrt((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]);
        double sign;
        if (m <= kWs) {
          erf_radial(r, a, K, rad.F);
          sign = -1.0;
        } else {
          erfc_radial(r, a, K, rad.F);
          sign = 1.0;
        }
        for (size_t g = 0; g < mi.size(); ++g)
          T[g] += sign * dG(mi[g][0], mi[g][1], mi[g][2], R, rad);
      }
  const double twopi = 2.0 * M_PI / L;
  for (int mx = -10; mx <= 10; ++mx)
    for (int my = -10; my <= 10; ++my)
      for (int mz = -10; mz <= 10; ++mz) {
        if (!mx && !my && !mz) continue;
        const double k[3] = {twopi * mx, twopi * my, twopi * mz};
        const double k2 = (k[0] * k[0] + k[1] * k[1]) + k[2] * k[2];
        const double w = 4.0 * M_PI / (L * L * L) * std::exp(-k2 / (4.0 * a * a)) / k2;
        for (size_t g = 0; g < mi.size(); ++g) {
          const int n = mi[g][0] + mi[g][1] + mi[g][2];
          if (n % 2) continue;
          const double sg = (n / 2) % 2 ? -1.0 : 1.0;
          T[g] += w * sg * ipow(k[0], mi[g][0]) * ipow(k[1], mi[g][1]) * ipow(k[2], mi[g][2]);
        }
      }
  // the neutralising background's constant of Ewald's split (the k = 0
  // term), which makes F, and T_0, independent of the split; it enters
  // potentials only
  T[0] -= M_PI / (a * a * L * L * L);
  // F is even in each coordinate (the cubic lattice is symmetric under each
  // reflection x_d -> -x_d): every T_gamma with an odd component vanishes
  // exactly; the sums above leave only rounding there
  for (size_t g = 0; g < mi.size(); ++g)
    if ((mi[g][0] | mi[g][1] | mi[g][2]) & 1) T[g] = 0.0;
  return T;
}

// psi(r) - 1/r at r -> 0 (the lattice's self potential; Madelung-type constant)
double ewald_self(double L, double split) {
  const double a = split / L;
  double s = -2.0 * a / kSqrtPi - M_PI / (a * a * L * L * L);
  for (int nx = -6; nx <= 6; ++nx)
    for (int ny = -6; ny <= 6; ++ny)
      for (int nz = -6; nz <= 6; ++nz) {
        if (!nx && !ny && !nz) continue;
        const double r = L * std::sqrt((double)(nx * nx + ny * ny + nz * nz));
        s += std::erfc(a * r) / r;
      }
  const double twopi = 2.0 * M_PI / L;
  for (int mx = -10; mx <= 10; ++mx)
    for (int my = -10; my <= 10; ++my)
      for (int mz = -10; mz <= 10; ++mz) {
        if (!mx && !my && !mz) continue;
        const double k2 = twopi * twopi * (double)(mx * mx + my * my + mz * mz);
        s += 4.0 * M_PI / (L * L * L) * std::exp(-k2 / (4.0 * a * a)) / k2;
      }
  return s;
}

// grad F(r) for r inside the doubled cube (max|r_d| < L), split a = split/L
void grad_far(const double r[3], double L, double split, double g[3]) {
  const double a = split / L;
  g[0] = g[1] = g[2] = 0.0;
  for (int nx = -4; nx <= 4; ++nx)
    for (int ny = -4; ny <= 4; ++ny)
      for (int nz = -4; nz <= 4; ++nz) {
        const int m = std::max(std::abs(nx), std::max(std::abs(ny), std::abs(nz)));
        const double p[3] = {r[0] + nx * L, r[1] + ny * L, r[2] + nz * L};
        const double rho = std::sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
        const double x = a * rho;
        double c;  // grad h = -c p
        if (m <= kWs) {
          // h = -erf(a rho)/rho: c = -a^3 q(a rho),
          // q(x) = (erf x - 2x/sqrt(pi) e^(-x^2)) / x^3
          double q;
          if (x < 0.5) {
            q = 0.0;
            double t = 1.0, f = 1.0;  // x^(2k-2), k!
            for (int k = 1; k <= 14; ++k) {
              f *= (double)k;
              q += ((k % 2) ? 1.0 : -1.0) * 2.0 * k * t / (f * (2 * k + 1));
              t *= x * x;
            }
            q *= 2.0 / kSqrtPi;
          } else {
            q = (std::erf(x) - 2.0 * x / kSqrtPi * std::exp(-x * x)) / (x * x * x);
          }
          c = -a * a * a * q;
        } else {
          // h = erfc(a rho)/rho: c = erfc(x)/rho^3 + 2a/sqrt(pi) e^(-x^2)/rho^2
          c = std::erfc(x) / (rho * rho * rho) + 2.0 * a / kSqrtPi * std::exp(-x * x) / (rho * rho);
        }
        for (int d = 0; d < 3; ++d) g[d] -= c * p[d];
      }
  const double twopi = 2.0 * M_PI / L;
  for (int mx = -5; mx <= 5; ++mx)
    for (int my = -5; my <= 5; ++my)
      for (int mz = -5; mz <= 5; ++mz) {
        if (!mx && !my && !mz) continue;
        const double k[3] = {twopi * mx, twopi * my, twopi * mz};
        const double k2 = (k[0] * k[0] + k[1] * k[1]) + k[2] * k[2];
        const double w = 4.0 * M_PI / (L * L * L) * std::exp(-k2 / (4.0 * a * a)) / k2;
        const double sn = std::sin((k[0] * r[0] + k[1] * r[1]) + k[2] * r[2]);
        for (int d = 0; d < 3; ++d) g[d] -= w * k[d] * sn;
      }
}

// F(r) = psi(r) - sum_near 1/|r + nL| itself (the potential of the far
// replicas and the background per unit mass, up to the sign), by Ewald's
// split; F(0) is finite (the n = 0 near term's singularity is removed).
double pot_far(const double r[3], double L, double split) {
  const double a = split / L;
  double f = -M_PI / (a * a * L * L * L);
  for (int nx = -4; nx <= 4; ++nx)
    for (int ny = -4; ny <= 4; ++ny)
      for (int nz = -4; nz <= 4; ++nz) {
        const int m = std::max(std::abs(nx), std::max(std::abs(ny), std::abs(nz)));
        const double p[3] = {r[0] + nx * L, r[1] + ny * L, r[2] + nz * L};
        const double rho = std::sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
        if (m <= kWs)
          f -= rho > 0.0 ? std::erf(a * rho) / rho : 2.0 * a / kSqrtPi;
        else
          f += std::erfc(a * rho) / rho;
      }
  const double twopi = 2.0 * M_PI / L;
  for (int mx = -5; mx <= 5; ++mx)
    for (int my = -5; my <= 5; ++my)
      for (int mz = -5; mz <= 5; ++mz) {
        if (!mx && !my && !mz) continue;
        const double k[3] = {twopi * mx, twopi * my, twopi * mz};
        const double k2 = (k[0] * k[0] + k[1] * k[1]) + k[2] * k[2];
        f += 4.0 * M_PI / (L * L * L) * std::exp(-k2 / (4.0 * a * a)) / k2 *
             std::cos((k[0] * r[0] + k[1] * r[1]) + k[2] * r[2]);
      }
  return f;
}

// periodic walk: the tree of image img (centres shifted), theta test as above
void walk_image(const Tree& t, const Cell& g, int64_t ci, const double sh[3], double theta,
                int direct_max, int img, std::vector<int32_t>& p2p, std::vector<int8_t>& pimg,
                std::vector<int32_t>& m2p, std::vector<int8_t>& mimg) {
  const Cell& c = t.cells[ci];
  double dx = g.centre[0] - (c.centre[0] + sh[0]);
  double dy = g.centre[1] - (c.centre[1] + sh[1]);
  double dz = g.centre[2] - (c.centre[2] + sh[2]);
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double rr = c.bmax / theta + g.bmax;
  if (d2 > rr * rr) {
    if (c.count <= direct_max) {
      p2p.push_back((int32_t)ci);
      pimg.push_back((int8_t)img);
    } else {
      m2p.push_back((int32_t)ci);
      mimg.push_back((int8_t)img);
    }
    return;
  }
  if (c.is_leaf) {
    p2p.push_back((int32_t)ci);
    pimg.push_back((int8_t)img);
    return;
  }
  for (int k = 0; k < c.n_child; ++k)
    walk_image(t, g, c.child_first + k, sh, theta, direct_max, img, p2p, pimg, m2p, mimg);
}

// periodic walk with the error-bound test (image img, centres shifted)
void walk_image_err(const Tree& t, const Cell& g, int64_t ci, const double sh[3], double tol,
                    double mmax, int pmax, int direct_max, int img, std::vector<int32_t>& p2p,
                    std::vector<int8_t>& pimg, std::vector<int32_t>& m2p,
                    std::vector<int8_t>& mimg, std::vector<int8_t>& m2p_q) {
  const Cell& c = t.cells[ci];
  double dx = g.centre[0] - (c.centre[0] + sh[0]);
  double dy = g.centre[1] - (c.centre[1] + sh[1]);
  double dz = g.centre[2] - (c.centre[2] + sh[2]);
  const int q = accept_order_d(dx, dy, dz, g, c, tol, mmax, pmax);
  if (q >= 0) {
    if (c.count <= direct_max) {
      p2p.push_back((int32_t)ci);
      pimg.push_back((int8_t)img);
    } else {
      m2p.push_back((int32_t)ci);
      mimg.push_back((int8_t)img);
      m2p_q.push_back((int8_t)q);
    }
    return;
  }
  if (c.is_leaf) {
    p2p.push_back((int32_t)ci);
    pimg.push_back((int8_t)img);
    return;
  }
  for (int k = 0; k < c.n_child; ++k)
    walk_image_err(t, g, c.child_first + k, sh, tol, mmax, pmax, direct_max, img, p2p, pimg, m2p,
                   mimg, m2p_q);
}

// ---------------------------------------------------------------------------
// Background subtraction (Background Subtraction section and its figure).
// The sources become density contrasts: from every source region the uniform
// mean density rho = M_total / L^3 is taken off, and the total taken off over
// the near zone (the 5L cube of the 125 images) is added back exactly, so
// with nothing truncated the result is that of the lists without subtraction.
// For a sink group g of side s_g its neighbourhood N(g) is the cube of side
// width * s_g about its centre (width odd; the section's figure draws 3, and
// the text asks for a region that roughly surrounds the nearby cells summed
// pair by pair, which a wider cube does when cells are pair-summed far out). Source cells inside N(g) interact as usual (matter
// only); the uniform background of N(g) is removed for all its sinks by the
// exact field of that cube. Outside N(g) every region of space interacts as
// matter minus background: an M2P cell through its moments minus those of its
// uniform cube (to the same order as the matter), a P2P cell through its
// pairs plus the exact field of its negative cube, an empty octant of an
// opened cell through the exact field of its negative cube. A cell straddling
// the border of N(g) is opened whatever the theta test says; if it is a leaf,
// or for an empty octant that straddles, the part outside N(g) is the box
// minus its intersection with N(g) (two exact box fields).
// ---------------------------------------------------------------------------

// ln(b + R) with R = sqrt(a^2 + b^2 + c^2), a^2 + c^2 > 0; for b < 0 written
// as ln((a^2 + c^2) / (R - b)) to avoid the cancellation.
double log_b_plus_r(double a, double b, double c, double R) {
  if (b >= 0.0) return std::log(b + R);
  return std::log(((a * a) + (c * c)) / (R - b));
}

// Phi(a, b, c) = a ln(b + R) + b ln(a + R) - c atan(a b / (c R)): a function
// whose mixed derivative d^2/da db is 1/R (terms that vanish with their
// factor are dropped, which is their limit).
double box_phi(double a, double b, double c) {
  const double R = std::sqrt((a * a + b * b) + c * c);
  double t = 0.0;
  if (a != 0.0) t += a * log_b_plus_r(a, b, c, R);
  if (b != 0.0) t += b * log_b_plus_r(b, a, c, R);
  if (c != 0.0) t -= c * std::atan((a * b) / (c * R));
  return t;
}

// Field at x of unit density filling the box [lo, hi] (G = 1, unsoftened):
//   a(x) = integral over the box of (y - x) / |y - x|^3 dy.
// Along z the w-integral of w / R^3 is -1/R at the end points and the u, v
// integrals of 1/R are double differences of Phi, so
//   a_z = - sum over the 8 corners of s_u s_v s_w Phi(u, v, w),
// u, v, w the corner's offsets from x and s = +1 at hi, -1 at lo; x and y
// follow by symmetry.
void box_field(const double lo[3], const double hi[3], const double x[3], double a[3]) {
  const double u[2] = {lo[0] - x[0], hi[0] - x[0]};
  const double v[2] = {lo[1] - x[1], hi[1] - x[1]};
  const double w[2] = {lo[2] - x[2], hi[2] - x[2]};
  a[0] = a[1] = a[2] = 0.0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) {
        const double s = ((i ^ j ^ k) & 1) ? 1.0 : -1.0;  // s_u s_v s_w: -1 x (-1)^(#lo)
        a[0] -= s * box_phi(v[j], w[k], u[i]);
        a[1] -= s * box_phi(u[i], w[k], v[j]);
        a[2] -= s * box_phi(u[i], v[j], w[k]);
      }
}

// ln(b + R) for the gradient of the box field, where its sum over the corners
// is finite: for b < 0 written as ln(rho2) - ln(R - b), rho2 the sum of the
// other two squares; when rho2 = 0 (the point lies on the line of a box edge)
// ln(rho2) is dropped: it cancels between the edge's two corners whenever the
// point lies beyond the edge, the only place the gradient is finite.
double log_edge(double b, double rho2, double R) {
  if (b >= 0.0) return R > 0.0 ? std::log(b + R) : 0.0;
  return rho2 > 0.0 ? std::log(rho2 / (R - b)) : -std::log(R - b);
}

// atan(num / (c R)) for the gradient; at c = 0 its one-sided limit from
// c > 0 (the gradient jumps across the plane of a face).
double atan_face(double num, double c, double R) {
  if (c != 0.0) return std::atan(num / (c * R));
  if (num == 0.0) return 0.0;
  return num > 0.0 ? M_PI / 2 : -M_PI / 2;
}

// Gradient of box_field, T[k][l] = d a_k / d x_l (symmetric). From
// a_z = - sum s Phi(u, v, w) with u, v, w = corner - x and the mixed
// derivatives of Phi: dPhi/da = ln(b + R) + (terms constant in b),
// dPhi/dc = -atan(ab / (cR)) + (terms constant in a or in b); the constant
// terms cancel in the corner sums, leaving
//   T_xx = -sum s atan(v w / (u R)),  T_xy = sum s ln(w + R),
// and the others by symmetry.
void box_grad(const double lo[3], const double hi[3], const double x[3], double T[3][3]) {
  const double u2[2] = {lo[0] - x[0], hi[0] - x[0]};
  const double v2[2] = {lo[1] - x[1], hi[1] - x[1]};
  const double w2[2] = {lo[2] - x[2], hi[2] - x[2]};
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) T[k][l] = 0.0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) {
        const double u = u2[i], v = v2[j], w = w2[k];
        const double R = std::sqrt((u * u + v * v) + w * w);
        const double s = ((i ^ j ^ k) & 1) ? 1.0 : -1.0;
        T[0][0] -= s * atan_face(v * w, u, R);
        T[1][1] -= s * atan_face(u * w, v, R);
        T[2][2] -= s * atan_face(u * v, w, R);
        T[0][1] += s * log_edge(w, u * u + v * v, R);
        T[0][2] += s * log_edge(v, u * u + w * w, R);
        T[1][2] += s * log_edge(u, v * v + w * w, R);
      }
  T[1][0] = T[0][1];
  T[2][0] = T[0][2];
  T[2][1] = T[1][2];
}

// Raw moments of unit density filling a cube of side s about its centre:
// prod_d 2 (s/2)^(alpha_d + 1) / (alpha_d + 1) for all alpha_d even, else 0.
double cube_moment(int a, int b, int c, double s) {
  if ((a & 1) || (b & 1) || (c & 1)) return 0.0;
  const int al[3] = {a, b, c};
  double m = 1.0;
  for (int d = 0; d < 3; ++d) m *= 2.0 * ipow(0.5 * s, al[d] + 1) / (double)(al[d] + 1);
  return m;
}

enum Rel { kInside = 0, kOutside = 1, kStraddle = 2 };

// Relation of the box [blo, bhi] to N = [nlo, nhi].
int box_rel(const double blo[3], const double bhi[3], const double nlo[3], const double nhi[3]) {
  bool inside = true, outside = false;
  for (int d = 0; d < 3; ++d) {
    inside = inside && blo[d] >= nlo[d] && bhi[d] <= nhi[d];
    outside = outside || bhi[d] <= nlo[d] || blo[d] >= nhi[d];
  }
  return inside ? kInside : (outside ? kOutside : kStraddle);
}

struct BgLists {
  std::vector<int8_t> msub;
  std::vector<double> boxes;
  std::vector<int8_t> sign;
  void push(const double lo[3], const double hi[3], int sg) {
    for (int d = 0; d < 3; ++d) boxes.push_back(lo[d]);
    for (int d = 0; d < 3; ++d) boxes.push_back(hi[d]);
    sign.push_back((int8_t)sg);
  }
  // negative background over [lo, hi] minus N
  void push_outside(const double lo[3], const double hi[3], int rel, const double nlo[3],
                    const double nhi[3]) {
    if (rel == kInside) return;
    push(lo, hi, -1);
    if (rel == kStraddle) {
      double ilo[3], ihi[3];
      for (int d = 0; d < 3; ++d) {
        ilo[d] = std::max(lo[d], nlo[d]);
        ihi[d] = std::min(hi[d], nhi[d]);
      }
      push(ilo, ihi, +1);
    }
  }
};

// periodic walk with background subtraction; N = [nlo, nhi] is N(g)
void walk_image_bs(const Tree& t, const Cell& g, const double nlo[3], const double nhi[3],
                   int64_t ci, const double sh[3], double theta, int direct_max, int img,
                   std::vector<int32_t>& p2p, std::vector<int8_t>& pimg,
                   std::vector<int32_t>& m2p, std::vector<int8_t>& mimg, BgLists& bl) {
  const Cell& c = t.cells[ci];
  const double cx[3] = {c.centre[0] + sh[0], c.centre[1] + sh[1], c.centre[2] + sh[2]};
  const double h = std::ldexp(t.side, -(c.level + 1));
  const double blo[3] = {cx[0] - h, cx[1] - h, cx[2] - h};
  const double bhi[3] = {cx[0] + h, cx[1] + h, cx[2] + h};
  const int rel = box_rel(blo, bhi, nlo, nhi);
  double dx = g.centre[0] - cx[0];
  double dy = g.centre[1] - cx[1];
  double dz = g.centre[2] - cx[2];
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double rr = c.bmax / theta + g.bmax;
  if (rel != kStraddle && d2 > rr * rr) {
    if (c.count <= direct_max) {
      p2p.push_back((int32_t)ci);
      pimg.push_back((int8_t)img);
      bl.push_outside(blo, bhi, rel, nlo, nhi);
    } else {
      m2p.push_back((int32_t)ci);
      mimg.push_back((int8_t)img);
      bl.msub.push_back((int8_t)(rel == kOutside));
    }
    return;
  }
  if (c.is_leaf) {
    p2p.push_back((int32_t)ci);
    pimg.push_back((int8_t)img);
    bl.push_outside(blo, bhi, rel, nlo, nhi);
    return;
  }
  // opened: its empty octants first (octant o = 4 x + 2 y + z, key order),
  // then its children
  if (rel != kInside) {
    bool has[8] = {false, false, false, false, false, false, false, false};
    for (int k = 0; k < c.n_child; ++k) has[t.cells[c.child_first + k].key & 7u] = true;
    for (int o = 0; o < 8; ++o) {
      if (has[o]) continue;
      const int bit[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
      double olo[3], ohi[3];
      for (int d = 0; d < 3; ++d) {
        olo[d] = bit[d] ? cx[d] : blo[d];
        ohi[d] = bit[d] ? bhi[d] : cx[d];
      }
      bl.push_outside(olo, ohi, box_rel(olo, ohi, nlo, nhi), nlo, nhi);
    }
  }
  for (int k = 0; k < c.n_child; ++k)
    walk_image_bs(t, g, nlo, nhi, c.child_first + k, sh, theta, direct_max, img, p2p, pimg, m2p,
                  mimg, bl);
}

// N(g): the cube of side width * s_g about the group's centre
void neighbourhood(const Tree& t, const Cell& g, int width, double nlo[3], double nhi[3]) {
  const double h3 = (double)width * std::ldexp(t.side, -(g.level + 1));
  for (int d = 0; d < 3; ++d) {
    nlo[d] = g.centre[d] - h3;
    nhi[d] = g.centre[d] + h3;
  }
}

}  // namespace

// ===========================================================================
// C ABI (host pointers only)
// ===========================================================================
extern "C" {

const char* oracle_last_error(void) { return g_err.c_str(); }

int oracle_nm(int p) { return nm(p); }

// Keys in caller order plus the root cube (lo[3], side) actually used.
int oracle_morton_keys(int64_t n, const double* pos, const double* box, double* lo_side,
                       uint64_t* keys) {
  if (n < 1 || !pos || !keys) return fail("bad arguments");
  double lo[3], side;
  if (box) {
    lo[0] = box[0], lo[1] = box[1], lo[2] = box[2], side = box[3];
    if (!is_pow2(side)) return fail("box side must be a positive power of two");
  } else {
    root_cube(n, pos, lo, &side);
  }
  int e;
  std::frexp(side, &e);
  double scale = std::ldexp(1.0, kBits - (e - 1));
  for (int64_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) q[d] = quantise(pos[3 * i + d], lo[d], scale);
    keys[i] = (1ull << 63) | interleave(q[0], q[1], q[2]);
  }
  if (lo_side) {
    lo_side[0] = lo[0], lo_side[1] = lo[1], lo_side[2] = lo[2], lo_side[3] = side;
  }
  return 0;
}

int oracle_tree_build(int64_t n, const double* pos, int n_leaf, int n_group, const double* box,
                      void** out) {
  ensure_alpha();
  if (n < 1 || !pos || !out) return fail("bad arguments");
  if (n_leaf < 1 || n_group < n_leaf) return fail("need 1 <= n_leaf <= n_group");
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(pos[i])) return fail("non-finite position");
  if (box) {
    if (!is_pow2(box[3])) return fail("box side must be a positive power of two");
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d)
        if (pos[3 * i + d] < box[d] || pos[3 * i + d] > box[d] + box[3])
          return fail("point outside the given box");
  }
  Tree* t = new Tree();
  t->n_leaf = n_leaf;
  t->n_group = n_group;
  int rc = build_tree(*t, n, pos, box);
  if (rc) {
    delete t;
    return rc;
  }
  *out = t;
  return 0;
}

void oracle_tree_destroy(void* h) { delete (Tree*)h; }

// counts: n, n_cells, n_groups, n_leaves, max_level, n_p2p_entries,
// n_m2p_entries, lo[3] and side as bits are not included (see get_root).
int oracle_tree_counts(void* h, int64_t* out) {
  Tree* t = (Tree*)h;
  int64_t leaves = 0;
  for (auto& c : t->cells) leaves += c.is_leaf;
  out[0] = t->n;
  out[1] = (int64_t)t->cells.size();
  out[2] = (int64_t)t->groups.size();
  out[3] = leaves;
  out[4] = t->max_level;
  out[5] = t->has_lists ? (int64_t)t->p2p.size() : -1;
  out[6] = t->has_lists ? (int64_t)t->m2p.size() : -1;
  return 0;
}

int oracle_tree_root(void* h, double* lo_side) {
  Tree* t = (Tree*)h;
  lo_side[0] = t->lo[0], lo_side[1] = t->lo[1], lo_side[2] = t->lo[2], lo_side[3] = t->side;
  return 0;
}

int oracle_tree_get_keys(void* h, uint64_t* keys, int64_t* perm) {
  Tree* t = (Tree*)h;
  if (keys) std::copy(t->key.begin(), t->key.end(), keys);
  if (perm) std::copy(t->perm.begin(), t->perm.end(), perm);
  return 0;
}

int oracle_tree_get_cells(void* h, int32_t* level, uint64_t* key, int64_t* first, int64_t* count,
                          int64_t* parent, int64_t* child_first, int32_t* n_child,
                          int32_t* is_leaf, double* centre, double* bmax) {
  Tree* t = (Tree*)h;
  for (size_t i = 0; i < t->cells.size(); ++i) {
    const Cell& c = t->cells[i];
    if (level) level[i] = c.level;
    if (key) key[i] = c.key;
    if (first) first[i] = c.first;
    if (count) count[i] = c.count;
    if (parent) parent[i] = c.parent;
    if (child_first) child_first[i] = c.child_first;
    if (n_child) n_child[i] = c.n_child;
    if (is_leaf) is_leaf[i] = c.is_leaf;
    if (centre)
      for (int d = 0; d < 3; ++d) centre[3 * i + d] = c.centre[d];
    if (bmax) bmax[i] = c.bmax;
  }
  return 0;
}

int oracle_tree_get_groups(void* h, int64_t* groups) {
  Tree* t = (Tree*)h;
  std::copy(t->groups.begin(), t->groups.end(), groups);
  return 0;
}

// Lists of every group, or only of the selected group ordinals (the others
// stay empty; evaluating a sink of an unselected group is then an error).
int oracle_build_lists(void* h, double theta, int direct_max, int64_t n_sel, const int64_t* sel) {
  Tree* t = (Tree*)h;
  if (!(theta > 0 && theta < 1)) return fail("theta must lie in (0, 1)");
  if (direct_max < 0) return fail("direct_max must be >= 0");
  std::vector<char> want;
  if (sel) {
    want.assign(t->groups.size(), 0);
    for (int64_t k = 0; k < n_sel; ++k) {
      if (sel[k] < 0 || sel[k] >= (int64_t)t->groups.size()) return fail("bad group ordinal");
      want[sel[k]] = 1;
    }
  }
  t->list_sel = want;
  return build_lists(*t, theta, direct_max, want);
}

// Error-bound lists (see accept_order) with orders up to pmax; mass in
// caller order (only its largest value is used).
int oracle_build_lists_err(void* h, const double* mass, double tol, int pmax, int direct_max,
                           int64_t n_sel, const int64_t* sel) {
  Tree* t = (Tree*)h;
  if (!mass) return fail("bad arguments");
  if (!(tol > 0) || !std::isfinite(tol)) return fail("tol must be finite and > 0");
  if (pmax < 0 || pmax > 8) return fail("pmax must lie in [0, 8]");
  if (direct_max < 0) return fail("direct_max must be >= 0");
  double mmax = 0.0;
  for (int64_t i = 0; i < t->n; ++i) mmax = std::max(mmax, mass[i]);
  std::vector<char> want;
  if (sel) {
    want.assign(t->groups.size(), 0);
    for (int64_t k = 0; k < n_sel; ++k) {
      if (sel[k] < 0 || sel[k] >= (int64_t)t->groups.size()) return fail("bad group ordinal");
      want[sel[k]] = 1;
    }
  }
  t->list_sel = want;
  return build_lists(*t, -1.0, direct_max, want, tol, mmax, pmax);
}

// Periodic lists: the walk above for each of the 125 images of the source
// tree (the cube and its neighbours, image = 25 (n_x + 2) + 5 (n_y + 2) +
// (n_z + 2)), images in that order, each a depth-first walk; the root cube is
// the periodic cell. The tree must have been built with a given box.
int build_lists_periodic(Tree* t, double theta, int direct_max, int64_t n_sel,
                         const int64_t* sel, bool bs, int width, double tol = 0.0,
                         double mmax = 0.0, int pmax = -1);

int oracle_build_lists_periodic(void* h, double theta, int direct_max, int64_t n_sel,
                                const int64_t* sel) {
  return build_lists_periodic((Tree*)h, theta, direct_max, n_sel, sel, false, 3);
}

// Periodic lists with background subtraction (see walk_image_bs); N(g) of
// side width (odd, 3 .. 9) group sides.
int oracle_build_lists_periodic_bs(void* h, double theta, int direct_max, int width,
                                   int64_t n_sel, const int64_t* sel) {
  if (width < 3 || width > 9 || !(width & 1)) return fail("width must be odd, in [3, 9]");
  return build_lists_periodic((Tree*)h, theta, direct_max, n_sel, sel, true, width);
}

// Periodic lists with the error-bound test of accept_order (orders up to
// pmax per entry); mass in caller order (only its largest value is used).
int oracle_build_lists_periodic_err(void* h, const double* mass, double tol, int pmax,
                                    int direct_max, int64_t n_sel, const int64_t* sel) {
  Tree* t = (Tree*)h;
  if (!mass) return fail("bad arguments");
  if (!(tol > 0) || !std::isfinite(tol)) return fail("tol must be finite and > 0");
  if (pmax < 0 || pmax > 8) return fail("pmax must lie in [0, 8]");
  double mmax = 0.0;
  for (int64_t i = 0; i < t->n; ++i) mmax = std::max(mmax, mass[i]);
  return build_lists_periodic(t, -1.0, direct_max, n_sel, sel, false, 3, tol, mmax, pmax);
}

int build_lists_periodic(Tree* t, double theta, int direct_max, int64_t n_sel,
                         const int64_t* sel, bool bs, int width, double tol, double mmax,
                         int pmax) {
  const bool err = theta < 0;
  if (!err && !(theta > 0 && theta < 1)) return fail("theta must lie in (0, 1)");
  if (direct_max < 0) return fail("direct_max must be >= 0");
  std::vector<char> want;
  if (sel) {
    want.assign(t->groups.size(), 0);
    for (int64_t k = 0; k < n_sel; ++k) {
      if (sel[k] < 0 || sel[k] >= (int64_t)t->groups.size()) return fail("bad group ordinal");
      want[sel[k]] = 1;
    }
  }
  const int64_t G = (int64_t)t->groups.size();
  std::vector<std::vector<int32_t>> lp(G), lm(G);
  std::vector<std::vector<int8_t>> ip(G), im(G), iq(G);
  std::vector<BgLists> bl(bs ? G : 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < G; ++g) {
    if (!(want.empty() || want[g])) continue;
    const Cell& gc = t->cells[t->groups[g]];
    double nlo[3], nhi[3];
    neighbourhood(*t, gc, width, nlo, nhi);
    for (int img = 0; img < kImages; ++img) {
      double sh[3];
      image_shift(img, t->side, sh);
      if (bs)
        walk_image_bs(*t, gc, nlo, nhi, 0, sh, theta, direct_max, img, lp[g], ip[g], lm[g], im[g],
                      bl[g]);
      else if (err)
        walk_image_err(*t, gc, 0, sh, tol, mmax, pmax, direct_max, img, lp[g], ip[g], lm[g], im[g],
                       iq[g]);
      else
        walk_image(*t, gc, 0, sh, theta, direct_max, img, lp[g], ip[g], lm[g], im[g]);
    }
  }
  t->bg = bs;
  t->bg_width = width;
  t->m2p_sub.clear();
  t->box_off.clear();
  t->boxes.clear();
  t->box_sign.clear();
  if (bs) {
    t->box_off.assign(G + 1, 0);
    for (int64_t g = 0; g < G; ++g) {
      t->box_off[g + 1] = t->box_off[g] + (int64_t)bl[g].sign.size();
      t->m2p_sub.insert(t->m2p_sub.end(), bl[g].msub.begin(), bl[g].msub.end());
      t->boxes.insert(t->boxes.end(), bl[g].boxes.begin(), bl[g].boxes.end());
      t->box_sign.insert(t->box_sign.end(), bl[g].sign.begin(), bl[g].sign.end());
    }
  }
  t->p2p_off.assign(G + 1, 0);
  t->m2p_off.assign(G + 1, 0);
  for (int64_t g = 0; g < G; ++g) {
    t->p2p_off[g + 1] = t->p2p_off[g] + (int64_t)lp[g].size();
    t->m2p_off[g + 1] = t->m2p_off[g] + (int64_t)lm[g].size();
  }
  t->p2p.resize(t->p2p_off[G]);
  t->m2p.resize(t->m2p_off[G]);
  t->p2p_img.resize(t->p2p_off[G]);
  t->m2p_img.resize(t->m2p_off[G]);
  for (int64_t g = 0; g < G; ++g) {
    std::copy(lp[g].begin(), lp[g].end(), t->p2p.begin() + t->p2p_off[g]);
    std::copy(lm[g].begin(), lm[g].end(), t->m2p.begin() + t->m2p_off[g]);
    std::copy(ip[g].begin(), ip[g].end(), t->p2p_img.begin() + t->p2p_off[g]);
    std::copy(im[g].begin(), im[g].end(), t->m2p_img.begin() + t->m2p_off[g]);
  }
  t->m2p_q.clear();
  t->list_p = -1;
  if (err) {
    t->m2p_q.resize(t->m2p_off[G]);
    for (int64_t g = 0; g < G; ++g)
      std::copy(iq[g].begin(), iq[g].end(), t->m2p_q.begin() + t->m2p_off[g]);
    t->list_p = pmax;
  }
  t->list_sel = want;
  t->has_lists = true;
  t->periodic = true;
  t->theta = theta;
  t->direct_max = direct_max;
  return 0;
}

// Background-subtracted lists: box CSR offsets (G + 1), boxes (6 per box:
// lo[3], hi[3]), their signs, and the subtraction flag of every M2P entry.
int oracle_get_background(void* h, int64_t* box_off, double* boxes, int8_t* box_sign,
                          int8_t* m2p_sub) {
  Tree* t = (Tree*)h;
  if (!t->has_lists || !t->bg) return fail("no background-subtracted lists");
  if (box_off) std::copy(t->box_off.begin(), t->box_off.end(), box_off);
  if (boxes) std::copy(t->boxes.begin(), t->boxes.end(), boxes);
  if (box_sign) std::copy(t->box_sign.begin(), t->box_sign.end(), box_sign);
  if (m2p_sub) std::copy(t->m2p_sub.begin(), t->m2p_sub.end(), m2p_sub);
  return 0;
}

// Raw moments, slots 0 .. nm(p) - 1, of unit density filling a cube of side s
// about its centre (for the pins).
int oracle_cube_moments(int p, double s, double* out) {
  ensure_alpha();
  if (p < 0 || p > 12) return fail("p must lie in [0, 12]");
  for (int sl = 0; sl < nm(p); ++sl)
    out[sl] = cube_moment(g_alpha[3 * sl], g_alpha[3 * sl + 1], g_alpha[3 * sl + 2], s);
  return 0;
}

// Gradient of the field of unit density filling [lo, hi] at n points, 9 per
// point, row k = d a_k / d x (for the pins).
int oracle_box_grad(const double* lo, const double* hi, int64_t n, const double* x, double* T) {
  for (int64_t i = 0; i < n; ++i) box_grad(lo, hi, &x[3 * i], (double(*)[3]) & T[9 * i]);
  return 0;
}

// Field of unit density filling [lo, hi] at n points (for the pins).
int oracle_box_field(const double* lo, const double* hi, int64_t n, const double* x, double* a) {
  for (int64_t i = 0; i < n; ++i) box_field(lo, hi, &x[3 * i], &a[3 * i]);
  return 0;
}

int oracle_get_list_images(void* h, int8_t* p2p_img, int8_t* m2p_img) {
  Tree* t = (Tree*)h;
  if (!t->has_lists || !t->periodic) return fail("no periodic lists");
  if (p2p_img) std::copy(t->p2p_img.begin(), t->p2p_img.end(), p2p_img);
  if (m2p_img) std::copy(t->m2p_img.begin(), t->m2p_img.end(), m2p_img);
  return 0;
}

// T_gamma of the far replicas for |gamma| <= K (slot order), split a = split/L.
int oracle_lattice_tensor(double L, int K, double split, double* out) {
  if (!(L > 0) || K < 0 || K > 20 || !(split > 0)) return fail("bad arguments");
  const auto T = lattice_tensor(L, K, split);
  std::copy(T.begin(), T.end(), out);
  return 0;
}

double oracle_ewald_self(double L, double split) { return ewald_self(L, split); }

// O-D periodic: the definition above, for the selected sinks (caller
// indices; all if null), near zone softened, far part by Ewald sums.
int oracle_ewald_direct(int64_t n, const double* pos, const double* mass, double L, double eps,
                        int64_t n_sinks, const int64_t* sinks, double* acc, double* pot) {
  if (n < 1 || !pos || !mass || !acc || !(L > 0)) return fail("bad arguments");
  std::vector<int64_t> todo;
  if (sinks) {
    todo.assign(sinks, sinks + n_sinks);
  } else {
    todo.resize(n);
    for (int64_t i = 0; i < n; ++i) todo[i] = i;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < (int64_t)todo.size(); ++k) {
    const int64_t i = todo[k];
    const double* xi = &pos[3 * i];
    NSum s[3], sp;
    for (int64_t j = 0; j < n; ++j) {
      const double* xj = &pos[3 * j];
      double a[3] = {0, 0, 0}, ph = 0.0;
      for (int img = 0; img < kImages; ++img) {
        if (j == i && img == kImages / 2) continue;
        double sh[3];
        image_shift(img, L, sh);
        double r[3] = {(xj[0] + sh[0]) - xi[0], (xj[1] + sh[1]) - xi[1], (xj[2] + sh[2]) - xi[2]};
        p2p_pair(mass[j], r, Soft{kPlummer, eps}, a, pot ? &ph : nullptr);
      }
      const double r[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
      if (j != i) {
        double g[3];
        grad_far(r, L, kSplit, g);
        for (int d = 0; d < 3; ++d) a[d] += mass[j] * g[d];
      }
      // the far replicas of j (of i itself too) and the background
      if (pot) ph -= mass[j] * pot_far(r, L, kSplit);
      for (int d = 0; d < 3; ++d) s[d].add(a[d]);
      sp.add(ph);
    }
    for (int d = 0; d < 3; ++d) acc[3 * k + d] = s[d].value();
    if (pot) pot[k] = sp.value();
  }
  return 0;
}

int oracle_get_m2p_orders(void* h, int8_t* out) {
  Tree* t = (Tree*)h;
  if (!t->has_lists) return fail("no lists");
  if (t->list_p < 0) return fail("lists have no per-entry orders");
  std::copy(t->m2p_q.begin(), t->m2p_q.end(), out);
  return 0;
}

int oracle_group_of(void* h, int64_t* out) {
  Tree* t = (Tree*)h;
  std::copy(t->group_of.begin(), t->group_of.end(), out);
  return 0;
}

int oracle_get_lists(void* h, int64_t* p2p_off, int32_t* p2p, int64_t* m2p_off, int32_t* m2p) {
  Tree* t = (Tree*)h;
  if (!t->has_lists) return fail("no lists");
  if (p2p_off) std::copy(t->p2p_off.begin(), t->p2p_off.end(), p2p_off);
  if (p2p) std::copy(t->p2p.begin(), t->p2p.end(), p2p);
  if (m2p_off) std::copy(t->m2p_off.begin(), t->m2p_off.end(), m2p_off);
  if (m2p) std::copy(t->m2p.begin(), t->m2p.end(), m2p);
  return 0;
}

// Moments of the selected cells (all cells if sel is null) from the given
// positions (caller order); the tree's membership and centres stay fixed.
int oracle_compute_moments(void* h, const double* pos, const double* mass, int p, int64_t n_sel,
                           const int64_t* sel) {
  Tree* t = (Tree*)h;
  if (p < 0 || p > 10) return fail("p must lie in [0, 10]");
  const int64_t n = t->n;
  std::vector<double> spos(3 * n), sm(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) spos[3 * i + d] = pos[3 * t->perm[i] + d];
    sm[i] = mass[t->perm[i]];
  }
  const int K = nm(p);
  const int64_t C = (int64_t)t->cells.size();
  if (t->p != p || (int64_t)t->mom.size() != C * K) {
    t->mom.assign(C * K, 0.0);
    t->mom_valid.assign(C, 0);
    t->p = p;
  }
  std::vector<int64_t> todo;
  if (sel) {
    todo.assign(sel, sel + n_sel);
  } else {
    todo.resize(C);
    for (int64_t i = 0; i < C; ++i) todo[i] = i;
  }
  // Largest cells first so that the long ones start early.
  std::sort(todo.begin(), todo.end(),
            [&](int64_t a, int64_t b) { return t->cells[a].count > t->cells[b].count; });
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < (int64_t)todo.size(); ++k) {
    int64_t ci = todo[k];
    p2m_direct(spos.data(), sm.data(), t->cells[ci], p, &t->mom[ci * K]);
    t->mom_valid[ci] = 1;
  }
  return 0;
}

int oracle_get_moments(void* h, double* out) {
  Tree* t = (Tree*)h;
  std::copy(t->mom.begin(), t->mom.end(), out);
  return 0;
}

// O-T: treecode accelerations (and potentials) for the selected sinks (caller
// indices; all if null), accumulated in FP64 in list order: P2P entries first,
// then M2P entries. counts[0] = P2P pairs (including the skipped self slot),
// counts[1] = M2P pairs, over the evaluated sinks. absum (nullable): per sink
// the sum of the magnitudes of the terms that make up its acceleration (every
// pair, every expansion entry, every background box, the far replicas): the
// scale against which the rounding of a sum of those terms is measured
// (|a| much below it means cancellation). condsum (nullable): the same sum
// with each term weighted by its condition with respect to rounding its
// relative coordinates from the offsets of the mixed-precision path, whose
// positions are offsets from the centre of their sink group: a pair term by
// 1 + (|x_i - c_g(i)| + |x_j - c_g(j)|) / |r|, an expansion term by
// 1 + |x_i - c_g(i)| / |R| (the rest by 1).
int oracle_eval_tree(void* h, const double* pos, const double* mass, int kernel, double eps,
                     int64_t n_sinks, const int64_t* sinks, double* acc, double* pot,
                     int64_t* counts, double* absum, double* condsum) {
  Tree* t = (Tree*)h;
  if (!t->has_lists) return fail("lists not built");
  if (t->p < 0) return fail("moments not computed");
  if (t->p < t->list_p) return fail("moments of lower order than the lists");
  if (check_soft(kernel, eps)) return -1;
  const Soft sf{kernel, eps};
  const int64_t n = t->n;
  const int K = nm(t->p);
  std::vector<int64_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[t->perm[i]] = i;
  std::vector<int64_t> todo;
  if (sinks) {
    todo.assign(sinks, sinks + n_sinks);
  } else {
    todo.resize(n);
    for (int64_t i = 0; i < n; ++i) todo[i] = i;
  }
  const int64_t T = (int64_t)todo.size();
  // every sink's group must have lists and every M2P cell used must have moments
  for (int64_t k = 0; k < T; ++k) {
    int64_t g = t->group_of[inv[todo[k]]];
    if (!t->list_sel.empty() && !t->list_sel[g]) return fail("sink of a group without lists");
    for (int64_t e = t->m2p_off[g]; e < t->m2p_off[g + 1]; ++e)
      if (!t->mom_valid[t->m2p[e]]) return fail("moments missing for an M2P cell");
  }
  // periodic lists: local coefficients of the far replicas from the root's
  // moments, L_beta = sum_{|alpha| <= p} (-1)^|alpha|/alpha! M_alpha T_{alpha+beta}
  std::vector<std::array<int, 3>> far_mi;
  std::vector<double> far_L;
  if (t->periodic) {
    if (!t->mom_valid[0]) return fail("moments of the root are needed for periodic lists");
    const int p = t->p;
    const auto Tg = lattice_tensor(t->side, 2 * p + 1, kSplit);
    far_mi = multi_upto(p + 1);
    far_L.assign(far_mi.size(), 0.0);
    const double* M = &t->mom[0];
    for (size_t b = 0; b < far_mi.size(); ++b)
      for (int sl = 0; sl < K; ++sl) {
        const int* al = &g_alpha[3 * sl];
        const int n = al[0] + al[1] + al[2];
        const double w = ((n % 2) ? -1.0 : 1.0) / (factorial(al[0]) * factorial(al[1]) * factorial(al[2]));
        const std::array<int, 3> gsum = {al[0] + far_mi[b][0], al[1] + far_mi[b][1], al[2] + far_mi[b][2]};
        far_L[b] += w * M[sl] * Tg[slot_of(gsum)];
      }
  }
  // background subtraction: the mean density, total mass (the root's
  // monopole) over the cube's volume
  double bg_rho = 0.0;
  if (t->bg) {
    if (!t->mom_valid[0]) return fail("moments of the root are needed for the background");
    bg_rho = t->mom[0] / (t->side * t->side * t->side);
  }
  int64_t c_p2p = 0, c_m2p = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : c_p2p, c_m2p)
  for (int64_t k = 0; k < T; ++k) {
    const int64_t ci = todo[k];
    const int64_t si = inv[ci];
    const int64_t g = t->group_of[si];
    const double* xi = &pos[3 * ci];
    double a[3] = {0, 0, 0}, ph = 0.0, ab = 0.0, cs = 0.0;
    auto norm3 = [](const double* v) { return std::sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]); };
    // distance of a particle (sorted index) from its group's centre
    auto goff = [&](int64_t sj, const double* x) {
      const double* c = t->cells[t->groups[t->group_of[sj]]].centre;
      const double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
      return norm3(d);
    };
    const double oi = (absum || condsum) ? goff(si, xi) : 0.0;
    for (int64_t e = t->p2p_off[g]; e < t->p2p_off[g + 1]; ++e) {
      const Cell& c = t->cells[t->p2p[e]];
      double sh[3] = {0, 0, 0};
      const int img = t->periodic ? (int)t->p2p_img[e] : kImages / 2;
      if (t->periodic) image_shift(img, t->side, sh);
      c_p2p += c.count;
      for (int64_t j = c.first; j < c.first + c.count; ++j) {
        if (j == si && img == kImages / 2) continue;
        const double* xj = &pos[3 * t->perm[j]];
        double r[3] = {(xj[0] + sh[0]) - xi[0], (xj[1] + sh[1]) - xi[1], (xj[2] + sh[2]) - xi[2]};
        if (absum || condsum) {
          double da[3] = {0, 0, 0}, dph = 0.0;
          p2p_pair(mass[t->perm[j]], r, sf, da, &dph);
          const double m = norm3(da), rn = norm3(r);
          ab += m;
          if (m > 0.0) cs += m * (1.0 + (oi + goff(j, xj)) / rn);
        }
        p2p_pair(mass[t->perm[j]], r, sf, a, &ph);
      }
    }
    std::vector<double> msub(t->bg ? K : 0);
    for (int64_t e = t->m2p_off[g]; e < t->m2p_off[g + 1]; ++e) {
      const int64_t cid = t->m2p[e];
      const Cell& c = t->cells[cid];
      double sh[3] = {0, 0, 0};
      if (t->periodic) image_shift((int)t->m2p_img[e], t->side, sh);
      double R[3] = {xi[0] - (c.centre[0] + sh[0]), xi[1] - (c.centre[1] + sh[1]),
                     xi[2] - (c.centre[2] + sh[2])};
      double da[3], dphi;
      const int q = t->list_p >= 0 ? (int)t->m2p_q[e] : t->p;
      const double* Mc = &t->mom[cid * K];
      if (t->bg && t->m2p_sub[e]) {
        // matter minus the uniform cube of the cell, order by order up to p
        const double s = std::ldexp(t->side, -c.level);
        for (int sl = 0; sl < K; ++sl) {
          const int* al = &g_alpha[3 * sl];
          msub[sl] = Mc[sl] - bg_rho * cube_moment(al[0], al[1], al[2], s);
        }
        Mc = msub.data();
      }
      m2p_one(Mc, q, R, sf, da, &dphi);
      a[0] += da[0], a[1] += da[1], a[2] += da[2];
      ph += dphi;
      ab += norm3(da);
      cs += norm3(da) * (1.0 + oi / norm3(R));
      c_m2p += 1;
    }
    if (t->bg) {
      // background: the listed boxes, minus N(g), plus the 5L cube of the
      // near zone (exact fields, FP64)
      double f[3];
      for (int64_t b = t->box_off[g]; b < t->box_off[g + 1]; ++b) {
        box_field(&t->boxes[6 * b], &t->boxes[6 * b + 3], xi, f);
        const double sg = (double)t->box_sign[b];
        for (int d = 0; d < 3; ++d) a[d] += sg * bg_rho * f[d];
        ab += bg_rho * norm3(f);
        cs += bg_rho * norm3(f);
      }
      double nlo[3], nhi[3];
      neighbourhood(*t, t->cells[t->groups[g]], t->bg_width, nlo, nhi);
      box_field(nlo, nhi, xi, f);
      for (int d = 0; d < 3; ++d) a[d] -= bg_rho * f[d];
      ab += bg_rho * norm3(f);
      cs += bg_rho * norm3(f);
      double zlo[3], zhi[3];
      for (int d = 0; d < 3; ++d) {
        zlo[d] = t->lo[d] - (double)kWs * t->side;
        zhi[d] = t->lo[d] + (double)(kWs + 1) * t->side;
      }
      box_field(zlo, zhi, xi, f);
      for (int d = 0; d < 3; ++d) a[d] += bg_rho * f[d];
      ab += bg_rho * norm3(f);
      cs += bg_rho * norm3(f);
    }
    if (t->periodic) {
      // far replicas: a_k = sum_{|beta| <= p} u^beta/beta! L_{beta+e_k}
      const double* c0 = t->cells[0].centre;
      const double u[3] = {xi[0] - c0[0], xi[1] - c0[1], xi[2] - c0[2]};
      const double a_near[3] = {a[0], a[1], a[2]};
      for (size_t b = 0; b < far_mi.size(); ++b) {
        const auto& be = far_mi[b];
        if (be[0] + be[1] + be[2] > t->p) break;
        const double mono = ipow(u[0], be[0]) * ipow(u[1], be[1]) * ipow(u[2], be[2]) /
                            (factorial(be[0]) * factorial(be[1]) * factorial(be[2]));
        for (int d = 0; d < 3; ++d) {
          std::array<int, 3> bk = be;
          bk[d] += 1;
          a[d] += mono * far_L[slot_of(bk)];
        }
        // potential: phi = -sum_beta u^beta/beta! L_beta
        ph -= mono * far_L[slot_of(be)];
      }
      const double far[3] = {a[0] - a_near[0], a[1] - a_near[1], a[2] - a_near[2]};
      ab += norm3(far);
      cs += norm3(far);
    }
    for (int d = 0; d < 3; ++d) acc[3 * k + d] = a[d];
    if (pot) pot[k] = ph;
    if (absum) absum[k] = ab;
    if (condsum) condsum[k] = cs;
  }
  if (counts) {
    counts[0] = c_p2p;
    counts[1] = c_m2p;
  }
  return 0;
}

// O-D: exact softened direct sum for the selected sinks (caller indices; all
// if null) over all sources, j = i skipped, compensated sums.
int oracle_direct(int64_t n, const double* pos, const double* mass, int kernel, double eps,
                  int64_t n_sinks, const int64_t* sinks, double* acc, double* pot) {
  if (n < 1 || !pos || !mass || !acc) return fail("bad arguments");
  if (check_soft(kernel, eps)) return -1;
  const Soft sf{kernel, eps};
  const int64_t T = sinks ? n_sinks : n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < T; ++k) {
    const int64_t i = sinks ? sinks[k] : k;
    NSum a[3], ph;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1],
                     pos[3 * j + 2] - pos[3 * i + 2]};
      PairTerms pt;
      if (!pair_terms(sf, (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2], &pt)) continue;
      for (int d = 0; d < 3; ++d) a[d].add(mass[j] * r[d] * pt.K);
      ph.add(-mass[j] * pt.psi);
    }
    for (int d = 0; d < 3; ++d) acc[3 * k + d] = a[d].value();
    if (pot) pot[k] = ph.value();
  }
  return 0;
}

// VJP of O-D: xbar_k = sum_{j != k} H(r_kj) (m_k abar_j - m_j abar_k), with
// r_kj = x_j - x_k and H(r) = K I + B r r^T the pair Hessian (Plummer:
// K = s^(-3/2), B = -3 s^(-5/2), s = |r|^2 + eps^2);
// mbar_k = sum_{i != k} abar_i . (x_k - x_i) K.
int oracle_direct_vjp(int64_t n, const double* pos, const double* mass, int kernel, double eps,
                      const double* abar, int64_t n_rows, const int64_t* rows, double* xbar,
                      double* mbar) {
  if (n < 1 || !pos || !mass || !abar || !xbar) return fail("bad arguments");
  if (check_soft(kernel, eps)) return -1;
  const Soft sf{kernel, eps};
  const int64_t T = rows ? n_rows : n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < T; ++q) {
    const int64_t k = rows ? rows[q] : q;
    NSum xb[3], mb;
    for (int64_t j = 0; j < n; ++j) {
      if (j == k) continue;
      double r[3] = {pos[3 * j] - pos[3 * k], pos[3 * j + 1] - pos[3 * k + 1],
                     pos[3 * j + 2] - pos[3 * k + 2]};
      PairTerms pt;
      if (!pair_terms(sf, (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2], &pt)) continue;
      double v[3];
      for (int d = 0; d < 3; ++d) v[d] = mass[k] * abar[3 * j + d] - mass[j] * abar[3 * k + d];
      double rv = (r[0] * v[0] + r[1] * v[1]) + r[2] * v[2];
      for (int d = 0; d < 3; ++d) xb[d].add(v[d] * pt.K + pt.B * r[d] * rv);
      // d a_j / d m_k = (x_k - x_j) K = -r K
      double ra = (r[0] * abar[3 * j] + r[1] * abar[3 * j + 1]) + r[2] * abar[3 * j + 2];
      mb.add(-ra * pt.K);
    }
    for (int d = 0; d < 3; ++d) xbar[3 * q + d] = xb[d].value();
    if (mbar) mbar[q] = mb.value();
  }
  return 0;
}

// VJP of O-T with the topology (membership, centres, b_max, lists) held
// fixed: the gradient of sum_i abar_i . a_i with respect to every position
// (and mass). Moments are functions of the positions through their
// definition; centres do not move.
int oracle_tree_vjp(void* h, const double* pos, const double* mass, int kernel, double eps,
                    const double* abar, double* xbar, double* mbar) {
  Tree* t = (Tree*)h;
  if (check_soft(kernel, eps)) return -1;
  const Soft sf{kernel, eps};
  if (!t->has_lists) return fail("lists not built");
  if (!t->list_sel.empty()) return fail("the VJP needs the lists of every group");
  if (t->p < 0) return fail("moments not computed");
  if (t->p < t->list_p) return fail("moments of lower order than the lists");
  const int64_t n = t->n;
  const int p = t->p;
  const int K = nm(p);
  const int64_t C = (int64_t)t->cells.size();
  const int64_t G = (int64_t)t->groups.size();
  for (int64_t c = 0; c < C; ++c)
    if (!t->mom_valid[c]) return fail("all moments are needed for the VJP");
  // background subtraction: the mean density and, per group, the derivative
  // of the loss with respect to it (every mass enters through it)
  const double L3 = t->side * t->side * t->side;
  const double bg_rho = t->bg ? t->mom[0] / L3 : 0.0;
  std::vector<double> drho(G, 0.0);
  std::vector<double> xb(3 * n, 0.0), mb(n, 0.0);   // indexed by sorted position
  std::vector<double> Mbar(C * K, 0.0);
  std::vector<char> used(C, 0);
  // (1) P2P pairs and (2) M2P sink side, per group; P2P source side and M2P
  // cell cotangents are collected per group and then added in group order.
  std::vector<std::vector<double>> src_x(G), src_m(G), cellbar(G);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t g = 0; g < G; ++g) {
    const Cell& gc = t->cells[t->groups[g]];
    // P2P source contributions of this group, in list order
    int64_t nsrc = 0;
    for (int64_t e = t->p2p_off[g]; e < t->p2p_off[g + 1]; ++e) nsrc += t->cells[t->p2p[e]].count;
    src_x[g].assign(3 * nsrc, 0.0);
    src_m[g].assign(nsrc, 0.0);
    const int64_t nm2p = t->m2p_off[g + 1] - t->m2p_off[g];
    cellbar[g].assign(nm2p * K, 0.0);
    for (int64_t si = gc.first; si < gc.first + gc.count; ++si) {
      const int64_t ci = t->perm[si];
      const double* xi = &pos[3 * ci];
      const double* ab = &abar[3 * ci];
      int64_t off = 0;
      for (int64_t e = t->p2p_off[g]; e < t->p2p_off[g + 1]; ++e) {
        const Cell& c = t->cells[t->p2p[e]];
        double sh[3] = {0, 0, 0};
        const int img = t->periodic ? (int)t->p2p_img[e] : kImages / 2;
        if (t->periodic) image_shift(img, t->side, sh);
        for (int64_t j = c.first; j < c.first + c.count; ++j, ++off) {
          if (j == si && img == kImages / 2) continue;
          const int64_t cj = t->perm[j];
          double r[3] = {(pos[3 * cj] + sh[0]) - xi[0], (pos[3 * cj + 1] + sh[1]) - xi[1],
                         (pos[3 * cj + 2] + sh[2]) - xi[2]};
          PairTerms pt;
          if (!pair_terms(sf, (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2], &pt)) continue;
          double ra = (r[0] * ab[0] + r[1] * ab[1]) + r[2] * ab[2];
          double mj = mass[cj];
          double Hab[3];
          for (int d = 0; d < 3; ++d) Hab[d] = ab[d] * pt.K + pt.B * r[d] * ra;
          for (int d = 0; d < 3; ++d) {
            xb[3 * si + d] -= mj * Hab[d];         // sink moves: r = x_j - x_i
            src_x[g][3 * off + d] += mj * Hab[d];  // source moves
          }
          src_m[g][off] += ra * pt.K;              // d a_i / d m_j = r K
        }
      }
      std::vector<double> msub(t->bg ? K : 0), cube(t->bg ? K : 0);
      for (int64_t e = t->m2p_off[g]; e < t->m2p_off[g + 1]; ++e) {
        const int64_t cid = t->m2p[e];
        const Cell& c = t->cells[cid];
        const double* M = &t->mom[cid * K];
        const bool subt = t->bg && t->m2p_sub[e];
        if (subt) {
          // matter minus the cell's uniform cube (see eval)
          const double s = std::ldexp(t->side, -c.level);
          for (int sl = 0; sl < K; ++sl) {
            const int* al = &g_alpha[3 * sl];
            cube[sl] = cube_moment(al[0], al[1], al[2], s);
            msub[sl] = M[sl] - bg_rho * cube[sl];
          }
          M = msub.data();
        }
        double sh[3] = {0, 0, 0};
        if (t->periodic) image_shift((int)t->m2p_img[e], t->side, sh);
        double R[3] = {xi[0] - (c.centre[0] + sh[0]), xi[1] - (c.centre[1] + sh[1]),
                       xi[2] - (c.centre[2] + sh[2])};
        const double r2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
        const int q = t->list_p >= 0 ? (int)t->m2p_q[e] : p;
        Radial rad = radial_soft(sf, r2, q + 2);
        double* Mb = &cellbar[g][(e - t->m2p_off[g]) * K];
        for (int sl = 0; sl < nm(q); ++sl) {
          const int* al = &g_alpha[3 * sl];
          int nn = al[0] + al[1] + al[2];
          double w = ((nn % 2) ? -1.0 : 1.0) /
                     (factorial(al[0]) * factorial(al[1]) * factorial(al[2]));
          // a_k = -sum w M d^{alpha+e_k} G ;  d a_k / d x_l = -sum w M d^{alpha+e_k+e_l} G
          for (int k = 0; k < 3; ++k) {
            int b[3] = {al[0], al[1], al[2]};
            b[k] += 1;
            double d1 = dG(b[0], b[1], b[2], R, rad);
            Mb[sl] -= w * ab[k] * d1;
            // d M_sub / d rho = -cube
            if (subt) drho[g] += w * ab[k] * d1 * cube[sl];
            for (int l = 0; l < 3; ++l) {
              int bb[3] = {b[0], b[1], b[2]};
              bb[l] += 1;
              xb[3 * si + l] -= w * M[sl] * ab[k] * dG(bb[0], bb[1], bb[2], R, rad);
            }
          }
        }
      }
      if (t->bg) {
        // exact box fields: rho (sum of signed boxes - N(g) + near zone);
        // the sink moves them, the mean density scales them
        double T[3][3], f[3], Bsum[3] = {0, 0, 0}, Tsum[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        auto add = [&](const double* lo, const double* hi, double sg) {
          box_field(lo, hi, xi, f);
          box_grad(lo, hi, xi, T);
          for (int k = 0; k < 3; ++k) {
            Bsum[k] += sg * f[k];
            for (int l = 0; l < 3; ++l) Tsum[k][l] += sg * T[k][l];
          }
        };
        for (int64_t b = t->box_off[g]; b < t->box_off[g + 1]; ++b)
          add(&t->boxes[6 * b], &t->boxes[6 * b + 3], (double)t->box_sign[b]);
        double nlo[3], nhi[3], zlo[3], zhi[3];
        neighbourhood(*t, gc, t->bg_width, nlo, nhi);
        add(nlo, nhi, -1.0);
        for (int d = 0; d < 3; ++d) {
          zlo[d] = t->lo[d] - (double)kWs * t->side;
          zhi[d] = t->lo[d] + (double)(kWs + 1) * t->side;
        }
        add(zlo, zhi, 1.0);
        for (int k = 0; k < 3; ++k) {
          drho[g] += ab[k] * Bsum[k];
          for (int l = 0; l < 3; ++l) xb[3 * si + l] += bg_rho * ab[k] * Tsum[k][l];
        }
      }
    }
  }
  // add the per-group source and cell parts in group order
  for (int64_t g = 0; g < G; ++g) {
    int64_t off = 0;
    for (int64_t e = t->p2p_off[g]; e < t->p2p_off[g + 1]; ++e) {
      const Cell& c = t->cells[t->p2p[e]];
      for (int64_t j = c.first; j < c.first + c.count; ++j, ++off) {
        for (int d = 0; d < 3; ++d) xb[3 * j + d] += src_x[g][3 * off + d];
        mb[j] += src_m[g][off];
      }
    }
    for (int64_t e = t->m2p_off[g]; e < t->m2p_off[g + 1]; ++e) {
      const int64_t cid = t->m2p[e];
      used[cid] = 1;
      for (int sl = 0; sl < K; ++sl) Mbar[cid * K + sl] += cellbar[g][(e - t->m2p_off[g]) * K + sl];
    }
  }
  // periodic lists: the far replicas. a_k(i) = sum_{|beta|<=p} u_i^beta/beta!
  // L_{beta+e_k} with L_beta = sum_alpha w_alpha M_alpha(root) T_{alpha+beta}:
  //   d/dx_{i,l}: sum_k abar_ik sum_{|beta|<=p-1} u^beta/beta! L_{beta+e_k+e_l}
  //   d/dM_alpha(root): w_alpha sum_i sum_k abar_ik sum_beta u^beta/beta! T_{alpha+beta+e_k}
  if (t->periodic) {
    const auto Tg = lattice_tensor(t->side, 2 * p + 1, kSplit);
    const auto bmi = multi_upto(p + 1);
    std::vector<double> Lb(bmi.size(), 0.0);
    const double* M0 = &t->mom[0];
    for (size_t b = 0; b < bmi.size(); ++b)
      for (int sl = 0; sl < K; ++sl) {
        const int* al = &g_alpha[3 * sl];
        const int nn = al[0] + al[1] + al[2];
        const double w = ((nn % 2) ? -1.0 : 1.0) / (factorial(al[0]) * factorial(al[1]) * factorial(al[2]));
        const std::array<int, 3> gs = {al[0] + bmi[b][0], al[1] + bmi[b][1], al[2] + bmi[b][2]};
        Lb[b] += w * M0[sl] * Tg[slot_of(gs)];
      }
    const double* c0 = t->cells[0].centre;
    std::vector<double> D(multi_upto(p + 1).size(), 0.0);  // sum_i sum_k abar_ik u^beta/beta! at beta+e_k
    for (int64_t j = 0; j < n; ++j) {
      const int64_t cj = t->perm[j];
      const double u[3] = {pos[3 * cj] - c0[0], pos[3 * cj + 1] - c0[1], pos[3 * cj + 2] - c0[2]};
      const double* ab = &abar[3 * cj];
      for (size_t b = 0; b < bmi.size(); ++b) {
        const auto& be = bmi[b];
        if (be[0] + be[1] + be[2] > p) break;
        const double mono = ipow(u[0], be[0]) * ipow(u[1], be[1]) * ipow(u[2], be[2]) /
                            (factorial(be[0]) * factorial(be[1]) * factorial(be[2]));
        for (int k = 0; k < 3; ++k) {
          std::array<int, 3> bk = be;
          bk[k] += 1;
          D[slot_of(bk)] += ab[k] * mono;
          if (be[0] + be[1] + be[2] > p - 1) continue;
          for (int l = 0; l < 3; ++l) {
            std::array<int, 3> bkl = bk;
            bkl[l] += 1;
            xb[3 * j + l] += ab[k] * mono * Lb[slot_of(bkl)];
          }
        }
      }
    }
    used[0] = 1;
    for (int sl = 0; sl < K; ++sl) {
      const int* al = &g_alpha[3 * sl];
      const int nn = al[0] + al[1] + al[2];
      const double w = ((nn % 2) ? -1.0 : 1.0) / (factorial(al[0]) * factorial(al[1]) * factorial(al[2]));
      double acc = 0.0;
      for (size_t gi = 0; gi < bmi.size(); ++gi) {
        const std::array<int, 3> gs = {al[0] + bmi[gi][0], al[1] + bmi[gi][1], al[2] + bmi[gi][2]};
        acc += Tg[slot_of(gs)] * D[gi];
      }
      Mbar[sl] += w * acc;
    }
  }
  // (3) moment cotangents to particles through the moment definition:
  // d M_alpha / d x_{j,d} = m_j alpha_d (x_j - c)^(alpha - e_d),
  // d M_alpha / d m_j = (x_j - c)^alpha.
  for (int64_t cid = 0; cid < C; ++cid) {
    if (!used[cid]) continue;
    const Cell& c = t->cells[cid];
    const double* Mb = &Mbar[cid * K];
#pragma omp parallel for schedule(static)
    for (int64_t j = c.first; j < c.first + c.count; ++j) {
      const int64_t cj = t->perm[j];
      double d[3] = {pos[3 * cj] - c.centre[0], pos[3 * cj + 1] - c.centre[1],
                     pos[3 * cj + 2] - c.centre[2]};
      double gx[3] = {0, 0, 0}, gm = 0.0;
      for (int sl = 0; sl < K; ++sl) {
        const int* al = &g_alpha[3 * sl];
        gm += Mb[sl] * ipow(d[0], al[0]) * ipow(d[1], al[1]) * ipow(d[2], al[2]);
        for (int q = 0; q < 3; ++q) {
          if (al[q] == 0) continue;
          int e3[3] = {al[0], al[1], al[2]};
          e3[q] -= 1;
          gx[q] += Mb[sl] * (double)al[q] * ipow(d[0], e3[0]) * ipow(d[1], e3[1]) * ipow(d[2], e3[2]);
        }
      }
      for (int q = 0; q < 3; ++q) xb[3 * j + q] += mass[cj] * gx[q];
      mb[j] += gm;
    }
  }
  // the mean density is the total mass over L^3: every mass gets d/d rho / L^3
  if (t->bg) {
    double dr = 0.0;
    for (int64_t g = 0; g < G; ++g) dr += drho[g];
    for (int64_t j = 0; j < n; ++j) mb[j] += dr / L3;
  }
  for (int64_t j = 0; j < n; ++j) {
    const int64_t cj = t->perm[j];
    for (int d = 0; d < 3; ++d) xbar[3 * cj + d] = xb[3 * j + d];
    if (mbar) mbar[cj] = mb[j];
  }
  return 0;
}

// Single cell-body expansion (for pins): acc[0..2], acc[3] = phi.
int oracle_m2p(int p, const double* M, const double* R, int kernel, double eps, double* acc4) {
  ensure_alpha();
  if (p < 0 || p > 10) return fail("p must lie in [0, 10]");
  if (check_soft(kernel, eps)) return -1;
  m2p_one(M, p, R, Soft{kernel, eps}, acc4, &acc4[3]);
  return 0;
}

// Moments of a point set about a centre (for pins).
int oracle_p2m(int p, int64_t n, const double* pos, const double* mass, const double* centre,
               double* out) {
  ensure_alpha();
  Cell c{};
  c.first = 0;
  c.count = n;
  for (int d = 0; d < 3; ++d) c.centre[d] = centre[d];
  p2m_direct(pos, mass, c, p, out);
  return 0;
}

// All derivatives d^alpha G(R), |alpha| <= order, in storage order (for pins).
int oracle_derivs(int order, const double* R, int kernel, double eps, double* out) {
  ensure_alpha();
  if (order < 0 || order > 12) return fail("order must lie in [0, 12]");
  if (check_soft(kernel, eps)) return -1;
  Radial rad = radial_soft(Soft{kernel, eps}, (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2], order);
  for (int sl = 0; sl < nm(order); ++sl) {
    const int* al = &g_alpha[3 * sl];
    out[sl] = dG(al[0], al[1], al[2], R, rad);
  }
  return 0;
}

// Re-centring of moments (Multipole Error Bounds section: M about a shifted
// centre written as powers of the shift): given M about z, return M about
// z' = z - shift, i.e. M'_alpha = sum_{beta <= alpha} C(alpha, beta)
// shift^(alpha - beta) M_beta, shift = z - z'.
int oracle_m2m(int p, const double* M, const double* shift, double* out) {
  ensure_alpha();
  const int K = nm(p);
  for (int s = 0; s < K; ++s) {
    const int* al = &g_alpha[3 * s];
    double acc = 0.0;
    for (int b0 = 0; b0 <= al[0]; ++b0)
      for (int b1 = 0; b1 <= al[1]; ++b1)
        for (int b2 = 0; b2 <= al[2]; ++b2) {
          double binom = factorial(al[0]) / (factorial(b0) * factorial(al[0] - b0)) *
                         factorial(al[1]) / (factorial(b1) * factorial(al[1] - b1)) *
                         factorial(al[2]) / (factorial(b2) * factorial(al[2] - b2));
          acc += binom * ipow(shift[0], al[0] - b0) * ipow(shift[1], al[1] - b1) *
                 ipow(shift[2], al[2] - b2) * M[mindex(b0, b1, b2)];
        }
    out[s] = acc;
  }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads for the following parallel regions (timing on one core and on all).
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
