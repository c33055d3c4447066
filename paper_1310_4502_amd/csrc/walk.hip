// Interaction lists: one depth-first walk of the source tree per sink group
// (the source/sink cell traversal of the Tree Construction and Traversal
// section, restricted to cell-body interactions; the m x n blocking of the
// Improving instruction-level parallelism section: one list per sink cell,
// shared by all its sinks).
//
// One wavefront walks one group. The unit of work is a run of sibling cells
// (contiguous in the canonical cell order): the lanes test the run against
// the acceptance criterion at once, the cells before the first opened one are
// emitted in order with ballot compaction, the rest of the run is kept on an
// LDS stack and the opened cell's children become the next run. The output is
// therefore exactly the depth-first preorder. The kernel runs twice: once to
// count, once to fill at offsets from a scan of the counts.
//
// Two acceptance tests: the theta criterion, and an absolute-error test that
// also picks the expansion order of each accepted cell (Multipole Error
// Bounds section: the cheapest order meeting the accuracy). The error test
// bounds the field of the truncated order-q cell-body expansion of 1/r by
// the tail sum over n > q of (n + 1) b^n / d^(n + 2):
//   E_q = M / (d - b)^2 * ((q + 2) - (q + 1) t) * t^(q + 1),  t = b / d,
// with d the distance from the cell centre to the group's bounding sphere,
// b the cell's b_max and M its particle count times the largest mass.
#include "common.h"

namespace hot {
namespace {

constexpr int kB = 256;
constexpr int kWavesPerBlock = kB / 64;
constexpr int kStack = kMaxLevel + 4;

enum { CLS_NONE = 0, CLS_P2P = 1, CLS_M2P = 2, CLS_OPEN = 3 };

// Parameters of the error-bound test (unused by the theta walk).
struct ErrMac {
  double tol;
  const double* mmax;  // device scalar: the largest particle mass
  int pmax;
  int8_t* m2p_q;       // fill pass: order of every M2P entry
};

// Periodic lists: the walk runs once per near image of the source tree
// (cell centres shifted by n L, max|n_d| <= 2), images in index order
// 25 (n_x + 2) + 5 (n_y + 2) + n_z + 2.
struct Images {
  double side;
  int8_t* p2p_img;  // fill pass: image of every entry
  int8_t* m2p_img;
};

// Background subtraction on periodic lists (Background Subtraction section
// and its figure). N(g), the cube of `width` (odd, 3 in the figure) group
// sides about the group's centre, splits the sources: cells inside it interact as usual; outside it
// every region is matter minus the uniform mean density -- M2P cells through
// their moments minus their cube's (flagged per entry), P2P cells and the
// empty octants of opened cells through the exact field of their negative
// cube (listed as boxes). A cell straddling the border of N(g) is opened
// whatever the theta test says; the part of a straddling leaf or empty
// octant outside N(g) is its box (sign -1) minus its intersection with N(g)
// (sign +1). Empty octants are listed when their cell is opened, in octant
// order, before its children are walked.
struct Background {
  int width;               // side of N(g) in group sides (odd)
  const int8_t* c_level;
  const uint64_t* c_key;
  int64_t* cnt_box;        // count pass: boxes per group
  const int64_t* off_box;  // fill pass: first box of each group
  double* boxes;           // fill pass: lo[3], hi[3] per box
  int8_t* box_sign;
  int8_t* m2p_sub;         // fill pass: 1 = the entry's cell lies outside N(g)
};

enum { REL_IN = 0, REL_OUT = 1, REL_STRADDLE = 2 };

__device__ __forceinline__ int box_rel(const double lo[3], const double hi[3],
                                       const double nlo[3], const double nhi[3]) {
  bool inside = true, outside = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    inside = inside && lo[d] >= nlo[d] && hi[d] <= nhi[d];
    outside = outside || hi[d] <= nlo[d] || lo[d] >= nhi[d];
  }
  return inside ? REL_IN : (outside ? REL_OUT : REL_STRADDLE);
}

// the box pieces of a region outside or straddling N(g), from slot `at`
__device__ __forceinline__ void put_pieces(const Background& bg, int64_t at, const double lo[3],
                                           const double hi[3], int rel, const double nlo[3],
                                           const double nhi[3]) {
  double* b = bg.boxes + 6 * at;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b[d] = lo[d];
    b[3 + d] = hi[d];
  }
  bg.box_sign[at] = -1;
  if (rel == REL_STRADDLE) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      b[6 + d] = fmax(lo[d], nlo[d]);
      b[9 + d] = fmin(hi[d], nhi[d]);
    }
    bg.box_sign[at + 1] = 1;
  }
}

__device__ __forceinline__ int n_pieces(int rel) {
  return rel == REL_IN ? 0 : (rel == REL_OUT ? 1 : 2);
}

// Order accepted for cell c (-1: not acceptable). FP64, no FMA; the same
// operations in the same order as the oracle's test.
__device__ __forceinline__ int accept_order(double dx, double dy, double dz, double gb, double b,
                                            int count, double mmax, double tol, int pmax) {
  const double d = sqrt((dx * dx + dy * dy) + dz * dz) - gb;
  if (!(d > b)) return -1;
  const double t = b / d;
  const double h = d - b;
  const double A = ((double)count * mmax) / (h * h);
  double tp = t;
  for (int q = 0; q <= pmax; ++q) {
    const double E = (A * ((double)(q + 2) - (double)(q + 1) * t)) * tp;
    if (E <= tol) return q;
    tp = tp * t;
  }
  return -1;
}

template <bool FILL, bool ERR, bool PER, bool BG>
__global__ __launch_bounds__(kB) void k_walk(
    const int32_t* __restrict__ g_cell, int64_t G, const double* __restrict__ c_centre,
    const double* __restrict__ c_bmax, const int32_t* __restrict__ c_count,
    const uint8_t* __restrict__ c_leaf, const int32_t* __restrict__ c_child,
    const int32_t* __restrict__ c_nchild, double theta, ErrMac em, Images im, Background bg,
    int direct_max,
    int64_t* __restrict__ cnt_p2p, int64_t* __restrict__ cnt_m2p, int64_t* __restrict__ pairs_p2p,
    const int64_t* __restrict__ off_p2p, const int64_t* __restrict__ off_m2p,
    int32_t* __restrict__ p2p, int32_t* __restrict__ m2p, int64_t C, unsigned* __restrict__ flags) {
  __shared__ int2 stk[kWavesPerBlock][kStack];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (g >= G) return;
  const int gc = g_cell[g];
  const double gx = c_centre[3 * gc], gy = c_centre[3 * gc + 1], gz = c_centre[3 * gc + 2];
  const double gb = c_bmax[gc];
  const double mmax = ERR ? *em.mmax : 0.0;
  const uint64_t lt = lanemask_lt();
  int64_t np = 0, nmm = 0, npairs = 0, nbox = 0;
  int64_t bp = 0, bm = 0, bb = 0;
  if (FILL) {
    bp = off_p2p[g];
    bm = off_m2p[g];
    if (BG) bb = bg.off_box[g];
  }
  double nlo[3] = {0.0, 0.0, 0.0}, nhi[3] = {0.0, 0.0, 0.0};
  if (BG) {
    const double h3 = (double)bg.width * ldexp(im.side, -((int)bg.c_level[gc] + 1));
    nlo[0] = gx - h3, nlo[1] = gy - h3, nlo[2] = gz - h3;
    nhi[0] = gx + h3, nhi[1] = gy + h3, nhi[2] = gz + h3;
  }
  bool bad = false;
  for (int img = 0; img < (PER ? 125 : 1) && !bad; ++img) {
  double shx = 0.0, shy = 0.0, shz = 0.0;
  if (PER) {
    shx = (double)(img / 25 - 2) * im.side;
    shy = (double)((img / 5) % 5 - 2) * im.side;
    shz = (double)(img % 5 - 2) * im.side;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) stk[w][0] = make_int2(0, 1);
  int top = 0;
  while (top >= 0) {
    __builtin_amdgcn_wave_barrier();
    const int2 r = stk[w][top];
    const int lo = uniform_i32(r.x), hi = uniform_i32(r.y);
    if (lo < 0 || hi > C || hi - lo > 8 || lo >= hi) {  // never true for a valid tree
      if (lane == 0) atomicOr(flags, FLAG_INTERNAL);
      bad = true;
      break;
    }
    const int c = lo + lane;
    int cls = CLS_NONE;
    int cnt = 0;
    int q = -1;
    int rel = REL_IN;
    double blo[3], bhi[3];
    if (c < hi) {
      double dx, dy, dz;
      if (PER) {
        const double cx = c_centre[3 * c] + shx;
        const double cy = c_centre[3 * c + 1] + shy;
        const double cz = c_centre[3 * c + 2] + shz;
        dx = gx - cx;
        dy = gy - cy;
        dz = gz - cz;
        if (BG) {
          const double h = ldexp(im.side, -((int)bg.c_level[c] + 1));
          blo[0] = cx - h, blo[1] = cy - h, blo[2] = cz - h;
          bhi[0] = cx + h, bhi[1] = cy + h, bhi[2] = cz + h;
          rel = box_rel(blo, bhi, nlo, nhi);
        }
      } else {
        dx = gx - c_centre[3 * c];
        dy = gy - c_centre[3 * c + 1];
        dz = gz - c_centre[3 * c + 2];
      }
      cnt = c_count[c];
      bool acc;
      if (ERR) {
        q = accept_order(dx, dy, dz, gb, c_bmax[c], cnt, mmax, em.tol, em.pmax);
        acc = q >= 0;
      } else {
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const double rr = c_bmax[c] / theta + gb;
        acc = d2 > rr * rr;
      }
      if (BG && rel == REL_STRADDLE) acc = false;
      if (acc)
        cls = cnt <= direct_max ? CLS_P2P : CLS_M2P;
      else
        cls = c_leaf[c] ? CLS_P2P : CLS_OPEN;
    }
    const uint64_t om = __ballot(cls == CLS_OPEN);
    const int k = om ? (__ffsll((long long)om) - 1) : 64;
    const uint64_t before = k >= 64 ? ~0ull : ((1ull << k) - 1ull);
    const uint64_t pm = __ballot(cls == CLS_P2P) & before;
    const uint64_t mm = __ballot(cls == CLS_M2P) & before;
    // boxes of the emitted P2P cells, in lane order (one or two per cell)
    uint64_t b1 = 0, b2 = 0;
    if (BG) {
      const bool mine = (pm >> lane) & 1ull;
      b1 = __ballot(mine && rel != REL_IN);
      b2 = __ballot(mine && rel == REL_STRADDLE);
    }
    if (FILL) {
      if ((pm >> lane) & 1ull) {
        p2p[bp + np + __popcll(pm & lt)] = c;
        if (PER) im.p2p_img[bp + np + __popcll(pm & lt)] = (int8_t)img;
        if (BG && rel != REL_IN)
          put_pieces(bg, bb + nbox + __popcll(b1 & lt) + __popcll(b2 & lt), blo, bhi, rel, nlo,
                     nhi);
      }
      if ((mm >> lane) & 1ull) {
        m2p[bm + nmm + __popcll(mm & lt)] = c;
        if (ERR) em.m2p_q[bm + nmm + __popcll(mm & lt)] = (int8_t)q;
        if (PER) im.m2p_img[bm + nmm + __popcll(mm & lt)] = (int8_t)img;
        if (BG) bg.m2p_sub[bm + nmm + __popcll(mm & lt)] = (int8_t)(rel == REL_OUT);
      }
    } else {
      if ((pm >> lane) & 1ull) npairs += cnt;
    }
    np += __popcll(pm);
    nmm += __popcll(mm);
    if (BG) nbox += __popcll(b1) + __popcll(b2);
    if (om) {
      const int oc = lo + k;
      const int cf = c_child[oc], nc = c_nchild[oc];
      int nt = top;
      if (nc < 1 || nc > 8 || cf < 0 || top + 2 >= kStack) {  // never true for a valid tree
        if (lane == 0) atomicOr(flags, FLAG_INTERNAL);
        bad = true;
        break;
      }
      if (BG) {
        // the opened cell's empty octants (octant = the key's last digit,
        // 4 x + 2 y + z), one lane each
        const double ocx = c_centre[3 * oc] + shx;
        const double ocy = c_centre[3 * oc + 1] + shy;
        const double ocz = c_centre[3 * oc + 2] + shz;
        const double h = ldexp(im.side, -((int)bg.c_level[oc] + 1));
        const double plo[3] = {ocx - h, ocy - h, ocz - h};
        const double phi[3] = {ocx + h, ocy + h, ocz + h};
        const double pc[3] = {ocx, ocy, ocz};
        if (box_rel(plo, phi, nlo, nhi) != REL_IN) {
          const int oct = lane < nc ? (int)(bg.c_key[cf + lane] & 7ull) : -1;
          unsigned present = 0u;
          for (int j = 0; j < nc; ++j) present |= 1u << __shfl(oct, j);
          int orel = REL_IN;
          double olo[3], ohi[3];
          if (lane < 8 && !((present >> lane) & 1u)) {
            const int bit[3] = {(lane >> 2) & 1, (lane >> 1) & 1, lane & 1};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              olo[d] = bit[d] ? pc[d] : plo[d];
              ohi[d] = bit[d] ? phi[d] : pc[d];
            }
            orel = box_rel(olo, ohi, nlo, nhi);
          }
          const uint64_t e1 = __ballot(orel != REL_IN);
          const uint64_t e2 = __ballot(orel == REL_STRADDLE);
          if (FILL && orel != REL_IN)
            put_pieces(bg, bb + nbox + __popcll(e1 & lt) + __popcll(e2 & lt), olo, ohi, orel, nlo,
                       nhi);
          nbox += __popcll(e1) + __popcll(e2);
        }
      }
      if (oc + 1 < hi) {
        if (lane == 0) stk[w][top] = make_int2(oc + 1, hi);
        nt = top + 1;
      }
      if (lane == 0) stk[w][nt] = make_int2(cf, cf + nc);
      top = nt;
    } else {
      --top;
    }
  }
  }
  if (!FILL) {
    // sum of P2P source particles over lanes
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) npairs += __shfl_xor(npairs, off);
    if (lane == 0) {
      cnt_p2p[g] = np;
      cnt_m2p[g] = nmm;
      pairs_p2p[g] = npairs;
      if (BG) bg.cnt_box[g] = nbox;
    }
  }
}

__global__ void k_pair_weights(const int32_t* __restrict__ g_count, int64_t G,
                               int64_t* __restrict__ pp, int64_t* __restrict__ mp) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  pp[g] *= g_count[g];
  mp[g] *= g_count[g];
}

// largest particle mass (the bit patterns of non-negative doubles order as
// their values); flags non-finite or negative masses
__global__ void k_mass_max(const double* __restrict__ mass, int64_t n,
                           unsigned long long* __restrict__ out, unsigned* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (i < n) {
    m = mass[i];
    if (!(isfinite(m) && m >= 0.0)) {
      atomicOr(flags, FLAG_BAD_MASS);
      m = 0.0;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

}  // namespace

namespace {

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

// Pair segments of every group's P2P list, one wavefront per group over its
// entries 64 at a time (the pair kernels then read one record per segment
// instead of following list entry -> cell -> particle range -> source group
// -> centre for every entry): consecutive entries whose particle ranges are
// contiguous (and, periodic, in one image) form a run, and a run is cut where
// a source group ends. The lane holding the last entry of a run walks the
// run's segments (a run still open at the end of a batch is closed by lane 0
// of the next); an exclusive scan over the lanes places them in list order.
// COUNT: per-group segment counts into cnt; else the records at off[g].
template <bool COUNT>
__global__ __launch_bounds__(kB) void k_pair_segs(
    int64_t G, const int64_t* __restrict__ p2p_off, const int32_t* __restrict__ p2p,
    const int8_t* __restrict__ p2p_img, double side, const int32_t* __restrict__ c_first,
    const int32_t* __restrict__ c_count, const int32_t* __restrict__ group_of,
    const int32_t* __restrict__ g_first, const int32_t* __restrict__ g_count,
    const int32_t* __restrict__ g_cell, const double* __restrict__ c_centre,
    int64_t* __restrict__ cnt, const int64_t* __restrict__ off, PairSeg* __restrict__ seg,
    unsigned* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (g >= G) return;
  const int gc = g_cell[g];
  const double cgx = c_centre[3 * gc], cgy = c_centre[3 * gc + 1], cgz = c_centre[3 * gc + 2];
  // segments of the run [a0, a1) in image im, counted, and written from o on
  // when emit (never in the counting pass)
  auto walk = [&](int a0, int a1, int im, int64_t o, bool emit) -> int {
    double shx = 0.0, shy = 0.0, shz = 0.0;
    if (p2p_img) image_shift(im, side, shx, shy, shz);
    int m = 0;
    for (int j = a0; j < a1;) {
      const int sg = group_of[j];
      const int sgend = g_first[sg] + g_count[sg];
      const int jend = a1 < sgend ? a1 : sgend;
      if (jend <= j) {
        atomicOr(flags, FLAG_INTERNAL);
        break;
      }
      if (!COUNT && emit) {
        const int sc = g_cell[sg];
        PairSeg r;
        r.first = j;
        r.end = jend;
        r.self = (sg == g && im == kCentreImage) ? 1 : 0;
        r.pad = 0;
        if (p2p_img) {
          r.dx = (c_centre[3 * sc] + shx) - cgx;
          r.dy = (c_centre[3 * sc + 1] + shy) - cgy;
          r.dz = (c_centre[3 * sc + 2] + shz) - cgz;
        } else {
          r.dx = c_centre[3 * sc] - cgx;
          r.dy = c_centre[3 * sc + 1] - cgy;
          r.dz = c_centre[3 * sc + 2] - cgz;
        }
        seg[o + m] = r;
      }
      ++m;
      j = jend;
    }
    return m;
  };
  int64_t k = COUNT ? 0 : off[g];
  const int64_t e0 = p2p_off[g], e1 = p2p_off[g + 1];
  // carried between batches: the previous entry's end and image, and the
  // first particle of the run still open (c_end < 0 before the first entry)
  int c_end = -1, c_img = kCentreImage, c_rf = 0;
  for (int64_t b = e0; b < e1; b += 64) {
    const int64_t e = b + lane;
    const bool valid = e < e1;
    int f = 0, en = 0, im = kCentreImage;
    if (valid) {
      const int c = p2p[e];
      f = c_first[c];
      en = f + c_count[c];
      if (p2p_img) im = (int)p2p_img[e];
    }
    int pe = __shfl_up(en, 1), pim = __shfl_up(im, 1);
    if (lane == 0) {
      pe = c_end;
      pim = c_img;
    }
    const bool start = valid && (f != pe || im != pim);
    const uint64_t smask = __ballot(start);
    const uint64_t vmask = __ballot(valid);
    const bool next_start = lane < 63 && ((smask >> (lane + 1)) & 1ull);
    const bool close = valid && (next_start || e + 1 == e1);
    // the lane's run starts at the highest start lane <= lane, or was carried
    const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t below = smask & le;
    const int sl = below ? 63 - __clzll(below) : 0;
    const int rf_l = __shfl(f, sl), rim_l = __shfl(im, sl);
    const int rf = below ? rf_l : c_rf;
    const int rim = below ? rim_l : c_img;
    // lane 0 closes the carried run first when its own entry starts a new one
    const bool carried = lane == 0 && start && c_end >= 0;
    int nseg = 0;
    if (carried) nseg += walk(c_rf, c_end, c_img, 0, false);
    if (close) nseg += walk(rf, en, rim, 0, false);
    int total;
    const int64_t at = k + wave_excl_scan(nseg, lane, &total);
    if (!COUNT && nseg > 0) {
      int64_t o = at;
      if (carried) o += walk(c_rf, c_end, c_img, o, true);
      if (close) walk(rf, en, rim, o, true);
    }
    k += total;
    // carry: the last valid entry's end and image, and its run's start
    const int lv = 63 - __clzll(vmask);
    c_end = __shfl(en, lv);
    c_img = __shfl(im, lv);
    c_rf = __shfl(rf, lv);
  }
  if (COUNT && lane == 0) cnt[g] = k;
}

// The same table when no listed cell spans two source groups (every listed
// cell then holds at most n_group particles: direct_max <= n_group), entry by
// entry in parallel: a segment starts at an entry that starts a run or, inside
// a run, changes the source group; the lane of its first entry writes the
// record and the lane of its last entry (or lane 0 of the next batch, for a
// segment still open at the end of one) writes its end.
template <bool COUNT>
__global__ __launch_bounds__(kB) void k_pair_segs_flat(
    int64_t G, const int64_t* __restrict__ p2p_off, const int32_t* __restrict__ p2p,
    const int8_t* __restrict__ p2p_img, double side, const int32_t* __restrict__ c_first,
    const int32_t* __restrict__ c_count, const int32_t* __restrict__ group_of,
    const int32_t* __restrict__ g_cell, const double* __restrict__ c_centre,
    int64_t* __restrict__ cnt, const int64_t* __restrict__ off, PairSeg* __restrict__ seg) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (g >= G) return;
  const int gc = g_cell[g];
  const double cgx = c_centre[3 * gc], cgy = c_centre[3 * gc + 1], cgz = c_centre[3 * gc + 2];
  int64_t k = COUNT ? 0 : off[g];
  const int64_t e0 = p2p_off[g], e1 = p2p_off[g + 1];
  // the previous entry's end, image and source group (c_end < 0 before the first)
  int c_end = -1, c_img = kCentreImage, c_sg = -1;
  for (int64_t b = e0; b < e1; b += 64) {
    const int64_t e = b + lane;
    const bool valid = e < e1;
    int f = 0, en = 0, im = kCentreImage, sg = -1;
    if (valid) {
      const int c = p2p[e];
      f = c_first[c];
      en = f + c_count[c];
      if (p2p_img) im = (int)p2p_img[e];
      sg = group_of[f];
    }
    int pe = __shfl_up(en, 1), pim = __shfl_up(im, 1), psg = __shfl_up(sg, 1);
    if (lane == 0) {
      pe = c_end;
      pim = c_img;
      psg = c_sg;
    }
    const bool sstart = valid && (f != pe || im != pim || sg != psg);
    const uint64_t smask = __ballot(sstart);
    const uint64_t vmask = __ballot(valid);
    const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    // this entry's segment (k - 1 for one carried over from the last batch)
    const int64_t idx = k + (int64_t)__popcll(smask & le) - 1;
    const bool last = valid && ((lane < 63 && ((smask >> (lane + 1)) & 1ull)) || e + 1 == e1);
    if (!COUNT) {
      if (sstart) {
        double shx = 0.0, shy = 0.0, shz = 0.0;
        if (p2p_img) image_shift(im, side, shx, shy, shz);
        const int sc = g_cell[sg];
        PairSeg* r = seg + idx;
        r->first = f;
        r->self = (sg == g && im == kCentreImage) ? 1 : 0;
        r->pad = 0;
        if (p2p_img) {
          r->dx = (c_centre[3 * sc] + shx) - cgx;
          r->dy = (c_centre[3 * sc + 1] + shy) - cgy;
          r->dz = (c_centre[3 * sc + 2] + shz) - cgz;
        } else {
          r->dx = c_centre[3 * sc] - cgx;
          r->dy = c_centre[3 * sc + 1] - cgy;
          r->dz = c_centre[3 * sc + 2] - cgz;
        }
      }
      if (last) seg[idx].end = en;
      if (lane == 0 && sstart && c_end >= 0) seg[k - 1].end = c_end;
    }
    k += (int64_t)__popcll(smask);
    const int lv = 63 - __clzll(vmask);
    c_end = __shfl(en, lv);
    c_img = __shfl(im, lv);
    c_sg = __shfl(sg, lv);
  }
  if (COUNT && lane == 0) cnt[g] = k;
}

// The pair-segment table of the current P2P lists (count, scan, one host
// sync for the total, fill).
void build_pair_segs(hot_ctx* ctx, hot_tree* t) {
  hipStream_t st = ctx->stream;
  const int64_t G = t->n_groups;
  const int8_t* img = t->periodic ? t->p2p_img.as<int8_t>() : nullptr;
  t->pseg_off.alloc(ctx, (G + 1) * sizeof(int64_t));
  // listed cells lie inside one source group when they hold at most n_group
  // particles (leaves hold at most n_leaf <= n_group)
  const bool flat = t->direct_max <= t->n_group;
  if (flat)
    k_pair_segs_flat<true><<<grid_for(G, kWavesPerBlock), kB, 0, st>>>(
        G, t->p2p_off.as<int64_t>(), t->p2p.as<int32_t>(), img, t->side,
        t->c_first.as<int32_t>(), t->c_count.as<int32_t>(), t->group_of.as<int32_t>(),
        t->g_cell.as<int32_t>(), t->c_centre.as<double>(), t->pseg_off.as<int64_t>(), nullptr,
        nullptr);
  else
    k_pair_segs<true><<<grid_for(G, kWavesPerBlock), kB, 0, st>>>(
        G, t->p2p_off.as<int64_t>(), t->p2p.as<int32_t>(), img, t->side, t->c_first.as<int32_t>(),
        t->c_count.as<int32_t>(), t->group_of.as<int32_t>(), t->g_first.as<int32_t>(),
        t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(), t->c_centre.as<double>(),
        t->pseg_off.as<int64_t>(), nullptr, nullptr, ctx->d_flags + kFlagLocal);
  HOT_CHECK_LAUNCH();
  int64_t* so = t->pseg_off.as<int64_t>();
  scan_i64(ctx, so, so, G, so + G);
  int64_t ns = 0;
  unsigned fl = 0;
  HOT_HIP(hipMemcpyAsync(&ns, so + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(&fl, ctx->d_flags + kFlagLocal, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipStreamSynchronize(st));
  if (fl & FLAG_INTERNAL) throw Error{HOT_E_DEVICE, "pair segment consistency check failed"};
  t->n_psegs = ns;
  t->pseg.alloc(ctx, (size_t)std::max<int64_t>(1, ns) * sizeof(PairSeg));
  if (flat)
    k_pair_segs_flat<false><<<grid_for(G, kWavesPerBlock), kB, 0, st>>>(
        G, t->p2p_off.as<int64_t>(), t->p2p.as<int32_t>(), img, t->side,
        t->c_first.as<int32_t>(), t->c_count.as<int32_t>(), t->group_of.as<int32_t>(),
        t->g_cell.as<int32_t>(), t->c_centre.as<double>(), nullptr, so, t->pseg.as<PairSeg>());
  else
    k_pair_segs<false><<<grid_for(G, kWavesPerBlock), kB, 0, st>>>(
        G, t->p2p_off.as<int64_t>(), t->p2p.as<int32_t>(), img, t->side, t->c_first.as<int32_t>(),
        t->c_count.as<int32_t>(), t->group_of.as<int32_t>(), t->g_first.as<int32_t>(),
        t->g_count.as<int32_t>(), t->g_cell.as<int32_t>(), t->c_centre.as<double>(), nullptr, so,
        t->pseg.as<PairSeg>(), ctx->d_flags + kFlagLocal);
  HOT_CHECK_LAUNCH();
}

template <bool ERR, bool PER, bool BG = false>
void walk_lists(hot_ctx* ctx, hot_tree* t, double theta, ErrMac em, int direct_max,
                int width = 3) {
  Images im{t->side, nullptr, nullptr};
  Background bg{width, t->c_level.as<int8_t>(), t->c_key.as<uint64_t>(), nullptr, nullptr,
                nullptr, nullptr, nullptr};
  hipStream_t st = ctx->stream;
  const int64_t G = t->n_groups;
  t->has_lists = false;
  t->has_transpose = false;
  t->list_p = -1;
  t->periodic = false;
  t->bg = false;
  t->p2p_off.alloc(ctx, (G + 1) * sizeof(int64_t));
  if (BG) {
    t->box_off.alloc(ctx, (G + 1) * sizeof(int64_t));
    bg.cnt_box = t->box_off.as<int64_t>();
  }
  t->m2p_off.alloc(ctx, (G + 1) * sizeof(int64_t));
  DBuf pairs, mcount, totals;
  pairs.alloc(ctx, (G + 1) * sizeof(int64_t));
  mcount.alloc(ctx, (G + 1) * sizeof(int64_t));
  totals.alloc(ctx, 4 * sizeof(int64_t));
  const unsigned grid = grid_for(G, kWavesPerBlock);
  k_walk<false, ERR, PER, BG><<<grid, kB, 0, st>>>(
      t->g_cell.as<int32_t>(), G, t->c_centre.as<double>(), t->c_bmax.as<double>(),
      t->c_count.as<int32_t>(), t->c_leaf.as<uint8_t>(), t->c_child.as<int32_t>(),
      t->c_nchild.as<int32_t>(), theta, em, im, bg, direct_max, t->p2p_off.as<int64_t>(),
      t->m2p_off.as<int64_t>(), pairs.as<int64_t>(), nullptr, nullptr, nullptr, nullptr,
      t->n_cells, ctx->d_flags + kFlagLocal);
  HOT_CHECK_LAUNCH();
  // pair counts: P2P sources x sinks, M2P cells x sinks
  HOT_HIP(hipMemcpyAsync(mcount.p, t->m2p_off.p, G * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  k_pair_weights<<<grid_for(G, kB), kB, 0, st>>>(t->g_count.as<int32_t>(), G, pairs.as<int64_t>(),
                                                 mcount.as<int64_t>());
  HOT_CHECK_LAUNCH();
  int64_t* tot = totals.as<int64_t>();
  scan_i64(ctx, pairs.as<int64_t>(), pairs.as<int64_t>(), G, tot + 2);
  scan_i64(ctx, mcount.as<int64_t>(), mcount.as<int64_t>(), G, tot + 3);
  scan_i64(ctx, t->p2p_off.as<int64_t>(), t->p2p_off.as<int64_t>(), G, t->p2p_off.as<int64_t>() + G);
  scan_i64(ctx, t->m2p_off.as<int64_t>(), t->m2p_off.as<int64_t>(), G, t->m2p_off.as<int64_t>() + G);
  if (BG)
    scan_i64(ctx, t->box_off.as<int64_t>(), t->box_off.as<int64_t>(), G,
             t->box_off.as<int64_t>() + G);
  int64_t h[5] = {0, 0, 0, 0, 0};
  unsigned fw[2] = {0u, 0u};
  HOT_HIP(hipMemcpyAsync(fw, ctx->d_flags, sizeof(fw), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(&h[0], t->p2p_off.as<int64_t>() + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(&h[1], t->m2p_off.as<int64_t>() + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HOT_HIP(hipMemcpyAsync(&h[2], tot + 2, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if (BG)
    HOT_HIP(hipMemcpyAsync(&h[4], t->box_off.as<int64_t>() + G, sizeof(int64_t),
                           hipMemcpyDeviceToHost, st));
  HOT_HIP(hipStreamSynchronize(st));
  raise_deferred(ctx, fw[kFlagDeferred]);
  const unsigned flags = fw[kFlagLocal];
  if (flags & FLAG_INTERNAL) throw Error{HOT_E_DEVICE, "walk consistency check failed"};
  if (ERR && (flags & FLAG_BAD_MASS)) throw Error{HOT_E_INVALID, "non-finite or negative mass"};
  t->n_p2p = h[0];
  t->n_m2p = h[1];
  t->p2p_pairs = h[2];
  t->m2p_pairs = h[3];
  t->p2p.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_p2p) * sizeof(int32_t));
  t->m2p.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_m2p) * sizeof(int32_t));
  if (ERR) {
    t->m2p_q.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_m2p) * sizeof(int8_t));
    em.m2p_q = t->m2p_q.as<int8_t>();
  } else {
    t->m2p_q.release();
  }
  if (PER) {
    t->p2p_img.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_p2p) * sizeof(int8_t));
    t->m2p_img.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_m2p) * sizeof(int8_t));
    im.p2p_img = t->p2p_img.as<int8_t>();
    im.m2p_img = t->m2p_img.as<int8_t>();
  } else {
    t->p2p_img.release();
    t->m2p_img.release();
  }
  t->n_boxes = h[4];
  if (BG) {
    t->boxes.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_boxes) * 6 * sizeof(double));
    t->box_sign.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_boxes) * sizeof(int8_t));
    t->m2p_sub.alloc(ctx, (size_t)std::max<int64_t>(1, t->n_m2p) * sizeof(int8_t));
    bg.cnt_box = nullptr;
    bg.off_box = t->box_off.as<int64_t>();
    bg.boxes = t->boxes.as<double>();
    bg.box_sign = t->box_sign.as<int8_t>();
    bg.m2p_sub = t->m2p_sub.as<int8_t>();
  } else {
    t->box_off.release();
    t->boxes.release();
    t->box_sign.release();
    t->m2p_sub.release();
  }
  k_walk<true, ERR, PER, BG><<<grid, kB, 0, st>>>(
      t->g_cell.as<int32_t>(), G, t->c_centre.as<double>(), t->c_bmax.as<double>(),
      t->c_count.as<int32_t>(), t->c_leaf.as<uint8_t>(), t->c_child.as<int32_t>(),
      t->c_nchild.as<int32_t>(), theta, em, im, bg, direct_max, nullptr, nullptr, nullptr,
      t->p2p_off.as<int64_t>(), t->m2p_off.as<int64_t>(), t->p2p.as<int32_t>(),
      t->m2p.as<int32_t>(), t->n_cells, ctx->d_flags + kFlagDeferred);
  HOT_CHECK_LAUNCH();
  t->theta = theta;
  t->direct_max = direct_max;
  t->list_p = ERR ? em.pmax : -1;
  t->periodic = PER;
  t->bg = BG;
  t->bg_width = width;
  build_pair_segs(ctx, t);
  t->has_lists = true;
}

}  // namespace

void build_lists(hot_ctx* ctx, hot_tree* t, double theta, int direct_max) {
  zero_flag_word(ctx, kFlagLocal);
  ErrMac em{0.0, nullptr, 0, nullptr};
  walk_lists<false, false>(ctx, t, theta, em, direct_max);
}

void build_lists_periodic(hot_ctx* ctx, hot_tree* t, double theta, int direct_max) {
  zero_flag_word(ctx, kFlagLocal);
  ErrMac em{0.0, nullptr, 0, nullptr};
  lattice_tensor(ctx, t);
  walk_lists<false, true>(ctx, t, theta, em, direct_max);
}

void build_lists_periodic_bs(hot_ctx* ctx, hot_tree* t, double theta, int direct_max, int width) {
  zero_flag_word(ctx, kFlagLocal);
  ErrMac em{0.0, nullptr, 0, nullptr};
  lattice_tensor(ctx, t);
  walk_lists<false, true, true>(ctx, t, theta, em, direct_max, width);
}

namespace {
// the largest particle mass on the device, for the error-bound test
void mass_max(hot_ctx* ctx, hot_tree* t, const double* mass, DBuf& mm) {
  mm.alloc(ctx, sizeof(unsigned long long));
  k_zero_u64<<<1, 1, 0, ctx->stream>>>(mm.as<unsigned long long>());
  HOT_CHECK_LAUNCH();
  k_mass_max<<<grid_for(t->n, kB), kB, 0, ctx->stream>>>(mass, t->n, mm.as<unsigned long long>(),
                                                         ctx->d_flags + kFlagLocal);
  HOT_CHECK_LAUNCH();
}
}  // namespace

void build_lists_periodic_err(hot_ctx* ctx, hot_tree* t, const double* mass, double tol,
                              int p_max, int direct_max) {
  zero_flag_word(ctx, kFlagLocal);
  DBuf mm;
  mass_max(ctx, t, mass, mm);
  ErrMac em{tol, mm.as<double>(), p_max, nullptr};
  lattice_tensor(ctx, t);
  walk_lists<true, true>(ctx, t, 0.0, em, direct_max);
}

void build_lists_err(hot_ctx* ctx, hot_tree* t, const double* mass, double tol, int p_max,
                     int direct_max) {
  zero_flag_word(ctx, kFlagLocal);
  DBuf mm;
  mm.alloc(ctx, sizeof(unsigned long long));
  k_zero_u64<<<1, 1, 0, ctx->stream>>>(mm.as<unsigned long long>());
  HOT_CHECK_LAUNCH();
  k_mass_max<<<grid_for(t->n, kB), kB, 0, ctx->stream>>>(mass, t->n, mm.as<unsigned long long>(),
                                                         ctx->d_flags + kFlagLocal);
  HOT_CHECK_LAUNCH();
  ErrMac em{tol, mm.as<double>(), p_max, nullptr};
  walk_lists<true, false>(ctx, t, 0.0, em, direct_max);
}

}  // namespace hot
