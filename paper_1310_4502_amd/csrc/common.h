// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hot.h"

namespace hot {

constexpr int kBits = 21;          // bits per axis in a key
constexpr int kMaxLevel = 21;      // deepest cell level
constexpr int kMaxP = 8;           // highest expansion order
constexpr int kWave = 64;

__host__ __device__ constexpr int nm(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
// moment slot of (a, b, c): by order, then a descending, then b descending
__host__ __device__ constexpr int mslot(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 +
         (b + c) * (b + c + 1) / 2 + c;
}
// padded stride (floats) of one cell's FP32 expansion coefficients
__host__ __device__ constexpr int nm_pad(int p) { return (nm(p) + 3) & ~3; }

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

#define HOT_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::hot::Error{HOT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HOT_CHECK_LAUNCH() HOT_HIP(hipGetLastError())

inline void invalid(const std::string& m) { throw Error{HOT_E_INVALID, m}; }
// clear one flag word (stream-ordered)
void zero_flag_word(hot_ctx* ctx, int word);
// after a stream synchronisation: if deferred flags f were read, clear the
// device word and fail with the check they name
void raise_deferred(hot_ctx* ctx, unsigned f);
inline void state(const std::string& m) { throw Error{HOT_E_STATE, m}; }

// Body of a C entry point: runs f with the context's device current and turns
// a thrown Error (or a host allocation failure) into its status code and the
// context's message.
template <class F>
int guard(hot_ctx* ctx, F&& f);

// Device-side error flags (bits set by kernels, read by the host). Two words:
// kernels of asynchronous calls (moments, evaluation, adjoint, the fill pass
// of the walk) set the deferred word, which hot_sync and the next
// synchronising call report; synchronous calls (tree_build, the list
// builders) clear and read their own local word.
enum : int { kFlagDeferred = 0, kFlagLocal = 1 };
// a third word, set by the evaluation's offset pass when some particle's mass
// differs from the first one's (not an error: it selects the pair kernels'
// general-mass loop)
enum : int { kFlagMass = 2 };
enum : unsigned {
  FLAG_NONFINITE_POS = 1u,
  FLAG_BAD_MASS = 2u,
  FLAG_OUTSIDE_BOX = 4u,
  FLAG_HASH_FULL = 8u,
  FLAG_INTERNAL = 16u,  // a kernel's own consistency check failed
};

// The precision argument of the evaluation calls: HOT_MIXED or HOT_FP64,
// optionally ORed with HOT_K1 (the softening kernel).
inline bool valid_precision(int precision) {
  const int base = precision & ~HOT_K1;
  return base == HOT_MIXED || base == HOT_FP64;
}
inline bool fp64_mode(int precision) { return (precision & ~HOT_K1) == HOT_FP64; }
// K1 with eps = 0 is the Newtonian kernel, which the Plummer kernels give.
inline bool use_k1(int precision, double eps) { return (precision & HOT_K1) && eps > 0.0; }

}  // namespace hot

// ---------------------------------------------------------------------------
// Context and tree (opaque in the C ABI)
// ---------------------------------------------------------------------------
struct hot_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hot_allocator alloc{};
  bool user_alloc = false;
  std::string err;
  unsigned* d_flags = nullptr;     // device error flags: [kFlagDeferred], [kFlagLocal]
  hipEvent_t ev[8]{};
  // a second stream of the library's own (default priority) on which the
  // adjoint builds its transposed lists while the sink-side kernels run on
  // `stream`, and the two events that order it against `stream`; created on
  // first use
  hipStream_t aux = nullptr;
  hipEvent_t xev[2]{};
  // phase timers (hot_set_timing): start and end event of every phase, and
  // whether the phase has been recorded since timing was switched on
  bool timing = false;
  hipEvent_t tev[2 * HOT_T_COUNT]{};
  bool trec[HOT_T_COUNT]{};
  // lattice sums of the far periodic replicas (host FP64) for one cube side
  std::vector<double> lattice;
  double lattice_side = 0.0;
  void* malloc_dev(size_t bytes);
  void free_dev(void* p);
};

namespace hot {

// Phase markers: record the start or end event of a phase on the context
// stream when timing is on.
inline void tmark(hot_ctx* ctx, int phase, bool end) {
  if (!ctx->timing) return;
  HOT_HIP(hipEventRecord(ctx->tev[2 * phase + (end ? 1 : 0)], ctx->stream));
  if (end) ctx->trec[phase] = true;
}
// Scope of one phase: start marker now, end marker at scope exit (also when
// the phase throws, so that hot_get_timings never waits on an event that was
// not recorded).
struct Phase {
  hot_ctx* ctx;
  int phase;
  Phase(hot_ctx* c, int p) : ctx(c), phase(p) { tmark(ctx, phase, false); }
  ~Phase() {
    if (ctx->timing && hipEventRecord(ctx->tev[2 * phase + 1], ctx->stream) == hipSuccess)
      ctx->trec[phase] = true;
  }
  Phase(const Phase&) = delete;
  Phase& operator=(const Phase&) = delete;
};

// A device allocation owned by a tree or by a call.
struct DBuf {
  hot_ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p && ctx) ctx->free_dev(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(hot_ctx* c, size_t b) {
    if (p && bytes >= b && ctx == c) return;
    release();
    ctx = c;
    bytes = b;
    p = b ? c->malloc_dev(b) : nullptr;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
  void swap(DBuf& o) {
    std::swap(ctx, o.ctx);
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
};

}  // namespace hot

struct hot_tree {
  hot_ctx* ctx = nullptr;
  bool valid = false;
  int64_t n = 0;
  int n_leaf = 16, n_group = 64;
  double lo[3] = {0, 0, 0};
  double side = 1.0;
  // particles (sorted order)
  hot::DBuf key, perm, spos, lambda, group_of, leaf_of, item_of;
  hot::DBuf leaf_list;  // leaf cells in particle order (n_leaves of them)
  // root cube on device: lo[3], side, scale = 2^21 / side
  hot::DBuf root;
  // cells
  int64_t n_cells = 0, n_leaves = 0;
  int max_level = 0;
  std::vector<int64_t> level_off;  // host: first cell of each level, size 23
  hot::DBuf c_key, c_level, c_first, c_count, c_parent, c_child, c_nchild, c_leaf, c_centre,
      c_bmax2, c_bmax;
  // hash table key -> cell
  uint64_t hash_slots = 0;
  hot::DBuf h_keys, h_vals;
  // groups
  int64_t n_groups = 0;
  hot::DBuf g_cell, g_first, g_count;
  // moments
  int p = -1;
  hot::DBuf mom64, mom32, momw64;
  bool momw64_valid = false;
  // P2P / M2P pair counts of the current lists (host copies)
  int64_t p2p_pairs = 0, m2p_pairs = 0;
  // lists
  bool has_lists = false;
  double theta = 0;
  int direct_max = 0;
  int64_t n_p2p = 0, n_m2p = 0;
  hot::DBuf p2p_off, p2p, m2p_off, m2p;
  // error-bound lists: expansion order (int8) of every M2P entry and the
  // highest order allowed; list_p = -1 for theta lists (every entry at p)
  hot::DBuf m2p_q;
  int list_p = -1;
  // periodic lists (root cube = periodic cell, given by the caller): the
  // image 0 .. 124 of every entry, image = 25 (n_x + 2) + 5 (n_y + 2) + n_z + 2
  // for the replica shifted by n L, and the far replicas' lattice sums
  bool box_given = false;
  bool periodic = false;
  hot::DBuf p2p_img, m2p_img, lattice;
  // background subtraction (periodic lists only): per M2P entry 1 if its
  // cell's uniform cube is subtracted; per group (CSR) the boxes whose exact
  // uniform field enters with sign +1 / -1 (lo[3], hi[3] each); the
  // subtracted weighted moments built at evaluation
  bool bg = false;
  int bg_width = 3;  // side of N(g) in group sides
  int64_t n_boxes = 0;
  hot::DBuf m2p_sub, box_off, boxes, box_sign, momsub;
  // pair segments of the P2P lists (CSR per group, built with the lists):
  // consecutive entries with contiguous particle ranges (and one image) form
  // a run, cut at source-group boundaries into segments
  int64_t n_psegs = 0;
  hot::DBuf pseg_off, pseg;
  // eval work items: (group, first sink) per wave
  int64_t n_items = 0;
  hot::DBuf items;
  // items of at most 32 sinks and the others (split at tree build; -1: not yet)
  int64_t n_items_small = -1, n_items_big = 0;
  hot::DBuf items_small, items_big;
  // adjoint caches built from the lists on first use
  bool has_transpose = false;
  // P2P by source item: records sorted by (item, group); rec_off per item
  int64_t n_srec = 0;
  int srec_gbits = 1;
  hot::DBuf srec_key, srec_val, srec_off;
  // work units of the source-side pair adjoint: (item, first record, end
  // record, single-unit flag) and each item's first unit
  int64_t n_schunk = 0;
  hot::DBuf schunk, schunk_off;
  // M2P by source cell: records sorted by (cell, group), split in items of
  // at most kCellItemGroups groups; citem_rec: first record of each item
  int64_t n_mrec = 0, n_citems = 0, n_mcells = 0;
  hot::DBuf mrec_key, mrec_val, citem_rec, citem_cell, mcell_rec, mcell_item;
  // lists with per-entry orders: items hold records of one order only;
  // citem_end: one past the item's last record; qitems: item ids sorted by
  // order, qitem_off[q] .. qitem_off[q + 1] those of order q (host copy)
  hot::DBuf citem_end, qitems;
  int64_t qitem_off[hot::kMaxP + 2] = {};
  // a cell's item partials are summed in rounds of at most 64 values when it
  // has more items than that: per round, chunk offsets per cell (C + 1) and
  // the number of chunks
  int mred_levels = 0;
  int64_t mred_n[3] = {};
  hot::DBuf mred_off[3];
};

namespace hot {

// ---------------------------------------------------------------------------
// Building blocks implemented in the .hip files
// ---------------------------------------------------------------------------
// Exclusive prefix sums (in place allowed), element types u32 -> u32 and
// i64 -> i64. total (device, may be null) receives the sum.
void scan_u32(hot_ctx* ctx, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total);
void scan_i64(hot_ctx* ctx, const int64_t* in, int64_t* out, int64_t n, int64_t* total);

// Stable LSD radix sort of the first n (key, value) pairs on key bits
// [lo, bits): a caller whose pairs are already ordered by the bits below lo
// passes lo > 0 and gets the order of a sort on all `bits` bits with fewer
// passes. The passes alternate between the caller's buffers and scratch; after
// an odd number of passes the buffers are exchanged (keys and vals then own
// the former scratch) rather than copied back.
void radix_sort(hot_ctx* ctx, DBuf& keys, DBuf& vals, int64_t n, int bits, int lo = 0);

void build_tree(hot_ctx* ctx, hot_tree* t, const double* pos, const double* box);
// the work items split by sink count (at most 32, or more), at tree build
void split_items(hot_ctx* ctx, hot_tree* t);
void gather_sorted(hot_ctx* ctx, const hot_tree* t, const double* pos, const double* mass,
                   double* spos, double* smass, int check_mass);
void build_moments(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, int p);
void weighted_fp64(hot_ctx* ctx, hot_tree* t);
void build_lists(hot_ctx* ctx, hot_tree* t, double theta, int direct_max);
void build_lists_err(hot_ctx* ctx, hot_tree* t, const double* mass, double tol, int p_max,
                     int direct_max);
void build_lists_periodic(hot_ctx* ctx, hot_tree* t, double theta, int direct_max);
void build_lists_periodic_bs(hot_ctx* ctx, hot_tree* t, double theta, int direct_max, int width);
void build_lists_periodic_err(hot_ctx* ctx, hot_tree* t, const double* mass, double tol,
                              int p_max, int direct_max);
// weighted scaled moments minus those of each cell's uniform cube of the mean
// density (into t->momsub, FP32 or FP64 as asked)
void weighted_sub(hot_ctx* ctx, hot_tree* t, bool fp64);
// exact background fields of the listed boxes, minus N(g), plus the near zone
void background_boxes(hot_ctx* ctx, hot_tree* t, const double* pos, double* acc);
// their adjoint and that of the mean density (through every mass)
void background_adjoint(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass,
                        double eps, int precision, const double* abar, double* xbar, double* mbar);
// weighted scaled moments of every cell's uniform cube per unit density, negated
// (C x nm_pad(p), FP32 or FP64)
void weighted_cube(hot_ctx* ctx, hot_tree* t, bool fp64, void* out);
// field (caller order, N x 3) of the flagged M2P entries' uniform cubes per
// unit mean density, with the sign they enter the forces with
void cube_field(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
                int precision, double* out);
void lattice_tensor(hot_ctx* ctx, hot_tree* t);
// lc_mem (nullable): room for the far replicas' local coefficients
// (far_local_count(p) doubles); allocated by the call when null
void far_replicas(hot_ctx* ctx, hot_tree* t, const double* pos, double* acc, double* pot,
                  double* lc_mem = nullptr);
constexpr int far_local_count(int p) { return (p + 2) * (p + 3) * (p + 4) / 6; }
void far_replicas_mbar(hot_ctx* ctx, hot_tree* t, const double* pos, const double* abar,
                       double* mbar_root);
void far_replicas_xbar(hot_ctx* ctx, hot_tree* t, const double* pos, const double* abar,
                       double* xbar);
// Device memory of one evaluation supplied by the caller (every pointer
// nullable: the call allocates what is null): FP32 or FP64 offsets and masses
// (N x 4), the per-sink compensated sums (N x 8), the far replicas' local
// coefficients (periodic lists).
struct EvalMem {
  void* off = nullptr;
  void* state = nullptr;
  double* far_local = nullptr;
};
void forces(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
            int precision, double* acc, double* pot, hot_stats* stats,
            const EvalMem* mem = nullptr);
void adjoint(hot_ctx* ctx, hot_tree* t, const double* pos, const double* mass, double eps,
             int precision, const double* abar, double* xbar, double* mbar);
void hash_lookup(hot_ctx* ctx, const hot_tree* t, const uint64_t* keys, int32_t* out, int64_t nq);

inline unsigned grid_for(int64_t n, int block) {
  return (unsigned)((n + block - 1) / block);
}

// Row and column of entry t of a row-major array with w columns: 32-bit
// division below 2^32 entries (a few instructions), 64-bit above.
__device__ __forceinline__ void row_col(int64_t t, int w, int64_t& r, int& col) {
  if (t < (int64_t)0xffffffffll) {
    const uint32_t q = (uint32_t)t / (uint32_t)w;
    r = (int64_t)q;
    col = (int)((uint32_t)t - q * (uint32_t)w);
  } else {
    r = t / w;
    col = (int)(t - r * w);
  }
}

// base^k for base an exact power of two (cell sides and their inverses): the
// exponent scaled, the same value as k repeated multiplications
__device__ __forceinline__ double pow2_pow(double base, int k) {
  return ldexp(1.0, ilogb(base) * k);
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
constexpr int kXcdCount = 8;

// Blocks of the kernels with one block per expansion order and run of 256
// cells (P2M, M2M and its transpose): the orders of a run are consecutive
// blocks on one XCD, so the run's particles, children or parents are fetched
// from HBM once and re-read from that XCD's L2 for the other orders: block
// b = 8 (p + 1) q + 8 o + x serves order o of cell run 8 q + x.
inline unsigned order_grid(int64_t runs, int p) {
  return (unsigned)(((runs + kXcdCount - 1) / kXcdCount) * kXcdCount * (p + 1));
}
__device__ __forceinline__ void order_block(int p, int64_t& run, int& ord) {
  const int64_t b = blockIdx.x;
  const int64_t grp = kXcdCount * (p + 1);
  const int64_t rem = b % grp;
  ord = (int)(rem / kXcdCount);
  run = (b / grp) * kXcdCount + rem % kXcdCount;
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = __lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Image index of a periodic list entry -> shift of the source replica, n L
// with n_d = digit - 2 of the index in base 5 (x most significant).
__device__ __forceinline__ void image_shift(int img, double side, double& sx, double& sy,
                                           double& sz) {
  sx = (double)(img / 25 - 2) * side;
  sy = (double)((img / 5) % 5 - 2) * side;
  sz = (double)(img % 5 - 2) * side;
}
constexpr int kCentreImage = 62;  // n = (0, 0, 0)

// One pair segment: sources [first, end) of one source group, all in one
// image, for the sinks of one group; d = (source group centre + image shift)
// - sink group centre in FP64 (rounded to the kernel's type where used);
// self = 1 when the sources are the sink group itself in the central image.
struct PairSeg {
  int32_t first, end, self, pad;
  double dx, dy, dz;
};
// sources summed in plain FP32 between two compensated adds of a pair kernel
constexpr int kSumRun = 256;

__device__ __forceinline__ float hot_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double hot_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// s^(-1/2): the hardware reciprocal square root in FP32, IEEE divide and
// square root in FP64.
__device__ __forceinline__ float hot_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double hot_rsq(double x) { return 1.0 / sqrt(x); }

// 64-bit mixer for the cell hash table (splitmix64 finaliser).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}
constexpr uint64_t kEmptyKey = 0;  // cell keys always carry the placeholder bit

__device__ __forceinline__ int32_t hash_find(const uint64_t* __restrict__ hk,
                                             const int32_t* __restrict__ hv, uint64_t mask,
                                             uint64_t key) {
  uint64_t s = mix64(key) & mask;
  while (true) {
    uint64_t k = hk[s];
    if (k == key) return hv[s];
    if (k == kEmptyKey) return -1;
    s = (s + 1) & mask;
  }
}

}  // namespace hot

namespace hot {

template <class F>
int guard(hot_ctx* ctx, F&& f) {
  if (!ctx) return HOT_E_INVALID;
  try {
    HOT_HIP(hipSetDevice(ctx->device));
    f();
    return HOT_OK;
  } catch (const Error& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return HOT_E_OOM;
  } catch (...) {
    ctx->err = "unexpected exception";
    return HOT_E_DEVICE;
  }
}

inline void need_tree(hot_ctx* ctx, hot_tree* t) {
  if (!t) invalid("null tree");
  if (t->ctx != ctx) invalid("tree belongs to another context");
  if (!t->valid) state("tree is invalid (a previous call failed)");
}

}  // namespace hot
