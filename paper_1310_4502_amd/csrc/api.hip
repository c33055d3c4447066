// C ABI entry points: argument checks, context and tree lifetime, error
// reporting, host-copy getters. The computation itself lives in the other
// translation units.
#include <cmath>
#include <mutex>
#include <new>

#include "common.h"

void* hot_ctx::malloc_dev(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) return nullptr;
  if (user_alloc) {
    p = alloc.alloc(alloc.user, bytes, (void*)stream);
    if (!p) throw hot::Error{HOT_E_OOM, "allocator returned NULL"};
  } else {
    hipError_t e = hipMallocAsync(&p, bytes, stream);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw hot::Error{HOT_E_OOM, "hipMallocAsync failed for " + std::to_string(bytes) + " bytes"};
    }
  }
  return p;
}

void hot_ctx::free_dev(void* p) {
  if (!p) return;
  if (user_alloc)
    alloc.free(alloc.user, p, (void*)stream);
  else
    (void)hipFreeAsync(p, stream);
}

// ---------------------------------------------------------------------------
// Device scratch of eval_forces_noalloc, for callers that cannot allocate
// device memory. One array per GPU, held from the library's load until the
// process ends: the FP32 offsets and masses (16 B) and the compensated sums
// (32 B) of at most kNoAllocMaxN particles, then the far replicas' local
// coefficients. Host code never uses the array's name as an address: the
// device address of each GPU's copy is looked up once per device (with that
// device current) and kept in scratch_ptr.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxN = int64_t(1) << 20;
constexpr size_t kScratchOff = 0;
constexpr size_t kScratchState = (size_t)kNoAllocMaxN * 16;
constexpr size_t kScratchLocal = kScratchState + (size_t)kNoAllocMaxN * 32;
constexpr size_t kScratchBytes = kScratchLocal + 4096;
static_assert(hot::far_local_count(hot::kMaxP) * sizeof(double) <= 4096, "local coefficients");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];


namespace {

using hot::Error;
using hot::guard;
using hot::need_tree;

__global__ void k_zero_flags(unsigned* f) { *f = 0u; }
__global__ void k_zero_flag_words(unsigned* f) { f[threadIdx.x] = 0u; }

bool pow2(double s) {
  if (!(s > 0) || !std::isfinite(s)) return false;
  int e;
  return std::frexp(s, &e) == 0.5;
}

template <typename T>
void d2h(hot_ctx* ctx, void* dst, const void* src, size_t count) {
  if (!dst || count == 0) return;
  HOT_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
}

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) hot::invalid("device index beyond the library's device table");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[device]) {
    void* ptr = nullptr;
    HOT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw hot::Error{HOT_E_DEVICE, "no device address for the scratch array"};
    scratch_ptr[device] = ptr;
  }
  return scratch_ptr[device];
}

}  // namespace

namespace hot {

void zero_flag_word(hot_ctx* ctx, int word) {
  k_zero_flags<<<1, 1, 0, ctx->stream>>>(ctx->d_flags + word);
  HOT_CHECK_LAUNCH();
}

void raise_deferred(hot_ctx* ctx, unsigned f) {
  if (!f) return;
  zero_flag_word(ctx, kFlagDeferred);
  HOT_HIP(hipStreamSynchronize(ctx->stream));
  if (f & FLAG_NONFINITE_POS) invalid("non-finite position (deferred from an earlier call)");
  if (f & FLAG_BAD_MASS) invalid("non-finite or negative mass (deferred from an earlier call)");
  if (f & FLAG_OUTSIDE_BOX) invalid("point outside the box (deferred from an earlier call)");
  if (f & FLAG_INTERNAL)
    throw Error{HOT_E_DEVICE, "kernel consistency check failed (deferred from an earlier call)"};
  invalid("device error flags set (deferred from an earlier call)");
}

}  // namespace hot

extern "C" {

int hot_ctx_create(int device, void* hip_stream, const hot_allocator* allocator, hot_ctx** out) {
  if (!out) return HOT_E_INVALID;
  *out = nullptr;
  hot_ctx* c = nullptr;
  try {
    c = new hot_ctx();
  } catch (...) {
    return HOT_E_OOM;
  }
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (allocator) {
    if (!allocator->alloc || !allocator->free) {
      delete c;
      return HOT_E_INVALID;
    }
    c->alloc = *allocator;
    c->user_alloc = true;
  }
  int rc = guard(c, [&] {
    int ndev = 0;
    HOT_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) hot::invalid("no such device");
    (void)scratch_address(device);
    HOT_HIP(hipMalloc(&c->d_flags, 64));
    k_zero_flag_words<<<1, 16, 0, c->stream>>>(c->d_flags);
    HOT_CHECK_LAUNCH();
    for (auto& e : c->ev) HOT_HIP(hipEventCreate(&e));
    HOT_HIP(hipStreamSynchronize(c->stream));
  });
  if (rc != HOT_OK) {
    // keep nothing: free what was created
    for (auto& e : c->ev)
      if (e) (void)hipEventDestroy(e);
    if (c->d_flags) (void)hipFree(c->d_flags);
    delete c;
    return rc;
  }
  *out = c;
  return HOT_OK;
}

int hot_ctx_destroy(hot_ctx* ctx) {
  if (!ctx) return HOT_E_INVALID;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  for (auto& e : ctx->xev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->tev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->d_flags) (void)hipFree(ctx->d_flags);
  delete ctx;
  return HOT_OK;
}

int hot_set_timing(hot_ctx* ctx, int on) {
  return guard(ctx, [&] {
    if (on && !ctx->tev[0])
      for (auto& e : ctx->tev) HOT_HIP(hipEventCreate(&e));
    for (auto& r : ctx->trec) r = false;
    ctx->timing = on != 0;
  });
}

int hot_get_timings(hot_ctx* ctx, double* ms) {
  return guard(ctx, [&] {
    if (!ms) hot::invalid("null output");
    HOT_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < HOT_T_COUNT; ++k) {
      ms[k] = -1.0;
      if (!ctx->trec[k]) continue;
      float t = 0.f;
      HOT_HIP(hipEventElapsedTime(&t, ctx->tev[2 * k], ctx->tev[2 * k + 1]));
      ms[k] = t;
    }
  });
}

const char* hot_last_error(hot_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int hot_sync(hot_ctx* ctx) {
  return guard(ctx, [&] {
    unsigned f = 0;
    HOT_HIP(hipMemcpyAsync(&f, ctx->d_flags + hot::kFlagDeferred, sizeof(unsigned),
                           hipMemcpyDeviceToHost, ctx->stream));
    HOT_HIP(hipStreamSynchronize(ctx->stream));
    hot::raise_deferred(ctx, f);
  });
}

int tree_build(hot_ctx* ctx, int64_t n, const double* pos, const hot_build_opts* opts,
               hot_tree** out) {
  if (!ctx) return HOT_E_INVALID;
  hot_tree* t = nullptr;
  int rc = guard(ctx, [&] {
    if (!out) hot::invalid("null output");
    *out = nullptr;
    if (!pos) hot::invalid("null positions");
    if (n < 1 || n > (int64_t)INT32_MAX - 1) hot::invalid("n must lie in [1, 2^31 - 2]");
    int n_leaf = 16, n_group = 64;
    const double* box = nullptr;
    if (opts) {
      n_leaf = opts->n_leaf ? opts->n_leaf : 16;
      n_group = opts->n_group ? opts->n_group : 64;
      box = opts->box;
    }
    if (n_group < 1 || n_group > 4096) hot::invalid("n_group must lie in [1, 4096]");
    if (n_leaf < 1 || n_leaf > n_group) hot::invalid("n_leaf must lie in [1, n_group]");
    if (box) {
      for (int d = 0; d < 3; ++d)
        if (!std::isfinite(box[d])) hot::invalid("box corner must be finite");
      if (!pow2(box[3])) hot::invalid("box side must be a positive power of two");
    }
    t = new hot_tree();
    t->ctx = ctx;
    t->n = n;
    t->n_leaf = n_leaf;
    t->n_group = n_group;
    t->box_given = box != nullptr;
    hot::Phase ph(ctx, HOT_T_TREE_BUILD);
    hot::build_tree(ctx, t, pos, box);
    t->valid = true;
    *out = t;
  });
  if (rc != HOT_OK && t) {
    (void)hipStreamSynchronize(ctx->stream);
    delete t;
  }
  return rc;
}

int tree_destroy(hot_ctx* ctx, hot_tree* tree) {
  if (!ctx || !tree) return HOT_E_INVALID;
  if (tree->ctx != ctx) {
    ctx->err = "tree belongs to another context";
    return HOT_E_INVALID;
  }
  (void)hipSetDevice(ctx->device);
  delete tree;  // buffers are freed stream-ordered
  return HOT_OK;
}

int compute_moments(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass, int p) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!pos || !mass) hot::invalid("null positions or masses");
    if (p < 0 || p > hot::kMaxP) hot::invalid("p must lie in [0, 8]");
    hot::Phase ph(ctx, HOT_T_MOMENTS);
    try {
      hot::build_moments(ctx, tree, pos, mass, p);
    } catch (...) {
      tree->p = -1;
      throw;
    }
  });
}

int build_interaction_lists(hot_ctx* ctx, hot_tree* tree, double theta, int direct_max) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!(theta > 0.0 && theta < 1.0)) hot::invalid("theta must lie in (0, 1)");
    if (direct_max < 0) hot::invalid("direct_max must be >= 0");
    hot::Phase ph(ctx, HOT_T_LISTS);
    try {
      hot::build_lists(ctx, tree, theta, direct_max);
    } catch (...) {
      tree->has_lists = false;
      throw;
    }
  });
}

int build_interaction_lists_err(hot_ctx* ctx, hot_tree* tree, const double* mass, double err_tol,
                                int p_max, int direct_max) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!mass) hot::invalid("null masses");
    if (!(err_tol > 0.0) || !std::isfinite(err_tol)) hot::invalid("err_tol must be finite and > 0");
    if (p_max < 0 || p_max > 8) hot::invalid("p_max must lie in [0, 8]");
    if (direct_max < 0) hot::invalid("direct_max must be >= 0");
    hot::Phase ph(ctx, HOT_T_LISTS);
    try {
      hot::build_lists_err(ctx, tree, mass, err_tol, p_max, direct_max);
    } catch (...) {
      tree->has_lists = false;
      throw;
    }
  });
}

int build_interaction_lists_periodic_err(hot_ctx* ctx, hot_tree* tree, const double* mass,
                                         double err_tol, int p_max, int direct_max) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!tree->box_given) hot::state("periodic lists need a tree built with a given box");
    if (!mass) hot::invalid("null masses");
    if (!(err_tol > 0.0) || !std::isfinite(err_tol)) hot::invalid("err_tol must be finite and > 0");
    if (p_max < 0 || p_max > 8) hot::invalid("p_max must lie in [0, 8]");
    if (direct_max < 0) hot::invalid("direct_max must be >= 0");
    hot::Phase ph(ctx, HOT_T_LISTS);
    try {
      hot::build_lists_periodic_err(ctx, tree, mass, err_tol, p_max, direct_max);
    } catch (...) {
      tree->has_lists = false;
      tree->periodic = false;
      throw;
    }
  });
}

int build_interaction_lists_periodic(hot_ctx* ctx, hot_tree* tree, double theta, int direct_max) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!tree->box_given) hot::state("periodic lists need a tree built with a given box");
    if (!(theta > 0.0 && theta < 1.0)) hot::invalid("theta must lie in (0, 1)");
    if (direct_max < 0) hot::invalid("direct_max must be >= 0");
    hot::Phase ph(ctx, HOT_T_LISTS);
    try {
      hot::build_lists_periodic(ctx, tree, theta, direct_max);
    } catch (...) {
      tree->has_lists = false;
      tree->periodic = false;
      throw;
    }
  });
}

int build_interaction_lists_periodic_bs(hot_ctx* ctx, hot_tree* tree, double theta,
                                        int direct_max, int width) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!tree->box_given) hot::state("periodic lists need a tree built with a given box");
    if (!(theta > 0.0 && theta < 1.0)) hot::invalid("theta must lie in (0, 1)");
    if (direct_max < 0) hot::invalid("direct_max must be >= 0");
    if (width < 3 || width > 9 || !(width & 1)) hot::invalid("width must be odd, in [3, 9]");
    hot::Phase ph(ctx, HOT_T_LISTS);
    try {
      hot::build_lists_periodic_bs(ctx, tree, theta, direct_max, width);
    } catch (...) {
      tree->has_lists = false;
      tree->periodic = false;
      tree->bg = false;
      throw;
    }
  });
}

int eval_forces(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass, double eps,
                int precision, double* acc, double* pot, hot_stats* stats) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!pos || !mass || !acc) hot::invalid("null positions, masses or output");
    if (!(eps >= 0.0) || !std::isfinite(eps)) hot::invalid("eps must be finite and >= 0");
    if (!hot::valid_precision(precision)) hot::invalid("unknown precision or kernel flag");
    if (!tree->has_lists) hot::state("build_interaction_lists first");
    if (tree->p < 0) hot::state("compute_moments first");
    if (tree->p < tree->list_p) hot::state("moments of lower order than the lists");
    if (tree->bg && pot)
      hot::invalid("potentials are not available with background-subtracted lists");
    hot::Phase ph(ctx, HOT_T_EVAL);
    hot::forces(ctx, tree, pos, mass, eps, precision, acc, pot, stats);
    if (tree->periodic) hot::far_replicas(ctx, tree, pos, acc, pot);
    if (tree->bg) hot::background_boxes(ctx, tree, pos, acc);
  });
}

int eval_forces_noalloc(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass,
                        double eps, int precision, double* acc, double* pot, hot_stats* stats) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!pos || !mass || !acc) hot::invalid("null positions, masses or output");
    if (!(eps >= 0.0) || !std::isfinite(eps)) hot::invalid("eps must be finite and >= 0");
    if (!hot::valid_precision(precision)) hot::invalid("unknown precision or kernel flag");
    if (hot::fp64_mode(precision))
      hot::invalid("eval_forces_noalloc computes in HOT_MIXED only (FP64 needs per-tree moments)");
    if (!tree->has_lists) hot::state("build_interaction_lists first");
    if (tree->p < 0) hot::state("compute_moments first");
    if (tree->p < tree->list_p) hot::state("moments of lower order than the lists");
    if (tree->bg)
      hot::invalid("eval_forces_noalloc does not take background-subtracted lists "
                   "(their subtracted moments need device memory)");
    if (tree->n > kNoAllocMaxN)
      throw hot::Error{HOT_E_CAPACITY, "eval_forces_noalloc takes at most " +
                                           std::to_string(kNoAllocMaxN) + " particles, the tree has " +
                                           std::to_string(tree->n)};
    unsigned char* base = static_cast<unsigned char*>(scratch_address(ctx->device));
    hot::EvalMem mem;
    mem.off = base + kScratchOff;
    mem.state = base + kScratchState;
    mem.far_local = reinterpret_cast<double*>(base + kScratchLocal);
    hot::Phase ph(ctx, HOT_T_EVAL);
    hot::forces(ctx, tree, pos, mass, eps, precision, acc, pot, stats, &mem);
    if (tree->periodic) hot::far_replicas(ctx, tree, pos, acc, pot, mem.far_local);
  });
}

int eval_forces_adjoint(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass,
                        double eps, int precision, const double* acc_bar, double* pos_bar,
                        double* mass_bar) {
  return guard(ctx, [&] {
    need_tree(ctx, tree);
    if (!pos || !mass || !acc_bar || !pos_bar) hot::invalid("null argument");
    if (!(eps >= 0.0) || !std::isfinite(eps)) hot::invalid("eps must be finite and >= 0");
    if (!hot::valid_precision(precision)) hot::invalid("unknown precision or kernel flag");
    if (!tree->has_lists) hot::state("build_interaction_lists first");
    if (tree->p < 0) hot::state("compute_moments first");
    if (tree->p < tree->list_p) hot::state("moments of lower order than the lists");
    hot::Phase ph(ctx, HOT_T_ADJOINT);
    hot::adjoint(ctx, tree, pos, mass, eps, precision, acc_bar, pos_bar, mass_bar);
  });
}

int tree_get_counts(hot_ctx* ctx, hot_tree* t, int64_t* out) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (!out) hot::invalid("null output");
    std::vector<uint8_t> leaf(t->n_cells);
    d2h<uint8_t>(ctx, leaf.data(), t->c_leaf.p, t->n_cells);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
    int64_t nl = 0;
    for (auto v : leaf) nl += v;
    for (int k = 0; k < 16; ++k) out[k] = 0;
    out[0] = t->n;
    out[1] = t->n_cells;
    out[2] = t->n_groups;
    out[3] = nl;
    out[4] = t->max_level;
    out[5] = t->has_lists ? t->n_p2p : -1;
    out[6] = t->has_lists ? t->n_m2p : -1;
    out[7] = t->p;
    out[8] = t->n_items;
    out[9] = (int64_t)t->hash_slots;
    out[10] = t->has_lists ? t->p2p_pairs : -1;
    out[11] = t->has_lists ? t->m2p_pairs : -1;
    out[12] = t->has_lists && t->bg ? t->n_boxes : -1;
    out[13] = t->n_leaves;
  });
}

int tree_get_root(hot_ctx* ctx, hot_tree* t, double* lo_side) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    lo_side[0] = t->lo[0];
    lo_side[1] = t->lo[1];
    lo_side[2] = t->lo[2];
    lo_side[3] = t->side;
  });
}

int tree_get_keys(hot_ctx* ctx, hot_tree* t, uint64_t* keys, uint32_t* perm) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    d2h<uint64_t>(ctx, keys, t->key.p, t->n);
    d2h<uint32_t>(ctx, perm, t->perm.p, t->n);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_get_cells(hot_ctx* ctx, hot_tree* t, int32_t* level, uint64_t* key, int32_t* first,
                   int32_t* count, int32_t* parent, int32_t* child_first, int32_t* n_child,
                   int32_t* is_leaf, double* centre, double* bmax) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    const int64_t C = t->n_cells;
    std::vector<int8_t> lv(level ? C : 0);
    std::vector<uint8_t> lf(is_leaf ? C : 0);
    d2h<int8_t>(ctx, level ? lv.data() : nullptr, t->c_level.p, C);
    d2h<uint8_t>(ctx, is_leaf ? lf.data() : nullptr, t->c_leaf.p, C);
    d2h<uint64_t>(ctx, key, t->c_key.p, C);
    d2h<int32_t>(ctx, first, t->c_first.p, C);
    d2h<int32_t>(ctx, count, t->c_count.p, C);
    d2h<int32_t>(ctx, parent, t->c_parent.p, C);
    d2h<int32_t>(ctx, child_first, t->c_child.p, C);
    d2h<int32_t>(ctx, n_child, t->c_nchild.p, C);
    d2h<double>(ctx, centre, t->c_centre.p, 3 * C);
    d2h<double>(ctx, bmax, t->c_bmax.p, C);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; level && i < C; ++i) level[i] = lv[i];
    for (int64_t i = 0; is_leaf && i < C; ++i) is_leaf[i] = lf[i];
  });
}

int tree_get_groups(hot_ctx* ctx, hot_tree* t, int32_t* groups) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    d2h<int32_t>(ctx, groups, t->g_cell.p, t->n_groups);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_get_lists(hot_ctx* ctx, hot_tree* t, int64_t* p2p_off, int32_t* p2p, int64_t* m2p_off,
                   int32_t* m2p) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (!t->has_lists) hot::state("no lists");
    d2h<int64_t>(ctx, p2p_off, t->p2p_off.p, t->n_groups + 1);
    d2h<int64_t>(ctx, m2p_off, t->m2p_off.p, t->n_groups + 1);
    d2h<int32_t>(ctx, p2p, t->p2p.p, t->n_p2p);
    d2h<int32_t>(ctx, m2p, t->m2p.p, t->n_m2p);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_get_list_images(hot_ctx* ctx, hot_tree* t, int8_t* p2p_img, int8_t* m2p_img) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (!t->has_lists || !t->periodic) hot::state("no periodic lists");
    d2h<int8_t>(ctx, p2p_img, t->p2p_img.p, t->n_p2p);
    d2h<int8_t>(ctx, m2p_img, t->m2p_img.p, t->n_m2p);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_get_background(hot_ctx* ctx, hot_tree* t, int64_t* box_off, double* boxes,
                        int8_t* box_sign, int8_t* m2p_sub) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (!t->has_lists || !t->bg) hot::state("no background-subtracted lists");
    if (box_off) d2h<int64_t>(ctx, box_off, t->box_off.p, t->n_groups + 1);
    if (boxes) d2h<double>(ctx, boxes, t->boxes.p, 6 * t->n_boxes);
    if (box_sign) d2h<int8_t>(ctx, box_sign, t->box_sign.p, t->n_boxes);
    if (m2p_sub) d2h<int8_t>(ctx, m2p_sub, t->m2p_sub.p, t->n_m2p);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_get_m2p_orders(hot_ctx* ctx, hot_tree* t, int8_t* orders) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (!t->has_lists || t->list_p < 0) hot::state("no error-bound lists");
    if (!orders) hot::invalid("null output");
    d2h<int8_t>(ctx, orders, t->m2p_q.p, t->n_m2p);
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_get_moments(hot_ctx* ctx, hot_tree* t, double* out) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (t->p < 0) hot::state("no moments");
    d2h<double>(ctx, out, t->mom64.p, (size_t)t->n_cells * hot::nm(t->p));
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int tree_lookup(hot_ctx* ctx, hot_tree* t, int64_t nq, const uint64_t* keys, int32_t* cells) {
  return guard(ctx, [&] {
    need_tree(ctx, t);
    if (nq <= 0) return;
    if (!keys || !cells) hot::invalid("null argument");
    hot::DBuf dk, dc;
    dk.alloc(ctx, nq * sizeof(uint64_t));
    dc.alloc(ctx, nq * sizeof(int32_t));
    HOT_HIP(hipMemcpyAsync(dk.p, keys, nq * sizeof(uint64_t), hipMemcpyHostToDevice, ctx->stream));
    hot::hash_lookup(ctx, t, dk.as<uint64_t>(), dc.as<int32_t>(), nq);
    HOT_HIP(hipMemcpyAsync(cells, dc.p, nq * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HOT_HIP(hipStreamSynchronize(ctx->stream));
  });
}

}  // extern "C"
