/*
 * hot.h -- C ABI of the MI355X hashed oct-tree gravitational force library.
 *
 * The library evaluates the softened Newtonian accelerations of N particles
 * (eq. "eom" of the Mathematical Approach section at scale factor a = 1 and
 * G = 1, with the Plummer smoothing of the Force Smoothing section) by the
 * cell-body multipole treecode of the paper: integer Morton keys and a sort
 * (Domain Decomposition section), an oct-tree of key-addressed cells kept in
 * a hash table (Tree Construction and Traversal section), moments about
 * geometric cell centres (Background Subtraction and Multipole Error Bounds
 * sections), a multipole acceptance walk per sink cell with m x n blocking
 * (Improving instruction-level parallelism section) and the Cartesian
 * expansion with Delta = 0 (Multipole Error Bounds section). It also gives
 * the reverse derivative (vector-Jacobian product) of that evaluation with the
 * tree topology held fixed.
 *
 * Conventions shared by every call:
 *  - All array arguments are DEVICE pointers unless the comment says host.
 *  - pos / acc / pos_bar / acc_bar: N x 3 row-major float64 (x0 y0 z0 x1 ...).
 *    mass / pot / mass_bar: N float64. Outputs are in caller order.
 *  - Work is enqueued on the context's HIP stream and may still be running
 *    when a call returns. The caller keeps its buffers alive until the stream
 *    has passed the call. Calls that must size device buffers from device
 *    results (tree_build, build_interaction_lists) synchronise the stream.
 *  - Return value: HOT_OK (0) or a negative HOT_E_* code; hot_last_error()
 *    gives a message. A failed call leaves the tree as it was before the call
 *    or marks it invalid (then only tree_destroy is accepted); nothing leaks.
 *  - One context per host thread. A tree belongs to the context that built it.
 */
#ifndef HOT_H
#define HOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HOT_OK = 0,
  HOT_E_INVALID = -1,  /* bad argument: see each call */
  HOT_E_STATE = -2,    /* call out of order (e.g. eval before moments) */
  HOT_E_OOM = -3,      /* device allocation failed */
  HOT_E_DEVICE = -4,   /* a HIP runtime error */
  HOT_E_CAPACITY = -5  /* a size limit of the library was exceeded */
};

enum { HOT_MIXED = 0, HOT_FP64 = 1 };

/* Softening kernel (Force Smoothing section), ORed into the precision
 * argument of eval_forces, eval_forces_noalloc and eval_forces_adjoint:
 * without it the Plummer kernel, phi = -m (r^2 + eps^2)^(-1/2); with HOT_K1
 * Dehnen's compensating kernel K1 with compact support of radius eps, the
 * one the section names for production runs. Its density, in x = r / eps < 1,
 *   rho(r) = 1575 / (128 pi eps^3) (1 - x^2)^2 (1 - 11 x^2 / 5)
 * (zero beyond eps), is the lowest-degree even polynomial that vanishes with
 * its slope at eps and has unit mass and a zero second moment (the
 * compensation that cancels the leading force bias); its potential per unit
 * mass is -(945 - 2100 x^2 + 2646 x^4 - 1620 x^6 + 385 x^8) / (256 eps)
 * inside and exactly -1/r outside, so the force is Newtonian beyond eps.
 * eps = 0 gives the Newtonian kernel with either choice. */
enum { HOT_K1 = 16 };

typedef struct hot_ctx hot_ctx;
typedef struct hot_tree hot_tree;

/* Optional device allocator. alloc returns NULL on failure; both run on the
 * caller's thread and receive the stream that first uses the block: the
 * context stream, except for the adjoint's transposed lists, which the
 * library builds on a second stream of its own (it starts after all work
 * queued on the context stream before the call, and the context stream waits
 * for it before reading them). The allocator must order reuse by that
 * stream: a block freed on one stream may go to another only once the work
 * queued before the free has finished. NULL selects hipMallocAsync /
 * hipFreeAsync on the given stream, which does so. */
typedef struct hot_allocator {
  void* (*alloc)(void* user, size_t bytes, void* stream);
  void (*free)(void* user, void* ptr, void* stream);
  void* user;
} hot_allocator;

/* Tree shape. n_leaf: a cell holding more than n_leaf particles is split
 * (1 <= n_leaf <= n_group). n_group: sink groups are the topmost cells with at
 * most n_group particles, or leaves that still hold more (1 <= n_group <=
 * 4096). box (HOST pointer, may be NULL): lo[3], side -- the root cube, side
 * a positive power of two, every point inside [lo, lo + side]; NULL derives
 * it from the data (per-axis minimum, next power of two of the largest
 * extent). Unless set, n_leaf = 16 and n_group = 64. */
typedef struct hot_build_opts {
  int n_leaf;
  int n_group;
  const double* box;
} hot_build_opts;

/* Counters filled by eval_forces when stats is not NULL (HOST struct). The
 * call then synchronises the stream and times its kernels. */
typedef struct hot_stats {
  int64_t p2p_pairs;     /* sum over sinks of the particles in their P2P cells */
  int64_t m2p_pairs;     /* sum over sinks of their M2P cells */
  double ms_p2p;
  double ms_m2p;
  double ms_total;
} hot_stats;

/* Phases timed by the context when timing is on (hot_set_timing): each
 * entry point and, inside the evaluation and the adjoint, each interaction
 * kernel. The adjoint's transpose phase is the first call's construction of
 * the transposed lists, recorded on the context's second stream: it runs
 * beside the sink-side kernels, so its duration is the wall time it spans
 * while sharing the GPU with them, not its cost alone; its downward phase is the moment cotangents' pass
 * down the tree (M2M transposed), the moment-to-particle transpose, the far
 * replicas and background terms, and the final write-back. */
enum {
  HOT_T_TREE_BUILD = 0,
  HOT_T_MOMENTS,
  HOT_T_LISTS,
  HOT_T_EVAL,
  HOT_T_EVAL_P2P,
  HOT_T_EVAL_M2P,
  HOT_T_ADJOINT,
  HOT_T_ADJ_TRANSPOSE,
  HOT_T_ADJ_P2P_SINK,
  HOT_T_ADJ_P2P_SOURCE,
  HOT_T_ADJ_M2P_SINK,
  HOT_T_ADJ_M2P_CELL,
  HOT_T_ADJ_DOWNWARD,
  HOT_T_COUNT
};

/* Context on one device. hip_stream (hipStream_t) may be NULL for the null
 * stream. allocator may be NULL (see hot_allocator). */
int hot_ctx_create(int device, void* hip_stream, const hot_allocator* allocator, hot_ctx** out);
int hot_ctx_destroy(hot_ctx* ctx);
/* Message of the last failure on this context (never NULL). */
const char* hot_last_error(hot_ctx* ctx);
/* Wait for the stream; returns a deferred device-side error (e.g. a
 * non-finite position or mass found by an asynchronous call) as
 * HOT_E_INVALID, or a HIP error as HOT_E_DEVICE. A deferred error is
 * reported once: by hot_sync or by the next call that synchronises the stream
 * (tree_build, the build_interaction_lists* calls), which then fails with it
 * and does nothing else. */
int hot_sync(hot_ctx* ctx);

/* Phase timers. hot_set_timing(ctx, 1) makes every later call record HIP
 * events on the context stream at the start and end of its phases (the
 * HOT_T_* list above; recording adds no synchronisation), and forgets earlier
 * records; 0 stops recording. hot_get_timings waits for the stream and writes
 * ms[HOT_T_COUNT] (HOST): the duration of each phase in its most recent
 * recorded run, -1 for phases not run since timing was switched on. */
int hot_set_timing(hot_ctx* ctx, int on);
int hot_get_timings(hot_ctx* ctx, double* ms);

/*
 * tree_build -- keys, sort, cells, hash table, sink groups and b_max.
 * Domain Decomposition section (keys mapped from coordinates, sorted) and
 * Tree Construction and Traversal section (hashed oct-tree cells).
 * Keys: 21 bits per axis quantised as floor((x - lo) 2^21 / side), clamped to
 * 2^21 - 1; octant digit 4x + 2y + z from the most significant level; a
 * leading placeholder bit (the root key is 1). Sort: stable by key. A cell at
 * level L < 21 with more than n_leaf particles has its non-empty octants as
 * children. Centres are the geometric cube centres, b_max the largest
 * particle distance from the centre.
 * n: 1 .. 2^31 - 1. pos: N x 3 (device). Errors: HOT_E_INVALID for bad sizes
 * or options, non-finite positions, a box side that is not a power of two, a
 * point outside the given box. The tree holds device memory until
 * tree_destroy.
 */
int tree_build(hot_ctx* ctx, int64_t n, const double* pos, const hot_build_opts* opts,
               hot_tree** out);
int tree_destroy(hot_ctx* ctx, hot_tree* tree);

/*
 * compute_moments -- raw Cartesian moments of every cell to order p about its
 * geometric centre, M_alpha = sum_j m_j (x_j - c)^alpha, |alpha| <= p (the
 * moment tensor of the Multipole Error Bounds section; order p = 2 is the
 * quadrupole, 4 the hexadecapole). Leaves from their particles, other cells by
 * re-centring their children's moments. FP64. pos may differ from the
 * positions the tree was built from: membership and centres stay fixed.
 * mass: N (device), finite and >= 0 (checked asynchronously, reported by the
 * next synchronising call). p: 0 .. 8.
 */
int compute_moments(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass, int p);

/*
 * build_interaction_lists -- for every sink group g, a depth-first walk of the
 * source tree from the root, children in octant order: a cell c passing the
 * acceptance test goes to the M2P list (or to the P2P list if it holds at
 * most direct_max particles); a leaf failing it goes to the P2P list; any
 * other cell is opened. Acceptance: with d the distance between the group and
 * cell centres, d^2 > (b_c / theta + b_g)^2 (FP64, no fused multiply-add);
 * the group form of the b_max criterion in the source/sink geometry of the
 * Multipole Error Bounds section. Lists are in depth-first preorder. Every
 * list builder also tabulates each group's P2P list as pair segments
 * (consecutive entries with contiguous particle ranges, cut at source-group
 * boundaries, with their FP64 centre offsets), which the pair kernels read.
 * theta: (0, 1). direct_max: >= 0. Synchronises the stream twice (list
 * sizes, then the segment count).
 */
int build_interaction_lists(hot_ctx* ctx, hot_tree* tree, double theta, int direct_max);

/*
 * build_interaction_lists_err -- the same walk with an absolute-error
 * acceptance test that also picks the expansion order of each interaction
 * (Multipole Error Bounds section: an error-based MAC that chooses the
 * cheapest order meeting a given accuracy). For cell c and group g, with
 * d = |centre_g - centre_c| - b_g, b = b_c, t = b / d and M = count_c times the
 * largest particle mass, the field error of the order-q expansion at any sink
 * of g is bounded (unsoftened) by
 *   E_q = M / (d - b)^2 * ((q + 2) - (q + 1) t) * t^(q + 1);
 * c is accepted at the smallest q in [0, p_max] with E_q <= err_tol (FP64, no
 * fused multiply-add, d > b required), otherwise opened (P2P if a leaf).
 * Accepted cells with at most direct_max particles go to the P2P list. The
 * M2P entries carry their order (tree_get_m2p_orders); evaluation and adjoint
 * need moments of order >= p_max.
 * mass: N (device; only its maximum is used). err_tol: finite, > 0 (an
 * acceleration). p_max: 0 .. 8. direct_max: >= 0. Synchronises the stream.
 */
int build_interaction_lists_err(hot_ctx* ctx, hot_tree* tree, const double* mass, double err_tol,
                                int p_max, int direct_max);

/*
 * build_interaction_lists_periodic -- periodic boundaries (Boundary
 * Conditions section): the root cube, which must have been given to
 * tree_build as opts->box, is the periodic cell of side L. The theta walk
 * above runs over each of the 125 near images of the source tree (the cube
 * shifted by n L, max|n_d| <= 2; image = 25 (n_x + 2) + 5 (n_y + 2) + n_z + 2),
 * images in that order, entries tagged with their image (tree_get_list_images);
 * the self pair is skipped in the unshifted image only. eval_forces then adds
 * the far replicas with a uniform neutralising background (Ewald's split of
 * the lattice sum, no surface term) through their lattice sums: a local
 * expansion about the cube centre built from the root's moments, derivatives
 * of the far function to order 2p + 1, applied to order p. eval_forces_adjoint
 * differentiates all of it, the far replicas included (through the sink
 * positions and the root's moments). Potentials, where asked for, are those
 * of the same split: with the background, whose constant enters the order-0
 * lattice sum, a lone particle at the cube centre has phi = +2.8373 m / L.
 * theta: (0, 1); direct_max: >= 0.
 * Synchronises the stream.
 */
int build_interaction_lists_periodic(hot_ctx* ctx, hot_tree* tree, double theta, int direct_max);

/*
 * build_interaction_lists_periodic_err -- the periodic lists above with the
 * error-bound test of build_interaction_lists_err in place of the theta test
 * (per image entry, on the shifted centre; every M2P entry carries its order,
 * tree_get_m2p_orders, and its image, tree_get_list_images). Evaluation,
 * potentials and adjoint as for periodic lists; moments of order >= p_max
 * are needed.
 * mass: N (device; only its maximum is used). err_tol: finite, > 0.
 * p_max: 0 .. 8. direct_max: >= 0. Synchronises the stream.
 */
int build_interaction_lists_periodic_err(hot_ctx* ctx, hot_tree* tree, const double* mass,
                                         double err_tol, int p_max, int direct_max);

/*
 * build_interaction_lists_periodic_bs -- the periodic lists above with
 * background subtraction (Background Subtraction section and its figure):
 * the sources become density contrasts, matter minus the mean density
 * rho = M_total / L^3 (M_total the root's monopole at evaluation). For a
 * sink group of side s, N(g) is the cube of side width * s about its centre
 * (width odd, 3 .. 9; the section's figure draws 3: a region that roughly
 * surrounds the pair-summed cells keeps their exact box fields few).
 * Source cells inside N(g) interact as usual. Outside it every M2P entry
 * uses its cell's moments minus those of its uniform cube, to the same
 * order as the matter (flagged per entry, tree_get_background), and P2P
 * cells and empty octants of opened cells contribute the exact field of
 * their negative uniform cube, listed per group as boxes with sign -1; a
 * cell straddling the border of N(g) is opened whatever the theta test
 * says, and where a straddling leaf or empty octant remains, its
 * intersection with N(g) is listed with sign +1. eval_forces then adds, per
 * sink, rho times the exact fields of its group's boxes, minus N(g)'s, plus
 * that of the whole 5L cube of the near zone (unsoftened, FP64), so that
 * with no truncation the result equals that of the periodic lists without
 * subtraction. eval_forces_adjoint differentiates all of it: the
 * subtracted moments at the sink, the box fields through the sink position,
 * and the mean density through every mass. Potentials are not available
 * with these lists (HOT_E_INVALID). theta: (0, 1); direct_max: >= 0.
 * Synchronises the stream.
 */
int build_interaction_lists_periodic_bs(hot_ctx* ctx, hot_tree* tree, double theta,
                                        int direct_max, int width);

/*
 * eval_forces -- accelerations (and optionally potentials) of all particles:
 *   a_i = sum over P2P cells, j != i:  m_j (x_j - x_i) (|x_j - x_i|^2 + eps^2)^(-3/2)
 *       + sum over M2P cells c:  -sum_{|alpha|<=p} (-1)^|alpha|/alpha! M_alpha
 *                                 d^(alpha+e_k) G(x_i - c),  G(R) = -(|R|^2+eps^2)^(-1/2)
 * (pair kernel of eq. "eom" with Plummer smoothing; the cell-body expansion
 * with Delta = 0 of the Multipole Error Bounds section, softened G).
 * precision HOT_MIXED: pair and expansion arithmetic in FP32 on offsets from
 * FP64 group centres, expansions scaled by the source cell side, per-sink
 * compensated (Kahan) FP32 sums, FP64 output; HOT_FP64: all FP64.
 * eps: finite, >= 0. acc: N x 3 out. pot: N out or NULL (phi_i = -sum m_j
 * (r^2+eps^2)^(-1/2) + expansion). stats: HOST or NULL. Needs
 * compute_moments and build_interaction_lists on this tree first.
 */
int eval_forces(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass, double eps,
                int precision, double* acc, double* pot, hot_stats* stats);

/*
 * eval_forces_adjoint -- the vector-Jacobian product of eval_forces with the
 * topology (membership, centres, b_max, lists) held fixed:
 *   pos_bar = d(sum_i acc_bar_i . a_i)/d pos,  mass_bar = d(...)/d mass.
 * Pair terms move both the sink and the source; expansion terms move the sink
 * (second derivatives of the expansion) and the source particles through the
 * moments (centres fixed). acc_bar: N x 3 (device). pos_bar: N x 3 out.
 * mass_bar: N out or NULL. Same precision modes as eval_forces. The first call
 * on a tree builds and caches transposed lists, on a second stream of the
 * context (created on first use) while the sink-side terms run on the
 * context stream; it waits for them on the host twice (list counts) and the
 * context stream waits for them before the source-side terms. Later calls
 * use only the context stream.
 */
int eval_forces_adjoint(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass,
                        double eps, int precision, const double* acc_bar, double* pos_bar,
                        double* mass_bar);

/*
 * eval_forces_noalloc -- eval_forces for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, results and errors as eval_forces
 * (bit-identical results: the same kernels run), and it allocates nothing:
 * the per-particle buffers of the evaluation (FP32 offsets and masses, the
 * compensated sums) and the far replicas' local coefficients live in one
 * fixed device array of the library, 48 MiB + 4 KiB on every GPU it runs on,
 * held from the library's load until the process ends. Limits: precision
 * HOT_MIXED only (HOT_E_INVALID otherwise); at most 2^20 particles
 * (HOT_E_CAPACITY beyond); theta, error-bound and periodic lists, not
 * background-subtracted ones (HOT_E_INVALID). Every call on one GPU uses
 * that GPU's array: calls that overlap on one GPU (on other streams, from
 * other threads or contexts) race, and the caller must order them; calls on
 * one stream are ordered by it. The array keeps the last call's contents;
 * nothing in it needs clearing (every element is written before it is read).
 */
int eval_forces_noalloc(hot_ctx* ctx, hot_tree* tree, const double* pos, const double* mass,
                        double eps, int precision, double* acc, double* pot, hot_stats* stats);

/* ---- host-copy getters (synchronise; for tests and diagnostics) ---------- */

/* out[16]: n, n_cells, n_groups, n_leaves, max_level, n_p2p_entries,
 * n_m2p_entries, p (or -1), n_work_items, hash_slots, p2p_pairs, m2p_pairs,
 * n_background_boxes, entries of the particle-ordered leaf list (equal to
 * n_leaves), 0... (-1 where not yet built or not applicable). */
int tree_get_counts(hot_ctx* ctx, hot_tree* tree, int64_t* out);
/* HOST: lo_side[4] = root cube lo[3], side. */
int tree_get_root(hot_ctx* ctx, hot_tree* tree, double* lo_side);
/* HOST: sorted keys [N] and perm [N] (sorted position -> caller index). */
int tree_get_keys(hot_ctx* ctx, hot_tree* tree, uint64_t* keys, uint32_t* perm);
/* HOST arrays of n_cells entries (any may be NULL), canonical order
 * (level, key): level, key (with placeholder), first particle (sorted
 * position), count, parent (-1 root), first child (-1 none), number of
 * children, leaf flag, centre (x y z per cell), b_max. */
int tree_get_cells(hot_ctx* ctx, hot_tree* tree, int32_t* level, uint64_t* key, int32_t* first,
                   int32_t* count, int32_t* parent, int32_t* child_first, int32_t* n_child,
                   int32_t* is_leaf, double* centre, double* bmax);
/* HOST: group cell ids [n_groups], ordered by first particle. */
int tree_get_groups(hot_ctx* ctx, hot_tree* tree, int32_t* groups);
/* HOST: CSR lists over groups: p2p_off [n_groups+1], p2p [n_p2p_entries],
 * m2p_off, m2p (cell ids); any may be NULL. */
int tree_get_lists(hot_ctx* ctx, hot_tree* tree, int64_t* p2p_off, int32_t* p2p,
                   int64_t* m2p_off, int32_t* m2p);

/* Expansion order of every M2P entry (host out, n_m2p int8, list order);
 * HOT_E_STATE unless the lists came from build_interaction_lists_err. */
int tree_get_m2p_orders(hot_ctx* ctx, hot_tree* tree, int8_t* orders);

/* Background-subtracted lists (host outs, each may be NULL): box_off
 * n_groups + 1 (CSR offsets), boxes 6 per box (lo[3], hi[3]), box_sign one
 * per box (+1 / -1), m2p_sub one per M2P entry (1: the cell's uniform cube is
 * subtracted). HOT_E_STATE unless the lists came from
 * build_interaction_lists_periodic_bs. */
int tree_get_background(hot_ctx* ctx, hot_tree* tree, int64_t* box_off, double* boxes,
                        int8_t* box_sign, int8_t* m2p_sub);

/* Image (0 .. 124) of every P2P and M2P entry of periodic lists (host out,
 * n_p2p and n_m2p int8, list order; either may be NULL); HOT_E_STATE unless
 * the lists came from build_interaction_lists_periodic. */
int tree_get_list_images(hot_ctx* ctx, hot_tree* tree, int8_t* p2p_img, int8_t* m2p_img);

/* HOST: FP64 moments [n_cells x (p+1)(p+2)(p+3)/6], slot order by order n,
 * then x exponent descending, then y exponent descending. */
int tree_get_moments(hot_ctx* ctx, hot_tree* tree, double* out);
/* Hash-table lookup of cell keys (HOST arrays): cell id or -1. */
int tree_lookup(hot_ctx* ctx, hot_tree* tree, int64_t nq, const uint64_t* keys, int32_t* cells);

#ifdef __cplusplus
}
#endif
#endif /* HOT_H */
