/*
 * dem.h -- C ABI of the MI355X (gfx950) multiresolution contact-detection
 * library (libdem.so).
 *
 * The operations follow Noble & Weinzierl, "A multiresolution Discrete
 * Element Method for triangulated objects with implicit time stepping"
 * (arXiv 2105.12415):
 *
 *   - particles are closed triangulated surfaces, each surrounded by an
 *     epsilon environment (Section 2, Definition "contact point");
 *   - two triangles are in contact iff their epsilon environments overlap,
 *     i.e. iff their distance d <= eps_i + eps_j; the contact point lies on
 *     the shortest path between the triangles with normal n(c) pointing to a
 *     triangle (Section 2, minimisation problem for x(c));
 *   - findContacts over a pair of particles (Algorithm 2) is answered either
 *     over all fine triangle pairs (DEM_MODE_FLAT) or by descending a
 *     surrogate tree that prunes the children of surrogate pairs whose
 *     epsilon environments do not overlap (Algorithm 5, Section 5.1);
 *   - every triangle pair is evaluated with the batched, fixed-iteration,
 *     penalty-regularised closest-point iteration (Section 3, iterative
 *     functional and its modified Newton update; Algorithm 4), and pairs
 *     the iteration cannot settle ("not terminated") fall back to the exact
 *     comparison-based distance (Section 3, direct distance calculation);
 *   - surrogate trees are built offline (Section 4, surrogate tree
 *     definition; Appendix B, Algorithm 7) with the smallest epsilon that
 *     keeps each surrogate conservative (Section 4, Definition
 *     "conservative").
 *
 * Conventions for every call:
 *   - All pointers documented "device" are caller-owned device memory
 *     (e.g. torch tensors); the library allocates no device memory and keeps
 *     no state between calls.  Host pointers are read during the call only.
 *   - Calls that take a stream enqueue work on it and return without
 *     synchronising; they contain no host-device copies or allocations, so
 *     they can be captured into a HIP graph.  Errors the host can see
 *     (bad arguments, undersized workspace, launch failures) are returned
 *     as dem_status; conditions only the device can see are OR-ed into
 *     *dev_status (DEM_DEV_* bits) for the caller to read after the stream
 *     has completed.
 *   - Coordinates are float (DEM_F32) or double (DEM_F64) as selected by
 *     dem_scene.precision; all floating-point device buffers of a call use
 *     that type unless stated otherwise.
 */
#ifndef DEM_H_
#define DEM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DEM_OK = 0,
  DEM_ERR_ARG = -1,               /* invalid argument (null pointer, size, layout) */
  DEM_ERR_CAPACITY = -2,          /* workspace smaller than dem_workspace_bytes() */
  DEM_ERR_HIP = -3,               /* a HIP runtime call or kernel launch failed */
  DEM_ERR_NOT_CONSERVATIVE = -4,  /* hierarchy input violates the surrogate-tree rules */
  DEM_ERR_OOM = -5                /* host allocation failed (dem_build_hierarchy) */
} dem_status;

typedef enum { DEM_F32 = 0, DEM_F64 = 1 } dem_precision;
typedef enum { DEM_MODE_FLAT = 0, DEM_MODE_HIER = 1 } dem_mode;

/* Bits OR-ed into *dev_status by the device. */
#define DEM_DEV_CONTACT_OVERFLOW 0x1u /* more contacts than dem_contacts.capacity */
#define DEM_DEV_QUEUE_OVERFLOW 0x2u   /* a level work queue exceeded queue_capacity */
#define DEM_DEV_NEAR_OVERFLOW 0x4u    /* near-pair list exceeded near_capacity */
#define DEM_DEV_NONFINITE 0x8u        /* a non-finite coordinate or distance was met */
#define DEM_DEV_BAD_TREE 0x10u        /* a child count outside 0..DEM_MAX_CHILDREN, or a surrogate pair
                                         surviving at depth n_levels_max - 1 (a tree deeper than
                                         dem_scene.n_levels_max states: its pairs below were not tested) */
#define DEM_DEV_FRONTIER_OVERFLOW 0x20u /* active sets outgrew dem_frontier's capacity or memory set */
#define DEM_DEV_STALLED 0x40u         /* persistent descent: a grid barrier gave up waiting (results invalid) */

#define DEM_MAX_LEVELS 32
#define DEM_MAX_CHILDREN 16           /* children per surrogate (N_surrogate <= 16) */

typedef void* dem_stream_t; /* a hipStream_t (0 = the null stream) */

/* ------------------------------------------------------------------ hierarchy */

typedef struct {
  /* Upper bound on |coordinate| the mesh will take in the world frame.  Sets
   * an absolute slack of coord_scale * 2^-19 on every stored surrogate
   * epsilon, which covers the FP32 rounding of vertices that are rigidly
   * moved after the build.  0 = use the largest |coordinate| of verts. */
  double coord_scale;
  /* Relative slack added to surrogate epsilons (>= 0; default 1e-6). */
  double rel_slack;
} dem_build_opts;

typedef struct {
  int32_t n_tris;        /* triangles of all levels */
  int32_t n_levels;
  int32_t* tri_verts;    /* [n_tris][3] vertex ids (as given) */
  int32_t* child_begin;  /* [n_tris] id of the first child (0 if none) */
  int32_t* child_count;  /* [n_tris] number of children; 0 marks a fine triangle */
  int32_t* level_begin;  /* [n_levels + 1] first triangle id of each level */
  double* eps;           /* [n_tris] epsilon in FP64: eps0 for fine triangles,
                            eps0 + max deviation of the fine descendants for surrogates */
  float* eps_f32;        /* [n_tris] eps with slack, rounded up to float */
  double* eps_f64;       /* [n_tris] eps with slack (double) */
  int32_t root_begin, root_count; /* level 0 = the coarsest model (tree root) */
  int32_t fine_begin, fine_count; /* last level = the particle triangulation */
  double max_dev;        /* largest surrogate deviation (eps - eps0) */
} dem_hierarchy;

/*
 * dem_build_hierarchy -- offline, host, FP64 (Section 4, surrogate tree
 * definition; Appendix B, Algorithm 7 "assign the smallest epsilon such that
 * the surrogate is conservative").
 *
 * verts     [n_verts][3] host, FP64: vertex positions of one particle (any
 *           frame; distances are invariant under the rigid motions applied
 *           later).
 * tris      [n_tris][3] host: vertex ids of all triangles, levels
 *           concatenated from the coarsest (level 0, the root model) to the
 *           finest (the particle triangulation).
 * parent    [n_tris] host: for a triangle of level l >= 1 the id (into
 *           tris) of its parent: in level l-1 for surrogate levels, in any
 *           earlier level for the last (fine) level, so that leaf sets may
 *           sit at different depths; ignored for level 0.  Children of one
 *           parent must be contiguous and levels sorted by parent.
 * level_sizes [n_levels] host: triangles per level (sum = n_tris).
 * eps0      epsilon of the fine triangles (uniform per particle, Section 2).
 * opts      may be NULL (defaults).
 * out       filled with library-allocated host arrays; release with
 *           dem_hierarchy_free.  Every triangle of levels < n_levels-1 must
 *           have between 1 and DEM_MAX_CHILDREN children and the last level
 *           must have none.
 *
 * Each surrogate gets eps = eps0 + max over the vertices of its fine
 * descendants of their distance to the surrogate triangle: the distance to
 * a triangle is convex, so the maximum over a fine triangle is at a vertex,
 * and that eps is the smallest for which the surrogate's environment holds
 * every fine descendant's eps0 environment (Definition "conservative").
 * Returns DEM_ERR_ARG / DEM_ERR_NOT_CONSERVATIVE on malformed input.
 */
dem_status dem_build_hierarchy(const double* verts, int32_t n_verts, const int32_t* tris,
                               const int32_t* parent, const int32_t* level_sizes, int32_t n_levels,
                               double eps0, const dem_build_opts* opts, dem_hierarchy* out);
void dem_hierarchy_free(dem_hierarchy* h);

/*
 * Surrogate trees for generic meshes (Appendix B, Algorithm 7, with the
 * surrogate triangles of Appendix A).  Offline, host, FP64.
 */
typedef struct {
  int32_t fanout;        /* N_surrogate: subsets per split and largest leaf set (2..DEM_MAX_CHILDREN) */
  int32_t kmeans_iters;  /* Lloyd iterations of each k-means split */
  int32_t fit_iters;     /* descent steps of each surrogate fit */
  double beta_size;      /* exponent of the size term (>= 2) */
  double alpha_area;     /* weight of the anti-degeneracy term (> 0; coordinates scaled by the set radius) */
  double alpha_inside;   /* weight of the outer-normal term (>= 0) */
  double beta_normal;    /* exponent of the outer-normal term (>= 1) */
} dem_tree_opts;

typedef struct {
  int32_t n_verts;       /* the mesh's vertices, then three per surrogate */
  double* verts;         /* [n_verts][3] */
  int32_t n_tris;        /* surrogates + mesh triangles */
  int32_t* tris;         /* [n_tris][3]: surrogates depth by depth, then the mesh triangles grouped by parent */
  int32_t* parent;       /* [n_tris]: -1 for the root; a surrogate of depth d >= 1 hangs below depth
                            d-1, a mesh triangle below any surrogate */
  int32_t n_levels;      /* surrogate depths + 1 */
  int32_t* level_sizes;  /* [n_levels]: surrogates per depth, then the number of mesh triangles */
  int32_t* fine_order;   /* [number of mesh triangles]: input index of each mesh triangle in output order */
} dem_surrogate_tree;

/* Fill o with the defaults (fanout 8, 12 k-means iterations, 60 fit steps,
 * beta_size 8, alpha_area 1e-3, alpha_inside 1, beta_normal 2). */
void dem_default_tree_opts(dem_tree_opts* o);

/*
 * dem_build_surrogate_tree -- top-down surrogate tree of one particle.
 *
 * verts     [n_verts][3] host, FP64; tris [n_tris][3] host: the particle's
 *           triangulation (any closed or open mesh).
 * opts      may be NULL (defaults).
 * out       library-allocated host arrays, released by
 *           dem_surrogate_tree_free; its verts, tris, parent, level_sizes
 *           and n_levels are the arguments dem_build_hierarchy takes.
 *
 * A set of more than fanout triangles is split into at most fanout subsets
 * by k-means on the triangle centroids (farthest-point start), each subset
 * gets a surrogate triangle, and the recursion continues; a set of at most
 * fanout triangles becomes the children of its surrogate.  A surrogate
 * triangle minimises Appendix A's functional: a high power of the distances
 * from its vertices to the set's triangles (small), a penalty on its inverse
 * squared area (not degenerate) and one on its vertices lying outside the
 * set's triangles along its outer normal (nestled).  Epsilons are not set
 * here: dem_build_hierarchy gives every surrogate the smallest conservative
 * one, so any surrogate triangle is correct and the fit only matters for
 * how much it prunes.  Returns DEM_ERR_ARG on malformed input.
 */
dem_status dem_build_surrogate_tree(const double* verts, int32_t n_verts, const int32_t* tris,
                                    int32_t n_tris, const dem_tree_opts* opts, dem_surrogate_tree* out);
void dem_surrogate_tree_free(dem_surrogate_tree* t);

/* ------------------------------------------------------------------ scene */

/* A scene: all particles, all levels, in one global numbering (device). */
typedef struct {
  int32_t precision;      /* dem_precision of verts and tri_eps */
  int32_t n_verts;
  int32_t n_tris;         /* all levels of all particles */
  int32_t n_particles;
  int32_t n_levels_max;   /* largest number of levels of any particle (<= DEM_MAX_LEVELS) */
  const void* verts;      /* [3][n_verts] SoA world coordinates */
  const int32_t* tri_verts;   /* [3][n_tris] SoA global vertex ids */
  const int32_t* child_begin; /* [n_tris] global id of the first child */
  const int32_t* child_count; /* [n_tris] 0 marks a fine triangle */
  const int32_t* tri_particle;/* [n_tris] owning particle */
  const void* tri_eps;        /* [n_tris] epsilon (surrogate eps with slack) */
  const int32_t* root_begin;  /* [n_particles] coarsest-level triangles */
  const int32_t* root_count;
  const int32_t* fine_begin;  /* [n_particles] fine (particle) triangles */
  const int32_t* fine_count;
  /* Optional [n_particles][12] rigid motion per particle (row-major R, then
   * c): the kernels use world = R v + c for the vertices v of verts, applied
   * while flattening each step's triangle soup (Section 3, triangle soup:
   * every coordinate undergoes the update's affine transformation).  NULL:
   * verts already are world coordinates.  Gradients are always with respect
   * to world positions. */
  const void* pose;
  /* Optional lazy flattening (HIER mode): the surrogates whose children are
   * fine triangles, grouped by tree depth: group d = fine_parents[
   * fine_parent_begin[d] .. fine_parent_begin[d+1]) holds the depth-d
   * parents (device array; fine_parent_begin is a host array inside this
   * struct, fine_parent_begin[0] = 0, non-decreasing up to n_levels_max).
   * With it, each step writes soup records for the surrogates and root
   * triangles only; the fine children of a surrogate are written after the
   * depth at which a pair containing that surrogate survived, so fine
   * triangles that no descent reaches are never touched.  NULL: every
   * triangle is written every step (always so in FLAT mode). */
  const int32_t* fine_parents;
  int32_t fine_parent_begin[DEM_MAX_LEVELS + 1];
  /* Needed by dem_frontier_step only (may be NULL for the other calls):
   * the parent of every triangle (-1 for root triangles) and its depth in its
   * particle's tree (root triangles 0, children one more than their parent). */
  const int32_t* tri_parent;  /* [n_tris] */
  const uint8_t* tri_depth;   /* [n_tris] */
} dem_scene;

/* ------------------------------------------------------------------ parameters */

typedef struct {
  int32_t mode;           /* DEM_MODE_FLAT (Algorithm 2) or DEM_MODE_HIER (Algorithm 5) */
  int32_t n_iter;         /* fixed Newton iteration count N_iterative, 0..8 (paper: 4) */
  float omega;            /* damping of the diagonal-Newton step (1 = undamped) */
  float alpha_reg_rel;    /* alpha_regulariser of a triangle = alpha_reg_rel * (|e1|^2 + |e2|^2) / 2 */
  float alpha_it_ratio;   /* alpha_iterative / alpha_regulariser */
  int32_t init_centroid;  /* 0: start the iteration at (a,b) = 0 as the paper does; 1: at the centroids */
  int32_t dense_distance; /* 1: threshold = +inf, every fine pair is reported with its exact distance */
  int32_t certify;        /* 1: settle a near pair from its iterate snapped to the closest
                             features when the separation bound certifies the distance
                             (FP32: within 4e-6 d + 1e-7 size), else send it to the exact
                             fallback; 0 (default): every near pair takes the exact fallback */
  int32_t prune_exact;    /* dem_frontier_step: 1 = decide "in range" with the exact comparison-based
                             distance (Section 3) instead of the iteration's lower bound; 0 (default) =
                             the iteration, as in dem_find_contacts */
  double energy_k;        /* k of E = k sum max(0, delta - d)^2 (used when dev_energy != NULL) */
  int32_t block;          /* threads per block of the descent / near kernels: 64, 128 or 256 */
  int32_t grid;           /* blocks of the descent and near-pair kernels (0 = 2048, else >= 8; default 1024) */
  int32_t batch_items;    /* work items a block claims at once (1..block; default 128) */
  int32_t flat_tile_i;    /* flat mode: i-triangles per tile (multiple of 64, <= 1024) */
  int32_t flat_tile_j;    /* flat mode: j-triangles staged in LDS per tile (1..64) */
  int32_t seed_chunk;     /* root-pair items are seed_chunk x seed_chunk triangle ranges (1..16; default 8) */
  int32_t frontier_grid;  /* dem_frontier_step: blocks of the per-leaf kernels (0 = 4096; <= 8192) */
  int32_t half_depths;    /* FP32 scenes, HIER mode: the descent at tree depths d < half_depths runs
                             the Newton iteration in half precision (reduced precision on coarse
                             surrogate levels, an extension named in the conclusion, Section 7).
                             The bound along its direction stays FP32 with its rounding slack, so the
                             contact set is unchanged.  0 (default) = off */
  /* Per-depth overrides of grid and batch_items for the descent launches
   * (index = tree depth; 0 = use grid / batch_items).  Depths differ in item
   * count and shape (few large root chunks at depth 0, millions of 4 x 4
   * child products further down), so their best launch shapes differ. */
  int32_t level_grid[DEM_MAX_LEVELS];
  int32_t level_batch[DEM_MAX_LEVELS];
  int64_t queue_capacity; /* items per level queue (>= 8; split into 8 equal segments, one
                             filled per XCD, so allow for uneven fills) */
  int64_t near_capacity;  /* fine pairs the lower bound could not prune (8 segments likewise) */
  /* Optional timing: an array of n_events hipEvent_t (host handles, created
   * by the caller).  events[0] is recorded before the first kernel launch of
   * dem_find_contacts and events[k] right after its k-th launch slot, in
   * order: reset, flatten, seed, then per tree depth d < n_levels_max two
   * slots, the descent at depth d and the lazy flattening of the children of
   * its surviving surrogates (an empty slot when nothing is launched) (HIER),
   * or the flat tile kernel (FLAT), then the certify kernel (if certify) and
   * the exact fallback kernel.  Slots beyond n_events - 1 are not
   * bracketed.  NULL / 0 disables (use that when the
   * call is captured into a graph). */
  void* const* events;
  int32_t n_events;
  /* 1: the whole descent (seeding, every depth, the lazy flattening) runs as
   * one persistent kernel with a device work queue: a grid of co-resident
   * blocks (sized from the kernel's occupancy) claims batches of each
   * depth's items dynamically, stealing across the per-XCD segments, with
   * grid barriers between depths.  Timing slots are then: reset, flatten,
   * descent, certify (if certify), fallback.  0 (default): one launch per
   * depth. */
  int32_t persistent;
  /* Polls a block of the persistent descent makes at a grid barrier before
   * it gives up and sets DEM_DEV_STALLED (0 = about a second's worth). */
  int32_t persistent_spins;
} dem_params;

/* Fill p with the defaults (N_it = 4, HIER mode, exact fallback, no per-depth overrides). */
void dem_default_params(dem_params* p);

/* ------------------------------------------------------------------ outputs */

/* Contacts (device SoA, caller-owned).  Contact c joins global triangles
 * ti[c] (particle pi[c]) and tj[c] (particle pj[c]) at exact distance d[c];
 * x = contact point, n = normal n(c) = p_i - x where p_i, p_j are the closest
 * points and x lies on the segment between them at the centre of the overlap
 * of the two epsilon environments (Section 2: centre of the shortest path
 * for equal eps, shifted by (eps_i - eps_j)/2 otherwise); for d = 0, x = p_i
 * and n = 0.  Order is unspecified.
 *
 * adjoint (optional, NULL = none): [DEM_ADJOINT_ROWS][capacity] values of the
 * scene's precision that the call producing the contacts writes beside
 * them and dem_contact_backward reads instead of solving each pair's
 * closest points again: row 0 delta = eps_i + eps_j; rows 1-3 the unit
 * direction u = (p_j - p_i) / d (0 for d = 0); rows 4-6 the barycentric code
 * of p_i on t_i, rows 7-8 the parameters of p_j on t_j, as
 *   row 4 = code_i + 8 code_j (codes below), rows 5, 6 = a_i, b_i,
 *   rows 7, 8 = a_j, b_j;
 * code 0: weights (1 - a - b, a, b) on the triangle's vertices (v0, v1, v2);
 * code 1..4: the point of a segment with weight a at its second end,
 * segments v0->v1, v1->v2, v2->v0, v0->v2 (a = 0: the first end).  The
 * weights are formed from these codes by the producing kernel itself, so
 * the gradient from stored rows equals the one from a fresh solve bit for
 * bit.  dem_sort_contacts moves the rows with their contacts. */
#define DEM_ADJOINT_ROWS 9
typedef struct {
  int64_t capacity;
  int32_t* pi;
  int32_t* pj;
  int32_t* ti;
  int32_t* tj;
  void* d;          /* [capacity] */
  void* x;          /* [3][capacity] */
  void* n;          /* [3][capacity] */
  uint32_t* count;  /* device scalar: contacts found (may exceed capacity) */
  void* adjoint;    /* [DEM_ADJOINT_ROWS][capacity] or NULL (see above) */
} dem_contacts;

/* Per-call counters (device memory, cleared by dem_find_contacts). */
typedef struct {
  unsigned long long evals[DEM_MAX_LEVELS];     /* triangle-pair evaluations at each depth */
  unsigned long long survivors[DEM_MAX_LEVELS]; /* surrogate pairs not pruned at each depth */
  unsigned long long near;      /* fine pairs the lower bound did not prune */
  unsigned long long certified; /* near pairs whose distance the iterate's bound certified */
  unsigned long long fallback;  /* near pairs sent to the comparison-based distance */
  unsigned long long contacts;  /* contacts found */
  unsigned long long items[DEM_MAX_LEVELS];     /* work items consumed at each depth */
  unsigned long long frontier_leaves;    /* active pairs evaluated by dem_frontier_step */
  unsigned long long frontier_unfolded;  /* active pairs replaced by their child pairs (widening) */
  unsigned long long frontier_collapsed; /* child groups replaced by their parent pair (narrowing) */
  unsigned long long fine_records;       /* triangle records the lazy flattening wrote */
} dem_stats;

/* Bytes of device workspace dem_find_contacts needs for this scene and
 * parameters (soup, level queues, near list, counters).  0 on bad input. */
size_t dem_workspace_bytes(const dem_scene* scene, int32_t n_pairs, const dem_params* p);

/*
 * dem_find_contacts -- all contacts between the candidate particle pairs
 * (Algorithm 2 in DEM_MODE_FLAT, Algorithm 5 in DEM_MODE_HIER; both give
 * the same set, Lemma 1).
 *
 * scene      device arrays as described in dem_scene (host struct).
 * pairs      device [2][n_pairs]: particle ids (pairs[0][k], pairs[1][k]).
 * p          parameters (host); NULL = defaults.
 * out        contact buffers (host struct of device pointers).
 * workspace  device, >= dem_workspace_bytes(scene, n_pairs, p) bytes.
 * dev_stats  device dem_stats or NULL.
 * dev_status device uint32: cleared, then DEM_DEV_* bits.  Every input
 *            vertex is checked: a non-finite coordinate sets
 *            DEM_DEV_NONFINITE (the contacts of such a call are meaningless,
 *            but the call completes).
 * dev_energy device double or NULL: receives k * sum max(0, delta - d)^2
 *            over every contact found, including contacts beyond
 *            out->capacity (DEM_DEV_CONTACT_OVERFLOW): rerun with a larger
 *            capacity before differentiating.
 * stream     hipStream_t to enqueue on.
 */
dem_status dem_find_contacts(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs,
                             const dem_params* p, const dem_contacts* out, void* workspace,
                             size_t workspace_bytes, dem_stats* dev_stats, uint32_t* dev_status,
                             double* dev_energy, dem_stream_t stream);

/*
 * dem_find_contacts_noalloc -- dem_find_contacts for callers that cannot
 * allocate device memory: code under HIP graph capture that may not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, kernels and results as dem_find_contacts, except that the
 * workspace is a library-owned static device array of DEM_SCRATCH_BYTES
 * (one per GPU, allocated when the library's code object is loaded on that
 * device and held until the process ends) instead of a caller buffer.  The
 * call itself allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the caller still passes pairs, contact buffers and status.
 *
 * Returns DEM_ERR_CAPACITY when dem_workspace_bytes(scene, n_pairs, p)
 * exceeds DEM_SCRATCH_BYTES (lower p->queue_capacity / near_capacity or use
 * dem_find_contacts), DEM_ERR_HIP when the scratch address of the current
 * device cannot be looked up (the first call on each device does that
 * lookup; make it outside graph capture), and the argument errors of
 * dem_find_contacts.  The current device must be the device of `stream`.
 *
 * Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents (counters are cleared by the call's first kernel): calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  The triangle soup it leaves is not available to
 * dem_contact_backward: contacts from this call are differentiated through
 * their adjoint rows (out->adjoint set), which need no workspace.
 */
#define DEM_SCRATCH_BYTES (64u << 20)
dem_status dem_find_contacts_noalloc(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs,
                                     const dem_params* p, const dem_contacts* out, dem_stats* dev_stats,
                                     uint32_t* dev_status, double* dev_energy, dem_stream_t stream);

/*
 * dem_contact_backward -- adjoint of the penalty contact energy
 * E = k * sum over contacts of max(0, delta - d)^2 (delta = eps_i + eps_j).
 *
 * With u = (p_j - p_i) / d and barycentric weights w_i, w_j of the closest
 * points, dE/dv = +2k (delta - d) w_i u for the vertices of t_i and
 * -2k (delta - d) w_j u for those of t_j (envelope theorem: d is a minimum
 * over the two triangles).  Intersecting pairs (d = 0) add energy but no
 * gradient.  With contacts->adjoint set, delta, u and the weights come from
 * its rows and d from contacts->d (no triangle data is read); otherwise the
 * closest points are solved again for each contact's triangle pair from
 * the workspace's triangle soup.
 *
 * contacts   the output of the immediately preceding dem_find_contacts (or
 *            dem_frontier_step) on this workspace (device count is read on
 *            device), possibly reordered by dem_sort_contacts.  A contact
 *            naming a triangle outside the scene is skipped and sets
 *            DEM_DEV_BAD_TREE; a contact list from another call reads soup
 *            records (or adjoint rows) that may not belong to it and gives a
 *            meaningless gradient.
 * grad_E     device double scalar multiplying the gradient, or NULL for 1.
 * grad_verts device [3][n_verts] with respect to world positions,
 *            ACCUMULATED into (caller zeroes it); NULL for energy only.
 *            Contributions are first summed per vertex within a block in
 *            64-bit fixed point scaled to the block's largest bound
 *            2k |grad_E| delta (exact sums; each contribution rounded to
 *            2^-29 of that bound in FP32, 2^-52 in FP64), then added to
 *            grad_verts with one FP32/FP64 atomic per vertex and component
 *            (order unspecified).  A contribution above 2^100 or not finite
 *            is left out and sets DEM_DEV_NONFINITE.
 * energy_out device double or NULL: set to E.
 * workspace  without adjoint rows: the workspace of the dem_find_contacts
 *            call that produced `contacts`, unchanged since, with the
 *            scene's verts and pose unchanged: the triangle soup flattened
 *            there is reused.  Needs workspace_bytes >= the soup's end (any
 *            size dem_workspace_bytes returned for this scene suffices).
 *            With contacts->adjoint set it is not read (may be NULL).
 * dev_status device uint32: DEM_DEV_* bits are OR-ed in (not cleared).
 */
dem_status dem_contact_backward(const dem_scene* scene, const dem_contacts* contacts, double k,
                                const double* grad_E, void* grad_verts, double* energy_out,
                                const void* workspace, size_t workspace_bytes,
                                uint32_t* dev_status, dem_stream_t stream);

/*
 * dem_sort_contacts -- a deterministic order for a contact list: contacts
 * sorted by (ti, tj), the global triangle numbers (a contact's triangle pair
 * is unique, so the order is total and the same on every run, whatever order
 * the kernels' atomics produced).  All fields (pi, pj, ti, tj, d, x, n) move
 * together, in place, with the adjoint rows when contacts->adjoint is set;
 * the count is unchanged.  Contacts naming a triangle
 * outside the scene come last in their input order and set DEM_DEV_BAD_TREE.
 * Kernels only (no memset, no host synchronisation): graph-capturable.
 *
 * scene      the scene the contacts refer to (its n_tris sizes the buckets).
 * contacts   device SoA as written by dem_find_contacts or dem_frontier_step;
 *            the first min(*count, capacity) entries are sorted.
 * workspace  device, >= dem_sort_contacts_workspace_bytes(scene, capacity)
 *            bytes, 256-byte aligned; scratch only.
 * dev_status device uint32: DEM_DEV_* bits are OR-ed in (not cleared).
 * Cost: O(n_tris + count) plus an insertion sort within each t_i bucket.
 */
size_t dem_sort_contacts_workspace_bytes(const dem_scene* scene, int64_t contact_capacity);
dem_status dem_sort_contacts(const dem_scene* scene, const dem_contacts* contacts, void* workspace,
                             size_t workspace_bytes, uint32_t* dev_status, dem_stream_t stream);

/* ------------------------------------------------------------------ frontier */

/*
 * Persistent active sets (Section 5.3: the multiscale Picard scheme of
 * Algorithm 6, which keeps an active set per particle pair between Picard
 * iterations and time steps, unfolds at most one tree level per iteration,
 * widens and narrows the sets, and vetoes repeated removals with a memory set
 * U).  Pairwise form, as in dem_find_contacts: the active set of a candidate
 * particle pair is a set of triangle pairs ("leaves") that covers every pair
 * of its fine triangles exactly once.
 *
 * Leaf record (four int32): {t_i, t_j, flags, info}
 *   t_i, t_j  global triangle ids (particles pairs[0][k], pairs[1][k]);
 *   flags     bit 0: the pair is in the memory set (its child pairs were once
 *             replaced by it); bit d (1..31): the pair's ancestor at depth
 *             d-1 is in the memory set, so the sibling group at depth d may
 *             not be narrowed;
 *   info      bits 0-7 index in the sibling group, 8-16 group size (0 for
 *             root pairs), 17-21 pair depth D (steps of unfolding from the
 *             root pair), bit 22/23: side i/j was unfolded to reach depth D.
 * The leaves of a buffer are in depth-first order: the root pairs of
 * candidate pair 0 (t_i-major), their descendants in place, then pair 1, ...
 * so every sibling group whose members are all leaves is contiguous.
 */
typedef struct {
  int64_t capacity;        /* leaves each buffer holds (< 2^32) */
  int32_t* leaves[2];      /* two device buffers of [capacity][4] leaf records */
  uint32_t* state;         /* device [4]: {buffer holding the active sets (0/1), leaf count,
                              leaves the last call needed, 0} */
  int64_t memory_capacity; /* slots of the memory set: a power of two >= 64 */
  uint64_t* memory;        /* device [memory_capacity]: hash set of pairs (t_i << 32 | t_j) */
} dem_frontier;

/* Bytes of device workspace dem_frontier_init / dem_frontier_step need
 * (triangle soup, near list, per-leaf outcome words, scan partials,
 * counters).  The step's soup sits where dem_contact_backward reads it, so
 * the workspace also serves the backward pass of the step's contacts.
 * 0 on bad input. */
size_t dem_frontier_workspace_bytes(const dem_scene* scene, int32_t n_pairs, const dem_params* p,
                                    int64_t frontier_capacity);

/*
 * dem_frontier_init -- active sets = all root-triangle pairs of every
 * candidate pair (Algorithm 6, initial statement); clears the memory set.
 *
 * pairs      device [2][n_pairs] particle ids, as for dem_find_contacts; a
 *            leaf's candidate pair is not stored, so the same pairs in the
 *            same order are expected for as long as the active sets are kept.
 * p          the parameters the steps will use (NULL = defaults).
 * f          host struct of device pointers (see dem_frontier).
 * workspace  >= dem_frontier_workspace_bytes(scene, n_pairs, p, f->capacity).
 * dev_status device uint32: cleared, then DEM_DEV_FRONTIER_OVERFLOW if the
 *            root pairs exceed f->capacity (state then holds 0 leaves and
 *            the number needed).
 */
dem_status dem_frontier_init(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs,
                             const dem_params* p, const dem_frontier* f, void* workspace,
                             size_t workspace_bytes, uint32_t* dev_status, dem_stream_t stream);

/*
 * dem_frontier_step -- one Picard iteration's contact detection on the
 * active sets at the scene's current positions.
 *
 * Every leaf is evaluated once (the iteration's lower bound, or the exact
 * distance if p->prune_exact):
 *   - out of range (d > eps_i + eps_j certainly): "no contact";
 *   - two fine triangles in range: settled by the exact comparison-based
 *     distance and reported in `out` if d <= eps_i + eps_j (else "no
 *     contact");
 *   - a surrogate in range: replaced by its child pairs (only the non-fine
 *     side unfolds), one level per call (widening).
 * A sibling group whose members are all leaves and all "no contact" is
 * replaced by its parent pair, which enters the memory set, unless the
 * parent already is in it (narrowing with the veto of the memory set).
 * If nothing widens or narrows, the active sets stay where they are;
 * otherwise the rewritten sets go to the other buffer and state[0] flips.
 *
 * scene      as for dem_find_contacts, with tri_parent and tri_depth set.
 * p          parameters (mode is ignored); NULL = defaults.
 * out, dev_energy  as for dem_find_contacts (this call's contacts).
 * dev_stats  evals[] counts leaves by pair depth; frontier_* counters.
 * dev_status cleared, then DEM_DEV_* bits.  On DEM_DEV_FRONTIER_OVERFLOW
 *            the active sets are left unchanged and state[2] holds the
 *            leaf count the rewrite needed.
 * The contacts can be differentiated with dem_contact_backward on this
 * call's workspace.
 */
dem_status dem_frontier_step(const dem_scene* scene, const dem_params* p, const dem_frontier* f,
                             const dem_contacts* out, void* workspace, size_t workspace_bytes,
                             dem_stats* dev_stats, uint32_t* dev_status, double* dev_energy,
                             dem_stream_t stream);

/* ------------------------------------------------------------------ forces */

/*
 * Merged contact points and their forces (Section 2: force of a contact
 * point; implementation note on redundant contact points).  Device SoA,
 * caller-owned.  Merged contact m joins particles pi[m] and pj[m]; x is the
 * mean of its group's contact points, n the mean of their normals n(c), f the
 * force on pi[m] (pj[m] receives -f).  Order is unspecified.
 */
typedef struct {
  int64_t capacity;
  int32_t* pi;        /* [capacity] */
  int32_t* pj;        /* [capacity] */
  void* x;            /* [3][capacity] */
  void* n;            /* [3][capacity] */
  void* f;            /* [3][capacity] */
  int32_t* members;   /* [capacity] contacts merged into it */
  uint32_t* count;    /* device scalar: merged contacts (may exceed capacity) */
} dem_merged;

/* Bytes of device workspace dem_contact_forces needs for contact lists of
 * up to contact_capacity entries (hash of cells, links, group sums).  0 on
 * bad input. */
size_t dem_contact_forces_workspace_bytes(int64_t contact_capacity);

/*
 * dem_contact_forces -- merge redundant contact points and apply the force
 * law to every merged point.
 *
 * Merging (implementation note of Section 2: points closer than eps become
 * one average point): two contact points of the same particle pair whose
 * distance is below merge_scale * (eps_i + eps_j) / 2 are in the same group,
 * transitively; a group becomes one merged contact at the mean point with
 * the mean normal.  merge_scale = 1 is the paper's rule; 0 keeps every
 * contact on its own.
 * Force (Section 2): F = n/|n| K_s (1 - |n|/eps_i) sqrt(1/(1/M_i + 1/M_j))
 * on p_i and -F on p_j, with n the merged normal; n = 0 (intersecting
 * triangles) gives no force.  Torque about the given centres:
 * (x - centre) x force.
 *
 * contacts   the output of dem_find_contacts or dem_frontier_step (its device
 *            count is read on the device).
 * mass       device [n_particles], centre device [3][n_particles] (scene
 *            precision).
 * out        merged contacts; overflow sets DEM_DEV_CONTACT_OVERFLOW.
 * group      device [contacts->capacity] or NULL: merged index of every input
 *            contact.
 * force, torque  device [3][n_particles] or NULL, ACCUMULATED into (caller
 *            zeroes them).
 * dev_status DEM_DEV_* bits are OR-ed in (not cleared); a full cell hash or a
 *            merge that does not settle within its step bound sets
 *            DEM_DEV_QUEUE_OVERFLOW.
 */
dem_status dem_contact_forces(const dem_scene* scene, const dem_contacts* contacts, const void* mass,
                              const void* centre, double k_s, double merge_scale, const dem_merged* out,
                              int32_t* group, void* force, void* torque, void* workspace,
                              size_t workspace_bytes, uint32_t* dev_status, dem_stream_t stream);

const char* dem_status_string(dem_status s);

/* Library version string ("dem <major>.<minor> gfx950"). */
const char* dem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DEM_H_ */
