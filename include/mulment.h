/*
 * mulment: multilevel maxent-stress graph layout on one MI355X (gfx950).
 *
 * C-ABI of libmulment.so.  Plain pointers and sizes only.  Every call returns
 * an mm_status; on failure the outputs are left untouched and
 * mm_last_error() describes the failure (thread-local, valid until the next
 * call on the same thread).  No exception or abort crosses this boundary.
 *
 * Memory.  Unless a parameter says "host", pointers are device pointers
 * (HBM) and are used in place on the context's HIP stream; the caller owns
 * them and keeps them alive until mm_sync() returns.  Objects the library
 * allocates (mm_khop, mm_coarse) are released with their *_free call.
 * A context is bound to one device and one stream and is not thread-safe;
 * separate contexts are independent.
 *
 * Graphs are undirected simple graphs (Preliminaries, "Basic Concepts"):
 * CSR with int32 row_ptr[n+1] and col[nnz], both directions stored, rows
 * strictly ascending, no self-loops; node weights c >= 1 and edge weights
 * w >= 1 (NULL = all 1, the paper's default inputs).
 */
#ifndef MULMENT_H
#define MULMENT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_EINVAL = 1,       /* invalid argument or malformed graph */
  MM_ENOMEM = 2,       /* device allocation failed */
  MM_EDEVICE = 3,      /* HIP runtime / kernel error */
  MM_EUNSUPPORTED = 4, /* valid request outside the implemented range */
  MM_EINTERNAL = 5
} mm_status;

typedef enum { MM_HOST = 0, MM_DEVICE = 1 } mm_mem;

typedef struct mm_context mm_context;
typedef struct mm_khop mm_khop;
typedef struct mm_coarse mm_coarse;

typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t* row_ptr; /* n+1 */
  const int32_t* col;     /* nnz */
  const int32_t* node_w;  /* n, or NULL (all 1) */
  const int32_t* edge_w;  /* nnz, or NULL (all 1) */
  int32_t mem;            /* mm_mem: where the four arrays live */
} mm_graph;

/* Layout parameters.  mm_params_default() gives the paper's configuration
 * (Section 4, "Algorithm Configuration"; Section 3.2 for the alpha decay). */
typedef struct {
  int32_t k;               /* stress set S = pairs within k hops (1 = edges, Eq. 1) */
  double q;                /* entropy exponent: r_q = (x_u-x_v)/|x_u-x_v|^(q+2); 0 = ln */
  double theta;            /* Barnes-Hut opening angle; < 0 = exact all-pairs far field */
  double alpha0;           /* initial entropy weight (1) */
  double alpha_decay;      /* alpha := decay * alpha per round (0.3) */
  double alpha_min;        /* final alpha (0.008) */
  int32_t iters_per_round; /* a: iterations per alpha round (2) */
  double eps_round;        /* early alpha drop when relative change < eps_round (1e-4) */
  double eps_final;        /* stop at alpha_min when relative change < eps_final (1e-4) */
  int32_t max_final_iters; /* cap on iterations at alpha_min (200) */
  int32_t max_levels;      /* max number of contractions (62) */
  int32_t coarsest_n;      /* stop coarsening at <= this many vertices (2) */
  double b, f;             /* W = min(b^h, |V|/f) (2, 20) */
  int32_t lp_rounds;       /* label-propagation rounds per level (10) */
  double coarse_dist_scale;/* d = hop (sqrt c_u + sqrt c_v) scale on coarse levels (1) */
  uint64_t seed;
  int32_t validate;        /* 1: full host-side graph validation (default) */
  const float* mlp_weights;/* device, MM_MLP_PARAMS floats: learned far-field correction
                              (Barnes-Hut only, q = 0); NULL = plain Barnes-Hut (default) */
  int32_t use_graphs;      /* 1: replay the iterations of levels with <= 2^18 vertices from
                              HIP graphs (default; same results, fewer launches); 0: direct */
  int32_t autotune;        /* 1: pick each level's sweep kernel, tile size and lanes per row
                              or chunk by timing the candidates on the level itself, once per
                              level shape, and keep the choice in the context (later layouts
                              reuse it, so their results are reproducible); 0: fixed rules
                              (default) */
  int32_t exact_below;     /* levels with at most this many vertices use the exact all-pairs
                              far field instead of Barnes-Hut (0 = none, default); mm_layout
                              only (mm_layout_batch requires 0) */
  int32_t approx_h;        /* h > 0: MulMent_h, the cluster far field of Eq. 3 with the graph
                              h levels beneath (else the coarsest) on every level that has a
                              coarser one, replacing theta / exact_below / mlp_weights there
                              (the coarsest level keeps those); 0 = off (default).  Needs the
                              hierarchy: ignored with init_xy; mm_layout only */
  int32_t khop_direct;     /* 1 (default): on levels swept tile-major with k = 2, rows whose
                              2-hop search used a bitmap are copied to the tile-major layout
                              straight from that bitmap, without writing their canonical ids
                              (same layout, bit for bit); 0: always via the canonical ids.
                              mm_layout only */
} mm_params;

#define MM_MAX_LEVELS 64
typedef struct {
  int32_t levels;                        /* graphs in the hierarchy incl. the input */
  int32_t level_n[MM_MAX_LEVELS];
  int64_t level_nnz[MM_MAX_LEVELS];
  int64_t level_khop[MM_MAX_LEVELS];     /* sum |S(u)| */
  int32_t level_iters[MM_MAX_LEVELS];
  int32_t level_final_iters[MM_MAX_LEVELS];
  int32_t level_cap_hit[MM_MAX_LEVELS];  /* final phase stopped by max_final_iters */
  double level_delta[MM_MAX_LEVELS];     /* last relative change */
  double level_sweep_ms[MM_MAX_LEVELS];  /* summed HIP-event time of the sweep launches */
  double level_far_ms[MM_MAX_LEVELS];    /* summed HIP-event time of the far-field launches */
  double level_khop_ms[MM_MAX_LEVELS];   /* wall time of the k-hop build */
  double t_total_ms, t_coarsen_ms, t_khop_ms, t_farfield_ms, t_sweep_ms, t_other_ms;
  int64_t vertex_updates;                /* sum over levels of n * iterations */
  int64_t finest_updates;                /* n_0 * iterations on the input graph */
  int32_t level_tile_bits[MM_MAX_LEVELS];/* sweep of the level: tile size 2^bits (0 = row kernel) */
  int32_t level_group[MM_MAX_LEVELS];    /* lanes per chunk (tiled) or per row (row kernel) */
  double t_tune_ms;                      /* time spent timing candidates (autotune) */
  int32_t level_blocks[MM_MAX_LEVELS];   /* tiled sweep: 16-byte entry blocks per lane and step */
  /* The far field runs on a second stream, concurrently with the part of the
   * sweep that does not read it, so the far-field and sweep times above
   * overlap; these are the elapsed times of the iterations themselves. */
  double t_iterate_ms;                   /* all iterations of all levels */
  double level_wall_ms[MM_MAX_LEVELS];   /* iterations of the level */
} mm_stats;

mm_status mm_params_default(mm_params* p);

/* device: HIP device ordinal; stream: hipStream_t or NULL (default stream).
 * The library allocates its buffers stream-ordered from the device's default
 * memory pool and raises that pool's release threshold, so memory it frees
 * stays mapped for its next allocations; mm_context_destroy trims the pool. */
mm_status mm_context_create(mm_context** out, int32_t device, void* stream);
void mm_context_destroy(mm_context* ctx);
/* Forgets the sweep configurations the autotuner chose in this context. */
mm_status mm_tune_clear(mm_context* ctx);
/* The autotuner's choices as records of MM_TUNE_FIELDS int64 each:
 * (coarse level?, n, sum |S(u)|, k, tile bits (0 = row kernel), lanes,
 * blocks per lane and step (tiled: 2 or 4; row kernel: 0)).
 * mm_tune_export writes at most cap records to recs (host) and the number
 * the context holds to *count (so cap = 0 asks for the size).
 * mm_tune_import adds or replaces count records; a record whose tile bits
 * are not 0 or 11..13, whose lanes are not a power of two in 1..64 (8..64 for
 * the row kernel, 1..16 tiled), or whose blocks are not 0 (row kernel) or
 * 0, 2, 4 (tiled; 0 = the default rule) is rejected with MM_EINVAL and
 * nothing is imported.  Used to keep a tuned
 * configuration across processes. */
#define MM_TUNE_FIELDS 7
mm_status mm_tune_export(mm_context* ctx, int64_t* recs, int32_t cap, int32_t* count);
mm_status mm_tune_import(mm_context* ctx, const int64_t* recs, int32_t count);
/* Waits for the context's stream; reports asynchronous device errors. */
mm_status mm_sync(mm_context* ctx);
const char* mm_last_error(void);

/* Full multilevel layout (Section 3): coarsening, initial layout,
 * prolongation and local improvement on every level.  init_xy (n*2,
 * interleaved, same memory kind as the graph, or NULL): when given, the
 * hierarchy is skipped and only the finest level is iterated starting at
 * alpha_min (the warm start of the dynamic-graph update).  out_xy: n*2 in
 * the graph's memory kind.  stats: host, may be NULL. */
mm_status mm_layout(mm_context* ctx, const mm_graph* g, const mm_params* p,
                    const float* init_xy, float* out_xy, mm_stats* stats);

/* Batched layout of G independent graphs (an extension: the paper lays out
 * one graph at a time).  g is their block-diagonal union: graph i owns the
 * vertices [graph_off[i], graph_off[i+1]) (graph_off: host, G+1, from 0 to
 * n; every graph has >= 2 vertices and no edge leaves its graph).  Every
 * graph is laid out as mm_layout would lay it out alone -- its own
 * hierarchy (U, f, stopping point), draws keyed by its local vertex ids,
 * its own quadtree and alpha schedule -- while each step runs as one set of
 * launches over the whole batch.  theta >= 0 (Barnes-Hut) only; no learned
 * far field.  init_xy (n*2 or NULL): warm start of every graph as in
 * mm_layout.  out_xy: n*2 in the graph's memory kind.  graph_levels (host,
 * G, may be NULL): levels of each graph's hierarchy.  stats: per union
 * level sizes, the iterations of its longest-running graph
 * (level_iters, level_final_iters), the number of its graphs stopped by
 * max_final_iters (level_cap_hit), the sweep configuration, and totals
 * (vertex_updates counts each graph's own iterations).  Each graph's alpha
 * schedule and stop run on the device; the host checks the number of
 * running graphs once per replay of several captured iterations (iterations
 * after a graph's stop leave its coordinates unchanged). */
mm_status mm_layout_batch(mm_context* ctx, int32_t G, const int64_t* graph_off, const mm_graph* g,
                          const mm_params* p, const float* init_xy, float* out_xy,
                          int32_t* graph_levels, mm_stats* stats);

/* ---- step-level entry points (device graphs) ---------------------------- */

/* k-hop distance sets S_k(u) = {v != u : hop(u,v) <= k}, sorted by (hop, v)
 * (stress superset S of the general model, footnote to Eq. 1).  g must be
 * MM_DEVICE.  Row offsets int64 off[n+1]; hend[u*k + h-1] = entries of row u
 * with hop <= h; ids int32. */
mm_status mm_khop_build(mm_context* ctx, const mm_graph* g, int32_t k, mm_khop** out);
void mm_khop_free(mm_khop* kh);
/* host: n, k, total entries */
mm_status mm_khop_info(const mm_khop* kh, int32_t* n, int32_t* k, int64_t* total);
/* device pointers of the sets (valid until mm_khop_free) */
mm_status mm_khop_arrays(const mm_khop* kh, const int64_t** off, const int32_t** hend,
                         const int32_t** nbr);
/* copy the sets into caller buffers (off n+1, hend n*k, nbr total) of kind mem */
mm_status mm_khop_export(mm_context* ctx, const mm_khop* kh, int64_t* off, int32_t* hend,
                         int32_t* nbr, int32_t mem);

/* General stress sets (the footnote to Eq. 1: any S ⊇ E, each pair with its
 * target distance d_uv).  The caller's arrays use the layout of the k-hop
 * sets above: row offsets off[n+1] (off[0] = 0, non-decreasing, total =
 * off[n]); hend[u*k + h-1] = entries of row u with d_uv <= h, for integer
 * distances h in 1..k (k in [1, 8]); nbr[total] ids, strictly increasing
 * inside each distance group; no row is empty (Eq. 2 divides by rho_u, the
 * sum of its weights).  S is a set of unordered pairs: an entry v at
 * distance h in row u needs u at distance h in row v.  No id repeats in a
 * row, none equals its row, all lie in [0, n).  That S contains E is the
 * caller's model choice and is not checked (no graph is passed).
 *
 * mm_khop_validate checks host arrays only (no device work, no context):
 * MM_OK, or MM_EINVAL naming the first violation (mm_last_error).
 * mm_khop_import copies the arrays (kind mem: MM_HOST or MM_DEVICE; device
 * arrays are read back to the host for the same checks) into a new set that
 * mm_sweep, mm_sweep_ex, mm_sweep_cfg, mm_objective and the mm_khop_*
 * queries accept like a built one; the caller keeps ownership of its
 * arrays.  Errors: MM_EINVAL as above, MM_ENOMEM. */
mm_status mm_khop_validate(int32_t n, int32_t k, const int64_t* off, const int32_t* hend,
                           const int32_t* nbr);
mm_status mm_khop_import(mm_context* ctx, int32_t n, int32_t k, const int64_t* off,
                         const int32_t* hend, const int32_t* nbr, int32_t mem, mm_khop** out);

/* Far field F_u = sum_{v != u} r_q(u,v) (the entropy term of Eq. 2 before
 * removing S).  theta < 0: exact all-pairs; theta >= 0: Barnes-Hut quadtree.
 * xy, F: n*2 FP32 device.  codes (n, Morton codes in id order), order (n,
 * ids sorted by (code, id)), nodes (5 int64 per node, pre-order: depth,
 * first sorted index, count, is_leaf, prefix) are optional device outputs
 * (Barnes-Hut only; nodes needs room for 2n entries); counters (host, 4
 * int64: accepted cells, exact leaf pairs, reserved, node count) optional. */
mm_status mm_repulsion(mm_context* ctx, int32_t n, const float* xy, double q, double theta,
                       float* F, uint64_t* codes, int32_t* order, int64_t* nodes,
                       int64_t* counters);

/* Cluster far field, the first two sums of Eq. 3 (Section 3.2, "Faster Local
 * Improvement"; MulMent_h): for each u,
 *   F_u = sum_{v != u, cluster1[v] == cluster1[u]} r_q(u,v)
 *       + sum_{j != cluster_h[u]} nu_j r_q(x_u, xp_j),
 * nu_j = #{v : cluster_h[v] == j}, xp_j = node-weighted midpoint of those v
 * (node_w NULL: weights 1).  cluster1 (n values in [0, n1)) maps to the next
 * coarser level, cluster_h (n values in [0, nh)) to the level used for the
 * approximation; vertices sharing u's cluster_h value but not its cluster1
 * value contribute nothing (the merged-vertex error of that section).  With
 * both maps the identity this is the exact sum.  All arrays are device
 * arrays; xy, F are n*2 FP32.  Out-of-range cluster ids are MM_EINVAL.
 * Synchronous on the context's stream. */
mm_status mm_repulsion_cluster(mm_context* ctx, int32_t n, const float* xy, const int32_t* node_w,
                               const int32_t* cluster1, int32_t n1, const int32_t* cluster_h,
                               int32_t nh, double q, float* F);

/* ---- learned far-field correction (an extension; the paper has none) ----
 * Barnes-Hut as in mm_repulsion (q = 0) where every accepted cell C adds,
 * besides m r(x_u - com), the correction kappa (h0 e + h1 p): d = |x_u - com|,
 * e = (x_u - com)/d, p = (-e_y, e_x), t = s/d with s the side of C's tight
 * cell, kappa = m t^2/d, h = MLP(f).  Features f (8): t; offset of com from
 * the cell centre along e and p, over s; central second moments per unit
 * mass rotated into (e, p) (ee, pp, ep), over s^2; log2(m)/16; 0.
 * MLP: h = W3 relu(W2 relu(W1 f + b1) + b2) + b3, W1 64x8, W2 64x64, W3 2x64
 * row-major; weights packed W1, b1, W2, b2, W3, b3 as MM_MLP_PARAMS FP32
 * values.  Evaluated with BF16 weights and activations and FP32
 * accumulation.  All pointers are device pointers; the calls are
 * synchronous on the context's stream. */
#define MM_MLP_PARAMS 4866

/* F (n*2) from xy (n*2) with the correction of `weights`.  theta >= 0. */
mm_status mm_repulsion_learned(mm_context* ctx, int32_t n, const float* xy, double theta,
                               const float* weights, float* F);

/* Training samples: every (u, C) the traversal at theta accepts, in
 * ascending Morton rank of u and visit order within u.  Per sample: u,
 * node (pre-order index of C), feat (8), target = exact residual
 * R = sum_{v in C} r(x_u - x_v) - m r(x_u - com) in h units,
 * ((R.e)/kappa, (R.p)/kappa) (2, computed in FP64), coef = kappa e (2).
 * At most cap samples are written; *count (host) receives the total, so
 * cap = 0 counts only. */
mm_status mm_far_samples(mm_context* ctx, int32_t n, const float* xy, double theta, int64_t cap,
                         int32_t* u_out, int32_t* node_out, float* feat, float* target,
                         float* coef, int64_t* count);

/* Initial weights for mm_mlp_train: W1 ~ N(0, 2/8) and W2 ~ N(0, 2/64)
 * (He), W3 ~ N(0, (out_scale/8)^2), zero biases; normal draws by the
 * Box-Muller transform of SplitMix64 draws 2p and 2p+1 of stream (seed, level
 * 0, tag 65) for parameter p.  weights: MM_MLP_PARAMS floats (device). */
mm_status mm_mlp_init(mm_context* ctx, uint64_t seed, double out_scale, float* weights);

/* h = MLP(feat) for count rows (feat count*8, out count*2). */
mm_status mm_mlp_forward(mm_context* ctx, int64_t count, const float* feat, const float* weights,
                         float* out);

/* Loss L = 1/(2 count) sum_rows |h - target|^2 and its gradient
 * (grad: MM_MLP_PARAMS floats, packed like the weights; loss: 1 float). */
mm_status mm_mlp_grad(mm_context* ctx, int64_t count, const float* feat, const float* target,
                      const float* weights, float* grad, float* loss);

/* `steps` Adam steps (beta 0.9/0.999, eps 1e-8, bias-corrected, step
 * numbers step0+1 ...) on minibatches of `batch` rows drawn with replacement
 * (SplitMix64 keyed by seed and step) from the count samples.  weights
 * (FP32, updated in place); adam: 2*MM_MLP_PARAMS floats of moment state
 * (zero before the first step); losses (steps floats, may be NULL): the
 * minibatch loss before each step. */
mm_status mm_mlp_train(mm_context* ctx, int64_t count, const float* feat, const float* target,
                       float* weights, float* adam, int32_t steps, int32_t batch, double lr,
                       uint64_t seed, int32_t step0, float* losses);

/* One Jacobi iteration of Eq. 2 at entropy weight alpha: xy_out from xy_in
 * only.  level 0: d = hop; level > 0: d = hop (sqrt c_u + sqrt c_v) scale
 * with c = node_w (device, n; NULL = 1).  F: far field from mm_repulsion.
 * delta (host, 2 doubles, may be NULL): |x'-x|^2 and |x|^2. */
mm_status mm_sweep(mm_context* ctx, const mm_khop* kh, int32_t level, const int32_t* node_w,
                   double scale, const float* xy_in, const float* F, double alpha, double q,
                   float* xy_out, double* delta);

/* mm_sweep without any device allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernel and result (bit
 * for bit) as mm_sweep.  Its temporaries -- the per-work-group partial sums,
 * the two relative-change sums and, on levels > 0, sqrt of the node weights
 * -- live in a fixed device array of the library (about 8 MiB), one copy per
 * device, held until the process ends; nothing in it needs to start at zero,
 * since every call writes what it reads.  The sets must have at most
 * MM_SWEEP_NOALLOC_MAX_N vertices, else MM_EINVAL (nothing is launched).
 * All calls on one device share that device's array: calls that overlap on
 * one device (several streams, contexts or host threads) race and must be
 * serialised by the caller.  MM_EDEVICE if the array's address could not be
 * looked up when the context was created. */
#define MM_SWEEP_NOALLOC_MAX_N (1 << 20)
mm_status mm_sweep_noalloc(mm_context* ctx, const mm_khop* kh, int32_t level,
                           const int32_t* node_w, double scale, const float* xy_in,
                           const float* F, double alpha, double q, float* xy_out, double* delta);

/* Kernel choice for mm_sweep_ex.  Both compute the same update.
 * MM_SWEEP_ROWS: a group of lanes per row gathers x_v from HBM/L2.
 * MM_SWEEP_TILED: the sets are re-laid tile-major (tiles of 8192 vertices,
 * 16-bit entries) and each workgroup stages one tile's coordinates in LDS;
 * needs k <= 7 and n <= 2^25 (else MM_EUNSUPPORTED).  The tile-major copy is
 * built on first use and cached in the mm_khop.
 * MM_SWEEP_AUTO: tiled when supported and the mean (row, tile) chunk has at
 * least 8 entries, rows otherwise (what mm_layout does on every level). */
enum { MM_SWEEP_AUTO = 0, MM_SWEEP_ROWS = 1, MM_SWEEP_TILED = 2 };
mm_status mm_sweep_ex(mm_context* ctx, mm_khop* kh, int32_t level, const int32_t* node_w,
                      double scale, const float* xy_in, const float* F, double alpha, double q,
                      float* xy_out, double* delta, int32_t mode);
/* As mm_sweep_ex with the configuration forced, the way the autotuner runs
 * its candidates: tile_bits = 0 runs the row kernel with group lanes per row
 * (8, 16, 32 or 64; blocks must be 0); tile_bits = 11, 12 or 13 runs the
 * tiled kernel with tiles of 2^tile_bits vertices, group lanes per chunk (1,
 * 2, 4, 8 or 16) and blocks 16-byte entry blocks per lane and step (2 or 4; 0 = the
 * default rule).  Any other combination is MM_EINVAL; tiled configurations the sets do not allow (k > 7, too
 * many tiles) are MM_EUNSUPPORTED.  The update is the same for every
 * configuration up to the order of FP32 summation. */
mm_status mm_sweep_cfg(mm_context* ctx, mm_khop* kh, int32_t level, const int32_t* node_w,
                       double scale, const float* xy_in, const float* F, double alpha, double q,
                       float* xy_out, double* delta, int32_t tile_bits, int32_t group,
                       int32_t blocks);

/* One coarsening step (Section 3.1): size-constrained label propagation with
 * bound U at hierarchy level level_h, then contraction.  cluster (device, n)
 * receives the coarse vertex of every vertex; *out the coarse graph
 * (device arrays owned by the library).  rounds_run / moves (host) optional. */
mm_status mm_coarsen(mm_context* ctx, const mm_graph* g, double U, int32_t lp_rounds,
                     uint64_t seed, int32_t level_h, int32_t* cluster, mm_coarse** out,
                     int32_t* rounds_run, int64_t* moves);
/* view of a coarse graph (device arrays, node_w and edge_w always set) */
mm_status mm_coarse_graph(const mm_coarse* cg, mm_graph* view);
/* copy the coarse graph into caller buffers (n+1, nnz, n, nnz) of kind mem */
mm_status mm_coarse_export(mm_context* ctx, const mm_coarse* cg, int32_t* row_ptr, int32_t* col,
                           int32_t* node_w, int32_t* edge_w, int32_t mem);
void mm_coarse_free(mm_coarse* cg);

/* Initial layout of the coarsest graph (replaces the placement of Section
 * 3.1, "Initial Layout", whose coarsest graph has two vertices at their
 * optimal distance): x_v uniform in [0,1)^2, coordinate j of vertex v from
 * the top 24 bits of SplitMix64 draw 2v+j of stream (seed, level, tag 1), so
 * every value is exact in FP32.  mm_layout applies the two-vertex optimum
 * itself when the coarsest graph has exactly two vertices.  xy: n*2 device. */
mm_status mm_init_layout(mm_context* ctx, int32_t n, uint64_t seed, int32_t level, float* xy);

/* Prolongation (Section 3.2): fine v placed uniformly in angle and radius
 * around coarse_xy[cluster[v]] within sqrt(coarse_w). */
mm_status mm_prolong(mm_context* ctx, int32_t n_fine, const int32_t* cluster,
                     const int32_t* coarse_w, const float* coarse_xy, uint64_t seed,
                     int32_t level, float* fine_xy);

/* Maxent-stress of Eq. 1 over the stress set S of kh at entropy weight
 * alpha: out (host, 4) = {M_S = stress - alpha * entropy, stress = sum over
 * unordered pairs of S of w (|x_u - x_v| - d_uv)^2, entropy = sum over the
 * other pairs u < v of ln |x_u - x_v| (q = 0; -|x_u - x_v|^-q / q otherwise),
 * coincident pairs (distance 0, left out of the entropy sum)}.  Target
 * distances as in mm_sweep (level, node_w, scale).  The paper's metric M_E is
 * the same call on the k = 1 sets (S = E); the full stress at the optimal
 * scale s* (Section 4, "Methodology") is mm_full_stress.  Sums in FP64. */
mm_status mm_objective(mm_context* ctx, const mm_khop* kh, int32_t level, const int32_t* node_w,
                       double scale, const float* xy, double alpha, double q, double* out);

/* Full stress over all connected pairs with hop distances (Section 4):
 * out (host, 3) = {F(x), s*, F(s* x)}; the graph in device memory.  Hop
 * distances come from breadth-first searches on the GPU: one search per
 * source for n <= 65536; above, a bit-parallel search of 256 sources at a
 * time over all vertices when the graph's diameter is low (the first 256
 * sources finish within 64 levels), otherwise the banded search: vertices
 * renumbered in Morton order of xy, 64 neighbouring sources per search, each
 * level visiting only the 64-vertex tiles next to the vertices reached at
 * the level before (n <= 2^23, else MM_EUNSUPPORTED).  Fast when the layout
 * roughly follows graph distances; correct for any xy.  Every method sums in
 * a fixed order (bit-identical reruns). */
mm_status mm_full_stress(mm_context* ctx, const mm_graph* g, const float* xy, double* out);
/* As mm_full_stress with the method chosen: 0 as above, 1 the multi-source
 * search over all vertices (any n and diameter), 2 one search per source
 * (n <= 1179648), 3 the banded search (n <= 2^23).  The results agree up to
 * the order of the FP64 sums. */
mm_status mm_full_stress_ex(mm_context* ctx, const mm_graph* g, const float* xy, int32_t method,
                            double* out);

#ifdef __cplusplus
}
#endif
#endif
