/*
 * FP64 CPU oracle for multilevel maxent-stress layout.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain restatement of
 * the method against which the GPU library is checked.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it.  It shares no code with the GPU library.
 *
 * Everything is double precision, every per-vertex loop is independent, and
 * every reduction is summed in ascending vertex (then neighbour) order, so
 * results do not depend on the OpenMP thread count.
 *
 * Readings of points the paper leaves open are listed beside each function.
 */
#ifndef MM_ORACLE_H
#define MM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based random numbers ------------------------------------
 * SplitMix64 (Steele, Lea, Flood 2014): the i-th output (0-based) of the
 * generator whose state starts at s is mix(s + (i+1)*0x9E3779B97F4A7C15).
 * A stream is selected by seed ^ (level << 48) ^ (tag << 32).
 * Tags: 1 initial layout (i = 2v + j), 2 prolongation (i = 2v + j),
 *       16 + r label-propagation round r (i = v, colour = bit 0).
 * A unit draw is (r >> 40) * 2^-24, exactly representable in FP32. */
uint64_t orc_splitmix64_at(uint64_t state, uint64_t i);
uint64_t orc_stream(uint64_t seed, uint32_t level, uint32_t tag);
void orc_draws(uint64_t seed, uint32_t level, uint32_t tag, uint64_t i0,
               int64_t count, uint64_t* out);

/* ---- execution ----------------------------------------------------------
 * Threads of the oracle's OpenMP loops from now on (n >= 1); returns the
 * previous maximum.  Results do not depend on it (fixed-order sums). */
int orc_set_threads(int n);

/* ---- input validation (Preliminaries: undirected simple graph, c, w) --
 * 0 ok, 1 n < 2, 2 bad row_ptr, 3 column out of range, 4 self-loop,
 * 5 row not strictly ascending (duplicate), 6 asymmetric edge or weight,
 * 7 isolated vertex, 8 weight < 1. */
int orc_validate(int32_t n, const int32_t* row_ptr, const int32_t* col,
                 const int32_t* node_w, const int32_t* edge_w);

/* ---- k-hop distance sets (stress superset S of the maxent-stress model) -
 * S_k(u) = { v != u : hop(u,v) <= k }, sorted by (hop, v).
 * off[n+1] (int64) row offsets; hend[u*k + h-1] = number of entries of row u
 * with hop <= h; nbr holds the ids.  Pass nbr == NULL (and hend == NULL)
 * to compute off only. */
int orc_khop_build(int32_t n, const int32_t* row_ptr, const int32_t* col,
                   int32_t k, int64_t* off, int32_t* hend, int32_t* nbr);

/* ---- far field: sum over v != u of r_q(u,v) = (x_u-x_v)/|x_u-x_v|^(q+2) -
 * Exact all-pairs sum in ascending v; coincident pairs contribute 0. */
void orc_farfield_exact(int32_t n, const double* xy, double q, double* F);

/* Cluster far field, the first two sums of Eq. 3 (Section 3.2): exact terms
 * within the own cluster of the next coarser level (cl1, values < n1), plus
 * each other vertex j of the approximation level (clh, values < nh) as
 * nu_j r_q(x_u, xp_j), nu_j = number of level vertices it represents, xp_j
 * their node-weighted midpoint (c may be NULL: weights 1).  Returns -1 on
 * an out-of-range cluster id, -2 on allocation failure. */
int orc_cluster_far(int32_t n, const double* xy, const int32_t* c, const int32_t* cl1,
                    int32_t n1, const int32_t* clh, int32_t nh, double q, double* F);

/* Barnes-Hut quadtree approximation (the quadtree far field the paper cites
 * as related work and as the method of the solver it compares against).
 * Box: origin (min x, min y), side 2^e >= extent; point cell index
 * floor((x - min) * 2^(24-e)) clamped to [0, 2^24-1]; Morton code
 * interleaves x bits (even) and y bits (odd).  Geometric quadtree by
 * recursive subdivision, a cell holding all its points in one child is the
 * same node as that child; one point or depth 24 is a leaf.  Traversal in
 * child order 0..3: leaves add exact terms for every v != u; an internal
 * cell C not containing u is accepted iff
 *     theta^2 * |2*(iu + 1/2) - 2*centre_C|^2  >  4 * side_C^2
 * (quantised units, evaluated exactly as written in FP64), contributing
 * mass_C * r_q(x_u, com_C); otherwise its children are visited.
 * codes (n) / order (n, sorted (code,id)) / nodes (5 per node:
 * depth, first sorted index, count, is_leaf, prefix code) may be NULL.
 * stats[0] accepted cells, stats[1] exact leaf pairs, stats[2] coincident
 * pairs skipped, stats[3] node count.  Returns 0, or -1 on allocation
 * failure. */
int orc_bh(int32_t n, const double* xy, double q, double theta, double* F,
           uint64_t* codes, int32_t* order, int64_t* nodes, int64_t node_cap,
           int64_t* stats);

/* ---- learned far-field correction (q = 0; an extension, not in the paper)
 * Same tree, opening test and visit order as orc_bh.  An accepted cell C
 * for target u adds m r(x_u - com) + kappa (h0 e + h1 p) where
 * e = (x_u - com)/d, p = (-e_y, e_x), t = s/d (s: side of C's tight cell),
 * kappa = m t^2/d and h = MLP(f), f = [t, offset of com from the cell
 * centre along e and p / s, rotated central second moments per unit mass
 * (ee, pp, ep) / s^2, log2(m)/16, 0].
 * MLP: h = W3 relu(W2 relu(W1 f + b1) + b2) + b3 with W1 64x8, W2 64x64,
 * W3 2x64 (row-major), packed W1, b1, W2, b2, W3, b3 (4866 doubles).
 * orc_far_samples records, for u ascending and cells in visit order, the
 * node id (pre-order index), f (8 per sample), the exact residual
 * R = sum_{v in C} r(x_u - x_v) - m r(x_u - com) in h units
 * ((R.e, R.p)/kappa, 2 per sample) and kappa e (2 per sample); at most cap
 * are stored, *count receives the total.  Return 0, or -1 on allocation
 * failure. */
int orc_far_samples(int32_t n, const double* xy, double theta, int64_t cap, int32_t* u_out,
                    int64_t* node_out, double* feat_out, double* target_out, double* coef_out,
                    int64_t* count);
int orc_bh_learned(int32_t n, const double* xy, double theta, const double* weights,
                   double* F);
/* The same field for the listed points only (F: nrows x 2), for checks of
 * large inputs on a sample. */
int orc_bh_learned_rows(int32_t n, const double* xy, double theta, const double* weights,
                        const int32_t* rows, int32_t nrows, double* F);
void orc_mlp_forward(const double* weights, int64_t count, const double* feat, double* out);

/* ---- one Jacobi iteration of the local update (Eq. 2) ----------------
 * For every u, from the old x only:
 *   A_u = sum_{v in S(u)} w_uv (x_v + d_uv (x_u-x_v)/|x_u-x_v|)
 *   C_u = sum_{v in S(u)} r_q(u,v)
 *   x'_u = (A_u + alpha (F_u - C_u)) / rho_u,  rho_u = sum_{S(u)} w_uv
 * F is the far field over all v != u; subtracting C leaves the entropy
 * term over v not in S(u) (the subtraction of Eq. 3's last sum).
 * d_uv = hop at level 0, hop*(sqrt c_u + sqrt c_v)*scale above it;
 * w = d^-2.  A coincident pair adds w*x_v to A and nothing to C.
 * delta[0] = sum (x'-x)^2, delta[1] = sum x^2 (vertex order). */
int orc_sweep(int32_t n, int32_t level, int32_t k, const int64_t* off,
              const int32_t* hend, const int32_t* nbr, const int32_t* c,
              double scale, const double* x, const double* F, double alpha,
              double q, double* xout, double* delta);

/* The same update with the entropy term summed directly over v not in S(u),
 * v != u (Eq. 2 as printed, no subtraction).  O(n^2). */
int orc_sweep_direct(int32_t n, int32_t level, int32_t k, const int64_t* off,
                     const int32_t* hend, const int32_t* nbr, const int32_t* c,
                     double scale, const double* x, double alpha, double q,
                     double* xout, double* delta);

/* The update for selected rows only, with S(u) found by BFS per row instead
 * of a stored set (for graphs whose sets do not fit in host memory). */
int orc_sweep_rows(int32_t n, const int32_t* row_ptr, const int32_t* col,
                   int32_t level, int32_t k, const int32_t* c, double scale,
                   const double* x, const double* F, double alpha, double q,
                   const int32_t* rows, int32_t nrows, double* xout_rows,
                   int64_t* set_sizes);

/* ---- size-constrained label propagation, synchronous two-colour form ----
 * Labels start as label[v] = v (or as given when keep_init != 0).  For round
 * r and colour s, v is active iff bit 0 of draw(seed, level_h, 16+r, v)
 * equals s.  Cluster weights W are frozen per sub-round.  An active v scores
 * each neighbouring label by the sum of edge weights to it; a label is
 * feasible iff it is v's own or W(L) + c(v) <= U; the best feasible label
 * has the largest score, ties going to v's own label and then to the
 * smallest id; labels of score 0 other than its own are never chosen.
 * Moves to L are admitted in ascending v while W(L) plus the sum of c over
 * proposals to L up to v stays <= U.  Stops after a round without moves.
 * moves[r] receives the number of moves of round r.  Returns rounds run. */
int orc_lp(int32_t n, const int32_t* row_ptr, const int32_t* col,
           const int32_t* c, const int32_t* w, double U, int32_t rounds,
           uint64_t seed, int32_t level_h, int32_t* label, int32_t* moves);

/* ---- contraction of a clustering ---------------------------------------
 * Coarse id = rank of the label among distinct labels.  c' = sum c,
 * w'(U,V) = sum of w over fine edges between the blocks; intra-block edges
 * dropped; coarse rows ascending.  Output arrays must hold n (+1) and nnz
 * entries.  Returns the coarse vertex count; *cnnz receives 2m'. */
int32_t orc_contract(int32_t n, const int32_t* row_ptr, const int32_t* col,
                     const int32_t* c, const int32_t* w, const int32_t* label,
                     int32_t* cluster, int32_t* crow_ptr, int32_t* ccol,
                     int32_t* cc, int32_t* cw, int64_t* cnnz);

/* ---- initial layout and prolongation ------------------------------------
 * init: x_v = (U0, U1) with U_j = unit draw(seed, level, tag 1, 2v+j).
 * prolong (uncoarsening): fine v of coarse v' = cluster[v] is placed at
 * x'_{v'} + rho (cos phi, sin phi), phi = 2 pi U0, rho = sqrt(c(v')) U1,
 * U_j = unit draw(seed, level, tag 2, 2v+j): angle uniform in [0, 2pi),
 * radius uniform in [0, sqrt c(v')]. */
void orc_init_layout(int32_t n, uint64_t seed, int32_t level, double* xy);
void orc_prolong(int32_t n_fine, const int32_t* cluster, const int32_t* coarse_c,
                 const double* coarse_xy, uint64_t seed, int32_t level,
                 double* fine_xy);

/* ---- objectives (Eq. 1 and the full-stress measure) --------------------
 * Pairs u < v.  stress = sum over v in S(u) of w (D - d)^2;
 * ent = sum over v not in S(u) of E_q(D), E_0 = ln D, E_q = -D^-q / q, so
 * M = stress - alpha * ent.  Coincident pairs are skipped in ent and
 * counted in out[2].  out = {stress, ent, coincident}. */
int orc_objective(int32_t n, int32_t level, int32_t k, const int64_t* off,
                  const int32_t* hend, const int32_t* nbr, const int32_t* c,
                  double scale, const double* x, double q, double* out);

/* Full stress over all pairs with BFS hop distances d and w = d^-2:
 * out = {F(x), s*, F(s* x)} with s* = sum(D/d) / sum((D/d)^2), the
 * minimiser of sum w (s D - d)^2. Pairs in different components skipped. */
int orc_full_stress(int32_t n, const int32_t* row_ptr, const int32_t* col,
                    const double* x, double* out);

#ifdef __cplusplus
}
#endif
#endif
