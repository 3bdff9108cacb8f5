/*
 * fa2lay.h -- C ABI of libfa2lay.so, an MI355X (gfx950) implementation of the
 * graph layout method of "Graph Visualization for Blockchain Data"
 * (Dietl, Gemuend, Oeltz, Thiele, Werner, 2024):
 *
 *   - split the graph into connected components, ignoring edge directions
 *     (sec. 4);
 *   - lay out small components with Kamada-Kawai on shortest-path (hop)
 *     distances (sec. 3.1, sec. 4);
 *   - lay out large components with ForceAtlas2, whose all-pairs repulsion is
 *     evaluated by a 2D Fast Multipole Method over a quadtree (sec. 3.2,
 *     sec. 3.2.1), with the swing/traction step-size control of sec. 3.2.
 *
 * Conventions (every entry point):
 *   - Pointers are DEVICE pointers on the context's device, owned by the
 *     caller, unless marked [host].  Arrays are dense, 0-based, and laid out
 *     as stated.  The library never frees or retains a caller pointer.
 *   - Work is enqueued on the context's stream (the stream passed to
 *     fl_create / fl_set_stream).  A call returns before the work finishes
 *     unless it returns a [host] value, in which case it synchronises the
 *     stream first.
 *   - The context owns its workspace (sort buffers, tree, lists, expansions)
 *     and grows it on demand with hipMalloc; repeated calls at the same or
 *     smaller sizes allocate nothing.
 *   - Errors are returned as fl_status; nothing is thrown or aborted across
 *     the ABI.  Arguments are validated on the host before any launch; a
 *     failed call launches nothing.  fl_last_error() describes the last
 *     failure of the context.  A context is not thread-safe: use one per
 *     host thread and stream.
 *   - Node ids are int32 in [0, n).  Positions are FP32, structure-of-arrays
 *     (x[n], y[n]).
 */
#ifndef FA2LAY_H
#define FA2LAY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FL_OK = 0,
    FL_EINVAL = -1,       /* bad argument (null pointer, size, id out of range, parameter) */
    FL_ENOMEM = -2,       /* device allocation failed or exceeds the context budget */
    FL_EHIP = -3,         /* a HIP runtime call failed; see fl_last_error */
    FL_ENONFINITE = -4,   /* a non-finite position was found */
    FL_EBUSY = -5,        /* serving: no free slot / budget (try later) */
    FL_ECANCELED = -6,    /* serving: job cancelled */
    FL_EUNSUPPORTED = -7  /* valid but not supported by this build (e.g. expansion order) */
} fl_status;

typedef struct fl_ctx fl_ctx;

/* Create a context on HIP device `device`, enqueueing on `stream` (a
 * hipStream_t; NULL = the device's null stream).  *out receives the handle.
 * workspace_budget_bytes bounds the device workspace the context may hold,
 * its branch contexts included (0: no bound); a call whose workspace would
 * pass it fails with FL_ENOMEM (after the buffers replaced by larger ones
 * have been freed and the sum checked again). */
fl_status fl_create(fl_ctx **out, int device, void *stream, size_t workspace_budget_bytes);
/* Release the context and its workspace (synchronises its stream). */
void fl_destroy(fl_ctx *ctx);
/* Text of the last error on this context; valid until the next call on it. */
const char *fl_last_error(const fl_ctx *ctx);
/* Switch the stream later calls enqueue on. */
fl_status fl_set_stream(fl_ctx *ctx, void *stream);
/* Block until the context's stream has drained; then free the workspace
 * buffers that were replaced by larger ones (see fl_workspace_bytes). */
fl_status fl_synchronize(fl_ctx *ctx);
/* Bytes of device workspace the context holds.  A buffer replaced by a
 * larger one is kept (it may still be in use by enqueued work) and counted
 * until fl_synchronize, fl_destroy or a later growth frees it. [host] */
size_t fl_workspace_bytes(const fl_ctx *ctx);
/* Library version string, e.g. "fa2lay 0.1 gfx950". [host] */
const char *fl_version(void);

/* ------------------------------------------------------------------------
 * Graph preparation (sec. 2: bipartite address/transaction graph with input
 * and output edges; sec. 4: components are taken ignoring edge directions).
 * ------------------------------------------------------------------------ */

/* Build the simple undirected graph of a directed edge list in CSR form:
 * direction ignored, self loops and duplicate pairs dropped, each row sorted
 * ascending.  deg[i] = number of distinct neighbours.
 *   src, dst [m] int32 in [0, n);  row_ptr [n+1];  col_idx capacity 2m;
 *   deg [n];  *nnz_out [host] = row_ptr[n].  Synchronises.
 * Errors: FL_EINVAL for n < 1, m < 0, n*n >= 2^62 or an id outside [0, n)
 * (checked on the device before any output is written). Bit-exact. */
fl_status fl_build_csr(fl_ctx *ctx, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       int32_t *row_ptr, int32_t *col_idx, int32_t *deg, int64_t *nnz_out);

/* Connected components of a CSR graph (sec. 4): label[v] = the smallest node
 * id of v's component.  *n_comp_out [host] = number of components.
 * Synchronises.  Bit-exact. */
fl_status fl_components(fl_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        int32_t *label, int32_t *n_comp_out);

/* ------------------------------------------------------------------------
 * Quadtree hooks (sec. 3.2.1: a square covering all particles, divided into
 * four while it holds more than leaf_size particles).  Exposed for testing.
 * ------------------------------------------------------------------------ */

/* Root square and Morton keys of the points (x[i], y[i]):
 *   xmin, ymin = exact minima (FP64 of FP32 values), L = max(xmax-xmin,
 *   ymax-ymin) (1 if 0), S = 2^bits / L (FP64, correctly rounded);
 *   q = min(floor((x - xmin) * S), 2^bits - 1), same for y with ymin;
 *   key = q_x bits in the even positions, q_y bits in the odd ones.
 * key [n] uint32; root4 [4] double (xmin, ymin, L, S) may be NULL.
 * bits in [1, 16]. */
fl_status fl_morton(fl_ctx *ctx, int32_t n, const float *x, const float *y, int32_t bits, uint32_t *key,
                    double *root4);

/* Stable ascending sort of key[n] (uint32; only the low 2*bits bits are
 * significant): key_out [n] sorted keys, perm [n] = source index of each
 * output position (ties keep ascending index). */
fl_status fl_sort_keys(fl_ctx *ctx, int32_t n, const uint32_t *key, int32_t bits, uint32_t *key_out,
                       int32_t *perm);

/* Build the adaptive quadtree of the points and copy it out.  cells
 * [cap * 10] int32, one row per cell: level, ix, iy, begin, end, parent,
 * child0..child3 (-1 = empty quadrant; child q covers (2ix + (q&1),
 * 2iy + (q>>1))); [begin, end) indexes the Morton-sorted order.  Cells are
 * in depth-first pre-order (sorted by (begin, level)).  A cell is a leaf iff
 * it holds <= leaf_size points or sits at level `bits`.  *n_cells_out [host].
 * Synchronises.  FL_EINVAL if cap is too small (n_cells_out still set). */
fl_status fl_tree(fl_ctx *ctx, int32_t n, const float *x, const float *y, int32_t bits, int32_t leaf_size,
                  int32_t *cells, int32_t cap, int32_t *n_cells_out);

/* ------------------------------------------------------------------------
 * ForceAtlas2 (sec. 3.2) with FMM repulsion (sec. 3.2.1)
 * ------------------------------------------------------------------------ */

enum { FL_GRAV_STRONG_MASS = 0, FL_GRAV_FA2_CONST = 1, FL_GRAV_STRONG_UNIT = 2 };
enum { FL_SWING_PAPER = 0, FL_SWING_FA2 = 1 };
/* FL_REP_AUTO: per system of n nodes, the context's tuning table decides
 * (exact below its crossover, else FMM with the p and leaf_size of n's size
 * bucket; see fl_autotune). */
enum { FL_REP_EXACT = 0, FL_REP_FMM = 1, FL_REP_AUTO = 2 };

/* Forces (mass m_i = deg_i + 1):
 *   repulsion  F_r,i = kr m_i sum_{j != i} m_j (p_i - p_j) / |p_i - p_j|^2
 *              (coincident pairs contribute 0);
 *   attraction F_a,i = ka sum_{j in N(i)} (p_j - p_i);
 *   gravity    STRONG_MASS: -kg m_i p_i;  STRONG_UNIT: -kg p_i;
 *              FA2_CONST: -kg m_i p_i / |p_i| (0 at the origin).
 * Step (sec. 3.2): swg_i = |F_i - F'_i|, tra_i = |F_i + F'_i| with F' the
 *   previous iteration's forces (0 on the first); SWING_PAPER: SWG = sum
 *   swg_i, TRA = sum tra_i; SWING_FA2: SWG = sum m_i swg_i, TRA = sum
 *   m_i tra_i / 2.  s_G = tau TRA / SWG, capped at (1 + max_rise) s_prev after
 *   the first iteration (SWG = 0: 1 on the first, the cap afterwards);
 *   s_i = ks s_G / (1 + s_G sqrt(swg_i)), capped at ksmax / |F_i|;
 *   p_i += s_i F_i.  Sums, s_G and s_i are FP64. */
typedef struct {
    double kr, kg, ka;
    int32_t gravity_mode;  /* FL_GRAV_* */
    int32_t swing_mode;    /* FL_SWING_* */
    double tau, ks, ksmax, max_rise;
    int32_t repulsion;     /* FL_REP_EXACT (O(n^2)), FL_REP_FMM or FL_REP_AUTO */
    int32_t p;             /* FMM expansion order: 4, 6, 8, 10, 12, 16 */
    int32_t leaf_size;     /* FMM: a cell holding more points is divided (1..1024) */
    int32_t morton_bits;   /* FMM: quadtree depth cap, 1..16 */
    int32_t list_lanes;    /* FMM: lanes per cell that build the interaction lists, 1 or 8 (0: chosen
                              by size); a launch shape only, the results are the same */
} fl_fa2_params;

/* Defaults: kr = kg = ka = 1, STRONG_MASS, SWING_PAPER, tau = 1, ks = 0.1,
 * ksmax = 10, max_rise = 0.5, FMM, p = 8, leaf_size = 64, morton_bits = 16,
 * list_lanes = 0. */
void fl_fa2_default_params(fl_fa2_params *prm);

/* Caller-owned iteration state. fx_prev/fy_prev [n]: forces of the previous
 * iteration (ignored when iter == 0), overwritten with this iteration's.
 * iter [host] counts completed iterations and is advanced by the step/run
 * calls.
 * Systems (sec. 4: every component is laid out separately): with n_comp <= 1
 * all n nodes form one system; with n_comp >= 2, comp_offsets [host,
 * n_comp + 1] (0 = comp_offsets[0] < ... < comp_offsets[n_comp] = n) splits
 * the nodes into systems k = [comp_offsets[k], comp_offsets[k+1]), no CSR
 * edge may join two of them (FL_EINVAL), and every system has its own
 * repulsion (only its own nodes repel), swing, traction and global speed,
 * so that each system's result is bitwise the one it gets alone.
 * scalars [4 * max(n_comp, 1)] double on the device, four per system: [0]
 * s_G of the previous iteration (read when iter > 0), overwritten with this
 * iteration's s_G; [1] SWG; [2] TRA of the last iteration.  The [host]
 * statistics of fl_fa2_step / fl_fa2_run are system 0's.  With
 * FL_REP_AUTO the tuning table is read at the largest system's size. */
typedef struct {
    float *fx_prev;
    float *fy_prev;
    double *scalars;
    int64_t iter;
    int32_t n_comp;
    const int32_t *comp_offsets;
} fl_fa2_state;

typedef struct {
    double swg, tra, speed;
} fl_step_stats;

/* The three force terms at positions (x, y) of a CSR graph (deg [n] as from
 * fl_build_csr; row_ptr/col_idx symmetric).  Any output pair may be NULL. */
fl_status fl_fa2_forces(fl_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        const int32_t *deg, const float *x, const float *y, const fl_fa2_params *prm,
                        float *frx, float *fry, float *fax, float *fay, float *fgx, float *fgy);

/* One iteration, in place on x, y and the state.  stats [host] may be NULL
 * (if not, the call synchronises).  FL_ENONFINITE if a force or position is
 * not finite (a system whose forces are not finite is left unmodified; the
 * others move). */
fl_status fl_fa2_step(fl_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                      const int32_t *deg, float *x, float *y, fl_fa2_state *state, const fl_fa2_params *prm,
                      fl_step_stats *stats);

/* `iters` iterations with no host synchronisation inside the loop.
 * per_iter [host, iters entries] may be NULL (if not, synchronises at the
 * end).  Checks for non-finite values at the end of the run.  When per_iter
 * is NULL, timing is off, graphs are on (fl_set_graphs) and iters >= 4, the
 * first iteration runs eagerly and one more is captured into a HIP graph on
 * the context's private streams and replayed; the results are bitwise those
 * of eager iterations.  The call returns after the work is done. */
fl_status fl_fa2_run(fl_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const int32_t *deg, float *x, float *y, fl_fa2_state *state, const fl_fa2_params *prm,
                     int32_t iters, fl_step_stats *per_iter);

/* fl_fa2_step for callers that cannot allocate device memory while they run
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same iteration, the same kernels and, bitwise, the same
 * results as fl_fa2_step, but every buffer the iteration needs beyond the
 * caller's arrays (sort buffers, tree, hash table, lists, expansions, force
 * and reduction buffers) is carved from a fixed array of
 * FL_NOALLOC_SCRATCH_BYTES bytes of device memory that the library holds on
 * each GPU it runs on until the process ends.  The call allocates and frees
 * nothing (the context, created earlier by fl_create, supplies its stream
 * and its small host staging buffer; its own workspace is neither used nor
 * grown).  Every call on a GPU uses that GPU's array from its start and
 * leaves the last call's contents in it: calls that overlap on one GPU (on
 * other streams or threads, or any fl_fa2_step_noalloc in flight) race.
 * The iteration runs in line on the context's stream (no branch streams).
 * Errors as fl_fa2_step, and FL_ENOMEM when the iteration's buffers do not
 * fit the array (then x, y and the state are left unmodified): with FMM at
 * p = 8 and leaf_size = 64, graphs of the bipartite transaction generator
 * fit up to 2e5 nodes (2.5e5 do not); with the exact repulsion, 4e6 nodes
 * without edges fit. */
#define FL_NOALLOC_SCRATCH_BYTES (256u << 20)
fl_status fl_fa2_step_noalloc(fl_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              const int32_t *deg, float *x, float *y, fl_fa2_state *state,
                              const fl_fa2_params *prm, fl_step_stats *stats);

/* Statistics of the FMM evaluations on this context [host, synchronises]:
 * last evaluation: out[0] cells, [1] leaves, [2] near-field (P2P) particle
 * pairs, [3] M2L (V-list) entries, [4] W-list entries, [5] X-list entries,
 * [6] deepest level, [7] U-list entries; totals since the last reset:
 * [8] near-field pairs, [9] M2L entries, [10] evaluations, [11] particles
 * evaluated.  reset != 0 zeroes the totals after reading them. */
enum { FL_NSTATS = 12 };
fl_status fl_fmm_stats(fl_ctx *ctx, int64_t *out, int reset);

/* Barnes-Hut repulsion (comparator: sec. 3.2.1 names it as the O(N log N)
 * method the FMM improves on; Barnes & Hut 1986).  The quadtree is the
 * FMM's (leaf_size, morton_bits); every cell carries its total mass and
 * centre of mass (FP64 sums, stored FP32).  For node i the tree is walked
 * from the root in depth-first order: a cell that does not hold i, with side
 * s and distance d from p_i to its centre of mass such that s < theta d,
 * acts as one particle (its mass at its centre of mass); any other cell is
 * opened, and an opened leaf is summed directly.  frx, fry [n] receive F_r
 * with the masses (deg + 1) and kr of fl_fa2_forces; theta = 0 gives the
 * exact sum.  All nodes form one system.  theta in [0, 10]. */
fl_status fl_bh_repulsion(fl_ctx *ctx, int32_t n, const float *x, const float *y, const int32_t *deg, double kr,
                          double theta, int32_t leaf_size, int32_t morton_bits, float *frx, float *fry);

/* ------------------------------------------------------------------------
 * Kamada-Kawai for small components (sec. 3.1): hop distances d_ij by
 * breadth-first search (exact for unit weights, equal to the Floyd-Warshall
 * distances the paper names), then localized stress majorization of the
 * energy  E = sum_{i<j} d_ij^-2 (|p_i - p_j| - l d_ij)^2: every node of a
 * component moves together from the previous positions to
 *   p_i' = sum_{j!=i} w_ij (p_j + l d_ij u_ij) / sum_{j!=i} w_ij,
 * w_ij = d_ij^-2, u_ij = (p_i - p_j)/|p_i - p_j| (0 when they coincide);
 * in a 2-node component, where this maps the distance r to |2l - r|, each
 * node moves half way (the pair lands at distance l about its midpoint).
 * Components are given as node ranges: comp_offsets [host, n_comp+1]
 * increasing, component k = nodes [comp_offsets[k], comp_offsets[k+1]), each
 * of 1..256 nodes, with no edge leaving its range.
 * ------------------------------------------------------------------------ */
enum { FL_KK_MAJORIZATION = 0, FL_KK_NEWTON = 1 };
/* Minimisers:
 *   FL_KK_MAJORIZATION: `steps` steps of the update above, every node of a
 *     component at once;
 *   FL_KK_NEWTON (the paper's Newton-Raphson, after Kamada and Kawai): a
 *     move takes the node m with the largest gradient norm |dE/dp_m| (lowest
 *     index on a tie) and makes up to 16 Newton-Raphson steps on p_m alone:
 *     the 2x2 system of E's second derivatives in x_m, y_m when that Hessian
 *     is positive definite, else -g / (2 sum_i d_mi^-2); each step is halved
 *     (at most 30 times) until the part of E that depends on p_m decreases,
 *     and a step that finds no decrease ends the move.  Moves stop when every
 *     gradient norm is below eps * l, or after steps * n moves for a
 *     component of n nodes.  One wave per component. */
/* Reductions (sec. 3.1, clustering before the layout, declustering after;
 * fl_kk_layout and fl_layout only, as they need the graph):
 *   FL_KK_REDUCE_LEAVES: a node with one edge whose neighbour has two or
 *     more is contracted into the neighbour (one round; a 2-node component
 *     keeps both);
 *   FL_KK_REDUCE_CHAINS: among the remaining nodes, those with exactly two
 *     remaining neighbours form chains; a chain between two distinct kept
 *     nodes is removed and counts as one edge of its length (loops, pure
 *     cycles and all but the chain with the smallest node id between the
 *     same two ends stay).
 * Both keep the hop distances between the remaining nodes, so these are laid
 * out with their distances in the full component.  Declustering: the i-th of
 * k nodes of a removed chain from end a (the smaller id) to end b goes to
 * p_a + i/(k+1) (p_b - p_a); then the j-th of k contracted leaves of node v
 * (id order) goes to distance l from p_v at angle phi + (j - (k-1)/2) pi/k,
 * phi the direction from the centre of gravity c of the placed nodes to p_v,
 * or at angle 2 pi j / k when |p_v - c| <= 1e-4 (R + l), R the largest
 * |p - c| of a placed node. */
enum { FL_KK_REDUCE_LEAVES = 1, FL_KK_REDUCE_CHAINS = 2 };
typedef struct {
    double l;           /* rescaling constant: desired length per hop (> 0) */
    int32_t steps;      /* majorization: steps; Newton-Raphson: moves per node */
    int32_t minimiser;  /* FL_KK_MAJORIZATION or FL_KK_NEWTON */
    double eps;         /* Newton-Raphson: gradient-norm tolerance, in units of l (>= 0) */
    int32_t reduce;     /* FL_KK_REDUCE_* flags (0: none) */
} fl_kk_params;

/* Defaults: l = 1, steps = 200, minimiser FL_KK_MAJORIZATION, eps = 1e-3,
 * reduce 0. */
void fl_kk_default_params(fl_kk_params *prm);

/* Hop distances of every component: dist [sum n_k^2] int32, component k's
 * n_k x n_k row-major matrix of local ids starting at dist_offsets[k] =
 * sum_{k'<k} n_k'^2 (written to dist_offsets [host, n_comp+1] if not NULL).
 * Synchronises.  FL_EINVAL if an edge leaves its component or a component is
 * not connected.  Bit-exact. */
fl_status fl_hop_distances(fl_ctx *ctx, int32_t n_comp, const int32_t *comp_offsets, const int32_t *row_ptr,
                           const int32_t *col_idx, int32_t *dist, int64_t *dist_offsets);

/* The minimiser of prm on every component, in place on x, y, given the
 * distances of fl_hop_distances.  For majorization, one workgroup runs all
 * steps of one component, each node's sum split over up to 16 lanes (a
 * launch per size class: up to 16, 64 and 256 nodes); for Newton-Raphson,
 * one wave per component.  Synchronises. */
fl_status fl_kk_steps(fl_ctx *ctx, int32_t n_comp, const int32_t *comp_offsets, const int32_t *dist, float *x,
                      float *y, const fl_kk_params *prm);

/* fl_hop_distances then fl_kk_steps (with the reductions of prm->reduce),
 * distances in the context workspace.  FL_EINVAL from fl_kk_steps when
 * prm->reduce is not 0. */
fl_status fl_kk_layout(fl_ctx *ctx, int32_t n_comp, const int32_t *comp_offsets, const int32_t *row_ptr,
                       const int32_t *col_idx, float *x, float *y, const fl_kk_params *prm);

/* ------------------------------------------------------------------------
 * The whole method (sec. 4): connected components of the CSR graph; single
 * nodes to the origin; components of 2..kk_max_nodes nodes by Kamada-Kawai;
 * larger ones by fa2_iters ForceAtlas2 iterations each (FMM repulsion when
 * fa2->repulsion is FL_REP_FMM and the component has >= fmm_min_nodes nodes,
 * exact otherwise; with FL_REP_AUTO the context's tuning table decides per
 * component and fmm_min_nodes is not used).  x, y in place, caller's node order.  Components are laid
 * out independently, each about its own centre.  The ForceAtlas2 components
 * run concurrently: they are dealt, largest first, to up to 8 branch streams
 * owned by the context, and one HIP graph holding an iteration of every
 * component is replayed (results bitwise those of each component run alone
 * by fl_fa2_run).  With graphs off (fl_set_graphs) the components run one
 * after the other as eager launches on the context's stream.  Synchronises.
 * FL_ENONFINITE when a ForceAtlas2 component's forces or positions turned
 * non-finite: every component has its own status word, so that component
 * stops moving (at its last finite positions when a force was the first
 * non-finite value) while the others are laid out as usual, and all
 * positions are written back before the call returns the error.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_comp, n_single, n_kk, n_fa2;
    int64_t kk_nodes, fa2_nodes;
    double ms_setup, ms_kk, ms_fa2;
} fl_layout_stats;

fl_status fl_layout(fl_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const int32_t *deg,
                    float *x, float *y, const fl_fa2_params *fa2, int32_t fa2_iters, const fl_kk_params *kk,
                    int32_t kk_max_nodes, int32_t fmm_min_nodes, fl_layout_stats *stats);

/* ------------------------------------------------------------------------
 * Assembly of the component layouts into one drawing (sec. 4): every
 * component is rescaled to a common density, the components become the
 * nodes of a tree ("meta-graph": in a random order, each component is linked
 * to the largest one before it by an edge of half the two diameters summed
 * plus a constant), and the tree is laid out by Kamada-Kawai; a tree too
 * large for one layout is cut into groups that are laid out separately and
 * then assembled the same way.  Definitions (the paper leaves them open):
 *   centroid c_k and RMS distance rho_k of component k's nodes from it;
 *   scale s_k = sqrt(n_k / (2 pi density)) / rho_k (1 when rho_k = 0): the
 *     nodes then fill an equivalent uniform disc (same second moment) at the
 *     target density;
 *   radius R_k = s_k max_i |p_i - c_k| (diameter 2 R_k);
 *   "largest" = most nodes, the earliest in the order on a tie;
 *   groups: the order is cut into consecutive runs of max_group components,
 *     each with its own meta-graph; the runs, in order, are the components of
 *     the next level (nodes added up, centre = node-weighted centroid,
 *     radius = smallest circle about it holding the members' circles), until
 *     one run remains;
 *   a group's layout starts with item t at distance d(0, t) from the origin
 *     at angle 2 pi t / g and runs `sweeps` sweeps of sequential localized
 *     stress majorization of E = sum_{i<j} d_ij^-2 (|p_i - p_j| - d_ij)^2
 *     (d = path length in the meta-graph): items 0..g-1 in turn move to
 *     sum_{j!=i} w_ij (p_j + d_ij u_ij) / sum_{j!=i} w_ij, w_ij = d_ij^-2;
 *   finally node i of component k goes to s_k (p_i - c_k) + shift_k, with the
 *     drawing's node centroid at the origin.
 * Precision: frames and group centres FP64; the meta-graph layout FP32.
 * ------------------------------------------------------------------------ */
typedef struct {
    double density;     /* target nodes per unit area (> 0) */
    double gap;         /* constant added to every meta-edge length (> 0) */
    int32_t max_group;  /* largest meta-graph laid out in one piece, 2..256 */
    int32_t sweeps;     /* majorization sweeps per meta-graph (>= 0) */
} fl_assemble_params;

/* Defaults: density 1, gap 1, max_group 256, sweeps 100. */
void fl_assemble_default_params(fl_assemble_params *prm);

typedef struct {
    int32_t n_comp, levels, groups;
    double ms;
} fl_assemble_stats;

/* Assemble, in place on x, y [n], the components given by label [n] (device,
 * int32 in [0, n), e.g. fl_components' labels; component k = the k-th
 * smallest distinct label, n_comp of them).  order [host, n_comp] is the
 * random order: a permutation of 0..n_comp-1 drawn by the caller.
 * Optional device outputs (NULL: not written):
 *   frame [n_comp * 6] FP64: c_k (x, y), s_k, R_k, shift_k (x, y);
 *   parent [n_comp]: the component linked to in the first-level meta-graph,
 *     -1 for the first of each group.
 * stats [host] may be NULL.  Synchronises.  FL_EINVAL for a label outside
 * [0, n), a count of distinct labels other than n_comp, an order that is not
 * a permutation, or parameters out of range. */
fl_status fl_assemble(fl_ctx *ctx, int32_t n, const int32_t *label, int32_t n_comp, const int32_t *order, float *x,
                      float *y, const fl_assemble_params *prm, double *frame, int32_t *parent,
                      fl_assemble_stats *stats);

/* ------------------------------------------------------------------------
 * Autotuning (project addition; the paper fixes no FMM parameters).
 * The table maps a system size to exact or FMM repulsion and the FMM's
 * expansion order p and leaf size; FL_REP_AUTO reads it.
 * ------------------------------------------------------------------------ */
enum { FL_TUNE_MAX_BUCKETS = 16 };
typedef struct {
    int32_t fmm_min_nodes;  /* exact repulsion below this size, FMM from it */
    int32_t n_buckets;      /* 1..FL_TUNE_MAX_BUCKETS */
    int32_t bucket_max[FL_TUNE_MAX_BUCKETS]; /* bucket b: sizes <= bucket_max[b], ascending (the last
                                                bucket also takes every larger size) */
    int32_t p[FL_TUNE_MAX_BUCKETS];          /* expansion order per bucket (4, 6, 8, 10, 12, 16) */
    int32_t leaf_size[FL_TUNE_MAX_BUCKETS];  /* leaf size per bucket (1..1024) */
    int32_t list_lanes[FL_TUNE_MAX_BUCKETS]; /* lanes per cell of the list kernels (1 or 8; 0: by size) */
    double max_rel_err;     /* error bound the table was tuned for (0: not tuned) */
} fl_tuning;

/* The table a new context starts with: fmm_min_nodes 4096, one bucket with
 * p = 8, leaf_size = 64, list_lanes = 0, max_rel_err 0. */
void fl_default_tuning(fl_tuning *out);
/* Copy a table into the context (NULL: the default); FL_EINVAL if malformed. */
fl_status fl_set_tuning(fl_ctx *ctx, const fl_tuning *tuning);
fl_status fl_get_tuning(fl_ctx *ctx, fl_tuning *out);

/* One measurement of fl_autotune: p = 0 is the exact repulsion. */
typedef struct {
    int32_t size, p, leaf_size, list_lanes, feasible;
    double ms;       /* median over the repetitions (tree, lists and passes for FMM) */
    double rel_err;  /* |F - F_exact|_2 / |F_exact|_2 over all nodes of the prefix */
} fl_tune_sample;

/* Measure and build a tuning table; the table is also installed in the
 * context.  For each size s of sizes [host, ascending, 1..16 entries, each
 * in [2, n]], the first s points of x, y, deg [device, n] (pass them in
 * random order, so that a prefix is a uniform subsample; deg gives the
 * masses) are evaluated by the exact repulsion and by the FMM for every
 * p in {4, 6, 8, 10, 12, 16}, leaf_size in {16, 24, 32, 48, 64, 96, 128}
 * and list_lanes in {1, 8}, `reps` timed repetitions each (HIP events on the context's stream).  At
 * each size the fastest FMM configuration whose error against the exact
 * forces is <= max_rel_err is chosen (the most accurate one if none is);
 * the crossover is the geometric mean of the largest size at which exact
 * repulsion is faster and the next one (sizes[0] if the FMM wins at every
 * size, past the last size if it wins at none).  max_rel_err in [1e-6, 1]
 * (the exact reference itself is good to about 1e-7); reps in [1, 20].
 * samples [host, samples_cap entries] may be NULL; n_samples [host] gets the
 * number of measurements.  Synchronises. */
fl_status fl_autotune(fl_ctx *ctx, int32_t n, const float *x, const float *y, const int32_t *deg, int32_t n_sizes,
                      const int32_t *sizes, double max_rel_err, int32_t reps, fl_tuning *out,
                      fl_tune_sample *samples, int32_t samples_cap, int32_t *n_samples);

/* ------------------------------------------------------------------------
 * Layout server: continuous batching of layout jobs on one GPU.  Jobs are
 * copied at submission and queued FIFO; `max_slots` workers (one HIP stream
 * and context each) admit the head of the queue whenever the workers' charges
 * (below) with the head's estimated device bytes fit `mem_budget_bytes`; a
 * worker that ends a job holding more than the budget allows gives its
 * memory back, and so does an idle one whose memory keeps the head out, so
 * the device bytes the workers hold stay within the budget.  Jobs that
 * arrive while others run start as soon as a slot and memory free up, and
 * their kernels overlap on the device.  A job runs fl_build_csr + fl_layout
 * (kk_max_nodes 256, fmm_min_nodes 4096) and its positions come back to host
 * memory.  Results do not depend on the other jobs in flight.  All server
 * calls are thread-safe.  Times are seconds since the server was created.
 * ------------------------------------------------------------------------ */
typedef struct fl_server fl_server;
enum { FL_JOB_QUEUED = 0, FL_JOB_RUNNING = 1, FL_JOB_DONE = 2, FL_JOB_FAILED = 3, FL_JOB_CANCELED = 4 };

typedef struct {
    int32_t n;                /* nodes */
    int64_t m;                /* directed edge records */
    const int32_t *src, *dst; /* [host, m] */
    const float *x0, *y0;     /* [host, n] initial positions */
    int32_t iters;            /* ForceAtlas2 iterations per large component */
    fl_fa2_params params;
} fl_job;

/* bytes_in_use / peak_bytes: the sum of the workers' charges against the
 * budget (a worker between jobs is charged the device bytes it holds, a
 * worker running a job the larger of those and the job's estimate);
 * held_bytes / peak_held_bytes: device bytes the workers hold between jobs
 * (context workspace, branch contexts, job buffers; measured, not estimated);
 * trims: times a worker gave its memory back to keep the charges within the
 * budget; over_estimate: jobs that grew their worker's memory past what they
 * were charged (the larger of the job's estimate and what the worker held). */
typedef struct {
    int64_t submitted, admitted, completed, failed, canceled, queued, running;
    int64_t bytes_in_use, peak_bytes, node_updates;
    int64_t held_bytes, peak_held_bytes, trims, over_estimate;
} fl_server_stats;

fl_status fl_server_create(fl_server **out, int device, size_t mem_budget_bytes, int32_t max_slots);
/* Tuning table (see fl_autotune) for jobs admitted from now on whose
 * params.repulsion is FL_REP_AUTO; NULL restores the default. */
fl_status fl_server_set_tuning(fl_server *srv, const fl_tuning *tuning);
/* Test hook: a server whose workers sleep ns_per_node_update * n * iters
 * nanoseconds instead of using the GPU (results = initial positions). */
fl_status fl_server_create_fake(fl_server **out, size_t mem_budget_bytes, int32_t max_slots,
                                double ns_per_node_update);
/* Copies the job's arrays; never waits for the GPU.  FL_ENOMEM if the job
 * alone exceeds the budget, FL_EINVAL for a malformed job. */
fl_status fl_server_submit(fl_server *srv, const fl_job *job, uint64_t *job_id);
fl_status fl_server_poll(fl_server *srv, uint64_t job_id, int32_t *state);
/* Block until the job is done, failed or cancelled (timeout_s < 0: no limit;
 * FL_EBUSY on timeout). */
fl_status fl_server_wait(fl_server *srv, uint64_t job_id, double timeout_s, int32_t *state);
/* Positions [host, n each; either may be NULL] and times3 [host, 3]:
 * arrival, start, completion.  FL_EBUSY while queued/running, FL_EHIP if the
 * job failed (fl_server_last_error has its message), FL_ECANCELED. */
fl_status fl_server_result(fl_server *srv, uint64_t job_id, float *x_host, float *y_host, double *times3);
/* Forget a finished job and free its host results. */
fl_status fl_server_release(fl_server *srv, uint64_t job_id);
/* Cancel a queued job (FL_EBUSY once it runs). */
fl_status fl_server_cancel(fl_server *srv, uint64_t job_id);
fl_status fl_server_stats_get(fl_server *srv, fl_server_stats *out);
const char *fl_server_last_error(const fl_server *srv);
/* Cancels queued jobs, waits for running ones, frees everything. */
void fl_server_destroy(fl_server *srv);

/* Per-phase device timing (HIP events on the context's stream).  When
 * enabled, fl_fa2_step/run (FL_PH_EVAL: the near field, FL_PH_FAR: the far
 * field added to it; fl_bh_repulsion: tree, then FL_PH_BH for
 * the cell moments and the walk) record events around their phases; fl_get_timing
 * returns the accumulated milliseconds and launch counts per phase
 * (FL_NPHASE entries each) and clears them [host, synchronises]. */
enum { FL_PH_TREE = 0, FL_PH_LISTS, FL_PH_UPWARD, FL_PH_M2L, FL_PH_EVAL, FL_PH_ATTRACT, FL_PH_UPDATE,
       FL_PH_EXACT, FL_PH_BH, FL_PH_FAR, FL_NPHASE };
fl_status fl_set_timing(fl_ctx *ctx, int enable);
/* Graph replay of fl_fa2_run and concurrent components in fl_layout (on by
 * default); 0 runs every iteration as eager launches on the context's stream
 * (the same results, bitwise). */
fl_status fl_set_graphs(fl_ctx *ctx, int enable);
fl_status fl_get_timing(fl_ctx *ctx, double *ms, int64_t *counts);

#ifdef __cplusplus
}
#endif

#endif /* FA2LAY_H */
