/*
 * rdist.h -- C ABI of the MI355X (gfx950) R-distance engine.
 *
 * The engine computes, for a directed graph with adjacency A and a gain
 * gamma, the R-distance matrix of Jing & Meister (arXiv 2308.07403):
 *
 *     Y = (I - gamma*A)^{-1}                      (Sec. 2, Eq. Y-defined)
 *     R = log_gamma Y,  D = ceil(R - eta)         (Eq. R-defined; Sec. 4.1.1,
 *                                                  rounded distance function)
 *     Y == 0  ->  D = RDIST_UNREACHABLE           (no walk: Eq. Y-series)
 *
 * and the greedy next hop toward a goal g (Sec. 4.2, Eq. descent):
 *
 *     i <- argmax over successors j of i of Y[g, j]   (ascent on Y, as in the
 *                                                       proof of Theorem 4)
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Adjacency (Sec. 2, adjacency equation): A is n x n, row-major uint8,
 *    A[i*n + j] = 1 iff there is a directed edge from node j to node i.
 *    Entries must be 0 or 1 and the diagonal must be 0 (Sec. 3.1 footnote).
 *  - D is n x n, row-major int16: D[i*n + j] is the R-distance from j to i.
 *    eta = 1e-9 (ceil at exact integers: an exactly representable integer R
 *    rounds to itself).  D is clamped to [-32767, 32766] and counted as
 *    saturated when clamped; RDIST_UNREACHABLE (0x7FFF) marks Y == 0.
 *  - Out-degree of node j is the column sum sum_i A[i*n + j]; Delta is its
 *    maximum (Theorem 2).
 *  - gamma > 0: explicit gain, must satisfy 0 < gamma < 1.
 *    gamma < 0: AUTO, gamma := |gamma| / Delta (one IEEE double division),
 *    or |gamma| when the graph has no edge.
 *  - Gate: the solve requires gamma * Delta < 1.  Then I - gamma*A is
 *    column-wise strictly diagonally dominant, so elimination needs no
 *    pivoting, Y >= 0 entrywise, and greedy ascent on Y reaches the goal
 *    (Theorem 4's hypothesis).  Graphs that fail it are not solved: their
 *    status is RDIST_E_NOT_DD and D is filled with RDIST_UNREACHABLE.
 *  - Pointers named *_dev are device pointers on the context's device; the
 *    caller allocates and owns them.  Other pointers are host pointers.
 *  - Every call is asynchronous on the caller's HIP stream (hipStream_t
 *    passed as void*; NULL = the null stream).  Argument errors are
 *    returned synchronously.  Conditions only the device can detect (bad
 *    adjacency, NOT_DD) are reported in rdist_info.status, which is valid
 *    once the stream has reached the end of the call.  rdist_info should be
 *    pinned host memory (hipHostMalloc); with pageable memory the call
 *    returns only after the device has finished it.
 *  - No C++ exception crosses this interface.  A context may be used from
 *    several threads only if created with RDIST_THREADSAFE.
 */
#ifndef RDIST_H
#define RDIST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rdist_ctx_s *rdist_ctx;
typedef struct rdist_graph_s *rdist_graph;

typedef enum rdist_status {
    RDIST_OK = 0,
    RDIST_E_ARG = 1,     /* invalid argument (synchronous) */
    RDIST_E_ADJ = 2,     /* A has an entry other than 0/1 or a self-loop */
    RDIST_E_NOT_DD = 3,  /* gamma * Delta >= 1: the gate refused the graph */
    RDIST_E_NOMEM = 4,   /* device allocation failed or the request can never fit the budget */
    RDIST_E_AGAIN = 5,   /* the HBM budget is currently in use; retry after releases */
    RDIST_E_HIP = 6,     /* a HIP runtime call failed (see rdist_last_error) */
    RDIST_E_STATE = 7    /* a handle was used in a way its state does not allow */
} rdist_status;

#define RDIST_UNREACHABLE 0x7FFF

/* ---- flags for rdist_solve / rdist_solve_batched ---- */
#define RDIST_F64 0x0u              /* FP64 inversion (default) */
#define RDIST_MIXED_F32 0x1u        /* FP32-MFMA trailing updates, FP64 panel,
                                       per-entry certification, FP64 recompute */
#define RDIST_KEEP_Y 0x10u          /* keep Y resident in a graph handle (for rdist_next_hop) */
#define RDIST_PLAN_SMALL 0x100u     /* force the single-workgroup register-resident plan (n <= 128) */
#define RDIST_PLAN_BLOCKED 0x200u   /* force the blocked multi-kernel plan, whatever n */
#define RDIST_UNFUSED_EPILOGUE 0x400u /* run the readout as a standalone pass over Y */
#define RDIST_BLOCK_128 0x800u      /* blocked plan: force block width b = 128 */
#define RDIST_BLOCK_256 0x1000u     /* blocked plan: force block width b = 256 (default for n > 6400) */
#define RDIST_NO_GRAPH 0x2000u      /* rdist_solve_batched: launch eagerly, no HIP graph capture or replay */
#define RDIST_WEIGHTED 0x4000u      /* rdist_solve: A_dev holds positive integer weights (Sec. 3.2) */

/* ---- flags for rdist_create ---- */
#define RDIST_THREADSAFE 0x1u

typedef struct rdist_info {
    int32_t status;          /* rdist_status detected for this graph */
    int32_t delta;           /* largest out-degree */
    double gamma;            /* gain actually used */
    int64_t n_unreachable;   /* entries with Y == 0 */
    int64_t n_subnormal;     /* entries with 0 < Y < DBL_MIN (reachable, low precision) */
    int64_t n_saturated;     /* entries clamped to the int16 range */
    int64_t n_ambiguous;     /* entries whose R - eta lies within 1e-10 of an integer */
    int64_t n_negative;      /* entries with Y < 0 (never expected under the gate) */
    int64_t n_uncertified;   /* RDIST_MIXED_F32: entries recomputed in FP64;
                                edge change: entries its error bounds lost */
    double fallback_fraction;/* RDIST_MIXED_F32: n_uncertified / n^2;
                                edge change: 1 when it re-inverted the graph */
} rdist_info;

/*
 * Creates a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context and its graph handles may hold (0: no bound).
 * tile_cache_path (nullable) names a JSON file of tuned launch shapes written
 * by the autotuner; missing or unreadable files fall back to built-in shapes.
 * flags: 0 or RDIST_THREADSAFE.  Returns RDIST_E_ARG for a bad device.
 */
rdist_status rdist_create(rdist_ctx *out, int device, size_t hbm_budget_bytes,
                          const char *tile_cache_path, uint32_t flags);

/* Frees everything the context owns, including graph handles not yet released.
 * The caller must have synchronised every stream the context was used on. */
void rdist_destroy(rdist_ctx ctx);

/*
 * One graph: D = ceil(log_gamma (I - gamma*A)^{-1} - eta) (see above).
 *   A_dev : n x n uint8 adjacency (read only).
 *   n     : 1 <= n <= 65536.
 *   gamma : explicit (0,1) or AUTO (< 0, |gamma| in (0, 1]).
 *   flags : RDIST_F64 or RDIST_MIXED_F32, optionally | RDIST_KEEP_Y and a plan flag.
 *           With RDIST_WEIGHTED (Sec. 3.2, extension to weighted graphs),
 *           A_dev[i*n + j] is the positive integer weight W_ij of the edge
 *           j -> i (1 .. 255; 0: no edge, gamma^inf = 0), Y = (I - gamma^W)^{-1}
 *           elementwise-powered, and D is the weighted distance (Eq.
 *           distance-function-integer, same readout).  Delta counts out-edges
 *           and the gate is gamma * Delta < 1 as for 0/1 graphs (every column
 *           sum of gamma^W is then below 1); self-loops are refused
 *           (RDIST_E_ADJ).  Always the blocked plan; not with
 *           RDIST_MIXED_F32 or RDIST_PLAN_SMALL, nor in rdist_solve_batched.
 *   D_dev : n x n int16 output, written by the device.
 *   keep  : with RDIST_KEEP_Y, receives a graph handle owning Y and the
 *           out-neighbour lists (release with rdist_graph_release); else NULL.
 *   info  : nullable host pointer, one rdist_info.
 *   stream: hipStream_t.
 * Errors: RDIST_E_ARG (synchronous), RDIST_E_NOMEM/RDIST_E_AGAIN (workspace
 * does not fit the budget), RDIST_E_HIP.
 */
rdist_status rdist_solve(rdist_ctx ctx, const uint8_t *A_dev, int32_t n, double gamma,
                         uint32_t flags, int16_t *D_dev, rdist_graph *keep,
                         rdist_info *info, void *stream);

/*
 * Many independent graphs per call (Sec. 3, Eq. of the inverse, applied to
 * each graph on its own).  Graphs with n <= T (T = 128 unless tuned) go to
 * one persistent launch in which each workgroup solves whole graphs, longest
 * first; graphs with T < n <= 4096 take the blocked steps together, one
 * launch per step phase for the whole set (128-wide blocks; a large graph's
 * tiles spread over the whole device); larger graphs are solved one after
 * another with the blocked plan.  A graph's arithmetic does not depend on the
 * rest of the batch, only on T.
 * Host arrays of length `count` (0 .. 2^20): n[g], A_dev[g], gamma[g], D_dev[g]
 * (device pointers), info[g] (nullable array, preferably pinned).  flags as
 * rdist_solve plus RDIST_NO_GRAPH (RDIST_KEEP_Y fills keep[g]).  Each
 * graph's status is in info[g].status.
 * Without RDIST_KEEP_Y / RDIST_NO_GRAPH the launch sequence is captured into
 * a HIP graph keyed by (stream, flags, n[], A_dev[], gamma[], D_dev[]) and
 * replayed on later identical calls; the context keeps the last 4 such plans
 * and their device buffers (about n^2 + 256 n doubles per graph).  With a
 * tile cache file (rdist_create), the first batch of each size class is
 * first timed under every candidate T and persistent grid (the call then
 * blocks until those trial runs end) and the fastest is recorded in the file.
 */
rdist_status rdist_solve_batched(rdist_ctx ctx, int32_t count, const int32_t *n,
                                 const uint8_t *const *A_dev, const double *gamma,
                                 uint32_t flags, int16_t *const *D_dev, rdist_graph *keep,
                                 rdist_info *info, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * solve of rdist_solve for graphs with n <= RDIST_NOALLOC_MAX_N, with no
 * device allocation, no stream or event creation and no event timing.  Its
 * kernels use a static device scratch of about 17.6 MiB (the blocked plan's
 * matrix and step buffers for n = 1024, plus out-degrees and the device
 * info) that every GPU the library runs on holds until the process ends;
 * rdist_create takes its address for the context's device.  Every call on
 * one GPU shares that scratch, whatever the context: calls that overlap on
 * one GPU (on different streams, contexts or threads) race and must be
 * serialised by the caller.  All steps run on `stream` in order (no
 * lookahead stream), so a solve may take longer than with rdist_solve; D and
 * info are those of rdist_solve with the same arguments (bit for bit).
 *   flags: RDIST_F64 with optional RDIST_WEIGHTED, RDIST_PLAN_SMALL,
 *          RDIST_PLAN_BLOCKED, RDIST_UNFUSED_EPILOGUE, RDIST_BLOCK_128,
 *          RDIST_BLOCK_256 as for rdist_solve; RDIST_MIXED_F32, RDIST_KEEP_Y
 *          and RDIST_NO_GRAPH are refused (RDIST_E_ARG).
 *   info : nullable; pinned host memory (a pageable target makes the copy
 *          synchronous).
 * RDIST_E_ARG for n outside [1, RDIST_NOALLOC_MAX_N] or the flags above;
 * RDIST_E_HIP if the scratch's device address could not be taken.
 */
#define RDIST_NOALLOC_MAX_N 1024
rdist_status rdist_solve_noalloc(rdist_ctx ctx, const uint8_t *A_dev, int32_t n, double gamma, uint32_t flags,
                                 int16_t *D_dev, rdist_info *info, void *stream);

/*
 * Greedy local pursuit on a kept graph (Sec. 4.2, Eq. descent; Theorem 4 and
 * its corollary).  Each hop moves from node i to the successor j of i (edge
 * i -> j) with the largest Y[goal, j], the lowest j on exact ties.  For query
 * q with start cur_dev[q] and goal goal_dev[q]:
 *   max_hops == 1 (next hop):  out_dev[q] = the next node from the start; the
 *     start itself when it is the goal; -1 when no successor has
 *     Y[goal, j] > 0 (goal unreachable) or a node id is out of range.
 *   max_hops > 1 (paths), rows of max_hops + 1 entries:
 *     out_dev[q*(max_hops+1) + 0] = start,
 *     out_dev[q*(max_hops+1) + h] = node reached after h hops;
 *     the row ends at the goal and the remaining entries are -1.  A hop that
 *     finds no successor with Y[goal, j] > 0 writes -1 and ends the row; an
 *     out-of-range start or goal leaves the whole row -1.
 * q >= 0, 1 <= max_hops <= 65535.  Needs a graph kept with RDIST_KEEP_Y.
 */
rdist_status rdist_next_hop(rdist_ctx ctx, rdist_graph g, const int32_t *cur_dev,
                            const int32_t *goal_dev, int32_t q, int32_t max_hops,
                            int32_t *out_dev, void *stream);

/* Frees a kept graph's Y and lists and returns their bytes to the budget.
 * The caller must have synchronised streams that still use the graph. */
void rdist_graph_release(rdist_graph g);

/*
 * Device view of a kept graph's Y (read only; valid until release):
 * Y[i*ld + j] for 0 <= i, j < n.  Returns RDIST_E_ARG for a NULL handle.
 */
rdist_status rdist_graph_y(rdist_graph g, const double **Y_dev, int32_t *n, int32_t *ld);

/*
 * Edge change on a kept graph without a new inversion (the dynamic
 * re-planning of the Discussion, Applications): the edge src -> dst gets
 * weight `weight` (0 removes it; 0/1 for graphs solved without
 * RDIST_WEIGHTED, 0 .. 255 with it).  With delta the change of the entry
 * gamma^w of X (Sec. 3.2), Y becomes
 *   Y + f Y[:, dst] Y[src, :],  f = delta / (1 - delta Y[src, dst])
 * (Sherman-Morrison), i.e. (I - X')^{-1} for the changed graph at the graph's
 * gain, in one pass over Y; the graph's adjacency, out-degrees and successor
 * lists follow.  D_dev (nullable, n x n int16) receives the changed graph's D.
 *
 * Every entry of Y carries a bound on its relative error (2 bytes per entry,
 * allocated by the first change and counted in the budget), carried through
 * each change.  Entries whose bound no longer vouches for them (a removal
 * that cancels an entry to zero or to its rounding error; a D readout whose
 * integer boundary lies within the bound) are counted in
 * info->n_uncertified, and the call then re-inverts the changed graph from
 * its kept adjacency (info->fallback_fraction = 1, info's counters those of
 * the new inversion).  So D_dev equals, up to the readout's own ambiguity
 * band, the D of a fresh rdist_solve of the changed graph at the same gain.
 *
 * The change is applied only if the changed graph passes the gate
 * gamma * Delta' < 1; otherwise Y, D_dev and the graph stay as they were and
 * info->status is RDIST_E_NOT_DD.  info (nullable, host) receives the call's
 * status, Delta', gamma and D's counters.  RDIST_E_ARG for bad nodes or
 * weight.  The call returns when the change is complete (it waits for the
 * stream); changes to one graph must not overlap.
 */
rdist_status rdist_graph_update_edge(rdist_ctx ctx, rdist_graph g, int32_t src, int32_t dst, int32_t weight,
                                     int16_t *D_dev, rdist_info *info, void *stream);

/*
 * Several edge changes, applied in order (a later change to the same edge
 * wins): src[e] -> dst[e] gets weight[e] (host arrays of count entries,
 * rules as rdist_graph_update_edge).  Changes go in chunks of up to 8 per
 * pass over Y: change a of a chunk is the rank-one step of the graph left by
 * changes 0 .. a-1 (its column and row of Y are built from Y and the earlier
 * terms), and one pass adds all of a chunk's terms to Y, carrying each
 * entry's error bound through every term; re-inversion as for one change.
 * A chunk is applied only if every intermediate graph passes the gate (a
 * bound on its Delta: the largest of Delta and every out-degree a change of
 * the chunk passes through); otherwise info->status is RDIST_E_NOT_DD, that
 * chunk and the rest are not applied, the chunks before it stay applied, and
 * D_dev is left as it was.  D_dev (nullable) receives the final graph's D.
 * info->n_uncertified sums the lost entries of all chunks,
 * info->fallback_fraction is 1 if any chunk re-inverted.  count = 0 changes
 * nothing: D_dev is not written and info receives the graph's status,
 * Delta and gamma (its counters zero).
 * Synchronous.
 */
rdist_status rdist_graph_update_edges(rdist_ctx ctx, rdist_graph g, int32_t count, const int32_t *src,
                                      const int32_t *dst, const int32_t *weight, int16_t *D_dev,
                                      rdist_info *info, void *stream);

/*
 * Goal rows without an inversion (the recurrent network of Sec. 2 and its
 * walk series, Eq. Y-series): for each of q goals g = goals[k], row k of the
 * output is row g of Y = (I - X)^{-1}, the fixed point of
 *   y_j = [j == g] + sum over successors i of j of x y_i,  x = gamma^w of edge j -> i
 * (the network on the reversed edges, driven at the goal), found by
 * iterating from y = 0 until a step changes no entry (the iterates never
 * decrease, so this takes finitely many steps).  Row g is what the next hop
 * toward g reads (Sec. 4.2), so greedy paths need only these rows.
 *
 * Graph: successor lists in CSR, on the device: the successors of node j
 * are succ_idx[succ_ptr[j] .. succ_ptr[j+1]) (int64 offsets, int32 ids,
 * strictly increasing, no self-loop; succ_ptr[0] = 0, succ_ptr[n] = nnz).
 * weights (nullable, device, nnz bytes in 1..255): integer edge weights
 * (Sec. 3.2); NULL means weight 1.  gamma: explicit in (0, 1), or < 0 for
 * AUTO = |gamma| / Delta (Delta = the largest out-degree).  Malformed lists
 * give info->status RDIST_E_ADJ, a failed gate RDIST_E_NOT_DD; then Y rows
 * are 0 and D rows the sentinel.  goals (device, q ids; an id outside
 * [0, n) gives a row of zeros).
 *
 * Y_dev (nullable, device, q x n doubles, row k at Y_dev + k*n) and D_dev
 * (nullable, device, q x n int16: the readout of rdist_solve) receive the
 * rows; steps (nullable, host) the number of iteration steps.  Needs 2 n q'
 * doubles of workspace (q' = q rounded up to a power of two up to 64, then
 * to a multiple of 64).  1 <= q <= 65535.  The call waits for its stream
 * (it reads back, every 16 steps, whether the rows have settled).
 */
rdist_status rdist_goal_rows(rdist_ctx ctx, int32_t n, const int64_t *succ_ptr, const int32_t *succ_idx,
                             int64_t nnz, const uint8_t *weights, double gamma, const int32_t *goals,
                             int32_t q, double *Y_dev, int16_t *D_dev, int32_t *steps, rdist_info *info,
                             void *stream);

/*
 * Greedy paths over goal rows (Sec. 4.2): query k walks from starts[k]
 * toward goals[k], each hop to the successor j (CSR as above) with the
 * largest Y_rows[k*n + j], the lowest j on exact ties; out_dev layout and
 * ending as rdist_next_hop (q int32 for max_hops == 1, else q x (max_hops+1)).  Y_rows as written by
 * rdist_goal_rows for the same goals (successor offsets are clamped to
 * [0, nnz), ids outside [0, n) skipped).  Asynchronous on the stream.
 */
rdist_status rdist_goal_paths(rdist_ctx ctx, int32_t n, const int64_t *succ_ptr, const int32_t *succ_idx,
                              int64_t nnz, const double *Y_rows, const int32_t *goals, const int32_t *starts, int32_t q,
                              int32_t max_hops, int32_t *out_dev, void *stream);

/*
 * Bounds on the gain for one graph (Sec. 4.1: the critical gain
 * Eq. critical-gain, Theorem 2's sufficient bound, Theorem 3's bound for
 * trees; Sec. 5.1: the machine-precision bound Eq. gamma-precision), to
 * choose gamma before a solve.  rho(A) is bracketed by power iteration on
 * A + I with Collatz-Wielandt ratios, which bound the spectral radius for
 * any positive vector: rho_lo <= rho(A) <= rho_hi rigorously (rounding
 * included); on graphs that are not strongly connected the lower bound may
 * stay loose.
 */
typedef struct rdist_gain_report {
    int32_t status;          /* RDIST_OK, or RDIST_E_ADJ (entries other than 0/1, or a self-loop) */
    int32_t delta;           /* largest out-degree Delta */
    int32_t steps;           /* power-iteration steps taken */
    int32_t diameter;        /* d used below: the caller's, else n - 1 (a bound) */
    double rho_lo, rho_hi;   /* bracket of the spectral radius of A (0 <= rho <= Delta) */
    double gamma_c_lo, gamma_c_hi; /* 1 / rho_hi and 1 / rho_lo: the critical gain (HUGE_VAL for 0) */
    double gamma_gate;       /* 1 / Delta: gains below it pass this library's gate gamma Delta < 1 */
    double gamma_global;     /* Theorem 2: below 1 / (Delta + Delta^(d-1)) D is globally correct */
    double gamma_tree;       /* Theorem 3 (undirected trees): (-1 + sqrt(1 + 4 Delta (d+2))) / (2 Delta (d+2)) */
    double gamma_precision;  /* Eq. gamma-precision: gamma^d stays above the smallest double above this */
} rdist_gain_report;

/*
 * A_dev: n x n adjacency as for rdist_solve (0/1).  diameter: the graph's
 * diameter if the caller knows it, else 0 (then n - 1 is used).  Iterates
 * at most max_steps steps, stopping once rho_hi - rho_lo <= rel_tol rho_hi.
 * Synchronous (reads the bounds back every 16 steps).
 */
rdist_status rdist_gain_bounds(rdist_ctx ctx, const uint8_t *A_dev, int32_t n, int32_t diameter,
                               int32_t max_steps, double rel_tol, rdist_gain_report *out, void *stream);

/*
 * Per-entry certificate of a kept graph's D (Sec. 3.1, Eq. Y-series-trunc
 * with the walk-count bound Eq. Nijk-limit, as in the proof of Theorem 2):
 * with k = D_ij the readout of Y_ij, the true distance is at least k, and a
 * true distance of k + 1 or more would give
 *   Y_ij <= gamma^(k+1) Delta^k / (1 - gamma Delta)           (Eq. Y-bracket).
 * An entry with Y_ij above that bound by a relative margin for Y's error
 * has D_ij equal to the graph distance.  The margin is the largest of
 * 2^-30, the inversion's error bound 8 n u / (1 - gamma Delta) (u = 2^-53)
 * and, when Y carries edge changes made since its last inversion, the cap
 * 2^-20 on the error bounds of changed entries.  Y_ij = 0 certifies
 * "unreachable" when e gamma^(n-1) > DBL_MIN (then no reachable entry can
 * underflow); entries below DBL_MIN are not certified.  mask_dev
 * (nullable, device, n x n bytes) receives 1 for certified entries;
 * *n_certified (host) their count.  For graphs solved with RDIST_WEIGHTED
 * the bound covers positive integer weights: a true distance of k + 1 or
 * more makes every walk of l edges weigh at least max(l, k + 1), so
 *   Y_ij <= gamma^(k+1) (Delta^(k+1) - 1) / (Delta - 1)
 *           + (gamma Delta)^(k+2) / (Delta (1 - gamma Delta))
 * ((k + 1) gamma^(k+1) + gamma^(k+2) / (1 - gamma) for Delta = 1), with
 * Delta the largest number of out-edges.  Synchronous.
 */
rdist_status rdist_certify(rdist_ctx ctx, rdist_graph g, uint8_t *mask_dev, int64_t *n_certified, void *stream);

/*
 * Standalone readout over a caller-provided Y (the unfused form of the
 * epilogue): D[i*n + j] from Y_dev[i*ld + j] for 0 <= i, j < n with the
 * given gain (0 < gamma < 1).  info (nullable) receives the counters.
 */
rdist_status rdist_epilogue(rdist_ctx ctx, const double *Y_dev, int32_t n, int32_t ld,
                            double gamma, int16_t *D_dev, rdist_info *info, void *stream);

/*
 * ---- Serving: a request loop with continuous batching ----
 *
 * A server owns `slots` HIP streams of its context (each with its own
 * workspace) and a queue.  rdist_server_submit only queues a request;
 * rdist_server_poll (non-blocking) collects finished requests and then
 * dispatches queued ones, oldest first, while a slot is free and the HBM
 * footprint of the requests in flight stays within the server's budget:
 * the requests with n <= 4096 that are waiting, both kinds, are solved
 * together in one batched solve on one slot (as rdist_solve_batched with
 * T = 128, eager launches), up to max_batch of them; a path request keeps
 * its Y in the slot's buffers and its greedy paths (as rdist_next_hop) run
 * on the slot right after the batch.  While at most 8 requests wait, one
 * with n > 1024 stays out of the batch.  A request above 4096, and one with
 * n > 1024 that is not batched, runs on a slot of its own as
 * rdist_solve, its greedy paths (as rdist_next_hop) on the Y that solve
 * leaves in the slot's workspace, so no graph handle is made or released
 * per request.  Requests on different slots run concurrently on the
 * device.  A slot's device buffers grow with
 * headroom and are kept until rdist_server_destroy.  Results are
 * bit-for-bit those of the same request solved alone (rdist_solve_batched
 * with count 1 and no tile cache for n <= 4096, rdist_solve above; for
 * n <= 4096 the two give the same bits): every slot has its own workspace
 * and no kernel's arithmetic depends on what else runs.  For the paper's query modes see Sec. 4.1 (full distance
 * matrix) and Sec. 4.2 (greedy routing).
 */
typedef struct rdist_server_s *rdist_server;

#define RDIST_QUERY_D 0       /* full n x n D */
#define RDIST_QUERY_PATHS 1   /* greedy paths for q (start, goal) pairs */

typedef struct rdist_request {
    int64_t id;                /* caller's tag, reported by rdist_server_poll */
    const uint8_t *A_dev;      /* n x n adjacency (device); kept alive by the caller until done */
    int32_t n;
    int32_t kind;              /* RDIST_QUERY_D or RDIST_QUERY_PATHS */
    double gamma;              /* explicit or AUTO (< 0), as rdist_solve */
    int16_t *D_host;           /* RDIST_QUERY_D: n*n int16 host buffer (pinned) receiving D */
    const int32_t *cur_host;   /* RDIST_QUERY_PATHS: q start nodes (host) */
    const int32_t *goal_host;  /* RDIST_QUERY_PATHS: q goal nodes (host) */
    int32_t q;                 /* RDIST_QUERY_PATHS: pairs, 0 <= q <= 4096 */
    int32_t max_hops;          /* RDIST_QUERY_PATHS: 1 .. 65535 */
    int32_t *paths_host;       /* RDIST_QUERY_PATHS: host buffer (pinned) of q int32 for max_hops == 1,
                                  else q*(max_hops+1); layout as rdist_next_hop's out */
    rdist_info *info_host;     /* nullable: the solve's info, valid once the request is reported done */
} rdist_request;

/* Creates a server on ctx with `slots` streams (1..64), an HBM budget for
 * the footprint of requests in flight (0: unbounded) and a batch limit
 * (1..1024).  A request's footprint is 8 np^2 + 4096 np bytes (np = n
 * rounded up to 128), twice that for path requests (the kept Y). */
rdist_status rdist_server_create(rdist_ctx ctx, int32_t slots, size_t hbm_budget_bytes, int32_t max_batch,
                                 rdist_server *out);

/* Queues a copy of *req.  RDIST_E_ARG for bad fields; RDIST_E_NOMEM when
 * its footprint alone exceeds the budget (it could never be admitted). */
rdist_status rdist_server_submit(rdist_server s, const rdist_request *req);

/* Finished requests since the last call: their ids into done_ids (up to
 * max), their count into *n_done; then dispatches what fits.  Never blocks
 * on the device.  A request whose solve failed to launch is reported done
 * with info_host->status set (when given) and counted in rdist_server_stats. */
rdist_status rdist_server_poll(rdist_server s, int64_t *done_ids, int32_t max, int32_t *n_done);

typedef struct rdist_server_stats {
    int64_t submitted, completed, failed;
    int64_t queued, in_flight;         /* now */
    int64_t batches, batched_requests; /* batched dispatches and the requests they carried */
    int64_t max_in_flight;             /* most requests in flight at once */
    size_t footprint_in_flight, max_footprint_in_flight;
} rdist_server_stats;

rdist_status rdist_server_stats_get(rdist_server s, rdist_server_stats *out);

/* Waits for everything in flight, then frees the server (not the context). */
void rdist_server_destroy(rdist_server s);

/* Per-kernel timing collected with HIP events on the launching stream. */
typedef struct rdist_kernel_stats {
    int64_t launches;        /* timed launches since the last reset */
    double total_ms;         /* summed event-to-event duration */
    double flops;            /* algorithmic flops of those launches */
    double bytes;            /* algorithmic bytes of those launches */
} rdist_kernel_stats;

#define RDIST_K_UPDATE 0      /* trailing rank-b update over all tiles outside the next block's
                                 row and column (the FP64/FP32 MFMA hot loop); batched plans
                                 (eager launches, RDIST_NO_GRAPH): the level plan's rest tiles */
#define RDIST_K_PANEL 1       /* diagonal-block inverse */
#define RDIST_K_ROWCOL 2      /* pivot row/column block preparation */
#define RDIST_K_INGEST 3      /* adjacency -> M, degrees, gate */
#define RDIST_K_EPILOGUE 4    /* standalone readout */
#define RDIST_K_SMALL 5       /* single-workgroup solve */
#define RDIST_K_BATCHED 6     /* persistent batched solve */
#define RDIST_K_NEXTHOP 7     /* next-hop queries */
#define RDIST_K_CERTIFY 8     /* mixed precision: certification + recompute; rdist_certify */
#define RDIST_K_UPDATE_EDGE 9 /* update of the next block's row and column (lookahead) and the
                                 last, readout-fused update; batched plans (eager launches): the
                                 level plan's diagonal and edge tiles */
#define RDIST_K_MIXED_GEMM 10  /* mixed precision: the FP32 trailing updates (row products, -U^T and
                                  P^T count as RDIST_K_ROWCOL) */
#define RDIST_K_REFINE 11     /* mixed precision: residual, correction product and recompute */
#define RDIST_K_EDGE_UPDATE 12 /* rdist_graph_update_edge: the rank-1 pass over Y (and D) */
#define RDIST_K_ROWS_STEP 13   /* rdist_goal_rows: one iteration step */
#define RDIST_K_COUNT 14

/* Per-kernel event timing: 0 off, 1 every kernel class, or a mask of
 * RDIST_TIMING_CLASS(k) bits timing only those classes (each timed launch
 * records two events on its stream, so a narrow mask disturbs a timed run
 * less).  Enabling resets the counters; RDIST_E_ARG for a negative value. */
#define RDIST_TIMING_CLASS(k) (2 << (k))
rdist_status rdist_set_timing(rdist_ctx ctx, int enable);
/* Holds (hold != 0) or resumes event timing without draining or resetting
 * anything: launches enqueued while held are not timed, the counters and
 * the timed launches still in flight are kept.  Lets a caller time a sample
 * of the launches of a run it does not want to stall.  Cheap, never
 * synchronises; RDIST_E_ARG for a NULL context. */
rdist_status rdist_timing_hold(rdist_ctx ctx, int hold);
/* Reads the counters of kernel class `which` (RDIST_K_*); synchronises the
 * streams the timed launches ran on. */
rdist_status rdist_kernel_stats_get(rdist_ctx ctx, int which, rdist_kernel_stats *out);

/* Bytes of device memory currently held by the context and its graphs. */
size_t rdist_hbm_in_use(rdist_ctx ctx);

/* Thread-local description of the last failure in this thread ("" if none). */
const char *rdist_last_error(void);
const char *rdist_status_string(rdist_status s);

#ifdef __cplusplus
}
#endif
#endif /* RDIST_H */
