/*
 * skim.h -- C ABI of the MI355X (gfx950) library for sketch-based influence
 * computation under binary Independent Cascade (Cohen, Delling, Pajor,
 * Werneck, "Sketch-based Influence Maximization and Computation", 2014).
 *
 * Conventions shared by every call
 * --------------------------------
 * Graph: a directed graph as a forward CSR (out-edges).  row_ptr[n+1]
 *   (uint64, row_ptr[0] = 0, non-decreasing, row_ptr[n] = m), col[m] (uint32
 *   heads, strictly increasing within a row: no duplicate edges), no
 *   self-loops, every head < n.  n >= 1, n * 64 < 2^32.
 * Edge probabilities (binary IC, Section 1 and 2 of the paper): thr[m]
 *   (uint32) encodes p = (thr + 1) / 2^32; the edge (u -> v) is live in
 *   instance i iff the 32-bit coin of (seed, u, v, i) is <= thr.  A
 *   probability p is encoded as floor((2^32 - 1) * p); p = 1 is 0xFFFFFFFF.
 * Instances: l in [1, 64] Monte-Carlo instances G^(i) (Section 2); they are
 *   never stored by the caller: ranks and coins come from SplitMix64
 *   (Steele, Lea, Flood 2014) seeded with `seed`:
 *     SM(c)   = mix64(seed + (c + 1) * 0x9E3779B97F4A7C15)
 *     r(v, i) = SM(64 v + i)                      rank of node-instance pair
 *     coin    = high (i even) / low (i odd) 32 bits of
 *               SM(2^62 + 32 (u n + v) + floor(i / 2))
 * Sketch k: 2 <= k <= 256 (skim_greedy: 2 <= k <= 65535).
 * Pointers: every array argument is a DEVICE pointer (HIP global memory on
 *   the current device) unless stated otherwise.  The caller owns every
 *   buffer; inputs must stay valid and unmodified until the stream reaches
 *   the end of the call's work.  `stream` is a hipStream_t (NULL = the
 *   default stream).
 * Errors: argument and graph validation runs before any result is written;
 *   on failure the call returns SKIM_EINVAL and leaves outputs untouched.
 *   A HIP runtime failure returns SKIM_EDEVICE; an allocation failure
 *   SKIM_ENOMEM.  skim_last_error() describes the last failure of the
 *   calling thread.  Nothing throws across this boundary.
 * Synchronisation: skim_sketches_query, skim_sketches_create and
 *   skim_query_plan_launch only enqueue work on `stream` (results are
 *   complete when the stream reaches them).  The other calls may synchronise
 *   `stream` internally (they read small device counters to schedule their
 *   work: the build's search is driven level by level from the host); their
 *   results are complete when they return SKIM_OK.
 * Determinism: for the same inputs every call returns the same bits, on any
 *   stream and in any batch mix.
 */
#ifndef SKIM_H
#define SKIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SKIM_ABI_VERSION 9u

typedef enum {
    SKIM_OK = 0,
    SKIM_EINVAL = 1,       /* bad argument or invalid graph               */
    SKIM_ENOMEM = 2,       /* device allocation failed                    */
    SKIM_EDEVICE = 3,      /* HIP runtime or kernel failure               */
    SKIM_EBUSY = 4,        /* server queue / budget full, retry later     */
    SKIM_EUNSUPPORTED = 5  /* valid request outside the supported limits  */
} skim_status;

typedef struct {
    uint32_t n;               /* nodes                                     */
    uint64_t m;               /* edges                                     */
    const uint64_t *row_ptr;  /* [n+1] device                              */
    const uint32_t *col;      /* [m]   device                              */
    const uint32_t *thr;      /* [m]   device                              */
} skim_graph;

/* ABI version (SKIM_ABI_VERSION of the built library). */
uint32_t skim_abi_version(void);

/* Text of the last failure on the calling thread ("" if none). */
const char *skim_last_error(void);

/*
 * Fault injection, for tests of the error paths.  Host side only: nothing
 * is done wrong on the device.  what = SKIM_FAULT_ALLOC: the next `count`
 * device allocations the library makes fail as if the device were out of
 * memory (the call that makes one returns SKIM_ENOMEM and writes no
 * result); SKIM_FAULT_SERVE: the next `count` batch copies or launches of
 * the serving loop are treated as failed (the batch's requests complete
 * with status -5 and its slot is freed); SKIM_FAULT_IC_RECORDS: the next
 * `count` skim_build_ic_sketches calls give their single record-appending
 * pass room for one record, so that they take the counting path (same
 * results).  count = 0 disarms.  Process-wide.  SKIM_EINVAL for an unknown
 * kind.
 */
#define SKIM_FAULT_ALLOC 1u
#define SKIM_FAULT_SERVE 2u
#define SKIM_FAULT_IC_RECORDS 3u
skim_status skim_debug_inject(uint32_t what, uint32_t count);

/*
 * skim_build_sketches -- combined bottom-k reachability sketches of every
 * node over l instances (Section 3, eq. combinedrs; built as Section 5.2,
 * Algorithm 2, describes: per instance, pairs by increasing rank, reverse
 * searches pruned at nodes whose instance-local sketch already holds k
 * ranks, merged into the global bottom-k sketch) and, optionally, the
 * influence estimate of every node (Section 3, eq. combinedthresh; Section
 * 5.1 divides by l).
 *
 *   ranks [n*k] out, device: row v = X_v ascending, padded with UINT64_MAX.
 *   size  [n]   out, device: |X_v| = min(k, |R_v|).
 *   est   [n]   out, device, may be NULL: |X_v| / l if |X_v| < k, else
 *         ((k-1) / rho(tau_v)) / l with tau_v = ranks[v*k + k-1] and
 *         rho(T) = ((T >> 11) + 1) * 2^-53 (IEEE double, correctly rounded).
 *   work  [6]   out, HOST, may be NULL: work the device did, in order:
 *         accepted visits (node-instance-source), live-edge scans, records
 *         kept for the merge, rank windows processed, restarts of the
 *         window phase after a buffer overflow, and the overflow bits.
 */
skim_status skim_build_sketches(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                uint64_t *ranks, uint32_t *size, double *est,
                                uint64_t *work, void *stream);

/*
 * skim_build_sketches_perm -- combined bottom-k sketches with structured
 * permutation ranks instead of hashed ones (Section 3.1, structured
 * permutation ranks): the n l pairs take positions 1 .. n l in l chunks of n
 * positions; chunk c holds every node once, in the order of
 * h_c(v) = SM(2^63 + c n + v); the instance a node takes in chunk c is drawn
 * from those it has not taken before (instance i goes to the chunk given by
 * the place of SM(2^61 + 64 v + i) among the node's l keys).  The instances
 * (live edges) are those of skim_build_sketches.  Only the first
 * min(k, l) n positions can enter a sketch.
 *   ranks [n*k] out, device: X_v, the k smallest positions (as uint64) of
 *         the pairs v reaches, ascending, padded with UINT64_MAX.
 *   size  [n]   out, device; est [n] out, device, may be NULL:
 *         |X_v| / l if |X_v| < k, else (1 + (k-1)(D-1)/(T-1)) / l with
 *         D = n l and T = the k-th position (IEEE double, in that order).
 *   work as for skim_build_sketches.  n l < 2^32.
 */
skim_status skim_build_sketches_perm(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                     uint64_t *ranks, uint32_t *size, double *est,
                                     uint64_t *work, void *stream);

/*
 * skim_perm_query_batch -- union estimates over sketches of permutation
 * positions (skim_build_sketches_perm), as skim_query_batch (mode 0) with
 * the permutation reading: estimator 0 applies the estimator above to the
 * k-th smallest distinct position of the union; estimator 1 (Cohen-Kaplan,
 * Section 5.1, last paragraph) reads a threshold position T as the uniform
 * rank r = (T - 1)/(l n - 1), so a held value weighs (l n - 1)/(T_max - 1)
 * (1 when a holder is not full), summed in increasing order, divided by l.
 */
skim_status skim_perm_query_batch(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                  uint32_t k, uint32_t ell, uint64_t q, const uint64_t *qoff,
                                  const uint32_t *qnodes, uint32_t estimator, double *est,
                                  int32_t *qstatus, void *stream);

/*
 * skim_estimates -- per-node estimates from existing sketches, same formula
 * as the `est` output of skim_build_sketches.
 *   ranks [n*k], size [n] in, device; est [n] out, device.
 */
skim_status skim_estimates(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                           uint32_t ell, double *est, void *stream);

/*
 * skim_query_batch -- influence of q seed sets from the sketches (Section
 * 5.1).  Set j is qnodes[qoff[j] .. qoff[j+1]) (duplicates act once).
 *   estimator 0: bottom-k of the union of the sketches: U = the distinct
 *     ranks of the union; |U| / l if |U| < k, else ((k-1)/rho(U[k-1])) / l.
 *   estimator 1: Cohen-Kaplan (eq. unionest): each distinct rank z that a
 *     member sketch holds as a non-threshold element weighs
 *     1 / rho(max tau_u over such holders), a non-full sketch weighing 1;
 *     the weights are summed in increasing order of z, then divided by l.
 *   ranks [n*k], size [n]: sketches as skim_build_sketches writes them.
 *   qoff [q+1] (qoff[0] = 0, non-decreasing), qnodes [qoff[q]]: device.
 *   est [q] out, device.  qstatus [q] out, device, may be NULL: 0, or -1
 *   when the set names a node >= n, or -2 when it has more than 1024
 *   entries, or -3 when its offsets are out of order (only a replayed plan
 *   can see that; that query's est is 0, the rest of the batch is
 *   unaffected).  An empty set gives est 0, status 0.
 *   mode 0: one persistent launch for the whole batch (default);
 *   mode 1: one launch per query (the plain path, for comparison).
 * The call validates qoff, launches, and waits for the stream.
 */
skim_status skim_query_batch(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                             uint32_t k, uint32_t ell, uint64_t q, const uint64_t *qoff,
                             const uint32_t *qnodes, uint32_t estimator, uint32_t mode,
                             double *est, int32_t *qstatus, void *stream);

/*
 * Resident sketches: a library-owned copy of a sketch table (ranks, sizes and
 * per-node estimates) kept in device memory for answering queries (Section 5:
 * the sketches are computed once and every query is answered from them).
 *   skim_sketches_create: copies ranks [n*k] and size [n] (device, as
 *     skim_build_sketches writes them) and computes the estimates, all
 *     enqueued on `stream` without waiting; the sources may be released once
 *     the stream has passed the copies.  *out receives the handle.
 *   skim_build_sketches_resident: skim_build_sketches straight into a new
 *     handle's buffers (synchronises as that call does); work as there.
 *   skim_sketches_data: the handle's device arrays (read-only) and shape;
 *     any output pointer may be NULL.
 *   skim_sketches_query: the union estimates of skim_query_batch (mode 0,
 *     same estimators and statuses) for q sets, ENQUEUED ONLY: no host check
 *     and no wait, so the call may be captured into a HIP graph.  qoff
 *     [q+1], qnodes [nnodes] (device); the offsets are checked by the
 *     kernel: a set whose offsets are out of order or reach past qoff[q] or
 *     nnodes gets status -3 and est 0.  workspace: NULL, or 128 device bytes
 *     of the caller's for the launch's work counter (give one when capturing
 *     into a graph or when more than 64 calls on one handle may be in flight
 *     at once: without it, calls take the handle's 64 counters in turn).
 *   skim_sketches_free: waits for the device, then releases the handle
 *     (NULL is ignored).
 * Errors: SKIM_EINVAL (bad shape or NULL), SKIM_ENOMEM, SKIM_EDEVICE.
 */
typedef struct skim_sketches skim_sketches;

skim_status skim_sketches_create(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                 uint32_t k, uint32_t ell, void *stream, skim_sketches **out);
skim_status skim_build_sketches_resident(const skim_graph *g, uint32_t ell, uint32_t k,
                                         uint64_t seed, uint64_t *work, void *stream,
                                         skim_sketches **out);
skim_status skim_sketches_data(const skim_sketches *sk, const uint64_t **ranks,
                               const uint32_t **size, const double **est, uint32_t *n,
                               uint32_t *k, uint32_t *ell);
skim_status skim_sketches_query(const skim_sketches *sk, uint64_t q, const uint64_t *qoff,
                                const uint32_t *qnodes, uint64_t nnodes, uint32_t estimator,
                                double *est, int32_t *qstatus, void *workspace, void *stream);
void skim_sketches_free(skim_sketches *sk);

/*
 * Query plans: the batched launch of skim_query_batch (mode 0) for fixed
 * buffers, captured once into a HIP graph.
 *   skim_query_plan_create: validates qoff as skim_query_batch does, then
 *     captures the launch (arguments as for skim_query_batch; q >= 1).  The
 *     buffers must stay allocated while the plan lives; their contents may
 *     change between launches (sets may be rewritten in place as long as
 *     qoff[q] does not exceed qnodes' length: a set whose offsets are out of
 *     order or beyond qoff[q] gets status -3).
 *   skim_query_plan_launch: replays the graph on `stream` without waiting
 *     (the caller synchronises); SKIM_EDEVICE on a launch failure.
 *   skim_query_plan_free: releases the plan (NULL is ignored).
 * For callers that answer batches of a fixed shape repeatedly (serving loops,
 * benchmarks): a replay costs one graph launch instead of validation, two
 * launches and a wait.
 */
typedef struct skim_query_plan skim_query_plan;

skim_status skim_query_plan_create(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                   uint32_t k, uint32_t ell, uint64_t q, const uint64_t *qoff,
                                   const uint32_t *qnodes, uint32_t estimator, double *est,
                                   int32_t *qstatus, void *stream, skim_query_plan **plan);
skim_status skim_query_plan_launch(skim_query_plan *plan, void *stream);
void skim_query_plan_free(skim_query_plan *plan);

/*
 * skim_greedy -- SKIM seed selection (Section 4, Algorithm 1) for s seeds.
 * Pairs are taken by increasing rank; each uncovered pair runs a complete
 * reverse search that adds one to size[v] of every node it reaches; the
 * first node whose size reaches k (smallest id among nodes reaching k on
 * the same pair) is the next seed; once every rank is processed the seed is
 * the unselected node of largest size (smallest id on ties).  The residual
 * problem then covers every pair the seed reaches (forward search per
 * instance, not entering covered pairs) and removes their ranks from the
 * partial sketches.  Here 2 <= k <= 65535 (sizes are 16-bit counters): a k
 * above every reach set gives exact greedy on the instances.
 *   seeds      [s] out, device: selected nodes in order.
 *   gain_pairs [s] out, device: newly covered node-instance pairs of each
 *              seed (l times its exact marginal influence, Section 4.1.1).
 *   gain       [s] out, device, may be NULL: gain_pairs / l.
 *   state: NULL = one-shot.  Otherwise *state = NULL starts a fresh run and
 *     returns its state in *state; a non-NULL *state resumes that run and
 *     selects the next s seeds (g, l, k, seed must be those of the run;
 *     the graph buffers must stay valid while the state lives).  Resuming
 *     in steps gives exactly the one-shot sequence.  s may not exceed the
 *     number of unselected nodes.
 */
typedef struct skim_greedy_state skim_greedy_state;

skim_status skim_greedy(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed, uint32_t s,
                        uint32_t *seeds, uint64_t *gain_pairs, double *gain,
                        skim_greedy_state **state, void *stream);

/* Release a state returned by skim_greedy (NULL is ignored). */
void skim_greedy_state_free(skim_greedy_state *state);

/* Seeds selected so far by a state (0 for NULL). */
uint32_t skim_greedy_state_selected(const skim_greedy_state *state);

/*
 * skim_greedy_state_save / skim_greedy_state_load -- suspend a SKIM run and
 * resume it later, in this or another process (Section 4: sketch building
 * is suspended when a seed is found and resumed after the residual update;
 * a saved state is the run between two such steps).  The saved image holds
 * the run's progress: covered pairs, partial sketch sizes, selected nodes,
 * the inverted index and its pool, the rank cursor and the per-seed error
 * records; what follows from (g, l, k, seed) alone (live lists, rank order)
 * is rebuilt by the load.
 *   save: buf [*bytes] out, HOST; buf NULL stores the size needed in
 *         *bytes; otherwise *bytes must be at least that size and receives
 *         it.  The state is unchanged.
 *   load: g, l, k, seed as for the saved run (the graph must be the same:
 *         n and m are checked, and the image records them); buf [bytes] in,
 *         HOST.  *state receives a new state; resuming it with skim_greedy
 *         selects what the saved run would have selected next.
 * Errors: SKIM_EINVAL for a NULL state or bytes, a buffer too small, or an
 * image that is not a saved state of this graph and parameters (nothing is
 * returned in *state then).  Both calls synchronise the stream.
 */
skim_status skim_greedy_state_save(const skim_greedy_state *state, void *buf, uint64_t *bytes,
                                   void *stream);
skim_status skim_greedy_state_load(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                   const void *buf, uint64_t bytes, skim_greedy_state **state,
                                   void *stream);

/*
 * skim_build_ic_sketches -- sketches for the IC model itself (Section 3,
 * "Sketches for an IC model"), with structured permutation ranks (Section 3,
 * "Structured permutation ranks") in the limit of infinitely many instances,
 * so that nothing depends on l.
 *   Positions t = 1 .. k n form k chunks of n; chunk c holds every node once,
 *   node v at position c n + 1 + |{w : h_c(w) < h_c(v)}| with
 *   h_c(v) = SM(2^63 + c n + v).  Every position has an instance of its own:
 *   edge (u -> w) is live in the instance of position t iff the high
 *   (t - 1 even) or low (t - 1 odd) 32 bits of output floor((t - 1) / 2) of
 *   the SplitMix64 stream seeded with SM(2^63 + 2^62 + u n + w) are <= thr.
 *   The sketch of u is the k smallest positions t whose node u reaches in the
 *   instance of t; the influence estimate is n (k - 1) / (T - 1), T the k-th
 *   smallest (every node reaches itself in every chunk, so T <= k n).
 *   positions [n k] out, device (uint32): row u ascending.
 *   est       [n] out, device, may be NULL.
 * k in [2, 256], k n < 2^32; same graph conventions and validation as
 * skim_build_sketches.  Every position runs a complete reverse search (an
 * instance has one source, so nothing prunes): the work is about k times
 * the sum of all nodes' influence.  Scratch: a visited bitmap (n / 8 bytes)
 * and a 4 KiB queue per search thread, at most 8 GiB in all, plus n / 8 + 4 n
 * bytes per workgroup for the searches that reach more than 1024 nodes, at
 * most 2 GiB; this suits graphs up to about 2^20 nodes.
 */
skim_status skim_build_ic_sketches(const skim_graph *g, uint32_t k, uint64_t seed,
                                   uint32_t *positions, double *est, void *stream);

/*
 * skim_ic_query_batch -- union queries over IC-model sketches (Section 3,
 * permutation ranks; Section 5.1, union estimators) for q seed sets.
 *   positions  [n k] device: as written by skim_build_ic_sketches.
 *   qoff, qnodes: as for skim_query_batch (qoff[0] = 0, non-decreasing;
 *     qnodes may be NULL when every set is empty; duplicates act once).
 *   estimator 0 (bottom-k): n (k - 1) / (T - 1), T the k-th smallest distinct
 *     position of the union of the members' sketches.
 *   estimator 1 (Cohen-Kaplan, eq. unionest with permutation ranks): every
 *     distinct position z some member u holds outside its own threshold
 *     T_u = X_u[k-1] weighs n / (T_max(z) - 1), T_max(z) the largest T_u over
 *     those members; the weights are added in increasing z.
 *   est [q] out, device; qstatus [q] out, device, may be NULL: 0; -1 for a
 *     node >= n and -2 for more than 1024 members (est 0 for both); an empty
 *     set gives 0.
 */
skim_status skim_ic_query_batch(const uint32_t *positions, uint32_t n, uint32_t k, uint64_t q,
                                const uint64_t *qoff, const uint32_t *qnodes, uint32_t estimator,
                                double *est, int32_t *qstatus, void *stream);

/*
 * skim_influence_batch -- exact influence of q seed sets over the l
 * instances of `seed` (Section 2, eqs. (Inf) and (timedinf)):
 * reach_pairs[j] = sum_i |reach_i(S_j)| = l Inf({G^(i)}, S_j), the number of
 * node-instance pairs reachable from S_j over live edges.  For a quality
 * harness: with a seed other than the one the sketches or SKIM used, it
 * scores their seed sets on fresh instances (call it with several seeds for
 * more than 64 instances).  Same graph conventions and validation as
 * skim_build_sketches; l in [1, 64].
 *   qoff        [q+1] device: set j is qnodes[qoff[j] .. qoff[j+1]); qoff[0]
 *               must be 0 and qoff non-decreasing (SKIM_EINVAL otherwise).
 *   qnodes      [qoff[q]] device (may be NULL when every set is empty).
 *               Duplicate nodes act once; an empty set reaches 0 pairs.
 *   reach_pairs [q] out, device.
 *   qstatus     [q] out, device, may be NULL: 0, or -1 when the set holds a
 *               node >= n (its reach_pairs is then 0).
 * Scratch: the live out-lists of the graph (8 (64 n + 1) bytes plus 4 bytes
 * per live edge-instance) and up to 2 GiB of per-query search state.
 */
skim_status skim_influence_batch(const skim_graph *g, uint32_t ell, uint64_t seed, uint64_t q,
                                 const uint64_t *qoff, const uint32_t *qnodes,
                                 uint64_t *reach_pairs, int32_t *qstatus, void *stream);

/*
 * skim_greedy_exact -- exact greedy on the l instances of `seed`, for
 * graphs small enough to score every node at every step (a reference for a
 * quality harness; Section 4 compares SKIM against it).  Step j selects the
 * unselected node of largest exact marginal gain (newly covered
 * node-instance pairs; smallest id on ties) and covers the pairs it reaches.
 *   seeds      [s] out, device.
 *   gain_pairs [s] out, device: l times each seed's exact marginal influence.
 * s <= n; same graph conventions and validation as skim_build_sketches;
 * l in [1, 64].  Each step runs n searches (pruned at covered pairs).
 */
skim_status skim_greedy_exact(const skim_graph *g, uint32_t ell, uint64_t seed, uint32_t s,
                              uint32_t *seeds, uint64_t *gain_pairs, void *stream);

/*
 * skim_greedy_records -- per-seed records of a SKIM run for its adaptive
 * error estimate (Section 4, adaptive error estimation), taken when the seed
 * is chosen, before its residual update.  For seeds first .. first+count-1
 * of the run (in selection order):
 *   tau    [count] out, device, may be NULL: the rank r(v, i) of the pair
 *          whose reverse search filled the seed's sketch (the seed's
 *          threshold rank); 2^64 - 1 for a seed chosen by the exhaustion rule.
 *   second [count] out, device, may be NULL: the second largest sketch k',
 *          the largest size among the other unselected nodes, where a node
 *          reached by the search of the pair of rank tau counts one less (so
 *          k' <= k - 1); for an exhaustion seed, the largest size among the
 *          other unselected nodes.
 * first + count must not exceed skim_greedy_state_selected(state)
 * (SKIM_EINVAL otherwise); tau and second may not both be NULL when count > 0.
 */
skim_status skim_greedy_records(const skim_greedy_state *state, uint32_t first, uint32_t count,
                                uint64_t *tau, uint32_t *second, void *stream);

/*
 * skim_discrepancy_tail -- confidence distribution of the total discrepancy
 * of a SKIM seed sequence (Section 4, adaptive error estimation,
 * eq. (chernoff)).  The discrepancy of seed j is the largest marginal gain of
 * any node minus the seed's exact gain Delta_j (node-instance pairs).  For a
 * filled-sketch seed, P[D_j > eps Delta_j] <= (e^-nu / (1-nu)^(1-nu))^mu with
 * mu = rho(tau_j) Delta_j (1 + eps), nu = 1 - k'_j / mu, rho(T) =
 * ((T >> 11) + 1) 2^-53 (1 where mu <= k'_j); an exhaustion seed has D_j = 0;
 * a filled-sketch record with Delta_j = 0 gives no bound.  Each D_j is
 * rounded up to the grid of step h = max_rel_error * I / bins pairs,
 * I = sum_j Delta_j, with everything at or beyond bins * h kept in the last
 * cell, and the per-seed distributions are convolved (treated as
 * independent, as in the paper).
 *   s                 number of seeds (records); 0 gives tail = (1, 0, ..., 0).
 *   tau, second       [s] device: as returned by skim_greedy_records.
 *   gain_pairs        [s] device: the seeds' gains as returned by skim_greedy.
 *   bins              1 .. 65536; s * (bins + 1) <= 2^30 (else
 *                     SKIM_EUNSUPPORTED).
 *   max_rel_error     > 0, finite: the grid covers total discrepancies of
 *                     0 .. max_rel_error * I.
 *   tail              [bins + 1] out, device (double): tail[t] is an upper
 *                     bound on P[D_1 + ... + D_s >= t h]; tail[0] = 1.
 *                     With I = 0 the result is (1, 0, ..., 0).
 * Scratch: 12 * s * (bins + 1) bytes of device memory for the call.
 */
skim_status skim_discrepancy_tail(uint32_t s, const uint64_t *tau, const uint32_t *second,
                                  const uint64_t *gain_pairs, uint32_t bins,
                                  double max_rel_error, double *tail, void *stream);

/*
 * skim_discrepancy_tail_noalloc -- skim_discrepancy_tail for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * result; it allocates nothing and only enqueues its work on `stream` (the
 * caller synchronises).  Its scratch is a file-scope device array of about
 * 12.3 MiB that each GPU the library runs on holds until the process ends:
 * s * (bins + 1) may be at most 2^20 (1,048,576), else SKIM_EUNSUPPORTED
 * with nothing enqueued.  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams or threads, before the
 * previous call's work has finished) race and must be serialised by the
 * caller.
 */
skim_status skim_discrepancy_tail_noalloc(uint32_t s, const uint64_t *tau, const uint32_t *second,
                                          const uint64_t *gain_pairs, uint32_t bins,
                                          double max_rel_error, double *tail, void *stream);

/*
 * Serving: a request loop over resident sketches.  Union queries are
 * admitted when their bytes (4 per node + 20) fit the free part of
 * budget_bytes, else SKIM_EBUSY (retry later); a request that can never fit
 * gives SKIM_EUNSUPPORTED.  A worker thread keeps up to `streams` batches in
 * flight and packs every waiting query that fits a free slot (max_batch sets,
 * budget_bytes / 4 / streams nodes) into one persistent launch as soon as
 * the slot frees up (continuous batching); incremental SKIM requests run in
 * order on their own stream, resuming one device-resident state, and overlap
 * with the query batches.  Each result is the one the batch call gives for
 * the same input.  Latencies run from arrival to completion seen by the host.
 * The sketches (ranks, size: device, caller-owned) and the SKIM graph must
 * stay valid while the server lives.  Calls on one server are thread-safe.
 */
typedef struct skim_server skim_server;

typedef struct {
    uint64_t budget_bytes;  /* bytes of admitted, unfinished query requests */
    uint32_t max_batch;     /* queries per launch                           */
    uint32_t streams;       /* batches in flight, 1..16                     */
    uint32_t estimator;     /* 0 bottom-k, 1 Cohen-Kaplan                   */
} skim_server_config;

skim_status skim_server_create(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                               uint32_t ell, const skim_server_config *cfg, skim_server **out);
void skim_server_destroy(skim_server *server);

/* Submit one seed set (HOST array of count node ids); returns a ticket. */
skim_status skim_server_submit(skim_server *server, const uint32_t *nodes, uint32_t count,
                               uint64_t *ticket);

/* SKIM_OK with the result (HOST pointers, may be NULL; status as in
 * skim_query_batch) and the ticket retired; SKIM_EBUSY while in flight;
 * SKIM_EINVAL for an unknown ticket. */
skim_status skim_server_poll(skim_server *server, uint64_t ticket, double *est, int32_t *status,
                             double *latency_us);

/* Cancel query request `ticket`: it completes with status -6 and est 0
 * (skim_server_poll then returns SKIM_OK).  A request still waiting is
 * withdrawn at once; one already in a batch on the GPU finishes there and
 * its result is dropped.  SKIM_EINVAL for an unknown or finished ticket. */
skim_status skim_server_cancel(skim_server *server, uint64_t ticket);

/* Attach the graph for SKIM requests (once per server). */
skim_status skim_server_set_graph(skim_server *server, const skim_graph *g, uint32_t ell,
                                  uint32_t k, uint64_t seed);

/* Request the next s seeds of the server's SKIM run (skim_greedy semantics).
 * Admitted when its result bytes (12 per seed + 64) fit the free part of
 * budget_bytes beside the queries in flight, else SKIM_EBUSY (retry later);
 * SKIM_EUNSUPPORTED if it could never fit. */
skim_status skim_server_submit_greedy(skim_server *server, uint32_t s, uint64_t *ticket);

/* seeds [s], gain_pairs [s]: HOST arrays; SKIM_EBUSY while running. */
skim_status skim_server_poll_greedy(skim_server *server, uint64_t ticket, uint32_t *seeds,
                                    uint64_t *gain_pairs, double *latency_us);

/*
 * Open-loop replay, for measurement: submits set j (HOST offsets[q+1],
 * nodes) at arrival_s[j] seconds after the call starts (retrying on
 * SKIM_EBUSY; latency still counts from the scheduled arrival) and collects
 * every result into HOST arrays est[q], status[q] (-4 = rejected, -5 = the
 * batch's copy, launch or completion failed; est is 0 for both),
 * latency_us[q] (may be NULL).  busy_retries (HOST, may be NULL) counts
 * admission refusals.
 */
skim_status skim_server_replay(skim_server *server, uint64_t q, const uint64_t *offsets,
                               const uint32_t *nodes, const double *arrival_s, double *est,
                               int32_t *status, double *latency_us, uint64_t *busy_retries);

/*
 * Launch shapes of the sketch build's pruned search (process-wide; they
 * change speed only, never results):
 *   small_frontier   frontiers of at most this many entries go in batches of
 *                    small_batch levels launched without reading back the
 *                    frontier size (default 65536);
 *   small_batch      levels per such batch (default 8, 1..64);
 *   large_batch      levels per batch of larger frontiers (default 3, 1..64);
 *   thread_frontier  frontiers of at most this many entries are expanded one
 *                    entry per thread, larger ones 1024 entries per
 *                    workgroup per round (default 524288);
 *   heavy_visits     a rank window whose visited pairs took more than this
 *                    many visits each on average is followed by a window of
 *                    one rank bucket instead of two (default 4, >= 1);
 *   sort_frontier    frontiers of more than this many entries are sorted by
 *                    pair before they are expanded, so that live lists are
 *                    read in order (0 = never, the default);
 *   window_span      rank buckets per window after a window with few visits
 *                    per pair (default 2, 1..8); bucket 0 holds about k/2
 *                    ranks per instance and each later bucket doubles the
 *                    rank range.  Wider windows mean fewer search levels and
 *                    more visits past k;
 *   first_span       rank buckets of the first window (default 5, 1..16);
 *                    a first window that outgrows its buffers is given up
 *                    and the build starts again from bucket 0 alone;
 *   pull_frontier    levels whose frontier holds at least this many entries
 *                    are taken by pull: every pair reads its live out-list
 *                    and takes the sources of the frontier entries it meets
 *                    (the frontier sorted by pair and indexed over pairs),
 *                    instead of each entry pushing over its live in-list.
 *                    Both directions make the same visits (Section 5.2, the
 *                    pruned searches of Algorithm 2), so the sketches do not
 *                    depend on it.  Nonzero also builds the out-lists with
 *                    the in-lists; 0 = never (the default).
 * skim_set_build_params(NULL) restores the defaults; fields out of range give
 * SKIM_EINVAL and change nothing.
 */
typedef struct {
    uint32_t small_frontier;
    uint32_t small_batch;
    uint32_t large_batch;
    uint32_t thread_frontier;
    uint32_t heavy_visits;
    uint32_t sort_frontier;
    uint32_t window_span;
    uint32_t first_span;
    uint32_t pull_frontier;
} skim_build_params;

skim_status skim_set_build_params(const skim_build_params *params);
void skim_get_build_params(skim_build_params *params);

/*
 * Autotuner for the build's launch shapes: builds the sketches of (g, l, k,
 * seed) into ranks/size (device, as for skim_build_sketches) with the
 * current parameters and then with candidate values of one parameter at a
 * time (coordinate descent over small_frontier, small_batch, large_batch,
 * thread_frontier, sort_frontier, window_span, first_span, pull_frontier:
 * never, from 2^21 or from 2^23 entries), each timed as the best of `reps` builds
 * with HIP events on `stream` after one warm-up build.  The fastest set becomes the current
 * parameters and is written to *best (HOST); *best_ms and *start_ms (HOST,
 * may be NULL) receive its time and that of the parameters in force at the
 * call.  Results of every build are identical; ranks/size hold the last.
 */
skim_status skim_tune_build(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                            uint64_t *ranks, uint32_t *size, uint32_t reps,
                            skim_build_params *best, double *best_ms, double *start_ms,
                            void *stream);

/*
 * skim_tune_build_cached -- skim_tune_build behind a persistent cache keyed
 * by the device (architecture name, compute units) and the configuration
 * (n, m, l, k, seed and 64 evenly spaced samples of each graph array).
 * cache_path (HOST string) names a text file, one line per key; it is read
 * and created or appended to as needed.  On a hit the stored shapes are put
 * in force without timing anything (*hit = 1, *best_ms = the stored time,
 * *start_ms = 0, ranks/size untouched); on a miss the tuner runs as
 * skim_tune_build and its choice is appended (*hit = 0).  Unreadable lines
 * are skipped.  best, hit: HOST out; best_ms, start_ms: HOST out, may be
 * NULL.  Concurrent calls in one process are serialised; calls from several
 * processes on one file may both tune and both append (the first matching
 * line wins).
 */
skim_status skim_tune_build_cached(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                   uint64_t *ranks, uint32_t *size, uint32_t reps,
                                   const char *cache_path, skim_build_params *best,
                                   double *best_ms, double *start_ms, uint32_t *hit,
                                   void *stream);

/*
 * Kernel timing, for measurement: while a kernel name is enabled, every
 * launch of that kernel (e.g. "k_expand", the level expansion of the pruned
 * reverse search) made by the calling thread is bracketed by HIP events on
 * the call's stream.  Totals accumulate across calls until reset.
 *   skim_timing_enable(names): time launches of the kernels named in the
 *     comma-separated list `names` (NULL or "" = off).
 *   skim_timing_read(name, total_ms, launches): totals so far (HOST
 *   pointers, may be NULL); returns 1 if the kernel has entries, else 0.
 */
void skim_timing_enable(const char *kernel);
void skim_timing_reset(void);
int skim_timing_read(const char *kernel, double *total_ms, uint64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* SKIM_H */
