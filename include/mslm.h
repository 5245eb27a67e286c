/*
 * mslm — exact multislice-modularity Leiden on one AMD MI355X (gfx950).
 *
 * The operation: community detection in a snapshot temporal network by Leiden optimisation
 * (local moving, refinement, aggregation) of the multislice modularity Q_MS of Eq. 6
 * (Section 3.2) on the supra-graph of Eq. 3 (Section 3.1): T snapshots over the same N
 * node ids, supra-node (i, s) numbered v = s*N + i, intra-snapshot edges on the diagonal
 * blocks and an ordinal coupling omega between (i, s) and (i, s+1) for every node i.
 * Resolution gamma and coupling omega are exact fractions; all arithmetic is integer or
 * exact rational, so results are bit-for-bit reproducible and independent of batching.
 *
 * Conventions shared by every entry point
 *   - Return value: MSLM_OK or a negative mslm_status; mslm_last_error() gives the text.
 *     On error outputs are left untouched and a valid handle stays valid.
 *   - Host pointers unless a flag says device.  Inputs are copied; the caller keeps
 *     ownership of everything it passes and may free it on return.
 *   - Streams: device work runs on the hipStream_t given at creation (NULL = default
 *     stream).  Calls return after their outputs are written.
 *   - A handle is used by one thread at a time; distinct handles are independent.
 */
#ifndef MSLM_H
#define MSLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MSLM_OK = 0,
  MSLM_EINVAL = -1,       /* invalid argument or malformed graph                        */
  MSLM_ENOMEM = -2,       /* device or host allocation failed                           */
  MSLM_EOVERFLOW = -3,    /* exact integer head-room precondition violated              */
  MSLM_EUNSUPPORTED = -4, /* outside this version's limits (T > 64, N*T*33 >= 2^32)         */
  MSLM_EHIP = -5,         /* HIP runtime error                                          */
  MSLM_EBUSY = -6         /* server: result not ready before the timeout                */
} mslm_status;

typedef struct mslm_graph mslm_graph;   /* owns the device supra-CSR of one temporal graph */
typedef struct mslm_server mslm_server; /* continuous-batching request loop               */

enum { MSLM_INPUT_ON_DEVICE = 1u, MSLM_OUTPUT_ON_DEVICE = 2u, MSLM_PROFILE = 4u, MSLM_COUNT = 8u,
       MSLM_COUPLE_PRESENT = 16u };

/* The objective a solve maximises.  MULTISLICE: Q_MS of Eq. 6, a null model per snapshot
 * (gamma^(s) k_i^s k_j^s / 2m_s).  GLOBAL: the modularity of Eq. 5 over the whole supra-graph
 * of Eq. 3 (null model gamma kappa_u kappa_v / 2mu with kappa the supra-degree, intra weight
 * plus coupling), the objective the paper's GPU path optimised on the supra-graph in place of
 * Q_MS (Section 3.2).  CPM: the multislice Constant Potts Model that Section 3.2 names as a
 * quality function of the same supra-graph strategy, read as Eq. 6 with the null term
 * gamma^(s) n_i n_j, node weight n = 1 per supra-node (no 2m_s), under the same 1/2mu. */
enum { MSLM_NULL_MULTISLICE = 0, MSLM_NULL_GLOBAL = 1, MSLM_NULL_CPM = 2 };

/* One temporal graph.  Slice s holds edges [slice_offsets[s], slice_offsets[s+1]) of
 * src/dst/weight: undirected, each edge listed once in either orientation, ids in [0, N),
 * no self-loops, weight >= 1 (NULL = unit weights).  Repeated pairs inside a slice add
 * their weights.  slice_offsets is always host memory; src/dst/weight are device
 * pointers when flags has MSLM_INPUT_ON_DEVICE.  Limits: 1 <= T <= 64, N >= 1,
 * N*T*33 < 2^32, every slice's total degree 2m_s < 2^31.
 * Coupling (Eq. 6's omega^(sr)): coupling (host, NULL = ordinal) is a T*T row-major matrix of
 * integers c_sr in [0, 2^16), symmetric with a zero diagonal; copies (i,s) and (i,r) are
 * coupled with weight omega^(sr) = omega * c_sr (the ordinal coupling of Eq. 3 is c_sr = 1 for
 * |s - r| = 1; categorical coupling is c_sr = 1 for all s != r).  With MSLM_COUPLE_PRESENT in
 * flags only copies present in both slices are coupled, a copy being present when it has an
 * edge in its slice (the supra-graph of data whose nodes are absent from some snapshots);
 * under the CPM an absent copy then carries node weight 0.  2mu = sum_s 2m_s + omega * C with
 * C the coupling total (sum of c_sr over ordered coupled copy pairs; 2N(T-1) for the ordinal
 * coupling of every copy), reported in mslm_result.coupling_total. */
typedef struct {
  int32_t n_nodes;
  int32_t n_slices;
  const int64_t *slice_offsets;
  const int32_t *src;
  const int32_t *dst;
  const int32_t *weight;
  int64_t omega_num, omega_den;   /* default coupling omega = num/den, num >= 0, den >= 1 */
  uint32_t flags;
  const int32_t *coupling;
} mslm_graph_desc;

/* One solve.  gamma = gamma_num/gamma_den (num >= 0, den >= 1).  omega_den == 0 keeps the
 * graph's default coupling.  max_levels >= 1 bounds the aggregation levels of one Leiden
 * iteration; max_iterations <= 0 runs iterations until the partition is stable (at most
 * 32); max_sweeps <= 0 means 32 local-moving sweeps per level.  The seed only changes the
 * hash priorities of the schedule.  Numerators and denominators must be below 2^31.
 * null_model: MSLM_NULL_MULTISLICE (0), MSLM_NULL_GLOBAL (1) or MSLM_NULL_CPM (2); with GLOBAL
 * the scaled total weight 2mu' = b * sum_s 2m_s + 2 a N (T-1) (omega = a/b) must stay below
 * 2^31 and max(p, q) * 2mu'^2 below 2^62 (else EOVERFLOW).
 * gamma_slices (host, NULL = gamma in every slice): T pairs (num, den), the resolution
 * gamma^(s) of each slice (Eq. 6), each positive with num, den < 2^31; not with GLOBAL
 * (EINVAL).  The kernels fold them into the slice denominators (see mslm_leiden's errors).
 * initial_membership (host, NULL = singletons): the start partition of the first Leiden
 * iteration (warm start, or resume from an earlier result), T*N labels in [0, T*N) in
 * supra-node order (equal labels = one community; any labelling of a partition gives the same
 * solve).  Both arrays are read during the call (copied by mslm_server_submit). */
typedef struct {
  int64_t gamma_num, gamma_den;
  int64_t omega_num, omega_den;
  int32_t max_levels;
  int32_t max_iterations;
  int32_t max_sweeps;
  int32_t null_model;
  uint64_t seed;
  uint32_t flags;                 /* MSLM_OUTPUT_ON_DEVICE: membership is a device pointer;
                                     MSLM_PROFILE: time every level-0 local-moving decision
                                     launch with HIP events on the graph's stream (the short
                                     launches of aggregated levels are left untimed);
                                     MSLM_COUNT: count the work of those kernels            */
  uint32_t reserved1;
  const int64_t *gamma_slices;
  const int32_t *initial_membership;
} mslm_params;

/* Per-solve outcome.  q_components (3T+1 int64) are the exact integer pieces of Q:
 * W_s (weight inside communities in slice s, both directions), SS_s (sum over communities
 * of the squared slice-s degree; for the CPM of the squared slice-s supra-node count), 2m_s,
 * and I (sum of c_sr over the ordered coupled copy pairs sharing a community: their count for
 * the ordinal coupling); mslm_q_exact (mslm_q_exact_variant
 * for per-slice resolutions and the CPM) turns them into the reduced fraction Q.  For the GLOBAL null model
 * the T slots of SS hold one value, SS' = sum over communities of (sum of kappa')^2 with
 * kappa' = b * (intra degree) + a * (coupling count), then zeros; mslm_q_exact_global reduces
 * them. */
typedef struct {
  double q;                       /* Q rounded to double                                    */
  int32_t n_communities, levels_run, iterations_run, colours_level0;
  int64_t sweeps, moves, sweep_cap_hits, refine_rounds, merges, splits;
  int64_t exact_fallbacks;        /* big-integer evaluations this solve's units needed; how many
                                     depends on the order in which the kernels meet candidates
                                     (batching may change it), the result never does           */
  double ms_total;                /* host wall clock of the call                            */
  double ms_colour, ms_local_move, ms_refine, ms_aggregate, ms_finish;   /* device, by phase */
  double lm_kernel_ms;            /* summed durations of the timed decision launches
                                     (MSLM_PROFILE: level 0 only, equal to lm0_kernel_ms)     */
  int64_t lm_launches;            /* number of those launches (MSLM_PROFILE)                 */
  int64_t lm_units, lm_entries, lm_candidates;   /* work of those kernels: units decided,
                                     adjacency entries scanned, candidate communities (COUNT) */
  int64_t q_components[3 * 64 + 1];
  double lm0_kernel_ms;           /* level-0 decision kernel time (MSLM_PROFILE)              */
  int64_t lm0_launches;           /* level-0 decision launches (MSLM_PROFILE)                 */
  int64_t lm0_units, lm0_entries, lm0_candidates;   /* level-0 share of the work (COUNT)   */
  int64_t coupling_total;         /* the graph's coupling total C (2mu = sum 2m_s + omega C)  */
} mslm_result;

/* Build the device supra-CSR (Eq. 3) of a temporal graph: both directions of every intra
 * edge with repeated pairs summed, plus the coupling entries (i,s)<->(i,r) of every coupled
 * pair of copies (for the ordinal coupling (i,s)<->(i,s+1) for all i).
 * *out is NULL on failure.  Errors: EINVAL (ids, self-loops, weights, sizes), EOVERFLOW
 * (2m_s >= 2^31), EUNSUPPORTED (T > 64 or N*T too large), ENOMEM, EHIP. */
mslm_status mslm_create(const mslm_graph_desc *desc, void *hip_stream, mslm_graph **out);

/* Run the deterministic Leiden schedule on a resident graph (Section 3.2, Eq. 6).
 * membership[T*N] receives the community of supra-node v = s*N + i, labelled 0..K-1 in
 * order of first appearance; every community is connected.  res may be NULL.
 * Errors: EINVAL (parameters), EOVERFLOW (int64 gain head-room: q*2m_s*w and p*b*k*Sigma
 * must stay below 2^62, with k and Sigma bounded by N under the CPM; with per-slice
 * resolutions, Q = lcm of their denominators and C = lcm over s of gamma^(s)*Q take the places
 * of q and p, each slice's 2m_s (1 under the CPM) is multiplied by C / (gamma^(s)*Q) and must
 * stay below 2^31), ENOMEM, EHIP. */
mslm_status mslm_leiden(mslm_graph *g, const mslm_params *params, int32_t *membership,
                        mslm_result *res);

/* Release a graph handle and its device memory.  NULL is allowed. */
void mslm_destroy(mslm_graph *g);

/* Exact Q of Eq. 6 from the 3T+1 components, as a reduced fraction written in decimal
 * into num/den (NUL-terminated).  Errors: EINVAL (buffers too small, den <= 0). */
mslm_status mslm_q_exact(const int64_t *q_components, int32_t n_slices, int32_t n_nodes,
                         int64_t gamma_num, int64_t gamma_den, int64_t omega_num,
                         int64_t omega_den, char *num, size_t num_cap, char *den, size_t den_cap);

/* The same for the GLOBAL null model: Q_G = (q 2mu' W' - p SS') / (q 2mu'^2) with
 * W' = b * sum_s W_s + a * I and 2mu' = b * sum_s 2m_s + 2 a N (T-1).  Errors: EINVAL. */
mslm_status mslm_q_exact_global(const int64_t *q_components, int32_t n_slices, int32_t n_nodes,
                                int64_t gamma_num, int64_t gamma_den, int64_t omega_num,
                                int64_t omega_den, char *num, size_t num_cap, char *den,
                                size_t den_cap);

/* Exact value of any objective from a solve's 3T+1 components: null_model MULTISLICE (Eq. 6,
 * as mslm_q_exact), GLOBAL (as mslm_q_exact_global) or CPM, whose SS_s slots hold the sum over
 * communities of the squared number of their slice-s supra-nodes:
 *   Q = (sum_s [W_s - gamma^(s) SS_s] + omega I) / (sum_s 2m_s + omega C).
 * gamma_slices as in mslm_params (NULL: gamma_num/gamma_den in every slice; not with GLOBAL).
 * coupling_total: the graph's C (mslm_result.coupling_total); < 0 means 2N(T-1), the ordinal
 * coupling of every copy that mslm_q_exact and mslm_q_exact_global assume.  Errors: EINVAL. */
mslm_status mslm_q_exact_variant(const int64_t *q_components, int32_t n_slices, int32_t n_nodes,
                                 int32_t null_model, const int64_t *gamma_slices,
                                 int64_t gamma_num, int64_t gamma_den, int64_t omega_num,
                                 int64_t omega_den, int64_t coupling_total, char *num,
                                 size_t num_cap, char *den, size_t den_cap);

/* Execution choices that change the speed of a solve and never its result (the same
 * memberships, Q components and statistics for every value).  Each graph handle holds one;
 * mslm_batch_leiden uses the one of the graph its first solve names, the server the defaults.
 *   graphs             1: the sweeps of an aggregated level are replayed from a captured HIP graph
 *                      after the second sweep (default 0: plain launches)
 *   latency_units      aggregated levels: colour batches of at most this many units take the
 *                      one-launch latency path (64..65536, default 1024)
 *   split_group_units  level 0: a colour batch with at least this many lane-group units gives
 *                      them a launch of their own (0..2^30, default 16384)
 *   copy_moves         level 0: the per-entry neighbour-label copy is kept through sweeps that
 *                      moved at most (units / copy_moves) units (1..2^30, default 1024)
 *   lat_parts_max      latency path: most blocks sharing one unit's candidates (1..16, default 16)
 *   batch_units        mslm_batch_leiden: most supra-nodes per union, in units of 2^20 (1..100,
 *                      default 24)
 * Errors: EINVAL for a value out of range or a NULL pointer. */
typedef struct {
  int32_t graphs;
  int32_t latency_units;
  int32_t split_group_units;
  int32_t copy_moves;
  int32_t lat_parts_max;
  int32_t batch_units;
  int32_t reserved[2];
} mslm_tuning;

mslm_status mslm_get_tuning(const mslm_graph *g, mslm_tuning *out);
mslm_status mslm_set_tuning(mslm_graph *g, const mslm_tuning *t);

/* Autotuner: times full solves of (g, params) under candidate tunings, one setting changed at a
 * time from the best so far (graphs, latency_units, split_group_units, copy_moves,
 * lat_parts_max; `rounds` passes over them, 1..4), keeps a change only when it is at least 2%
 * faster, checks that every candidate's membership and Q components equal those of the
 * starting tuning (MSLM_EHIP with the error text if one ever differs, which would be a library
 * bug), installs the best tuning on the handle and writes it to `out`.  ms_start / ms_best
 * (may be NULL) receive the solve times of the starting and the chosen tuning. */
mslm_status mslm_autotune(mslm_graph *g, const mslm_params *params, int32_t rounds,
                          mslm_tuning *out, double *ms_start, double *ms_best);

/* Device bytes a graph and one solve on it need (admission estimate). */
size_t mslm_footprint_bytes(const mslm_graph_desc *desc);

/* Graph sizes: supra-nodes, directed CSR entries (coupling entries included). */
mslm_status mslm_graph_info(const mslm_graph *g, int64_t *n_supra, int64_t *nnz, int64_t *two_m);

/* Text of the last error on this thread (valid until the next call on this thread). */
const char *mslm_last_error(void);

/* Route the library's device allocations through a caller's allocator, for example PyTorch's
 * caching allocator (the package's Python binding installs one); alloc == release == NULL
 * restores hipMalloc/hipFree.  alloc(bytes, ctx) returns device memory of the current device
 * (NULL = out of memory, reported as MSLM_ENOMEM); release(ptr, ctx) takes back a block alloc
 * returned.  Every buffer is released through the pair that allocated it, so the pair may be
 * changed while graphs exist.  Before a release the library waits for all device work
 * (hipDeviceSynchronize), so a block can be handed to other work at once.  The pair is global
 * to the process; the callbacks may run on any thread that calls into the library (including
 * the request loop's workers).  Errors: EINVAL (one of the two is NULL). */
mslm_status mslm_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                               void (*release)(void *ptr, void *ctx), void *ctx);

/* ------------------------------------------------------------------ allocation-free solve */
/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  mslm_leiden on a resident graph, same arguments
 * and same results, except that every work buffer of the solve is carved from a static device
 * array of MSLM_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on from load
 * until the process ends; no hipMalloc, hipFree or allocating library routine is called (the
 * graph and the caller's outputs are the only other device memory touched).  The array keeps
 * the last call's contents; every call clears what it needs.  Calls on one GPU share its
 * array: the library runs them one at a time (a per-device lock), and a call's device work is
 * finished when it returns, so calls from several threads never overlap on the array.
 * Errors: EUNSUPPORTED when the solve needs more than the array holds (estimate: 96 bytes per
 * CSR entry plus 384 per supra-node plus 1 MiB: about 400k supra-nodes with 1M entries), EINVAL for
 * MSLM_PROFILE (it records HIP events) or when the current device is not the graph's, and as
 * mslm_leiden otherwise. */
#define MSLM_STATIC_SCRATCH_BYTES (256ull << 20)
mslm_status mslm_leiden_static(mslm_graph *g, const mslm_params *params, int32_t *membership,
                               mslm_result *res);

/* ------------------------------------------------------------------ batching */
/* Many solves (graph x gamma x omega) run as one disjoint-union solve: every kernel launch
 * covers all solves that are still active, and each solve's result is bit-identical to a
 * plain mslm_leiden call with the same graph and parameters (the schedule only ever
 * compares units of the same solve, and priorities use solve-local ids). */
typedef struct {
  int32_t graph;                  /* index into graphs[]                                    */
  int32_t reserved;
  mslm_params params;
  int32_t *membership;            /* host [T*N] of that graph                               */
  mslm_result *result;            /* may be NULL                                            */
} mslm_solve;

mslm_status mslm_batch_leiden(mslm_graph *const *graphs, int32_t n_graphs,
                              const mslm_solve *solves, int32_t n_solves, void *hip_stream);

/* ------------------------------------------------------------------ long sequences */
/* Windowed optimisation of a snapshot sequence of any length T (Section 4 names it for the
 * 7375-snapshot School data, whose one supra-graph is out of reach): windows of `window`
 * consecutive snapshots (1..64), each starting window - overlap snapshots after the previous
 * one (0 <= overlap < window), the last one ending at the last snapshot.  Each window is solved
 * as mslm_leiden solves its supra-graph (same parameters, ordinal coupling, MSLM_COUPLE_PRESENT
 * honoured); a later window starts from the earlier windows' labels on its overlapping
 * snapshots and singletons elsewhere.  A window's community that holds overlapping copies takes
 * the label of its first such copy (smallest supra-node), any other a new label; overlapping
 * copies keep their labels, the window labels its other snapshots; labels are finally
 * renumbered by first appearance.  desc: host edge lists, slice_offsets[T+1], coupling NULL;
 * params: initial_membership NULL, gamma_slices (if given) T pairs.  membership[T*N] (host).
 * Errors: EINVAL (arguments), and those of mslm_create / mslm_leiden for a window. */
typedef struct {
  int32_t windows;         /* windows solved                                                 */
  int32_t n_communities;   /* communities of the final labels                                */
  double ms_total;         /* host wall clock of the call                                    */
} mslm_window_result;

mslm_status mslm_leiden_windowed(const mslm_graph_desc *desc, const mslm_params *params,
                                 int32_t window, int32_t overlap, void *hip_stream,
                                 int32_t *membership, mslm_window_result *res);

/* ------------------------------------------------------------------ spectral pathway */
/* The Bethe-Hessian pathway of Section 3.1 (the paragraphs after Eq. 4) on a resident graph:
 * H(r) = (r^2 - 1) I - r A + D with A the supra-adjacency of Eq. 3 (intra weights, coupling
 * omega * c_sr) and D its weighted degrees; the k algebraically smallest eigenpairs of H (its
 * informative, negative end) by Lanczos with full reorthogonalisation in float64 (classical
 * Gram-Schmidt against every Lanczos vector, a second pass when the first removed more than half
 * of the vector's squared norm), the small tridiagonal matrix's eigenpairs by implicit QR steps
 * with the Wilkinson shift, Ritz vectors; k-means of the n = N*T rows of the eigenvector
 * embedding into k clusters.
 *   k                  eigenvectors and clusters, 1..32 and below n
 *   lanczos_steps      Krylov dimension m, k..min(256, n) (0: min(n, 256, max(4k, k + 152));
 *                      without restarts the returned pairs converge only when m is large enough
 *                      for the graph: res->residual_max reports how far they are)
 *   kmeans_iterations  Lloyd iteration cap (0: 100)
 *   r                  0: sqrt(<d^2>/<d> - 1) (1 when that is not above 1), the degree-corrected
 *                      sqrt(average degree); else the value given (1 gives the Laplacian D - A)
 *   omega_den == 0     keeps the graph's coupling omega
 *   seed               the Lanczos start vector (SplitMix64 of seed ^ i, uniform in [-1, 1))
 * k-means is deterministic: the first point, then the point farthest from the centroids chosen
 * so far (lowest index on ties), then Lloyd steps until no label changes (nearest centroid,
 * lowest index on ties; distances summed over the coordinates in order, each operation
 * rounded; centroid sums exact on the fixed-point values round(x * 2^40)). */
typedef struct {
  int32_t k;
  int32_t lanczos_steps;
  int32_t kmeans_iterations;
  int32_t reserved;
  double r;
  int64_t omega_num, omega_den;
  uint64_t seed;
} mslm_spectral_params;

typedef struct {
  double r;                /* the r used                                                     */
  double residual_max;     /* largest ||H y - lambda y|| of the returned eigenpairs         */
  int32_t lanczos_steps;   /* Krylov dimension reached (less than asked when it closed)     */
  int32_t tridiagonal_steps; /* implicit QR steps of the tridiagonal eigensolver             */
  int32_t kmeans_iterations;
  int32_t second_passes;   /* Lanczos steps whose reorthogonalisation took a second pass     */
  double spmv_ms;          /* summed duration of the Lanczos operator launches (HIP events) */
  int64_t spmv_launches;
  double ms_total;         /* host wall clock of the call                                     */
} mslm_spectral_result;

/* eigenvalues[k] (host, ascending), embedding (host n x k row-major, may be NULL), labels
 * (host n, may be NULL: no k-means).  Errors: EINVAL (arguments), EUNSUPPORTED (the Krylov
 * space closed before k vectors), ENOMEM, EHIP. */
mslm_status mslm_bethe_hessian(mslm_graph *g, const mslm_spectral_params *params,
                               double *eigenvalues, double *embedding, int32_t *labels,
                               mslm_spectral_result *res);
/* y = H(r) x for host vectors of n = N*T (the operator alone, for checking it).  omega_den == 0
 * keeps the graph's coupling.  Errors: EINVAL, ENOMEM, EHIP. */
mslm_status mslm_bh_apply(mslm_graph *g, double r, int64_t omega_num, int64_t omega_den,
                          const double *x, double *y);
/* The k-means of the pathway on caller points (host, n x dim row-major, 1 <= dim <= 32,
 * 1 <= k <= 32, k <= n): labels[n], centroids[k x dim] (may be NULL) and the Lloyd iterations
 * run; work on hip_stream (NULL: the default stream).  Errors: EINVAL, ENOMEM, EHIP. */
mslm_status mslm_kmeans(const double *points, int64_t n, int32_t dim, int32_t k,
                        int32_t max_iterations, int32_t *labels, double *centroids,
                        int32_t *iterations, void *hip_stream);

/* ------------------------------------------------------------------ serving */
/* A continuous-batching request loop (no counterpart in the paper: a systems layer around the
 * solve).  Requests are admitted in arrival order; each of max_slots worker slots takes all
 * admitted requests waiting when it becomes free (up to 64 per group) and runs them as one
 * batched solve, so up to max_slots groups are on the device at once and requests that arrive
 * meanwhile join the next free slot.  Device memory: a slot keeps its buffers between groups,
 * and the sum over slots of the larger of (bytes a slot holds, footprint estimate of the group
 * it runs) never exceeds hbm_budget_bytes; an idle slot whose buffers keep the queue's head
 * out releases them.  hip_stream: NULL gives every slot a stream of its own (created on the
 * current device); otherwise all slots queue their device work on that stream (groups are
 * still formed concurrently, their device work runs in stream order).  Every result equals
 * plain mslm_create + mslm_leiden on the same request.  Errors: EINVAL (max_slots outside
 * 1..16, zero budget), EHIP, ENOMEM. */
mslm_status mslm_server_create(size_t hbm_budget_bytes, int32_t max_slots, void *hip_stream,
                               mslm_server **out);
/* Copies the graph (host pointers only) and queues it.  Errors, before anything is queued:
 * EINVAL (the graph as for mslm_create, device inputs, parameters, or a footprint above the
 * budget), EOVERFLOW (2m_s >= 2^31 in a slice or the int64 gain head-room of these gamma and
 * omega), EUNSUPPORTED.  A request that is accepted cannot fail on these later; should its
 * group fail on the device, its requests are run again one at a time, so one request's error
 * is never another's result. */
mslm_status mslm_server_submit(mslm_server *s, const mslm_graph_desc *desc,
                               const mslm_params *params, uint64_t *ticket);
/* Waits up to timeout_ms (< 0: forever) for a ticket; EBUSY on timeout (the ticket stays
 * valid), EINVAL for an unknown ticket (each ticket is collected once).  latency_s is the time
 * from submit to completion. */
mslm_status mslm_server_wait(mslm_server *s, uint64_t ticket, int32_t timeout_ms,
                             int32_t *membership, mslm_result *res, double *latency_s);
/* Device bytes the slots hold now; the largest total seen at any group's start or end; the
 * largest total charged against the budget (never above it). */
mslm_status mslm_server_memory(mslm_server *s, size_t *held_bytes, size_t *peak_held_bytes,
                               size_t *peak_charged_bytes);
/* Stops the loop: queued requests end with EINVAL ("server destroyed"), running groups
 * finish, threads blocked in mslm_server_wait return, then the server is freed.  No call on
 * the server may start once destroy has begun. */
void mslm_server_destroy(mslm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MSLM_H */
