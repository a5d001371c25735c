/*
 * ef.h - Expected Force (EF) on AMD Instinct MI355X (gfx950).
 *
 * Expected Force of a node s (Sylos Labini et al., "Scaling Expected Force:
 * Efficient Identification of Key Nodes in Network-based Epidemic Models",
 * Sec. 3.3, Eq. 1): list every infected cluster reachable from s by two
 * transmission events (s infects a neighbour y, then s or y infects a still
 * susceptible neighbour z); a cluster's degree d is the number of edges that
 * leave it; EF(s) = -sum_c p_c ln p_c with p_c = d_c / sum_c d_c. Clusters are
 * counted with the multiplicities of the paper's Algorithm 1 (a star y-s-z is
 * reached twice, a path s-y-z once; a triangle lowers d by 2).
 *
 * Per seed the library also returns the exact integers
 *   N(s) = number of event sequences (clusters with multiplicity) and
 *   D(s) = sum of their degrees.
 *
 * Conventions for every entry point:
 *   - Each returns an ef_status; none throws, aborts or exits. On failure
 *     ef_last_error() returns a thread-local, human-readable message.
 *   - Node ids are the caller's ids, 0..n-1, in inputs and outputs.
 *   - The graph is simple and undirected, given as int32 CSR: row_ptr[n+1]
 *     offsets, col_idx[nnz] neighbour ids, each edge stored in both rows,
 *     rows sorted ascending, no self-loops, no duplicates, nnz < 2^31.
 *   - Ownership: the caller owns every buffer it passes. Handles are opaque
 *     and released only by the matching *_free. A handle must not be used by
 *     two threads at once.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     With host output pointers a call returns after its results are on the
 *     host. With EF_OUT_DEVICE the outputs are device pointers and the call
 *     is asynchronous on hip_stream.
 */
#ifndef EF_H_
#define EF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EF_OK = 0,
  EF_ERR_ARG = 1,            /* null pointer, negative size, bad enum or flag */
  EF_ERR_NOT_SYMMETRIC = 2,  /* an arc u->v without v->u */
  EF_ERR_SELF_LOOP = 3,      /* an arc u->u */
  EF_ERR_DUPLICATE = 4,      /* an arc listed twice in a row */
  EF_ERR_UNSORTED = 5,       /* a row not ascending, or row_ptr decreasing */
  EF_ERR_RANGE = 6,          /* a neighbour id outside 0..n-1, or row_ptr[0] != 0 */
  EF_ERR_OVERFLOW = 7,       /* nnz >= 2^31, or an int64 result could overflow */
  EF_ERR_NOMEM = 8,          /* device allocation failed or exceeds EF_MAX_DEVICE_BYTES */
  EF_ERR_DEVICE = 9,         /* no usable gfx950 device, or a HIP runtime error */
  EF_ERR_STATE = 10          /* call not valid for this handle */
} ef_status;

/* The exact formulations (all return identical N and D):
 *   EF_ALGO_CLUSTER     - cluster-centric, Algorithm 1: every cluster is
 *                         scored once and credited to its three nodes.
 *   EF_ALGO_PER_SEED    - the original per-seed formulation (Sec. 4): each
 *                         seed visits all of its own clusters (stars around
 *                         it, and paths through each neighbour).
 *   EF_ALGO_CLUSTER_AGG - as EF_ALGO_CLUSTER, but the pair sums of centres of
 *                         degree > 1024 are formed per class of equal
 *                         neighbour degree (Algorithm 1, Phase 2 regrouped:
 *                         clusters with the same three degrees have the same
 *                         score), so such a centre costs M^2 scores for M
 *                         distinct neighbour degrees instead of k(k-1)/2;
 *                         centres with more than 4096 distinct neighbour
 *                         degrees take the EF_ALGO_CLUSTER path. Same results
 *                         up to rounding order; clusters are accounted, not
 *                         enumerated one by one. */
typedef enum { EF_ALGO_CLUSTER = 0, EF_ALGO_PER_SEED = 1, EF_ALGO_CLUSTER_AGG = 2 } ef_algo;

/* Precision of the cluster-degree logarithms and their sums:
 *   EF_PREC_FP64  - every term and sum in double precision.
 *   EF_PREC_FP32C - terms in single precision with compensated (double-float)
 *                   sums; the final EF of seeds with more than 2^24 clusters is
 *                   formed in double precision; seeds whose EF would lose
 *                   accuracy to cancellation are recomputed from non-negative
 *                   terms (see ef_run_stats.promoted). */
typedef enum { EF_PREC_FP64 = 0, EF_PREC_FP32C = 1 } ef_prec;

/* flags */
#define EF_VALIDATE     0x1u  /* load: check that the CSR is simple and symmetric */
#define EF_DEVICE_PTRS  0x2u  /* load: row_ptr/col_idx are device pointers, borrowed
                                 (they must outlive the graph handle) */
#define EF_OUT_DEVICE   0x4u  /* compute/topk: outputs are device pointers, async */
#define EF_PROFILE      0x8u  /* compute: time each phase with HIP events
                                 (read back with ef_stats) */

typedef struct ef_graph ef_graph;

typedef struct {
  int32_t n;              /* nodes */
  int64_t nnz;            /* arcs = 2 * undirected edges */
  int32_t max_degree;
  int64_t clusters;       /* W = sum_v k_v (k_v - 1) / 2: the cluster set of Algorithm 1 */
  int64_t sum_sq_degree;  /* sum_v k_v^2 (the per-seed formulation's 2-hop stream length) */
  int64_t up_arcs;        /* arcs oriented from lower to higher (degree, id) rank = nnz / 2 */
  int64_t wedge_checks;   /* membership tests of the triangle pass: sum_w up(w) * down(w) */
} ef_graph_info;

/* Timings of the last ef_compute that ran with EF_PROFILE (milliseconds, from
 * HIP events on the call's stream), and counters of the last ef_compute. */
typedef struct {
  double t_bin_ms;        /* degree binning and work-list construction */
  double t_pairs_ms;      /* cluster generation and scoring (all pair-loop kernels) */
  double t_pairs_small_ms;/* pair loop, centres with k <= 64 (one wavefront each) */
  double t_pairs_mid_ms;  /* pair loop, centres with 64 < k <= 1024 (one workgroup each) */
  double t_pairs_big_ms;  /* pair loop, 1024x1024 super-tiles of centres with k > 1024 */
  double t_reduce_ms;     /* per-arc reduction of super-tile partial sums */
  double t_triangles_ms;  /* triangle pass (cluster-centric) */
  double t_stream_ms;     /* 2-hop path stream (per-seed) */
  double t_finalize_ms;   /* per-seed sums and Eq. 1 */
  double t_pass2_ms;      /* recomputation of cancellation-prone seeds (FP32C) */
  double t_total_ms;      /* first to last event of the call */
  int64_t pairs_small;    /* clusters scored by each pair-loop kernel */
  int64_t pairs_mid;
  int64_t pairs_big;
  int64_t pair_tiles;     /* super-tiles launched for centres with k > 1024 */
  int64_t promoted;       /* FP32C seeds recomputed from non-negative terms */
  int64_t fp64_finalized; /* FP32C seeds with more than 2^24 clusters */
  int64_t seeds;          /* seeds computed */
} ef_run_stats;

/* Text of the last error on this thread ("" when none). Never NULL. */
const char *ef_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t ef_version(void);

/* Number of visible gfx950 devices (0 is not an error). */
ef_status ef_device_count(int32_t *count);

/* Check on the host that (n, nnz, row_ptr, col_idx) is a simple undirected
 * graph in the CSR form described above. Returns the first violation found
 * (EF_ERR_RANGE, EF_ERR_UNSORTED, EF_ERR_DUPLICATE, EF_ERR_SELF_LOOP,
 * EF_ERR_NOT_SYMMETRIC, EF_ERR_OVERFLOW) and names the row in ef_last_error().
 * Needs no device. Input for Algorithm 1 is such a graph (Sec. 4). */
ef_status ef_validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx);

/* Load a graph (Algorithm 1's input, Sec. 4). Without EF_DEVICE_PTRS the
 * arrays are host memory and are copied; with it they are device memory and
 * are borrowed. EF_VALIDATE runs ef_validate_csr first (device inputs are
 * copied to the host for it). The library allocates its own device arrays
 * (degrees, arc sources, reverse arcs, the degree-oriented half adjacency)
 * and keeps them until ef_graph_free. */
ef_status ef_graph_load_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col_idx, uint32_t flags, void *hip_stream,
                            ef_graph **out);

/* Build and load a graph from m host edges (src[i], dst[i]) over nodes
 * 0..n-1, in either orientation; self-loops are dropped, duplicates merged. */
ef_status ef_graph_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                              void *hip_stream, ef_graph **out);

/* Release a graph handle and every device array the library allocated for it
 * (host-loaded CSR copies included; borrowed EF_DEVICE_PTRS arrays stay the
 * caller's). hipFree waits for work still queued on the graph, so the handle
 * may be freed right after an asynchronous ef_compute. Bookkeeping only: no
 * step of the method. EF_ERR_ARG for a null handle; g is invalid afterwards. */
ef_status ef_graph_free(ef_graph *g);

/* Copy the load-time figures of g (sizes, W of Algorithm 1, degree sums) into
 * the caller's *out. Host only, no device work. EF_ERR_ARG if g or out is null. */
ef_status ef_graph_info_get(const ef_graph *g, ef_graph_info *out);

/* Expected Force (Eq. 1) of all nodes (seeds == NULL: outputs indexed by node
 * id, length n) or of seeds[0..n_seeds) (outputs position-aligned with seeds;
 * duplicates allowed). ef receives EF as double; D and N (nullable) receive
 * the exact int64 sums. Selected seeds always use the per-seed formulation.
 * Flags: EF_OUT_DEVICE, EF_PROFILE. */
ef_status ef_compute(ef_graph *g, ef_algo algo, ef_prec prec, const int32_t *seeds,
                     int32_t n_seeds, double *ef, int64_t *D, int64_t *N, uint32_t flags,
                     void *hip_stream);

/* Expected Force with three transmission events: Sec. 3.3 defines EF for a
 * number j of events and evaluates j = 2 (ef_compute); this is j = 3. Every
 * ordered sequence of three events from the seed counts once, as Algorithm 1
 * counts the two-event sequences: event 1 s -> y, event 2 from s or y, event
 * 3 from s, y or the second node, each to a susceptible neighbour of its
 * infector. The cluster degree is the number of edges leaving the four
 * infected nodes; N, D and EF then follow Eq. 1 as for j = 2 (EF = +0.0 when
 * D = 0 or N <= 1). N(s) equals the two-event D(s).
 * Arguments, outputs, seeds, duplicates and flags (EF_OUT_DEVICE,
 * EF_PROFILE) as ef_compute; ef_stats reports the item, finalize and FP64
 * recompute times (t_stream_ms, t_finalize_ms, t_pass2_ms) and the number of
 * recomputed seeds (promoted). FP32C scores in FP32 and sums in double; a
 * seed whose EF cancels (kappa = (S/D)/EF > 16 or EF <= 0) is recomputed in
 * FP64. The work is the number of sequences, about k_s^3 for a seed of
 * degree k_s: intended for graphs of moderate degree. EF_ERR_OVERFLOW when a
 * requested seed's sums could exceed int64. Synchronises the stream in FP32C
 * mode (the recompute list is built on the host). */
ef_status ef_compute_j3(ef_graph *g, ef_prec prec, const int32_t *seeds, int32_t n_seeds,
                        double *ef, int64_t *D, int64_t *N, uint32_t flags, void *hip_stream);

/* SIR outbreaks on the graph (Sec. 3.1) and the empirical spreading power of
 * every node (Sec. 3.3), to check EF against simulated spreading. Discrete
 * steps: every node infected at the start of a step infects each susceptible
 * neighbour with probability beta (the smallest successful infector is the
 * node's infector), then recovers with probability mu; an outbreak ends when
 * no node is infected or after t_max steps. The paper's calibration is
 * mu = 1/3, beta = 1.3 / (3 <k>). Every decision is a SplitMix64 draw on a
 * counter of (seed, simulation, step, arc or node), so results are
 * reproducible and independent of scheduling:
 *   stream(r, t) = mix(mix(seed ^ r) ^ (t + 1)) for simulation r, step t;
 *   the attempt along arc e draws mix(stream ^ (2e) K), the recovery of node
 *   u draws mix(stream ^ (2u + 1) K), K = 0xD1B54A32D192ED03; the index case
 *   is the high 64 bits of mix(mix(seed ^ r) ^ ~0) * n; a decision of
 *   probability p succeeds when (draw >> 11) < floor(p 2^53).
 * Outputs (host memory): per simulation r < n_sims the index case, size
 * (nodes ever infected), t_end (steps run) and t_peak (first step with the
 * most infected nodes); over the global simulations (size >= n/4, rounded
 * up): inf_count[v] = those in which v was infected, and sp_sum[(d-1) n + v]
 * = the sum over them of v's descendants within d generations of the
 * infection tree, d = 1..4 (divide by inf_count for the empirical spreading
 * power of order d). Nullable: work[0] = arcs walked by the attempts (one draw
 * each), work[1] = frontier node-steps (infected nodes summed over the steps
 * run); phase_ms[0..2] = kernel time of the attempts, of the updates with
 * their prefix kernels, and of the descendant counts, from HIP events on the
 * stream. Simulations run in batches of up to 1024 sharing about 3 GB of the
 * graph's scratch memory (13 bytes per node and simulation). The stream is
 * synchronised every 8 steps and at the end. EF_ERR_ARG for beta or mu
 * outside [0, 1], negative n_sims or t_max, null outputs, or simulations on
 * a graph without nodes. */
ef_status ef_sir(ef_graph *g, double beta, double mu, uint64_t seed, int32_t n_sims,
                 int32_t t_max, int32_t *index, int32_t *size, int32_t *t_end, int32_t *t_peak,
                 int64_t *sp_sum, int64_t *inf_count, int64_t *work, double *phase_ms,
                 void *hip_stream);

/* The k nodes of largest EF ("key nodes", the paper's title and Sec. 1):
 * computes EF of all nodes with `algo` / `prec`, then writes nodes[0..k) and
 * (nullable) ef[0..k) in EF-descending order, ties by node id ascending.
 * 0 <= k <= n, else EF_ERR_ARG. Flags: EF_OUT_DEVICE (nodes / ef are device
 * pointers, asynchronous on hip_stream), EF_PROFILE. */
ef_status ef_topk(ef_graph *g, ef_algo algo, ef_prec prec, int32_t k, int32_t *nodes,
                  double *ef, uint32_t flags, void *hip_stream);

/* Top-k selection alone (the ranking step of ef_topk, for EF a caller already
 * holds, e.g. from ef_compute with EF_OUT_DEVICE): ef_in is a device array of
 * the graph's n values, non-negative (a value that is not positive counts as
 * 0); writes nodes[0..k) and (nullable) ef[0..k) in descending order, ties by
 * node id ascending. The selection runs on the device with scratch memory
 * held by the handle. 0 <= k <= n, else EF_ERR_ARG. Flags: EF_OUT_DEVICE
 * (nodes / ef are device pointers, asynchronous on hip_stream); without it
 * they are host memory and the call synchronises the stream. */
ef_status ef_topk_values(ef_graph *g, const double *ef_in, int32_t k, int32_t *nodes,
                         double *ef, uint32_t flags, void *hip_stream);

/* ef_topk_values without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc. Same selection and order (descending, ties by id
 * ascending) over the n device values ef_in, written to the device arrays
 * nodes[0..k) and (nullable) ef[0..k); no graph handle. Its scratch is a fixed
 * 3 MiB array in device memory that each GPU holds from the library's load to
 * process end; it is resolved on the calling thread's current device (which
 * must own ef_in, nodes, ef and hip_stream) on the first call there. The call
 * makes no hipMalloc / hipFree and no other allocating call, and no memset
 * (every scratch word it reads is written by the same call first), so it can
 * be captured. Calls that overlap on one GPU (two streams, two threads) share
 * that array and race: serialise them. Asynchronous on hip_stream.
 * EF_ERR_ARG unless 0 <= k <= n and k <= 65536, flags == EF_OUT_DEVICE, and
 * ef_in / nodes are non-null when k > 0; EF_ERR_DEVICE if the array's address
 * cannot be obtained or a launch fails. */
ef_status ef_topk_values_noalloc(const double *ef_in, int32_t n, int32_t k, int32_t *nodes,
                                 double *ef, uint32_t flags, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Batches: many graphs computed together. The caller concatenates the graphs
 * into one disjoint union: graph i owns nodes node_off[i] .. node_off[i+1]-1,
 * row_ptr / col_idx are the union's CSR (global ids, host memory, copied).
 * EF of a node of the union equals its EF in its own graph, since a cluster
 * never spans two components (Sec. 3.3). One call computes every graph, in
 * one of two designs:
 *   phased      each phase of the exact path runs once over the whole batch
 *               (one launch per phase and degree bin);
 *   persistent  a single launch of a persistent kernel whose workgroups take
 *               (graph, bin, chunk) work items from an atomic cursor; each
 *               graph moves to its next phase as soon as its own items of
 *               the previous one are done.
 * The launch sequence of a design is captured into a HIP graph on its first
 * use and replayed afterwards. On first use the batch is tuned: both designs
 * are timed with several settings (small-degree bin thresholds; chunk sizes
 * of the persistent items) and the fastest is kept; the choice is cached for
 * the process per size class (graphs, nodes, arcs, largest degree, each
 * rounded up to a power of two) and precision, so a later batch of the same
 * class is not timed again. Outputs are per node of the union, in union
 * order (cluster-centric).
 * ------------------------------------------------------------------------- */
typedef struct ef_batch ef_batch;

#define EF_BATCH_PHASED     0x10u  /* batch compute: use the phased design */
#define EF_BATCH_PERSISTENT 0x20u  /* batch compute: use the persistent design */

typedef struct {
  int32_t n_graphs;
  int32_t n;              /* nodes of the union */
  int64_t nnz;            /* arcs of the union */
  int64_t clusters;       /* W of the union */
  double replay_ms;       /* last graph replay (set when called with EF_PROFILE) */
  float tune_ms[8];       /* phased design: eager pass time of each threshold candidate */
  int32_t tuned_choice;   /* phased design: index of the chosen candidate */
  int32_t thr8, thr16, thr32; /* phased design: chosen small-bin thresholds */
  float persist_tune_ms[8];   /* persistent design: time of each candidate (thresholds x
                                 chunk sizes) */
  int32_t persist_choice;     /* persistent design: index of the chosen candidate */
  int32_t design;             /* design used without a flag: 0 phased, 1 persistent */
  int32_t items;              /* work items of the persistent schedule */
  int32_t from_cache;         /* 1: the tuning came from the size-class cache */
  int32_t size_class;         /* the batch's size class */
  int32_t persist_pass2;      /* last synchronised persistent launch: pass-2 seeds */
  int32_t persist_fp64;       /*   and FP64-finalised seeds */
} ef_batch_stats;

/* EF_VALIDATE also checks that no arc leaves its graph (EF_ERR_RANGE). */
ef_status ef_batch_create(int32_t n_graphs, const int32_t *node_off, int64_t nnz,
                          const int32_t *row_ptr, const int32_t *col_idx, uint32_t flags,
                          void *hip_stream, ef_batch **out);

/* Tune the batch (see above): time every candidate of both designs on this
 * batch (eager passes) and keep the fastest, or take the size class's cached
 * choice; drops any captured graph. */
ef_status ef_batch_autotune(ef_batch *b, ef_prec prec);

/* EF, D, N (D, N nullable) of every node of the union. Host outputs: returns
 * after the copy. EF_OUT_DEVICE: asynchronous on hip_stream. EF_PROFILE:
 * records the replay time (ef_batch_stats_get). EF_BATCH_PHASED or
 * EF_BATCH_PERSISTENT runs that design (untuned settings if the batch was
 * never tuned); without either, the tuned design (tuning on first use).
 * EF_ERR_DEVICE if, in a synchronised call, the persistent kernel reports a
 * wait that exceeded its bound (no result is then complete). */
ef_status ef_batch_compute(ef_batch *b, ef_prec prec, double *ef, int64_t *D, int64_t *N,
                           uint32_t flags, void *hip_stream);

/* Copy the batch's sizes, tuning record and last replay time into the
 * caller's *out. Host only, no device work. EF_ERR_ARG if b or out is null. */
ef_status ef_batch_stats_get(const ef_batch *b, ef_batch_stats *out);

/* Release a batch: its captured graph, persistent-kernel schedule, device
 * arrays, events and own stream. hipFree waits for queued work. Bookkeeping
 * only: no step of the method. EF_ERR_ARG for a null handle; b is invalid
 * afterwards. */
ef_status ef_batch_free(ef_batch *b);

/* ---------------------------------------------------------------------------
 * Learned surrogate. A small MLP (16 features -> 64 -> GELU -> 64 -> GELU -> 1;
 * BF16 weights and activations, FP32 accumulation on the matrix cores) that
 * predicts the residual ln N(s) - EF(s) from cheap per-node features; it is
 * trained on the GPU on exact EF from this library, and the exact kernel
 * rescores its candidates, judges its rank agreement and stands in for it
 * when the agreement is too low. The surrogate is not part of the paper's
 * method; it is a production pattern around the exact path.
 * ------------------------------------------------------------------------- */
typedef struct ef_surrogate ef_surrogate;

typedef struct {
  float lr;            /* Adam step size */
  int32_t epochs;      /* maximum passes over the training rows */
  int32_t batch;       /* rows per step (>= 32) */
  uint64_t seed;       /* shuffling and split */
  float weight_decay;  /* decoupled weight decay per step (0 = none) */
  float val_fraction;  /* held-out share for early stopping, in [0, 0.9) */
  int32_t patience;    /* epochs without validation improvement before stopping */
  float lr_end;        /* step size of the last step as a share of lr, in (0, 1]: the
                          step size follows a half cosine from lr down to lr * lr_end
                          over the configured epochs (1: constant) */
} ef_train_cfg;

typedef struct {
  int32_t epochs_run;
  float train_loss;    /* mean squared error on the training rows (final weights) */
  float val_loss;      /* best validation mean squared error */
  float train_ms;      /* GPU time of the training loop */
  int64_t rows, val_rows;
} ef_train_report;

typedef struct {
  int32_t candidates;  /* nodes rescored exactly */
  int32_t sample;      /* nodes in the judge's random sample */
  float spearman;      /* rank correlation of surrogate and exact EF on the sample */
  int32_t fallback;    /* 1 if the exact top-k of the whole graph was returned */
  float t_predict_ms, t_rescore_ms, t_judge_ms;
} ef_judge_report;

/* A surrogate with random (He-normal) weights and identity standardisation. */
ef_status ef_surrogate_create(uint64_t seed, ef_surrogate **out);
ef_status ef_surrogate_free(ef_surrogate *s);
/* params: 5313 FP32 values (W1 16x64, b1 64, W2 64x64, b2 64, w3 64, b3;
 * row-major, input index first); mean / inv_std: 16 values each. Any may be
 * NULL. set_params resets the optimiser state. */
ef_status ef_surrogate_get_params(ef_surrogate *s, float *params, float *mean, float *inv_std);
ef_status ef_surrogate_set_params(ef_surrogate *s, const float *params, const float *mean,
                                  const float *inv_std);
ef_status ef_surrogate_save(ef_surrogate *s, const char *path);
ef_status ef_surrogate_load(ef_surrogate *s, const char *path);

/* The 16 raw per-node features (row-major n x 16) and ln N(s) per node:
 * ln(1+k), ln(1+A), ln(1+B), asinh(m3), asinh(m4), ln(1+A-k), ln(1+N),
 * ln(1+D'), ln(D'/N), max/min/mean/std of ln(neighbour degree), ln(1+Q),
 * share of degree-1 neighbours, ln(1+max(m2, 0)); A, B = sums of neighbour
 * degrees and of their squares, Q = sum over neighbours of their
 * neighbour-degree sums, N in closed form, D' the sum of the cluster degrees
 * taken without the triangle term, and m_j = E[x^j] over the node's N event
 * sequences with x = d / (D'/N) - 1 (sums of d^2, d^3, d^4 in closed form
 * per arc, triangle clusters without their -2). ln N - EF =
 * m2/2 - m3/6 + m4/12 - ... when the triangle terms are left out. No
 * triangle pass is run: a call costs the arcs' neighbour-sum gathers.
 * EF_OUT_DEVICE: X and lnN are device pointers. */
ef_status ef_features(ef_graph *g, float *X, float *lnN, uint32_t flags, void *hip_stream);

/* Gradient of the mean squared error of the network on (X, y) (host, rows x
 * 16 inputs used as given) into grad[5313]; loss = the mean squared error.
 * For checking the training kernels against a CPU reference. */
ef_status ef_surrogate_gradients(ef_surrogate *s, const float *X, const float *y, int64_t rows,
                                 float *grad, float *loss, void *hip_stream);

/* The network's output y[i] (the predicted ln N - EF) for rows of 16 inputs
 * X (row-major, used as given: standardise raw features first), on the same
 * BF16-operand MFMA kernel that ef_surrogate_predict runs. Host X and y
 * (copied; the call synchronises), or device pointers with EF_OUT_DEVICE
 * (asynchronous on hip_stream). rows >= 0, else EF_ERR_ARG. */
ef_status ef_surrogate_forward(ef_surrogate *s, const float *X, int64_t rows, float *y,
                               uint32_t flags, void *hip_stream);

/* Train on host rows: X raw features (rows x 16), y targets (ln N - exact EF).
 * Standardises the features (stored with the surrogate), then runs Adam on the
 * GPU, its step size decaying along a half cosine (cfg->lr_end), with early
 * stopping on a held-out share. */
ef_status ef_surrogate_train(ef_surrogate *s, const float *X, const float *y, int64_t rows,
                             const ef_train_cfg *cfg, ef_train_report *rep, void *hip_stream);

/* Predicted EF of every node of g (double, length n). EF_OUT_DEVICE: device
 * output, asynchronous. */
ef_status ef_surrogate_predict(ef_surrogate *s, ef_graph *g, double *ef_pred, uint32_t flags,
                               void *hip_stream);

/* Top-k by the surrogate with exact rescoring: the rerank_factor * k best
 * nodes by predicted EF are rescored by the exact per-seed kernel and the k
 * best by exact EF returned (host arrays nodes[k], ef_exact[k] nullable).
 * The judge compares surrogate and exact EF on judge_sample random nodes
 * (seeded); if their Spearman correlation is below min_spearman, the exact
 * top-k of the whole graph is returned instead (rep->fallback = 1). */
ef_status ef_topk_surrogate(ef_graph *g, ef_surrogate *s, int32_t k, int32_t rerank_factor,
                            int32_t judge_sample, float min_spearman, uint64_t seed,
                            int32_t *nodes, double *ef_exact, ef_judge_report *rep,
                            void *hip_stream);

/* Copy the counters and (with EF_PROFILE) phase times of the last ef_compute
 * on g into the caller's *out. Host only: the figures are those the call left
 * after its stream was synchronised. EF_ERR_ARG if g or out is null. */
ef_status ef_stats(const ef_graph *g, ef_run_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* EF_H_ */
