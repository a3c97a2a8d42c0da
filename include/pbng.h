/*
 * pbng.h -- C ABI of the MI355X (gfx950) butterfly-peeling library.
 *
 * The library computes, for a simple bipartite graph G(W = (U, V), E):
 *   - per-vertex and per-edge butterfly counts (Section 2.1, Algorithm 1),
 *   - tip numbers of every vertex of one side (Section 2.2, Definition 2;
 *     two-phase peeling of Section 3.2),
 *   - wing numbers of every edge (Section 2.2, Definition 1; two-phase
 *     peeling with the BE-Index of Sections 2.3 and 3.3, Algorithms 4-6).
 * All counts, supports and results are uint64 and exact; they never depend
 * on the number of partitions, the bound rule, tuning or batching.
 *
 * Graph format (pbng_csr): the U-side CSR.
 *   row_ptr : int64[n_u + 1], row_ptr[0] == 0, row_ptr[n_u] == m,
 *             non-decreasing.
 *   col_idx : int32[m], V ids in [0, n_v), strictly increasing in each row
 *             (no duplicate edges).
 *   Edge id e is the CSR slot: edge e joins the row u with
 *   row_ptr[u] <= e < row_ptr[u+1] to V-vertex col_idx[e].  Per-edge outputs
 *   are in edge-id order.
 *   on_device: 1 when row_ptr / col_idx are HIP device pointers; 0 for host
 *   memory.  Output buffers live in the same memory space as the graph.
 *
 * Ownership: the caller owns the graph and every output buffer.  The library
 * keeps no pointer to them after a call returns.  Work memory belongs to the
 * context and is released by pbng_destroy.
 *
 * Synchronicity: every compute call enqueues on the context's stream and
 * returns after the results are complete in the output buffers.
 * Threads: a context must not be used by two host threads at once.
 *
 * Errors: functions return 0 on success or a negative PBNG_E_* code; the
 * output contents are then unspecified.  pbng_last_error gives a message.
 * No C++ exception crosses this interface.
 */
#ifndef PBNG_H
#define PBNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBNG_OK 0
#define PBNG_E_ARG (-1)         /* null pointer, negative size, bad enum    */
#define PBNG_E_GRAPH (-2)       /* unsorted row, duplicate or out-of-range id */
#define PBNG_E_NOMEM (-3)       /* device allocation failed                   */
#define PBNG_E_DEVICE (-4)      /* HIP runtime error (see pbng_last_error)    */
#define PBNG_E_OVERFLOW (-5)    /* size beyond the library's index widths     */
#define PBNG_E_TIMEOUT (-6)     /* reserved: no call of this version returns
                                   it (no device wait here is bounded by
                                   time; every wait ends by construction)  */
#define PBNG_E_UNSUPPORTED (-7) /* reserved: option not available (every
                                   option of this version is built)        */

typedef struct pbng_ctx pbng_ctx;

typedef struct {
    int64_t n_u, n_v, m;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    int32_t on_device;
} pbng_csr;

typedef enum {
    PBNG_COUNT_VERTEX_U = 0, /* out: uint64[n_u], butterflies containing each u */
    PBNG_COUNT_VERTEX_V = 1, /* out: uint64[n_v]                              */
    PBNG_COUNT_EDGE = 2      /* out: uint64[m], butterflies containing each edge */
} pbng_count_kind;

typedef enum { PBNG_SIDE_U = 0, PBNG_SIDE_V = 1 } pbng_side;

/* Bound rules for the coarse-grained ranges (Section 3.1.3).  Ranges only
 * shape the schedule; results are identical under every rule.             */
typedef enum {
    PBNG_BOUND_PLAIN = 0,   /* the paper's work-estimate rule with adaptive
                               target and scaling factor; tip ranges also
                               end at a vertex-count target, and a small
                               heavy core is peeled one level per partition */
    PBNG_BOUND_LEARNED = 1, /* predicted entity numbers from a loaded MLP;
                               the plain rule when no predictor is loaded   */
    PBNG_BOUND_RANDOM = 2,  /* seeded random increasing bounds (tests)      */
    PBNG_BOUND_PAPER = 3    /* the paper's rule alone (Section 3.1.3): tip
                               ranges end at the work crossing only, with
                               neither the library's vertex-count target nor
                               its single-level partitions (PLAIN has both;
                               wing is the same under both rules)          */
} pbng_bound_rule;

/* flags */
#define PBNG_F_NO_DYNAMIC 0x1   /* keep peeled entities in the lists (no
                                   dynamic graph updates, Section 5.2)     */
#define PBNG_F_NO_BATCH 0x2     /* tip: never recount; wing: per-edge update
                                   in the coarse-grained rounds (every peeled
                                   edge walks its blooms) instead of one
                                   bloom-aggregated update per bloom
                                   (Section 5.1; with PBNG_F_NO_DYNAMIC the
                                   PBNG-- ablation of Section 6)            */
#define PBNG_F_NO_DENSE_TILE 0x4 /* counting: scalar path for hub pairs too */
#define PBNG_F_KERNEL_TIMING 0x8 /* time kernel classes with HIP events on
                                    the context stream (fills
                                    pbng_stats.kstat); coarse-grained tip
                                    rounds are then driven from the host    */
#define PBNG_F_HOST_ROUNDS 0x10  /* tip and wing: coarse-grained rounds
                                    driven from the host, one
                                    synchronisation per round, instead of
                                    replays of a captured HIP graph of
                                    several rounds                           */
#define PBNG_F_SHORT_PROBE 0x20  /* tip: the key-range peel kernel gives up
                                    after one LDS probe, so most of its
                                    items take the exact HBM overflow pass
                                    (a test hook for that path; results are
                                    unchanged, only slower)                  */

/* Kernel classes timed under PBNG_F_KERNEL_TIMING. */
enum {
    PBNG_K_COUNT = 0,   /* wedge-traversal counting / recounting            */
    PBNG_K_TIP_PEEL = 1,/* coarse-grained tip peel rounds                   */
    PBNG_K_FD = 2,      /* fine-grained (per-partition) peeling             */
    PBNG_K_WING_CD = 3, /* coarse-grained wing batch updates                */
    PBNG_K_DENSE = 4,   /* int8 matrix-core hub tiles                       */
    PBNG_K_TIP_HRANGE = 5, /* coarse-grained tip peel: the (vertex, key
                              range) LDS hash kernel alone                  */
    PBNG_K_TIP_TILED = 6,  /* coarse-grained tip peel: the (vertex, key
                              tile) LDS counter kernel alone                */
    PBNG_K_NCLASS = 7
};

typedef struct {
    double ms;          /* summed event time of the class's launches         */
    uint64_t launches;  /* timed intervals (one per round / pass)            */
    uint64_t bytes;     /* algorithmic bytes the method moves in them        */
    uint64_t wedges;    /* wedges (or links) walked in them                  */
} pbng_kernel_stat;

typedef struct {
    int32_t P;          /* partitions; 0 = default (tip 150; wing 400 below
                           1e8 edges, 1000 at or above), clamped to the
                           work-efficiency bound of Section 4.2, minimum 1   */
    int32_t bound_rule; /* pbng_bound_rule                                   */
    int32_t flags;      /* PBNG_F_*                                          */
    int32_t seed;       /* seed of PBNG_BOUND_RANDOM                         */
    int32_t dense_cut;  /* degree above which hub pairs use the int8 matrix-
                           core path in counting; 0 = library default,
                           negative = never                                 */
    int32_t tile_w;     /* coarse-grained tip rounds: active vertices with
                           more live wedges than this count in LDS key tiles,
                           others in LDS hash ranges; 0 = library default
                           (the larger of 2^16 and 16384 per 2^16-vertex
                           tile of the side), negative = never (schedule
                           only)                                             */
    int32_t batch_edges;/* batch calls: most edges packed into one union
                           graph; 0 = library default (2^26)                 */
    int32_t wide_work;  /* wing: fine-grained work above which a partition
                           is peeled by device-wide kernels; 0 = library
                           default (2^24), negative = never (schedule only)  */
    int32_t level_alive;/* tip: coarse-grained partitions of one support
                           level each (they need no fine-grained peeling)
                           once at most this many vertices are alive; 0 =
                           library default (1024 vertices holding at least
                           2^30 wedges of work, 2^21 per vertex), positive =
                           at that count whatever the work, negative = never
                           (schedule only)                                  */
    int32_t recount_w;  /* tip: a coarse-grained round recounts the remaining
                           graph instead of peeling when its active set's
                           live wedges exceed this (Section 5.1); 0 = the
                           paper's bound, the sum over edges of
                           min(d_u, d_v) in the input graph; negative = never
                           (schedule only)                                  */
} pbng_opts;

/* Per-call counters and phase times of the last compute call. */
typedef struct {
    double ms_total, ms_prep, ms_count, ms_cd, ms_fd_prep, ms_fd;
    uint64_t wedges;          /* wedges walked by all traversal kernels      */
    uint64_t wedges_count;    /* of which by counting / recounting           */
    uint64_t wedges_cd;       /* of which by coarse-grained peeling          */
    uint64_t wedges_fd;       /* of which by fine-grained peeling            */
    uint64_t updates;         /* support updates applied (wing)              */
    uint64_t links;           /* bloom-edge links walked (wing)              */
    uint64_t blooms, bloom_pairs; /* BE-Index size (wing)                    */
    uint64_t rho;             /* coarse-grained peeling rounds (syncs)       */
    uint64_t recounts;        /* tip rounds done by recounting (Section 5.1) */
    int32_t partitions;       /* partitions actually created; tip may exceed
                                 P when a small heavy core is peeled one
                                 support level per partition               */
    int32_t P_used;           /* partitions requested after clamping         */
    int32_t bound_rule_used;  /* pbng_bound_rule the call actually used      */
    int32_t fd_wide;          /* wing: partitions peeled by device-wide
                                 kernels instead of one workgroup            */
    uint64_t fd_work_max, fd_work_sum; /* estimated fine-grained work        */
    uint64_t dense_pairs;     /* hub pairs counted on matrix cores           */
    pbng_kernel_stat kstat[PBNG_K_NCLASS];
} pbng_stats;

/* Create a context bound to the current HIP device and the given stream
 * (hipStream_t, may be NULL for the default stream).                      */
int pbng_create(pbng_ctx **ctx, void *hip_stream);
void pbng_destroy(pbng_ctx *ctx);
const char *pbng_last_error(pbng_ctx *ctx);
int pbng_last_stats(pbng_ctx *ctx, pbng_stats *out);

/* Butterfly counts (Section 2.1, Algorithm 1; hub pairs optionally by an
 * int8 matrix product on matrix cores).  out: see pbng_count_kind.        */
int pbng_count(pbng_ctx *ctx, const pbng_csr *g, pbng_count_kind kind,
               const pbng_opts *opts, uint64_t *out);

/* pbng_count without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same results as pbng_count.  The graph (on_device
 * must be 1) and out are the caller's device buffers; every other byte the
 * call needs comes from one static 64 MiB array per device that the library
 * holds until the process ends.  Graphs whose relabelled vertex and edge
 * arrays alone exceed it (40 bytes per edge plus 32 per vertex) return
 * PBNG_E_OVERFLOW before any work; a graph that passes that check but needs
 * more scratch (dense counters of large starts, hub tiles) returns
 * PBNG_E_NOMEM.  Calls on one device share the array and keep the last
 * call's contents: calls that overlap on one device (two contexts, two host
 * threads, two streams) race and must be serialised by the caller.        */
int pbng_count_noalloc(pbng_ctx *ctx, const pbng_csr *g, pbng_count_kind kind,
                       const pbng_opts *opts, uint64_t *out);

/* Tip numbers of one side (Definition 2; Section 3.2).  tip_out: uint64
 * [n_u] for PBNG_SIDE_U, [n_v] for PBNG_SIDE_V.  opts may be NULL.       */
int pbng_tip(pbng_ctx *ctx, const pbng_csr *g, pbng_side side,
             const pbng_opts *opts, uint64_t *tip_out);

/* Tip numbers with the learned range bounds taken from caller-supplied
 * predicted tip numbers instead of the predictor (Section 3.1.3 with the
 * support key replaced by a prediction): theta_hint uint64[n_side], in the
 * graph's memory space, read only.  Results never depend on the hint; with
 * the exact tip numbers as hint it shows what a perfect predictor would do
 * to the schedule.                                                         */
int pbng_tip_hinted(pbng_ctx *ctx, const pbng_csr *g, pbng_side side,
                    const pbng_opts *opts, const uint64_t *theta_hint,
                    uint64_t *tip_out);

/* Tip numbers plus the coarse-grained schedule that produced them (Section
 * 3.1, Algorithm 4; Theorem 1 states what it must satisfy).  Outputs, all in
 * the graph's memory space:
 *   tip_out    uint64[n_side]  tip numbers, as pbng_tip;
 *   part_out   int32[n_side]   partition of each vertex (0-based; the
 *                              partition during which it was peeled);
 *   init_out   uint64[n_side]  its support when its partition began, i.e.
 *                              its butterflies inside the vertices of its own
 *                              and later partitions (the initialisation
 *                              vector of the fine-grained phase);
 *   bounds_out uint64[bounds_cap]  exclusive upper bound theta(i+1) of
 *                              partition i for i < min(partitions, cap)
 *                              (UINT64_MAX for a final partition that takes
 *                              every remaining vertex);
 *   *nparts    number of partitions created (may exceed bounds_cap).
 * By Theorem 1 every vertex of partition i has theta(i) <= tip < theta(i+1)
 * with theta(0) = 0.  bounds_out may be NULL when bounds_cap is 0.        */
int pbng_tip_schedule(pbng_ctx *ctx, const pbng_csr *g, pbng_side side,
                      const pbng_opts *opts, uint64_t *tip_out,
                      int32_t *part_out, uint64_t *init_out,
                      uint64_t *bounds_out, int32_t bounds_cap,
                      int32_t *nparts);

/* Wing numbers of every edge (Definition 1; Section 3.3, Algorithms 4-6).
 * wing_out: uint64[m].  opts may be NULL.                                 */
int pbng_wing(pbng_ctx *ctx, const pbng_csr *g, const pbng_opts *opts,
              uint64_t *wing_out);

/* ---- Hierarchy retrieval (Section 2.2, Definitions 1-2) -------------------
 *
 * The k-tips of one side are the butterfly-connected components of its
 * vertices with tip number >= k (with all of the other side): two vertices
 * are joined when they share at least two neighbours, i.e. lie in a common
 * butterfly.  The k-wings are the butterfly-connected components of the
 * edges with wing number >= k: two edges are joined when a butterfly whose
 * four edges all have wing number >= k holds both.  theta: the entity
 * numbers from pbng_tip (uint64[n_side]) or pbng_wing (uint64[m]); comp_out:
 * int32 of the same length, the smallest id in the entity's k-tip / k-wing,
 * or -1 for entities below k.  Both in the graph's memory space.  Levels
 * nest: every (k+1)-tip lies inside one k-tip, and likewise for wings.     */
int pbng_tip_components(pbng_ctx *ctx, const pbng_csr *g, pbng_side side,
                        const uint64_t *theta, uint64_t k, int32_t *comp_out);
int pbng_wing_components(pbng_ctx *ctx, const pbng_csr *g,
                         const uint64_t *theta, uint64_t k,
                         int32_t *comp_out);

/* ---- Many graphs per call ------------------------------------------------
 *
 * Tip numbers of one side / wing numbers of every edge of ng graphs.  A
 * butterfly never spans two connected components, so the graphs are packed
 * into their disjoint union (ids shifted by the totals of the graphs before)
 * and decomposed together: every launch, every coarse-grained round and the
 * one persistent fine-grained launch serve all graphs of a chunk, and its
 * fine-grained queue holds partitions of every graph.  Chunks are runs of
 * consecutive graphs with at most opts->batch_edges edges (a larger graph
 * forms a chunk of its own).  Results equal the single-graph calls'.
 *
 * g: host array of ng descriptors, all with the same on_device; outs: host
 * array of ng output pointers in that memory space, outs[k] of n_u[k] / n_v[k]
 * (tip) or m[k] (wing) entries.  Statistics sum over chunks.                */
int pbng_tip_batch(pbng_ctx *ctx, const pbng_csr *g, int32_t ng,
                   pbng_side side, const pbng_opts *opts,
                   uint64_t *const *outs);
int pbng_wing_batch(pbng_ctx *ctx, const pbng_csr *g, int32_t ng,
                    const pbng_opts *opts, uint64_t *const *outs);

/* ---- Autotuner -------------------------------------------------------------
 *
 * Times one call of `kind` (0: tip numbers of side U, 1: of side V, 2: wing
 * numbers) on g under schedule settings picked by coordinate descent from
 * *base (NULL = defaults): (tip, when the base rule is PLAIN or PAPER) the
 * bound rule, PLAIN against PAPER; the int8 hub cut-over dense_cut in
 * {-1 (off), 256, 1024, 4096}; (tip) the key-tile threshold tile_w in
 * {2^16, 2^18, 2^20, -1 (never)} and the recount bound recount_w in
 * {0 (Section 5.1), -1 (never)}; (wing) the device-wide partition threshold
 * wide_work, its default 2^24 against {2^22, 2^26, -1 (never)}; then the
 * partition count P:
 * the base value against P0/2 and 2 P0 (P0 = base P, else 150 for tip and
 * 400 for wing).  One untimed warm
 * run precedes the timed ones; each setting is timed once.  The fastest
 * setting goes to *best and its time in ms to *ms_best (may be NULL).  The
 * context caches it under the graph's signature (n_u, n_v, m, largest
 * degree, kind): a later call for the same signature returns the cached
 * setting without running anything.  Results never depend on the setting.  */
int pbng_autotune(pbng_ctx *ctx, const pbng_csr *g, int32_t kind,
                  const pbng_opts *base, pbng_opts *best, double *ms_best);

/* ---- Learned range bounds (Section 3.1.3 replaced by a predictor) -------
 *
 * The coarse-grained phase needs each partition's upper bound.  The paper
 * picks it from current supports with a work estimate; PBNG_BOUND_LEARNED
 * instead takes the work-weighted quantile of predicted tip numbers
 * theta_hat = r_hat * support, where r_hat in [0, 1] is the output of a
 * multilayer perceptron (8 inputs, three hidden layers of 64 ReLU units,
 * sigmoid output; fp32) on per-vertex features.  Results never depend on the
 * predictor: only the partition schedule does.
 *
 * Parameters: one flat float vector of PBNG_MLP_NPARAM entries laid out as
 * W1[64][8], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], w4[64], b4
 * (row-major, output index first).  Features, 8 per vertex of one side, with
 * d = degree, w = sum of neighbour degrees, dmax/dmin = largest/smallest
 * neighbour degree, S = butterfly support, Smax/Wmax = maxima over the side,
 * m = edges, L = natural log1p:
 *   L(d)/8, L(S)/32, L(w)/16, L(dmax)/12, L(dmin)/12, L(S)/L(Smax),
 *   L(w)/L(Wmax), L(m)/24   (0 for a vertex of degree 0, except the last;
 *   0 where a divisor is 0).
 * Training target: r = theta / S (0 when S = 0).  Loss: sum wt (r_hat - r)^2
 * / sum wt.  Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias
 * correction; one step per minibatch, rows in the order given.
 *
 * The parameters and Adam state belong to the context; the calls below run
 * on the context's stream and return when done.                            */
#define PBNG_MLP_NPARAM 8961

/* Features of every vertex of one side: feat[n_side * 8] (row-major), in the
 * same memory space as the graph.                                          */
int pbng_tip_features(pbng_ctx *ctx, const pbng_csr *g, pbng_side side,
                      float *feat);
/* Load predictor parameters from a file: a NumPy .npy array of
 * PBNG_MLP_NPARAM little-endian float32 values (version 1 or 2 header, C
 * order), in the layout above; Adam state cleared.  PBNG_E_ARG for a
 * missing or malformed file (the context then keeps its previous
 * parameters; without any, PBNG_BOUND_LEARNED runs the plain rule).        */
int pbng_predictor_load(pbng_ctx *ctx, const char *path);
/* He-uniform weights and zero biases from a seed; Adam state cleared.     */
int pbng_mlp_init(pbng_ctx *ctx, uint64_t seed);
/* Copy parameters in from / out to host memory (PBNG_MLP_NPARAM floats);
 * set clears the Adam state.  get fails with PBNG_E_ARG before any init.  */
int pbng_mlp_set(pbng_ctx *ctx, const float *params);
int pbng_mlp_get(pbng_ctx *ctx, float *params);
/* r_hat for n rows of x (device [n * 8]) into y (device [n]).            */
int pbng_mlp_forward(pbng_ctx *ctx, const float *x, int64_t n, float *y);
/* Loss and gradient over n rows (device x [n*8], r [n], wt [n]); grad is
 * device [PBNG_MLP_NPARAM], loss a host float.                             */
int pbng_mlp_loss_grad(pbng_ctx *ctx, const float *x, const float *r,
                       const float *wt, int64_t n, float *grad, float *loss);
/* epochs passes of minibatch Adam over n rows (device pointers) with the
 * given batch size and learning rate; epoch_loss (host [epochs], may be
 * NULL) receives each epoch's mean loss as the epoch went.                 */
int pbng_mlp_train(pbng_ctx *ctx, const float *x, const float *r,
                   const float *wt, int64_t n, int32_t batch, int32_t epochs,
                   float lr, float *epoch_loss);

#ifdef __cplusplus
}
#endif
#endif /* PBNG_H */
