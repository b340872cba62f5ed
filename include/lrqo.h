/*
 * liblrqo — low-rank K-ary quadratic maximisation on one MI355X (gfx950).
 *
 * Problem (Sec. 1, eq. max_quad with the K-th roots of unity of eq. AK_def,
 * in the factor form of Sec. 2.2, eq. quad_max-norm):
 *
 *        maximise  ||V^H z||^2 = z^H (V V^H) z   over  z in A_K^n,
 *        A_K = { exp(2 pi i k / K) : k = 0 .. K-1 }.
 *
 * An assignment is returned as uint8 labels k_i (z_i = exp(2 pi i k_i / K)),
 * so K <= 255.  The objective is always the FP64 value ||V^H z||^2 of the
 * returned labels.
 *
 * Memory: every array argument named "device" must be device memory of the
 * current HIP device; host arguments are ordinary host memory.  The caller
 * owns all of them; the library never frees or keeps caller memory.  The
 * library's own scratch (per device, grown on demand) is released by
 * lrqo_shutdown().  The environment variable LRQO_ARENA_LIMIT (bytes), read
 * at every call, caps the scratch one call may need: a call needing more
 * returns LRQO_ENOMEM before any device work (as it does when the device
 * allocation itself fails).
 *
 * Ordering: work is enqueued on the stream set by lrqo_set_stream (the null
 * stream by default) and every solve call synchronises that stream before it
 * returns, because results are delivered to host memory.
 *
 * Errors: every call returns an lrqo_status; no exception crosses the ABI.
 * Argument errors are detected before any device work is issued.  A short
 * description of the last failure of the calling thread is available from
 * lrqo_last_error().  On error the contents of outputs are unspecified.
 */
#ifndef LRQO_H
#define LRQO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lrqo_status {
    LRQO_OK = 0,
    LRQO_EINVAL = -1,     /* argument out of range, null pointer, bad layout */
    LRQO_ENOMEM = -2,     /* device scratch could not be allocated */
    LRQO_EDEVICE = -3,    /* a HIP runtime call failed (message says which) */
    LRQO_ETOOBIG = -4,    /* exact enumeration larger than the cap */
    LRQO_ENOTFINITE = -5, /* V holds a NaN or an infinity */
    LRQO_EDEGENERATE = -6 /* warning only, never returned: reported in
                             lrqo_exact_result.warning */
} lrqo_status;

#define LRQO_MAX_R 8
#define LRQO_MAX_K 255
#define LRQO_MAX_TOPK 64

/* Version as major*10000 + minor*100 + patch. */
int32_t lrqo_version(void);

/* Text of the calling thread's last error ("" if none). */
const char* lrqo_last_error(void);

/* Stream used by later calls of the calling thread (a hipStream_t; NULL is
 * the null stream).  Returns LRQO_OK. */
lrqo_status lrqo_set_stream(void* hip_stream);

/* Release the library's device scratch on every device it touched. */
lrqo_status lrqo_shutdown(void);

/* --------------------------------------------------------------------------
 * Sampled maximisation (Sec. 4.2, eq. def_f; Thm. rr_tail).
 *
 * Draws directions c_s, s = first_index .. first_index + S - 1, uniformly on
 * the complex unit sphere of C^r as c = g / ||g||, g a standard Gaussian in
 * R^{2r} (proof of Lemma innerIsBeta), rounds each row by the decision rule
 * (Sec. 3, eq. decision_rule: z_i = the K-th root nearest in phase to
 * (V c)_i) and keeps the best f(c) = ||V^H z(c)||^2.
 *
 * Direction stream (the paper fixes none): Philox4x32-10 with key
 * (seed & 0xffffffff, seed >> 32) and counter (s & 0xffffffff, s >> 32,
 * instance, b) for blocks b = 0..ceil(2r/4)-1; word t of block b is uniform
 * u[4b+t] = ((x >> 9) + 1/2) * 2^-23; g[2j] = sqrt(-2 ln u[2j]) cos(2 pi u[2j+1]),
 * g[2j+1] = sqrt(-2 ln u[2j]) sin(2 pi u[2j+1]); c_j = (g[2j] + i g[2j+1])/||g||.
 * The device evaluates this stream in FP32.
 *
 * Scoring: every candidate is scored in FP32; the best `rescore_topk` FP32
 * scores (ties to the lower index) are re-evaluated in FP64 from the same
 * FP32 direction widened to FP64; the FP64 arg-max (ties to the lower index)
 * is the result.  Labels and objective are therefore exactly those of the
 * FP64 decision rule at the returned direction.
 *
 * V (device): n x r, row-major.  complex layout: interleaved FP32 (re, im),
 * element (i, j) at V[2*(i*r + j)]; real layout (options->real_v = 1):
 * FP32, element (i, j) at V[i*r + j].
 * z (device): n uint8 labels of the winner.
 * Ranges: 1 <= n <= 2^31 - 1, 1 <= r <= 8, 2 <= K <= 255,
 * 1 <= S <= 2^32 - 1; otherwise LRQO_EINVAL.
 * ------------------------------------------------------------------------ */

typedef struct lrqo_sampled_options {
    int32_t real_v;          /* 0: complex64 V; 1: real FP32 V */
    int32_t precision;       /* 0: FP32 scorer; 1: precision form (r <= 4,
                                else LRQO_EINVAL).  K = 2, 3, 4: V c and V^H z
                                on BF16 MFMA from three-part BF16 splits of V
                                and c (FP32-grade w; a label can differ from
                                the FP64 rule only within 256 u sum_j
                                |V_ij||c_j| of a decision boundary, u = 2^-24);
                                other K: V c on BF16 MFMA with hi + lo parts,
                                rows inside the BF16 error margin recomputed in
                                FP32.  The FP64 rescore is the same in both.
                                LRQO_BF16_FORM=w4 (read once per process)
                                selects the second form for every K */
    int32_t rescore_topk;    /* 1..64; 0 means 64 */
    uint32_t instance;       /* counter word 2 of the direction stream */
    uint64_t first_index;    /* index of the first direction (range splitting) */
    float* f_out;            /* optional device [S]: FP32 score of every direction */
    const float* directions; /* optional device [S][2r]: unit directions to score in
                                place of the stream ((re, im) pairs, FP32); then
                                first_index must be 0 and best_index indexes this list */
    /* Inspection outputs (each may be NULL / 0; they do not change the result): */
    float* dirs_out;         /* optional device [S][2r]: the FP32 direction each candidate
                                was scored with, (re, im) pairs */
    int32_t probe_count;     /* 0..64 candidates whose per-row labels the scorer writes */
    int32_t probe_pad;
    const int64_t* probe;    /* host [probe_count]: their positions 0..S-1 in this call */
    uint16_t* probe_labels;  /* device [probe_count][n]: the scorer's label of row i for
                                probe t at [t*n + i], | 0x100 when the precision form
                                recomputed that row in FP32 */
} lrqo_sampled_options;

typedef struct lrqo_sampled_result {
    int64_t best_index;      /* absolute stream index s of the winner */
    double obj;              /* FP64 ||V^H z||^2 of the returned labels */
    double fp32_obj;         /* the FP32 scorer's value for the same direction */
    double best_c[2 * LRQO_MAX_R]; /* winner's direction, FP64 copy of the FP32 values, (re, im) pairs */
    int64_t flagged_rows;    /* precision 1: row-candidates recomputed in FP32
                                (always 0 for K = 2, 3, 4, which recompute none) */
    float device_ms;         /* device time of the call, from stream events */
    float score_ms;          /* device time of the fused scoring kernel alone */
    int32_t rescored;        /* candidates that went through the FP64 rescore */
    int32_t slices;          /* row slices of the scoring launch */
} lrqo_sampled_result;

/* Complex V, FP32 scorer, 64-way FP64 rescore, instance 0, first index 0. */
lrqo_status lrqo_solve_sampled(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                               uint64_t seed, uint8_t* z, double* obj);

/* Full form.  opt may be NULL (defaults above); res (host) may be NULL. */
lrqo_status lrqo_solve_sampled_ex(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                                  uint64_t seed, const lrqo_sampled_options* opt, uint8_t* z,
                                  lrqo_sampled_result* res);

/* Allocation-free form of lrqo_solve_sampled_ex, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, semantics and results, but the library's
 * scratch (result record, roots, scores, slice sums, selection and rescore
 * buffers) lives in a static device array of LRQO_NOALLOC_SCRATCH_BYTES,
 * one per GPU, held until the process ends; the call allocates no device or
 * host memory.  A call whose scratch would exceed the array returns
 * LRQO_ETOOBIG before any device work (S up to 2^20 fits at any n for r <= 4
 * when the scorer needs one row slice, S = 65,536 with eight slices).  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (from
 * several host threads or streams) race, so callers serialise them.  The
 * array keeps the last call's contents; each call rewrites everything it
 * reads (the result record and the flag counter are cleared first). */
#define LRQO_NOALLOC_SCRATCH_BYTES (64u << 20)

lrqo_status lrqo_solve_sampled_noalloc(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                                       uint64_t seed, const lrqo_sampled_options* opt, uint8_t* z,
                                       lrqo_sampled_result* res);

/* --------------------------------------------------------------------------
 * Exact maximisation by arrangement-vertex enumeration (Sec. 3, Alg. 2,
 * Thm. rankr).
 *
 * Builds the augmented real rows a_{i,m} = [Im(rho_m V_i), Re(rho_m V_i)],
 * rho_m = exp(-i pi (2m+1)/K), m < B_K (eq. tildeV, Def. BK), enumerates every
 * set of 2d-1 rows with at most two per coordinate (d = r, r-1, ..., 1, the
 * recursion of Alg. 2 on the leading d columns) in colex order within each
 * level, solves the FP64 null vector of each set (twice-orthogonalised
 * Gram-Schmidt, by one thread per set up to d = 4 and by sixteen lanes per
 * set above; the set is full rank when its smallest residual exceeds
 * 1e-10 times its largest row norm), takes both signs, labels untouched rows
 * by the decision rule and tries, for coordinates in the set, both labels
 * beside the boundary (one row in the set) or all K labels (two rows:
 * V_i c = 0, Cor. two_implies_all).  Candidates are scored in FP32; the sets
 * are taken in chunks, and after each chunk its best sets join a shortlist of
 * the 64 best distinct FP32 scores (equal scores keep the set with the lowest
 * global index: every vertex of one cell gives the same score, and keeping
 * one of them leaves room for other assignments).  The shortlist is rescored
 * in FP64 and the FP64 maximum is returned (ties to the lower set index).
 *
 * V (device): n x r complex128, interleaved (re, im), row-major.
 * z (device): n uint8 labels.  obj (host): FP64 objective.
 * Ranges: 1 <= r <= 8, r <= n <= 2^31 - 1, 2 <= K <= 255, at most 2^20
 * label combinations per vertex (2^(2r-1-2p) K^p); the number of index sets
 * sum_d C(n B_K, 2d-1) must not exceed the cap: max_sets when positive, 2^34
 * when 0, and 2^62 when negative (the cap lifted); otherwise LRQO_ETOOBIG
 * before any device work.  Set indices are 64-bit.
 * A factor that violates general position (Assumption 1; for instance a real
 * V with K = 2, whose augmented rows only constrain Re c) makes valid sets
 * rank deficient: res->warning is LRQO_EDEGENERATE and the result is the best
 * candidate found, with no claim of optimality.
 * Environment (inspection only, the result does not depend on them):
 * LRQO_EXACT_CHUNK sets per chunk (default 2^26); LRQO_EXACT_FORM=fused
 * scores every set in one pass over all rows, =split runs the vertex /
 * row-slice / combine kernels; unset, the split form is taken only where it
 * slices the rows (n of 2,048 and more with few sets) and a chunk's per-set
 * buffers fit in 128 MB.
 * ------------------------------------------------------------------------ */

typedef struct lrqo_exact_result {
    double obj;              /* FP64 objective of the returned labels */
    int64_t index_sets;      /* valid index sets enumerated (all levels) */
    int64_t rank_deficient;  /* sets rejected by the rank test */
    int64_t candidates;      /* scored label vectors */
    float device_ms;
    int32_t warning;         /* LRQO_OK, or LRQO_EDEGENERATE when some valid set was rank
                                deficient: V is not in general position (Assumption 1);
                                the result is still the best candidate found */
} lrqo_exact_result;

lrqo_status lrqo_solve_exact(const double* V, int64_t n, int32_t r, int32_t K, uint8_t* z,
                             double* obj);

/* max_sets: the cap above; res (host) may be NULL. */
lrqo_status lrqo_solve_exact_ex(const double* V, int64_t n, int32_t r, int32_t K,
                                int64_t max_sets, uint8_t* z, lrqo_exact_result* res);

/* Null-vector randomized sampler (the randomized form of Alg. 2 compared
 * with uniform sphere sampling in Sec. 5, Table samplers): S draws of 2r-1
 * rows of the augmented matrix of the full factor; a draw whose rows are
 * distinct, hold at most two rows per coordinate and pass the rank test is
 * feasible and its vertex is scored exactly as lrqo_solve_exact_ex scores an
 * enumerated index set; the best FP64 objective wins (ties to the earlier
 * draw).  Draw s (the paper fixes no generator): with M = 2r-1 and N = n B_K,
 * row j = (2^32 w[2j+1] + w[2j]) mod N, w[4b+t] = word t of Philox4x32-10
 * with key (seed & 0xffffffff, seed >> 32) and counter (s & 0xffffffff,
 * s >> 32, 0x4E554C4C, b); the set is the sorted rows.  Same layouts and
 * limits as lrqo_solve_exact_ex except the cap and 1 <= S <= 2^31 - 1.
 * res->index_sets counts draws with distinct rows and at most two per
 * coordinate, res->rank_deficient those of them that fail the rank test.
 * No feasible draw returns LRQO_EINVAL. */
lrqo_status lrqo_solve_nullvec(const double* V, int64_t n, int32_t r, int32_t K, int64_t S, uint64_t seed,
                               uint8_t* z, lrqo_exact_result* res);

/* --------------------------------------------------------------------------
 * Batched sampled maximisation: many small instances in one persistent,
 * work-queue-driven launch (the sampled method of Sec. 4.2 on each).
 *
 * Instance t has factor V_t (n_t x r_t) starting at float offset
 * v_offset[t] of the device array V (complex64 interleaved, or real FP32
 * with options->real_v = 1), and is solved exactly as lrqo_solve_sampled_ex
 * would solve it alone with instance = t (counter word 2 of the direction
 * stream), the same seed and the same S.
 * z (device) receives the labels of instance t at offset
 * n_0 + ... + n_{t-1}; obj (host, count doubles) the FP64 objectives.
 * Ranges: 1 <= count <= 2^22, 1 <= n_t <= 256, 1 <= r_t <= 4,
 * 2 <= K <= 255, 1 <= S <= 4096.
 * The launch shape (directions per lane, persistent blocks per CU) is either
 * given in options or picked by timing the candidates on the device the
 * first time a batch signature (K, S, max r, mean-n bucket, count bucket)
 * is seen; choices are appended to the JSON-lines file named by
 * LRQO_TUNE_CACHE (default ~/.cache/lrqo_batched_tune.json).  The whole
 * sequence is captured once into a hipGraph per device and replayed while
 * count, K, S, seed, T, shape, pointers and the total row count stay the
 * same.  Calls are serialised per device.
 * ------------------------------------------------------------------------ */

typedef struct lrqo_batch_options {
    int32_t real_v;          /* 0: complex64 factors; 1: real FP32 factors */
    int32_t rescore_topk;    /* 1..64; 0 means min(64, S) */
    int32_t cpl;             /* directions per lane 1, 2 or 4; 0: tuned */
    int32_t blocks_per_cu;   /* persistent blocks per CU 1..16; 0: tuned */
    int32_t no_graph;        /* 1: launch directly instead of replaying a hipGraph */
    int32_t pad;
    int64_t* best_index;     /* optional host [count]: winning stream index per instance */
} lrqo_batch_options;

typedef struct lrqo_batch_result {
    float device_ms;         /* device time of the scoring sequence (graph replay) */
    int32_t cpl;             /* launch shape used */
    int32_t blocks_per_cu;
    int32_t items;           /* (instance, tile) work items */
    int32_t tuned_now;       /* 1 if the shape was tuned during this call */
    int32_t graph_captured_now;
    int64_t row_candidates;  /* sum over instances of n_t * S */
} lrqo_batch_result;

lrqo_status lrqo_solve_batched(const float* V, int32_t count, const int64_t* v_offset,
                               const int32_t* n, const int32_t* r, int32_t K, int64_t S,
                               uint64_t seed, const lrqo_batch_options* opt, uint8_t* z,
                               double* obj, lrqo_batch_result* res);

/* --------------------------------------------------------------------------
 * Learned direction proposal (rank 3).  A permutation-invariant network over
 * the rows of V (in a canonical gauge: V -> V G, G unitary from the fourth
 * moment sum_i |v_i|^2 v_i^H v_i and the K-th and first column moments)
 * gives a 32-component von Mises-Fisher mixture on the unit sphere of C^3;
 * lrqo_proposal_sample draws directions from it (every
 * round(1/uniform_fraction)-th one is the uniform stream's direction instead)
 * for lrqo_solve_sampled_ex(options.directions).  Parameters: 21,248 floats,
 * packed [W1 64x6, b1 64, W2 64x64, b2 64, W3 256x64, b3 256] row-major.
 * Training: lrqo_proposal_train_step computes the mean over a batch of
 * -log((1/K) sum_t p(omega^t c*_can)) for target directions c*, its gradient
 * (hand-written backward) and, with update = 1, one Adam step
 * (beta = 0.9, 0.999, eps = 1e-8).  V here is complex64 (n x 3) only.
 * A handle belongs to the device current at creation; calls on one handle
 * must not overlap.
 * ------------------------------------------------------------------------ */

typedef struct lrqo_proposal lrqo_proposal;

int32_t lrqo_proposal_param_count(void);

/* init (host): parameter count doubles.  *out receives the handle. */
lrqo_status lrqo_proposal_create(const double* init, int32_t K, lrqo_proposal** out);
lrqo_status lrqo_proposal_destroy(lrqo_proposal* p);

/* Parameters and Adam state to / from host memory (checkpoint / resume);
 * m, v and step may be NULL. */
lrqo_status lrqo_proposal_get_state(lrqo_proposal* p, float* theta, float* m, float* v, int64_t* step);
lrqo_status lrqo_proposal_set_state(lrqo_proposal* p, const float* theta, const float* m, const float* v,
                                    int64_t step);

/* V (device): instances concatenated, instance t at float offset
 * v_offset[t] (host), n[t] rows (host); targets (host): count x 6 floats,
 * the best direction of each instance as (re, im) pairs.  mean_loss (host)
 * and grad_out (host, parameter count floats) may be NULL. */
lrqo_status lrqo_proposal_train_step(lrqo_proposal* p, const float* V, int32_t count,
                                     const int64_t* v_offset, const int64_t* n,
                                     const float* targets, float lr, int32_t update,
                                     double* mean_loss, float* grad_out);

/* S directions (device dirs, S x 6 floats) for the factor V (device, n x 3
 * complex64); uniform directions come from stream (seed, instance). */
lrqo_status lrqo_proposal_sample(lrqo_proposal* p, const float* V, int64_t n, int64_t S, uint64_t seed,
                                 uint32_t instance, float uniform_fraction, float* dirs);

/* Canonical gauge of V (device, n x 3 complex64): frame_out (host, 19
 * doubles) = G (3x3 complex row-major, (re, im)) then the scale s. */
lrqo_status lrqo_proposal_frame(lrqo_proposal* p, const float* V, int64_t n, double* frame_out);

/* --------------------------------------------------------------------------
 * Exact rank-1 maximisation by the phase sweep (Sec. 2.5, Alg. 1,
 * Thm. rank1): maximise |z^H q|^2 over z in A_K^n for one vector q (the
 * rank-1 case of the problem; with q_i = v1_i + i v2_i built from two real
 * eigenvectors this is the two-eigenvector rounding of the appendix
 * "Rank-1 at Scale").
 *
 * q: device complex128 [n], interleaved (re, im); z: device uint8 [n] out.
 * Boundary points phi_i = (2 pi/K)(1/2 + floor(x_i) - x_i), x_i =
 * K arg(q_i)/(2 pi), are evaluated in FP64 with the operations in that order
 * and sorted stably (equal points keep coordinate order); the n+1 cells are
 * scored by FP64 prefix sums in a fixed order and the best cell wins (ties
 * to the earlier cell).  1 <= n <= 2^31 - 1, 2 <= K <= 255.  A non-finite
 * entry of q returns LRQO_ENOTFINITE.
 * ------------------------------------------------------------------------ */

typedef struct lrqo_rank1_result {
    double obj;              /* |z^H q|^2 of the returned labels (FP64, fixed-order sum) */
    double sweep_obj;        /* the chosen cell's value from the sweep's prefix sums */
    int64_t best_cell;       /* 0: assignment at phi = -pi/K; l: after the l-th boundary point */
    float device_ms;
    int32_t sort_passes;     /* 8-bit radix passes run: 4 over 32-bit images of the points, plus
                                those over the exact 64-bit keys (digits that differ) when a run
                                of more than 16 equal images holds distinct points */
} lrqo_rank1_result;

lrqo_status lrqo_solve_rank1(const double* q, int64_t n, int32_t K, uint8_t* z, lrqo_rank1_result* res);

/* --------------------------------------------------------------------------
 * Objective on the graph and greedy local refinement (the step after the
 * low-rank solve: labels scored on the original sparse matrix and improved by
 * single-vertex moves; appendix "Rank-1 at Scale", eq. incremental and the
 * hybrid warm start).
 *
 * Graph on n vertices as a symmetric adjacency in CSR, all arrays device
 * memory: row_ptr[n+1] (int64: row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz), col[nnz] (int32: 0 <= col < n, no self loop) and
 * w[nnz] (FP64 edge weights, finite) or NULL for unit weights.  Every edge
 * {i, j} must appear as (i, j) and (j, i) with equal weights (not checked).
 * The matrix is the Laplacian Q = L = D - A, as for Max-K-Cut (Sec. 5), so
 *     z^H L z = sum over edges {i, j} of w_ij |z_i - z_j|^2,
 * and the cut weight is the sum of w_ij over edges whose ends carry
 * different labels (for K = 3, z^H L z = 3 cut).  The CSR layout, the
 * range of every index and every label of z (< K) are checked on the device
 * before use; a violation returns LRQO_EINVAL.  n <= 2^31 - 1.
 * ------------------------------------------------------------------------ */

typedef struct lrqo_graph {
    const int64_t* row_ptr;  /* device [n + 1] */
    const int32_t* col;      /* device [nnz] (may be NULL when nnz = 0) */
    const double* w;         /* device [nnz] or NULL (unit weights) */
    int64_t n;
    int64_t nnz;
} lrqo_graph;

/* z^H L z and the cut weight of labels z (device uint8 [n], labels < K,
 * 2 <= K <= 255), as FP64 host values; sums are taken in a fixed order. */
lrqo_status lrqo_graph_objective(const lrqo_graph* g, int32_t K, const uint8_t* z, double* quad,
                                 double* cut);

/* Greedy local search on z^H L z from the labels in z (device uint8 [n],
 * updated in place), 2 <= K <= 16.  One round: every vertex finds its best
 * other label b (gain 2 sum_k c_k (cos(2 pi (a-k)/K) - cos(2 pi (b-k)/K)),
 * c_k the weight of its neighbours with label k; ties to the lowest b), is a
 * candidate when the gain exceeds 1e-12 of its weighted degree, and moves
 * when its (gain, -index) beats that of every neighbouring candidate.  Moving
 * vertices are pairwise non-adjacent, so each round raises z^H L z by the sum
 * of their gains; rounds repeat until none moves (a single-vertex local
 * optimum) or max_rounds have moved. */
typedef struct lrqo_refine_options {
    int32_t max_rounds;      /* rounds that move at least one vertex; 0: 1,000,000 */
    int32_t check_every;     /* rounds launched between host checks, 1..64; 0: 8 */
} lrqo_refine_options;

typedef struct lrqo_refine_result {
    double quad_before;      /* z^H L z of the input labels */
    double quad_after;       /* z^H L z of the returned labels */
    double cut_before;
    double cut_after;
    int64_t moves;           /* vertex moves over all rounds */
    int32_t rounds;          /* rounds that moved at least one vertex */
    int32_t converged;       /* 1: no vertex has a positive gain */
    float device_ms;         /* device time of the launched rounds */
    int32_t launched;        /* rounds launched (the last check interval may run past convergence) */
} lrqo_refine_result;

lrqo_status lrqo_refine_greedy(const lrqo_graph* g, int32_t K, uint8_t* z,
                               const lrqo_refine_options* opt, lrqo_refine_result* res);

/* --------------------------------------------------------------------------
 * Spectral truncation (the step before the solvers): the r largest
 * eigenpairs of a Hermitian matrix by Lanczos with full reorthogonalisation
 * (FP64), returned as the factor V = U diag(sqrt(max(lambda, 0))) that the
 * solvers take (device complex128 n x r, row-major interleaved; for the
 * Laplacian the imaginary parts are zero to rounding).  Eigenvalues in
 * descending order; each eigenvector is rotated so that its largest-modulus
 * entry (lowest index among equals) is real and positive.  Convergence: the
 * residual bound |beta_m s_{m,k}| of every pair is at most tol times the
 * largest Ritz value, checked every check_every steps; an invariant Krylov
 * space ends the iteration early (exact pairs).
 * ------------------------------------------------------------------------ */

typedef struct lrqo_eigs_options {
    int32_t max_iter;        /* Lanczos steps, at most min(n, 2000); 0: 300 */
    int32_t check_every;     /* steps between convergence checks; 0: 10 for the
                                Laplacian, 1 for the phase-sync operator */
    double tol;              /* 0: 1e-10 */
    uint64_t seed;           /* start vector: complex Gaussian entries from Philox4x32-10,
                                counter (i lo, i hi, 0x5354524C, 0) */
} lrqo_eigs_options;

typedef struct lrqo_eigs_result {
    double eigenvalues[LRQO_MAX_R];
    double residuals[LRQO_MAX_R];
    int32_t iterations;      /* Lanczos steps taken */
    int32_t converged;
    float device_ms;
    int32_t pad;
} lrqo_eigs_result;

/* Top-r factor of the Laplacian L = D - A of a graph (layout as for
 * lrqo_graph_objective, checked on the device), 1 <= r <= 8. */
lrqo_status lrqo_laplacian_factor(const lrqo_graph* g, int32_t r, const lrqo_eigs_options* opt, double* V,
                                  lrqo_eigs_result* res);

/* Top-r factor of Q = U U^H + sigma W (phase synchronisation), applied
 * matrix-free: U device complex128 n x p (row-major interleaved, 0 <= p <= 8)
 * and W the Hermitian Gaussian matrix defined by w_seed: for i <= j,
 * Philox4x32-10 with key (w_seed lo, w_seed hi) and counter
 * (i, j >> 1, 0x57484D41, 0) gives words (w0, w1, w2, w3); column j takes
 * (w0, w1) for even j and (w2, w3) for odd j, as u = ((w >> 9) + 1/2) 2^-23;
 * W_ij = sqrt(-log u0) e^{2 pi i u1} (i < j), W_ii = sqrt(-2 log u0)
 * cos(2 pi u1), W_ji = conj(W_ij) (evaluated in FP32 with the hardware
 * log2, sqrt, sin and cos, accumulated in FP64).  Each product costs n^2/2
 * entry evaluations; check_every = 0 checks convergence after every step. */
lrqo_status lrqo_phase_sync_factor(const double* U, int64_t n, int32_t p, double sigma, uint64_t w_seed, int32_t r,
                                   const lrqo_eigs_options* opt, double* V, lrqo_eigs_result* res);

#ifdef __cplusplus
}
#endif

#endif /* LRQO_H */
