/*
 * ph.h -- C ABI of the MI355X adaptive-FMM photoionization library (libph.so).
 *
 * The library evaluates the discrete Zheleznyak photoionization integral of
 * Lin & Zhuang, "Adaptive Strategies to Fast Multipole Method in
 * Photoionization Calculations" (arXiv 2112.10059):
 *
 *   S_ph(x_i) = P * sum_{j in S, j != i} w_j I_j K(|x_i - x_j|) + P [i in S] c_self I_i,   i in T
 *
 * with K(r) = g(r) / (4 pi r^2) and g of Sec. 2.1 eq. (3),
 * P = p_q/(p+p_q) * xi*omega/alpha (eq. (2)), the quadrature form of
 * Sec. 2.4 eq. (15), and the adaptive source set S (Sec. 3 eq. (18),
 * Sec. 4.3 eq. (22)) and target set T (Sec. 3 strategy 2; field rule of
 * Sec. 5).  The far field is approximated by a fast multipole method with
 * artificial sources fitted at check points (Sec. 2.4 eq. (17) and the
 * figure of artificial/check points), the near field of Sec. 2.4 eq. (16)
 * is summed exactly.
 *
 * Conventions shared by every entry point:
 *  - Every function returns ph_status; nothing throws across the ABI.
 *    A failed call leaves outputs unspecified and sets a thread-local detail
 *    string readable with ph_last_error().
 *  - "device" pointers are HIP device allocations on the GPU that was current
 *    when the plan was created; "host" pointers are ordinary CPU memory.
 *  - The caller owns every buffer it passes in; the plan owns its internal
 *    device buffers (sorted points, tree, operators) and frees them in
 *    ph_plan_destroy.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is enqueued on it; the call returns without
 *    waiting unless stated otherwise.
 *  - A plan owns one per-call workspace: ph_evaluate calls on it must not overlap on the
 *    device (keep them on one stream, or order their streams).  Calls that bring their own
 *    workspace (ph_evaluate_ws) may overlap each other and the plan's own calls.  Host
 *    calls on one plan from several threads are serialised by a lock in the plan.
 */
#ifndef PH_H_
#define PH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ph_plan ph_plan; /* opaque */

typedef enum {
    PH_OK = 0,
    PH_EINVAL = 1,        /* an argument failed host-side validation (no device work was done) */
    PH_ENOMEM = 2,        /* device or host allocation failed, or the workspace cap was hit   */
    PH_EDEVICE = 3,       /* a HIP runtime call failed                                        */
    PH_ENUMERIC = 4,      /* a non-finite or negative source value was seen on the device     */
    PH_EUNSUPPORTED = 5,  /* a valid request the library does not implement                   */
    PH_EFALLBACK = 6      /* informational: the learned selector fell back to the threshold rule;
                             the output is valid                                              */
} ph_status;

typedef enum {
    PH_FP64 = 0,            /* every step in FP64                                              */
    PH_FP32 = 1,            /* FP32 kernels, Kahan-compensated near field, FP64 final combine  */
    PH_FP32_BF16SPLIT = 2   /* as PH_FP32 with M2L on split BF16 (hi/lo) operands              */
} ph_precision;

typedef enum {
    PH_SEL_THRESHOLD = 0,   /* the source rule I >= src_rel * max I (Sec. 3 eq. (18))          */
    PH_SEL_LEARNED = 1      /* learned per-leaf keep/drop on top of the threshold rule          */
} ph_selector;

typedef enum {
    PH_METHOD_FMM = 0,      /* adaptive fast multipole evaluation                               */
    PH_METHOD_DIRECT = 1    /* all-pairs direct sum over the selected sets (O(|S| |T|))         */
} ph_method;

/* Quadrature points (Sec. 2.4 eq. (15)).  Host pointers, read only during ph_plan_create. */
typedef struct {
    int64_t n;              /* number of points, >= 1                                          */
    const double *xyz;      /* n x 3, cm, array of structures, caller order                    */
    const double *w;        /* n quadrature volumes (cm^3); NULL => uniform grid, w = h^3      */
    double h;               /* grid spacing (cm) for a uniform cell-centred grid, else 0       */
    double self_coeff;      /* own-cell coefficient c_self; NaN => integral of K over the cube
                               of side h (requires h > 0); 0 for point clouds                  */
    double cube_lo[3];      /* lower corner of the octree root cube (cm)                        */
    double cube_size;       /* edge of the root cube (cm); <= 0 => bounding cube of the points */
} ph_points;

/* Gas (Sec. 2.1 eqs. (2)-(3)).  pO2 = o2_fraction * p_torr. */
typedef struct {
    double p_torr;          /* gas pressure p (Torr), > 0                                       */
    double o2_fraction;     /* pO2 / p, in (0, 1]                                              */
    double pq_torr;         /* quenching pressure p_q (Torr), >= 0                             */
    double xi_omega_over_alpha; /* xi * omega / alpha, >= 0                                    */
    double chi_min;         /* cm^-1 Torr^-1, 0 < chi_min < chi_max                            */
    double chi_max;
} ph_gas;

/* Adaptive selection (Sec. 3; Sec. 4.3 eq. (22); Sec. 5 field rule). */
typedef struct {
    double src_rel;         /* keep source j iff I_j >= src_rel * max_k I_k; 0 => every point  */
    double e_abs;           /* keep target i iff |E_i| >= e_abs (V/m); < 0 => rule off         */
    double e_applied;       /* keep target i iff |E_i| >= e_applied + e_rel (max|E| - e_applied) */
    double e_rel;           /*   ... < 0 => rule off.  Both rules off => every point a target   */
    double r_s;             /* third strategy of Sec. 3 (r_s skip), 0 = off: at a target of leaf B
                               the sources of B's W list (near boxes not adjacent to B, Fig. of
                               the near-field cross section) are left out when
                               sum_A Q_A K(d_min(A, B)) < r_s * (the rest of S at the target),
                               Q_A the weighted strength of box A; that changes S by at most
                               r_s relative.  The paper's streamer runs use 1e-4 (Sec. 5)     */
} ph_thresholds;

typedef struct {
    ph_precision precision;
    ph_selector selector;
    ph_method method;
    int order_q;            /* lattice points per box edge (2..8); 0 => FP64: 6 on uniform grids,
                               7 on point clouds; other precisions: 4                      */
    int leaf_capacity;      /* split a box while max(#sources, #targets) > this; 0 => 64         */
    int max_depth;          /* 0 => depth of the tree over all points (bounded by 16)           */
    double pinv_rel_cutoff; /* singular values below cutoff * sigma_max are dropped; 0 => 1e-15 for
                               FP64, 1e-7 for FP32 on uniform grids, 1e-4 for FP32 on clouds */
    const float *selector_weights; /* host, PH_MLP_NPARAM floats (learned selector) or NULL     */
    float selector_logit_threshold;/* keep a source leaf iff its logit >= threshold           */
    double selector_fallback_rel;  /* source rule I >= rel * max I used when the learned
                                      selector falls back; 0 => 1e-4                         */
    size_t workspace_cap_bytes;    /* 0 => unlimited                                           */
    int validate;           /* learned selector only: 1 => every call also runs the plain FMM under
                               the threshold rule (selector_fallback_rel) and keeps the learned
                               result only if ||S_learned - S_threshold||_2 <= tol ||S_threshold||_2,
                               else returns the threshold result and reports the fallback        */
    double tol;             /* that tolerance; 0 with validate = 1 keeps only identical results;
                               default (0, validate = 0) 1e-3                                   */
} ph_options;

#define PH_NPHASES 12
typedef struct {
    int64_t n_src;          /* selected sources                                                 */
    int64_t n_tgt;          /* selected targets                                                 */
    int64_t n_boxes;        /* boxes of the per-call tree                                       */
    int64_t n_leaves;       /* source leaves the learned selector decided on (learned plans)    */
    int32_t levels;         /* deepest level + 1                                                */
    int32_t fell_back;      /* 1 if the learned selector fell back                              */
    int64_t n_src_dropped;  /* sources removed by the learned selector                          */
    double t_ms[PH_NPHASES];/* per-phase device time (hipEvent), filled only when requested     */
    int64_t work[12];       /* algorithmic work: [0] near pairs (P2P), [1] local-to-target kernel
                               evaluations, [2] W-list evaluations, [3] P2M kernel evaluations,
                               [4] X-list evaluations, [5] M2L box pairs, [6] M2M child
                               translations, [7] L2L translations, [8] grid local-to-target
                               multiply-adds, [9] grid P2M multiply-adds, [10] targets of leaves
                               with a non-empty U list (those the near-field kernel visits),
                               [11] those of the near pairs ([0]) whose kernel value is read from
                               the uniform-grid table of cell offsets                           */
    double check_rel_l2;    /* validated learned calls: ||S_learned - S_threshold|| / ||S_threshold||
                               as measured on the device; -1 otherwise                           */
} ph_stats;

/* Returns a static description of a status code. */
const char *ph_status_string(ph_status s);

/* Detail of the last failure on the calling thread ("" if none). */
const char *ph_last_error(void);

/* Fills *opt with the defaults described above (FP32, threshold selector, FMM). */
void ph_options_default(ph_options *opt);

/*
 * Builds a plan over a fixed point set for the discretised integral of Sec. 2.4 (eq. (15):
 * weights w_j, the own-cell term on grids) and its fast multipole evaluation (eqs. (16)-(17):
 * an octree whose near and far parts are summed directly and through equivalent densities):
 * validates every argument on the host (no device call happens before validation passes),
 * copies the points to the device, computes 63-bit Morton keys and radix-sorts them, builds
 * the octree over all points, and precomputes the per-level FMM operators of the gas
 * (Sec. 2.1, eq. (3)) in FP64 on the host.
 * Errors: PH_EINVAL (bad argument), PH_ENOMEM, PH_EDEVICE, PH_EUNSUPPORTED.
 * Synchronous.  *out is set only on success.
 */
ph_status ph_plan_create(const ph_points *pts, const ph_gas *gas, const ph_thresholds *thr,
                         const ph_options *opt, ph_plan **out);

/* Releases the plan and its device memory; NULL is allowed.  Synchronises the device. */
void ph_plan_destroy(ph_plan *plan);

/*
 * One evaluation of S_ph (Sec. 2.4 eqs. (15)-(17) with the adaptive sets of Sec. 3).
 *   I     device, n values in caller order: double for PH_FP64, float otherwise.
 *         Must be finite and >= 0 (else PH_ENUMERIC is reported, see below).
 *   absE  device, n floats |E| (V/m); may be NULL only if both field rules are off.
 *   S_out device, n values, same type as I: S_ph at selected targets, 0 elsewhere.
 *   stats host, nullable.  When non-NULL the call waits for the stream, fills
 *         the counts and per-phase times, and reports this call's faults:
 *         PH_ENUMERIC if the device saw a bad source value, PH_ENOMEM if an
 *         interaction list overflowed its capacity (the lists are then cut, reads
 *         stay in bounds, S_out is not valid).  When NULL the call is fully
 *         asynchronous; its faults are reported by the next ph_plan_check().
 * The interaction lists and the near field run on a second stream, and the V/X
 * target lists with the deepest level's M2L products on a third (both library-owned,
 * shared by the plans of the device), both
 * forked from `stream` after the octree and joined back into it (the third before
 * the other levels' M2L products, the second, lists and near field, before the
 * gathers; events, no host synchronisation): the call stays ordered on `stream`.  Calls on one plan's own workspace must not overlap.
 */
ph_status ph_evaluate(ph_plan *plan, const void *I, const float *absE, void *S_out,
                      void *stream, ph_stats *stats);

/*
 * Another evaluation on the sets of the previous ph_evaluate on this plan (Sec. 5 evaluates S_ph
 * twice per time step, on fields that change little between the two): the source and target
 * sets, the learned decisions, the octree and every interaction list are those that call built
 * on the plan's own workspace; only the source strengths are new.  It runs the compaction of
 * the new I on the old flags (which also clears S_out at the points that are not targets and
 * checks the selected sources' values), the upward and downward passes, the near field and
 * the far field; the maxima pass, the selection pass, the tree and the list builds are left
 * out, and so are the FP32 scale (2^-e from the previous call's maximum) and, on learned plans,
 * the validation.  I and S_out as for ph_evaluate (absE is not read).  Errors as ph_evaluate,
 * plus PH_EINVAL when no ph_evaluate has completed its launches on the plan since it was
 * created or its target set was changed, PH_EUNSUPPORTED for the direct method.  Results equal
 * a plan whose selection gave those sets: for an I whose sets and maximum are those of the
 * previous call, bit for bit equal to ph_evaluate.
 */
ph_status ph_evaluate_same_sets(ph_plan *plan, const void *I, void *S_out, void *stream, ph_stats *stats);

/*
 * Size in bytes of the per-call workspace of ph_evaluate_ws (0 for NULL).  Every per-call
 * array of the hot path lives in it: selection flags and compacted records, the per-call
 * tree and interaction lists, equivalent densities and check values, translation products,
 * the near field, the learned selector's rows, and the threshold-rule field of a validated
 * call.
 */
size_t ph_evaluate_workspace_bytes(const ph_plan *plan);

/*
 * ph_evaluate with a caller-owned workspace (device, ph_evaluate_workspace_bytes bytes,
 * 256-byte aligned; torch allocations are).  The workspace must be all zero before its first
 * call with this plan and must not be written by the caller between calls: it carries the
 * call number and the box tags that let the lists skip clearing.  It may be reused across
 * calls of the same plan only.  Calls with distinct workspaces may run concurrently on
 * different streams (their device work overlaps, except the list building and near field,
 * which share the second and third streams and run one call after the other; those two
 * streams belong to all plans of a device, so that several plans never hold more streams than
 * the device has hardware queues).
 * Results are bit-identical to ph_evaluate.  Errors as ph_evaluate, plus PH_EINVAL for a
 * null or misaligned workspace.
 */
ph_status ph_evaluate_ws(ph_plan *plan, const void *I, const float *absE, void *S_out, void *workspace,
                         void *stream, ph_stats *stats);

/*
 * Demand-oriented target set (Sec. 3, second strategy: only the points where S_ph is needed,
 * e.g. a cross-section or a line of interest, Sec. 4.1).  mask: host, n bytes in caller order,
 * nonzero = the point may be a target; every later call evaluates S only there (intersected
 * with the field rules of the thresholds, if on) and writes 0 elsewhere.  NULL restores "every
 * point".  n must equal the plan's point count.  Waits for the device; must not run while a
 * call on the plan is still executing on another thread's stream.
 */
ph_status ph_plan_set_targets(ph_plan *plan, const uint8_t *mask, int64_t n);

/*
 * Moves the plan to another gas (Sec. 2.1, eq. (3); the pressure study of Sec. 4.2): the
 * constants a = chi_min p_O2, b = chi_max p_O2 and P, the own-cell coefficient (unless the
 * plan was created with a fixed self_coeff) and every operator are rebuilt; the point order,
 * the octree and the per-call buffers are kept.  The kernel depends on the pressure only
 * through a r and b r, so the far-field operators of a box of half-width hw depend on a hw
 * and b hw alone, up to powers of hw: the plan keeps every level it has built, and a level
 * whose a hw and b hw it has seen before (for instance after halving or doubling the
 * pressure, when level l takes the operators of level l +- 1) is rescaled from the cache
 * instead of being built, bit for bit equal to a fresh build.  *levels_reused (nullable)
 * receives how many levels came from the cache.  Results of later calls equal those of a
 * plan created with this gas, bit for bit.  Waits for the device; must not run while a call
 * on the plan is still executing.  Errors: PH_EINVAL (bad gas), PH_EDEVICE.
 */
ph_status ph_plan_set_gas(ph_plan *plan, const ph_gas *gas, int *levels_reused);

/*
 * Graph replay of ph_evaluate: not available in this library.  enable = 0 returns
 * PH_OK (calls launch eagerly, as always); enable != 0 returns PH_EUNSUPPORTED.
 */
ph_status ph_plan_set_graph(ph_plan *plan, int enable);

/*
 * Per-phase device time.  ms_sum (host, PH_NPHASES doubles, nullable) receives the
 * summed hipEvent time of every call recorded since the previous query, per phase:
 *   0 maxima of I and |E|
 *   1 selection flags, one pass over the points (with the learned selector, the list
 *     of its rows too)
 *   2 the learned selector's decisions (learned plans) and the compaction of the
 *     selected points                     3 octree        4 interaction lists
 *   5 upward pass (P2M, M2M)   6 downward pass (M2L, L2L, P2L; waits for the lists)
 *   7 far field at the targets (L2P, M2P, own cell) and the output (waits for 8)
 *   8 near field (P2P), or the whole direct sum
 *   9 the M2L product launches alone (the deepest level's on the third stream plus the
 *     others' on the caller's; their events bracket just those launches)
 * Phases 4 and 8 run on the plan's second stream beside phases 5-7, so their
 * times overlap those; the V/X target lists and the deepest level's M2L products
 * run on a third stream (not timed apart: their time shows in phases 5 and 6).
 * *n_calls (nullable) the number of calls.  The sums are then reset.  record = 1
 * turns recording on for every later ph_evaluate (events on the caller's stream,
 * no extra synchronisation), 0 turns it off, -1 leaves it unchanged.  Synchronous.
 */
ph_status ph_phase_times(ph_plan *plan, int record, double *ms_sum, int64_t *n_calls);

/*
 * Waits for the stream and reports the faults of every ph_evaluate call on this plan since
 * the previous ph_plan_check (whether or not a call with stats already reported them):
 * PH_ENOMEM if an interaction list overflowed, else PH_ENUMERIC if a bad source value was
 * seen, else PH_OK.  The record is cleared, so a second check right after returns PH_OK.
 */
ph_status ph_plan_check(ph_plan *plan, void *stream);

/* Number of points of the plan, or -1 for NULL. */
int64_t ph_plan_size(const ph_plan *plan);

/*
 * Test/inspection access to plan-internal device arrays after the last
 * ph_evaluate (or after ph_plan_create for the plan-time arrays).  Copies at
 * most cap_bytes into the host buffer dst and stores the array length (in
 * elements; in rows for the two-dimensional arrays 4 and 8) in *n_out.
 * Synchronous.  what:
 *   0 sorted Morton keys (uint64, n)      1 permutation sorted->caller (int32, n)
 *   2 selected sources, sorted positions (int32, n_src)
 *   3 selected targets, sorted positions (int32, n_tgt)
 *   4 box table (int32, n_boxes x PH_BOX_FIELDS, fields below)
 *   5 level offsets (int32, levels + 1)   6 own-cell coefficient (double, 1)
 *   7 scale exponent e of the FP32 forms (int32, 1)
 *   8 learned-selector row features (float, rows x 8)
 *   9 learned-selector row boxes: plan-tree box ids (int32, rows)
 *  10 third strategy (r_s > 0): per sorted point, 1 where the W list of its leaf was left
 *     out (uint8, n; defined at the targets of leaves with a W list)
 */
#define PH_BOX_FIELDS 10  /* level, ax, ay, az, src_first, src_count, tgt_first, tgt_count, parent, flags */
ph_status ph_debug_fetch(ph_plan *plan, int what, void *dst, int64_t cap_bytes, int64_t *n_out);

/*
 * Learned leaf selector network: 8 inputs -> 64 -> 64 -> 1 logit, exact-erf
 * GELU after each hidden layer.  Parameter vector layout (PH_MLP_NPARAM floats):
 *   W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3[1]   (row-major, out x in)
 * These calls carry the training loop; buffers are device, caller-owned, FP32.
 */
#define PH_MLP_NIN 8
#define PH_MLP_NHID 64
#define PH_MLP_NPARAM (64 * 8 + 64 + 64 * 64 + 64 + 64 + 1)

/* logits[m] = net(X[m][8]); bf16 != 0 rounds weights and activations to BF16 (FP32 accumulate). */
ph_status ph_mlp_forward(const float *params, const float *X, int64_t m, float *logits, int bf16,
                         void *stream);

/*
 * Mean binary cross-entropy with logits over m rows, positive rows weighted by
 * pos_weight, and its gradient: grad[PH_MLP_NPARAM] (overwritten) and loss[1].
 */
ph_status ph_mlp_backward(const float *params, const float *X, const float *y, float pos_weight,
                          int64_t m, float *grad, float *loss, void *stream);

/*
 * ph_mlp_backward for callers that cannot allocate device memory (code under stream capture,
 * tight training loops, hosts that forbid allocation): the same result bit for bit, with the
 * per-block gradient partials in a fixed array inside the library (4.9 MB per GPU, kept until
 * the process ends) instead of memory allocated at the call.  It makes no allocation of any
 * kind.  m must be in 1..PH_MLP_NOALLOC_MAX_ROWS (else PH_EINVAL, nothing launched).  Every
 * call on one GPU shares that array, so calls that overlap on one GPU (different streams or
 * host threads) race; calls ordered on one stream do not.
 */
#define PH_MLP_NOALLOC_MAX_ROWS 8192
ph_status ph_mlp_backward_noalloc(const float *params, const float *X, const float *y, float pos_weight,
                                  int64_t m, float *grad, float *loss, void *stream);

/* One Adam step (bias-corrected, step >= 1) on nparam values in place. */
ph_status ph_adam_step(float *params, float *m1, float *m2, const float *grad, int64_t nparam,
                       float lr, float beta1, float beta2, float eps, int64_t step, void *stream);

/*
 * Learned selector rows (adaptive source selection of Sec. 3, decided per leaf by the
 * network; not in the paper): the leaves of the plan's tree over all points that hold at
 * least one candidate source, I >= thresholds.src_rel * I_max, in box order.  Eight
 * features per row b (E_max = max |E|, I_max = max I over all points, w_ref = h^3 on grids
 * else cube volume / n; sums and maxima of I over b's candidates):
 *   0 log10(max_b I / I_max)              1 log10(sum_b w I / (I_max w_ref))
 *   2 log2(side_b / w_ref^(1/3))          3 log10(1 + |centre_b - x_Emax| / side_b)
 *   4 max |E| / E_max over b's points     5 mean |E| / E_max    6 std |E| / E_max
 *   7 max |E| / E_max over the 27 boxes around b (features 3-7 are 0 without |E|)
 * x_Emax is the point of largest |E| (first in caller order among ties).  A learned plan
 * keeps row b iff the network's BF16 logit is >= selector_logit_threshold.
 * I (device, plan precision) and absE (device, nullable) are a call's inputs; this call
 * resets the plan's per-call scalars (run ph_evaluate again before fetching its results).
 * feats: device, cap_leaves x 8 floats (nullable); *n_leaves receives the row count, rows
 * beyond cap_leaves are not written.  Synchronous.
 */
ph_status ph_selector_features(ph_plan *plan, const void *I, const float *absE, float *feats,
                               int64_t cap_leaves, int64_t *n_leaves, void *stream);

/*
 * Training labels: for the first n_rows rows of the last ph_selector_features call (same
 * I), the field of each row's candidate sources at the given targets, in the units of
 * S_out (Sec. 2.4 eq. (15) restricted to those sources, own-cell term included, times P):
 *   out[r * ld + t] = P sum_{j in row r} G(x_{targets[t]}, y_j) I_j.
 * Every such field is non-negative, so the Gram matrix of the rows bounds exactly how
 * much S changes when a set of rows is dropped.  targets: device, n_targets caller-order
 * indices; out: device, n_rows x ld floats, ld >= n_targets.  Kernel values in the plan's
 * precision, sums in FP64.  PH_EINVAL if n_rows exceeds the row count.  Synchronous.
 */
ph_status ph_selector_fields(ph_plan *plan, const void *I, const int32_t *targets, int64_t n_targets,
                             float *out, int64_t ld, int64_t n_rows, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PH_H_ */
