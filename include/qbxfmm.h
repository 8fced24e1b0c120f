/*
 * qbxfmm: FMM-accelerated Global QBX for 2D Helmholtz single- and
 * double-layer potentials on MI355X (gfx950).
 *
 * Method: Rachh, Kloeckner, O'Neil, "Fast algorithms for Quadrature by
 * Expansion I: Globally valid expansions".  For a curve discretised by
 * Gauss-Legendre panels (Sec. 2.2) with one QBX centre per node, the library
 * evaluates
 *
 *     u(t) = S[sigma_s](t) + D[sigma_d](t),
 *     S[s](t) = sum_j (i/4) w_j H0(omega |t - s_j|) s_j        (Sec. 1, 3.2)
 *     D[s](t) = sum_j (i/4) w_j d/dn_j H0(omega |t - s_j|) s_j
 *
 * with QBX (Sec. 2.1, eqs. (jexp), (graf-coefficient), (phiapprox)) at every
 * target associated with a centre and the plain Gauss rule elsewhere
 * (Sec. 3.2, eq. (gauss-layerpot)).  QBX coefficients are formed either
 * directly over all sources, or by the FMM of Sec. 7.2 (Stages 1-8 with the
 * QBX additions P2QBXL, M2QBXL and L2QBXL).  Centres lie on the exterior
 * side, so on-curve targets receive the exterior one-sided limits (Sec. 2,
 * eq. (oneside)); no jump term is added.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - All functions are extern "C", never throw, and return a qbx_status.  On
 *   failure qbx_last_error() returns a message for the calling thread, and
 *   qbx_ctx_last_error(ctx) the message of the last failed call on a context.
 * - Evaluations (qbx_eval, qbx_eval_noalloc, qbx_eval_batch,
 *   qbx_geom_autotune), qbx_krylov_dot and qbx_ctx_set_stream use the
 *   context's streams, events and buffers, so one thread at a time may be
 *   inside one of them: such a call made while another thread is inside one
 *   on the same context returns QBX_E_BUSY and does nothing.  Geometry
 *   creation and destruction, area queries and the other calls may run from
 *   other threads alongside (a server builds geometries on worker threads
 *   while it evaluates others).
 * - Geometry arrays (qbx_plan_create, qbx_geom_create) are HOST pointers to
 *   float64 arrays; the library copies what it needs.  The caller keeps
 *   ownership.
 * - Density, potential and coefficient arrays of the evaluation calls are
 *   complex128 data, i.e. interleaved (re, im) float64.  Where each lives is
 *   found with hipPointerGetAttributes.  Device memory of the context's
 *   device (or managed memory) is read and written in place, asynchronously
 *   on the context's stream; the caller synchronises that stream before
 *   reading the results on the host.  qbx_eval also takes host memory
 *   (pageable or pinned): it copies those arrays through buffers of its own
 *   and returns once the results are back in host memory.  The other
 *   evaluation calls refuse host memory with QBX_E_INVAL.
 * - Indices are 0-based; counts are int64_t.
 */
#ifndef QBXFMM_H
#define QBXFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QBX_ABI_VERSION 3

typedef enum {
    QBX_OK = 0,
    QBX_E_INVAL = -1,        /* invalid argument (size, non-finite value, range) */
    QBX_E_NOMEM = -2,        /* host or device allocation failed */
    QBX_E_DEVICE = -3,       /* a HIP call failed (no device, launch error) */
    QBX_E_ASSOC = -4,        /* a target in Gamma_near has no eligible centre (Sec. 6.1) */
    QBX_E_UNSUPPORTED = -5,  /* valid request outside what the library implements */
    QBX_E_BUSY = -6          /* the context is inside a call made by another thread */
} qbx_status;

typedef struct qbx_ctx_s *qbx_ctx;    /* device + stream */
typedef struct qbx_plan_s *qbx_plan;  /* host-side tree, lists, orders, association */
typedef struct qbx_geom_s *qbx_geom;  /* device-resident plan + translation tables */

typedef struct {
    int32_t p;            /* QBX expansion order (Sec. 2.1, eq. (phiapprox)); 0..40 */
    int32_t p_add;        /* FMM order increment (Sec. 7.1, Table p_add); -1 = default rule */
    int32_t leaf_max;     /* n_max: split a box holding more sources + centres (Stage 1) */
    int32_t direct;       /* 1 = form QBX coefficients directly over all sources (no FMM) */
    int32_t far_fp32;     /* 1 = M2L and L2L on FP32 matrix cores with complex-float
                             tables (the scaled entries are bounded by one); allowed
                             only when eps >= 1e-6.  Everything else stays FP64. */
    int32_t w_direct;     /* W-list boxes (Stage 5) whose sources enter the centre's
                             coefficients directly, as in P2QBXL, instead of through
                             M2QBXL: -1 = when cheaper by operation count (default),
                             0 = never (every W box through M2QBXL, as in Stage 5),
                             n > 0 = boxes holding at most n sources.  Direct sums
                             are exact, so the choice only removes truncation. */
    int32_t level_restrict; /* 1 (default) = refine the adaptive tree until leaves
                             that touch differ by at most one level (2:1 balance, the
                             level-restricted trees of the paper's experiments, Sec. 8);
                             0 = the plain adaptive tree of Stage 1 */
    int32_t keep_x_rows;  /* 1 (default) = keep the X-list P2L basis rows (Stage 6; one
                             row of 2 P_b + 3 values per source of each X-list box,
                             geometry only) in device memory from the first evaluation
                             on, when they take at most 1 GiB; 0 = rebuild them inside
                             every evaluation (less memory, a slower X-list stage) */
    double eps_assoc;     /* association slack epsilon_assoc (Sec. 6.1); default 0.05 */
} qbx_options;

typedef struct {
    int64_t n_src, n_ctr, n_tgt;
    int32_t n_levels;     /* levels 0 .. n_levels-1 */
    int32_t n_boxes, n_leaves;
    int32_t p, p_add;
    int64_t n_u_pairs, n_v_pairs, n_w_pairs, n_x_pairs;  /* box-box list entries */
    int64_t n_p2qbxl_pairs;   /* (centre, source) pairs over U lists */
    int64_t n_m2qbxl_pairs;   /* (centre, W-box) pairs */
    int64_t n_x_src_pairs;    /* (box, source) pairs over X lists */
    int64_t n_smooth_targets; /* targets served by the smooth rule */
    double root_radius;       /* |b0| (half the side of the root square) */
    size_t device_bytes;      /* resident device footprint of the geometry */
} qbx_stats;

enum { QBX_LIST_U = 0, QBX_LIST_V = 1, QBX_LIST_W = 2, QBX_LIST_X = 3 };

int32_t qbx_abi_version(void);
const char *qbx_last_error(void);

/* The message of the last call on ctx (or on one of its geometries) that
 * failed, "" if none has; the text stays valid until the calling thread
 * calls this again.  ctx NULL gives "". */
const char *qbx_ctx_last_error(qbx_ctx ctx);
void qbx_options_default(qbx_options *opt);

/* ---- context ------------------------------------------------------------
 * qbx_ctx_create: bind a device and a HIP stream (hipStream_t passed as
 * void*; NULL = the null stream).  Errors: QBX_E_DEVICE if the device cannot
 * be set. */
qbx_status qbx_ctx_create(int32_t device, void *stream, qbx_ctx *out);
qbx_status qbx_ctx_set_stream(qbx_ctx ctx, void *stream);
/* qbx_ctx_destroy releases the caller's handle; the context's streams and
 * events live on until the last geometry made on it is destroyed, so
 * geometries may be destroyed before or after their context. */
qbx_status qbx_ctx_destroy(qbx_ctx ctx);

/* ---- host planning (no GPU needed) ---------------------------------------
 * qbx_plan_create builds, on the host:
 *  - the adaptive quadtree over sources and centres (Sec. 4; Sec. 7.2,
 *    Stage 1): root = smallest origin-centred square holding all sources and
 *    centres (enlarged by a relative 1e-12), split while a box holds more
 *    than leaf_max sources + centres; with level_restrict, leaves touching
 *    a box two or more levels finer are split further (2:1 balance);
 *  - the U, V, W, X lists (Sec. 7.2 definitions);
 *  - FMM orders P_l = p_FMM(l) + p_add, with p_FMM(l) the smallest P such
 *    that |H_n(3 omega R_l) J_n(sqrt(2) omega R_l)| <= eps for all n > P,
 *    R_l the box radius at level l (Sec. 7.1);
 *  - target association (Sec. 6.1): for targets with tgt_ctr[m] == -1 (or
 *    every target when tgt_ctr is NULL) the nearest centre i with
 *    |t - c_i| <= cr_i (1 + eps_assoc), ties to the lowest index; with no
 *    such centre a target within sh_j/4 of a source j fails (QBX_E_ASSOC),
 *    any other is served by the smooth rule.  tgt_ctr[m] >= 0 fixes target
 *    m to that centre (e.g. on-curve nodes and their own centres).
 * Arguments: sources (sx, sy) with full arclength weights w, outward unit
 * normals (nx, ny) and the length sh of the panel each source lies on;
 * centres (cx, cy) with expansion radii cr; targets (tx, ty).  Sources and
 * centres may be different point sets (oversampled sources, Sec. 2.2).
 * Errors: QBX_E_INVAL (n < 0, non-finite input, cr <= 0, w < 0, |n| not 1
 * within 1e-6, omega <= 0, eps outside [1e-15, 1e-2], p outside 0..40,
 * leaf_max < 1, far_fp32 with eps < 1e-6, level_restrict not 0 or 1),
 * QBX_E_ASSOC, QBX_E_NOMEM. */
qbx_status qbx_plan_create(double omega, double eps, const qbx_options *opt,
                           int64_t n_src, const double *sx, const double *sy,
                           const double *w, const double *nx, const double *ny,
                           const double *sh,
                           int64_t n_ctr, const double *cx, const double *cy,
                           const double *cr,
                           int64_t n_tgt, const double *tx, const double *ty,
                           const int32_t *tgt_ctr, qbx_plan *out);
qbx_status qbx_plan_destroy(qbx_plan plan);
qbx_status qbx_plan_stats(qbx_plan plan, qbx_stats *out);
/* Boxes in (level, Morton) order: level, integer index (ix, iy) at that
 * level, parent (-1 for the root), leaf flag, source and centre counts.
 * Each array holds n_boxes entries; any pointer may be NULL. */
qbx_status qbx_plan_boxes(qbx_plan plan, int32_t *level, int32_t *ix, int32_t *iy,
                          int32_t *parent, int32_t *leaf, int32_t *n_src_in,
                          int32_t *n_ctr_in);
/* One list in CSR form: start[n_boxes + 1], idx[start[n_boxes]] (box
 * indices, ascending within a box).  which = QBX_LIST_U/V/W/X.  With idx
 * NULL only start is written. */
qbx_status qbx_plan_list(qbx_plan plan, int32_t which, int32_t *start, int32_t *idx);
/* FMM order P_l per level (n_levels entries). */
qbx_status qbx_plan_orders(qbx_plan plan, int32_t *P);
/* Centre index per target (user numbering) or -1 for the smooth rule. */
qbx_status qbx_plan_association(qbx_plan plan, int32_t *tgt_ctr_out);

/* ---- device geometry -----------------------------------------------------
 * qbx_geom_create = qbx_plan_create + upload to the context's device of the
 * sorted points, tree, lists and translation tables; they stay resident
 * until qbx_geom_destroy.  Same arguments and errors as qbx_plan_create,
 * plus QBX_E_DEVICE / QBX_E_NOMEM for device failures. */
qbx_status qbx_geom_create(qbx_ctx ctx, double omega, double eps, const qbx_options *opt,
                           int64_t n_src, const double *sx, const double *sy,
                           const double *w, const double *nx, const double *ny,
                           const double *sh,
                           int64_t n_ctr, const double *cx, const double *cy,
                           const double *cr,
                           int64_t n_tgt, const double *tx, const double *ty,
                           const int32_t *tgt_ctr, qbx_geom *out);
qbx_status qbx_geom_from_plan(qbx_ctx ctx, qbx_plan plan, qbx_geom *out);
qbx_status qbx_geom_destroy(qbx_geom geom);
qbx_status qbx_geom_stats(qbx_geom geom, qbx_stats *out);
qbx_status qbx_geom_association(qbx_geom geom, int32_t *tgt_ctr_out);
/* qbx_geom_area_query: area queries (Sec. 5: the area query definition,
 * peer boxes and the guiding-box algorithm) on the geometry's tree, on the
 * device.  Query i is the closed square |x - (qx[i], qy[i])|_inf <= qr[i];
 * its result is every leaf box (plan numbering, as qbx_plan_boxes) whose
 * closed square meets it, in the order the query visits them.  A query
 * centre outside the root square is answered from the root (all leaves
 * examined); a negative or NaN radius gives no leaves.  qx, qy, qr: device
 * arrays of n doubles.  start: device int64[n + 1], written with the
 * offsets of each query's leaves (start[n] = total).  leaves: device
 * int32[total], or NULL to count only.  *total_out (host, may be NULL)
 * receives the total.  Runs on the context's stream and synchronises it.
 * Errors: QBX_E_INVAL (n < 0, null arrays), QBX_E_NOMEM, QBX_E_DEVICE. */
qbx_status qbx_geom_area_query(qbx_geom geom, int64_t n, const double *qx, const double *qy,
                               const double *qr, int64_t *start, int32_t *leaves,
                               int64_t *total_out);
/* qbx_geom_points_near: disk tests through area queries (Sec. 5): hit_out[i]
 * = 1 if one of the geometry's sources (which = 0) or centres (which = 1)
 * lies within distance qr[i] of (qx[i], qy[i]), else 0.  The leaves an area
 * query over the disk's bounding square returns are scanned, with the exact
 * test dx^2 + dy^2 <= qr^2.  The geometric refinement conditions of Sec. 5
 * are such tests: Condition 1 (centres as queries, radius h/2, against the
 * panels' points) and Condition 3 (panel points as queries, radius h/4,
 * against the centres).  qx, qy, qr: device arrays of n doubles; hit_out:
 * device int32[n].  A negative or NaN radius gives 0.  Runs on the
 * context's stream and synchronises it.  Errors: QBX_E_INVAL (n < 0, which
 * not 0 or 1, null arrays), QBX_E_NOMEM, QBX_E_DEVICE. */
qbx_status qbx_geom_points_near(qbx_geom geom, int32_t which, int64_t n, const double *qx,
                                const double *qy, const double *qr, int32_t *hit_out);
/* qbx_geom_associate: target association (Sec. 6.1) on the device through
 * area queries, by the rule of qbx_plan_create: the nearest centre i with
 * |t - c_i| <= cr_i (1 + eps_assoc), ties to the lowest index.  As in the
 * paper, each centre is entered in the lists of the leaves its square meets
 * (an area query per centre, with the centre's own eligibility radius), and
 * each source in those its sh/4 square meets; a target then scans the list
 * of the leaf that holds it (quadrants the tree leaves empty count as
 * leaves of their own).  tx, ty: device arrays of n_tgt doubles (any
 * points; targets outside the root square are handled exactly).
 * tgt_ctr_out: device int32[n_tgt], the centre (user numbering) or -1 for
 * the smooth rule.  *n_fail_out (host, may be NULL): targets within sh_j/4
 * of a source j with no eligible centre, where qbx_plan_create fails with
 * QBX_E_ASSOC.  The comparisons round as the host's, so results agree with
 * qbx_plan_association bit for bit.  Runs on the context's stream and
 * synchronises it; temporary device buffers.  Errors: QBX_E_INVAL,
 * QBX_E_NOMEM, QBX_E_DEVICE. */
qbx_status qbx_geom_associate(qbx_geom geom, int64_t n_tgt, const double *tx, const double *ty,
                              int32_t *tgt_ctr_out, int64_t *n_fail_out);
/* qbx_geom_bytes: device memory the geometry holds once it has evaluated
 * n_dens densities: the resident part (points, tree, lists, tables) plus the
 * evaluation scratch (charges, expansions, per-pair rows, radial sequences,
 * coefficients), whether or not the scratch is allocated yet.  The scratch
 * serves chunks of up to 4 densities, so the figure grows with n_dens only
 * by the small GEMM tile lists of the chunk sizes used.  For admission by an
 * HBM budget (a serving loop).  0 for a NULL geometry. */
size_t qbx_geom_bytes(qbx_geom geom, int32_t n_dens);
/* qbx_plan_bytes: the same figure for the geometry qbx_geom_from_plan would
 * make from this plan (its resident part, evaluation scratch and the
 * order-0 geometry of smooth-rule targets), computed on the host without
 * allocating device memory: admission by an HBM budget can decide before
 * anything is allocated.  It runs the host part of the upload (tables
 * included) once.  0 for a NULL plan or on failure. */
size_t qbx_plan_bytes(qbx_plan plan, int32_t n_dens);

/* ---- per-stage timing and work ----------------------------------------------
 * Stages of one evaluation, in launch order (Sec. 7.2 stage names). */
enum {
    QBX_STAGE_CHARGES = 0,  /* qS, qD = (i/4) w sigma, reordered to tree order */
    QBX_STAGE_P2M,          /* Stage 2, leaves */
    QBX_STAGE_M2M,          /* Stage 2, upward pass */
    QBX_STAGE_M2L,          /* Stage 4 */
    QBX_STAGE_P2L_X,        /* Stage 6 */
    QBX_STAGE_L2L,          /* Stage 7 */
    QBX_STAGE_P2QBXL,       /* Stage 3, new */
    QBX_STAGE_M2QBXL,       /* Stage 5, new */
    QBX_STAGE_L2QBXL,       /* Stage 8, new */
    QBX_STAGE_EVAL,         /* QBX evaluation at associated targets */
    QBX_STAGE_SMOOTH,       /* smooth Gauss rule at the other targets */
    QBX_STAGE_DIRECT,       /* direct-mode coefficient sum */
    QBX_STAGE_COEF_OUT,     /* optional coefficient export */
    QBX_N_STAGES
};

/* qbx_geom_profile: enable (1) or disable (0) HIP-event timing of every
 * stage of later qbx_eval calls on this geometry (events are recorded on
 * the context's stream around each stage's launches).  While profiling is
 * on, every stage runs in order on the context's stream (no second stream,
 * no graph), so each stage's time is its own. */
qbx_status qbx_geom_profile(qbx_geom geom, int32_t enable);
/* qbx_eval_batch: evaluate several resident geometries at once (one matvec
 * each), as a serving loop or a multi-geometry solve does.  Geometry i takes
 * n_dens[i] densities sigma_s[i] / sigma_d[i] (arrays of device pointers;
 * either array, or an entry of it, may be NULL as in qbx_eval) and writes
 * u[i]; no coefficient export.  Every FMM stage is one launch over all the
 * geometries (per kernel variant the geometries need): the grid is the
 * concatenation of each geometry's own grid for the stage, and a per-block
 * map names the geometry whose arguments a block takes.  The geometries go
 * through the pipeline together in passes of up to 4 densities each; a
 * geometry listed twice, or with more than 4 densities, takes several
 * passes.  The launches run on the context's stream (and its side stream,
 * forked from and joined back to it).  Each result is bitwise the same as
 * from qbx_eval alone.  The launch records are built on the host and copied
 * to the device once per call; the call waits for the previous call's copy
 * to finish.  The record buffers belong to the context: calls on one
 * context from several threads must not overlap.  If stage profiling or graph replay is on for any geometry, the
 * evaluations run one after another through qbx_eval.  Errors: QBX_E_INVAL
 * (null or foreign geometry, n_dens outside 1..64, missing u or densities),
 * QBX_E_DEVICE, QBX_E_NOMEM. */
qbx_status qbx_eval_batch(qbx_ctx ctx, int32_t n_geom, const qbx_geom *geoms, const int32_t *n_dens,
                          const void *const *sigma_s, const void *const *sigma_d, void *const *u);
/* qbx_geom_autotune: pick the M2L kernel configuration that makes this
 * geometry's evaluation fastest.  The candidates take turns over 9 passes,
 * each a sample of 4 whole evaluations with n_dens zero densities (HIP
 * events on the context's stream; the first pass warms up; temporary device
 * buffers; synchronises the stream), and each keeps its fastest sample.
 * Candidates: columns staged in LDS with w waves per tile, w the row-block
 * count of most V pairs (the default) or about half of it, and the
 * direct-load kernel; another candidate replaces the default only when at
 * least 1% faster.  They compute the same sums in the same order, so results
 * do not change.  *choice_out (may be NULL) receives the waves per tile chosen, 0
 * for the direct kernel.  Overwrites the geometry's scratch (no evaluation
 * may be in flight on it). */
qbx_status qbx_geom_autotune(qbx_geom geom, int32_t n_dens, int32_t *choice_out);
/* qbx_geom_graph: enable (1) or disable (0) graph replay of later qbx_eval
 * calls on this geometry (the "execution modes" of a served matvec loop,
 * where the same evaluation repeats with new density values in the same
 * buffers).  The first call with a given (n_dens, sigma_s, sigma_d, u, coef)
 * captures the whole evaluation into a HIP graph on a stream of the
 * library's own; later calls with the same pointers replay it.  The graph
 * stream waits for the context's stream and the context's stream waits for
 * the graph, so ordering against the caller is unchanged.  Up to 8 argument
 * sets are kept per geometry (least recently used evicted).  Results are
 * identical to the plain path.  QBX_E_UNSUPPORTED if the context could not
 * create its streams. */
qbx_status qbx_geom_graph(qbx_geom geom, int32_t enable);
/* Accumulated milliseconds and launch counts per stage since the last reset
 * (synchronises the stream).  ms and launches hold QBX_N_STAGES entries
 * (either may be NULL); reset != 0 clears the accumulators. */
qbx_status qbx_geom_stage_times(qbx_geom geom, double *ms, int64_t *launches, int32_t reset);
/* Algorithmic floating-point work of one evaluation with n_dens densities,
 * per stage (QBX_N_STAGES entries): the translations count 8 flops per
 * complex multiply-add of the dense operator (M2L: 8 (2P+1)^2 per V pair and
 * density), the near-field kernels the multiply-adds of their coefficient
 * sums (P2QBXL: 24 (2p+1) per source-centre pair and density). */
qbx_status qbx_geom_work(qbx_geom geom, int32_t n_dens, double *flops);

/* ---- evaluation ----------------------------------------------------------
 * u[d][m] = S[sigma_s[d]](t_m) + D[sigma_d[d]](t_m) for d < n_dens, m < n_tgt.
 * sigma_s, sigma_d: device complex128 [n_dens][n_src] (either may be NULL,
 * meaning zero density); u: device complex128 [n_dens][n_tgt]; coef:
 * optional device complex128 [n_dens][2p+1][n_ctr] receiving the QBX
 * coefficients alpha_l (paper's convention, l = -p..p) per centre.
 * Work is enqueued on the context's stream; scratch device memory is owned
 * by the geometry and grows to fit n_dens.  Errors: QBX_E_INVAL (n_dens < 1
 * or > 64, u NULL, both densities NULL), QBX_E_DEVICE, QBX_E_NOMEM. */
qbx_status qbx_eval(qbx_geom geom, int32_t n_dens, const void *sigma_s,
                    const void *sigma_d, void *u, void *coef);

/* ---- GMRES building blocks (the solve of Sec. 8.3 on the device) ------------
 * The Arnoldi step of GMRES on a QBX matvec, run on the context's stream so
 * that the Krylov basis never leaves the device.  V holds Krylov vectors as
 * rows: vector i at V + i * ldv (complex128, device), n entries each.  Sums
 * run in a fixed order (results do not depend on timing).
 * qbx_krylov_dot:       h[i] = sum_j conj(V[i][j]) w[j] for i < k (Gram-Schmidt
 *                       coefficients; k = 1, V = w gives |w|^2 in h[0]).
 *                       h: device complex128[k].  Uses a workspace of the
 *                       context (grown on demand: the call may allocate).
 * qbx_krylov_update:    w[j] -= sum_i h[i] V[i][j], i < k (h device [k]).
 * qbx_krylov_normalize: v[j] = w[j] / sqrt(Re nrm2[0]), nrm2 a device
 *                       complex128 (e.g. from qbx_krylov_dot); 0 if it is 0.
 *                       v may equal w.
 * qbx_upsample:         densities on Gauss panels of q nodes carried to the
 *                       same panels with qs nodes (Sec. 3.2, Table 1):
 *                       yd[p qs + a] = sum_b L[a q + b] x[p q + b] and
 *                       ys = alpha yd (alpha = alpha_re + i alpha_im), for
 *                       the n_panels panels; L: device float64 [qs][q];
 *                       either output may be NULL.
 * Errors: QBX_E_INVAL (sizes, ldv < n, null arrays), QBX_E_NOMEM,
 * QBX_E_DEVICE. */
qbx_status qbx_krylov_dot(qbx_ctx ctx, int64_t n, int32_t k, const void *V, int64_t ldv,
                          const void *w, void *h);
qbx_status qbx_krylov_update(qbx_ctx ctx, int64_t n, int32_t k, const void *V, int64_t ldv,
                             const void *h, void *w);
qbx_status qbx_krylov_normalize(qbx_ctx ctx, int64_t n, const void *w, const void *nrm2, void *v);
qbx_status qbx_upsample(qbx_ctx ctx, int64_t n_panels, int32_t q, int32_t qs, const double *L,
                        double alpha_re, double alpha_im, const void *x, void *ys, void *yd);

/* ---- evaluation without allocation ----------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * qbx_eval_noalloc computes exactly what qbx_eval computes (same kernels,
 * same sums in the same order: results are bitwise equal) but takes every
 * evaluation buffer (charges, expansions, per-pair rows, radial sequences,
 * coefficients) from one static device array of QBX_NOALLOC_SCRATCH_BYTES
 * bytes per device instead of the geometry's own scratch, and calls no
 * hipMalloc, hipFree or allocating routine.  The array is part of the
 * library's device code: each device the library runs on holds it from the
 * first qbx_ctx_create on that device until the process ends.  Densities
 * are taken in chunks of up to 4, as many as fit; a geometry whose buffers
 * for one density exceed the array is rejected with QBX_E_UNSUPPORTED
 * (the message gives the size needed) and must use qbx_eval.  The
 * geometry, its tables and GEMM tile lists must exist (qbx_geom_create);
 * sigma_s, sigma_d, u, coef are as in qbx_eval, on the context's stream.
 * Every call on one device shares that device's array and overwrites what
 * the previous call left there: calls that overlap on one device (other
 * threads, other contexts or streams of the same device, captured graphs
 * replayed concurrently) race and give wrong results; serialise them.
 * Stage profiling and graph replay settings of the geometry are ignored
 * (no events are taken, nothing is captured by the library).  Errors: as
 * qbx_eval, plus QBX_E_UNSUPPORTED. */
#define QBX_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)
qbx_status qbx_eval_noalloc(qbx_geom geom, int32_t n_dens, const void *sigma_s,
                            const void *sigma_d, void *u, void *coef);

#ifdef __cplusplus
}
#endif
#endif
