/*
 * ft.h - stochastic conservative field transfer on MI355X (gfx950).
 *
 * C ABI of the hot path of the control-variate Monte Carlo (CV-MC) Galerkin
 * projection of Paudel, Smith and Merson (arXiv 2603.00538): a field f^s that
 * can only be queried at points is projected onto a P1 target space,
 *
 *     b_i = integral f^s psi_i   (sec. 2, Eq. load_vector),
 *     M x = b                    (sec. 2, Eq. galerkin_system),
 *
 * with b estimated per target element as the exact control part plus a Monte
 * Carlo estimate of the residual (sec. 4.1, Eq. cv_element_load_residual_operator
 * and the seven-step algorithm that closes sec. 4.1).
 *
 * A transfer is four calls, matching the algorithm's steps:
 *
 *   ft_target_create    setup, once per target mesh (mass matrix, incidence)
 *   ft_sample_points    step 1 + 3: the point-query list (nodes, then samples)
 *   -- the caller evaluates f^s at every query point (the black box) --
 *   ft_consume_queries  steps 4-6: residual, per-element MC sums, assembly
 *   ft_project          steps 2 + 7: control load, M x = b, conservation report
 *
 * plus a mesh-backed P1 source with uniform-grid point localization
 * (ft_source_*), standing in for the black box in benchmarks (sec. 5.3).
 *
 * Conventions (all calls):
 *  - Pointers marked "device" are HIP device memory owned by the caller; the
 *    library never retains them after the call returns.  "host" pointers are
 *    ordinary host memory.
 *  - Arrays are structure-of-arrays: coords[c * ld + i] is coordinate c of
 *    point i; values[f * ld + q] is field f at query q.
 *  - Every call enqueues its work on `stream` and returns without waiting,
 *    except ft_target_create, ft_source_create_p1, ft_source_stats and
 *    ft_project, which synchronize `stream` before returning.
 *  - Argument, ordering and mesh errors are returned immediately with no work
 *    enqueued; a failed HIP call returns FT_E_DEVICE.  ft_last_error() gives a
 *    message for the last failure on the calling thread.
 *  - A handle may be used by one host thread at a time.
 */
#ifndef FT_H
#define FT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FT_OK = 0,
    FT_E_ARG = -1,         /* invalid argument: null pointer, size or enum out of range      */
    FT_E_MESH = -2,        /* degenerate element or connectivity out of range                 */
    FT_E_ORDER = -3,       /* call out of order (e.g. project before consume)                 */
    FT_E_DEVICE = -4,      /* a HIP runtime call failed                                       */
    FT_E_NOCONV = -5,      /* CG stopped at max_iter above rtol (x is still written)          */
    FT_E_NONFINITE = -6,   /* NaN/Inf query values were consumed (x is still written)         */
    FT_E_OOM = -7,         /* device allocation failed                                        */
    FT_E_UNSUPPORTED = -8  /* valid but not implemented combination                           */
} ft_status;

typedef enum {
    FT_F64 = 0,            /* points and values in binary64                                   */
    FT_F32 = 1,            /* points and values in binary32 (coordinates converted inside)    */
    FT_SPLIT_F16 = 2,      /* binary32 points and values; element sums of many fields on the
                              matrix cores as hi+lo binary16 products, binary32 accumulation   */
    FT_SPLIT_BF16 = 3      /* as FT_SPLIT_F16 with hi+lo bfloat16 products                    */
} ft_precision;

/* How the samples of an element are drawn (sec. 4.1 step 3; sec. 7 names better
 * sampling schemes as the way forward). */
typedef enum {
    FT_SAMPLING_PLAIN = 0,       /* independent uniform samples                                     */
    FT_SAMPLING_STRATIFIED = 1   /* the d' uniforms of the samples stratified over the unit cube:   */
                                 /* m = floor(N^(1/d')) cells per axis (d' = 2 for triangles, 3 for */
                                 /* tetrahedra); sample j < m^d' takes cell (j mod m, (j/m) mod m,  */
                                 /* j/m^2), its uniforms u -> min((cell + u)/m, 1 - 2^-53), then the  */
                                 /* same maps; samples j >= m^d' stay plain.  Unbiased.              */
} ft_sampling;

/* How the control-variate coefficient is chosen (sec. 4.1, Eq. cv_centered_integrand;
 * sec. 5.1 studies alpha in [0, 1]). */
typedef enum {
    FT_ALPHA_FIXED = 0,          /* cfg.alpha for every element                                     */
    FT_ALPHA_ELEMENT = 1         /* per element, the coefficient minimizing the sample variance of   */
                                 /* the residual terms, estimated from that element's own samples   */
                                 /* (see ft_consume_queries)                                        */
} ft_alpha_mode;

/* Layout of the query values handed to ft_consume_queries (field f at query q). */
typedef enum {
    FT_VALUES_FIELD_MAJOR = 0,   /* values[f * Q + q] (q in the query-list order)                   */
    FT_VALUES_ELEMENT_TILES = 1  /* node v: values[f * n_nodes + v]; sample j of element t:         */
                                 /* values[F * n_nodes + (t * F + f) * N + j], i.e. [F][n_nodes]      */
                                 /* then one F x N tile per element (one field: the same as          */
                                 /* FT_VALUES_FIELD_MAJOR).  Many fields read and write one element's */
                                 /* values as one contiguous block.                                  */
} ft_values_layout;

typedef struct ft_target ft_target;
typedef struct ft_source ft_source;

/* Sampling configuration of one transfer (sec. 4.1 steps 3-5).  Zero-initialized
 * sampling and alpha_mode give plain samples and a fixed alpha. */
typedef struct {
    int32_t  samples_per_elem;  /* N >= 1: samples per target element (the paper uses N = 20)     */
    int32_t  n_fields;          /* F >= 1: fields transferred together, sharing the samples       */
    double   alpha;             /* control-variate coefficient (Eq. cv_centered_integrand); 1.0    */
    uint64_t seed;              /* Philox4x32-10 key                                               */
    uint32_t stream_id;         /* realization id: Philox counter word 2                           */
    int32_t  precision;         /* ft_precision of the query points and values                     */
    int32_t  sampling;          /* ft_sampling                                                     */
    int32_t  alpha_mode;        /* ft_alpha_mode                                                   */
    int32_t  values_layout;     /* ft_values_layout of the values given to ft_consume_queries      */
    int32_t  reserved;          /* 0                                                               */
} ft_sample_cfg;

/* Mass solve configuration (sec. 4.1 step 7). */
typedef struct {
    double  rtol;               /* stop when ||b - M x||_2 <= rtol ||b||_2 (recurrence residual)   */
    int32_t max_iter;           /* Jacobi-PCG iteration cap per field (per refinement step)        */
    int32_t refine_steps;       /* 0: binary64 PCG.  k > 0 (one field): up to k steps of binary64  */
                                /* residual + iterative refinement around a binary32 inner PCG     */
                                /* (binary64 dot products), stopping on the true residual          */
} ft_solve_cfg;

/* Per-field result of ft_project (conservation: sec. 2 Eq. conservation, App. B).
 * sum_b and int_x are compensated sums (each addition's rounding error is
 * carried along, as in Neumaier's summation). */
typedef struct {
    double  sum_b;              /* sum_i b_i                                                       */
    double  int_x;              /* m^T x = integral of the transferred field, m = M 1             */
    double  cons_defect;        /* |int_x - sum_b| / |sum_b|                                       */
    double  rel_resid;          /* true residual ||b - M x||_2 / ||b||_2 after the solve           */
    int32_t iters;              /* CG iterations taken                                             */
    int32_t status;             /* FT_OK, FT_E_NOCONV or FT_E_NONFINITE for this field             */
    int64_t n_nonfinite;        /* non-finite query values seen by the last consume                */
    int64_t n_out_of_domain;    /* query points outside the source mesh (extrapolated), counted by  */
                                /* the built-in source routes (ft_transfer_p1, plans, batches);    */
                                /* -1 after ft_consume_queries: the caller's black box evaluated   */
                                /* the points (ft_source_stats counts ft_source_eval's)            */
    double  sum_b_stderr;       /* estimated standard error of sum_b from the samples themselves    */
                                /* (App. B, Eq. cv_global_integral_estimator: the element totals    */
                                /* |Omega_t|/N sum_j r_tj are independent, so Var(sum b) is the     */
                                /* sum of |Omega_t|^2 s_t^2 / N, s_t^2 the unbiased sample variance */
                                /* of element t's residuals r = y - alpha g; with each element's    */
                                /* own alpha, that alpha).  Its square estimates E[E_cons^2] of     */
                                /* Eq. conservation_residual_bound.  Reported after                 */
                                /* ft_consume_queries (FT_F64, FT_F32), ft_transfer_p1 and plans    */
                                /* with N >= 2; 0 after ft_transfer_supermesh (exact b); -1 where   */
                                /* not estimated (N = 1, the split matrix-core forms, batches)      */
} ft_report;

/* Sizes of a target after setup. */
typedef struct {
    int32_t dim;
    int64_t n_nodes;
    int64_t n_elems;
    int64_t nnz;                /* stored entries of M (CSR)                                        */
    int64_t n_inverted;         /* elements with negative orientation (accepted; |det J| is used) */
    int32_t order;              /* polynomial degree of the target elements: 1 or 2                */
} ft_target_info;

/*
 * ft_target_create - setup of a P1 target mesh (sec. 2: M_ki = int psi_k psi_i,
 * computed exactly; the element measure |Omega_t| = |det J_t| / d! used by
 * sec. 4.1).
 *   dim      2 (triangles), 3 (tetrahedra), or 4 to 6 (d-simplices: sec. 2
 *            states the formulation for any dimension, sec. 7 names 5D/6D
 *            distribution-function transfers).  A d-simplex sample takes
 *            ceil(d/2) Philox blocks (u_(i+1) from block i/2, words (0,1)
 *            for even i, (2,3) for odd i), sorted, whose spacings are its
 *            barycentric weights.  Targets of dimension 4 to 6 take the
 *            black-box route (ft_sample_points, ft_consume_queries, their
 *            per-element-count forms, ft_project) in the FT_F64 and FT_F32
 *            forms (plain or stratified samples, the strata given by the
 *            base-m digits of the sample index over the d uniforms); there is
 *            no built-in source of those dimensions, and the split forms and
 *            batches return FT_E_UNSUPPORTED.
 *   coords   device, binary64, [dim][n_nodes] (SoA)
 *   conn     device, int32, [n_elems][dim+1] vertex ids in [0, n_nodes)
 *   out      host; receives a new handle (library-owned device memory:
 *            copies of the mesh, CSR mass matrix, Jacobi diagonal, lumped
 *            mass, node->element incidence, work vectors)
 * Errors: FT_E_ARG (dim, sizes, null), FT_E_MESH (id out of range, or an
 * element with |det J| <= 1e-12 h^d, h its longest edge), FT_E_OOM.
 * Synchronizes `stream`.
 */
ft_status ft_target_create(int32_t dim, int64_t n_nodes, const double* coords, int64_t n_elems,
                           const int32_t* conn, hipStream_t stream, ft_target** out);

/*
 * ft_target_create_p2 - setup of a target of quadratic (P2) Lagrange elements
 * on straight-sided triangles or tetrahedra (sec. 2 states the projection for
 * any target space V_t = span{psi_i}; App. A bounds its error for degree p).
 * Every transfer then follows sec. 4.1 with the P2 basis: the query list's
 * node block holds every P2 node (the control g = I_h f^s is f^s there), the
 * samples are drawn from the element's vertices exactly as for P1, and
 * g(X) = sum_i g_i psi_i(X) and the element loads use the P2 basis
 *   vertex k: l_k (2 l_k - 1),   edge e = (a, b): 4 l_a l_b,
 * (l: barycentric coordinates of the sample), which adds up to 1, so the
 * conservation identity holds as for P1.  M is assembled exactly from the
 * simplex moments.
 *   coords   device, binary64, [dim][n_nodes] (SoA): vertices and edge nodes
 *   conn     device, int32, [n_elems][(dim+1)(dim+2)/2]: the element's dim+1
 *            vertices, then its edge nodes in the order of the vertex pairs
 *            (0,1) (0,2) (1,2) for triangles, (0,1) (0,2) (0,3) (1,2) (1,3)
 *            (2,3) for tetrahedra; each edge node at the midpoint of its edge
 * Supported for P2 targets: ft_sample_points, ft_consume_queries (FT_F64 and
 * FT_F32, one fixed alpha, either value layout), ft_transfer_p1, ft_project;
 * the other routes return FT_E_UNSUPPORTED.
 * Errors: as ft_target_create; FT_E_MESH also for an edge node off its
 * edge's midpoint (relative 1e-10).  Synchronizes `stream`.
 */
ft_status ft_target_create_p2(int32_t dim, int64_t n_nodes, const double* coords, int64_t n_elems,
                              const int32_t* conn, hipStream_t stream, ft_target** out);

/* Release a target and all its device memory (null is accepted).  The
 * caller must make sure no work using it is still pending on any stream. */
ft_status ft_target_destroy(ft_target* t);

ft_status ft_target_get_info(const ft_target* t, ft_target_info* info /* host */);

/* Number of query points of a transfer: Q = n_nodes + n_elems * N (-1 on bad args). */
int64_t ft_query_count(const ft_target* t, int32_t samples_per_elem);

/*
 * ft_sample_points - the point-query list (sec. 4.1 step 1 and step 3).
 * Entries [0, n_nodes) are the target nodes (the control g = I_h f^s is
 * f^s at the nodes); entry n_nodes + t*N + j is sample j of element t:
 * Philox4x32-10 at counter (j, t, stream_id, blk) with key seed gives
 * uniforms, mapped to area/volume-uniform barycentric weights (Osada map for
 * triangles, sorted spacings for tetrahedra and d-simplices) and then to the physical point
 * sum_k lambda_k x_{v_k}.
 *   points   device, [dim][Q] in cfg->precision (Q = ft_query_count)
 * Errors: FT_E_ARG.  Asynchronous on `stream`.
 */
ft_status ft_sample_points(ft_target* t, const ft_sample_cfg* cfg, void* points, hipStream_t stream);

/*
 * ft_consume_queries - steps 4-6 of sec. 4.1 for the caller's point values.
 *   values   device, F*Q values in cfg->precision: f^s at every query point,
 *            [F][Q] in the order of ft_sample_points (nodes first, then
 *            samples), or element tiles (cfg->values_layout)
 * For every element t and local vertex k:
 *   beta_tk = |Omega_t| / N * sum_j (y_tj - alpha sum_l lambda_l g_{v_l}) lambda_k,
 * with lambda regenerated from the same Philox stream (cfg must match the
 * one given to ft_sample_points), then b_res,v = sum of beta_tk over the
 * (t, k) at node v in a fixed order (no floating-point atomics, so results
 * are bitwise reproducible).  With cfg->alpha_mode == FT_ALPHA_ELEMENT (forms
 * FT_F64 and FT_F32) each element uses its own coefficient, the one that
 * minimizes the sample variance of its residual terms summed over k:
 *   alpha_t = (P/N - sum_k A_k B_k / N^2) / (Q/N - sum_k B_k^2 / N^2),
 * A_k = sum_j y_tj lambda_k, B_k = sum_j g(X_tj) lambda_k, P = sum_j y_tj g(X_tj) w_j,
 * Q = sum_j g(X_tj)^2 w_j, w_j = sum_k lambda_k^2, clipped to [0, 2] (1 when the
 * denominator is not positive), and beta_tk also carries the element's exact
 * control part alpha_t (M_t g_t)_k; ft_project then adds no control and starts
 * from x = 0.  Estimating alpha_t from the same samples biases the estimate by
 * O(1/N).  The control values g (the first n_nodes
 * entries of each field) are copied into the target.  Non-finite values are
 * counted and reported by ft_project.
 * Errors: FT_E_ARG, FT_E_OOM.  Asynchronous on `stream`.
 */
ft_status ft_consume_queries(ft_target* t, const ft_sample_cfg* cfg, const void* values, hipStream_t stream);

/*
 * ft_consume_queries_noalloc - ft_consume_queries for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results
 * (bitwise) as ft_consume_queries; it calls no allocation routine and does
 * not synchronize.  The per-element loads (F * n_elems * (dim+1) binary64
 * values, between the element kernel and the node assembly) live in a fixed
 * 64 MiB device array of the library instead of the target: each GPU holds
 * its own copy until the process ends, every call on a GPU shares it and
 * leaves its contents behind, so calls that overlap on one GPU (any targets,
 * any streams) race and must be ordered by the caller.  The control values
 * and assembled loads go to the target's field buffers: a new target holds
 * them for one field, and a larger field count needs one ft_consume_queries
 * with that count first.
 * Errors: FT_E_ARG (as ft_consume_queries; element loads larger than 64 MiB;
 * n_fields above the target's field buffers), FT_E_ORDER, FT_E_UNSUPPORTED.
 * Asynchronous on `stream` (which must belong to the current device).
 */
ft_status ft_consume_queries_noalloc(ft_target* t, const ft_sample_cfg* cfg, const void* values, hipStream_t stream);

/* Result of ft_allocate_samples (host). */
typedef struct {
    int64_t total;              /* sum of the counts: samples of the new query list     */
    double  weight_sum;         /* W = sum_t a_t, a_t = |Omega_t| sigma_t as the pilot  */
                                /* estimated it                                          */
    double  predicted_stderr;   /* sqrt(sum_t a_t^2 / N_t): the standard error of sum b  */
                                /* the allocation should reach ((W^2 / total)^(1/2) when */
                                /* no count is clamped or rounded)                       */
} ft_allocation;

/*
 * ft_allocate_samples - samples per element from the element variances (sec. 7:
 * better sampling; App. B, Eq. cv_global_integral_estimator: with N_t
 * independent samples in element t, Var(sum b) = sum_t |Omega_t|^2 sigma_t^2 / N_t,
 * smallest for a total B when N_t is proportional to a_t = |Omega_t| sigma_t,
 * the Neyman allocation, where it equals W^2 / B).  The last transfer of the
 * target is the pilot: a fixed N0 >= 2 samples per element on a route that
 * estimates the element variances (ft_consume_queries in FT_F64 or FT_F32,
 * ft_transfer_p1, plans, ft_batch_consume_run); its variance terms
 * v_t = |Omega_t|^2 s_t^2 / N0 of field `field` give a_t = sqrt(N0 v_t)
 * (non-finite terms count as 0), and
 *   N_t = min(max(floor(budget a_t / W + 1/2), n_min), n_max)
 * (n_min everywhere when W = 0), W = sum_t a_t summed in a fixed order, so
 * the counts are the same on every run.
 *   budget        total samples wanted, in [1, 2^40] (ft_budget_for_tolerance
 *                 gives one for an error target); clamping makes the total differ
 *   n_min, n_max  1 <= n_min <= n_max <= 2^20 (n_min >= 2 keeps the standard
 *                 error of the next transfer estimable)
 *   offsets       device, int64 [n_elems + 1], written: exclusive prefix sums of
 *                 the counts, offsets[n_elems] = total (the input of
 *                 ft_sample_points_adaptive and ft_consume_queries_adaptive)
 *   out           host: total, W and the predicted standard error
 * Errors: FT_E_ARG, FT_E_ORDER (no such pilot), FT_E_OOM (scratch of about
 * n_elems / 64 doubles, kept by the target).  Synchronizes `stream`.
 */
ft_status ft_allocate_samples(ft_target* t, int32_t field, int64_t budget, int32_t n_min, int32_t n_max,
                              int64_t* offsets, ft_allocation* out, hipStream_t stream);

/* The total samples for which the Neyman prediction W / sqrt(B) reaches
 * rel_tol |sum_b|: ceil((weight_sum / (rel_tol |sum_b|))^2), at least 1, at
 * most 2^40 (1 when weight_sum or sum_b is 0; -1 on invalid arguments).
 * Host-only, touches no device memory. */
int64_t ft_budget_for_tolerance(double weight_sum, double sum_b, double rel_tol);

/*
 * ft_sample_points_adaptive - ft_sample_points with N_t = offsets[t+1] -
 * offsets[t] samples in element t: entries [0, n_nodes) are the nodes, entry
 * n_nodes + offsets[t] + j (j < N_t) is sample j of element t, the same
 * Philox counter (j, t, stream_id, blk) and map as ft_sample_points (so
 * N_t = N everywhere reproduces its samples).  cfg->samples_per_elem must be
 * 0; plain sampling; FT_F64 or FT_F32 points.
 *   offsets  device, int64 [n_elems + 1] (ft_allocate_samples, or the
 *            caller's: non-decreasing, 1 <= N_t <= 2^20, offsets[0] = 0,
 *            offsets[n_elems] = total); an element whose range is not valid
 *            gets no samples written, and ft_consume_queries_adaptive counts it
 *   total    host, the total number of samples, in [n_elems, 2^40]
 *   points   device, [dim][n_nodes + total] in cfg->precision
 * The caller keeps offsets unchanged until the matching consumption.
 * Errors: FT_E_ARG, FT_E_UNSUPPORTED.  Asynchronous on `stream`.
 */
ft_status ft_sample_points_adaptive(ft_target* t, const ft_sample_cfg* cfg, const int64_t* offsets, int64_t total,
                                    void* points, hipStream_t stream);

/*
 * ft_consume_queries_adaptive - ft_consume_queries for the list of
 * ft_sample_points_adaptive (the same cfg, offsets pointer and total):
 *   beta_tk = |Omega_t| / N_t * sum_{j < N_t} (y_tj - alpha g(X_tj)) psi_k(X_tj),
 * unbiased for every N_t >= 1, with fixed alpha or each element's own
 * (FT_ALPHA_ELEMENT, P1 targets), on P1 and P2 targets; values field-major
 * [F][n_nodes + total].  The element variances are |Omega_t|^2 s_t^2 / N_t,
 * so ft_project reports the standard error of sum b (-1 when an element has a
 * single sample).  An element with an invalid range contributes 0 and counts
 * as one non-finite value (ft_project then returns FT_E_NONFINITE).
 * Errors: FT_E_ARG, FT_E_ORDER, FT_E_UNSUPPORTED, FT_E_OOM.  Asynchronous on
 * `stream`.
 */
ft_status ft_consume_queries_adaptive(ft_target* t, const ft_sample_cfg* cfg, const int64_t* offsets, int64_t total,
                                      const void* values, hipStream_t stream);

/*
 * ft_transfer_p1_adaptive - ft_transfer_p1 with N_t = offsets[t+1] - offsets[t]
 * samples in element t (the counts of ft_allocate_samples): the same samples
 * as ft_sample_points_adaptive draws (so the same element loads as consuming
 * that list's values of the built-in source), with no query list in memory.
 * cfg->samples_per_elem must be 0; plain samples, FT_F64 or FT_F32, at most 4
 * fields, fixed alpha; P1 and P2 targets.  offsets and total as
 * ft_sample_points_adaptive (an invalid range contributes 0 and counts as a
 * non-finite value).  ft_project reports the standard error of sum b (-1 when
 * an element has a single sample).
 * Errors: FT_E_ARG, FT_E_UNSUPPORTED, FT_E_OOM.  Asynchronous on `stream`.
 */
ft_status ft_transfer_p1_adaptive(ft_target* t, ft_source* s, const ft_sample_cfg* cfg, const int64_t* offsets,
                                  int64_t total, hipStream_t stream);

/*
 * ft_project - step 2 and step 7 of sec. 4.1 and the conservation report.
 * Several fields (F > 1, at most 64) are solved together by a batched PCG that
 * reads M once per iteration for all of them, each field with its own
 * scalars and stopping test.
 * b = alpha M g + b_res (the control load integrated exactly), then Jacobi-PCG
 * on M y = b_res from y = 0 and x = alpha g + y (the same iterates as CG on
 * M x = b started at x = alpha g), stopping at ||b - M x|| <= rtol ||b||.
 *   x        device, binary64, [F][n_nodes]: the transferred coefficients
 *   b_out    device, binary64, [F][n_nodes] or null: the load vector b
 *   rep      host, [F] reports
 * Errors: FT_E_ORDER (no consume since the last sample), FT_E_ARG; per-field
 * FT_E_NOCONV / FT_E_NONFINITE are returned (the worst of them) after x is
 * written.  Synchronizes `stream`.
 */
ft_status ft_project(ft_target* t, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep,
                     hipStream_t stream);

/*
 * ft_transfer_p1 - steps 1 and 3-6 of sec. 4.1 with the built-in P1 source `s`
 * in place of a caller-side black box, without materializing the query list:
 * the same samples (Philox counters of cfg), the same localization rule and
 * the same element sums as ft_sample_points + ft_source_eval +
 * ft_consume_queries, fused into one pass over the samples.  Follow with
 * ft_project.  Requires cfg->precision FT_F64 or FT_F32 (the binary32 form:
 * binary32 samples and points, values rounded to binary32, as the query list
 * of that form holds them; sums in binary64), cfg->n_fields equal to the
 * source's field count (at most 4), and a source of the target's dimension.
 * Out-of-domain queries (nodes and samples) are counted for the transfer and
 * reported by ft_project (ft_report.n_out_of_domain).
 * Errors: FT_E_ARG, FT_E_UNSUPPORTED, FT_E_OOM.  Asynchronous on `stream`.
 */
ft_status ft_transfer_p1(ft_target* t, ft_source* s, const ft_sample_cfg* cfg, hipStream_t stream);

/*
 * ft_transfer_supermesh - the exact load vector b_i = integral f^s psi_i of
 * the built-in P1 source, by mesh intersection (sec. 3): every target
 * element is intersected with every source element that meets it (the
 * candidates come from the source's bin grid) and f^s psi_i, quadratic on
 * each intersection, is integrated exactly by a degree-2 rule.  Triangles:
 * the intersection polygon (target clipped by the three edge half-planes of
 * the source) is fanned from its first vertex, three-point rule per
 * sub-triangle.  Tetrahedra: the target is cut by the four face half-spaces
 * of the source, each cut leaving tetrahedra (a corner, or a prism split in
 * three), four-point rule per tetrahedron.  The reference the Monte Carlo
 * estimate converges to, and the paper's intersection-based comparator.
 * Follow with ft_project, which then solves M x = b with no control part
 * (alpha = 0, start x = 0); ft_report.n_out_of_domain counts the target
 * elements the source does not cover entirely.  At most 4 fields.
 *   area   device, binary64, [n_elems] or null: per target element, the sum
 *          of the areas (volumes) of its intersections (= |Omega_t| where the
 *          source covers it)
 * Errors: FT_E_ARG, FT_E_UNSUPPORTED, FT_E_OOM.  Asynchronous on `stream`.
 */
ft_status ft_transfer_supermesh(ft_target* t, ft_source* s, double* area, hipStream_t stream);

/*
 * ft_source_create_p1 - a P1 field on a source mesh, evaluated at points by
 * uniform-grid localization (sec. 5.3: grid cells per axis int(L sqrt(#elements))).
 *   coords         device, binary64, [dim][n_nodes]
 *   conn           device, int32, [n_elems][dim+1]
 *   nodal_values   device, binary64, [n_fields][n_nodes]
 *   bins           host, [dim] cells per axis, or null / zeros for the default
 *                  int(sqrt(n_elems)) along the longest axis in 2D,
 *                  round(0.75 cbrt(n_elems/6)) in 3D (ft_source_autotune refines it)
 * Localization rule: the element maximizing min_k mu_k(x) (mu: barycentric
 * coordinates); exact ties go to the lowest element id; a best min mu below
 * -1e-10 counts as out of domain and is evaluated by extrapolation from that
 * element, which is then searched among all elements (however far outside
 * the point lies; such points cost a pass over the whole mesh).
 * Errors: FT_E_ARG, FT_E_MESH, FT_E_OOM.  Synchronizes `stream`.
 */
ft_status ft_source_create_p1(int32_t dim, int64_t n_nodes, const double* coords, int64_t n_elems,
                              const int32_t* conn, int32_t n_fields, const double* nodal_values,
                              const int32_t* bins, hipStream_t stream, ft_source** out);

/*
 * ft_source_eval - evaluate the P1 source at points.
 *   points     device, [dim][ld] in `precision`, points 0..n_points-1 used
 *   values     device, [n_fields][ld_out] in `precision`
 *   elem_ids   device, int32, [n_points], or null: the containing source element
 * ld / ld_out are the leading dimensions (>= n_points).
 * Errors: FT_E_ARG.  Asynchronous on `stream`.
 */
ft_status ft_source_eval(ft_source* s, int64_t n_points, const void* points, int64_t ld, int32_t precision,
                         void* values, int64_t ld_out, int32_t* elem_ids, hipStream_t stream);

/*
 * ft_source_eval_queries - ft_source_eval over a query list from
 * ft_sample_points (sec. 4.1 steps 1 and 4): the first n_nodes points (the
 * target nodes) and the remaining n_points - n_nodes (the element-major
 * samples) are split into wavefronts separately, so that with N a multiple
 * of 256 every wavefront's points lie in one target element and share their
 * candidate source elements.  One launch.  Results are identical to
 * ft_source_eval on the same points for any n_nodes in [0, n_points].
 * Arguments as for ft_source_eval.  Errors: FT_E_ARG.  Asynchronous on `stream`.
 */
ft_status ft_source_eval_queries(ft_source* s, int64_t n_nodes, int64_t n_points, const void* points, int64_t ld,
                                 int32_t precision, void* values, int64_t ld_out, int32_t* elem_ids,
                                 hipStream_t stream);

/*
 * ft_source_eval_tiles - ft_source_eval_queries over the query list of a
 * transfer (n_nodes nodes, then n_elems x samples_per_elem samples), the
 * values written as FT_VALUES_ELEMENT_TILES: [F][n_nodes], then one F x N
 * tile per element (one element's samples of all fields contiguous, for
 * ft_consume_queries with cfg->values_layout = FT_VALUES_ELEMENT_TILES).
 *   points   device, [dim][ld] in `precision` (ld >= n_nodes + n_elems N)
 *   values   device, F (n_nodes + n_elems N) values in `precision`
 *   elem_ids device, int32, [n_nodes + n_elems N], or null
 * Errors: FT_E_ARG.  Asynchronous on `stream`.
 */
ft_status ft_source_eval_tiles(ft_source* s, int64_t n_nodes, int64_t n_elems, int32_t samples_per_elem,
                               const void* points, int64_t ld, int32_t precision, void* values, int32_t* elem_ids,
                               hipStream_t stream);

/*
 * ft_source_autotune - choose the bin grid for a query distribution.  For
 * each candidate resolution (cells along the longest axis of the source's
 * box, the other axes proportionally fewer) the bins are rebuilt and
 * ft_source_eval_queries is timed on `points` (a sample of the real queries,
 * laid out as for ft_source_eval_queries); the fastest grid is kept.
 *   candidates  host [n_candidates], 1..64 entries
 *   bins_out    host [3] or null: the chosen cells per axis
 * The tuning launches' out-of-domain counts are discarded (the count is
 * reset).  Errors: FT_E_ARG, FT_E_OOM, FT_E_DEVICE.  Synchronizes `stream`.
 */
ft_status ft_source_autotune(ft_source* s, int64_t n_nodes, int64_t n_points, const void* points, int64_t ld,
                             int32_t precision, int32_t n_candidates, const int32_t* candidates, int32_t* bins_out,
                             hipStream_t stream);

/* Sizes of a source after setup. */
typedef struct {
    int32_t dim;
    int32_t n_fields;
    int64_t n_nodes;
    int64_t n_elems;
    int32_t bins[3];            /* cells per axis of the localization grid (1 for unused axes)    */
    int64_t n_registrations;    /* element ids stored over all bins (one per element)              */
} ft_source_info;

ft_status ft_source_get_info(const ft_source* s, ft_source_info* info /* host */);

/*
 * ft_source_integral - the exact integral of each source field over the
 * source mesh, the quantity a conservative transfer preserves (sec. 2, Eq.
 * conservation; the relative conservation error of sec. 5.1 compares the
 * transferred integral m^T x with it):
 *     int f = sum_e |Omega_e| * (mean of f over e's vertices),
 * summed with compensation (each addition's rounding error carried along).
 *   integrals  host, [n_fields]
 * Errors: FT_E_ARG, FT_E_OOM.  Synchronizes `stream`.
 */
ft_status ft_source_integral(ft_source* s, double* integrals, hipStream_t stream);

/* Out-of-domain points seen by ft_source_eval and ft_source_eval_queries since
 * the last call (then reset); the transfer routes report theirs in
 * ft_report.n_out_of_domain.
 * Synchronizes `stream`. */
ft_status ft_source_stats(ft_source* s, int64_t* n_out_of_domain /* host */, hipStream_t stream);

ft_status ft_source_destroy(ft_source* s);

/*
 * Plans: the setup/online split of a transfer from the built-in source
 * (sec. 5.3: localization is paid once at initialization, later transfers
 * between the same meshes only evaluate, accumulate and solve).
 */
typedef struct ft_plan ft_plan;

/*
 * ft_plan_create - draw the samples of `cfg` on target `t` and localize every
 * target node and sample in source `s` once (the containing source element
 * of each query is kept on the device, 4 bytes per query).  cfg: FT_F64,
 * n_fields equal to the source's field count.  t and s are not owned and must
 * outlive the plan.  Out-of-domain queries are counted once here and reported
 * by ft_project after every ft_plan_transfer (ft_report.n_out_of_domain).
 * Errors: FT_E_ARG, FT_E_UNSUPPORTED, FT_E_OOM.  Synchronizes `stream`.
 */
ft_status ft_plan_create(ft_target* t, ft_source* s, const ft_sample_cfg* cfg, hipStream_t stream, ft_plan** out);

/*
 * ft_plan_transfer - sec. 4.1 steps 1 and 3-6 with the cached localization:
 * the source field given by `nodal_values` (device, binary64, [n_fields][n_nodes
 * of the source mesh]; null = the source's own values) is interpolated at the
 * plan's samples and nodes, and the residual element sums and node assembly
 * follow as in ft_transfer_p1 (bitwise equal to it for the source's own
 * values).  Follow with ft_project.  Asynchronous on `stream`.
 */
ft_status ft_plan_transfer(ft_plan* p, const double* nodal_values, hipStream_t stream);

ft_status ft_plan_destroy(ft_plan* p);

/*
 * Batches: many independent transfers from built-in P1 sources (one field
 * each, FT_F64 or FT_F32 as ft_transfer_p1), of mixed dimension, size and
 * samples per element, run as one sequence of launches.  Target elements of all transfers are the work
 * units of persistent kernels, one launch per element-kernel variant (sec.
 * 4.1: the element sums of step 5 are independent); the node sums and the
 * mass solves of all transfers share their launches.  Each transfer gives exactly the samples and element sums
 * of ft_transfer_p1 on the same target, source and cfg (samples_per_elem > 8),
 * and a solution of the same M x = b to the same tolerance.
 */
typedef struct ft_batch ft_batch;

enum { FT_BATCH_GRAPH = 1 };   /* capture a run as a HIP graph; later runs replay it */

/*
 * ft_batch_create - set up a batch of `count` transfers.
 *   targets, sources   host arrays [count] of handles; not owned: they must
 *                      outlive the batch, and no other call may use them while
 *                      ft_batch_run runs.  Targets must be distinct (P1).
 *                      sources may hold only null entries: a batch for
 *                      caller values (ft_batch_consume_run)
 *   cfgs               host [count]: per-transfer sample configuration
 *                      (n_fields = the source's field count, FT_F64 or FT_F32)
 *   flags              0 or FT_BATCH_GRAPH
 * A transfer of F fields runs as F systems, one per field, sharing its
 * target's mass matrix and samples (each field localizes its samples again:
 * a multi-field transfer costs about F one-field ones in the element stage).
 * Builds the work lists (node, element and row tiles; element tiles grouped
 * by variant, the dearest variants first) and the batch's solver vectors on
 * the device.
 * Errors: FT_E_ARG, FT_E_UNSUPPORTED, FT_E_OOM.  Synchronizes `stream`.
 */
ft_status ft_batch_create(int32_t count, ft_target* const* targets, ft_source* const* sources,
                          const ft_sample_cfg* cfgs, int32_t flags, hipStream_t stream, ft_batch** out);

/*
 * ft_batch_run - sec. 4.1 steps 1-7 for every transfer of the batch
 * (binary64 solve: cfg->refine_steps must be 0).
 *   x        host array [count] of device pointers: x[k] binary64 [n_fields][n_nodes] of transfer k
 *   b        host array [count] of device pointers (load vectors, as x) or null entries, or null
 *   reports  host [sum of n_fields], one report per field: transfer 0's fields, then transfer 1's, ...
 *   status   host [sum of n_fields] or null: per-field status
 * The solve launches exactly cfg->max_iter Jacobi-PCG iterations (a converged
 * system's tiles return at once), so a run has no host synchronization until
 * its end; with FT_BATCH_GRAPH the first run with a given (rtol, max_iter) is
 * captured and replayed afterwards.  Afterwards every target is in the state
 * ft_transfer_p1 leaves (ft_project may re-solve it).
 * Returns FT_OK, or the worst per-transfer status (FT_E_NONFINITE before
 * FT_E_NOCONV).  Synchronizes `stream`.
 */
ft_status ft_batch_run(ft_batch* b, const ft_solve_cfg* cfg, double* const* x, double* const* bvec,
                       ft_report* reports, int32_t* status, hipStream_t stream);

/*
 * ft_batch_consume_run - the black-box route for every transfer of a batch
 * (sec. 4.1 steps 4-7 from the caller's values): each transfer's values are
 * consumed as ft_consume_queries does, then all fields of all transfers are
 * assembled and solved together by the batched Jacobi-PCG and reported as
 * ft_batch_run does (n_out_of_domain -1, sum_b_stderr from the samples).
 * Each target must hold the query list of its transfer (ft_sample_points
 * with the transfer's cfg); the batch may have been created without sources
 * (sources[k] all null), and then only this call runs it.
 *   values   host array [count] of device pointers: the query values of
 *            transfer k, [n_fields][Q_k] (or element tiles, per its cfg),
 *            binary64 or binary32 as its cfg
 *   x, b, reports, status   as ft_batch_run
 * FT_F64 and FT_F32 transfers with one fixed alpha each.  Runs without a
 * graph.  Errors: FT_E_ARG, FT_E_ORDER (a target not sampled with its
 * transfer's configuration), FT_E_UNSUPPORTED; per-field FT_E_NOCONV /
 * FT_E_NONFINITE as ft_batch_run.  Synchronizes `stream`.
 */
ft_status ft_batch_consume_run(ft_batch* b, const ft_solve_cfg* cfg, const void* const* values, double* const* x,
                               double* const* bvec, ft_report* reports, int32_t* status, hipStream_t stream);

/*
 * ft_batch_autotune - pick, for each kind of transfer in the batch, the
 * element-stage variant and the bin grid of its source by timing them (a
 * kind: architecture, dimension, form, N, fields and the power-of-two
 * buckets of the target and source element counts).  For the largest
 * transfer of each kind not found in the cache: ft_source_autotune on a run
 * of that transfer's own samples (cells along the longest axis 0.6 to 1.6
 * times the default of ft_source_create_p1), then each of the five (lanes per element, samples per
 * lane) variants (64,4) (64,2) (64,1) (32,1) (16,1) of the batch's element
 * kernel on that transfer, the fastest kept; the other transfers of the kind
 * take the same variant and the same factor on their sources' cells.
 * Results stay those of the same transfers with other variants to rounding
 * (the variant fixes the order of each element's sums).
 *   cache_path  host, a JSON file (one entry per line) read before tuning and
 *               rewritten with every entry after it, or null (no cache)
 *   n_tuned     host, or null: kinds timed in this call (0 when all came
 *               from the cache)
 * Rebuilds the bins of the batch's sources and the element work lists; a
 * captured graph is captured again by the next run.  Uses temporary device
 * memory for the samples.  Errors: FT_E_ARG (cache not writable), FT_E_OOM,
 * FT_E_DEVICE.  Synchronizes `stream`.
 */
ft_status ft_batch_autotune(ft_batch* b, const char* cache_path, int32_t* n_tuned, hipStream_t stream);

/* The element-stage variant of transfer k: lanes per element and samples per lane per round. */
ft_status ft_batch_variant(const ft_batch* b, int32_t k, int32_t* lanes_per_elem, int32_t* samples_per_lane);

ft_status ft_batch_destroy(ft_batch* b);

/* Samples per element for a target relative standard error of sum b
 * (App. B, Eq. conservation_residual_bound: E[E_cons^2] falls as 1/N):
 * ceil(N (sum_b_stderr / (rel_tol |sum_b|))^2), at least 1, at most 2^20.
 *   rep               host, a report of a transfer made with N samples per element
 *   samples_per_elem  that N
 *   rel_tol           the target standard error relative to |sum_b| (> 0)
 * Returns 1 when the report's standard error is 0 (no sampling error) or
 * sum_b is 0; -1 when the report carries no estimate (sum_b_stderr < 0) or
 * an argument is invalid.  Host-only, touches no device memory. */
int32_t ft_samples_for_tolerance(const ft_report* rep, int32_t samples_per_elem, double rel_tol);

/* Message describing the last failure on this thread ("" if none). */
const char* ft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FT_H */
