/*
 * xrl.h -- C-ABI of the MI355X (gfx950) FMM-accelerated panel operator of the
 * XRL method (arXiv 2409.12375).
 *
 * The operator.  After the centroid-midpoint basis transformation (Sec. II-A,
 * Fig. 2, Algorithm 1) the surface current is carried by pulse functions on
 * flat triangle panels, one scalar density per Cartesian component
 * (eq. (4)), and the expensive part of every iteration of the solve is the
 * product of the panel matrix P with those densities (eq. (9), Sec. II-C):
 *
 *     (P x)_k = sum_l P_kl x_l,   P_kl = int_{S_k} int_{S_l} 1/|r - r'| dS' dS
 *
 * (eq. (6), second term, with the factor j*omega*mu0/(4*pi) taken outside the
 * integral as Sec. II-D describes, so P is frequency independent and shared by
 * every port and frequency).  P is real, symmetric and positive definite
 * (Sec. II-D); densities are complex.  The library applies P with a fast
 * multipole method on the panel centroids (Sec. II-C) and stores the
 * near-field entries on panels (Sec. II-C, last paragraph).
 *
 * Conventions (all entry points):
 *  - Every function returns xrl_status; 0 is success, negative is an error.
 *    Nothing throws across the ABI.  xrl_last_error() returns a thread-local
 *    message describing the last failure on the calling thread.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it; functions that must read results back to the host
 *    synchronise that stream before returning.
 *  - Handles are opaque and owned by the library; each create has a matching
 *    destroy.  Device memory for handles and temporaries comes from the
 *    allocator installed with xrl_set_allocator (hipMalloc/hipFree when none
 *    is).  Caller buffers (x, y, b) are never freed by the library.
 *  - On error the outputs are unspecified and the handles stay valid.
 *    Asynchronous kernel faults surface as XRL_E_HIP at the next call that
 *    synchronises.
 */
#ifndef XRL_H
#define XRL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xrl_status;
#define XRL_OK 0
#define XRL_E_INVALID_ARG (-1)      /* bad pointer, size, option or layout */
#define XRL_E_DEGENERATE_PANEL (-2) /* a panel with (near) zero area or a NaN vertex */
#define XRL_E_OOM (-3)              /* device or host allocation failed */
#define XRL_E_HIP (-4)              /* a HIP runtime call failed */
#define XRL_E_NOT_CONVERGED (-5)    /* GMRES stopped before reaching rtol */
#define XRL_E_UNSUPPORTED (-6)      /* option combination not implemented */
#define XRL_E_STATE (-7)            /* call out of order (e.g. matvec before assemble) */

/* Device-memory hand-off.  alloc returns `bytes` of device memory on the
 * current device (256-byte aligned), or NULL when it cannot; `stream` is the
 * stream of the library call that needs the memory (the buffer is first used
 * in stream order on it).  free releases a pointer alloc returned; the library
 * waits for the device to finish every use of the buffer before it calls free.
 * ctx is passed through.  The hooks may be called from any library entry point
 * except xrl_fmm_matvec_noalloc, which allocates nothing. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} xrl_allocator;

/* Install `a` (copied) for every later device allocation of the library, in
 * every thread; NULL restores hipMalloc/hipFree.  A buffer is always released
 * through the allocator that made it, also after the allocator is changed, so
 * the hooks and ctx must stay valid until every handle created while they
 * were installed is destroyed.  Errors: XRL_E_INVALID_ARG (one hook NULL). */
xrl_status xrl_set_allocator(const xrl_allocator *a);

/* Data types of densities and potentials (complex, interleaved re/im). */
#define XRL_C64 1  /* complex64: pairs of float  */
#define XRL_C128 2 /* complex128: pairs of double */

/* Arithmetic of the operator application. */
#define XRL_PREC_FP64 0  /* every phase in FP64 (M2L on FP64 MFMA)                      */
#define XRL_PREC_FP32 1  /* "plain FP32": every phase FP32, M2L on the vector ALUs,
                            near field by quadrature in FP32                             */
#define XRL_PREC_MIXED 2 /* FP32 M2L on MFMA with FP32 accumulation; self and touching
                            near-field integrals in FP64, stored FP32                   */

/* Translation engine (M2L, and M2M/L2L with it). */
#define XRL_M2L_AUTO 0    /* MFMA for FP64 and MIXED, vector ALU for FP32 */
#define XRL_M2L_MFMA 1    /* MFMA; M2M and L2L target-stationary; M2L follows the
                             column count of each call: offset-stationary below 16
                             real columns, target-stationary from 16 on               */
#define XRL_M2L_VALU 2    /* vector ALU, offset-stationary                             */
#define XRL_M2L_MFMA_OS 3 /* MFMA, always offset-stationary (pairs that share an
                             operator batched into one GEMM, per-target reduction)    */
#define XRL_M2L_MFMA_TS 4 /* MFMA, always target-stationary (one wave per target
                             accumulates its pairs in registers)                      */

const char *xrl_last_error(void);
/* Library version string (static storage). */
const char *xrl_version(void);

/* ------------------------------------------------------------------ */
/* Mesh and tree                                                       */
/* ------------------------------------------------------------------ */
/* An indexed surface mesh of flat panels (Sec. II-A: triangles, or the
 * hybrid mesh of triangles and rectangles of Fig. 1).
 * vertices: [n_vertices][3] float64.
 * tris: vertex indices (0-based), [n_panels][3] int32 when verts_per_panel is
 *   3 (or 0); [n_panels][4] when it is 4, a row (a, b, c, d) being the
 *   four-sided panel whose surface is the union of the triangles (a, b, c)
 *   and (a, c, d) (a rectangle, or any planar quadrilateral), and a row with
 *   d < 0 a triangle (a, b, c).  One pulse function per panel (eq. (4)): a
 *   four-sided panel is one unknown, integrated over both of its triangles.
 * Both arrays live on the host (on_device = 0) or on the current HIP device
 * (on_device = 1); they are copied during xrl_tree_build and not referenced
 * afterwards.  Vertex order only fixes the sign of the panel normal, which P
 * does not use. */
typedef struct {
    int64_t n_vertices;
    int64_t n_panels;
    const double *vertices;
    const int32_t *tris;
    int32_t on_device;
    int32_t verts_per_panel; /* 3 (0 reads as 3) or 4 */
} xrl_mesh_desc;

typedef struct xrl_tree xrl_tree;
typedef struct xrl_plan xrl_plan;

/* Panel geometry (centroid, area, normal, diameter), a cube around all
 * centroids, 63-bit Morton codes of the centroids, a radix sort and a
 * level-by-level split of every box holding more than max_leaf centroids,
 * all on the device (the octree of the FMM of Sec. II-C, built on panel
 * centroids).  A panel belongs to the box that holds its centroid.  On a
 * hybrid mesh the tree sorts elements: every triangle, and both triangles of
 * every four-sided panel, each by its own centroid; the FMM, the near field
 * and the leaf sizes count elements, and the matvec gathers each panel's
 * density to its elements and sums their potentials back (P = S P_tri S^T,
 * S the panel-element membership; the integral over a panel is the sum over
 * its triangles).
 *   max_leaf  : 1..128; near-field blocks are padded to a multiple of 4
 *               targets.  Larger leaves move work from the translations to
 *               the near field (fewer M2L pairs, more stored values).
 *   max_depth : 1..21; a box at max_depth is a leaf whatever its count
 *               (flagged in xrl_tree_info.n_overfull_leaves).
 * Errors: XRL_E_INVALID_ARG (sizes, indices out of range),
 *         XRL_E_DEGENERATE_PANEL (area <= 1e-14 * diameter^2, a non-finite
 *         vertex, or two panels with the same three vertex indices or the
 *         same three vertex positions: coincident panels make P singular),
 *         XRL_E_OOM, XRL_E_HIP. */
xrl_status xrl_tree_build(const xrl_mesh_desc *mesh, int32_t max_leaf, int32_t max_depth,
                          void *stream, xrl_tree **out);
void xrl_tree_destroy(xrl_tree *tree);

typedef struct {
    int64_t n_panels;
    int64_t n_boxes;
    int64_t n_leaves;
    int32_t depth;             /* deepest level present (root = 0) */
    int32_t n_overfull_leaves; /* leaves at max_depth with more than max_leaf elements */
    double root_center[3];
    double root_size;          /* side of the root cube */
    int64_t n_elements;        /* triangles the tree sorts: n_panels plus one per
                                  four-sided panel */
} xrl_tree_info;
xrl_status xrl_tree_get_info(const xrl_tree *tree, xrl_tree_info *info);

/* ------------------------------------------------------------------ */
/* Plan                                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t order;     /* expansion order p, even, 2..12 (other values: XRL_E_UNSUPPORTED);
                          (p+1)^2 real coefficients per column */
    int32_t precision; /* XRL_PREC_* */
    int32_t m2l_engine;/* XRL_M2L_* */
    int32_t max_cols;  /* largest number of complex columns one matvec will carry */
    double theta;      /* separation criterion of the M2L (V-list) pairs: a same-level
                          pair is translated only if r_t + r_s < theta * |c_t - c_s|
                          (r: panel-inclusive box radii), else applied directly as
                          near field.  0 selects the default (XRL_DEFAULT_THETA);
                          otherwise 0.5 <= theta <= 1. */
} xrl_plan_opts;
#define XRL_DEFAULT_THETA 0.9

/* Interaction lists of the adaptive octree (U: adjacent leaves, V: same-level
 * well-separated boxes, W and X: the adaptive lists), translated into a
 * near-field list per target leaf (U, W and X, applied directly) and M2L
 * pairs (V), plus the translation operators (M2M, L2L: 8 each; M2L: one per
 * integer offset in [-3,3]^3 outside [-1,1]^3) and the per-panel moment table
 * of the regular solid harmonics integrated exactly over each panel.
 * Several trees make one batched plan: the meshes are stacked in the order
 * given, densities are concatenated along the panel axis.  The trees must
 * outlive the plan.
 * Errors: XRL_E_INVALID_ARG, XRL_E_UNSUPPORTED (order or engine; or a leaf
 *         holding more than 128 panels at the maximum depth, i.e. nearly
 *         coincident centroids), XRL_E_OOM, XRL_E_HIP. */
xrl_status xrl_fmm_plan(xrl_tree *const *trees, int32_t n_trees, const xrl_plan_opts *opts,
                        void *stream, xrl_plan **out);
void xrl_plan_destroy(xrl_plan *plan);

typedef struct {
    int64_t n_panels;
    int64_t n_boxes;
    int64_t n_leaves;
    int64_t n_m2l_pairs;  /* V-list pairs over all levels */
    int64_t n_near_rows;  /* source rows over all target leaves */
    int64_t n_near_entries; /* stored near-field values (with target padding) */
    int64_t n_near_pairs; /* unpadded target-source panel pairs */
    int32_t order;
    int32_t precision;
    double max_sep_ratio; /* max over M2L pairs of (rad_t + rad_s) / |c_t - c_s| */
    int64_t n_demoted_pairs; /* V-list candidates whose panel-inclusive radii do not
                                separate them; applied directly as near field */
    double theta;            /* separation criterion in use (xrl_plan_opts.theta) */
    int64_t n_elements;      /* triangles the FMM and the near field work on */
} xrl_plan_info;
xrl_status xrl_plan_get_info(const xrl_plan *plan, xrl_plan_info *info);

/* ------------------------------------------------------------------ */
/* Near field                                                          */
/* ------------------------------------------------------------------ */
/* Optional learned surrogate for near-singular pairs: a 18 -> H -> H -> 2
 * multilayer perceptron with SiLU activations (H = 64 or 128).  Its first
 * output divided by rho^4 (rho: distance of the target centroid from the
 * source centroid in source diameters, from the features) predicts
 * P_kl / P_kl^(3x3 Gauss) - 1; its second output predicts log10 of the
 * absolute error of that prediction.  Weights are FP32, row-major [out][in],
 * on the host. */
typedef struct {
    int32_t hidden;          /* H (128) */
    const float *w1, *b1;    /* [H][18], [H] */
    const float *w2, *b2;    /* [H][H],  [H] */
    const float *w3, *b3;    /* [2][H],  [2] */
    const float *feat_lo, *feat_hi; /* [18] input range seen in training */
    float log10_err_bound;   /* fall back to quadrature when out[1] exceeds it */
} xrl_mlp;

typedef struct {
    double r_near;      /* non-touching pairs with |c_k-c_l|/max(diam) < r_near use the
                           semi-analytic rule (default 2.0) */
    double r_mid;       /* regular pairs below r_mid use the finer product rule (FP32
                           storage: 12-point symmetric triangle rules, FP64: 5x5
                           conical Gauss), above it the coarser (6-point; 4x4);
                           default 4.0, where the coarser rule is within 2e-7 of
                           the exact entry */
    const xrl_mlp *surrogate; /* NULL: quadrature everywhere */
    int32_t audit_every;      /* with a surrogate: every k-th accepted pair is also
                                 integrated by quadrature for the error report (0: off) */
} xrl_nf_opts;

typedef struct {
    int64_t n_entries;     /* stored values (padding included) */
    int64_t n_self, n_touching, n_near_singular, n_regular;
    int64_t n_mlp_accepted, n_mlp_fallback;
    double audit_max_rel_err, audit_rms_rel_err; /* surrogate audit, if any */
    double ms;             /* wall time of the assembly */
    int64_t n_regular_fine; /* regular pairs below r_mid (the finer product rule) */
} xrl_nf_stats;

/* Fill the near-field panel-panel entries P_kl (frequency independent, done
 * once and reused by every matvec, Sec. II-C and II-D).  Pair classes: self
 * (closed form), touching (shared vertex index: exact inner integral, graded
 * outer rule), near-singular (exact inner integral, subdivided outer rule, or
 * the surrogate), regular (product Gauss).  stats may be NULL.
 * Errors: XRL_E_INVALID_ARG, XRL_E_OOM, XRL_E_HIP. */
xrl_status xrl_nearfield_assemble(xrl_plan *plan, const xrl_nf_opts *opts, void *stream,
                                  xrl_nf_stats *stats);

/* Self-test of the 16x16x16 bf16 MFMA layout used by the surrogate's
 * inference: D[16][16] = bf16(A[16][16]) * bf16(B[16][16]), float host arrays. */
xrl_status xrl_selftest_mfma_bf16(const float *A, const float *B, float *D);

/* Surrogate support (the learned near-singular model above).
 * Features and cheap values of explicit triangle pairs, on the device:
 *   tri_k, tri_l : [n][9] float64 (target, source vertices)
 *   feat         : [n][18] float32 (canonical frame of the source, see the
 *                  surrogate source file), cheap: [n] float64 3x3 Gauss value
 *                  (may be NULL). */
xrl_status xrl_surrogate_features(const double *tri_k, const double *tri_l, int64_t n, float *feat,
                                  double *cheap, void *stream);

/* Training of the surrogate on the device with the library's own FP32
 * forward, backward and Adam kernels.  Weights w (device, packed
 * W1 b1 W2 b2 W3 b3, H*H + 22*H + 2 floats) hold the initial values on entry
 * and the trained values on exit.  Loss: mean (y0 - t)^2 +
 * calib_weight * mean (y1 - (log10(target_scale |y0 - t| / rho^4) - log_mu) / log_sigma)^2,
 * the second target taken as a constant (no gradient through y0).
 * X: [n][18] device features, t: [n] device targets.  loss_hist: host
 * [epochs] (mean first loss term over each epoch) or NULL. */
typedef struct {
    int32_t hidden, batch, epochs;
    float lr, lr_decay, beta1, beta2, eps;
    float calib_weight, log_mu, log_sigma, target_scale;
    uint64_t seed;
} xrl_mlp_train_opts;
xrl_status xrl_mlp_train(const float *X, const float *t, int64_t n, const xrl_mlp_train_opts *opts,
                         float *w, float *loss_hist, void *stream);

/* Loss (host [2]: the two terms) and gradient (device, packed like w) of one
 * batch; loss_args (host [4]) = calib_weight, log_mu, log_sigma, target_scale. */
xrl_status xrl_mlp_loss_grad(const float *w, int32_t hidden, const float *X, const float *t, int64_t n,
                             const float *loss_args, float *loss, float *grad, void *stream);

/* Forward pass, out: [n][2] device, first output already divided by rho^4.
 * bf16 = 0: FP32 kernels (training path); bf16 = 1: the BF16 MFMA inference
 * kernel used by the assembly. */
xrl_status xrl_mlp_forward(const float *w, int32_t hidden, const float *X, int64_t n, int32_t bf16,
                           float *out, void *stream);

/* ------------------------------------------------------------------ */
/* Operator application                                                */
/* ------------------------------------------------------------------ */
/* Per-column complex scalars for y = alpha_c * (P x)_c + beta_c * A .* x_c
 * (A = panel areas, i.e. the Galerkin mass term of eq. (6) first term with
 * beta = Z_s).  alpha, beta: host arrays of n_cols (re, im) double pairs;
 * either may be NULL (alpha = 1, beta = 0). */
typedef struct {
    const double *alpha;
    const double *beta;
} xrl_epilogue;

/* y = P x (plus the optional epilogue) for n_cols complex columns.
 *   x : device, [n_panels][ldx] complex (XRL_C64 or XRL_C128), user panel
 *       order, columns 0..n_cols-1 used; ldx >= n_cols (in complex elements).
 *   y : device, [n_panels][ldy] same dtype; only columns 0..n_cols-1 written.
 * n_cols <= max_cols of the plan.  Requires xrl_nearfield_assemble first.
 * x and y must not overlap.
 * Errors: XRL_E_INVALID_ARG, XRL_E_STATE, XRL_E_HIP. */
xrl_status xrl_fmm_matvec(const xrl_plan *plan, const void *x, int64_t ldx, int32_t n_cols,
                          int32_t dtype, void *y, int64_t ldy, const xrl_epilogue *ep,
                          void *stream);

/* The same product for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the call allocates nothing.  Its work arrays (sorted densities
 * and potentials, multipole and local expansions, epilogue scalars) live in
 * one fixed 64 MiB device array of the library, one copy per device, held
 * until the process ends; the plan, x and y are the caller's as above.
 *   - Needs 4*8*n_cols + 2*(N*2*n_cols + 256)*E + 2*(B*K*2*n_cols + 256)*E
 *     bytes (E = 8 for FP64 plans, else 4; each part rounded up to 256; N
 *     panels, B boxes, K = (p+1)^2); larger requests fail with
 *     XRL_E_INVALID_ARG and a message naming the size.
 *   - The translations always run target-stationary on the matrix cores (no
 *     per-pair scratch); results agree with xrl_fmm_matvec to rounding.
 *   - Runs eagerly: graph mode and profiling of the plan do not apply.
 *   - Every call on one device shares that device's array: calls that
 *     overlap on one device (concurrent streams or threads) race and give
 *     undefined results.  The array keeps the last call's contents; the call
 *     overwrites every element it reads.
 * Errors: XRL_E_INVALID_ARG, XRL_E_STATE, XRL_E_HIP. */
xrl_status xrl_fmm_matvec_noalloc(const xrl_plan *plan, const void *x, int64_t ldx, int32_t n_cols,
                                  int32_t dtype, void *y, int64_t ldy, const xrl_epilogue *ep, void *stream);

/* Per-phase device times (milliseconds), recorded with HIP events on the
 * matvec stream while profiling is on (no host wait inside the matvec):
 * xrl_plan_get_phase_ms waits for the recorded events and returns the mean
 * over the matvecs since profiling was switched on (the last 256 at most).
 * [0] gather [1] P2P [2] P2M [3] M2M [4] M2L [5] L2L [6] L2P [7] scatter. */
#define XRL_N_PHASES 8
xrl_status xrl_plan_set_profiling(xrl_plan *plan, int32_t on);
xrl_status xrl_plan_get_phase_ms(const xrl_plan *plan, double *ms /* [XRL_N_PHASES] */);

/* Kernel-shape knobs of a plan (results agree to rounding for every
 * setting; only speed changes).  Takes effect at the next matvec.
 *   XRL_TUNE_TS_KERNEL   (0..2, default 0): form of the target-stationary M2L:
 *       0  software-pipelined, one operator per offset;
 *       1  software-pipelined, the 64 operators of non-negative offsets with
 *          the others applied as sign-reflected copies (a smaller table);
 *       2  two waves per SIMD, no explicit pipeline, one operator per offset.
 *   XRL_TUNE_TS_MIN_COLS (>= 1, default 16): with XRL_M2L_MFMA, the
 *       translations run target-stationary from this many real columns on,
 *       offset-stationary below.
 *   XRL_TUNE_P2P_FORM    (0..2, default 0; 2 on XRL_M2L_VALU plans): P2P
 *       above 16 FP32 columns on the 16x16x4 MFMA, densities times the
 *       stored block (0), on the vector ALU with the source densities read
 *       as wave-uniform scalars (1, one lane per target), or on the vector
 *       ALU with the source densities staged in LDS (2).
 *   XRL_TUNE_TS_ORDER    (0/1, default 1): launch order of the
 *       target-stationary translations: the targets with the most pairs
 *       first (1) or in box order (0).
 *   XRL_TUNE_L2L_FORM    (0/1, default 1): the translations with one source
 *       per target (L2L) source-stationary, one wave per parent holding its
 *       local expansion for all its children (1), or target-stationary (0).
 *   XRL_TUNE_M2M_FORM    (0..2, default 2): the translations with at most
 *       eight pairs per target (M2M) with one wave per 16-row tile of each
 *       target (1), one wave per target (0), or the first on levels with
 *       fewer than 1024 targets and the second on the others (2).
 *   XRL_TUNE_LEAF_FORM   (0/1, default 1; 0 on XRL_M2L_VALU plans): P2M and
 *       L2P above 16 FP32 columns as per-leaf 16x16x4 MFMA products (1) or
 *       on the vector ALU with LDS-staged tiles (0).
 *   XRL_TUNE_TS_NARROW_COLS (0/1, default 1): FP32 target-stationary forms
 *       0 and 1 with 1..4 real columns past the last full 16-column tile
 *       (C = 16 n + 1 .. 16 n + 4, e.g. 18 complex columns): those columns
 *       on 4x4x1 MFMA blocks beside the n 16x16x4 tiles (1) or in a further,
 *       mostly padded 16x16x4 tile (0).
 *   XRL_TUNE_VALU_FORM   (0/1, default 1): the vector-ALU offset-stationary
 *       translations in FP32 up to order 8: one column per thread with all
 *       (p+1)^2 output rows in registers and the operator read from LDS as
 *       broadcasts (1), or 16 x 4 register tiles of 6 rows by 4 columns over
 *       64-column blocks (0).
 *   XRL_TUNE_LEAF_L2L    (0/1, default 1): FP32 plans whose P2M and L2P run
 *       on MFMA (more than 16 real columns): L2P adds the parent's local
 *       expansion through each leaf's L2L operator itself (a second
 *       contraction with precomputed moment rows), and L2L translates into
 *       the boxes with children only (1); or L2L into every box (0).
 * Errors: XRL_E_INVALID_ARG (null plan, unknown key, bad value). */
#define XRL_TUNE_TS_KERNEL 0
#define XRL_TUNE_TS_MIN_COLS 1
#define XRL_TUNE_P2P_FORM 2
#define XRL_TUNE_TS_NARROW_COLS 3
#define XRL_TUNE_TS_ORDER 4
#define XRL_TUNE_L2L_FORM 5
#define XRL_TUNE_M2M_FORM 6
#define XRL_TUNE_LEAF_FORM 7
#define XRL_TUNE_VALU_FORM 8
#define XRL_TUNE_LEAF_L2L 9
xrl_status xrl_plan_set_tuning(xrl_plan *plan, int32_t key, int32_t value);

/* Graph mode (on != 0): the first xrl_fmm_matvec with a new argument set
 * (x, y, leading dimensions, column count, dtype, which epilogue terms are
 * present) runs eagerly, then captures its kernel sequence into a HIP graph
 * on a plan-owned stream; later calls with the same arguments replay it
 * with a single hipGraphLaunch on the caller's stream (the epilogue values
 * themselves may change between calls).  Profiling (xrl_plan_set_profiling)
 * bypasses the graph.  Errors: XRL_E_INVALID_ARG, XRL_E_HIP. */
xrl_status xrl_plan_set_graph(xrl_plan *plan, int32_t on);

/* Autotuner result: every form tried, in order, with its mean matvec time. */
typedef struct {
    int32_t n_tried;
    int32_t engine[8];    /* XRL_M2L_* of each form tried */
    int32_t ts_kernel[8]; /* XRL_TUNE_TS_KERNEL value of each form tried */
    double ms[8];         /* mean time of one matvec, milliseconds */
    int32_t best_engine, best_ts_kernel;
    double best_ms;
    int32_t n_p2p_tried;  /* P2P forms timed with the best translation form (0 when one applies) */
    double p2p_ms[3];     /* mean matvec time with XRL_TUNE_P2P_FORM = 0, 1, 2 */
    int32_t best_p2p_form;
} xrl_tune_result;

/* Times `reps` matvecs (after one warm-up) with each translation form that
 * applies to the plan's precision (MFMA plans: offset-stationary and the three
 * target-stationary forms; the vector-ALU plan has one form) on the caller's
 * arguments, keeps the fastest in the plan, then does the same for the three
 * P2P forms when more than 16 FP32 columns are carried.  y is overwritten.
 * The forms agree to rounding, so the choice only changes speed.
 * Errors: XRL_E_INVALID_ARG, XRL_E_STATE (not assembled), XRL_E_HIP. */
xrl_status xrl_plan_autotune(xrl_plan *plan, const void *x, int64_t ldx, int32_t n_cols, int32_t dtype, void *y,
                             int64_t ldy, int32_t reps, void *stream, xrl_tune_result *result);

/* Debug export of plan internals to host memory (tests):
 *   item 0: perm        int32 [n_elements] sorted position -> global panel
 *                       (both elements of a four-sided panel name the panel)
 *   item 1: box_range   int32 [n_boxes][2] element range [begin, end) per box
 *   item 2: box_level   int32 [n_boxes]
 *   item 3: near_rows   int32 [n_leaves+1] CSR over leaves into item 4
 *   item 4: near_src    int32 [n_near_rows] sorted source element per row
 *   item 5: m2l_pairs   int32 [n_m2l_pairs][2] (target box, source box)
 *   item 6: leaf_box    int32 [n_leaves]   box index of each leaf
 *   item 7: box_parent  int32 [n_boxes]
 *   item 8: near_values float64 [n_near_entries] (per leaf [rows][tpad])
 *   item 9: leaf_tpad   int32 [n_leaves]   padded target count of each leaf block
 *                                          (its targets rounded up to a multiple of 4)
 *   item 10: m2l_ratio  float64 [n_m2l_pairs] (r_t + r_s) / |c_t - c_s| of each
 *                       pair of item 5, in the same order
 * With buf == NULL only *nbytes is set. */
xrl_status xrl_plan_export(const xrl_plan *plan, int32_t item, void *buf, int64_t *nbytes);

/* Host-only: the FP64 M2L operator of the plan's translations for the
 * integer offset (ox, oy, oz) = (target centre - source centre) / h, order p
 * (2..12, even), written row-major to out[(p+1)^2][(p+1)^2] (real harmonic
 * coefficients, rows: local, columns: multipole).  It is the translation of
 * the FMM of Sec. II-C between same-level boxes.  Needs no device.
 * Errors: XRL_E_INVALID_ARG (null out, offset inside [-1,1]^3 or outside
 * [-3,3]^3), XRL_E_UNSUPPORTED (order). */
xrl_status xrl_m2l_operator(int32_t order, int32_t ox, int32_t oy, int32_t oz, double *out);

/* Self-test of the 16x16x4 MFMA operand layout used by the M2L kernel:
 * D[16][16] = A[16][4] * B[4][16], row-major host arrays of float
 * (elem_bytes = 4) or double (8).  Runs one wave on the current device. */
xrl_status xrl_selftest_mfma(int32_t elem_bytes, const void *A, const void *B, void *D);

/* Self-test of the 16-block 4x4x1 FP32 MFMA layout used for the columns
 * past the last full tile of the target-stationary translation: for each
 * block b, D[b][4][4] = A[b][4] (column) * B[b][4] (row); A, B: [16][4],
 * D: [16][4][4] row-major host float arrays.  One wave on the current device. */
xrl_status xrl_selftest_mfma_4x4(const float *A, const float *B, float *D);

/* ------------------------------------------------------------------ */
/* Iterative solve                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t iterations;  /* total inner iterations (max over right-hand sides) */
    int32_t restarts;
    int32_t converged;   /* number of right-hand sides that reached rtol */
    double max_rel_residual; /* max over right-hand sides of ||b - A x|| / ||b|| */
} xrl_gmres_stats;

/* Solve (beta_c * diag(A) + alpha_c * P) x_c = b_c for n_rhs complex columns
 * together (multiple right-hand sides share every FMM matvec; Sec. III:
 * restarted GMRES, restart 50, relative residual 1e-4 or 1e-6).  Arnoldi
 * orthogonalisation (classical Gram-Schmidt, twice) and the least-squares
 * update are FP64 whatever the plan's precision.
 *   b, x : device, [n_panels][n_rhs] complex of type dtype (XRL_C64 or
 *          XRL_C128), user panel order; x holds the initial guess on entry
 *          and the solution on exit.  Complex64 data is widened to complex128
 *          for the iteration (the Krylov basis is always FP64) and the
 *          solution rounded back to complex64.
 * The solver's operator applications never replay a captured graph (each
 * Arnoldi step hands over a new vector), whatever xrl_plan_set_graph says.
 * Errors: XRL_E_INVALID_ARG, XRL_E_STATE, XRL_E_NOT_CONVERGED (stats filled),
 *         XRL_E_HIP. */
xrl_status xrl_gmres_solve(const xrl_plan *plan, const xrl_epilogue *op, const void *b, void *x,
                           int32_t n_rhs, int32_t dtype, int32_t restart, double rtol, int32_t max_iter,
                           void *stream, xrl_gmres_stats *stats);

/* ------------------------------------------------------------------ */
/* Loop analysis around the panel operator                             */
/* ------------------------------------------------------------------ */
/* PEEC graph of a closed conforming triangle mesh (Sec. II-A, Fig. 1):
 * panel centroids are nodes, each edge shared by panels i < j is a branch
 * whose global current runs from i to j.  The centroid-midpoint maps
 * A_1..A_3 of Algorithm 1 (row = branch: rho_{i,e} = m_e - c_i at column i,
 * -rho_{j,e} at column j) and a loop basis M (Sec. II-B, eq. (7); rows of
 * +-1 per branch): one fan of panels around every mesh vertex except one per
 * connected surface, plus two loops per handle from a tree-cotree split of
 * the mesh; the loops span exactly the branch currents that conserve charge
 * at every panel (eq. (2)), N_loops = N_edges - N_panels + components.
 * The mesh (host arrays, same panel order as the plan it is used with) is
 * read during the call only.  Errors: XRL_E_INVALID_ARG, XRL_E_UNSUPPORTED
 * (an edge not shared by exactly two panels, a non-manifold vertex),
 * XRL_E_OOM, XRL_E_HIP. */
typedef struct xrl_loops xrl_loops;
typedef struct {
    int64_t n_panels, n_edges, n_loops;
    int64_t n_vertex_loops, n_global_loops, n_components;
    int64_t nnz_loop_matrix;
} xrl_loops_info;
xrl_status xrl_loops_build(const xrl_mesh_desc *mesh, void *stream, xrl_loops **out);
void xrl_loops_destroy(xrl_loops *loops);
xrl_status xrl_loops_get_info(const xrl_loops *loops, xrl_loops_info *info);
/* Host copies (int32): item 0 the panels (i, j) of each branch [N_edges][2];
 * item 1 the mesh vertices of each branch [N_edges][2]; item 2 the loop
 * matrix as (loop, branch, sign) triples.  buf == NULL: only *nbytes. */
xrl_status xrl_loops_export(const xrl_loops *loops, int32_t item, void *buf, int64_t *nbytes);

/* Surface impedance of eq. (3) (double-plane model, Sec. II-A) at n
 * frequencies (Hz, > 0) for conductivity sigma (S/m) and thickness (m):
 * zs[2 i], zs[2 i + 1] = Re, Im Z_s(freq[i]).  Host only. */
xrl_status xrl_surface_impedance(double sigma, double thickness, const double *freq, int32_t n, double *zs);

/* Branch-space operator of eq. (5)-(6), V_edge = sum_t A_t (beta area +
 * alpha P) A_t^T I_edge, for n_cols columns (alpha_c = j omega mu0 / 4 pi,
 * beta_c = Z_s per column from op; NULL terms as in xrl_epilogue).  The
 * product with P runs through xrl_fmm_matvec on 3 n_cols columns, so the
 * plan (built on the same mesh) needs max_cols >= 3 n_cols.
 *   i_edge, v_edge : device, [N_edges][n_cols] complex128.
 * Errors: XRL_E_INVALID_ARG, XRL_E_STATE, XRL_E_HIP. */
xrl_status xrl_edge_matvec(const xrl_loops *loops, const xrl_plan *plan, const xrl_epilogue *op, const void *i_edge,
                           void *v_edge, int32_t n_cols, void *stream);

/* Solve the loop system eq. (8), M (sum_t A_t (beta area + alpha P) A_t^T)
 * M^T I_l = M V_edge, for n_rhs columns sharing every FMM matvec (restarted
 * GMRES, FP64 Arnoldi as in xrl_gmres_solve), and return the branch
 * currents I_edge = M^T I_l.
 *   v_edge, i_edge : device, [N_edges][n_rhs] complex128.
 *   precond: XRL_PRECOND_NONE, XRL_PRECOND_DIAG_P (eq. (10): M sum_t A_t
 *   (beta area + alpha P_d) A_t^T M^T with P_d the diagonal of P, applied
 *   from the right as in eq. (11)) or XRL_PRECOND_DIAG_L (the surface part
 *   plus the diagonal of the branch interaction matrix sum_t A_t P A_t^T).
 *   The preconditioner is factored once per column by the library's own
 *   sparse LDL^T (reverse Cuthill-McKee envelope, host) in place of a
 *   vendor solver; its entries of P come from the assembled near field.
 * Errors: XRL_E_INVALID_ARG, XRL_E_STATE, XRL_E_NOT_CONVERGED (stats
 * filled), XRL_E_HIP. */
#define XRL_PRECOND_NONE 0
#define XRL_PRECOND_DIAG_P 1
#define XRL_PRECOND_DIAG_L 2
xrl_status xrl_loop_gmres_solve(const xrl_loops *loops, const xrl_plan *plan, const xrl_epilogue *op,
                                const void *v_edge, void *i_edge, int32_t n_rhs, int32_t precond, int32_t restart,
                                double rtol, int32_t max_iter, void *stream, xrl_gmres_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* XRL_H */
