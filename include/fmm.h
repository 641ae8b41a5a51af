/*
 * fmm.h - C ABI of the MI355X (gfx950) DA-FMM library, libfmm_mi355x.so.
 *
 * The library computes, for N point charges q_i at positions r_i, the Coulomb
 * potential phi_i = sum_{j != i} q_j / |r_i - r_j| (left-hand side of the
 * paper's Eq. P2M_phi, no physical constant) and, on request, the field
 * E_i = -grad phi_i = sum_{j != i} q_j (r_i - r_j) / |r_i - r_j|^3, with the
 * differential-algebra fast multipole method of Zhang, arXiv 2508.02626:
 * Taylor (DA) multipole expansions in d = r / r^2 (Sec. 2.1), translated by
 * M2M (Sec. 2.2), converted by M2L (Sec. 2.3), P2L (Sec. 2.4), shifted by
 * L2L (Sec. 2.5), evaluated by L2P / M2P (Sec. 3.2), with the near field
 * summed pairwise (Sec. 1).  Pairs at distance zero contribute nothing.
 *
 * Conventions for every entry point
 *  - Pointers named *_dev are device pointers of the current HIP device;
 *    pointers named *_host are host pointers.  Arrays are contiguous, FP64,
 *    in the caller's (original) particle order; positions are [n][3].
 *  - All device work is enqueued on the stream argument (0 = null stream) and
 *    is asynchronous unless stated; the caller keeps inputs alive and outputs
 *    untouched until the stream has passed the call.
 *  - The plan copies what it needs from xyz_dev and never keeps the caller's
 *    pointers.  It owns its workspace (tree, lists, sorted particles,
 *    expansions), allocated through the caller's allocator or, when none is
 *    given, with stream-ordered hipMallocAsync, and released by
 *    fmm_plan_destroy.
 *  - Every function returns FMM_OK or a negative status; arguments are
 *    validated before anything is enqueued.  No function aborts or prints;
 *    fmm_last_error() gives the calling thread's last message.
 *  - Calls on different plans may run concurrently on different streams.
 *    Concurrent calls on one plan must be ordered by the caller.
 */
#ifndef FMM_MI355X_H
#define FMM_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FMM_OK = 0,
    FMM_EINVAL = -1,        /* invalid argument (also non-finite coordinates) */
    FMM_ENOMEM = -2,        /* device or host allocation failed              */
    FMM_EDEVICE = -3,       /* a HIP call failed; see fmm_last_error()        */
    FMM_EUNSUPPORTED = -4   /* valid but not supported by this build          */
};

/* Precision of the evaluation (fmm_options_t.precision): a set of parts run
 * in FP32; everything not named stays FP64.  FMM_MIXED is both. */
enum {
    FMM_FP64 = 0,
    FMM_P2P_F32 = 1,   /* P2P pair terms in FP32, compensated (Kahan) FP32 sum
                          per target and source range, FP64 combination       */
    FMM_M2L_F32 = 2,   /* M2L contraction on FP32 MFMA: all of it at orders
                          <= 8, the rows of higher degree (all but the first
                          16 of each parity class) from order 12; orders 9-11
                          keep M2L in FP64                                    */
    FMM_MIXED = 3
};

typedef struct fmm_plan_s *fmm_plan_t;

/* Optional stream-ordered allocator (e.g. a framework's caching allocator).
 * alloc returns NULL on failure; free must accept what alloc returned. */
typedef struct {
    void *(*alloc)(size_t bytes, hipStream_t stream, void *ctx);
    void (*free)(void *ptr, hipStream_t stream, void *ctx);
    void *ctx;
} fmm_allocator_t;

typedef struct {
    int32_t uniform_depth; /* >= 0: full octree of this depth (leaf_size unused);
                              -1: adaptive octree, a box with more than
                              leaf_size particles is subdivided (Sec. 3.5)    */
    int32_t max_depth;     /* adaptive depth cap, 1..21 (default 21)          */
    int32_t precision;     /* FMM_FP64, or a combination of FMM_P2P_F32 and
                              FMM_M2L_F32 (FMM_MIXED: both)                   */
    int32_t want_field;    /* nonzero: fmm_evaluate may be given a field array */
    const double *root;    /* host {lo_x, lo_y, lo_z, W} of the root cube, or
                              NULL for the bounding cube of the points        */
    int32_t m2l_method;    /* FMM_M2L_SIGN_CLASS (default): the derivative-
                              tensor contraction on the matrix cores, shared by
                              the offsets of a sign class; FMM_M2L_ROTATION:
                              the axis-rotation form of Sec. 3.4 on the vector
                              unit (rotate, one-variable axial map, rotate
                              back; FP64 whatever the precision)              */
    int32_t kernel;        /* FMM_KERNEL_COULOMB (default): phi_i = sum q_j /
                              |x_i - x_j|.  FMM_KERNEL_SOFTENED: the softened
                              (Plummer) kernel 1/sqrt(|x|^2 + eps^2), a second
                              non-oscillatory kernel (the DA formulation is not
                              tied to 1/r: closing remark of Sec. 3.4); every
                              j != i contributes, also at distance 0 when
                              eps > 0.  Softened plans use full Cartesian
                              Taylor expansions (the kernel is not harmonic, so
                              there is no fold) on uniform or adaptive trees,
                              need FMM_FP64, order <= 10 and the sign-class
                              M2L method, and are evaluated by fmm_evaluate
                              only                                            */
    double softening;      /* eps >= 0, in the units of the coordinates
                              (softened kernel only)                          */
} fmm_options_t;

enum { FMM_M2L_SIGN_CLASS = 0, FMM_M2L_ROTATION = 1 };
enum { FMM_KERNEL_COULOMB = 0, FMM_KERNEL_SOFTENED = 1 };

/* Default options: adaptive, max_depth 21, FP64, field on, bounding cube,
 * sign-class M2L, Coulomb kernel. */
void fmm_default_options(fmm_options_t *opt);

/*
 * fmm_plan - build the octree and interaction lists for n points.
 *   xyz_dev    [n][3] FP64 device positions (read during the call only)
 *   n          number of points, 1 <= n < 2^31
 *   order      truncation order p of the DA vectors, 0..16 (Sec. 3, "order")
 *   leaf_size  s >= 1 for adaptive trees (Sec. 3.5); ignored for uniform trees
 *   opt        options, or NULL for fmm_default_options
 *   alloc      allocator, or NULL for hipMallocAsync on `stream`
 *   stream     HIP stream for all device work
 *   out        receives the plan handle on success (untouched on failure)
 * Waits once for `stream` to learn tree and list sizes (the points have been
 * read by then); the last build steps are still enqueued on `stream` when the
 * call returns: later work on `stream` follows them, and evaluations and
 * exports on other streams wait for them (an event of the plan).  Returns
 * FMM_EINVAL for invalid arguments or non-finite coordinates, FMM_EUNSUPPORTED when the
 * tree has so many boxes that its folded multipoles (order >= 6: boxes + 1
 * rows of 16 ceil(k / 4) doubles, k the M2L k-steps, 24 at order 8) reach
 * 4 GiB.
 */
int fmm_plan(const double *xyz_dev, int64_t n, int32_t order, int32_t leaf_size,
             const fmm_options_t *opt, const fmm_allocator_t *alloc, hipStream_t stream,
             fmm_plan_t *out);

/*
 * fmm_plan_batch - build `count` independent plans (the many-small-problems
 * case of Sec. 1's recipe applied to each problem).  Arrays of length count:
 * xyz_dev[i] [n[i]][3] device coordinates, order[i], leaf_size[i]; opts is
 * NULL (defaults for all) or an array of count options.  With no allocator
 * the plans are built concurrently by up to `threads` host threads, each on a
 * stream of its own that first waits for the work already enqueued on
 * `stream`; with an allocator they are built one after the other on `stream`.
 * On return every plan is complete and behaves as one built by fmm_plan on
 * `stream` (destroy is ordered on `stream`).  On failure no plan is returned
 * (out[] is all NULL) and the status and message of the first failing plan
 * are reported.
 */
int fmm_plan_batch(int32_t count, const double *const *xyz_dev, const int64_t *n,
                   const int32_t *order, const int32_t *leaf_size, const fmm_options_t *opts,
                   const fmm_allocator_t *alloc, hipStream_t stream, int32_t threads,
                   fmm_plan_t *out);

/*
 * fmm_evaluate - potentials (and fields) for charges q.
 *   q_dev      [n] FP64 device charges, original order
 *   phi_dev    [n] FP64 device output potentials
 *   field_dev  [n][3] FP64 device output fields E = -grad phi, or NULL
 * Asynchronous on `stream`: P2P runs on a stream of the plan's own, in two
 * parts forked from `stream` (after the charges are sorted, after M2L) and
 * joined back (before M2L, before the output), so that it overlaps the
 * upward and downward passes; M2P (W lists) follows the second part there.
 * Deterministic: the
 * same plan and charges give bitwise identical results on every call.
 * Softened-kernel plans (full expansions) run P2P's parts beside the upward
 * pass and the downward pass (P2L, L2L), M2P after the second part; their
 * M2L runs alone.
 */
int fmm_evaluate(fmm_plan_t plan, const double *q_dev, double *phi_dev, double *field_dev,
                 hipStream_t stream);

/*
 * fmm_evaluate_batch - evaluate `count` independent plans, packing the work
 * of all of them into shared launches (one launch per pipeline stage instead
 * of one per stage and plan).  Arrays of length count; field[i] may be NULL.
 * Plans may differ in n, order and precision.  Each result is bitwise equal to
 * fmm_evaluate on the same plan alone.  Softened-kernel plans are refused
 * (FMM_EINVAL): they have their own pipeline, run by fmm_evaluate.
 */
int fmm_evaluate_batch(fmm_plan_t const *plans, const double *const *q_dev,
                       double *const *phi_dev, double *const *field_dev, int32_t count,
                       hipStream_t stream);

/*
 * fmm_evaluate_batch_noalloc - fmm_evaluate_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, same results (bitwise
 * equal to fmm_evaluate_batch and to fmm_evaluate on each plan).  Where
 * fmm_evaluate_batch allocates, on every call, device memory for the per-plan
 * views its kernels read, this call stages them in a fixed array of the
 * library: FMM_NOALLOC_MAX_PLANS views (a few hundred bytes each), one copy
 * per device, held until the process ends.  It calls no hipMalloc, hipFree or
 * other allocating routine.
 *   count  0..FMM_NOALLOC_MAX_PLANS (FMM_EINVAL beyond)
 * Every call on a device shares that device's array and leaves its last
 * contents there: calls on one stream are ordered and safe, but calls that
 * overlap on one device (different streams, or threads without ordering)
 * race and give wrong results.  All plans must belong to the current device.
 * The first evaluation of a plan on a stream may still create a HIP event,
 * and a plan's first evaluation its side stream.
 */
#define FMM_NOALLOC_MAX_PLANS 1024
int fmm_evaluate_batch_noalloc(fmm_plan_t const *plans, const double *const *q_dev,
                               double *const *phi_dev, double *const *field_dev, int32_t count,
                               hipStream_t stream);

/* Device bytes held by the plan (its workspace, as allocated: a chunk reused
 * from the library's cache counts with its full size), for admission control. */
int fmm_plan_footprint(fmm_plan_t plan, size_t *bytes);

/* Device bytes the library keeps on `device` outside any plan: chunks of
 * destroyed plans cached for reuse by later plans (at most 8 GiB per device;
 * returned to the device when an allocation fails).  Plans built without a
 * caller allocator also draw on HIP's default memory pool, which is set to
 * keep freed memory for reuse. */
int fmm_cached_bytes(int device, size_t *bytes);

/* Predicted device bytes of a plan before building it (upper bound used for
 * admission: tree, lists and expansions for n points at this order). */
int fmm_plan_estimate(int64_t n, int32_t order, int32_t leaf_size,
                      const fmm_options_t *opt, size_t *bytes);

/* Sizes of the plan: out[0]=boxes, [1]=|U|, [2]=|V|, [3]=|W|, [4]=|X|,
 * [5]=deepest level, [6]=key depth D, [7]=n, [8]=order, [9]=coefficients per
 * expansion (p+1)(p+2)(p+3)/6. */
int fmm_plan_sizes(fmm_plan_t plan, int64_t out[10]);

/*
 * fmm_plan_export_tree - copy the tree to host buffers (any may be NULL).
 *   root_host[4]  {lo_x, lo_y, lo_z, W}
 *   perm_host[n]  sorted position -> original index (particles sorted by
 *                 (Morton key, original index))
 *   per box (boxes in (level, Morton code) order): level, morton, first
 *   particle (sorted position), count, parent (-1 for the root), first child
 *   (-1 if none), number of children
 *   lists as CSR over boxes: *_off[boxes+1] (int64), *_src[|list|] (int32),
 *   sources of each box ascending; U (P2P), V (M2L), W (M2P), X (P2L).
 * Synchronous (waits for `stream`).
 */
int fmm_plan_export_tree(fmm_plan_t plan, hipStream_t stream, double *root_host,
                         int64_t *perm_host, int32_t *level_host, uint64_t *morton_host,
                         int64_t *first_host, int64_t *count_host, int32_t *parent_host,
                         int32_t *child_begin_host, int32_t *nchild_host,
                         int64_t *U_off_host, int32_t *U_src_host, int64_t *V_off_host,
                         int32_t *V_src_host, int64_t *W_off_host, int32_t *W_src_host,
                         int64_t *X_off_host, int32_t *X_src_host);

/*
 * fmm_plan_export_expansions - copy the multipole (M) and local (L) expansions
 * of the last fmm_evaluate to host buffers [boxes][(p+1)(p+2)(p+3)/6], in the
 * paper's DA convention: M holds the Taylor coefficients of phi_M in
 * d = r/r^2 about the box centre (Eq. P2M), L those of phi_L in d' = r - c
 * (Eq. P2L); monomials ordered by degree, then descending exponents of d1, d2
 * (Table 1).  Either pointer may be NULL.  Synchronous.  Leaves' M are the
 * P2M results; parents' M are rebuilt from the folded (harmonic) multipoles
 * the evaluation's M2M produced (levels 0 and 1, which the evaluation does
 * not need, are completed by the same M2M first); L of boxes at level >= 2
 * are unfolded from the harmonic local expansions after the L2L (zero above).
 * Softened-kernel plans hold Cartesian Taylor expansions instead: M the
 * moments M_a = sum_i q_i (c - x_i)^a / a! (phi = sum_a M_a d^a K(x - c)), L
 * the Taylor coefficients of the local expansion in x - c, in the same
 * monomial order (levels 0 and 1 of M completed as above, L zero there).
 */
int fmm_plan_export_expansions(fmm_plan_t plan, hipStream_t stream, double *M_host,
                               double *L_host);

/*
 * Stage timing of fmm_evaluate.  With timing on, every fmm_evaluate on the
 * plan brackets each stage with HIP events on the stream it runs on.
 * fmm_plan_read_timing waits for the recorded events, adds their durations
 * (milliseconds) per stage into ms[0..15] and the number of timed evaluations
 * into calls[0..15], and clears the records.  Stages: 0 permute charges,
 * 1 P2M raw moments, 2 M2M, 3 folded multipoles of the leaves (and full
 * ones of M2P sources), 4 M2L, 5 P2L, 6 unfold, 7 L2L, 8 L2P+output,
 * 9 and 10 the two parts of P2P and 11 M2P (on the plan's side stream,
 * concurrent with stages 1-3 and 5-7 respectively).
 */
int fmm_plan_set_timing(fmm_plan_t plan, int on);
int fmm_plan_read_timing(fmm_plan_t plan, double ms[16], int64_t calls[16]);

/*
 * fmm_order_table - copy one of the per-order constant tables, built on the
 * host from closed forms in long double exactly as the device tables are
 * (for tests of the closed forms; no device is touched).  Scaled units:
 * Mhat_a = w_|a| M_a / h^|a| with w_n = (-1)^n / (2n-1)!!, Lhat_b = b! L_b
 * h^(|b|+1), h the box width; monomials in the DA order of Table 1
 * (n_p = (p+1)(p+2)(p+3)/6 of them).
 *   which 0  derivative tables: [343][ld], offset k = (kx, ky, kz) in
 *            {-3..3}^3 at row (kx+3)*49 + (ky+3)*7 + (kz+3) (rows of the 27
 *            near offsets are zero); entry e of a row runs over z = 0..2,
 *            then i = 0.., then j = 0.. with i + j + z <= 2p, holding
 *            d^(i,j,z) (1/|x|) at x = k (Eq. m2l's derivatives of 1/r)
 *         1  M2M (Sec. 2.2): [8][n_p][n_p], S[o][a][b] = d Mhat'_b / d Mhat_a
 *            from the child of octant o (bits x, y, z: child centre above
 *            the parent's) to its parent, on harmonic multipoles
 *         2  L2L (Sec. 2.5): [8][n_p][n_p], G[o][g][b] = d Lhat'_b / d Lhat_g
 *            from a parent to its child of octant o
 *         3  P2M (Sec. 2.1, 3.1): [n_p][n_p], Mhat_a = sum_g P[g][a] Q_g with
 *            the raw moments Q_g = sum q u^g, u = (x - c)/h
 *         4  harmonic reconstruction: [(p+1)^2][n_p], the full harmonic Mhat
 *            from its components with z exponent <= 1 (harmonic order:
 *            degree n holds (i, n-i, 0) for i = n..0, then (i, n-1-i, 1))
 *         5  rotation-based M2L (Sec. 3.4), multipole side: [64][S] per class
 *            of offsets (|k_x|, |k_y|, |k_z|) at row |k_x| 16 + |k_y| 4 + |k_z|
 *            (rows of the near offsets zero), S = sum_n (2n+1)^2: per degree n
 *            a (2n+1)^2 block [folded component][mode], the map from the
 *            folded multipole to azimuthal mode coordinates about the offset
 *            (mode index 0 for m = 0, 2m - 1 + t for m > 0, t = 0 cos, 1 sin)
 *         6  local side: [64][S], per degree a block [mode][folded component]
 *         7  axial map: [distinct |k|^2][sum_m (p+1-m)^2], per m = 0..p a
 *            block [n - m][l - m] coupling mode m of multipole degree n to
 *            local degree l (the same for cos and sin)
 *         8  [64] the axial block of each class (-1 for near offsets)
 *            For a sign vector s, T(s o k) = R_s T(k) R_s, R_s = +-1 by the
 *            parities of a folded component's exponents; T(k) = B A F.
 *         9  layout of a folded multipole row: [1][ldmh], the component (index
 *            in the harmonic order of table 4) kept at each position, -1 for
 *            padding.  From order 6: the components sorted by parity class
 *            (x, y, z exponent parities, class 4 (x mod 2) + 2 (y mod 2) + z),
 *            each class padded to a multiple of 4 (one k-step of the
 *            matrix-core contraction); sorted column 4 s + g (k-step s, lane
 *            group g) sits at 8 (s / 2) + 2 g + (s mod 2), so that a lane's
 *            operands of two k-steps are adjacent; ldmh = 16 ceil(k / 4) for k
 *            k-steps.  Below order 6: the harmonic order, padded to 16.
 *   out_host   host buffer of `capacity` doubles, or NULL to query the size
 *   count      receives the number of doubles; ld the row length
 * Returns FMM_EINVAL for a bad order, table or a buffer too small.
 */
int fmm_order_table(int32_t order, int32_t which, double *out_host, int64_t capacity, int64_t *count,
                    int32_t *ld);

/* Release the plan.  Stream-ordered on the plan's build stream: memory is
 * returned after work already enqueued there, and the latest evaluation on
 * every other stream that evaluated the plan, have finished. */
int fmm_plan_destroy(fmm_plan_t plan);

/* Message of the calling thread's last failed call ("" if none). */
const char *fmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
