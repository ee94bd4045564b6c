/*
 * h2.h -- C ABI of the MI355X (gfx950) library for the data-driven H^2
 * construction of Cai, Huang, Chow and Xi (arXiv 2206.01885).
 *
 * The calls follow the paper's statement of the problem (Algorithm 2): the
 * input is a point set X, a kernel function kappa, an approximation tolerance
 * eps, a separation ratio tau and a leaf capacity q; the output is the H^2
 * representation (bases U, transfer matrices R, coupling blocks B and the
 * dense nearfield), which is then applied to vectors, y = Ktilde x.
 *
 * All numerical work of h2_build / h2_matvec runs in the library's HIP
 * kernels on the current device.  Pointers marked "device" must be device
 * memory of that device; pointers marked "host" are host memory.
 *
 * Thread safety: a handle must not be used by two calls at once; distinct
 * handles are independent.  Every non-OK status leaves a message readable with
 * h2_last_error() (thread-local).
 */
#ifndef H2_MI355X_H
#define H2_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_handle_s *h2_handle;

typedef enum {
    H2_OK = 0,
    H2_EINVAL = -1,       /* invalid argument (sizes, tolerance, non-finite points, ...) */
    H2_ENOMEM = -2,       /* device memory exhausted (H2_DEVICE_MEMORY_CAP=<bytes> in the
                             environment caps what the library takes, to test this) */
    H2_EDEVICE = -3,      /* HIP runtime error */
    H2_EUNSUPPORTED = -4, /* valid request outside what the library implements */
    H2_EINTERNAL = -5     /* internal consistency check failed */
} h2_status;

/* Kernel functions (Section 2 and Table 1 of the paper); params[0] is the
 * bandwidth h or the length scale l:
 *   H2_COULOMB      1/|x-y|, with kappa(x,x) = 0
 *   H2_GAUSSIAN     exp(-|x-y|^2 / h^2)
 *   H2_EXPONENTIAL  exp(-|x-y| / l)
 *   H2_MATERN32     (1 + sqrt(3)|x-y|/l) exp(-sqrt(3)|x-y|/l)
 *   H2_BUMP         exp(-1 / (1 - a|x-y|^2)), a = params[0] (kappa_4 of the
 *                   paper's Table 1, where a = 0.1); defined where
 *                   a|x-y|^2 < 1, which the caller's points must satisfy
 *                   (the formula is evaluated as written)
 *   H2_COSINE       cos(a x.y), a = params[0] (kappa_3 of Table 1, a = 1);
 *                   not a function of |x-y|, so the calibration of r1, r2
 *                   does not apply: options.r1 and options.r2 must be set
 *                   (H2_EINVAL otherwise)
 *   H2_ADVECTION    exp(a((x-y)_0 - |x-y|)) / |x-y|, a = params[0] > 0, 0 at
 *                   x = y: the Green's function of steady advection-diffusion
 *                   with the drift along axis 0 (not in the paper).  Not
 *                   symmetric: the build keeps a column basis V, W of its own
 *                   (Algorithm 2, getBasis on K(Y_i*, Xbar_i)^T) beside U, R.
 *                   Not a function of |x-y| either: options.r1 and
 *                   options.r2 must be set (H2_EINVAL otherwise)          */
typedef enum {
    H2_COULOMB = 0,
    H2_GAUSSIAN = 1,
    H2_EXPONENTIAL = 2,
    H2_MATERN32 = 3,
    H2_BUMP = 4,
    H2_COSINE = 5,
    H2_ADVECTION = 6
} h2_kernel_id;

/* Build options (h2_options_default fills the defaults).
 *   tau            separation ratio of Eq. (separation), 0 < tau < 1; default 0.7
 *   r1, r2         the maximum sizes of X_i^* and Y_i^* (Algorithm 1).  The
 *                  volume DataReduct samples X_i^*'s list with a grid of at
 *                  most r1 points and each of the two parts of Y_i^*'s list
 *                  (Y_p^* and the interaction-list part) with a grid of at
 *                  most r2/2 points.  0 = choose them from the tolerance
 *                  (Section 4.2: r1 = r, r2 = 2 r); > 0 = use as given
 *                  (r1 <= 2048, 2 <= r2 <= 4096)
 *   r_min          0, or a lower bound applied to the calibrated r (so r1 >=
 *                  r_min and r2 >= 2 r_min when they are chosen from the
 *                  tolerance)
 *   precision      64: FP64 throughout; 32: the coupling and nearfield blocks,
 *                  the apply and its vectors in FP32 (FP32 products per block,
 *                  compensated accumulation of the block products, FP64
 *                  interpolation sums); the tree, HiDR and the interpolative
 *                  decompositions stay FP64
 *   store_coupling 1: store the coupling and nearfield blocks (default);
 *                  0: store the nearfield blocks only; h2_matvec evaluates
 *                  each coupling block entry where it multiplies (no B in
 *                  memory: about 180 GB less at n = 2^20, at the cost of the
 *                  kernel evaluations in every apply); precision 64 only
 *                  (H2_EUNSUPPORTED otherwise)
 *   calib_seed     seed of the random points used to choose r1, r2
 *   profile        1: h2_matvec records HIP events around each of its sweeps on
 *                  its stream, and the build around its launches of the
 *                  interpolative decompositions and of the top-down
 *                  DataReduct; h2_query then reports the last apply's and the
 *                  build's times
 *   datareduct     DataReduct method of HiDR (Section 3.3): H2_DR_VOLUME
 *                  (default; the reference set is a tensor grid), H2_DR_FPS
 *                  (farthest point sampling from the list's first point; a
 *                  set gets at most r1 / r2 points) or H2_DR_SURFACE (the
 *                  reference set lies on three ellipsoids around each part
 *                  of the list, semi-axes 0.3, 0.6 and 1.2 times the part's
 *                  bounding-box widths).  The choice of r1, r2 from the
 *                  tolerance always uses the volume method.
 *   srrqr_f        0 (default): getBasis is the column-pivoted QR alone;
 *                  f > 1 (and <= 1e6): strong rank-revealing swaps follow it,
 *                  so that the interpolation matrix G of Eq. (SRRQR1) has
 *                  max |G| <= f (the rank stays the pivoted QR's)         */
enum { H2_DR_VOLUME = 0, H2_DR_FPS = 1, H2_DR_SURFACE = 2 };
typedef struct {
    double tau;
    int r1, r2;
    int precision;
    int store_coupling;
    uint64_t calib_seed;
    int profile;
    int r_min;
    int datareduct;
    double srrqr_f;
} h2_options;

void h2_options_default(h2_options *opt);

/* h2_build: Algorithm 2 of the paper.
 *   points     device, FP64, SoA layout [dim][n] (points[k*n + i] is
 *              coordinate k of point i), original order.  Read during the
 *              call only; the library keeps its own permuted copy.
 *   n          number of points, n >= 1 (and n < 2^31)
 *   dim        1, 2 or 3
 *   kernel_id  an h2_kernel_id
 *   params     host, params[0] = bandwidth / length scale (ignored for Coulomb,
 *              may then be NULL); must be finite and > 0 when used
 *   tol        approximation tolerance eps, 0 < tol < 1
 *   leaf_size  maximum number of points q of a leaf, >= 1
 *   out        receives the handle; set to NULL on failure (nothing leaks)
 * The call synchronises the current stream (level sizes are read back).   */
h2_status h2_build(const double *points, int64_t n, int dim, int kernel_id, const double *params,
                   double tol, int leaf_size, h2_handle *out);

/* As h2_build, with options (NULL = defaults) and a HIP stream (NULL = the
 * default stream) on which all work is ordered.                          */
h2_status h2_build_ex(const double *points, int64_t n, int dim, int kernel_id, const double *params,
                      double tol, int leaf_size, const h2_options *opt, void *hip_stream, h2_handle *out);

/* h2_build_batched: Algorithm 2 for nprob independent problems in one call.
 * Each problem is built exactly as h2_build_ex would build it alone (same
 * tree, lists, r1/r2, HiDR, bases and blocks), but two steps run over all
 * problems together: the choice of r1, r2 (Section 4.2; identical
 * calibration sets of different problems are evaluated once, and all sets
 * share each round's launches), and the nested-basis step -- kernel-block
 * evaluation and pivoted-QR ID of Section 4.1 -- level by level: round t
 * takes depth maxdepth_p - t of every problem p, and all its nodes go into
 * one batched launch.
 *   points     host array of nprob device pointers, each as in h2_build
 *   n, dim, kernel_id, tol, leaf_size   host arrays [nprob], as in h2_build
 *   params     host array [nprob]: params[p] is problem p's params[0]
 *              (ignored for Coulomb)
 *   opt        options shared by all problems (NULL = defaults)
 *   hip_stream stream of all work and of the returned handles (NULL = default)
 *   out        host array [nprob] of handles; all NULL on failure, and the
 *              message of h2_last_error() names the problem that failed a check.
 * Synchronises the stream.                                                */
h2_status h2_build_batched(int nprob, const double *const *points, const int64_t *n, const int *dim,
                           const int *kernel_id, const double *params, const double *tol, const int *leaf_size,
                           const h2_options *opt, void *hip_stream, h2_handle *out);

/* h2_rebuild: the representation of another kernel, kernel parameter or
 * tolerance on the same points, from the representor sets already computed
 * (Section 6, "HiDR once for all": HiDR depends on the points only, so a
 * kernel family -- e.g. the bandwidths of a Gaussian-process search -- needs
 * it once).  Keeps the tree, the lists, r1, r2 and every X_i^*, Y_i^*;
 * recomputes Algorithm 2 from the kernel blocks on: interpolative
 * decompositions, skeletons, coupling and nearfield blocks.  The result is
 * what h2_build_ex would return for the new kernel and tolerance with the
 * options r1, r2 set to this handle's values (r1, r2 are not recalibrated
 * for the new kernel).
 *   h          a built handle; its previous bases and blocks are replaced
 *   kernel_id, params, tol   as in h2_build
 * Waits for the handle's last apply; synchronises its stream.  On failure
 * the handle is left unusable for h2_matvec (h2_destroy still works).     */
h2_status h2_rebuild(h2_handle h, int kernel_id, const double *params, double tol);

/* h2_matvec: y = Ktilde x, the product of the H^2 representation with x
 * (Section 2.1: the O(n) apply of a matrix with nested bases -- upward pass
 * through the column bases and transfer matrices, coupling blocks of the
 * interaction lists, downward pass through the row bases, dense nearfield
 * blocks; Section 6 measures the construction by this product's error
 * ||K z - Ktilde z|| / ||z||).
 *   h      a built handle (h2_build*, h2_rebuild); H2_EINVAL if NULL or not
 *          ready (a failed h2_rebuild)
 *   x, y   device, [nrhs][n] (x[r*n + i] is entry i of right-hand side r),
 *          original point order; FP64 (double) for a handle built with
 *          precision 64, FP32 (float) for precision 32; must not overlap
 *   nrhs   number of right-hand sides, 1 <= nrhs <= 256
 * Stream-ordered on the handle's stream; returns without synchronising
 * except on the first call with a larger nrhs (workspace allocation).    */
h2_status h2_matvec(h2_handle h, const void *x, void *y, int nrhs);
h2_status h2_matvec_ex(h2_handle h, const void *x, void *y, int nrhs, void *hip_stream);

/* h2_matvec_noalloc: h2_matvec_ex for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, same kernels and the same result bit
 * for bit, but the apply's work vectors -- x and y in tree order and the
 * node coefficients, (2 n + sum of ranks of both bases) * ceil(nrhs/32)*32
 * values -- live in one array of H2_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds until the process ends; the call allocates nothing and
 * records no profile events.  H2_EUNSUPPORTED if the work vectors do not
 * fit (the message gives the bytes needed).  Every call on one GPU uses that
 * GPU's array: calls that overlap on one GPU (other streams, other threads,
 * other handles) race and must be ordered by the caller.  The device must be
 * the handle's and current.                                              */
#define H2_NOALLOC_SCRATCH_BYTES ((int64_t)1 << 28)
h2_status h2_matvec_noalloc(h2_handle h, const void *x, void *y, int nrhs, void *hip_stream);

/* Summary of a built representation (all host values). */
typedef struct {
    int64_t n;
    int dim, kernel_id;
    int nnode, maxdepth, nleaf;
    int r1, r2;
    int64_t nnz_il, nnz_near; /* interaction-list and near-list entries */
    int max_rank;
    int64_t sum_rank;
    int64_t bytes_U, bytes_B, bytes_D; /* stored interpolation, coupling, nearfield */
    int precision;
    double t_tree, t_lists, t_calib, t_hidr, t_basis, t_blocks; /* seconds */
    /* last h2_matvec with options.profile = 1 (milliseconds, HIP events on the
     * apply's stream; h2_query waits for that apply to finish); 0 otherwise */
    double mv_gather, mv_upward, mv_coupling, mv_downward, mv_leaves, mv_scatter;
    int mv_nrhs;
    /* build with options.profile = 1: HIP-event time (ms) of the launches of
     * the interpolative decompositions (all, and the one for nodes with more
     * than 64 candidate columns; launches of h2_build_batched are shared by
     * all its problems), and the algorithmic floating-point operations of
     * this handle's decompositions (pivoted QR to the rank found and the
     * solve for T); 0 otherwise */
    double id_ms, id_wide_ms, id_flops, id_wide_flops;
    /* build with options.profile = 1 and the volume DataReduct: HIP-event
     * time (ms) of the box-pruned top-down DataReduct launches of HiDR, and
     * the bytes of the candidate coordinates they reduce (each farfield list
     * T_i counted once); 0 otherwise */
    double hidr_down_ms, hidr_down_bytes;
    /* column basis V, W: 1 when the kernel is not symmetric and V, W are
     * built apart from U, R (max_rank, sum_rank and bytes_U describe U, R;
     * these describe V, W and equal them for a symmetric kernel, except
     * bytes_V = 0 there) */
    int nonsymmetric, max_rank_v;
    int64_t sum_rank_v, bytes_V;
    /* with hidr_down_ms: the squared distances the definition of the
     * top-down DataReduct evaluates (every reference point against every
     * candidate of T_i); the box-pruned search evaluates fewer */
    double hidr_down_evals;
} h2_info;

h2_status h2_query(h2_handle h, h2_info *info);

/* h2_export: copy one internal array to host memory for inspection and
 * parity tests.  `what` selects the array (H2_EXP_*); for the per-node
 * variable-length lists, `node` selects the node, otherwise it is ignored.
 * Point indices are tree positions (perm maps them to original indices).
 * If host_buf is NULL only the element count is returned in *count.
 * Otherwise `bytes` must hold the whole array.                            */
enum {
    H2_EXP_PERM = 0,        /* int32 [n] tree position -> original index */
    H2_EXP_PARENT = 1,      /* int32 [nnode] */
    H2_EXP_FIRST_CHILD = 2, /* int32 [nnode] (-1 for leaves) */
    H2_EXP_NCHILD = 3,      /* int32 [nnode] */
    H2_EXP_START = 4,       /* int32 [nnode] first tree position */
    H2_EXP_COUNT = 5,       /* int32 [nnode] */
    H2_EXP_DEPTH = 6,       /* int32 [nnode] */
    H2_EXP_CENTER = 7,      /* double [nnode][dim] */
    H2_EXP_SIDE = 8,        /* double [nnode] */
    H2_EXP_IL_PTR = 9,      /* int32 [nnode+1] */
    H2_EXP_IL_COL = 10,     /* int32 [nnz_il] */
    H2_EXP_NEAR_PTR = 11,   /* int32 [nnode+1] */
    H2_EXP_NEAR_COL = 12,   /* int32 [nnz_near] */
    H2_EXP_XSTAR = 13,      /* int32 list of node `node` */
    H2_EXP_YSTAR = 14,      /* int32 list of node `node` */
    H2_EXP_RANK = 15,       /* int32 [nnode] */
    H2_EXP_MBAR = 16,       /* int32 [nnode] rows of the node's ID problem */
    H2_EXP_PIV = 17,        /* int32 list of node `node` (mbar entries) */
    H2_EXP_SKEL = 18,       /* int32 list of node `node` (rank entries) */
    H2_EXP_T = 19,          /* double, node `node`: rank x (mbar-rank) row-major */
    H2_EXP_POINTS = 20,     /* double [dim][n] SoA, tree order */
    H2_EXP_B = 21,          /* double, IL entry `node` (CSR index): rank_i x rank_v_j column-major (precision 64) */
    H2_EXP_CALIB_R = 22,    /* int32 [maxdepth+1] r chosen per depth (0 if not calibrated) */
    /* the column basis V, W (the same arrays as U, R for a symmetric kernel) */
    H2_EXP_RANK_V = 23,     /* int32 [nnode] */
    H2_EXP_MBAR_V = 24,     /* int32 [nnode] */
    H2_EXP_PIV_V = 25,      /* int32 list of node `node` */
    H2_EXP_SKEL_V = 26,     /* int32 list of node `node` */
    H2_EXP_T_V = 27         /* double, node `node`: rank_v x (mbar_v-rank_v) row-major */
};
h2_status h2_export(h2_handle h, int what, int node, void *host_buf, size_t bytes, int64_t *count);

/* Release a handle and all its device memory.  NULL is accepted.  Waits for
 * the handle's last h2_matvec (on whatever stream it ran) to finish, not for
 * other work on those streams; the memory returns to the library's cache. */
h2_status h2_destroy(h2_handle h);

/* Message of the last non-OK status returned on this thread. */
const char *h2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* H2_MI355X_H */
