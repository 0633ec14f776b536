/*
 * pdd.h -- C ABI of libpdd, Poisson-disk decimation of int32 point clouds on
 * one AMD Instinct MI355X (gfx950).
 *
 * The method (arXiv 2311.17604):
 *   - cost of a point p (Eq. 12, Sec. 4.2): the sum of 1 / d(p, p')^2 over
 *     its k nearest remaining neighbours p';
 *   - greedy removal (Sec. 4, Sec. 4.2): remove the remaining point of highest
 *     cost, update the costs its removal changes, repeat until exactly the
 *     requested number of points is left (Sec. 3: |C'| = lambda |C| with
 *     lambda = m / |C|).
 *
 * Exact integer reading used throughout (the paper's Eq. 12 is real-valued
 * and silent on ties and coincident points):
 *   d2(i, j) = sum over axes of (P_i - P_j)^2, int64, P in int32 millimetres;
 *   term(D)  = floor(2^56 / D) for D >= 1, 2^58 for D = 0;
 *   W(i)     = sum of term over the min(k, alive - 1) smallest d2 from i to
 *              the other alive points (uint64; k <= 32 keeps it below 2^64);
 *   key(i)   = (W descending, original index ascending); the greedy removes
 *              the highest key.  Results are therefore unique, and the
 *              library returns them bit for bit.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are DEVICE pointers on the context's device; the
 *     caller allocates and owns them; the library never frees or keeps them
 *     after the call returns.
 *   - Points are int32 x, y, z (mm) at a byte stride of 12 (packed xyz) or
 *     16 (xyz + 4 bytes of attributes, e.g. RGB + pad), first point at d_xyz.
 *   - Per-axis extent (max - min) must be < 2^21 mm (PDD_ERANGE otherwise).
 *   - Work runs on the context's stream.  pdd_decimate and
 *     pdd_decimate_batch synchronise that stream before returning;
 *     pdd_knn_cost returns once its work is enqueued.
 *   - Return value is a status code (PDD_OK = 0).  On error the output
 *     buffers' contents are unspecified, but nothing is written outside
 *     them.  No C++ exception crosses this interface.
 */
#ifndef PDD_H
#define PDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PDD_OK = 0,
    PDD_EINVAL = 1,    /* bad argument: sizes, k, keep, null pointers */
    PDD_ERANGE = 2,    /* coordinate extent >= 2^21 mm on some axis */
    PDD_ENOMEM = 3,    /* device allocation failed */
    PDD_EHIP = 4,      /* a HIP runtime call failed (see pdd_last_error) */
    PDD_EINTERNAL = 5  /* internal invariant violated (a bug) */
};

typedef struct pdd_ctx pdd_ctx;   /* device, stream, scratch pool */
typedef struct pdd_grid pdd_grid; /* Morton-sorted points + voxel cell table, owned by a ctx */

/* Options of a decimation.  A zero field takes the default. */
typedef struct {
    int32_t k;              /* neighbours in the cost, 1..32 (no default: required) */
    int32_t b;              /* extra buffered neighbours, k + b <= 32 (default: 8, capped) */
    int32_t voxel_log2;     /* cell edge = 2^voxel_log2 mm, 2..20 (default: chosen from density) */
    float round_frac;       /* initial share of alive points ranked per removal round, (0, 1] (default 0.01);
                               adapted per round between 1e-5 and 4x the initial value */
    int32_t point_stride;   /* bytes between points: 12 or 16 (default 12) */
    int32_t flags;          /* PDD_F_* bits */
    int32_t round_blocks;   /* workgroups (256 threads) per launch of the removal-round kernels, 64..65535
                               (default 1024); the kernels loop over their items, so results never depend on it */
    int32_t reserved[3];
} pdd_opts;

#define PDD_F_CHECK 1       /* extra device-side invariant checks (slower) */
#define PDD_F_TIMING 2      /* record HIP events per phase (see pdd_last_timing) */
#define PDD_F_PROGRESS 4    /* print a progress line to stderr every 50 removal rounds */
#define PDD_F_EAGER 8       /* launch each round's kernels one by one; by default a round is
                               captured as a hipGraph (a batch's as two, around the host-sized
                               budget cut) and replayed every round */

/* Create a context on HIP device `hip_device` that enqueues its work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  *out receives the
 * handle.  Errors: PDD_EINVAL (out NULL), PDD_EHIP. */
int pdd_ctx_create(pdd_ctx **out, int hip_device, void *hip_stream);

/* Release a context, its grids and scratch memory.  NULL is a no-op. */
void pdd_ctx_destroy(pdd_ctx *ctx);

/*
 * Voxel grid (Sec. 5: the cloud is voxelised and neighbours are searched in
 * the point's voxel and the adjacent ones).  Points are ordered by the
 * 63-bit Morton code of their coordinates relative to the cloud's minimum
 * corner; cells are the runs of equal code >> (3 * voxel_log2).  The grid
 * keeps a copy of the points; d_xyz may be freed after the call returns.
 *   d_xyz, n, stride : input points (n >= 2, stride 12 or 16)
 *   voxel_log2       : cell edge 2^voxel_log2 mm (2..20), 0 = automatic
 *   out              : receives the grid handle (free with pdd_grid_free)
 * Synchronises the stream (the cell count sizes the cell table).
 * Errors: PDD_EINVAL, PDD_ERANGE, PDD_ENOMEM, PDD_EHIP.
 */
int pdd_build_grid(pdd_ctx *ctx, const int32_t *d_xyz, int64_t n, int32_t stride,
                   int32_t voxel_log2, pdd_grid **out);

/* Free a grid.  NULL is a no-op. */
void pdd_grid_free(pdd_ctx *ctx, pdd_grid *grid);

/* Number of occupied cells and the voxel_log2 of a grid (either may be NULL). */
int pdd_grid_info(const pdd_grid *grid, int64_t *ncells, int32_t *voxel_log2);

/*
 * k-nearest-neighbour cost of every point of a grid over all its points
 * (Eq. 12 in the exact reading above).  Row i of each output belongs to the
 * input point i (original order).
 *   k, b    : 1 <= k, k + b <= 32
 *   d_nbr   : [n * (k+b)] int32 or NULL: original indices of the k+b nearest,
 *             ascending d2; -1 past the end when n - 1 < k + b.  Among equal
 *             d2 the order and, at the last place, the choice of point are
 *             unspecified.
 *   d_r2k   : [n] int64 or NULL: d2 of the min(k, n-1)-th nearest
 *   d_cost  : [n] uint64: W over the min(k, n-1) nearest
 * Errors: PDD_EINVAL, PDD_ENOMEM, PDD_EHIP.
 */
int pdd_knn_cost(pdd_ctx *ctx, const pdd_grid *grid, int32_t k, int32_t b, int32_t *d_nbr,
                 int64_t *d_r2k, uint64_t *d_cost);

/*
 * Greedy decimation (Sec. 4, Sec. 4.2) to exactly keep_count points.
 *   d_xyz, n        : input points (n >= 2), stride opts->point_stride
 *   keep_count      : 1..n points to keep
 *   opts            : k required; other fields 0 for defaults
 *   d_kept          : [keep_count] int32: kept original indices, ascending
 *   d_order         : [n - keep_count] int32 or NULL: removed indices in the
 *                     sequential greedy's removal order
 *   d_order_cost    : [n - keep_count] uint64 or NULL: W of each removed
 *                     point at its removal
 * The result equals the sequential greedy's bit for bit (removal happens in
 * rounds that provably commute with it).  Synchronises the stream.
 * Errors: PDD_EINVAL, PDD_ERANGE, PDD_ENOMEM, PDD_EHIP, PDD_EINTERNAL.
 */
int pdd_decimate(pdd_ctx *ctx, const int32_t *d_xyz, int64_t n, int64_t keep_count,
                 const pdd_opts *opts, int32_t *d_kept, int32_t *d_order, uint64_t *d_order_cost);

/*
 * Batch of independent clouds (scans) decimated together: cloud s is
 * points [h_offsets[s], h_offsets[s+1]) of d_xyz and keeps h_keep[s] of them,
 * exactly as pdd_decimate would on that cloud alone (Sec. 3 and 4 per
 * cloud).  All clouds share one grid (the cloud is the top of the sort key,
 * so no neighbourhood crosses two clouds) and one set of round kernels; in
 * each round every cloud whose ranked set exceeds its remaining removals
 * keeps only its top keys.
 *   h_offsets   : host array of nscan + 1 offsets, h_offsets[0] = 0,
 *                 every cloud at least 2 points, total < 2^31
 *   h_keep      : host array of nscan counts, 1 <= h_keep[s] <= size of s
 *   d_kept      : [sum h_keep] int32: per cloud its kept indices (relative to
 *                 the cloud's first point), ascending, clouds in order
 *   d_order     : [sum (size - keep)] int32 or NULL: per cloud its removed
 *                 indices (relative) in removal order, clouds in order
 *   d_order_cost: [sum (size - keep)] uint64 or NULL: cost at removal
 * Clouds are taken in consecutive groups of at most 2^28 points, each
 * group one batched decimation (so the round state fits the device).
 * Within a group each cloud's extent must fit 2^b mm per axis and the
 * clouds 2^c ids with 3b + c <= 63 (else PDD_ERANGE).  Synchronises the
 * stream.
 * Errors: PDD_EINVAL, PDD_ERANGE, PDD_ENOMEM, PDD_EHIP, PDD_EINTERNAL.
 */
int pdd_decimate_batch(pdd_ctx *ctx, const int32_t *d_xyz, const int64_t *h_offsets, int32_t nscan,
                       const int64_t *h_keep, const pdd_opts *opts, int32_t *d_kept, int32_t *d_order,
                       uint64_t *d_order_cost);

/*
 * Autotuner: chooses voxel_log2, b and round_frac for pdd_decimate of this
 * cloud by timing trial decimations of a strided sample (every step-th
 * point, about `sample` points; 0 = 2M) with keep scaled alike: round share,
 * then list width, then the finest cell level relative to the automatic one.
 * None of them can change a decimation's result, only its time.
 *   base    : k and point_stride used; other fields are the starting point
 *   out     : receives base with the chosen voxel_log2, b and round_frac
 *   best_ms : (if not NULL) the best trial's time on the sample
 * Synchronises the stream.  Errors: PDD_EINVAL, PDD_ERANGE, PDD_ENOMEM,
 * PDD_EHIP, PDD_EINTERNAL.
 */
int pdd_autotune(pdd_ctx *ctx, const int32_t *d_xyz, int64_t n, int64_t keep, const pdd_opts *base,
                 int64_t sample, pdd_opts *out, float *best_ms);

/*
 * Autotuner for pdd_decimate_batch: chooses round_frac and b for this batch
 * by timing trial batched decimations of every step-th cloud (whole clouds,
 * about `sample` points in all; 0 = 8M), gathered into one smaller batch:
 * round share, then list width.  The finest level stays automatic.  Like
 * pdd_autotune, the choice changes only the time of the result, never the
 * result (the question of voxel and buffer sizes that Sec. 7 leaves open).
 *   d_xyz, h_offsets, nscan, h_keep : the batch, as for pdd_decimate_batch
 *   base    : k and point_stride used; other fields are the starting point
 *   out     : receives base with the chosen b and round_frac
 *   best_ms : (if not NULL) the best trial's time on the sample
 * Synchronises the stream.  Errors: PDD_EINVAL, PDD_ERANGE, PDD_ENOMEM,
 * PDD_EHIP, PDD_EINTERNAL.
 */
int pdd_autotune_batch(pdd_ctx *ctx, const int32_t *d_xyz, const int64_t *h_offsets, int32_t nscan,
                       const int64_t *h_keep, const pdd_opts *base, int64_t sample, pdd_opts *out,
                       float *best_ms);

/*
 * Quality of a (decimated) cloud, the measures of Sec. 6: for every point
 * the number of other points within each of R radii, exact in integers
 * (|p - q|^2 <= r2[r] on int32 millimetres); per radius their mean and the
 * fractiles 0.01, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99 (element of rank
 * floor(q (m - 1)) in ascending order); the least-squares line of count
 * against neighbourhood area (pi r^2 in m^2) over all (point, radius) pairs,
 * whose slope estimates the density, with its R^2 and RMSE, computed in
 * double from the exact sums; and the squared distance from every point to
 * its nearest other point, whose minimum Eq. 2 maximises.
 *   d_xyz        : [m] points, int32 x, y, z (12 bytes) or x, y, z, pad (16)
 *   h_r2         : host array of R squared radii (mm^2), strictly increasing,
 *                  1 <= R <= PDD_QUALITY_MAX_R
 *   d_counts     : [m * R] uint32 or NULL: counts, point-major
 *   d_nn2        : [m] int64 or NULL: squared nearest-neighbour distances
 *   out          : host; receives the summary
 * m >= 2.  Synchronises the stream.  Errors: PDD_EINVAL (also when the
 * largest radius exceeds what the grid's levels cover), PDD_ERANGE,
 * PDD_ENOMEM, PDD_EHIP.
 */
#define PDD_QUALITY_MAX_R 32
#define PDD_QUALITY_NFRAC 7
typedef struct {
    int32_t R;
    int32_t fractile_capped;                       /* 1 if a fractile reached the 4095 cap */
    int64_t m;
    double area_m2[PDD_QUALITY_MAX_R];
    double mean[PDD_QUALITY_MAX_R];
    uint32_t fractile[PDD_QUALITY_MAX_R][PDD_QUALITY_NFRAC];
    uint64_t sum[PDD_QUALITY_MAX_R];               /* exact sum of the counts per radius */
    uint64_t sum_sq[PDD_QUALITY_MAX_R];            /* exact sum of their squares */
    double slope, intercept, r_squared, rmse;      /* count = intercept + slope * area */
    int64_t nn2_min;                               /* smallest squared nearest-neighbour distance */
} pdd_quality;
int pdd_quality_measure(pdd_ctx *ctx, const int32_t *d_xyz, int64_t m, int32_t stride_bytes, const int64_t *h_r2,
                        int32_t R, uint32_t *d_counts, int64_t *d_nn2, pdd_quality *out);

/* Counters of the last pdd_decimate on this context, written to stats[0..n),
 * n <= 15:
 *   0 rounds, 1 re-searches (buffer exhausted), 2 danger checks, 3 reverse-list
 *   rebuilds, 4 device bytes the context's scratch pool holds after the call
 *   (its high-water mark), 5 finest cell level (log2 mm), 6 list width used,
 *   7 touched (re-costed) points, 8 points tested by the initial k-NN search,
 *   9 lists certified in predicted regions, 10 lists in predicted regions
 *   that were not (searched again by the shell search), 11 points whose
 *   tile could not certify their list (all searched again), 12 points tested
 *   by the re-searches, 13 survivors enumerated by the danger checks, 14
 *   rounds launched as a replay of the captured round graph.
 * Entries 8-10 are also written by pdd_knn_cost.  After pdd_decimate_batch
 * the counters are summed over its groups of clouds (4-6: the last group's).
 * Returns the number of counters written. */
int pdd_last_stats(const pdd_ctx *ctx, int64_t *stats, int n);

/* Phase durations in ms of the last pdd_decimate on this context that ran
 * with PDD_F_TIMING, from HIP events recorded on the context's stream,
 * written to ms[0..n): 0 grid build, 1 initial k-NN cost kernel, 2 reverse
 * lists, 3 removal rounds, 4 finalisation (kept set and removal order);
 * after pdd_decimate_batch, summed over its groups of clouds.
 * Returns the number written. */
int pdd_last_timing(const pdd_ctx *ctx, float *ms, int n);

/*
 * Learned search region (not part of the paper; it sizes the k-NN search of
 * Sec. 5, which the paper does over the 26 voxels around a point's own
 * voxel).  The initial k-NN runs in tiles, one per anchor cell: the finest
 * grid cell around a point that holds list-width + 1 points.  A tile scans a
 * region of cells around its anchor cell; by default the cell grown by half
 * its edge.  A network predicts, per anchor cell, log2(e / cell edge), e the
 * growth needed for the region to hold the list of every point anchored
 * there (the list's last distance less the point's distance to the outside
 * of the cell, maximised over the cell), from 64 features: log1p of the
 * point counts of the 4x4x4 cells of half the edge centred on the cell.
 * The tile then uses the cell grown by 2^margin * e when that region is
 * smaller than the default one.  A list whose last distance is not within
 * the region's distance to its outside is searched again by the shell
 * search, so the predictor changes which points are tested, never a result.
 * A network is trained for one list width (list(k + b) below).
 *
 * Network: 64 -> 64 -> 64 -> 1 with ReLU; PDD_PRED_NPARAM parameters in
 * fp32, flat: W1 [64 in][64 out], b1 [64], W2 [64][64], b2 [64], w3 [64],
 * b3.  The products run in bf16 on matrix cores with fp32 accumulation.
 * Loss: mean pinball loss at level tau, tau max(y - yhat, 0) +
 * (1 - tau) max(yhat - y, 0); Adam (0.9, 0.999, 1e-8, bias-corrected).
 * The parameters live in the context; the calls below are stream-ordered
 * and synchronise before returning.
 */
#define PDD_PRED_NPARAM 8385

/* Set (host array of n == PDD_PRED_NPARAM floats) or read back the
 * parameters; setting also clears the Adam state.  Errors: PDD_EINVAL
 * (wrong n, or reading before any set), PDD_ENOMEM, PDD_EHIP. */
int pdd_pred_set_weights(pdd_ctx *ctx, const float *params, int64_t n);
int pdd_pred_get_weights(pdd_ctx *ctx, float *params, int64_t n);

/* Use (on != 0) or not the predicted regions in the initial k-NN of
 * pdd_knn_cost and pdd_decimate; margin_log2 in [0, 8] is added to the
 * predicted log2 growth.  Errors: PDD_EINVAL (no parameters set). */
int pdd_pred_enable(pdd_ctx *ctx, int32_t on, float margin_log2);

/* Training rows from a grid: runs the plain k-NN with list width
 * list(k + b), then for every anchor cell (level >= 1) writes its 64 bf16
 * features (d_feat [cap][64], uint16 bit patterns) and target
 * log2(e) - log2(cell edge), e the growth described above in mm (d_target
 * [cap] float; -8 when no growth is needed).  *count receives the number of
 * anchor cells; rows beyond cap are not written.
 * Errors: PDD_EINVAL, PDD_ENOMEM, PDD_EHIP. */
int pdd_pred_samples(pdd_ctx *ctx, const pdd_grid *grid, int32_t k, int32_t b, uint16_t *d_feat,
                     float *d_target, int64_t cap, int64_t *count);

/* Network outputs of n feature rows (d_feat [n][64] bf16) into d_out [n].
 * Errors: PDD_EINVAL (no parameters), PDD_EHIP. */
int pdd_pred_forward(pdd_ctx *ctx, const uint16_t *d_feat, int64_t n, float *d_out);

/* Gradient of the mean pinball loss over rows 0..n-1, 1 <= n <= 128, into
 * d_grad [PDD_PRED_NPARAM]; the loss into d_loss [1] if not NULL.  No
 * update.  Errors: PDD_EINVAL, PDD_EHIP. */
int pdd_pred_grad(pdd_ctx *ctx, const uint16_t *d_feat, const float *d_target, int64_t n, float tau,
                  float *d_grad, float *d_loss);

/* `steps` Adam steps (learning rate lr) on minibatches of `batch` rows
 * (16..128, a multiple of 16) drawn with replacement from the n rows by a
 * counter-based hash of seed, step and row; the loss of each step into
 * d_loss [steps] if not NULL.  Errors: PDD_EINVAL, PDD_ENOMEM, PDD_EHIP. */
int pdd_pred_train(pdd_ctx *ctx, const uint16_t *d_feat, const float *d_target, int64_t n, int32_t steps,
                   int32_t batch, float lr, float tau, uint64_t seed, float *d_loss);

/* Static description of a status code. */
const char *pdd_strerror(int status);

/* Text of the last HIP or internal error on this context ("" if none). */
const char *pdd_last_error(const pdd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PDD_H */
