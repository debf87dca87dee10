/*
 * tpcf.h -- angular two-point correlation pair counting on AMD MI355X (gfx950).
 *
 * C ABI of libtpcf.so.  The library counts, for a catalog of objects on the
 * sky, the pairs of objects per bin of angular separation: DD within a data
 * catalog, RR within a random catalog, DR across the two (paper, Section 1,
 * the definitions under Eq. 1), and combines the three histograms into the
 * Landy-Szalay estimator w(theta) (Eq. 1).  The angle of a pair is the
 * arc-cosine of the dot product of the two unit vectors (Section 3, first
 * bullet); pairs are binned in theta, not in cos theta (Section 2), with
 * per-block partial histograms combined into one global histogram (Section 3,
 * second bullet).
 *
 * Conventions for every entry point:
 *   - plain C types only; no exception crosses the boundary;
 *   - every call returns an int status (TPCF_OK or a negative TPCF_E_* code);
 *     tpcf_last_error(ctx) returns a message for the calling thread;
 *   - sizes and row indices are int64_t; catalogs hold at most 2^31 - 1024
 *     objects;
 *   - host input arrays are read during the call only (copied if needed);
 *   - output arrays are written only when the call returns TPCF_OK;
 *   - a context is used by one host thread at a time;
 *   - counts are exact: for the same catalog and edges, every precision mode
 *     returns the same integers as a plain FP64 CPU double loop using host
 *     libm acos on the same machine (see "Counting rule" below).
 *
 * Counting rule (shared by every precision mode):
 *   unit vector   x = cos(dec) cos(ra), y = cos(dec) sin(ra), z = sin(dec),
 *                 angles in radians as deg * (pi / 180), FP64 libm;
 *   dot product   d = (x_i x_j + y_i y_j) + z_i z_j, FP64, no fused
 *                 multiply-add, evaluated left to right;
 *   angle         theta = acos(clamp(d, -1, 1)) (host libm);
 *   edges         e_k = edge_deg[k] * (pi / 180), k = 0..nbins;
 *   slot          number of edges with e_k <= theta: slot 0 is theta < e_0,
 *                 slot k+1 is e_k <= theta < e_{k+1}, slot nbins+1 is
 *                 theta >= e_nbins (a tie goes to the upper bin).
 *   DD and RR count unordered pairs i < j (self-pairs excluded, N(N-1)/2 in
 *   total); DR counts all N_D * N_R pairs.
 *   The GPU never evaluates acos: each edge is compiled on the host into the
 *   largest double D_k with acos(D_k) >= e_k, and a pair counts past edge k
 *   exactly when clamp(d) <= D_k.
 */
#ifndef TPCF_H
#define TPCF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpcf_ctx tpcf_ctx;   /* opaque; owns device state */

/* Pair kinds (Section 1). */
enum { TPCF_DD = 0, TPCF_DR = 1, TPCF_RR = 2 };

/* Precision modes (identical counts).
 * TPCF_FP32_CHORD: bulk pairs are classified from the FP32 squared chord
 *   |f_i - f_j|^2 of FP32 copies of the unit vectors, against FP32 chord^2
 *   bands proven to contain every edge; a pair inside a band is re-decided in
 *   FP64 with the exact counting rule.
 * TPCF_FP64: every pair's FP64 dot product d is computed as in the counting
 *   rule and compared with D_k (the plain path). */
enum { TPCF_FP32_CHORD = 0, TPCF_FP64 = 1 };

enum {
    TPCF_OK = 0,
    TPCF_E_INVALID = -1,    /* bad argument; nothing launched */
    TPCF_E_NOMEM = -2,      /* device or host allocation failed */
    TPCF_E_HIP = -3,        /* a HIP runtime call failed */
    TPCF_E_BADID = -4,      /* unknown catalog or job id */
    TPCF_E_BUDGET = -5,     /* request exceeds the configured HBM budget */
    TPCF_E_CANCELLED = -6,  /* job was cancelled */
    TPCF_E_INTERNAL = -7    /* an internal consistency check failed */
};

/* Open a context on HIP device `device`.  hip_stream: a hipStream_t to launch
 * on (borrowed; it must outlive the context), or NULL for a non-blocking
 * stream owned by the context (the null stream itself cannot be borrowed).
 * Device buffers that other streams write or read around tpcf_count_async
 * need an explicit ordering (tpcf_synchronize, or events) with a context
 * that owns its stream.  *out receives the context. */
int tpcf_open(int device, void *hip_stream, tpcf_ctx **out);

/* Release every catalog and device buffer of the context, then the context. */
int tpcf_close(tpcf_ctx *ctx);

/* Upload a catalog given right ascension and declination in degrees (host
 * FP64 arrays of n finite values).  The library builds the FP64 unit vectors
 * with the counting rule's formula on the host, keeps them on the device as
 * structure-of-arrays (x[], y[], z[]) together with FP32 copies rounded to
 * nearest, and returns a catalog id in *out_cat.  Device memory is owned by
 * the library until tpcf_release_catalog or tpcf_close.  n may be 0.
 * Rows are stored in a spatially coherent order (a Morton curve of the unit
 * vectors), which the counts do not depend on; tpcf_catalog_order returns
 * it.  Row ranges in tpcf_count refer to this stored order. */
int tpcf_upload_catalog(tpcf_ctx *ctx, const double *ra_deg, const double *dec_deg,
                        int64_t n, int32_t *out_cat);

/* Same, from caller-computed FP64 unit vectors (host arrays).  Each vector
 * must satisfy | x^2 + y^2 + z^2 - 1 | <= 2^-20, else TPCF_E_INVALID. */
int tpcf_upload_catalog_xyz(tpcf_ctx *ctx, const double *x, const double *y,
                            const double *z, int64_t n, int32_t *out_cat);

/* 3-D catalog: Cartesian positions (comoving coordinates, any length unit;
 * host FP64 arrays of n finite values with |x|, |y|, |z| <= 2^50).  The paper
 * notes that its method carries over from w(theta) to the spatial
 * correlation function xi(r) (Section 1).  Pairs of a 3-D catalog are binned
 * by their Euclidean distance r under the 3-D counting rule:
 *   squared distance  r2 = (dx*dx + dy*dy) + dz*dz, dx = x_i - x_j etc.,
 *                     FP64, no fused multiply-add, left to right;
 *   distance          r = sqrt(r2) (host libm, correctly rounded);
 *   slot              number of edges e_k <= r (edges in the coordinates'
 *                     unit, finite, strictly increasing, within [0, 1e150]).
 * Every counting call (tpcf_count, _async, _batch, tpcf_submit) takes 3-D
 * catalogs in place of sky catalogs; bin_edges_deg then holds distances.
 * Both catalogs of a DR count must be 3-D, and so must every catalog of a
 * batch.  Precisions: TPCF_FP32_CHORD (FP32 squared distances of FP32 copies
 * against a proven band, band pairs re-decided with the exact rule) and
 * TPCF_FP64 (the rule's r2 against S_k = the smallest double whose square
 * root reaches e_k).  Pruning (tuning field prune) uses bounding balls.  The
 * FP32 band widens with the largest
 * norm R of the catalogs (about 2^-23 R in r), so coordinates centred on the
 * survey keep fewer pairs on the exact path.  Rows are stored in Morton order
 * of the bounding box; tpcf_catalog_order returns it. */
int tpcf_upload_catalog_3d(tpcf_ctx *ctx, const double *x, const double *y,
                           const double *z, int64_t n, int32_t *out_cat);

/* tpcf_upload_catalog_3d with jackknife region labels (see
 * tpcf_upload_catalog_regions): stored grouped by label, Morton order of the
 * bounding box inside each region; tpcf_count_regions and tpcf_jackknife
 * then give delete-one errors of xi(r). */
int tpcf_upload_catalog_3d_regions(tpcf_ctx *ctx, const double *x, const double *y,
                                   const double *z, int64_t n, const int32_t *region,
                                   int32_t nreg, int32_t *out_cat);

/* Zero-copy attach of caller-owned device memory: d_xyz64 points to 3*n
 * doubles on the context's device laid out as x[0..n), y[0..n), z[0..n)
 * (unit vectors, same norm limit as above).  d_xyz32 is NULL, or 3*n floats
 * on the same device in the same layout holding the FP32 copies rounded to
 * nearest, (float)x[i] etc.; with NULL the library makes its own copy.  The
 * caller keeps both arrays alive and unchanged until the catalog is
 * released.  Checked on the device; TPCF_E_INVALID if a vector fails the
 * norm limit or is not finite, or if a given FP32 copy is not the rounded
 * FP64 value (the FP32 band is proven for round-to-nearest copies).  Rows
 * keep the caller's order. */
int tpcf_attach_catalog(tpcf_ctx *ctx, const double *d_xyz64, const float *d_xyz32, int64_t n,
                        int32_t *out_cat);

/* Storage order of a catalog: out_order (host, n int64) receives, for each
 * stored row r, the index of that object in the uploaded arrays.  Attached
 * catalogs keep the caller's order (identity). */
int tpcf_catalog_order(tpcf_ctx *ctx, int32_t cat, int64_t *out_order);

/* Number of objects of a catalog. */
int tpcf_catalog_size(tpcf_ctx *ctx, int32_t cat, int64_t *out_n);

/* Release a catalog id and the device memory the library owns for it.
 * Freeing device memory waits until all work on the device has finished
 * (jobs in flight on any stream included), so callers that keep jobs running
 * release catalogs in batches rather than at every completion. */
int tpcf_release_catalog(tpcf_ctx *ctx, int32_t cat);

/* Jackknife regions.  The paper judges its residuals against the statistical
 * error of a sky with few independent fields (Section 4, discussion of the
 * w(theta) residuals); a delete-one jackknife over sky regions estimates that
 * error from one pass of counting.  Regions are labels chosen by the caller
 * (contiguous patches of sky, typically). */
#define TPCF_MAX_REGIONS 1024

/* tpcf_upload_catalog with a region label per object: region (host, n int32)
 * holds values in [0, nreg), 1 <= nreg <= TPCF_MAX_REGIONS; NULL region
 * uploads an unlabelled catalog (nreg ignored).  Objects are stored grouped
 * by region (each region a contiguous run of rows, in label order), Morton
 * order within a region; tpcf_catalog_order returns the order.
 * TPCF_E_INVALID for a label out of range. */
int tpcf_upload_catalog_regions(tpcf_ctx *ctx, const double *ra_deg, const double *dec_deg,
                                int64_t n, const int32_t *region, int32_t nreg,
                                int32_t *out_cat);

/* Region count of a catalog in *out_nreg (0 if unlabelled) and, when
 * out_counts (host, nreg int64) is not NULL, the objects per region. */
int tpcf_catalog_regions(tpcf_ctx *ctx, int32_t cat, int32_t *out_nreg, int64_t *out_counts);

/* Counts of a whole-catalog request split by region (synchronous): the
 * pairs as tpcf_count with row_begin = row_end = -1 into out_total (nbins+2
 * slots), and into out_touch (host, nreg x (nbins+2) u64, region-major) for
 * every region r the pairs with at least one member in r (a pair inside one
 * region is counted once there).  The counts with region r deleted are then
 * out_total - out_touch[r], exactly.  Both catalogs (cat_b = -1 for DD/RR)
 * must carry labels with the same nreg.  Same kinds, edges and precisions as
 * tpcf_count; results are not cached. */
int tpcf_count_regions(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b,
                       const double *bin_edges_deg, int32_t nbins, int precision,
                       uint64_t *out_total, uint64_t *out_touch);

/* Count pairs (synchronous): the DD, DR or RR histogram of the paper's
 * estimator (Section 1, the pair counts defined below Eq. 1), binned in theta
 * (Section 2) by the counting rule above (Section 3, first bullet).
 * kind       TPCF_DD or TPCF_RR: unordered pairs i < j of cat_a, cat_b must be
 *            -1; TPCF_DR: every pair (i in cat_a, j in cat_b).
 * bin_edges_deg  nbins+1 finite, strictly increasing values in [0, 180]
 *            (host array); 1 <= nbins <= 256.
 * precision  TPCF_FP32_CHORD or TPCF_FP64 (identical results).
 * row_begin, row_end  restrict i to rows [row_begin, row_end) of cat_a, in
 *            the catalog's stored order (tpcf_catalog_order); -1, -1 selects
 *            all rows.  For DD/RR the pairs are (i, j) with i in the range and
 *            j > i in stored order.
 * out_u64    host array of nbins+2 slots: [theta < e_0, bin 0 .. bin nbins-1,
 *            theta >= e_nbins].  Written on TPCF_OK only.
 * The total over slots always equals the number of pairs in the request; a
 * mismatch is reported as TPCF_E_INTERNAL. */
int tpcf_count(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b,
               const double *bin_edges_deg, int32_t nbins, int precision,
               int64_t row_begin, int64_t row_end, uint64_t *out_u64);

/* Asynchronous count into device memory: d_out_u64 is a device pointer to
 * nbins+2 uint64 slots, overwritten (not accumulated) by work enqueued on the
 * context stream; the call returns once the work is enqueued.  Same
 * arguments and results as tpcf_count otherwise.  The totals check is not
 * performed (the caller may check the sum). */
int tpcf_count_async(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b,
                     const double *bin_edges_deg, int32_t nbins, int precision,
                     int64_t row_begin, int64_t row_end, uint64_t *d_out_u64);

/* tpcf_count for callers that cannot allocate device memory (code that
 * must not call hipMalloc or hipFree, such as tight serving loops or hosts
 * that forbid allocation during a run).  Same arguments, result, totals check
 * and errors as tpcf_count, and the same kernels, but every work buffer (the
 * histogram copies, the work-queue counter, the output slots, the edge and
 * cell tables and the work-unit list) lives in a fixed 16 MiB array in device
 * memory, one per device, set up by tpcf_open and held until the process
 * ends.  The call allocates no device memory, creates no event and does not
 * use the RR result cache; catalogs must already be uploaded or attached.
 * Exact tile pruning is not applied (its bounding caps are built on first
 * use, which allocates); the counts are the same.  Requests whose work-unit
 * list does not fit the array (beyond roughly 3e5 units, which the plan keeps
 * below by widening column chunks, e.g. a 1e6 x 2e6 DR fits) fail with
 * TPCF_E_INVALID.  Synchronous: the array is free again when the call
 * returns.  All calls on one device share its array, so calls that overlap
 * on the same device (from several threads or contexts) race; the caller
 * serialises them. */
int tpcf_count_noalloc(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b,
                       const double *bin_edges_deg, int32_t nbins, int precision,
                       int64_t row_begin, int64_t row_end, uint64_t *out_u64);

/* One counting request, as used by batches and submitted jobs.  Fields have
 * the meaning of the tpcf_count arguments of the same names; the edges array
 * is read during the call only. */
typedef struct tpcf_job_desc {
    int kind;
    int32_t cat_a, cat_b;
    const double *bin_edges_deg;
    int32_t nbins;
    int precision;
    int64_t row_begin, row_end;
} tpcf_job_desc;

enum { TPCF_BATCH_GRAPH = 1 };

/* Count many requests in one launch (e.g. many data catalogs of uneven size
 * against one resident random catalog, or jackknife subsamples): each job is
 * a DD, DR or RR count as tpcf_count (Section 1, the pair counts below
 * Eq. 1); the paper gives each histogram a GPU of its own (Section 3, third
 * bullet), here the work units of all jobs share one launch.  All jobs
 * must share the same edges, nbins and precision.  The work units of every
 * job form one list, largest first, processed by one kernel launch; each job
 * gets its own histogram.  out_u64: host array of njobs * (nbins+2) slots,
 * job k at offset k * (nbins+2), written on TPCF_OK only.  flags:
 * TPCF_BATCH_GRAPH captures the launch sequence in a hipGraph on the first
 * call for a given batch (same job descriptions and catalogs) and replays it
 * on later calls; the graph is dropped when any catalog is released.
 * Synchronous; totals are checked for every job. */
int tpcf_count_batch(tpcf_ctx *ctx, const tpcf_job_desc *jobs, int32_t njobs, int flags,
                     uint64_t *out_u64);

/* Asynchronous jobs for serving.  Each job is one DD, DR or RR count as
 * tpcf_count (Section 1, the pair counts below Eq. 1).  tpcf_submit
 * validates and enqueues one request on one of four library streams (jobs on
 * different streams overlap on the device) and returns a job id.  An RR request whose result is
 * cached (same catalog, edges, precision and rows; the cache is cleared for a
 * catalog when it is released) completes at submit without device work.
 * tpcf_poll sets *done = 1 and writes nbins+2 slots to out_u64 (may be NULL)
 * when the job has finished, and then retires the id; *done = 0 otherwise.
 * tpcf_wait blocks until the job finishes, then acts like tpcf_poll.
 * tpcf_cancel sets a flag in host memory that the kernel reads before every
 * work unit; the job's poll/wait then returns TPCF_E_CANCELLED and retires
 * it.  A catalog cannot be released while an unretired job uses it. */
int tpcf_submit(tpcf_ctx *ctx, const tpcf_job_desc *job, int64_t *out_job);
int tpcf_poll(tpcf_ctx *ctx, int64_t job, uint64_t *out_u64, int *done);
int tpcf_wait(tpcf_ctx *ctx, int64_t job, uint64_t *out_u64);
int tpcf_cancel(tpcf_ctx *ctx, int64_t job);

/* Launch shape of later launches (set by the autotuner; defaults are fine).
 * Every field 0 takes the default.
 * rows_per_lane   2 or 4 rows held in registers per lane (default 4);
 * hist_copies     LDS histogram copies per wavefront, 4, 8, 16 or 32
 *                 (default 16); a value above what the slot count allows
 *                 (32 up to 46 slots, 16 up to 94, 8 up to 190, else 4) is
 *                 lowered;
 * max_cols        largest column range of a work unit, multiple of 256 in
 *                 [256, 65536] (default 4096);
 * blocks_per_cu   grid size per compute unit, <= 64 (default: the blocks
 *                 that fit at once; wavefronts take work from a queue);
 * lut_bytes       largest cell table held in LDS, 4096..33792 bytes
 *                 (default 24576; for wrapped tables 32768, which then also
 *                 hold the histograms and thresholds);
 * lut_direct      1: FP32 byte tables in the wrapped layout: the kernel
 *                 starts its sum for q at a floor q0 (a power of two below
 *                 a quarter of the smallest threshold), so every key lies in
 *                 one window of cells, and reads cell (bits(q) >> shift)
 *                 mod 2^w with one bitfield extract instead of a shift, a
 *                 clamp and an add; the table's unused part holds the
 *                 histograms (see tpcf_compile_wrap32).  Falls back to the
 *                 clamped layout when nothing fits.  0 (default): the table
 *                 starts at the first edge and the key is clamped;
 * prune           1: exact tile pruning.  Bounding caps of the column
 *                 catalog's aligned 64-point groups (built on first use,
 *                 4 doubles per group) and of each wavefront's rows bound the
 *                 angles of a row block x 64-column block (widened by
 *                 1e-6 rad); the counting rule's dot products of the block's
 *                 pairs then lie in an interval that also covers the
 *                 catalogs' norm deviation | |v|^2 - 1 |, and when no
 *                 threshold D_k falls inside it all of the block's pairs go
 *                 to one slot without being evaluated.  3-D catalogs: bounding balls
 *                 (mean and largest distance from it) bound the distances,
 *                 widened by 2^-22 R (R the largest norm) and 1e-12
 *                 relative.  Counts are unchanged; 0 (default) evaluates
 *                 every pair.
 * Results never depend on these.  tpcf_get_tuning returns the fields as set
 * (0 standing for the default); NULL to tpcf_set_tuning restores defaults. */
typedef struct tpcf_tuning {
    int32_t rows_per_lane;
    int32_t hist_copies;
    int32_t max_cols;
    int32_t blocks_per_cu;
    int32_t lut_bytes;
    int32_t lut_direct;
    int32_t prune;
} tpcf_tuning;

int tpcf_set_tuning(tpcf_ctx *ctx, const tpcf_tuning *tuning);
int tpcf_get_tuning(tpcf_ctx *ctx, tpcf_tuning *out);

/* HBM budget for everything the context allocates (catalogs, tables, plans,
 * workspaces); 0 = unlimited.  An allocation that would exceed it fails with
 * TPCF_E_BUDGET and leaves the context unchanged.  tpcf_hbm_usage reports
 * the bytes in use and the budget. */
int tpcf_set_hbm_budget(tpcf_ctx *ctx, int64_t bytes);
int tpcf_hbm_usage(tpcf_ctx *ctx, int64_t *out_used, int64_t *out_budget);

/* Wait for all work enqueued by the context (its stream and job streams). */
int tpcf_synchronize(tpcf_ctx *ctx);

/* Kernel timing.  With timing on, the library records a HIP event pair on
 * the context stream around every pair-kernel launch.  tpcf_kernel_time
 * waits for them and returns the summed kernel time in milliseconds and the
 * number of launches since the last reset; reset = 1 clears the record. */
int tpcf_set_timing(tpcf_ctx *ctx, int on);
int tpcf_kernel_time(tpcf_ctx *ctx, double *out_ms, int64_t *out_launches, int reset);

/* Work statistics since the last reset. */
typedef struct tpcf_counters {
    uint64_t pairs;           /* pairs evaluated */
    uint64_t flagged;         /* pairs that left the table-driven path for a threshold comparison */
    uint64_t exact;           /* pairs re-decided with the exact FP64 rule (FP32_CHORD band
                                 pairs, FP64 ties) */
    uint64_t rare_steps;      /* wavefront steps (64 lanes x a few pairs each) that took the
                                 rare path */
    uint64_t beyond_steps;    /* steps whose pairs all lay certainly beyond the last edge,
                                 counted in registers without table lookups */
    uint64_t one_slot_steps;  /* steps where each lane's pairs all fell in one certain slot,
                                 added with one LDS atomic per lane */
    uint64_t pruned_pairs;    /* pairs binned by pruned blocks without being evaluated
                                 (tuning field prune) */
    uint64_t two_slot_steps;  /* steps where each lane's pairs fell in two adjacent slots,
                                 decided by one threshold comparison per pair and added with
                                 two LDS atomics per lane */
    uint64_t chord_steps;     /* FP32 angular steps that formed the squared chord: the
                                 dot product did not decide them, or the step lay at
                                 small angles where the chord comes first */
} tpcf_counters;

/* Copy the statistics to *out (may be NULL) and, with reset = 1, clear
 * them.  Waits for all of the context's streams. */
int tpcf_stats(tpcf_ctx *ctx, tpcf_counters *out, int reset);

/* Landy-Szalay estimator (Eq. 1), host FP64; no context needed.
 * dd, dr, rr  histograms of nbins+2 slots as returned by tpcf_count (DD and
 *             RR of unordered pairs); only the nbins in-range bins are used.
 * n_d, n_r    catalog sizes (>= 2 each).
 * form 0      w_k = (DD_k/n_DD - 2 DR_k/n_DR + RR_k/n_RR) / (RR_k/n_RR) with
 *             n_DD = N_D(N_D-1)/2, n_DR = N_D N_R, n_RR = N_R(N_R-1)/2;
 * form 1      Eq. 1 as printed, the exponent read as a square and DD, RR
 *             doubled to ordered counts:
 *             w_k = 1 + (N_R/N_D)^2 (2 DD_k)/(2 RR_k) - 2 (N_R/N_D) DR_k/(2 RR_k).
 * out_w       host array of nbins doubles; NaN where RR_k = 0. */
int tpcf_landy_szalay(const uint64_t *dd, const uint64_t *dr, const uint64_t *rr,
                      int32_t nbins, int64_t n_d, int64_t n_r, int form, double *out_w);

/* Delete-one jackknife of the Landy-Szalay w over nreg regions, host FP64; no
 * context needed.  dd, dr, rr: whole-catalog histograms (nbins+2 slots);
 * dd_touch, dr_touch, rr_touch: the matching tpcf_count_regions outputs
 * (nreg x (nbins+2)); n_d, n_r: catalog sizes; nd_reg, nr_reg: objects per
 * region (tpcf_catalog_regions).  For each region r, sample r is
 * tpcf_landy_szalay (same form) of the counts total - touch[r] with sizes
 * n_d - nd_reg[r], n_r - nr_reg[r].  Outputs (host): out_samples nreg x nbins
 * (region-major), out_mean nbins (may be NULL), out_cov nbins x nbins (may
 * be NULL), cov = (nreg-1)/nreg * sum_r (w_r - mean)(w_r - mean)^T.
 * 2 <= nreg <= TPCF_MAX_REGIONS; TPCF_E_INVALID as tpcf_landy_szalay for a
 * deleted catalog with fewer than 2 objects. */
int tpcf_jackknife(const uint64_t *dd, const uint64_t *dd_touch, const uint64_t *dr,
                   const uint64_t *dr_touch, const uint64_t *rr, const uint64_t *rr_touch,
                   int32_t nbins, int32_t nreg, int64_t n_d, const int64_t *nd_reg, int64_t n_r,
                   const int64_t *nr_reg, int form, double *out_samples, double *out_mean,
                   double *out_cov);

/* Host-side edge compilation, exposed for inspection and CPU tests of the
 * host logic (no device work).  For nbins+1 edges in degrees it writes:
 *   out_D    nbins+1 doubles: D_k = largest double d in [-1, 1] with
 *            acos(d) >= e_k (+inf if e_k == 0, -inf if acos(-1) < e_k);
 *   out_qlo, out_qhi  nbins+1 floats: the FP32 chord^2 band of edge k for
 *            catalogs whose squared norms deviate from 1 by at most
 *            delta_max: q < qlo_k implies d > D_k and q >= qhi_k implies
 *            d <= D_k for the kernel's q = fl32 |f_i - f_j|^2;
 * any output pointer may be NULL. */
int tpcf_compile_edges(const double *bin_edges_deg, int32_t nbins, double delta_max,
                       double *out_D, float *out_qlo, float *out_qhi);

/* The FP32 dot-product screen of the angular kernels (host only, for CPU
 * tests): for catalogs whose squared norms deviate from 1 by at most
 * delta_max, a pair whose FP32 copies have p = fl32(f_i . f_j) <= *out_p
 * (with any order of fused or separate roundings) has the rule's d <= D of
 * the last edge, i.e. lies at or beyond it (Section 3, first bullet: the
 * angle from the dot product).  -inf when no pair can pass the last edge. */
int tpcf_compile_screen(const double *bin_edges_deg, int32_t nbins, double delta_max, float *out_p);

/* Tables of the FP32 angular kernels' dot-product path (host only, for CPU
 * tests of the host logic).  A step first forms p = fl32(f_i . f_j) of the
 * FP32 copies (Section 3: the angle comes from the dot product); each lane
 * keys its largest and smallest p as q' = fl32(2 - 2p), a negative q' read
 * as +0, into the cell clamp(bits(q') >> shift, lo, hi), whose entry
 * cells[cell - lo] has the codes of tpcf_compile_cells.  Per edge k (nbins+1
 * floats each, any may be NULL): q' >= out_khi[k] proves that the FP64 rule
 * puts the pair at or past edge k and q' < out_klo[k] that it does not;
 * p <= out_plo[k] and p >= out_phi[k] prove the same directly on p.
 * out_cells holds max_cells entries (16..33792; the kernels use 1024 bytes).
 * Returns TPCF_E_INVALID for invalid edges, delta_max outside [0, 2^-20] or
 * NULL shift/lo/hi/cells. */
int tpcf_compile_dot(const double *bin_edges_deg, int32_t nbins, double delta_max, int32_t max_cells,
                     float *out_klo, float *out_khi, float *out_plo, float *out_phi, int32_t *out_shift,
                     int32_t *out_lo, int32_t *out_hi, uint16_t *out_cells);

/* Cell table of the pair kernels for the given edges (host only, for CPU
 * tests of the host logic).  precision selects the key: TPCF_FP32_CHORD uses
 * the bits of q = fl32 |f_i - f_j|^2, TPCF_FP64 the high 32 bits of e = 1 - d
 * as a signed integer.  A key maps to cell
 * clamp(key >> shift, lo, hi); entry cells[cell - lo] is a slot (< 0x8000),
 * 0x8000 | k when only edge k is undecided in the cell, or 0xFFFF when
 * several edges are.  direct = 1 (TPCF_FP32_CHORD only) asks for the cells
 * of the wrapped layout (tpcf_compile_wrap32 with max_bytes = max_cells and
 * the default launch's histogram and threshold bytes), in cell order lo..hi;
 * its key is that of q summed from the floor, which always lies in
 * [lo, hi].  It fails with TPCF_E_INVALID if that table would not fit.
 * out_cells must hold max_cells entries (16..33792; the kernels use up to
 * 32768 bytes for wrapped tables, 24576 for other byte tables, 12288 beyond
 * 125 bins); out_E (nbins+1 doubles, may be NULL) receives fl(1 - D_k). */
int tpcf_compile_cells(const double *bin_edges_deg, int32_t nbins, int precision, double delta_max,
                       int32_t max_cells, int32_t direct, int32_t *out_shift, int32_t *out_lo,
                       int32_t *out_hi, uint16_t *out_cells, double *out_E);

/* Wrapped FP32 byte table (host only, for CPU tests; the layout of
 * lut_direct = 1).  For unit vectors whose squared norms deviate from 1 by at
 * most delta_max, the kernel forms q = fl(dz^2 + fl(dy^2 + fl(dx^2 + q0)))
 * from the FP32 differences, with the floor q0 = *out_q0, a power of two at
 * most a quarter of the smallest positive threshold and at least 2^-100.  Then
 * q < out_qlo[k] implies d > D_k and q >= out_qhi[k] implies d <= D_k (nbins+1
 * floats each, may be NULL), the floor included in the bounds.  Every key
 * bits(q) >> *out_shift lies in [*out_lo, *out_hi]; cell c sits at entry
 * c mod 2^(*out_wrap_bits) of out_image (2^(*out_wrap_bits) bytes, may be
 * NULL), with the entry codes of tpcf_compile_cells in one byte (slot,
 * 0x80 | k, or 0xFF); entries no key reaches are 0, and aux_bytes of them
 * from the 16-aligned byte offset *out_aux_off on are free for the
 * histograms and thresholds; when placing them after the table takes fewer
 * bytes in all, *out_aux_off is the table's size instead.  The table is the
 * smallest shift, then the smallest layout whose bytes in all stay within
 * max_bytes (256..65536), that fits; at most 125 bins.  TPCF_E_INVALID if
 * nothing fits. */
int tpcf_compile_wrap32(const double *bin_edges_deg, int32_t nbins, double delta_max, int32_t max_bytes,
                        int32_t aux_bytes, int32_t *out_shift, int32_t *out_wrap_bits, int32_t *out_lo,
                        int32_t *out_hi, int32_t *out_aux_off, float *out_q0, float *out_qlo, float *out_qhi,
                        uint8_t *out_image);

/* 3-D edge compilation (host only, for CPU tests): for nbins+1 distance
 * edges (as tpcf_upload_catalog_3d) and points of FP64 norm at most rmax
 * (0 <= rmax <= 2^51):
 *   out_S    nbins+1 doubles: S_k = smallest double s with sqrt(s) >= e_k
 *            (-inf when e_k == 0: every pair is at or past it);
 *   out_qlo, out_qhi  nbins+1 floats: the FP32 band, q < qlo_k implies
 *            r2 < S_k and q >= qhi_k implies r2 >= S_k for the kernel's
 *            q = fl32 |f_i - f_j|^2 of the FP32 copies;
 * any output pointer may be NULL. */
int tpcf_compile_edges_3d(const double *bin_edges, int32_t nbins, double rmax, double *out_S,
                          float *out_qlo, float *out_qhi);

/* Message describing the last failed call on the calling thread ("" if none).
 * Messages are kept per host thread, not per context: ctx may be NULL (for
 * the calls that take no context, or a failed tpcf_open) and is not
 * dereferenced.  Valid until the next call on the same thread. */
const char *tpcf_last_error(const tpcf_ctx *ctx);

/* Library version string. */
const char *tpcf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TPCF_H */
