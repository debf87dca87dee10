/*
 * CPU oracle for angular pair counting -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  The product path (the HIP library) shares no code
 * with it and never calls it.
 *
 * What it computes (paper, Section 1 and Section 3, first two bullets):
 *   - every object is a unit vector on the sky, built from (RA, Dec);
 *   - the angle between two objects is the arc-cosine of the dot product of
 *     their unit vectors;
 *   - DD counts pairs of objects within the data catalog, RR within the
 *     random catalog, and DR pairs of one data and one random object, each
 *     as a histogram over angular-separation bins (theta space, not cos theta,
 *     Section 2).
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - DD and RR count unordered pairs i < j, self-pairs excluded; DR counts
 *     all N_D * N_R pairs, coincident positions included;
 *   - the dot product is evaluated in FP64 as (x_i x_j + y_i y_j) + z_i z_j,
 *     left to right, each operation rounded (no fused multiply-add), and is
 *     clamped to [-1, 1] before the arc-cosine (host libm acos);
 *   - edges are given in degrees and converted with edge * (pi / 180);
 *     slot s of the output is the number of edges e_k with e_k <= theta, so
 *     slot 0 is theta < e_0, slot k+1 is e_k <= theta < e_{k+1}, and slot
 *     nbins+1 is theta >= e_nbins (ties go to the upper bin).
 *
 * The same file counts pairs by 3-D distance (oracle_count3d): the paper
 * notes that the method carries over to the spatial correlation function
 * (Section 1); there the separation is the FP64 Euclidean distance
 * sqrt((dx^2 + dy^2) + dz^2) of the coordinate differences, each operation
 * rounded, and edges are distances.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fno-builtin -shared -fPIC
 * -pthread (no builtins: sin and cos stay separate libm calls).
 * Every loop below is the plain definition; threads only split the rows i.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Unit vector of an object at right ascension ra and declination dec, both
 * in degrees: x = cos(dec) cos(ra), y = cos(dec) sin(ra), z = sin(dec).  The
 * paper forms the angle from a dot product (Section 3), which presumes these
 * unit vectors. */
void oracle_radec_to_xyz(int64_t n, const double *ra_deg, const double *dec_deg,
                         double *x, double *y, double *z)
{
    const double deg = M_PI / 180.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = ra_deg[i] * deg;
        double b = dec_deg[i] * deg;
        x[i] = cos(b) * cos(a);
        y[i] = cos(b) * sin(a);
        z[i] = sin(b);
    }
}

/* Angle between two unit vectors: arc-cosine of the clamped dot product
 * (Section 3, first bullet). */
static double pair_angle(double xi, double yi, double zi,
                         double xj, double yj, double zj)
{
    double d = (xi * xj + yi * yj) + zi * zj;
    if (d < -1.0) d = -1.0;
    if (d > 1.0) d = 1.0;
    return acos(d);
}

/* Separation of two points in 3-D (the spatial variant of the correlation
 * function, Section 1): the Euclidean distance, in FP64, from the coordinate
 * differences, (dx^2 + dy^2) + dz^2 left to right with every operation
 * rounded, then the libm square root. */
static double pair_distance(double xi, double yi, double zi,
                            double xj, double yj, double zj)
{
    double dx = xi - xj;
    double dy = yi - yj;
    double dz = zi - zj;
    double d2 = (dx * dx + dy * dy) + dz * dz;
    return sqrt(d2);
}

/* Output slot of an angle (or a distance): the number of edges at or below it. */
static int slot_of(double t, const double *edge_rad, int nedges)
{
    int s = 0;
    for (int k = 0; k < nedges; ++k)
        if (edge_rad[k] <= t)
            ++s;
    return s;
}

typedef struct {
    int cross;                       /* 0: pairs i<j within A; 1: A x B */
    int metric;                      /* 0: angle on the sky; 1: distance in 3-D */
    int64_t na, nb;
    const double *ax, *ay, *az, *bx, *by, *bz;
    int nedges;
    const double *edge_rad;
    int64_t row_begin, row_end;
    int64_t next_row;                /* shared row counter (atomic) */
    int64_t chunk;
} job_t;

typedef struct {
    job_t *job;
    uint64_t *hist;                  /* nedges + 1 slots, private */
} worker_t;

static double separation(const job_t *jb, double xi, double yi, double zi,
                         double xj, double yj, double zj)
{
    return jb->metric ? pair_distance(xi, yi, zi, xj, yj, zj) : pair_angle(xi, yi, zi, xj, yj, zj);
}

static void *worker(void *arg)
{
    worker_t *w = (worker_t *)arg;
    job_t *jb = w->job;
    for (;;) {
        int64_t r0 = __atomic_fetch_add(&jb->next_row, jb->chunk, __ATOMIC_RELAXED);
        if (r0 >= jb->row_end)
            break;
        int64_t r1 = r0 + jb->chunk;
        if (r1 > jb->row_end)
            r1 = jb->row_end;
        for (int64_t i = r0; i < r1; ++i) {
            double xi = jb->ax[i], yi = jb->ay[i], zi = jb->az[i];
            if (jb->cross) {
                for (int64_t j = 0; j < jb->nb; ++j) {
                    double t = separation(jb, xi, yi, zi, jb->bx[j], jb->by[j], jb->bz[j]);
                    w->hist[slot_of(t, jb->edge_rad, jb->nedges)] += 1;
                }
            } else {
                for (int64_t j = i + 1; j < jb->na; ++j) {
                    double t = separation(jb, xi, yi, zi, jb->ax[j], jb->ay[j], jb->az[j]);
                    w->hist[slot_of(t, jb->edge_rad, jb->nedges)] += 1;
                }
            }
        }
    }
    return NULL;
}

/*
 * Pair-count histogram.
 *   cross = 0: unordered pairs i < j of catalog A with i in [row_begin,
 *              row_end) (DD or RR);
 *   cross = 1: pairs (i, j), i in rows [row_begin, row_end) of A, j in B (DR).
 * metric 0: angles, edges in degrees; metric 1: 3-D distances, edges in the
 * coordinates' unit.  edges: nbins+1 increasing values.  out: nbins+2 slots.
 * row_begin < 0 or row_end < 0 select all rows.  Returns 0, or -1 on bad
 * arguments.
 */
static int count_pairs(int cross, int metric, int64_t na, const double *ax, const double *ay,
                       const double *az, int64_t nb, const double *bx, const double *by,
                       const double *bz, int32_t nbins, const double *edges,
                       int64_t row_begin, int64_t row_end, int nthreads, uint64_t *out)
{
    if (nbins < 1 || na < 0 || (cross && nb < 0) || !out)
        return -1;
    const double deg = M_PI / 180.0;
    int nedges = nbins + 1;
    double *edge_rad = (double *)malloc(sizeof(double) * (size_t)nedges);
    if (!edge_rad)
        return -1;
    /* angular edges come in degrees; distances are used as given */
    for (int k = 0; k < nedges; ++k)
        edge_rad[k] = metric ? edges[k] : edges[k] * deg;

    if (row_begin < 0) row_begin = 0;
    if (row_end < 0 || row_end > na) row_end = na;
    if (row_begin > row_end) row_begin = row_end;
    if (nthreads < 1) nthreads = 1;

    job_t jb = {cross, metric, na, nb, ax, ay, az, bx, by, bz, nedges, edge_rad,
                row_begin, row_end, row_begin, 16};
    worker_t *ws = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t *hists = (uint64_t *)calloc((size_t)nthreads * (size_t)(nedges + 1), sizeof(uint64_t));
    if (!ws || !th || !hists) {
        free(ws); free(th); free(hists); free(edge_rad);
        return -1;
    }
    for (int t = 0; t < nthreads; ++t) {
        ws[t].job = &jb;
        ws[t].hist = hists + (size_t)t * (size_t)(nedges + 1);
    }
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, worker, &ws[t]);
    worker(&ws[0]);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);

    for (int s = 0; s <= nedges; ++s) {
        uint64_t acc = 0;
        for (int t = 0; t < nthreads; ++t)
            acc += ws[t].hist[s];
        out[s] = acc;
    }
    free(ws); free(th); free(hists); free(edge_rad);
    return 0;
}

int oracle_count(int cross, int64_t na, const double *ax, const double *ay,
                 const double *az, int64_t nb, const double *bx, const double *by,
                 const double *bz, int32_t nbins, const double *edges_deg,
                 int64_t row_begin, int64_t row_end, int nthreads, uint64_t *out)
{
    return count_pairs(cross, 0, na, ax, ay, az, nb, bx, by, bz, nbins, edges_deg,
                       row_begin, row_end, nthreads, out);
}

/*
 * The same histogram over 3-D separations (the spatial correlation function
 * the paper's method extends to, Section 1): points are given as Cartesian
 * coordinates (comoving positions, any length unit), the separation of a pair
 * is pair_distance above, and edges are distances in the same unit; slot s
 * is the number of edges e_k with e_k <= r.
 */
int oracle_count3d(int cross, int64_t na, const double *ax, const double *ay,
                   const double *az, int64_t nb, const double *bx, const double *by,
                   const double *bz, int32_t nbins, const double *edges,
                   int64_t row_begin, int64_t row_end, int nthreads, uint64_t *out)
{
    return count_pairs(cross, 1, na, ax, ay, az, nb, bx, by, bz, nbins, edges,
                       row_begin, row_end, nthreads, out);
}

/*
 * Pair counts with jackknife regions: every point carries a region label in
 * [0, nreg).  out_total (nbins+2 slots) is the histogram of oracle_count over
 * all pairs; out_touch (nreg x (nbins+2)) row r counts the pairs with at
 * least one member in region r (a pair whose members share a region counts
 * once there).  Removing region r from both catalogs removes exactly the
 * pairs of row r, so the delete-one jackknife histograms are
 * out_total - out_touch[r].  Single-threaded; returns 0, or -1 on bad
 * arguments (a label out of range included).
 */
static int count_regions(int cross, int metric, int64_t na, const double *ax, const double *ay,
                         const double *az, const int32_t *ra, int64_t nb, const double *bx,
                         const double *by, const double *bz, const int32_t *rb, int32_t nbins,
                         const double *edges, int32_t nreg, uint64_t *out_total,
                         uint64_t *out_touch)
{
    if (nbins < 1 || nreg < 1 || na < 0 || (cross && nb < 0) || !out_total || !out_touch)
        return -1;
    for (int64_t i = 0; i < na; ++i)
        if (ra[i] < 0 || ra[i] >= nreg)
            return -1;
    if (cross)
        for (int64_t j = 0; j < nb; ++j)
            if (rb[j] < 0 || rb[j] >= nreg)
                return -1;
    const double deg = M_PI / 180.0;
    const int nedges = nbins + 1;
    const int nslots = nbins + 2;
    double *edge_rad = (double *)malloc(sizeof(double) * (size_t)nedges);
    if (!edge_rad)
        return -1;
    for (int k = 0; k < nedges; ++k)
        edge_rad[k] = metric ? edges[k] : edges[k] * deg;
    memset(out_total, 0, sizeof(uint64_t) * (size_t)nslots);
    memset(out_touch, 0, sizeof(uint64_t) * (size_t)nreg * (size_t)nslots);
    for (int64_t i = 0; i < na; ++i) {
        const int64_t j0 = cross ? 0 : i + 1;
        const int64_t jn = cross ? nb : na;
        for (int64_t j = j0; j < jn; ++j) {
            const double xj = cross ? bx[j] : ax[j];
            const double yj = cross ? by[j] : ay[j];
            const double zj = cross ? bz[j] : az[j];
            const int32_t rj = cross ? rb[j] : ra[j];
            const double t = metric ? pair_distance(ax[i], ay[i], az[i], xj, yj, zj)
                                    : pair_angle(ax[i], ay[i], az[i], xj, yj, zj);
            const int s = slot_of(t, edge_rad, nedges);
            out_total[s] += 1;
            out_touch[(size_t)ra[i] * (size_t)nslots + (size_t)s] += 1;
            if (rj != ra[i])
                out_touch[(size_t)rj * (size_t)nslots + (size_t)s] += 1;
        }
    }
    free(edge_rad);
    return 0;
}

int oracle_count_regions(int cross, int64_t na, const double *ax, const double *ay,
                         const double *az, const int32_t *ra, int64_t nb, const double *bx,
                         const double *by, const double *bz, const int32_t *rb, int32_t nbins,
                         const double *edges_deg, int32_t nreg, uint64_t *out_total,
                         uint64_t *out_touch)
{
    return count_regions(cross, 0, na, ax, ay, az, ra, nb, bx, by, bz, rb, nbins, edges_deg, nreg,
                         out_total, out_touch);
}

/* The same for 3-D catalogs: separations are the distances of
 * oracle_count3d, edges distances. */
int oracle_count_regions3d(int cross, int64_t na, const double *ax, const double *ay,
                           const double *az, const int32_t *ra, int64_t nb, const double *bx,
                           const double *by, const double *bz, const int32_t *rb, int32_t nbins,
                           const double *edges, int32_t nreg, uint64_t *out_total,
                           uint64_t *out_touch)
{
    return count_regions(cross, 1, na, ax, ay, az, ra, nb, bx, by, bz, rb, nbins, edges, nreg,
                         out_total, out_touch);
}

/* Slot of each listed pair (i-th entry pairs point a_i with point b_i);
 * used for probes placed next to bin edges. */
int oracle_pair_slots(int64_t n, const double *ax, const double *ay, const double *az,
                      const double *bx, const double *by, const double *bz,
                      int32_t nbins, const double *edges_deg, int32_t *slots)
{
    if (nbins < 1 || n < 0)
        return -1;
    const double deg = M_PI / 180.0;
    int nedges = nbins + 1;
    double *edge_rad = (double *)malloc(sizeof(double) * (size_t)nedges);
    if (!edge_rad)
        return -1;
    for (int k = 0; k < nedges; ++k)
        edge_rad[k] = edges_deg[k] * deg;
    for (int64_t i = 0; i < n; ++i) {
        double t = pair_angle(ax[i], ay[i], az[i], bx[i], by[i], bz[i]);
        slots[i] = slot_of(t, edge_rad, nedges);
    }
    free(edge_rad);
    return 0;
}

/* The angle itself (radians) for listed pairs, for pin tests. */
int oracle_pair_angles(int64_t n, const double *ax, const double *ay, const double *az,
                       const double *bx, const double *by, const double *bz, double *theta)
{
    for (int64_t i = 0; i < n; ++i)
        theta[i] = pair_angle(ax[i], ay[i], az[i], bx[i], by[i], bz[i]);
    return 0;
}

/* 3-D distance of each listed pair (a_i, b_i), as pair_distance. */
int oracle_pair_distances(int64_t n, const double *ax, const double *ay, const double *az,
                          const double *bx, const double *by, const double *bz, double *out)
{
    if (n < 0 || !out)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        out[i] = pair_distance(ax[i], ay[i], az[i], bx[i], by[i], bz[i]);
    return 0;
}
