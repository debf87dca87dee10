// C ABI of libtpcf.so: contexts, catalogs, pair counting, batches, jobs,
// Landy-Szalay.
//
// Host side of the pair-counting path.  Everything here runs on the host:
// argument checks, the unit vectors of uploaded catalogs, the edge compiler
// (edges.cpp), the work-unit plan, device-memory accounting, and the
// launches.  Every pair is counted on the GPU by the kernels in kernels.hip;
// there is no host fallback.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "edges.h"
#include "internal.h"
#include "tpcf.h"

using namespace tpcf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? TPCF_E_NOMEM : TPCF_E_HIP,            \
                        std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define TRY(expr)          \
    do {                   \
        int r_ = (expr);   \
        if (r_)            \
            return r_;     \
    } while (0)

constexpr double kMaxDelta = 9.5367431640625e-07;   // 2^-20
constexpr double kMaxCoord3d = 1125899906842624.0;    // 2^50: largest |coordinate| of a 3-D catalog
constexpr int kPoolStreams = 4;

// Launch shape, set by tpcf_set_tuning (the autotuner) or left at defaults.
// Zero fields take the defaults, which are the shapes the autotuner picked on
// the large octant workload: 4 rows per lane, 16 histogram copies,
// 4096-column units, and clamped cell tables of up to 24 KB.
struct Tuning {
    int rows_per_lane = 0;   // 2 or 4
    int hist_copies = 0;     // 4..32, at most what the slot count allows
    int max_cols = 0;        // largest column range of a work unit
    int blocks_per_cu = 0;   // 0: the blocks that fit at once
    int lut_bytes = 0;       // largest cell table
    int lut_direct = 0;      // 1: FP32 byte tables in the direct layout
    int prune = 0;           // 1: exact tile pruning
};

int rows_per_lane_of(const Tuning &t) { return t.rows_per_lane ? t.rows_per_lane : 4; }

int max_cols_of(const Tuning &t) { return t.max_cols ? t.max_cols : 4096; }

// Device memory of one context, with an optional budget on the total.
struct MemAccount {
    int64_t used = 0;
    int64_t budget = 0;   // 0: unlimited
};

int dev_alloc(MemAccount &m, void **p, size_t bytes) {
    if (m.budget > 0 && m.used + (int64_t)bytes > m.budget) {
        char buf[160];
        snprintf(buf, sizeof buf, "allocation of %zu bytes exceeds the HBM budget (%lld of %lld in use)",
                 bytes, (long long)m.used, (long long)m.budget);
        return fail(TPCF_E_BUDGET, buf);
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(TPCF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    m.used += (int64_t)bytes;
    return TPCF_OK;
}

void dev_free(MemAccount &m, void *p, size_t bytes) {
    if (p) {
        (void)hipFree(p);
        m.used -= (int64_t)bytes;
    }
}

// Device buffer that grows on demand.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    int ensure(MemAccount &m, size_t bytes) {
        if (bytes <= cap && p)
            return TPCF_OK;
        release(m);
        size_t want = bytes < 256 ? 256 : bytes;
        TRY(dev_alloc(m, &p, want));
        cap = want;
        return TPCF_OK;
    }
    void release(MemAccount &m) {
        dev_free(m, p, cap);
        p = nullptr;
        cap = 0;
    }
};

struct Catalog {
    int64_t n = 0;
    double *d64 = nullptr;      // x[n], y[n], z[n]
    float *d32 = nullptr;       // x[n], y[n], z[n]
    size_t bytes64 = 0, bytes32 = 0;
    bool owns64 = true;
    bool owns32 = true;
    double delta = 0;           // bound on | |v|^2 - 1 |
    std::vector<int64_t> order; // stored row r holds upload row order[r] (empty: identity)
    double *dcaps = nullptr;    // bounding caps of aligned 64-point groups, built on first use
    size_t bytes_caps = 0;
    // jackknife regions: stored rows of region r are [reg_start[r], reg_start[r+1])
    int32_t nreg = 0;
    std::vector<int64_t> reg_start;
    // 0: unit vectors on the sky; 1: Cartesian points in 3-D (rmax bounds
    // their FP64 norms, for the FP32 band)
    int metric = 0;
    double rmax = 0;
    double band_param() const { return metric ? rmax : delta; }
};

struct Compiled {
    EdgeTables edges;
    DevBuf dD, dE, dqlo, dqhi, dlut, dErad;
    CellTable cells;
    Band32 band;
    // Angular FP32: cell table of the dot-product key q' = fl(2 - 2p), packed
    // after the chord table (at byte plut_src of dlut); no cells otherwise.
    CellTable pcells;
    int plut_src = 0;
    int precision = 0;
    int entry_bytes = 2;   // 1: byte entries (0x80 | k, 0xFF), 2: 16-bit codes
    double delta = 0;      // norm bound of the band (3-D: rmax)
    int metric = 0;
};

struct Plan {
    std::vector<Unit> units;
    DevBuf dunits;
    uint64_t pairs = 0;
};

// Launch resources of one stream.  Work on one stream runs in order, so the
// buffers are reused by consecutive launches on it.
struct Workspace {
    hipStream_t stream = nullptr;
    bool own = false;
    DevBuf copies;   // kGlobalCopies x nslots u64
    DevBuf out;      // kMaxSlots u64
    DevBuf stats;    // kStats u64
    DevBuf touch;    // nreg x kGlobalCopies x nslots u64 (jackknife regions)
    DevBuf tout;     // nreg x nslots u64
    int inflight = 0;
};

// A validated counting request.
struct Request {
    int kind = 0;
    bool auto_pairs = false;
    int32_t cat_a = -1, cat_b = -1;
    const Catalog *A = nullptr, *B = nullptr;
    int64_t rb = 0, re = 0;
    int nbins = 0, precision = 0;
    Compiled *cp = nullptr;
    Plan *plan = nullptr;
    uint64_t pairs = 0;
    int metric = 0;
    std::string cache_key;   // RR requests: key of the result cache
};

struct AsyncJob {
    Request req;
    int ws = -1;
    hipEvent_t ev = nullptr;
    uint64_t *hres = nullptr;   // pinned: kMaxSlots results, then the cancel word
    volatile int *hcancel = nullptr;
    bool cancelled = false;
    bool ready = false;          // result known at submit (result cache)
    std::vector<uint64_t> result;
};

struct BatchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevBuf copies, out, jobs, units;
};

}  // namespace

struct tpcf_ctx {
    int device = 0;
    MemAccount mem;
    Workspace main;                      // the context stream
    std::vector<Workspace> pool;         // streams for submitted jobs
    int32_t next_id = 1;
    int64_t next_job = 1;
    std::map<int32_t, Catalog> cats;
    std::map<std::string, std::unique_ptr<Compiled>> compiled;
    std::map<std::string, std::unique_ptr<Plan>> plans;
    std::map<int64_t, AsyncJob> jobs;
    std::map<std::string, std::unique_ptr<BatchGraph>> graphs;
    std::map<std::string, std::vector<uint64_t>> result_cache;
    // pinned result buffers of retired jobs, reused by later submits:
    // hipHostFree would wait for the whole device at every completion
    std::vector<uint64_t *> pinned_free;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    uint64_t pairs_since_reset = 0;
    Tuning tune;
};

namespace {

int set_device(tpcf_ctx *ctx) {
    HIP_TRY(hipSetDevice(ctx->device));
    return TPCF_OK;
}

int sync_all(tpcf_ctx *ctx) {
    HIP_TRY(hipStreamSynchronize(ctx->main.stream));
    for (auto &w : ctx->pool)
        HIP_TRY(hipStreamSynchronize(w.stream));
    return TPCF_OK;
}

int init_workspace(tpcf_ctx *ctx, Workspace &w, hipStream_t borrowed) {
    if (borrowed) {
        w.stream = borrowed;
        w.own = false;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
        w.own = true;
    }
    TRY(w.stats.ensure(ctx->mem, sizeof(unsigned long long) * kStats));
    HIP_TRY((hipError_t)tpcf_launch_zero_u64((unsigned long long *)w.stats.p, kStats, w.stream));
    return TPCF_OK;
}

void free_workspace(tpcf_ctx *ctx, Workspace &w) {
    w.copies.release(ctx->mem);
    w.touch.release(ctx->mem);
    w.tout.release(ctx->mem);
    w.out.release(ctx->mem);
    w.stats.release(ctx->mem);
    if (w.own && w.stream)
        (void)hipStreamDestroy(w.stream);
    w.stream = nullptr;
}

void free_graph(tpcf_ctx *ctx, BatchGraph &g) {
    if (g.exec)
        (void)hipGraphExecDestroy(g.exec);
    if (g.graph)
        (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    g.copies.release(ctx->mem);
    g.out.release(ctx->mem);
    g.jobs.release(ctx->mem);
    g.units.release(ctx->mem);
}

void drop_graphs(tpcf_ctx *ctx) {
    for (auto &kv : ctx->graphs)
        free_graph(ctx, *kv.second);
    ctx->graphs.clear();
}

// Bound on the exact | |v|^2 - 1 | of FP64 vectors: the largest computed
// deviation plus the rounding of computing it (a few units of 2^-53).
double norm_bound(const double *x, const double *y, const double *z, int64_t n, bool *finite) {
    double m = 0.0;
    *finite = true;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i])) {
            *finite = false;
            return HUGE_VAL;
        }
        double t = x[i] * x[i];
        double u = y[i] * y[i];
        double v = z[i] * z[i];
        double r = (t + u) + v;
        double dev = fabs(r - 1.0);
        if (dev > m)
            m = dev;
    }
    return m + 4.0 * ldexp(1.0, -53);
}

// Spatially coherent storage order: sort the points along a Morton (Z-order)
// curve of their unit vectors, 21 bits per coordinate.  Neighbouring rows are
// then close on the sky, so the 64 lanes of a wavefront see nearly the same
// separation to each column point.  Counts do not depend on the order.
uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

uint64_t quant21(double c, double lo = -1.0, double hi = 1.0) {
    double t = (c - lo) / (hi - lo) * 2097151.0;
    if (!(t > 0.0))
        return 0;
    if (t > 2097151.0)
        return 2097151;
    return (uint64_t)t;
}

// Host threads for catalog preparation: large catalogs are split into
// contiguous chunks, at most 16, none smaller than 32768 points.  Every
// per-point result is computed exactly as in a serial loop, so the stored
// catalog does not depend on the thread count.
int host_threads(int64_t n) {
    const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
    return (int)std::max<int64_t>(1, std::min<int64_t>({hw, 16, n / 32768}));
}

template <typename F>
void parallel_chunks(int64_t n, int nt, F fn) {
    if (nt <= 1) {
        fn(0, 0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back(fn, t, n * t / nt, n * (t + 1) / nt);
    for (auto &t : th)
        t.join();
}

// Stored order: Morton order of the unit vectors, grouped by region first
// when labels are given (so each region is a contiguous range of rows).  The
// key ends in the point index, so it is a strict total order: chunks sorted
// on their own and merged pairwise give the one sorted sequence.
std::vector<int64_t> morton_order(const double *x, const double *y, const double *z, int64_t n,
                                  const int32_t *region = nullptr, double lo = -1.0, double hi = 1.0) {
    using Key = std::tuple<int32_t, uint64_t, int64_t>;
    std::vector<Key> k((size_t)n), tmp;
    const int nt = host_threads(n);
    std::vector<int64_t> bound((size_t)nt + 1);
    for (int t = 0; t <= nt; ++t)
        bound[t] = n * t / nt;
    parallel_chunks(n, nt, [&](int, int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            k[i] = std::make_tuple(region ? region[i] : 0,
                                   spread3(quant21(x[i], lo, hi)) | spread3(quant21(y[i], lo, hi)) << 1 |
                                       spread3(quant21(z[i], lo, hi)) << 2,
                                   i);
        std::sort(k.begin() + b, k.begin() + e);
    });
    if (nt > 1)
        tmp.resize((size_t)n);
    // merge rounds: runs of w chunks become runs of 2w chunks
    for (int w = 1; w < nt; w *= 2) {
        std::vector<std::thread> th;
        for (int t = 0; t < nt; t += 2 * w) {
            const int64_t b = bound[t], m = bound[std::min(t + w, nt)], e = bound[std::min(t + 2 * w, nt)];
            th.emplace_back([&, b, m, e] {
                std::merge(k.begin() + b, k.begin() + m, k.begin() + m, k.begin() + e, tmp.begin() + b);
            });
        }
        for (auto &t : th)
            t.join();
        k.swap(tmp);
    }
    std::vector<int64_t> order((size_t)n);
    parallel_chunks(n, nt, [&](int, int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            order[i] = std::get<2>(k[i]);
    });
    return order;
}

int add_catalog(tpcf_ctx *ctx, const double *x, const double *y, const double *z, int64_t n,
                int32_t *out_cat, const int32_t *region = nullptr, int32_t nreg = 0, int metric = 0) {
    if (!out_cat)
        return fail(TPCF_E_INVALID, "out_cat is NULL");
    if (n < 0 || n > (int64_t)0x7fffffff - 1024)
        return fail(TPCF_E_INVALID, "catalog size out of range");
    if (n > 0 && (!x || !y || !z))
        return fail(TPCF_E_INVALID, "coordinate array is NULL");
    if (region) {
        if (nreg < 1 || nreg > TPCF_MAX_REGIONS)
            return fail(TPCF_E_INVALID, "nreg must be in [1, TPCF_MAX_REGIONS]");
        for (int64_t i = 0; i < n; ++i)
            if (region[i] < 0 || region[i] >= nreg)
                return fail(TPCF_E_INVALID, "region labels must lie in [0, nreg)");
    }
    Catalog c;
    c.n = n;
    c.metric = metric;
    double lo = -1.0, hi = 1.0;
    if (metric == 0) {
        bool finite = true;
        double delta = n > 0 ? norm_bound(x, y, z, n, &finite) : 0.0;
        if (!finite)
            return fail(TPCF_E_INVALID, "coordinates must be finite");
        if (delta > kMaxDelta)
            return fail(TPCF_E_INVALID, "unit vectors must satisfy | |v|^2 - 1 | <= 2^-20");
        c.delta = delta;
    } else {
        // 3-D: finite coordinates within 2^50; rmax bounds every FP64 norm
        // (the square root of the largest squared norm, widened)
        double r2 = 0.0;
        lo = HUGE_VAL;
        hi = -HUGE_VAL;
        for (int64_t i = 0; i < n; ++i) {
            const double v[3] = {x[i], y[i], z[i]};
            for (double w : v) {
                if (!isfinite(w) || fabs(w) > kMaxCoord3d)
                    return fail(TPCF_E_INVALID, "3-D coordinates must be finite with |c| <= 2^50");
                lo = std::min(lo, w);
                hi = std::max(hi, w);
            }
            r2 = std::max(r2, (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        }
        c.rmax = sqrt(r2) * (1.0 + ldexp(1.0, -40)) + ldexp(1.0, -1000);
        if (!(hi > lo)) {
            lo = n > 0 ? lo - 1.0 : -1.0;
            hi = lo + 2.0;
        }
    }
    TRY(set_device(ctx));
    c.order = morton_order(x, y, z, n, region, lo, hi);
    if (region) {
        c.nreg = nreg;
        c.reg_start.assign((size_t)nreg + 1, 0);
        for (int64_t i = 0; i < n; ++i)
            ++c.reg_start[(size_t)region[i] + 1];
        for (int32_t r = 0; r < nreg; ++r)
            c.reg_start[(size_t)r + 1] += c.reg_start[(size_t)r];
    }
    size_t alloc_n = (size_t)(n > 0 ? n : 1);
    std::vector<double> h64(3 * alloc_n, 0.0);
    std::vector<float> h32(3 * alloc_n, 0.0f);
    parallel_chunks(n, host_threads(n), [&](int, int64_t b, int64_t e) {
        for (int64_t r = b; r < e; ++r) {
            const int64_t i = c.order[r];
            h64[r] = x[i];
            h64[alloc_n + r] = y[i];
            h64[2 * alloc_n + r] = z[i];
            h32[r] = (float)x[i];
            h32[alloc_n + r] = (float)y[i];
            h32[2 * alloc_n + r] = (float)z[i];
        }
    });
    c.bytes64 = sizeof(double) * 3 * alloc_n;
    c.bytes32 = sizeof(float) * 3 * alloc_n;
    TRY(dev_alloc(ctx->mem, (void **)&c.d64, c.bytes64));
    int rc = dev_alloc(ctx->mem, (void **)&c.d32, c.bytes32);
    if (rc) {
        dev_free(ctx->mem, c.d64, c.bytes64);
        return rc;
    }
    // blocking copies: the host vectors go out of scope on return
    hipError_t e = hipMemcpy(c.d64, h64.data(), c.bytes64, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c.d32, h32.data(), c.bytes32, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(ctx->mem, c.d64, c.bytes64);
        dev_free(ctx->mem, c.d32, c.bytes32);
        return fail(TPCF_E_HIP, std::string("upload: ") + hipGetErrorString(e));
    }
    int32_t id = ctx->next_id++;
    ctx->cats[id] = std::move(c);
    *out_cat = id;
    return TPCF_OK;
}

std::string edges_key(const double *edges, int nbins, int precision, double delta, int metric,
                      const Tuning &t) {
    std::string k((const char *)edges, sizeof(double) * (size_t)(nbins + 1));
    k.append((const char *)&precision, sizeof precision);
    k.append((const char *)&metric, sizeof metric);
    if (precision == TPCF_FP32_CHORD || metric)
        k.append((const char *)&delta, sizeof delta);
    k.append((const char *)&t.lut_bytes, sizeof t.lut_bytes);
    k.append((const char *)&t.lut_direct, sizeof t.lut_direct);
    k.append((const char *)&t.hist_copies, sizeof t.hist_copies);   // sizes a wrapped table's free piece
    k.append((const char *)&t.prune, sizeof t.prune);               // pruned: no dot-product tables
    return k;
}

template <typename T>
int upload_blocking(MemAccount &m, DevBuf &b, const std::vector<T> &v) {
    TRY(b.ensure(m, sizeof(T) * (v.size() ? v.size() : 1)));
    if (!v.empty())
        HIP_TRY(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return TPCF_OK;
}

void free_compiled(tpcf_ctx *ctx, Compiled &c) {
    c.dD.release(ctx->mem);
    c.dE.release(ctx->mem);
    c.dqlo.release(ctx->mem);
    c.dqhi.release(ctx->mem);
    c.dlut.release(ctx->mem);
    c.dErad.release(ctx->mem);
}

int hist_copies_of(const Tuning &t, int nslots);

// Cell entries as the kernels read them, appended to *out: one byte (slot,
// 0x80 | k, 0xFF) or the 16-bit codes.
void pack_cells(const std::vector<uint16_t> &src, int entry_bytes, std::vector<uint8_t> *out) {
    const size_t at = out->size();
    if (entry_bytes == 1) {
        out->resize(at + src.size());
        for (size_t i = 0; i < src.size(); ++i) {
            const uint16_t v = src[i];
            (*out)[at + i] = v == kMulti ? 0xFF : (v & kMedium) ? (uint8_t)(0x80 | (v & 0x7F)) : (uint8_t)v;
        }
    } else {
        out->resize(at + src.size() * 2);
        memcpy(out->data() + at, src.data(), src.size() * 2);
    }
}

// Host part of the edge compiler: thresholds, FP32 band and cell table of
// one edges array for the given tuning, and the table packed as the kernels
// read it.  Allocates no device memory.
int compile_host(const Tuning &tune, const double *edges, int nbins, int precision, double delta, int metric,
                 Compiled *c, std::vector<uint8_t> *packed, std::vector<float> *qlo, std::vector<float> *qhi) {
    std::string err;
    if (!(metric ? compile_edges_3d(edges, nbins, &c->edges, &err) : compile_edges(edges, nbins, &c->edges, &err)))
        return fail(TPCF_E_INVALID, err);
    c->precision = precision;
    c->delta = delta;
    c->metric = metric;
    const int nslots = nbins + 2;
    c->entry_bytes = nslots <= kMaxSlots8 ? 1 : 2;
    // FP32: by default the table fits kLdsTarget with the histograms and
    // edges and, with the angular dot-product path, its table (kDotLutBytes)
    // and the column staging (kStageBytes).  Pruned angular kernels take the
    // chord path alone (the blocks they evaluate lie across edges) and give
    // the chord table the room.
    const bool angular32 = !metric && precision == TPCF_FP32_CHORD;
    const bool dot = angular32 && !tune.prune;
    const int aux = aux_lds_bytes(nslots, hist_copies_of(tune, nslots), nbins + 1);
    const int pbytes = dot ? kDotLutBytes : 0;
    const int extra = dot ? pbytes + kStageBytes + 32 : 0;
    int table_bytes = tune.lut_bytes ? tune.lut_bytes : kMaxLutBytes;
    if (precision == TPCF_FP32_CHORD && !tune.lut_bytes)
        table_bytes = std::min(table_bytes, std::max(4096, (kLdsTarget - aux - extra) & ~15));
    const int max_cells = std::min(table_bytes, kMaxLutBytes) / c->entry_bytes;
    qlo->assign(c->edges.D.size(), 0.0f);
    qhi->assign(c->edges.D.size(), 0.0f);
    if (metric && precision == TPCF_FP32_CHORD) {
        c->band = make_band32_3d(c->edges, delta);
        c->cells = make_cells32_top(c->edges, c->band, qtop_key_3d(delta), max_cells);
        *qlo = c->band.qlo;
        *qhi = c->band.qhi;
    } else if (metric) {
        const double top = 4.0 * delta * delta * (1.0 + ldexp(1.0, -10));
        c->cells = make_cells64(c->edges, max_cells, top > 1e-300 ? top : 1e-300);
    } else if (precision == TPCF_FP32_CHORD) {
        c->band = make_band32(c->edges, delta);
        if (c->entry_bytes == 1 && tune.lut_direct) {
            Band32 fb = make_band32(c->edges, delta, floor_for(c->band));
            const int wrap_bytes = tune.lut_bytes ? tune.lut_bytes : kWrapLutBytes - extra;
            c->cells = make_cells32_wrap(c->edges, fb, delta, wrap_bytes, aux);
            if (!c->cells.cells.empty())
                c->band = fb;
        }
        if (c->cells.cells.empty())
            c->cells = make_cells32(c->edges, c->band, delta, max_cells);
        *qlo = c->band.qlo;
        *qhi = c->band.qhi;
        // the dot-product key's table and the per-pair band in p, after the
        // chord band's entries in qlo / qhi
        if (dot) {
            c->pcells = make_cells32_top(c->edges, make_band_dot32(c->edges, delta), dot_top_key(delta),
                                         pbytes / c->entry_bytes);
            std::vector<float> plo, phi;
            make_pband32(c->edges, delta, &plo, &phi);
            qlo->insert(qlo->end(), plo.begin(), plo.end());
            qhi->insert(qhi->end(), phi.begin(), phi.end());
        }
    } else {
        c->cells = make_cells64(c->edges, max_cells);
    }
    packed->clear();
    pack_cells(c->cells.direct ? c->cells.image : c->cells.cells, c->entry_bytes, packed);
    if (!c->pcells.cells.empty()) {
        packed->resize((packed->size() + 15) & ~(size_t)15, 0);
        c->plut_src = (int)packed->size();
        pack_cells(c->pcells.cells, c->entry_bytes, packed);
    }
    return TPCF_OK;
}

int get_compiled(tpcf_ctx *ctx, const double *edges, int nbins, int precision, double delta, int metric,
                 Compiled **out) {
    std::string key = edges_key(edges, nbins, precision, delta, metric, ctx->tune);
    auto it = ctx->compiled.find(key);
    if (it != ctx->compiled.end()) {
        *out = it->second.get();
        return TPCF_OK;
    }
    if (ctx->compiled.size() >= 64) {   // bounded cache: drop all (in-flight work first)
        TRY(sync_all(ctx));
        drop_graphs(ctx);
        for (auto &kv : ctx->compiled)
            free_compiled(ctx, *kv.second);
        ctx->compiled.clear();
    }
    auto c = std::make_unique<Compiled>();
    std::vector<uint8_t> packed;
    std::vector<float> qlo, qhi;
    TRY(compile_host(ctx->tune, edges, nbins, precision, delta, metric, c.get(), &packed, &qlo, &qhi));
    int rc;
    if ((rc = upload_blocking(ctx->mem, c->dD, c->edges.D)) || (rc = upload_blocking(ctx->mem, c->dE, c->edges.E)) ||
        (rc = upload_blocking(ctx->mem, c->dqlo, qlo)) || (rc = upload_blocking(ctx->mem, c->dqhi, qhi)) ||
        (rc = upload_blocking(ctx->mem, c->dlut, packed)) ||
        (rc = upload_blocking(ctx->mem, c->dErad, c->edges.edge_rad))) {
        free_compiled(ctx, *c);
        return rc;
    }
    *out = c.get();
    ctx->compiled[key] = std::move(c);
    return TPCF_OK;
}

// Column chunk width of a plan: aim for >= ~4096 units on big requests,
// within [256, max_cols], but wide enough that the unit list stays below
// kMaxUnits (about 0.8 GB of units; catalogs of 1e8 points would otherwise
// need tens of GB of them).
constexpr double kMaxUnits = 16777216.0;

int64_t chunk_width(uint64_t pairs, int64_t T, int64_t max_cols, double max_units = kMaxUnits) {
    int64_t bj = (int64_t)((double)pairs / 4096.0 / (double)T);
    bj = (bj + 255) / 256 * 256;
    if (bj > max_cols)
        bj = max_cols;
    if (bj < 256)
        bj = 256;
    const double need = (double)pairs / (double)T / max_units;   // columns per unit for max_units units
    if ((double)bj < need)
        bj = ((int64_t)need + 256) / 256 * 256;
    return bj;
}

// Work units.  DR: every row tile against column chunks of the B catalog.
// DD/RR: every row tile [i0, i1) against j in [i0, n): one masked unit for the
// diagonal block [i0, i0 + T), then unmasked chunks from i0 + T on.
Unit mk_unit(int64_t i0, int64_t i1, int64_t j0, int64_t j1, int64_t row_lo, int64_t col_lo, int32_t reg_a,
             int32_t reg_b) {
    Unit u;
    memset(&u, 0, sizeof u);
    u.i0 = (int32_t)i0;
    u.i1 = (int32_t)i1;
    u.j0 = (int32_t)j0;
    u.j1 = (int32_t)j1;
    u.row_lo = (int32_t)row_lo;
    u.col_lo = (int32_t)col_lo;
    u.reg_a = reg_a;
    u.reg_b = reg_b;
    return u;
}

Plan make_plan(bool auto_pairs, int64_t na, int64_t nb, int64_t rb, int64_t re, int64_t T,
               int64_t max_cols, double max_units = kMaxUnits) {
    Plan p;
    uint64_t pairs = 0;
    if (auto_pairs) {
        // sum over i in [rb, re) of (na - 1 - i)
        const int64_t cnt = re - rb;
        pairs = (uint64_t)cnt * (uint64_t)(na - 1) - (uint64_t)((rb + re - 1) * cnt / 2);
    } else {
        pairs = (uint64_t)(re - rb) * (uint64_t)nb;
    }
    p.pairs = pairs;
    const int64_t bj = chunk_width(pairs, T, max_cols, max_units);
    // Row tiles start at rb (valid rows from row_lo = rb).
    // Column chunks lie on a common grid of multiples of bj, so units of
    // different row tiles cover the same column ranges; the list is ordered
    // column chunk first, so the units in flight at any time (a grid-stride
    // window of consecutive units) share their columns and the column data
    // stays in each XCD's L2.
    const int64_t i_first = rb;
    if (auto_pairs) {
        for (int64_t i0 = i_first; i0 < re; i0 += T) {
            const int64_t i1 = i0 + T < re ? i0 + T : re;
            const int32_t lo = (int32_t)(i0 > rb ? i0 : rb);
            const int64_t dend = i0 + T < na ? i0 + T : na;
            if (lo + 1 < dend)
                p.units.push_back(mk_unit(i0, i1, i0, dend, lo, i0, -1, -1));
            int64_t j0 = dend;
            while (j0 < na) {
                // up to the next multiple of bj; a short first piece joins the next chunk
                int64_t j1 = (j0 / bj + 1) * bj;
                if (j1 - j0 < 256)
                    j1 += bj;
                if (j1 > na)
                    j1 = na;
                p.units.push_back(mk_unit(i0, i1, j0, j1, lo, j0, -1, -1));
                j0 = j1;
            }
        }
        std::sort(p.units.begin(), p.units.end(), [](const Unit &x, const Unit &y) {
            return x.j1 != y.j1 ? x.j1 < y.j1 : x.i0 < y.i0;
        });
    } else {
        for (int64_t j0 = 0; j0 < nb; j0 += bj) {
            const int64_t j1 = j0 + bj < nb ? j0 + bj : nb;
            for (int64_t i0 = i_first; i0 < re; i0 += T) {
                const int64_t i1 = i0 + T < re ? i0 + T : re;
                const int32_t lo = (int32_t)(i0 > rb ? i0 : rb);
                p.units.push_back(mk_unit(i0, i1, j0, j1, lo, j0, -1, -1));
            }
        }
    }
    return p;
}

// Work units of a whole-catalog request with jackknife regions: no unit
// crosses a region boundary on either side, and each carries its two region
// ids.  Row tiles are cut at region ends (starting at the region start);
// columns are cut on the bj grid and at region starts.  Auto-pairs: per row
// tile a diagonal unit over the tile's own columns, then the columns after
// it.  Ordered column chunk first.
Plan make_plan_regions(bool auto_pairs, int64_t na, int64_t nb, int64_t T, int64_t max_cols,
                       const std::vector<int64_t> &sa, const std::vector<int64_t> &sb) {
    Plan p;
    p.pairs = auto_pairs ? (uint64_t)na * (uint64_t)(na > 0 ? na - 1 : 0) / 2 : (uint64_t)na * (uint64_t)nb;
    const int64_t bj = chunk_width(p.pairs, T, max_cols);
    const int nra = (int)sa.size() - 1;
    auto region_of = [](const std::vector<int64_t> &st, int64_t j) {
        return (int32_t)(std::upper_bound(st.begin(), st.end(), j) - st.begin() - 1);
    };
    // the column pieces [c0, c1) after column j: bj grid and region starts
    auto next_cut = [&](const std::vector<int64_t> &st, int64_t j, int64_t n) {
        int64_t c = (j / bj + 1) * bj;
        const auto it = std::upper_bound(st.begin(), st.end(), j);
        if (it != st.end() && *it < c)
            c = *it;
        return c < n ? c : n;
    };
    struct Tile { int64_t i0, i1, lo; int32_t reg; };
    std::vector<Tile> tiles;
    for (int r = 0; r < nra; ++r) {
        const int64_t s0 = sa[(size_t)r], s1 = sa[(size_t)r + 1];
        if (s0 == s1)
            continue;   // empty region
        for (int64_t i0 = s0; i0 < s1; i0 += T)
            tiles.push_back(Tile{i0, i0 + T < s1 ? i0 + T : s1, i0 > s0 ? i0 : s0, (int32_t)r});
    }
    if (auto_pairs) {
        for (const Tile &t : tiles) {
            if (t.lo + 1 < t.i1)
                p.units.push_back(mk_unit(t.i0, t.i1, t.i0, t.i1, t.lo, t.i0, t.reg, t.reg));
            for (int64_t j = t.i1; j < na;) {
                const int64_t c1 = next_cut(sa, j, na);
                p.units.push_back(mk_unit(t.i0, t.i1, j, c1, t.lo, j, t.reg, region_of(sa, j)));
                j = c1;
            }
        }
        std::sort(p.units.begin(), p.units.end(), [](const Unit &x, const Unit &y) {
            return x.j1 != y.j1 ? x.j1 < y.j1 : x.i0 < y.i0;
        });
    } else {
        for (int64_t j = 0; j < nb;) {
            const int64_t c1 = next_cut(sb, j, nb);
            const int32_t rj = region_of(sb, j);
            for (const Tile &t : tiles)
                p.units.push_back(mk_unit(t.i0, t.i1, j, c1, t.lo, j, t.reg, rj));
            j = c1;
        }
    }
    return p;
}

int get_plan(tpcf_ctx *ctx, bool auto_pairs, int64_t na, int64_t nb, int64_t rb, int64_t re, Plan **out) {
    // 64 lanes x rows_per_lane rows per wavefront, four wavefronts per tile
    const int64_t T = (int64_t)kWaves * kWaveSize * rows_per_lane_of(ctx->tune);
    const int64_t max_cols = max_cols_of(ctx->tune);
    char buf[160];
    snprintf(buf, sizeof buf, "%d:%lld:%lld:%lld:%lld:%lld:%lld", (int)auto_pairs, (long long)na,
             (long long)nb, (long long)rb, (long long)re, (long long)T, (long long)max_cols);
    auto it = ctx->plans.find(buf);
    if (it != ctx->plans.end()) {
        *out = it->second.get();
        return TPCF_OK;
    }
    if (ctx->plans.size() >= 256) {   // bounded cache: drop all (in-flight work first)
        TRY(sync_all(ctx));
        drop_graphs(ctx);
        for (auto &kv : ctx->plans)
            kv.second->dunits.release(ctx->mem);
        ctx->plans.clear();
    }
    auto p = std::make_unique<Plan>(make_plan(auto_pairs, na, nb, rb, re, T, max_cols));
    TRY(upload_blocking(ctx->mem, p->dunits, p->units));
    *out = p.get();
    ctx->plans[buf] = std::move(p);
    return TPCF_OK;
}

// Plan of a whole-catalog request with jackknife regions (cached like get_plan,
// keyed by the catalog ids, which are never reused).
int get_plan_regions(tpcf_ctx *ctx, bool auto_pairs, int32_t cat_a, int32_t cat_b, const Catalog &A,
                     const Catalog &B, Plan **out) {
    const int64_t T = (int64_t)kWaves * kWaveSize * rows_per_lane_of(ctx->tune);
    const int64_t max_cols = max_cols_of(ctx->tune);
    char buf[160];
    snprintf(buf, sizeof buf, "R%d:%d:%d:%lld:%lld", (int)auto_pairs, (int)cat_a, (int)cat_b, (long long)T,
             (long long)max_cols);
    auto it = ctx->plans.find(buf);
    if (it != ctx->plans.end()) {
        *out = it->second.get();
        return TPCF_OK;
    }
    if (ctx->plans.size() >= 256) {
        TRY(sync_all(ctx));
        drop_graphs(ctx);
        for (auto &kv : ctx->plans)
            kv.second->dunits.release(ctx->mem);
        ctx->plans.clear();
    }
    auto p = std::make_unique<Plan>(
        make_plan_regions(auto_pairs, A.n, B.n, T, max_cols, A.reg_start, B.reg_start));
    if (p->units.size() > (size_t)0x7fffffff / kWaves)
        return fail(TPCF_E_INVALID, "too many work units (region boundaries split the work too finely)");
    TRY(upload_blocking(ctx->mem, p->dunits, p->units));
    *out = p.get();
    ctx->plans[buf] = std::move(p);
    return TPCF_OK;
}

// Histogram copies per wavefront: 32 (conflict-free within a half-wave) while
// the four wavefronts' histograms stay within ~24 KB, fewer for many bins.
int hist_copies_for(int nslots) {
    if ((nslots + 1) <= 48)
        return 32;
    if ((nslots + 1) <= 96)
        return 16;
    if ((nslots + 1) <= 192)
        return 8;
    return 4;
}

// The copies a launch uses: at most what the slot count allows, 16 unless
// the tuning asks for another count.
int hist_copies_of(const Tuning &t, int nslots) {
    const int want = t.hist_copies > 0 ? t.hist_copies : 16;
    return std::min(hist_copies_for(nslots), want);
}

std::string cache_key(int32_t cat, const double *edges, int nbins, int precision, int64_t rb, int64_t re) {
    std::string k((const char *)&cat, sizeof cat);
    k.append((const char *)edges, sizeof(double) * (size_t)(nbins + 1));
    k.append((const char *)&precision, sizeof precision);
    k.append((const char *)&rb, sizeof rb);
    k.append((const char *)&re, sizeof re);
    return k;
}

// Bounding caps of a catalog's aligned 64-point groups, built on the device on
// first use (pruning).
int ensure_caps(tpcf_ctx *ctx, Catalog &c) {
    if (c.dcaps)
        return TPCF_OK;
    const int64_t groups = (c.n + 63) / 64 > 0 ? (c.n + 63) / 64 : 1;
    c.bytes_caps = sizeof(double) * 4 * (size_t)groups;
    TRY(dev_alloc(ctx->mem, (void **)&c.dcaps, c.bytes_caps));
    hipError_t e = hipSuccess;
    if (c.n > 0)
        e = (hipError_t)tpcf_launch_caps64(c.d64, c.n, c.dcaps, c.metric, ctx->main.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->main.stream);
    if (e != hipSuccess) {
        dev_free(ctx->mem, c.dcaps, c.bytes_caps);
        c.dcaps = nullptr;
        return fail(TPCF_E_HIP, std::string("bounding caps: ") + hipGetErrorString(e));
    }
    return TPCF_OK;
}

// Check one request and resolve its catalogs and row range (no allocation).
int validate(tpcf_ctx *ctx, const tpcf_job_desc &d, Request *r) {
    if (d.kind != TPCF_DD && d.kind != TPCF_DR && d.kind != TPCF_RR)
        return fail(TPCF_E_INVALID, "kind must be TPCF_DD, TPCF_DR or TPCF_RR");
    if (d.precision != TPCF_FP32_CHORD && d.precision != TPCF_FP64)
        return fail(TPCF_E_INVALID, "precision must be TPCF_FP32_CHORD or TPCF_FP64");
    if (d.nbins < 1 || d.nbins > 256)
        return fail(TPCF_E_INVALID, "nbins must be in [1, 256]");
    if (!d.bin_edges_deg)
        return fail(TPCF_E_INVALID, "bin_edges_deg is NULL");
    r->kind = d.kind;
    r->auto_pairs = d.kind != TPCF_DR;
    r->precision = d.precision;
    r->nbins = d.nbins;
    auto ia = ctx->cats.find(d.cat_a);
    if (ia == ctx->cats.end())
        return fail(TPCF_E_BADID, "unknown catalog id cat_a");
    r->cat_a = d.cat_a;
    r->A = &ia->second;
    r->B = r->A;
    r->cat_b = -1;
    if (r->auto_pairs) {
        if (d.cat_b != -1)
            return fail(TPCF_E_INVALID, "DD/RR take one catalog: cat_b must be -1");
    } else {
        auto ib = ctx->cats.find(d.cat_b);
        if (ib == ctx->cats.end())
            return fail(TPCF_E_BADID, "unknown catalog id cat_b");
        r->cat_b = d.cat_b;
        r->B = &ib->second;
    }
    int64_t rb = d.row_begin, re = d.row_end;
    if (rb == -1 && re == -1) {
        rb = 0;
        re = r->A->n;
    }
    if (rb < 0 || re < rb || re > r->A->n)
        return fail(TPCF_E_INVALID, "row range must satisfy 0 <= row_begin <= row_end <= n");
    r->rb = rb;
    r->re = re;
    r->metric = r->A->metric;
    if (r->B->metric != r->metric)
        return fail(TPCF_E_INVALID, "a sky catalog and a 3-D catalog cannot be paired");
    return TPCF_OK;
}

// Validate one request and get its tables and plan.  delta_override >= 0
// compiles the FP32 band for that norm bound (shared by every job of a batch)
// instead of the request's own.
int prepare(tpcf_ctx *ctx, const tpcf_job_desc &d, double delta_override, Request *r, bool regions = false) {
    TRY(validate(ctx, d, r));
    const int64_t rb = r->rb, re = r->re;
    TRY(set_device(ctx));
    const double delta = delta_override >= 0 ? delta_override : std::max(r->A->band_param(), r->B->band_param());
    TRY(get_compiled(ctx, d.bin_edges_deg, d.nbins, d.precision, delta, r->metric, &r->cp));
    if (ctx->tune.prune)
        TRY(ensure_caps(ctx, const_cast<Catalog &>(*r->B)));
    r->cache_key.clear();
    if (regions) {
        if (rb != 0 || re != r->A->n)
            return fail(TPCF_E_INVALID, "region counts cover whole catalogs");
        if (r->A->nreg < 1 || r->B->nreg != r->A->nreg)
            return fail(TPCF_E_INVALID, "both catalogs need region labels with the same number of regions");
        TRY(get_plan_regions(ctx, r->auto_pairs, r->cat_a, r->auto_pairs ? r->cat_a : r->cat_b, *r->A, *r->B,
                             &r->plan));
        r->pairs = r->plan->pairs;
        return TPCF_OK;
    }
    TRY(get_plan(ctx, r->auto_pairs, r->A->n, r->B->n, rb, re, &r->plan));
    r->pairs = r->plan->pairs;
    if (d.kind == TPCF_RR)
        r->cache_key = cache_key(d.cat_a, d.bin_edges_deg, d.nbins, d.precision, rb, re);
    return TPCF_OK;
}

JobDev job_of(const Request &r, unsigned long long *hist, const int *cancel) {
    JobDev j;
    memset(&j, 0, sizeof j);
    const size_t na = (size_t)(r.A->n > 0 ? r.A->n : 1), nb = (size_t)(r.B->n > 0 ? r.B->n : 1);
    j.ax32 = r.A->d32;
    j.ay32 = r.A->d32 + na;
    j.az32 = r.A->d32 + 2 * na;
    j.bx32 = r.B->d32;
    j.by32 = r.B->d32 + nb;
    j.bz32 = r.B->d32 + 2 * nb;
    j.ax64 = r.A->d64;
    j.ay64 = r.A->d64 + na;
    j.az64 = r.A->d64 + 2 * na;
    j.bx64 = r.B->d64;
    j.by64 = r.B->d64 + nb;
    j.bz64 = r.B->d64 + 2 * nb;
    j.bcaps = r.B->dcaps;
    j.hist = hist;
    j.cancel = cancel;
    j.auto_pairs = r.auto_pairs ? 1 : 0;
    j.na = (int32_t)r.A->n;
    j.nb = (int32_t)r.B->n;
    return j;
}

// Threshold of the FP32 dot-product screen for the edge with threshold D
// (angular catalogs, squared norms within 1 +- delta): p = fl32(f_i . f_j) of
// the FP32 copies satisfies |p - d| <= E = dot_error32(delta), so p <= D - E
// proves d <= D.  The result is rounded down to a float.
float dot_screen32(double D, double delta) {
    if (!(D > -HUGE_VAL))
        return -HUGE_VALF;          // no pair passes this edge
    if (D == HUGE_VAL)
        return HUGE_VALF;           // every pair passes it
    const double P = D - dot_error32(delta);
    float f = (float)P;
    if ((double)f > P)
        f = nextafterf(f, -HUGE_VALF);
    return f;
}

// Kernel arguments of a launch with compiled edges cp.  delta: bound on
// | |v|^2 - 1 | over the launch's sky catalogs (angular pruning).
PairArgs args_of(const tpcf_ctx *ctx, const Compiled &cp, int nbins, unsigned long long *stats, double delta) {
    PairArgs a;
    memset(&a, 0, sizeof a);
    a.lut = cp.dlut.p;
    a.lut_cells = (int32_t)(cp.cells.direct ? cp.cells.image.size() : cp.cells.cells.size());
    a.lut_wrap_bits = cp.cells.wrap_bits;
    a.aux_off = cp.cells.aux_off;
    a.q_floor = cp.cells.q0;
    a.lut_entry_bytes = cp.entry_bytes;
    a.lut_shift = cp.cells.shift;
    a.lut_lo = cp.cells.lo;
    a.lut_hi = cp.cells.hi;
    a.lut_direct = cp.cells.direct ? 1 : 0;
    a.metric = cp.metric;
    a.prune = ctx->tune.prune ? 1 : 0;
    // 3-D: the FP32 row copies move each point by at most 2^-24 R per
    // component (sqrt(3) 2^-24 R in all); cp.delta holds R for 3-D edges
    a.prune_margin = cp.metric ? ldexp(cp.delta, -22) + 1e-300 : 0.0;
    a.prune_delta = cp.metric ? 0.0 : delta;
    a.erad = (const double *)cp.dErad.p;
    // key of the last edge's certain side (see PairArgs::beyond_key)
    const size_t last = cp.edges.D.size() - 1;
    if (cp.precision == TPCF_FP32_CHORD) {
        float qh = cp.band.qhi[last];
        memcpy(&a.beyond_key, &qh, sizeof qh);
        a.p_beyond = cp.metric ? -HUGE_VALF : dot_screen32(cp.edges.D[last], cp.delta);
        if (!cp.pcells.cells.empty()) {
            a.plut_cells = (int32_t)cp.pcells.cells.size();
            a.plut_shift = cp.pcells.shift;
            a.plut_lo = cp.pcells.lo;
            a.plut_hi = cp.pcells.hi;
            a.plut_src = cp.plut_src;
            const int base = lds_bytes(nbins + 2, hist_copies_of(ctx->tune, nbins + 2), a.lut_cells, cp.entry_bytes,
                                       nbins + 1, cp.cells.direct ? cp.cells.aux_off : -1);
            a.plut_lds = (base + 15) & ~15;
            a.stage_lds = (a.plut_lds + a.plut_cells * cp.entry_bytes + 15) & ~15;
            // the chord loop hands steps to the dot product at chord^2 above
            // 0.018 (about 7.7 deg), where p's error is ~2e-5 of q and a
            // lane's pairs seldom span several bins: a heuristic, measured
            // best on the octant workloads (0.6 to 25 deg tried)
            a.q_dot = std::max(0.018f, (float)(400.0 * dot_error32(cp.delta)));
        }
    } else {
        const double t = cp.edges.E[last];
        uint64_t b;
        memcpy(&b, &t, sizeof b);
        a.beyond_key = (uint32_t)(b >> 32);
        a.p_beyond = -HUGE_VALF;
    }
    a.qlo = (const float *)cp.dqlo.p;
    a.qhi = (const float *)cp.dqhi.p;
    a.E = (const double *)cp.dE.p;
    a.D = (const double *)cp.dD.p;
    a.nedges = nbins + 1;
    a.nslots = nbins + 2;
    a.hist_copies = hist_copies_of(ctx->tune, nbins + 2);
    a.rows_per_lane = rows_per_lane_of(ctx->tune);
    a.blocks_per_cu = ctx->tune.blocks_per_cu;
    a.stats = stats;
    return a;
}

int record_start(tpcf_ctx *ctx, hipStream_t st, hipEvent_t *e0, hipEvent_t *e1) {
    *e0 = *e1 = nullptr;
    if (!ctx->timing)
        return TPCF_OK;
    HIP_TRY(hipEventCreate(e0));
    HIP_TRY(hipEventCreate(e1));
    HIP_TRY(hipEventRecord(*e0, st));
    return TPCF_OK;
}

int record_stop(tpcf_ctx *ctx, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (!e0)
        return TPCF_OK;
    HIP_TRY(hipEventRecord(e1, st));
    ctx->events.emplace_back(e0, e1);
    return TPCF_OK;
}

// Enqueue one request on a workspace: zero its histogram copies, count, and
// reduce into d_out (nslots u64).  Every argument travels by value in the
// kernel arguments, so nothing on the host must outlive the call.
// With regions (nreg > 0), every unit's counts also go to the copies of its
// two regions in w.touch, reduced into d_touch (nreg x nslots u64).
int launch_one(tpcf_ctx *ctx, Workspace &w, const Request &r, unsigned long long *d_out,
               const int *cancel, int32_t nreg = 0, unsigned long long *d_touch = nullptr) {
    const int nslots = r.nbins + 2;
    unsigned long long *touch = nullptr;
    if (nreg > 0) {
        const size_t per = (size_t)kGlobalCopies * (size_t)nslots;
        TRY(w.touch.ensure(ctx->mem, sizeof(unsigned long long) * per * (size_t)nreg));
        touch = (unsigned long long *)w.touch.p;
        HIP_TRY((hipError_t)tpcf_launch_zero_u64(touch, (int64_t)(per * (size_t)nreg), w.stream));
    }
    // the histogram copies, then the work-queue counter, zeroed together
    TRY(w.copies.ensure(ctx->mem, sizeof(unsigned long long) * ((size_t)kGlobalCopies * kMaxSlots + 1)));
    unsigned long long *copies = (unsigned long long *)w.copies.p;
    HIP_TRY((hipError_t)tpcf_launch_zero_u64(copies, (int64_t)kGlobalCopies * nslots + 1, w.stream));
    PairArgs a = args_of(ctx, *r.cp, r.nbins, (unsigned long long *)w.stats.p, std::max(r.A->delta, r.B->delta));
    a.jobs = nullptr;
    a.job0 = job_of(r, copies, cancel);
    a.job0.touch = touch;
    a.units = (const Unit *)r.plan->dunits.p;
    a.n_units = (int32_t)r.plan->units.size();
    a.queue = (unsigned int *)(copies + (size_t)kGlobalCopies * nslots);
    hipEvent_t e0, e1;
    if (a.n_units > 0)
        TRY(record_start(ctx, w.stream, &e0, &e1));
    else
        e0 = e1 = nullptr;
    int lrc = tpcf_launch_pairs(&a, r.precision, w.stream);
    if (lrc)
        return fail(TPCF_E_HIP, std::string("pair kernel launch: ") + hipGetErrorString((hipError_t)lrc));
    TRY(record_stop(ctx, w.stream, e0, e1));
    lrc = tpcf_launch_reduce_copies(copies, nslots, 1, d_out, w.stream);
    if (lrc == 0 && touch)
        lrc = tpcf_launch_reduce_copies(touch, nslots, nreg, d_touch, w.stream);
    if (lrc)
        return fail(TPCF_E_HIP, std::string("reduce launch: ") + hipGetErrorString((hipError_t)lrc));
    ctx->pairs_since_reset += r.pairs;
    return TPCF_OK;
}

int check_total(const uint64_t *h, int nslots, uint64_t expected) {
    uint64_t tot = 0;
    for (int s = 0; s < nslots; ++s)
        tot += h[s];
    if (tot != expected) {
        char buf[160];
        snprintf(buf, sizeof buf, "slot total %llu differs from the %llu pairs requested",
                 (unsigned long long)tot, (unsigned long long)expected);
        return fail(TPCF_E_INTERNAL, buf);
    }
    return TPCF_OK;
}

tpcf_job_desc desc_of(int kind, int32_t cat_a, int32_t cat_b, const double *edges, int32_t nbins,
                      int precision, int64_t rb, int64_t re) {
    tpcf_job_desc d;
    d.kind = kind;
    d.cat_a = cat_a;
    d.cat_b = cat_b;
    d.bin_edges_deg = edges;
    d.nbins = nbins;
    d.precision = precision;
    d.row_begin = rb;
    d.row_end = re;
    return d;
}

void retire_job(tpcf_ctx *ctx, std::map<int64_t, AsyncJob>::iterator it) {
    AsyncJob &j = it->second;
    if (j.ev)
        (void)hipEventDestroy(j.ev);
    if (j.hres)      // the job's event has completed: no GPU work reads it
        ctx->pinned_free.push_back(j.hres);
    if (j.ws >= 0)
        ctx->pool[j.ws].inflight--;
    ctx->jobs.erase(it);
}

// Finish a completed job: result into out (may be null), retire it.
int finish_job(tpcf_ctx *ctx, std::map<int64_t, AsyncJob>::iterator it, uint64_t *out) {
    AsyncJob &j = it->second;
    const int nslots = j.req.nbins + 2;
    if (j.cancelled) {
        retire_job(ctx, it);
        return fail(TPCF_E_CANCELLED, "job was cancelled");
    }
    std::vector<uint64_t> h;
    if (j.ready) {
        h = j.result;
    } else {
        h.assign(j.hres, j.hres + nslots);
        int rc = check_total(h.data(), nslots, j.req.pairs);
        if (rc) {
            retire_job(ctx, it);
            return rc;
        }
        if (!j.req.cache_key.empty())
            ctx->result_cache[j.req.cache_key] = h;
    }
    if (out)
        memcpy(out, h.data(), sizeof(uint64_t) * (size_t)nslots);
    retire_job(ctx, it);
    return TPCF_OK;
}

// Device memory of the context's device?
bool on_device(const tpcf_ctx *ctx, const void *p) {
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != ctx->device) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

const char *tpcf_last_error(const tpcf_ctx *) { return g_err.c_str(); }

const char *tpcf_version(void) { return "tpcf 0.2 (gfx950)"; }

int tpcf_open(int device, void *hip_stream, tpcf_ctx **out) {
    if (!out)
        return fail(TPCF_E_INVALID, "out is NULL");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(TPCF_E_INVALID, "device index out of range");
    auto ctx = std::make_unique<tpcf_ctx>();
    ctx->device = device;
    HIP_TRY(hipSetDevice(device));
    // the device address of this device's fixed work area (tpcf_count_noalloc)
    HIP_TRY((hipError_t)tpcf_scratch_init(device));
    TRY(init_workspace(ctx.get(), ctx->main, (hipStream_t)hip_stream));
    HIP_TRY(hipStreamSynchronize(ctx->main.stream));
    *out = ctx.release();
    return TPCF_OK;
}

int tpcf_close(tpcf_ctx *ctx) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    (void)hipSetDevice(ctx->device);
    (void)sync_all(ctx);
    while (!ctx->jobs.empty())
        retire_job(ctx, ctx->jobs.begin());
    for (uint64_t *p : ctx->pinned_free)
        (void)hipHostFree(p);
    ctx->pinned_free.clear();
    drop_graphs(ctx);
    for (auto &kv : ctx->cats) {
        if (kv.second.owns64)
            dev_free(ctx->mem, kv.second.d64, kv.second.bytes64);
        if (kv.second.owns32)
            dev_free(ctx->mem, kv.second.d32, kv.second.bytes32);
        dev_free(ctx->mem, kv.second.dcaps, kv.second.bytes_caps);
    }
    for (auto &kv : ctx->compiled)
        free_compiled(ctx, *kv.second);
    for (auto &kv : ctx->plans)
        kv.second->dunits.release(ctx->mem);
    for (auto &ev : ctx->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    for (auto &w : ctx->pool)
        free_workspace(ctx, w);
    free_workspace(ctx, ctx->main);
    delete ctx;
    return TPCF_OK;
}

int tpcf_upload_catalog_regions(tpcf_ctx *ctx, const double *ra_deg, const double *dec_deg, int64_t n,
                                const int32_t *region, int32_t nreg, int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (n < 0)
        return fail(TPCF_E_INVALID, "n must be >= 0");
    if (n > 0 && (!ra_deg || !dec_deg))
        return fail(TPCF_E_INVALID, "ra_deg/dec_deg is NULL");
    const double deg = M_PI / 180.0;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(ra_deg[i]) || !isfinite(dec_deg[i]))
            return fail(TPCF_E_INVALID, "ra/dec must be finite");
    std::vector<double> x((size_t)n), y((size_t)n), z((size_t)n);
    parallel_chunks(n, host_threads(n), [&](int, int64_t b0, int64_t e0) {
        for (int64_t i = b0; i < e0; ++i) {
            double a = ra_deg[i] * deg;
            double b = dec_deg[i] * deg;
            x[i] = cos(b) * cos(a);
            y[i] = cos(b) * sin(a);
            z[i] = sin(b);
        }
    });
    return add_catalog(ctx, x.data(), y.data(), z.data(), n, out_cat, region, region ? nreg : 0);
}

int tpcf_upload_catalog(tpcf_ctx *ctx, const double *ra_deg, const double *dec_deg, int64_t n,
                        int32_t *out_cat) {
    return tpcf_upload_catalog_regions(ctx, ra_deg, dec_deg, n, nullptr, 0, out_cat);
}

int tpcf_catalog_regions(tpcf_ctx *ctx, int32_t cat, int32_t *out_nreg, int64_t *out_counts) {
    if (!ctx || !out_nreg)
        return fail(TPCF_E_INVALID, "NULL argument");
    auto it = ctx->cats.find(cat);
    if (it == ctx->cats.end())
        return fail(TPCF_E_BADID, "unknown catalog id");
    const Catalog &c = it->second;
    *out_nreg = c.nreg;
    if (out_counts)
        for (int32_t r = 0; r < c.nreg; ++r)
            out_counts[r] = c.reg_start[(size_t)r + 1] - c.reg_start[(size_t)r];
    return TPCF_OK;
}

int tpcf_upload_catalog_3d_regions(tpcf_ctx *ctx, const double *x, const double *y, const double *z,
                                   int64_t n, const int32_t *region, int32_t nreg, int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    return add_catalog(ctx, x, y, z, n, out_cat, region, region ? nreg : 0, 1);
}

int tpcf_upload_catalog_3d(tpcf_ctx *ctx, const double *x, const double *y, const double *z, int64_t n,
                           int32_t *out_cat) {
    return tpcf_upload_catalog_3d_regions(ctx, x, y, z, n, nullptr, 0, out_cat);
}

int tpcf_upload_catalog_xyz(tpcf_ctx *ctx, const double *x, const double *y, const double *z,
                            int64_t n, int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    return add_catalog(ctx, x, y, z, n, out_cat);
}

int tpcf_attach_catalog(tpcf_ctx *ctx, const double *d_xyz64, const float *d_xyz32, int64_t n,
                        int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!out_cat)
        return fail(TPCF_E_INVALID, "out_cat is NULL");
    if (n < 1 || n > (int64_t)0x7fffffff - 1024)
        return fail(TPCF_E_INVALID, "attach needs 1 <= n < 2^31 - 1024");
    if (!d_xyz64)
        return fail(TPCF_E_INVALID, "d_xyz64 is NULL");
    TRY(set_device(ctx));
    if (!on_device(ctx, d_xyz64))
        return fail(TPCF_E_INVALID, "d_xyz64 is not device memory of the context's device");
    if (d_xyz32 && !on_device(ctx, d_xyz32))
        return fail(TPCF_E_INVALID, "d_xyz32 is not device memory of the context's device");
    Catalog c;
    c.n = n;
    c.owns64 = false;
    c.d64 = const_cast<double *>(d_xyz64);
    c.bytes32 = sizeof(float) * 3 * (size_t)n;
    if (d_xyz32) {
        c.owns32 = false;
        c.d32 = const_cast<float *>(d_xyz32);
    } else {
        TRY(dev_alloc(ctx->mem, (void **)&c.d32, c.bytes32));
    }
    auto drop32 = [&] {
        if (c.owns32)
            dev_free(ctx->mem, c.d32, c.bytes32);
    };
    Workspace &w = ctx->main;
    int rc = w.out.ensure(ctx->mem, sizeof(unsigned long long) * kMaxSlots);
    if (rc) {
        drop32();
        return rc;
    }
    unsigned long long *chk = (unsigned long long *)w.out.p;
    hipError_t e = (hipError_t)tpcf_launch_zero_u64(chk, 2, w.stream);
    if (e == hipSuccess)
        e = (hipError_t)tpcf_launch_to_float(c.d64, n, c.owns32 ? c.d32 : nullptr, d_xyz32, chk, w.stream);
    unsigned long long h[2] = {0, 0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, chk, sizeof h, hipMemcpyDeviceToHost, w.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(w.stream);
    if (e != hipSuccess) {
        drop32();
        return fail(TPCF_E_HIP, std::string("attach: ") + hipGetErrorString(e));
    }
    double dev;
    memcpy(&dev, &h[0], sizeof dev);
    const double delta = dev + 4.0 * ldexp(1.0, -53);
    if (!(delta <= kMaxDelta)) {
        drop32();
        return fail(TPCF_E_INVALID, "attached vectors must be finite with | |v|^2 - 1 | <= 2^-20");
    }
    if (h[1]) {
        drop32();
        return fail(TPCF_E_INVALID, "d_xyz32 must hold the FP64 vectors rounded to nearest FP32");
    }
    c.delta = delta;
    int32_t id = ctx->next_id++;
    ctx->cats[id] = std::move(c);
    *out_cat = id;
    return TPCF_OK;
}

int tpcf_catalog_size(tpcf_ctx *ctx, int32_t cat, int64_t *out_n) {
    if (!ctx || !out_n)
        return fail(TPCF_E_INVALID, "NULL argument");
    auto it = ctx->cats.find(cat);
    if (it == ctx->cats.end())
        return fail(TPCF_E_BADID, "unknown catalog id");
    *out_n = it->second.n;
    return TPCF_OK;
}

int tpcf_catalog_order(tpcf_ctx *ctx, int32_t cat, int64_t *out_order) {
    if (!ctx || !out_order)
        return fail(TPCF_E_INVALID, "NULL argument");
    auto it = ctx->cats.find(cat);
    if (it == ctx->cats.end())
        return fail(TPCF_E_BADID, "unknown catalog id");
    const Catalog &c = it->second;
    for (int64_t r = 0; r < c.n; ++r)
        out_order[r] = c.order.empty() ? r : c.order[(size_t)r];
    return TPCF_OK;
}

int tpcf_release_catalog(tpcf_ctx *ctx, int32_t cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    auto it = ctx->cats.find(cat);
    if (it == ctx->cats.end())
        return fail(TPCF_E_BADID, "unknown catalog id");
    for (auto &kv : ctx->jobs)
        if (kv.second.req.cat_a == cat || kv.second.req.cat_b == cat)
            return fail(TPCF_E_INVALID, "catalog is used by a job that has not been polled to completion");
    TRY(set_device(ctx));
    TRY(sync_all(ctx));
    drop_graphs(ctx);   // captured launches hold catalog pointers
    for (auto c = ctx->result_cache.begin(); c != ctx->result_cache.end();) {
        int32_t k;
        memcpy(&k, c->first.data(), sizeof k);
        if (k == cat)
            c = ctx->result_cache.erase(c);
        else
            ++c;
    }
    if (it->second.owns64)
        dev_free(ctx->mem, it->second.d64, it->second.bytes64);
    if (it->second.owns32)
        dev_free(ctx->mem, it->second.d32, it->second.bytes32);
    dev_free(ctx->mem, it->second.dcaps, it->second.bytes_caps);
    ctx->cats.erase(it);
    return TPCF_OK;
}

int tpcf_count(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *bin_edges_deg,
               int32_t nbins, int precision, int64_t row_begin, int64_t row_end, uint64_t *out_u64) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!out_u64)
        return fail(TPCF_E_INVALID, "out_u64 is NULL");
    Request r;
    TRY(prepare(ctx, desc_of(kind, cat_a, cat_b, bin_edges_deg, nbins, precision, row_begin, row_end), -1, &r));
    const int nslots = nbins + 2;
    if (!r.cache_key.empty()) {
        auto c = ctx->result_cache.find(r.cache_key);
        if (c != ctx->result_cache.end()) {
            memcpy(out_u64, c->second.data(), sizeof(uint64_t) * (size_t)nslots);
            return TPCF_OK;
        }
    }
    Workspace &w = ctx->main;
    TRY(w.out.ensure(ctx->mem, sizeof(unsigned long long) * kMaxSlots));
    TRY(launch_one(ctx, w, r, (unsigned long long *)w.out.p, nullptr));
    std::vector<uint64_t> h((size_t)nslots);
    HIP_TRY(hipMemcpyAsync(h.data(), w.out.p, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost, w.stream));
    HIP_TRY(hipStreamSynchronize(w.stream));
    TRY(check_total(h.data(), nslots, r.pairs));
    if (!r.cache_key.empty())
        ctx->result_cache[r.cache_key] = h;
    memcpy(out_u64, h.data(), sizeof(uint64_t) * h.size());
    return TPCF_OK;
}

int tpcf_count_regions(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *bin_edges_deg,
                       int32_t nbins, int precision, uint64_t *out_total, uint64_t *out_touch) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!out_total || !out_touch)
        return fail(TPCF_E_INVALID, "out_total/out_touch is NULL");
    Request r;
    TRY(prepare(ctx, desc_of(kind, cat_a, cat_b, bin_edges_deg, nbins, precision, -1, -1), -1, &r, true));
    const int nslots = nbins + 2;
    const int32_t nreg = r.A->nreg;
    Workspace &w = ctx->main;
    TRY(w.out.ensure(ctx->mem, sizeof(unsigned long long) * kMaxSlots));
    TRY(w.tout.ensure(ctx->mem, sizeof(unsigned long long) * (size_t)kMaxSlots * (size_t)nreg));
    TRY(launch_one(ctx, w, r, (unsigned long long *)w.out.p, nullptr, nreg, (unsigned long long *)w.tout.p));
    std::vector<uint64_t> h((size_t)nslots), t((size_t)nslots * (size_t)nreg);
    HIP_TRY(hipMemcpyAsync(h.data(), w.out.p, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost, w.stream));
    HIP_TRY(hipMemcpyAsync(t.data(), w.tout.p, sizeof(uint64_t) * t.size(), hipMemcpyDeviceToHost, w.stream));
    HIP_TRY(hipStreamSynchronize(w.stream));
    TRY(check_total(h.data(), nslots, r.pairs));
    // every pair touches one or two regions: the touch sums lie between the
    // total and twice the total, slot by slot, and no region exceeds the total
    for (int s = 0; s < nslots; ++s) {
        uint64_t sum = 0;
        for (int32_t g = 0; g < nreg; ++g) {
            const uint64_t v = t[(size_t)g * nslots + s];
            if (v > h[(size_t)s])
                return fail(TPCF_E_INTERNAL, "a region count exceeds the total");
            sum += v;
        }
        if (sum < h[(size_t)s] || sum > 2 * h[(size_t)s])
            return fail(TPCF_E_INTERNAL, "region counts do not cover the total");
    }
    memcpy(out_total, h.data(), sizeof(uint64_t) * h.size());
    memcpy(out_touch, t.data(), sizeof(uint64_t) * t.size());
    return TPCF_OK;
}

int tpcf_count_async(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *bin_edges_deg,
                     int32_t nbins, int precision, int64_t row_begin, int64_t row_end,
                     uint64_t *d_out_u64) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!d_out_u64)
        return fail(TPCF_E_INVALID, "d_out_u64 is NULL");
    Request r;
    TRY(prepare(ctx, desc_of(kind, cat_a, cat_b, bin_edges_deg, nbins, precision, row_begin, row_end), -1, &r));
    return launch_one(ctx, ctx->main, r, (unsigned long long *)d_out_u64, nullptr);
}

int tpcf_count_noalloc(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *bin_edges_deg,
                       int32_t nbins, int precision, int64_t row_begin, int64_t row_end, uint64_t *out_u64) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!out_u64)
        return fail(TPCF_E_INVALID, "out_u64 is NULL");
    Request r;
    TRY(validate(ctx, desc_of(kind, cat_a, cat_b, bin_edges_deg, nbins, precision, row_begin, row_end), &r));
    TRY(set_device(ctx));
    unsigned char *base = (unsigned char *)tpcf_scratch_ptr(ctx->device);
    if (!base)
        return fail(TPCF_E_HIP, "the fixed work area of this device has no address (tpcf_open sets it up)");
    // tables on the host; their device copies go into the work area
    const double delta = std::max(r.A->band_param(), r.B->band_param());
    Compiled c;
    std::vector<uint8_t> packed;
    std::vector<float> qlo, qhi;
    TRY(compile_host(ctx->tune, bin_edges_deg, nbins, precision, delta, r.metric, &c, &packed, &qlo, &qhi));
    const int nslots = nbins + 2, nedges = nbins + 1;
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_copies = take(sizeof(unsigned long long) * ((size_t)kGlobalCopies * nslots + 1));
    const size_t o_out = take(sizeof(unsigned long long) * (size_t)nslots);
    const size_t o_D = take(sizeof(double) * nedges), o_E = take(sizeof(double) * nedges);
    const size_t o_qlo = take(sizeof(float) * qlo.size()), o_qhi = take(sizeof(float) * qhi.size());
    const size_t o_rad = take(sizeof(double) * nedges);
    const size_t o_lut = take(packed.size());
    const size_t o_units = off;
    if (o_units >= kScratchBytes)
        return fail(TPCF_E_INVALID, "the tables do not fit the fixed work area");
    const size_t max_units = (kScratchBytes - o_units) / sizeof(Unit);
    // the unit list is sized for half the room (the triangular lists of
    // auto-pairs hold a few more units than the estimate), then checked
    const int64_t T = (int64_t)kWaves * kWaveSize * rows_per_lane_of(ctx->tune);
    Plan plan = make_plan(r.auto_pairs, r.A->n, r.B->n, r.rb, r.re, T, max_cols_of(ctx->tune), 0.5 * (double)max_units);
    if (plan.units.size() > max_units) {
        char buf[200];
        snprintf(buf, sizeof buf, "the request needs %zu work units; the fixed work area (%zu MiB) holds %zu",
                 plan.units.size(), kScratchBytes >> 20, max_units);
        return fail(TPCF_E_INVALID, buf);
    }
    for (const Unit &u : plan.units)   // each unit's LDS counts must stay below 2^32
        if ((uint64_t)(u.i1 - u.i0) * (uint64_t)(u.j1 - u.j0) >= ((uint64_t)1 << 32))
            return fail(TPCF_E_INVALID, "the request is too large for the fixed work area");
    hipStream_t st = ctx->main.stream;
    auto h2d = [&](size_t at, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(base + at, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    HIP_TRY(h2d(o_D, c.edges.D.data(), sizeof(double) * c.edges.D.size()));
    HIP_TRY(h2d(o_E, c.edges.E.data(), sizeof(double) * c.edges.E.size()));
    HIP_TRY(h2d(o_qlo, qlo.data(), sizeof(float) * qlo.size()));
    HIP_TRY(h2d(o_qhi, qhi.data(), sizeof(float) * qhi.size()));
    HIP_TRY(h2d(o_rad, c.edges.edge_rad.data(), sizeof(double) * c.edges.edge_rad.size()));
    HIP_TRY(h2d(o_lut, packed.data(), packed.size()));
    HIP_TRY(h2d(o_units, plan.units.data(), sizeof(Unit) * plan.units.size()));
    // the histogram copies and the queue counter start at zero (a kernel, not a memset)
    unsigned long long *copies = (unsigned long long *)(base + o_copies);
    HIP_TRY((hipError_t)tpcf_launch_zero_u64(copies, (int64_t)kGlobalCopies * nslots + 1, st));
    c.dD.p = base + o_D;
    c.dE.p = base + o_E;
    c.dqlo.p = base + o_qlo;
    c.dqhi.p = base + o_qhi;
    c.dErad.p = base + o_rad;
    c.dlut.p = base + o_lut;
    PairArgs a = args_of(ctx, c, nbins, (unsigned long long *)ctx->main.stats.p, delta);
    a.prune = 0;     // bounding caps are built on first use, which allocates: count every pair
    a.jobs = nullptr;
    a.job0 = job_of(r, copies, nullptr);
    a.units = (const Unit *)(base + o_units);
    a.n_units = (int32_t)plan.units.size();
    a.queue = (unsigned int *)(copies + (size_t)kGlobalCopies * nslots);
    int lrc = tpcf_launch_pairs(&a, r.precision, st);
    if (lrc == 0)
        lrc = tpcf_launch_reduce_copies(copies, nslots, 1, (unsigned long long *)(base + o_out), st);
    if (lrc)
        return fail(TPCF_E_HIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)lrc));
    std::vector<uint64_t> h((size_t)nslots);
    HIP_TRY(hipMemcpyAsync(h.data(), base + o_out, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    TRY(check_total(h.data(), nslots, plan.pairs));
    ctx->pairs_since_reset += plan.pairs;
    memcpy(out_u64, h.data(), sizeof(uint64_t) * h.size());
    return TPCF_OK;
}

int tpcf_count_batch(tpcf_ctx *ctx, const tpcf_job_desc *jobs, int32_t njobs, int flags, uint64_t *out_u64) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!jobs || !out_u64 || njobs < 1 || njobs > 65536)
        return fail(TPCF_E_INVALID, "need 1 <= njobs <= 65536 job descriptions and an output array");
    if (flags & ~TPCF_BATCH_GRAPH)
        return fail(TPCF_E_INVALID, "unknown batch flags");
    const int nbins = jobs[0].nbins;
    if (nbins < 1 || nbins > 256 || !jobs[0].bin_edges_deg)
        return fail(TPCF_E_INVALID, "nbins must be in [1, 256] and edges non-NULL");
    for (int32_t k = 1; k < njobs; ++k) {
        if (jobs[k].nbins != nbins || jobs[k].precision != jobs[0].precision || !jobs[k].bin_edges_deg ||
            memcmp(jobs[k].bin_edges_deg, jobs[0].bin_edges_deg, sizeof(double) * (size_t)(nbins + 1)) != 0)
            return fail(TPCF_E_INVALID, "every job of a batch must use the same edges and precision");
    }
    // one norm bound for the whole batch, so all jobs share one set of tables
    double delta = 0.0;
    for (int32_t k = 0; k < njobs; ++k) {
        auto a = ctx->cats.find(jobs[k].cat_a);
        if (a != ctx->cats.end())
            delta = std::max(delta, a->second.band_param());
        auto b = ctx->cats.find(jobs[k].cat_b);
        if (b != ctx->cats.end())
            delta = std::max(delta, b->second.band_param());
    }
    std::vector<Request> reqs((size_t)njobs);
    for (int32_t k = 0; k < njobs; ++k) {
        TRY(prepare(ctx, jobs[k], delta, &reqs[k]));
        if (reqs[k].metric != reqs[0].metric)
            return fail(TPCF_E_INVALID, "a batch cannot mix sky and 3-D catalogs");
    }
    const int nslots = nbins + 2;
    const int prec = jobs[0].precision;
    // every job's histogram copies, then the work-queue counter
    const size_t copies_bytes = sizeof(unsigned long long) * ((size_t)njobs * kGlobalCopies * nslots + 1);
    const size_t out_bytes = sizeof(unsigned long long) * (size_t)njobs * nslots;
    hipStream_t st = ctx->main.stream;
    const bool use_graph = (flags & TPCF_BATCH_GRAPH) != 0;

    std::string key;
    key.append((const char *)&njobs, sizeof njobs);
    for (int32_t k = 0; k < njobs; ++k) {
        tpcf_job_desc d = jobs[k];
        d.bin_edges_deg = nullptr;
        key.append((const char *)&d, sizeof d);
    }
    key.append((const char *)jobs[0].bin_edges_deg, sizeof(double) * (size_t)(nbins + 1));
    key.append((const char *)&delta, sizeof delta);
    key.append((const char *)&ctx->tune, sizeof ctx->tune);

    BatchGraph *g = nullptr;
    std::unique_ptr<BatchGraph> fresh;
    auto git = ctx->graphs.find(key);
    if (use_graph && git != ctx->graphs.end())
        g = git->second.get();
    if (!g) {
        fresh = std::make_unique<BatchGraph>();
        g = fresh.get();
        int rc;
        if ((rc = g->copies.ensure(ctx->mem, copies_bytes)) || (rc = g->out.ensure(ctx->mem, out_bytes))) {
            free_graph(ctx, *g);
            return rc;
        }
        std::vector<JobDev> hj((size_t)njobs);
        std::vector<Unit> hu;
        for (int32_t k = 0; k < njobs; ++k) {
            hj[k] = job_of(reqs[k], (unsigned long long *)g->copies.p + (size_t)k * kGlobalCopies * nslots, nullptr);
            for (Unit u : reqs[k].plan->units) {
                u.job = k;
                hu.push_back(u);
            }
        }
        // units of all jobs interleaved by size: largest units first
        std::stable_sort(hu.begin(), hu.end(), [](const Unit &x, const Unit &y) {
            return (int64_t)(x.i1 - x.i0) * (x.j1 - x.j0) > (int64_t)(y.i1 - y.i0) * (y.j1 - y.j0);
        });
        if ((rc = upload_blocking(ctx->mem, g->jobs, hj)) || (rc = upload_blocking(ctx->mem, g->units, hu))) {
            free_graph(ctx, *g);
            return rc;
        }
        PairArgs a = args_of(ctx, *reqs[0].cp, nbins, (unsigned long long *)ctx->main.stats.p, delta);
        a.jobs = (const JobDev *)g->jobs.p;
        a.units = (const Unit *)g->units.p;
        a.n_units = (int32_t)hu.size();
        a.queue = (unsigned int *)((unsigned long long *)g->copies.p + (size_t)njobs * kGlobalCopies * nslots);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (use_graph) {
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                free_graph(ctx, *g);
                return fail(TPCF_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
            }
        }
        int lrc = tpcf_launch_zero_u64((unsigned long long *)g->copies.p,
                                       (int64_t)njobs * kGlobalCopies * nslots + 1, st);
        if (!lrc && !use_graph)
            rc = record_start(ctx, st, &e0, &e1);
        if (!lrc && !rc)
            lrc = tpcf_launch_pairs(&a, prec, st);
        if (!lrc && !rc && !use_graph)
            rc = record_stop(ctx, st, e0, e1);
        if (!lrc && !rc)
            lrc = tpcf_launch_reduce_copies((unsigned long long *)g->copies.p, nslots, njobs,
                                            (unsigned long long *)g->out.p, st);
        if (use_graph) {
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(st, &graph);
            g->graph = graph;
            if (!lrc && !rc && e == hipSuccess)
                e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
            if (!lrc && !rc && e != hipSuccess) {
                free_graph(ctx, *g);
                return fail(TPCF_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            }
        }
        if (lrc || rc) {
            (void)hipStreamSynchronize(st);
            free_graph(ctx, *g);
            return rc ? rc : fail(TPCF_E_HIP, std::string("batch launch: ") + hipGetErrorString((hipError_t)lrc));
        }
    }
    if (use_graph) {
        hipEvent_t e0, e1;
        TRY(record_start(ctx, st, &e0, &e1));
        HIP_TRY(hipGraphLaunch(g->exec, st));
        TRY(record_stop(ctx, st, e0, e1));
    }
    std::vector<uint64_t> h((size_t)njobs * nslots);
    HIP_TRY(hipMemcpyAsync(h.data(), g->out.p, out_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int rc = TPCF_OK;
    for (int32_t k = 0; k < njobs && !rc; ++k) {
        ctx->pairs_since_reset += reqs[k].pairs;
        rc = check_total(h.data() + (size_t)k * nslots, nslots, reqs[k].pairs);
    }
    if (fresh) {
        if (use_graph && !rc) {
            if (ctx->graphs.size() >= 16)
                drop_graphs(ctx);
            ctx->graphs[key] = std::move(fresh);
        } else {
            free_graph(ctx, *fresh);
        }
    }
    if (rc)
        return rc;
    memcpy(out_u64, h.data(), sizeof(uint64_t) * h.size());
    return TPCF_OK;
}

int tpcf_submit(tpcf_ctx *ctx, const tpcf_job_desc *job, int64_t *out_job) {
    if (!ctx || !job || !out_job)
        return fail(TPCF_E_INVALID, "NULL argument");
    AsyncJob j;
    TRY(prepare(ctx, *job, -1, &j.req));
    const int nslots = j.req.nbins + 2;
    if (!j.req.cache_key.empty()) {
        auto c = ctx->result_cache.find(j.req.cache_key);
        if (c != ctx->result_cache.end()) {
            j.ready = true;
            j.result = c->second;
        }
    }
    if (!j.ready) {
        if (ctx->pool.empty()) {
            ctx->pool.resize(kPoolStreams);
            for (auto &w : ctx->pool)
                TRY(init_workspace(ctx, w, nullptr));
        }
        int best = 0;
        for (int s = 1; s < (int)ctx->pool.size(); ++s)
            if (ctx->pool[s].inflight < ctx->pool[best].inflight)
                best = s;
        Workspace &w = ctx->pool[best];
        TRY(w.out.ensure(ctx->mem, sizeof(unsigned long long) * kMaxSlots));
        void *pinned = nullptr;
        if (!ctx->pinned_free.empty()) {
            pinned = ctx->pinned_free.back();
            ctx->pinned_free.pop_back();
        } else {
            HIP_TRY(hipHostMalloc(&pinned, sizeof(uint64_t) * (kMaxSlots + 8), hipHostMallocCoherent));
        }
        j.hres = (uint64_t *)pinned;
        j.hcancel = (volatile int *)(j.hres + kMaxSlots);
        *j.hcancel = 0;
        int rc = launch_one(ctx, w, j.req, (unsigned long long *)w.out.p, (const int *)j.hcancel);
        hipError_t e = hipSuccess;
        if (!rc)
            e = hipMemcpyAsync(j.hres, w.out.p, sizeof(uint64_t) * (size_t)nslots, hipMemcpyDeviceToHost, w.stream);
        if (!rc && e == hipSuccess)
            e = hipEventCreateWithFlags(&j.ev, hipEventDisableTiming);
        if (!rc && e == hipSuccess)
            e = hipEventRecord(j.ev, w.stream);
        if (rc || e != hipSuccess) {
            (void)hipStreamSynchronize(w.stream);
            if (j.ev)
                (void)hipEventDestroy(j.ev);
            ctx->pinned_free.push_back((uint64_t *)pinned);
            return rc ? rc : fail(TPCF_E_HIP, std::string("submit: ") + hipGetErrorString(e));
        }
        j.ws = best;
        w.inflight++;
    }
    int64_t id = ctx->next_job++;
    ctx->jobs[id] = std::move(j);
    *out_job = id;
    return TPCF_OK;
}

int tpcf_poll(tpcf_ctx *ctx, int64_t job, uint64_t *out_u64, int *done) {
    if (!ctx || !done)
        return fail(TPCF_E_INVALID, "NULL argument");
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end())
        return fail(TPCF_E_BADID, "unknown job id");
    *done = 0;
    if (!it->second.ready) {
        hipError_t e = hipEventQuery(it->second.ev);
        if (e == hipErrorNotReady)
            return TPCF_OK;
        if (e != hipSuccess)
            return fail(TPCF_E_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
    }
    *done = 1;
    return finish_job(ctx, it, out_u64);
}

int tpcf_wait(tpcf_ctx *ctx, int64_t job, uint64_t *out_u64) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end())
        return fail(TPCF_E_BADID, "unknown job id");
    if (!it->second.ready)
        HIP_TRY(hipEventSynchronize(it->second.ev));
    return finish_job(ctx, it, out_u64);
}

int tpcf_cancel(tpcf_ctx *ctx, int64_t job) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end())
        return fail(TPCF_E_BADID, "unknown job id");
    it->second.cancelled = true;
    if (it->second.hcancel)
        *it->second.hcancel = 1;
    return TPCF_OK;
}

int tpcf_set_tuning(tpcf_ctx *ctx, const tpcf_tuning *tuning) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    tpcf_tuning t;
    memset(&t, 0, sizeof t);
    if (tuning)
        t = *tuning;
    if (t.rows_per_lane != 0 && t.rows_per_lane != 2 && t.rows_per_lane != 4)
        return fail(TPCF_E_INVALID, "rows_per_lane must be 0 (default), 2 or 4");
    if (t.hist_copies != 0 && t.hist_copies != 4 && t.hist_copies != 8 && t.hist_copies != 16 &&
        t.hist_copies != 32)
        return fail(TPCF_E_INVALID, "hist_copies must be 0 (default), 4, 8, 16 or 32");
    if (t.max_cols != 0 && (t.max_cols < 256 || t.max_cols > 65536 || t.max_cols % 256))
        return fail(TPCF_E_INVALID, "max_cols must be 0 (default) or a multiple of 256 in [256, 65536]");
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > 64)
        return fail(TPCF_E_INVALID, "blocks_per_cu must be in [0, 64]");
    if (t.lut_bytes != 0 && (t.lut_bytes < 4096 || t.lut_bytes > kMaxDirectLutBytes))
        return fail(TPCF_E_INVALID, "lut_bytes must be 0 (default) or in [4096, 33792]");
    if (t.lut_direct != 0 && t.lut_direct != 1)
        return fail(TPCF_E_INVALID, "lut_direct must be 0 or 1");
    if (t.prune != 0 && t.prune != 1)
        return fail(TPCF_E_INVALID, "prune must be 0 or 1");
    Tuning u;
    u.rows_per_lane = t.rows_per_lane;
    u.hist_copies = t.hist_copies;
    u.max_cols = t.max_cols;
    u.blocks_per_cu = t.blocks_per_cu;
    u.lut_bytes = t.lut_bytes;
    u.lut_direct = t.lut_direct;
    u.prune = t.prune;
    ctx->tune = u;
    return TPCF_OK;
}

int tpcf_get_tuning(tpcf_ctx *ctx, tpcf_tuning *out) {
    if (!ctx || !out)
        return fail(TPCF_E_INVALID, "NULL argument");
    out->rows_per_lane = ctx->tune.rows_per_lane;
    out->hist_copies = ctx->tune.hist_copies;
    out->max_cols = ctx->tune.max_cols;
    out->blocks_per_cu = ctx->tune.blocks_per_cu;
    out->lut_bytes = ctx->tune.lut_bytes;
    out->lut_direct = ctx->tune.lut_direct;
    out->prune = ctx->tune.prune;
    return TPCF_OK;
}

int tpcf_set_hbm_budget(tpcf_ctx *ctx, int64_t bytes) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (bytes < 0)
        return fail(TPCF_E_INVALID, "budget must be >= 0 (0: unlimited)");
    ctx->mem.budget = bytes;
    return TPCF_OK;
}

int tpcf_hbm_usage(tpcf_ctx *ctx, int64_t *out_used, int64_t *out_budget) {
    if (!ctx || !out_used || !out_budget)
        return fail(TPCF_E_INVALID, "NULL argument");
    *out_used = ctx->mem.used;
    *out_budget = ctx->mem.budget;
    return TPCF_OK;
}

int tpcf_synchronize(tpcf_ctx *ctx) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    return sync_all(ctx);
}

int tpcf_set_timing(tpcf_ctx *ctx, int on) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    ctx->timing = on != 0;
    return TPCF_OK;
}

int tpcf_kernel_time(tpcf_ctx *ctx, double *out_ms, int64_t *out_launches, int reset) {
    if (!ctx || !out_ms || !out_launches)
        return fail(TPCF_E_INVALID, "NULL argument");
    TRY(sync_all(ctx));
    double ms = 0.0;
    for (auto &ev : ctx->events) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, ev.first, ev.second));
        ms += t;
    }
    *out_ms = ms;
    *out_launches = (int64_t)ctx->events.size();
    if (reset) {
        for (auto &ev : ctx->events) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
        ctx->events.clear();
    }
    return TPCF_OK;
}

int tpcf_stats(tpcf_ctx *ctx, tpcf_counters *out, int reset) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    TRY(set_device(ctx));
    TRY(sync_all(ctx));
    unsigned long long tot[kStats] = {};
    std::vector<Workspace *> ws{&ctx->main};
    for (auto &w : ctx->pool)
        ws.push_back(&w);
    for (Workspace *w : ws) {
        unsigned long long h[kStats] = {};
        HIP_TRY(hipMemcpy(h, w->stats.p, sizeof h, hipMemcpyDeviceToHost));
        for (int i = 0; i < kStats; ++i)
            tot[i] += h[i];
        if (reset)
            HIP_TRY((hipError_t)tpcf_launch_zero_u64((unsigned long long *)w->stats.p, kStats, w->stream));
    }
    if (reset)
        TRY(sync_all(ctx));
    if (out) {
        out->pairs = ctx->pairs_since_reset;
        out->flagged = tot[1];
        out->exact = tot[2];
        out->rare_steps = tot[4];
        out->beyond_steps = tot[5];
        out->one_slot_steps = tot[6];
        out->pruned_pairs = tot[7];
        out->two_slot_steps = tot[0];
        out->chord_steps = tot[8];
    }
    if (reset)
        ctx->pairs_since_reset = 0;
    return TPCF_OK;
}

int tpcf_landy_szalay(const uint64_t *dd, const uint64_t *dr, const uint64_t *rr, int32_t nbins,
                      int64_t n_d, int64_t n_r, int form, double *out_w) {
    if (!dd || !dr || !rr || !out_w)
        return fail(TPCF_E_INVALID, "NULL argument");
    if (nbins < 1 || nbins > 256)
        return fail(TPCF_E_INVALID, "nbins must be in [1, 256]");
    if (n_d < 2 || n_r < 2)
        return fail(TPCF_E_INVALID, "catalog sizes must be >= 2");
    if (form != 0 && form != 1)
        return fail(TPCF_E_INVALID, "form must be 0 or 1");
    const double nd = (double)n_d, nr = (double)n_r;
    std::vector<double> w((size_t)nbins);
    for (int k = 0; k < nbins; ++k) {
        // in-range bin k is slot k + 1
        const double DDk = (double)dd[k + 1], DRk = (double)dr[k + 1], RRk = (double)rr[k + 1];
        if (RRk == 0.0) {
            w[k] = NAN;
            continue;
        }
        if (form == 0) {
            const double pairs_dd = nd * (nd - 1.0) / 2.0;
            const double pairs_dr = nd * nr;
            const double pairs_rr = nr * (nr - 1.0) / 2.0;
            const double rr_n = RRk / pairs_rr;
            w[k] = (DDk / pairs_dd - 2.0 * (DRk / pairs_dr) + rr_n) / rr_n;
        } else {
            const double ratio = nr / nd;
            w[k] = 1.0 + ratio * ratio * ((2.0 * DDk) / (2.0 * RRk)) - 2.0 * ratio * (DRk / (2.0 * RRk));
        }
    }
    memcpy(out_w, w.data(), sizeof(double) * (size_t)nbins);
    return TPCF_OK;
}

int tpcf_jackknife(const uint64_t *dd, const uint64_t *dd_touch, const uint64_t *dr, const uint64_t *dr_touch,
                   const uint64_t *rr, const uint64_t *rr_touch, int32_t nbins, int32_t nreg, int64_t n_d,
                   const int64_t *nd_reg, int64_t n_r, const int64_t *nr_reg, int form, double *out_samples,
                   double *out_mean, double *out_cov) {
    if (!dd || !dd_touch || !dr || !dr_touch || !rr || !rr_touch || !nd_reg || !nr_reg || !out_samples)
        return fail(TPCF_E_INVALID, "NULL argument");
    if (nbins < 1 || nbins > 256)
        return fail(TPCF_E_INVALID, "nbins must be in [1, 256]");
    if (nreg < 2 || nreg > TPCF_MAX_REGIONS)
        return fail(TPCF_E_INVALID, "nreg must be in [2, TPCF_MAX_REGIONS]");
    const size_t ns = (size_t)nbins + 2, K = (size_t)nreg, nb = (size_t)nbins;
    std::vector<uint64_t> d1(ns), d2(ns), d3(ns);
    for (size_t r = 0; r < K; ++r) {
        // region r deleted: the pairs that touch it leave every count
        for (size_t s = 0; s < ns; ++s) {
            if (dd_touch[r * ns + s] > dd[s] || dr_touch[r * ns + s] > dr[s] || rr_touch[r * ns + s] > rr[s])
                return fail(TPCF_E_INVALID, "a region count exceeds its total");
            d1[s] = dd[s] - dd_touch[r * ns + s];
            d2[s] = dr[s] - dr_touch[r * ns + s];
            d3[s] = rr[s] - rr_touch[r * ns + s];
        }
        TRY(tpcf_landy_szalay(d1.data(), d2.data(), d3.data(), nbins, n_d - nd_reg[r], n_r - nr_reg[r], form,
                              out_samples + r * nb));
    }
    std::vector<double> mean(nb, 0.0);
    for (size_t k = 0; k < nb; ++k) {
        double acc = 0.0;
        for (size_t r = 0; r < K; ++r)
            acc += out_samples[r * nb + k];
        mean[k] = acc / (double)K;
    }
    if (out_mean)
        memcpy(out_mean, mean.data(), sizeof(double) * nb);
    if (out_cov) {
        const double f = ((double)K - 1.0) / (double)K;
        for (size_t a = 0; a < nb; ++a)
            for (size_t b = 0; b < nb; ++b) {
                double acc = 0.0;
                for (size_t r = 0; r < K; ++r)
                    acc += (out_samples[r * nb + a] - mean[a]) * (out_samples[r * nb + b] - mean[b]);
                out_cov[a * nb + b] = f * acc;
            }
    }
    return TPCF_OK;
}

int tpcf_compile_cells(const double *bin_edges_deg, int32_t nbins, int precision, double delta_max,
                       int32_t max_cells, int32_t direct, int32_t *out_shift, int32_t *out_lo,
                       int32_t *out_hi, uint16_t *out_cells, double *out_E) {
    if (!out_shift || !out_lo || !out_hi || !out_cells)
        return fail(TPCF_E_INVALID, "NULL argument");
    if (precision != TPCF_FP32_CHORD && precision != TPCF_FP64)
        return fail(TPCF_E_INVALID, "precision must be TPCF_FP32_CHORD or TPCF_FP64");
    if (!(delta_max >= 0.0) || delta_max > kMaxDelta)
        return fail(TPCF_E_INVALID, "delta_max must be in [0, 2^-20]");
    if (max_cells < 16 || max_cells > kMaxDirectLutBytes)
        return fail(TPCF_E_INVALID, "max_cells must be in [16, 33792]");
    if (direct != 0 && (direct != 1 || precision != TPCF_FP32_CHORD))
        return fail(TPCF_E_INVALID, "direct must be 0, or 1 with TPCF_FP32_CHORD");
    EdgeTables t;
    std::string err;
    if (!compile_edges(bin_edges_deg, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    CellTable c;
    if (direct) {
        const Band32 fb = make_band32(t, delta_max, floor_for(make_band32(t, delta_max)));
        c = make_cells32_wrap(t, fb, delta_max, max_cells,
                              aux_lds_bytes(nbins + 2, hist_copies_of(Tuning{}, nbins + 2), nbins + 1));
        if (c.cells.empty())
            return fail(TPCF_E_INVALID, "no wrapped table fits in max_cells bytes");
    } else {
        const int m = std::min<int>(max_cells, kMaxLutCells);
        c = precision == TPCF_FP32_CHORD ? make_cells32(t, make_band32(t, delta_max), delta_max, m)
                                         : make_cells64(t, m);
    }
    *out_shift = c.shift;
    *out_lo = c.lo;
    *out_hi = c.hi;
    memcpy(out_cells, c.cells.data(), sizeof(uint16_t) * c.cells.size());
    if (out_E)
        for (int k = 0; k <= nbins; ++k)
            out_E[k] = t.E[k];
    return TPCF_OK;
}

int tpcf_compile_wrap32(const double *bin_edges_deg, int32_t nbins, double delta_max, int32_t max_bytes,
                        int32_t aux_bytes, int32_t *out_shift, int32_t *out_wrap_bits, int32_t *out_lo,
                        int32_t *out_hi, int32_t *out_aux_off, float *out_q0, float *out_qlo, float *out_qhi,
                        uint8_t *out_image) {
    if (!out_shift || !out_wrap_bits || !out_lo || !out_hi || !out_aux_off || !out_q0)
        return fail(TPCF_E_INVALID, "NULL argument");
    if (!(delta_max >= 0.0) || delta_max > kMaxDelta)
        return fail(TPCF_E_INVALID, "delta_max must be in [0, 2^-20]");
    if (max_bytes < 256 || max_bytes > 65536 || aux_bytes < 0 || aux_bytes > max_bytes)
        return fail(TPCF_E_INVALID, "max_bytes must be in [256, 65536] and aux_bytes in [0, max_bytes]");
    EdgeTables t;
    std::string err;
    if (!compile_edges(bin_edges_deg, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    if (nbins + 2 > kMaxSlots8)
        return fail(TPCF_E_INVALID, "wrapped tables hold one-byte entries (at most 125 bins)");
    const Band32 fb = make_band32(t, delta_max, floor_for(make_band32(t, delta_max)));
    const CellTable c = make_cells32_wrap(t, fb, delta_max, max_bytes, aux_bytes);
    if (c.cells.empty())
        return fail(TPCF_E_INVALID, "no wrapped table fits in max_bytes");
    *out_shift = c.shift;
    *out_wrap_bits = c.wrap_bits;
    *out_lo = c.lo;
    *out_hi = c.hi;
    *out_aux_off = c.aux_off;
    *out_q0 = c.q0;
    for (int k = 0; k <= nbins; ++k) {
        if (out_qlo)
            out_qlo[k] = fb.qlo[k];
        if (out_qhi)
            out_qhi[k] = fb.qhi[k];
    }
    if (out_image)
        for (size_t i = 0; i < c.image.size(); ++i) {
            const uint16_t v = c.image[i];
            out_image[i] = v == kMulti ? 0xFF : (v & kMedium) ? (uint8_t)(0x80 | (v & 0x7F)) : (uint8_t)v;
        }
    return TPCF_OK;
}

int tpcf_compile_edges(const double *bin_edges_deg, int32_t nbins, double delta_max, double *out_D,
                       float *out_qlo, float *out_qhi) {
    if (!(delta_max >= 0.0) || delta_max > kMaxDelta)
        return fail(TPCF_E_INVALID, "delta_max must be in [0, 2^-20]");
    EdgeTables t;
    std::string err;
    if (!compile_edges(bin_edges_deg, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    Band32 b = make_band32(t, delta_max);
    for (int k = 0; k <= nbins; ++k) {
        if (out_D)
            out_D[k] = t.D[k];
        if (out_qlo)
            out_qlo[k] = b.qlo[k];
        if (out_qhi)
            out_qhi[k] = b.qhi[k];
    }
    return TPCF_OK;
}

int tpcf_compile_screen(const double *bin_edges_deg, int32_t nbins, double delta_max, float *out_p) {
    if (!out_p)
        return fail(TPCF_E_INVALID, "out_p is NULL");
    if (!(delta_max >= 0.0) || delta_max > kMaxDelta)
        return fail(TPCF_E_INVALID, "delta_max must be in [0, 2^-20]");
    EdgeTables t;
    std::string err;
    if (!compile_edges(bin_edges_deg, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    *out_p = dot_screen32(t.D[(size_t)nbins], delta_max);
    return TPCF_OK;
}

int tpcf_compile_dot(const double *bin_edges_deg, int32_t nbins, double delta_max, int32_t max_cells,
                     float *out_klo, float *out_khi, float *out_plo, float *out_phi, int32_t *out_shift,
                     int32_t *out_lo, int32_t *out_hi, uint16_t *out_cells) {
    if (!out_shift || !out_lo || !out_hi || !out_cells)
        return fail(TPCF_E_INVALID, "NULL argument");
    if (!(delta_max >= 0.0) || delta_max > kMaxDelta)
        return fail(TPCF_E_INVALID, "delta_max must be in [0, 2^-20]");
    if (max_cells < 16 || max_cells > kMaxDirectLutBytes)
        return fail(TPCF_E_INVALID, "max_cells must be in [16, 33792]");
    EdgeTables t;
    std::string err;
    if (!compile_edges(bin_edges_deg, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    const Band32 b = make_band_dot32(t, delta_max);
    const CellTable c = make_cells32_top(t, b, dot_top_key(delta_max), max_cells);
    std::vector<float> plo, phi;
    make_pband32(t, delta_max, &plo, &phi);
    for (int k = 0; k <= nbins; ++k) {
        if (out_klo)
            out_klo[k] = b.qlo[k];
        if (out_khi)
            out_khi[k] = b.qhi[k];
        if (out_plo)
            out_plo[k] = plo[k];
        if (out_phi)
            out_phi[k] = phi[k];
    }
    *out_shift = c.shift;
    *out_lo = c.lo;
    *out_hi = c.hi;
    memcpy(out_cells, c.cells.data(), sizeof(uint16_t) * c.cells.size());
    return TPCF_OK;
}

int tpcf_compile_edges_3d(const double *bin_edges, int32_t nbins, double rmax, double *out_S, float *out_qlo,
                          float *out_qhi) {
    if (!(rmax >= 0.0) || rmax > 2.0 * kMaxCoord3d)
        return fail(TPCF_E_INVALID, "rmax must be in [0, 2^51]");
    EdgeTables t;
    std::string err;
    if (!compile_edges_3d(bin_edges, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    Band32 b = make_band32_3d(t, rmax);
    for (int k = 0; k <= nbins; ++k) {
        if (out_S)
            out_S[k] = t.E[k];   // -inf for a zero edge
        if (out_qlo)
            out_qlo[k] = b.qlo[k];
        if (out_qhi)
            out_qhi[k] = b.qhi[k];
    }
    return TPCF_OK;
}

}  // extern "C"
