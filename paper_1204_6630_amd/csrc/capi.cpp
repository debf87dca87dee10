// C ABI of libtpcf.so: contexts, catalogs, pair counting, Landy-Szalay.
//
// Host side of the pair-counting path.  Everything here runs on the host:
// argument checks, the unit vectors of uploaded catalogs, the edge compiler
// (edges.cpp), the work-unit plan, and the launches.  Every pair is counted
// on the GPU by the kernels in kernels.hip; there is no host fallback.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "tpcf.h"
#include "edges.h"
#include "internal.h"

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

// Device buffer that grows on demand.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap)
            return TPCF_OK;
        if (p)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = bytes < 256 ? 256 : bytes;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess)
            return fail(TPCF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        cap = want;
        return TPCF_OK;
    }
    void release() {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct Catalog {
    int64_t n = 0;
    double *d64 = nullptr;      // x[n], y[n], z[n]
    float *d32 = nullptr;       // x[n], y[n], z[n]
    std::vector<int64_t> order; // stored row r holds upload row order[r] (empty: identity)
    bool owns64 = true;
    double delta = 0;           // bound on | |v|^2 - 1 |
};

struct Compiled {
    EdgeTables edges;
    // device copies: D, E (nedges doubles each), per precision cell table and bands
    DevBuf dD, dE, dqlo, dqhi, dlut;
    CellTable cells;
    Band32 band;
    int precision = 0;
    int entry_bytes = 2;   // 1: byte entries (0x80 | k, 0xFF), 2: 16-bit codes
};

struct Plan {
    std::vector<Unit> units;
    DevBuf dunits;
    uint64_t pairs = 0;
};

}  // namespace

struct tpcf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t next_id = 1;
    std::map<int32_t, Catalog> cats;
    std::map<std::string, std::unique_ptr<Compiled>> compiled;
    std::map<std::string, std::unique_ptr<Plan>> plans;
    DevBuf copies;      // kGlobalCopies x kMaxSlots u64
    DevBuf outbuf;      // kMaxSlots u64 (synchronous path)
    DevBuf stats;       // 4 u64
    DevBuf scratch;     // small device scratch (attach)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    uint64_t pairs_since_reset = 0;
};

namespace {

int set_device(tpcf_ctx *ctx) {
    HIP_TRY(hipSetDevice(ctx->device));
    return TPCF_OK;
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

constexpr double kMaxDelta = 9.5367431640625e-07;   // 2^-20

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

uint64_t quant21(double c) {
    double t = (c + 1.0) * 0.5 * 2097151.0;
    if (!(t > 0.0))
        return 0;
    if (t > 2097151.0)
        return 2097151;
    return (uint64_t)t;
}

std::vector<int64_t> morton_order(const double *x, const double *y, const double *z, int64_t n) {
    std::vector<std::pair<uint64_t, int64_t>> k((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        k[i] = {spread3(quant21(x[i])) | spread3(quant21(y[i])) << 1 | spread3(quant21(z[i])) << 2, i};
    std::sort(k.begin(), k.end());
    std::vector<int64_t> order((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        order[i] = k[i].second;
    return order;
}

int add_catalog(tpcf_ctx *ctx, const double *x, const double *y, const double *z, int64_t n,
                int32_t *out_cat) {
    if (!out_cat)
        return fail(TPCF_E_INVALID, "out_cat is NULL");
    if (n < 0 || n > (int64_t)0x7fffffff - 1024)
        return fail(TPCF_E_INVALID, "catalog size out of range");
    if (n > 0 && (!x || !y || !z))
        return fail(TPCF_E_INVALID, "coordinate array is NULL");
    bool finite = true;
    double delta = n > 0 ? norm_bound(x, y, z, n, &finite) : 0.0;
    if (!finite)
        return fail(TPCF_E_INVALID, "coordinates must be finite");
    if (delta > kMaxDelta)
        return fail(TPCF_E_INVALID, "unit vectors must satisfy | |v|^2 - 1 | <= 2^-20");
    int rc = set_device(ctx);
    if (rc)
        return rc;
    Catalog c;
    c.n = n;
    c.delta = delta;
    c.order = morton_order(x, y, z, n);
    size_t alloc_n = (size_t)(n > 0 ? n : 1);
    std::vector<double> h64(3 * alloc_n, 0.0);
    std::vector<float> h32(3 * alloc_n, 0.0f);
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = c.order[r];
        h64[r] = x[i];
        h64[alloc_n + r] = y[i];
        h64[2 * alloc_n + r] = z[i];
        h32[r] = (float)x[i];
        h32[alloc_n + r] = (float)y[i];
        h32[2 * alloc_n + r] = (float)z[i];
    }
    hipError_t e = hipMalloc((void **)&c.d64, sizeof(double) * 3 * alloc_n);
    if (e != hipSuccess)
        return fail(TPCF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    e = hipMalloc((void **)&c.d32, sizeof(float) * 3 * alloc_n);
    if (e != hipSuccess) {
        (void)hipFree(c.d64);
        return fail(TPCF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipMemcpyAsync(c.d64, h64.data(), sizeof(double) * 3 * alloc_n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c.d32, h32.data(), sizeof(float) * 3 * alloc_n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(c.d64);
        (void)hipFree(c.d32);
        return fail(TPCF_E_HIP, std::string("upload: ") + hipGetErrorString(e));
    }
    int32_t id = ctx->next_id++;
    ctx->cats[id] = c;
    *out_cat = id;
    return TPCF_OK;
}

std::string edges_key(const double *edges, int nbins, int precision, double delta) {
    std::string k((const char *)edges, sizeof(double) * (size_t)(nbins + 1));
    k.append((const char *)&precision, sizeof precision);
    if (precision == TPCF_FP32_CHORD)
        k.append((const char *)&delta, sizeof delta);
    return k;
}

template <typename T>
int upload(DevBuf &b, const std::vector<T> &v, hipStream_t st) {
    int rc = b.ensure(sizeof(T) * (v.size() ? v.size() : 1));
    if (rc)
        return rc;
    if (!v.empty())
        HIP_TRY(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    return TPCF_OK;
}

int get_compiled(tpcf_ctx *ctx, const double *edges, int nbins, int precision, double delta,
                 Compiled **out) {
    std::string key = edges_key(edges, nbins, precision, delta);
    auto it = ctx->compiled.find(key);
    if (it != ctx->compiled.end()) {
        *out = it->second.get();
        return TPCF_OK;
    }
    auto c = std::make_unique<Compiled>();
    std::string err;
    if (!compile_edges(edges, nbins, &c->edges, &err))
        return fail(TPCF_E_INVALID, err);
    c->precision = precision;
    const int nslots = nbins + 2;
    c->entry_bytes = nslots <= kMaxSlots8 ? 1 : 2;
    const int max_cells = kMaxLutBytes / c->entry_bytes;
    std::vector<float> qlo, qhi;
    if (precision == TPCF_FP32_CHORD) {
        c->band = make_band32(c->edges, delta);
        c->cells = make_cells32(c->edges, c->band, delta, max_cells);
        qlo = c->band.qlo;
        qhi = c->band.qhi;
    } else {
        c->cells = make_cells64(c->edges, max_cells);
        qlo.assign(c->edges.D.size(), 0.0f);
        qhi.assign(c->edges.D.size(), 0.0f);
    }
    std::vector<uint8_t> packed;
    if (c->entry_bytes == 1) {
        packed.resize(c->cells.cells.size());
        for (size_t i = 0; i < packed.size(); ++i) {
            uint16_t v = c->cells.cells[i];
            packed[i] = v == kMulti ? 0xFF : (v & kMedium) ? (uint8_t)(0x80 | (v & 0x7F)) : (uint8_t)v;
        }
    } else {
        packed.resize(c->cells.cells.size() * 2);
        memcpy(packed.data(), c->cells.cells.data(), packed.size());
    }
    int rc;
    if ((rc = upload(c->dD, c->edges.D, ctx->stream)) || (rc = upload(c->dE, c->edges.E, ctx->stream)) ||
        (rc = upload(c->dqlo, qlo, ctx->stream)) || (rc = upload(c->dqhi, qhi, ctx->stream)) ||
        (rc = upload(c->dlut, packed, ctx->stream)))
        return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));   // host vectors stay alive; keep it simple
    if (ctx->compiled.size() > 64) {
        for (auto &kv : ctx->compiled) {
            kv.second->dD.release();
            kv.second->dE.release();
            kv.second->dqlo.release();
            kv.second->dqhi.release();
            kv.second->dlut.release();
        }
        ctx->compiled.clear();
    }
    *out = c.get();
    ctx->compiled[key] = std::move(c);
    return TPCF_OK;
}

constexpr int kRowsPerUnit = kWaves * kWaveSize * 4;   // four wavefronts x 4 rows per lane

// Work units.  DR: every row tile against column chunks of the B catalog.
// DD/RR: every row tile [i0, i1) against j in [i0, n): one masked unit for the
// diagonal block [i0, i0 + T), then unmasked chunks from i0 + T on.
Plan make_plan(bool auto_pairs, int64_t na, int64_t nb, int64_t rb, int64_t re) {
    Plan p;
    const int64_t T = kRowsPerUnit;
    uint64_t pairs = 0;
    if (auto_pairs) {
        for (int64_t i = rb; i < re; ++i)
            pairs += (uint64_t)(na - 1 - i);
    } else {
        pairs = (uint64_t)(re - rb) * (uint64_t)nb;
    }
    p.pairs = pairs;
    // column chunk: aim for >= ~4096 units on big requests, within [256, 16384]
    double per_unit = (double)pairs / 4096.0 / (double)T;
    int64_t bj = (int64_t)per_unit;
    bj = (bj + 255) / 256 * 256;
    if (bj < 256)
        bj = 256;
    if (bj > 16384)
        bj = 16384;
    for (int64_t i0 = rb; i0 < re; i0 += T) {
        int64_t i1 = i0 + T < re ? i0 + T : re;
        if (auto_pairs) {
            int64_t dend = i0 + T < na ? i0 + T : na;
            if (i0 + 1 < dend)
                p.units.push_back(Unit{(int32_t)i0, (int32_t)i1, (int32_t)i0, (int32_t)dend});
            for (int64_t j0 = dend; j0 < na; j0 += bj) {
                int64_t j1 = j0 + bj < na ? j0 + bj : na;
                p.units.push_back(Unit{(int32_t)i0, (int32_t)i1, (int32_t)j0, (int32_t)j1});
            }
        } else {
            for (int64_t j0 = 0; j0 < nb; j0 += bj) {
                int64_t j1 = j0 + bj < nb ? j0 + bj : nb;
                p.units.push_back(Unit{(int32_t)i0, (int32_t)i1, (int32_t)j0, (int32_t)j1});
            }
        }
    }
    return p;
}

int get_plan(tpcf_ctx *ctx, bool auto_pairs, int64_t na, int64_t nb, int64_t rb, int64_t re,
             Plan **out) {
    char buf[128];
    snprintf(buf, sizeof buf, "%d:%lld:%lld:%lld:%lld", (int)auto_pairs, (long long)na,
             (long long)nb, (long long)rb, (long long)re);
    auto it = ctx->plans.find(buf);
    if (it != ctx->plans.end()) {
        *out = it->second.get();
        return TPCF_OK;
    }
    auto p = std::make_unique<Plan>(make_plan(auto_pairs, na, nb, rb, re));
    int rc = upload(p->dunits, p->units, ctx->stream);
    if (rc)
        return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (ctx->plans.size() > 32) {
        for (auto &kv : ctx->plans)
            kv.second->dunits.release();
        ctx->plans.clear();
    }
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

// Validate and enqueue one count; the result lands in d_out (nslots u64).
int enqueue_count(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *edges,
                  int32_t nbins, int precision, int64_t row_begin, int64_t row_end,
                  unsigned long long *d_out, uint64_t *expected_pairs) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (kind != TPCF_DD && kind != TPCF_DR && kind != TPCF_RR)
        return fail(TPCF_E_INVALID, "kind must be TPCF_DD, TPCF_DR or TPCF_RR");
    if (precision != TPCF_FP32_CHORD && precision != TPCF_FP64)
        return fail(TPCF_E_INVALID, "precision must be TPCF_FP32_CHORD or TPCF_FP64");
    if (nbins < 1 || nbins > 256)
        return fail(TPCF_E_INVALID, "nbins must be in [1, 256]");
    if (!edges)
        return fail(TPCF_E_INVALID, "bin_edges_deg is NULL");
    const bool auto_pairs = kind != TPCF_DR;
    auto ia = ctx->cats.find(cat_a);
    if (ia == ctx->cats.end())
        return fail(TPCF_E_BADID, "unknown catalog id cat_a");
    const Catalog &A = ia->second;
    const Catalog *B = &A;
    if (auto_pairs) {
        if (cat_b != -1)
            return fail(TPCF_E_INVALID, "DD/RR take one catalog: cat_b must be -1");
    } else {
        auto ib = ctx->cats.find(cat_b);
        if (ib == ctx->cats.end())
            return fail(TPCF_E_BADID, "unknown catalog id cat_b");
        B = &ib->second;
    }
    int64_t rb = row_begin, re = row_end;
    if (rb == -1 && re == -1) {
        rb = 0;
        re = A.n;
    }
    if (rb < 0 || re < rb || re > A.n)
        return fail(TPCF_E_INVALID, "row range must satisfy 0 <= row_begin <= row_end <= n");
    int rc = set_device(ctx);
    if (rc)
        return rc;
    const double delta = A.delta > B->delta ? A.delta : B->delta;
    Compiled *cp = nullptr;
    if ((rc = get_compiled(ctx, edges, nbins, precision, delta, &cp)))
        return rc;
    Plan *plan = nullptr;
    if ((rc = get_plan(ctx, auto_pairs, A.n, B->n, rb, re, &plan)))
        return rc;
    const int nslots = nbins + 2;
    if ((rc = ctx->copies.ensure(sizeof(unsigned long long) * kGlobalCopies * kMaxSlots)))
        return rc;
    if ((rc = ctx->stats.ensure(sizeof(unsigned long long) * 4)))
        return rc;
    unsigned long long *copies = (unsigned long long *)ctx->copies.p;
    HIP_TRY((hipError_t)tpcf_launch_zero_u64(copies, (int64_t)kGlobalCopies * nslots, ctx->stream));

    PairArgs a;
    memset(&a, 0, sizeof a);
    const size_t na = (size_t)(A.n > 0 ? A.n : 1), nbb = (size_t)(B->n > 0 ? B->n : 1);
    a.ax32 = A.d32;
    a.ay32 = A.d32 + na;
    a.az32 = A.d32 + 2 * na;
    a.bx32 = B->d32;
    a.by32 = B->d32 + nbb;
    a.bz32 = B->d32 + 2 * nbb;
    a.ax64 = A.d64;
    a.ay64 = A.d64 + na;
    a.az64 = A.d64 + 2 * na;
    a.bx64 = B->d64;
    a.by64 = B->d64 + nbb;
    a.bz64 = B->d64 + 2 * nbb;
    a.auto_pairs = auto_pairs ? 1 : 0;
    a.units = (const Unit *)plan->dunits.p;
    a.n_units = (int32_t)plan->units.size();
    a.lut = cp->dlut.p;
    a.lut_cells = (int32_t)cp->cells.cells.size();
    a.lut_entry_bytes = cp->entry_bytes;
    a.lut_shift = cp->cells.shift;
    a.lut_lo = cp->cells.lo;
    a.lut_hi = cp->cells.hi;
    a.qlo = (const float *)cp->dqlo.p;
    a.qhi = (const float *)cp->dqhi.p;
    a.E = (const double *)cp->dE.p;
    a.D = (const double *)cp->dD.p;
    a.nedges = nbins + 1;
    a.nslots = nslots;
    a.hist_copies = hist_copies_for(nslots);
    a.hist = copies;
    a.stats = (unsigned long long *)ctx->stats.p;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing && a.n_units > 0) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, ctx->stream));
    }
    int lrc = tpcf_launch_pairs(&a, precision == TPCF_FP32_CHORD ? 0 : 1, ctx->stream);
    if (lrc)
        return fail(TPCF_E_HIP, std::string("pair kernel launch: ") + hipGetErrorString((hipError_t)lrc));
    if (e0) {
        HIP_TRY(hipEventRecord(e1, ctx->stream));
        ctx->events.emplace_back(e0, e1);
    }
    lrc = tpcf_launch_reduce_copies(copies, nslots, d_out, ctx->stream);
    if (lrc)
        return fail(TPCF_E_HIP, std::string("reduce launch: ") + hipGetErrorString((hipError_t)lrc));
    ctx->pairs_since_reset += plan->pairs;
    if (expected_pairs)
        *expected_pairs = plan->pairs;
    return TPCF_OK;
}

}  // namespace

extern "C" {

const char *tpcf_last_error(void) { return g_err.c_str(); }

const char *tpcf_version(void) { return "tpcf 0.1 (gfx950)"; }

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
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    int rc;
    if ((rc = ctx->stats.ensure(sizeof(unsigned long long) * 4)))
        return rc;
    HIP_TRY((hipError_t)tpcf_launch_zero_u64((unsigned long long *)ctx->stats.p, 4, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *out = ctx.release();
    return TPCF_OK;
}

int tpcf_close(tpcf_ctx *ctx) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->cats) {
        if (kv.second.owns64 && kv.second.d64)
            (void)hipFree(kv.second.d64);
        if (kv.second.d32)
            (void)hipFree(kv.second.d32);
    }
    for (auto &kv : ctx->compiled) {
        kv.second->dD.release();
        kv.second->dE.release();
        kv.second->dqlo.release();
        kv.second->dqhi.release();
        kv.second->dlut.release();
    }
    for (auto &kv : ctx->plans)
        kv.second->dunits.release();
    for (auto &ev : ctx->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    ctx->copies.release();
    ctx->outbuf.release();
    ctx->stats.release();
    ctx->scratch.release();
    if (ctx->own_stream)
        (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return TPCF_OK;
}

int tpcf_upload_catalog(tpcf_ctx *ctx, const double *ra_deg, const double *dec_deg, int64_t n,
                        int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (n < 0)
        return fail(TPCF_E_INVALID, "n must be >= 0");
    if (n > 0 && (!ra_deg || !dec_deg))
        return fail(TPCF_E_INVALID, "ra_deg/dec_deg is NULL");
    const double deg = M_PI / 180.0;
    std::vector<double> x((size_t)n), y((size_t)n), z((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(ra_deg[i]) || !isfinite(dec_deg[i]))
            return fail(TPCF_E_INVALID, "ra/dec must be finite");
        double a = ra_deg[i] * deg;
        double b = dec_deg[i] * deg;
        x[i] = cos(b) * cos(a);
        y[i] = cos(b) * sin(a);
        z[i] = sin(b);
    }
    return add_catalog(ctx, x.data(), y.data(), z.data(), n, out_cat);
}

int tpcf_upload_catalog_xyz(tpcf_ctx *ctx, const double *x, const double *y, const double *z,
                            int64_t n, int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    return add_catalog(ctx, x, y, z, n, out_cat);
}

int tpcf_attach_catalog(tpcf_ctx *ctx, const double *d_xyz64, int64_t n, int32_t *out_cat) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    if (!out_cat)
        return fail(TPCF_E_INVALID, "out_cat is NULL");
    if (n < 1 || n > (int64_t)0x7fffffff - 1024)
        return fail(TPCF_E_INVALID, "attach needs 1 <= n < 2^31 - 1024");
    if (!d_xyz64)
        return fail(TPCF_E_INVALID, "d_xyz64 is NULL");
    int rc = set_device(ctx);
    if (rc)
        return rc;
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, d_xyz64) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != ctx->device) {
        (void)hipGetLastError();
        return fail(TPCF_E_INVALID, "d_xyz64 is not device memory of the context's device");
    }
    Catalog c;
    c.n = n;
    c.owns64 = false;
    c.d64 = const_cast<double *>(d_xyz64);
    HIP_TRY(hipMalloc((void **)&c.d32, sizeof(float) * 3 * (size_t)n));
    if ((rc = ctx->scratch.ensure(64)))
        return rc;
    double *dmax = (double *)ctx->scratch.p;
    HIP_TRY((hipError_t)tpcf_launch_zero_u64((unsigned long long *)dmax, 1, ctx->stream));
    int lrc = tpcf_launch_to_float(c.d64, n, c.d32, dmax, ctx->stream);
    double dev = 0.0;
    hipError_t e = (hipError_t)lrc;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&dev, dmax, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(c.d32);
        return fail(TPCF_E_HIP, std::string("attach: ") + hipGetErrorString(e));
    }
    double delta = dev + 4.0 * ldexp(1.0, -53);
    if (!(delta <= kMaxDelta)) {
        (void)hipFree(c.d32);
        return fail(TPCF_E_INVALID, "attached vectors must be finite with | |v|^2 - 1 | <= 2^-20");
    }
    c.delta = delta;
    int32_t id = ctx->next_id++;
    ctx->cats[id] = c;
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
    (void)hipSetDevice(ctx->device);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (it->second.owns64 && it->second.d64)
        (void)hipFree(it->second.d64);
    if (it->second.d32)
        (void)hipFree(it->second.d32);
    ctx->cats.erase(it);
    return TPCF_OK;
}

int tpcf_count(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *bin_edges_deg,
               int32_t nbins, int precision, int64_t row_begin, int64_t row_end, uint64_t *out_u64) {
    if (!out_u64)
        return fail(TPCF_E_INVALID, "out_u64 is NULL");
    if (ctx) {
        int rc = ctx->outbuf.ensure(sizeof(unsigned long long) * kMaxSlots);
        if (rc)
            return rc;
    }
    uint64_t expected = 0;
    int rc = enqueue_count(ctx, kind, cat_a, cat_b, bin_edges_deg, nbins, precision, row_begin, row_end,
                           (unsigned long long *)(ctx ? ctx->outbuf.p : nullptr), &expected);
    if (rc)
        return rc;
    std::vector<uint64_t> h((size_t)nbins + 2);
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->outbuf.p, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    uint64_t tot = 0;
    for (uint64_t v : h)
        tot += v;
    if (tot != expected) {
        char buf[160];
        snprintf(buf, sizeof buf, "slot total %llu differs from the %llu pairs requested",
                 (unsigned long long)tot, (unsigned long long)expected);
        return fail(TPCF_E_INTERNAL, buf);
    }
    memcpy(out_u64, h.data(), sizeof(uint64_t) * h.size());
    return TPCF_OK;
}

int tpcf_count_async(tpcf_ctx *ctx, int kind, int32_t cat_a, int32_t cat_b, const double *bin_edges_deg,
                     int32_t nbins, int precision, int64_t row_begin, int64_t row_end,
                     uint64_t *d_out_u64) {
    if (!d_out_u64)
        return fail(TPCF_E_INVALID, "d_out_u64 is NULL");
    return enqueue_count(ctx, kind, cat_a, cat_b, bin_edges_deg, nbins, precision, row_begin, row_end,
                         (unsigned long long *)d_out_u64, nullptr);
}

int tpcf_synchronize(tpcf_ctx *ctx) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return TPCF_OK;
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
    HIP_TRY(hipStreamSynchronize(ctx->stream));
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

int tpcf_stats(tpcf_ctx *ctx, uint64_t *out_pairs, uint64_t *out_flagged, uint64_t *out_exact, int reset) {
    if (!ctx)
        return fail(TPCF_E_INVALID, "context is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    unsigned long long h[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, ctx->stats.p, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (out_pairs)
        *out_pairs = ctx->pairs_since_reset;
    if (out_flagged)
        *out_flagged = h[1];
    if (out_exact)
        *out_exact = h[2];
    if (reset) {
        HIP_TRY((hipError_t)tpcf_launch_zero_u64((unsigned long long *)ctx->stats.p, 4, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        ctx->pairs_since_reset = 0;
    }
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

int tpcf_compile_cells(const double *bin_edges_deg, int32_t nbins, int precision, double delta_max,
                       int32_t max_cells, int32_t *out_shift, int32_t *out_lo, int32_t *out_hi,
                       uint16_t *out_cells, double *out_E) {
    if (!out_shift || !out_lo || !out_hi || !out_cells)
        return fail(TPCF_E_INVALID, "NULL argument");
    if (precision != TPCF_FP32_CHORD && precision != TPCF_FP64)
        return fail(TPCF_E_INVALID, "precision must be TPCF_FP32_CHORD or TPCF_FP64");
    if (!(delta_max >= 0.0) || delta_max > kMaxDelta)
        return fail(TPCF_E_INVALID, "delta_max must be in [0, 2^-20]");
    if (max_cells < 16 || max_cells > kMaxLutCells)
        return fail(TPCF_E_INVALID, "max_cells must be in [16, 24576]");
    EdgeTables t;
    std::string err;
    if (!compile_edges(bin_edges_deg, nbins, &t, &err))
        return fail(TPCF_E_INVALID, err);
    CellTable c = precision == TPCF_FP32_CHORD ? make_cells32(t, make_band32(t, delta_max), delta_max, max_cells)
                                               : make_cells64(t, max_cells);
    *out_shift = c.shift;
    *out_lo = c.lo;
    *out_hi = c.hi;
    memcpy(out_cells, c.cells.data(), sizeof(uint16_t) * c.cells.size());
    if (out_E)
        for (int k = 0; k <= nbins; ++k)
            out_E[k] = t.E[k];
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

}  // extern "C"
