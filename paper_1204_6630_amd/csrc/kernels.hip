// Pair-counting kernels for gfx950 (MI355X).
//
// The method (paper, Section 3): form the angle of every pair of objects from
// the dot product of their unit vectors, and histogram it with atomic
// updates of per-block partial histograms in on-chip memory that are later
// combined in one histogram in global memory.
//
// gfx950 design:
//   * one work unit = a tile of rows i (four wavefronts, each holding P = 2
//     or 4 points per lane in registers) against a range of columns
//     j; every wavefront walks the same j range, reading each j through the
//     scalar unit (the address is uniform), so no LDS staging of j is needed;
//   * a pair is classified with one table lookup in LDS: the key is the top
//     bits of q = fl32 |f_i - f_j|^2 (FP32_CHORD) or of e = fl64(1 - d)
//     (FP64); a cell whose whole range lies between two edges gives the slot
//     directly, a cell that straddles one edge's band is settled by one
//     threshold comparison, and anything closer is re-decided with the
//     exact FP64 rule d <= D_k;
//   * every wavefront owns a private LDS histogram, layout [slot][copy] with
//     copy = lane mod copies, updated with ds_add_u32; with 32 copies the
//     lanes of each half-wave (the LDS serves 32 lanes per pass) always hit
//     32 distinct banks;
//   * after each unit a wavefront sums its histogram and adds it with 64-bit
//     atomics into one of kGlobalCopies global copies, which a final kernel
//     reduces into the output slots.
//
// The whole file is compiled with -ffp-contract=off: the FP64 dot product is
// evaluated unfused and left to right exactly like the counting rule; the
// FP32 chord^2 uses explicit fmaf, which the error band accounts for.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

using namespace tpcf;

namespace {

// Columns per step of the vector paths (each lane evaluates P x this many
// pairs between two wavefront-wide tests).  Measured on the octant workload:
// 4 columns are 8 % faster than 2 on the FP32 path (fewer tests and loop
// trips per pair), while the FP64 path, with twice the registers per value,
// is 12 % slower at 4 than at 2.
constexpr int kColsPerStepF32 = 4;
constexpr int kColsPerStepF64 = 2;

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// Column coordinates are read through the constant address space: every lane
// of a wavefront reads the same j, so these become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) float *cfloat_p;
typedef const __attribute__((address_space(4))) double *cdouble_p;
typedef const __attribute__((address_space(4))) uint32_t *cword_p;
typedef const __attribute__((address_space(1))) double *gdouble_p;

// Unit and job descriptors are read-only and wavefront-uniform as well: copy
// them word by word through the constant address space (scalar loads).
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    T out;
    cword_p src = (cword_p)p;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(T) / 4); ++w)
        dst[w] = src[w];
    return out;
}

// Clamp into [lo, hi] in one instruction (all operands in VGPRs: gfx9 VOP3
// reads at most one SGPR, which keeps the compiler from forming v_med3).
__device__ __forceinline__ uint32_t med3_u32(uint32_t x, uint32_t lo, uint32_t hi) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

__device__ __forceinline__ int32_t med3_i32(int32_t x, int32_t lo, int32_t hi) {
    int32_t r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// Copy a wavefront-uniform value into a VGPR once, so loops do not
// re-materialise it for every VOP3 that needs a VGPR operand.
__device__ __forceinline__ uint32_t to_vgpr(uint32_t x) {
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// LDS access by 32-bit byte address.
template <bool LUT8>
__device__ __forceinline__ uint32_t lds_read_entry(uint32_t addr) {
    if (LUT8)
        return *(const lds_u8 *)(uintptr_t)addr;
    return *(const lds_u16 *)(uintptr_t)addr;
}

__device__ __forceinline__ void lds_add(uint32_t addr, uint32_t v) {
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// True when `pred` holds on every lane of the (fully active) wavefront.
__device__ __forceinline__ bool wave_all(bool pred) {
    return __builtin_amdgcn_ballot_w64(pred) == ~0ull;
}

// Balanced reductions of the JN x P values of a step (depth ~log3 instead
// of a chain of JN * P dependent instructions).
template <typename T, typename F, int N>
__device__ __forceinline__ T tree_reduce(const T (&v)[N], F f) {
    if constexpr (N == 1) {
        return v[0];
    } else if constexpr (N == 2) {
        return f(v[0], v[1]);
    } else {
        constexpr int M = (N + 2) / 3;
        T w[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            T x = v[3 * i];
            if (3 * i + 1 < N)
                x = f(x, v[3 * i + 1]);
            if (3 * i + 2 < N)
                x = f(x, v[3 * i + 2]);
            w[i] = x;
        }
        return tree_reduce<T, F, M>(w, f);
    }
}

__device__ __forceinline__ void lds_inc(uint32_t addr) {
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)addr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Cell entry codes: a slot (certain for the whole cell), flag | k (edge k
// undecided), or flag | kmask (several edges undecided).  Every test of an
// entry takes the flag bit from a register (Consts::flag): with literal masks
// the compiler narrows the tests to 8 or 16 bits and then spends an extra
// instruction per entry to widen the loaded value again.
template <bool LUT8>
struct Code {
    static constexpr uint32_t flag = LUT8 ? 0x80u : 0x8000u;
    static constexpr uint32_t kmask = LUT8 ? 0x7Fu : 0x7FFFu;
};

// Number of k with d <= D[k]; D is non-increasing in k.
__device__ __forceinline__ uint32_t count_le(double d, const double *D, int n) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (d <= D[mid])
            lo = mid + 1;
        else
            hi = mid;
    }
    return (uint32_t)lo;
}

// FP64 dot product of the counting rule: (x_i x_j + y_i y_j) + z_i z_j with
// every operation rounded (contraction is off for this file).
__device__ __forceinline__ double exact_dot(double xi, double yi, double zi,
                                            double xj, double yj, double zj) {
    double t = xi * xj;
    double u = yi * yj;
    double s = t + u;
    double v = zi * zj;
    return s + v;
}

// 3-D: squared distance of the counting rule, (dx^2 + dy^2) + dz^2 of the
// FP64 coordinate differences, every operation rounded.
__device__ __forceinline__ double exact_d2(double xi, double yi, double zi,
                                           double xj, double yj, double zj) {
    double dx = xi - xj;
    double dy = yi - yj;
    double dz = zi - zj;
    double t = dx * dx;
    double u = dy * dy;
    double s = t + u;
    double v = dz * dz;
    return s + v;
}

// The value the thresholds D_k are compared with (past edge k when
// value <= D_k): the dot product for angles, minus the squared distance in
// 3-D (where D_k = -S_k).
template <bool M3>
__device__ __forceinline__ double rule_value(double xi, double yi, double zi,
                                             double xj, double yj, double zj) {
    return M3 ? -exact_d2(xi, yi, zi, xj, yj, zj) : exact_dot(xi, yi, zi, xj, yj, zj);
}

struct Smem {
    uint32_t *hist;      // kWaves x (nslots + 1) x copies
    double *D;
    double *E;
    float2 *qband;       // FP32 band (qlo_k, qhi_k), one 8-byte read per edge
    float2 *pband;       // band in p (plo_k, phi_k), dot-product path
    double *erad;        // edges in radians (pruning)
    unsigned char *lut;
    uint32_t hist_addr;  // LDS byte address of hist
    uint32_t lut_addr;   // LDS byte address of lut
    uint32_t plut_addr;  // LDS byte address of the dot-product key's table
    uint32_t stage_addr; // LDS byte address of the wavefronts' column staging buffers
};

// LDS layout: the cell table first (at the start of the block's LDS, so a
// wrapped table is indexed by the masked key itself), then the histograms
// and the edge thresholds: after the table, or for a wrapped table at
// aux_off, inside the part of the table that no key reaches.
__device__ __forceinline__ Smem carve(unsigned char *base, const PairArgs &a) {
    Smem s;
    const int aux = a.lut_direct ? a.aux_off : (a.lut_cells * a.lut_entry_bytes + 15) & ~15;
    int hist_words = kWaves * (a.nslots + 1) * a.hist_copies;
    s.lut = base;
    s.hist = reinterpret_cast<uint32_t *>(base + aux);
    s.D = reinterpret_cast<double *>(base + aux + hist_words * 4);
    s.E = s.D + a.nedges;
    s.erad = s.E + a.nedges;
    s.qband = reinterpret_cast<float2 *>(s.erad + a.nedges);
    s.pband = s.qband + a.nedges;
    s.hist_addr = (uint32_t)(uintptr_t)(lds_u32 *)s.hist;
    s.lut_addr = (uint32_t)(uintptr_t)(lds_u8 *)s.lut;
    s.plut_addr = s.lut_addr + (uint32_t)a.plut_lds;
    s.stage_addr = s.lut_addr + (uint32_t)a.stage_lds;
    return s;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, kWaveSize));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, kWaveSize);
    return v;
}

// Sum one wavefront's LDS histogram into a global copy and clear it; with
// region copies (r0, r1 non-null) the sums also go there.
__device__ void flush_wave(const PairArgs &a, const Smem &s, unsigned long long *hist, unsigned long long *r0,
                           unsigned long long *r1, int wave, int lane, int copy) {
    const int C = a.hist_copies;
    uint32_t *h = s.hist + wave * (a.nslots + 1) * C;
    const size_t off = (size_t)copy * a.nslots;
    for (int s0 = 0; s0 < a.nslots; s0 += kWaveSize) {
        int slot = s0 + lane;
        if (slot < a.nslots) {
            uint32_t acc = 0;
            uint32_t *row = h + slot * C;
            // skewed walk over the copies: lanes of a half-wave hit distinct banks
            for (int c = 0; c < C; ++c) {
                int cc = (c + lane) & (C - 1);
                acc += row[cc];
                row[cc] = 0;
            }
            if (acc) {
                atomicAdd(&hist[off + slot], (unsigned long long)acc);
                if (r0)
                    atomicAdd(&r0[off + slot], (unsigned long long)acc);
                if (r1)
                    atomicAdd(&r1[off + slot], (unsigned long long)acc);
            }
        }
    }
}

// A flagged entry: edge k alone is undecided in the cell (its FP32 band,
// one 8-byte LDS read, settles q outside [qlo_k, qhi_k); inside it the exact
// FP64 rule compares d with D_k), or several are (the rule counts them).
template <bool LUT8, bool M3>
__device__ __forceinline__ uint32_t resolve_fp32(uint32_t ent, uint32_t flag, float q, const Smem &s,
                                                 const PairArgs &a, const JobDev &jb, int i, int j,
                                                 uint32_t &n_exact) {
    if (ent != (flag | Code<LUT8>::kmask)) {
        const int k = (int)(ent ^ flag);
        const float2 b = s.qband[k];
        if (q < b.x)
            return (uint32_t)k;
        if (q >= b.y)
            return (uint32_t)(k + 1);
        ++n_exact;
        const double d = rule_value<M3>(jb.ax64[i], jb.ay64[i], jb.az64[i], jb.bx64[j], jb.by64[j], jb.bz64[j]);
        return (uint32_t)k + (d <= s.D[k] ? 1u : 0u);
    }
    ++n_exact;
    const double d = rule_value<M3>(jb.ax64[i], jb.ay64[i], jb.az64[i], jb.bx64[j], jb.by64[j], jb.bz64[j]);
    return count_le(d, s.D, a.nedges);
}

template <bool LUT8>
__device__ __forceinline__ uint32_t resolve_fp64(uint32_t ent, uint32_t flag, double e, double d,
                                                 const Smem &s, const PairArgs &a,
                                                 uint32_t &n_exact) {
    if (ent != (flag | Code<LUT8>::kmask)) {
        int k = (int)(ent ^ flag);
        double Ek = s.E[k];
        if (e > Ek)
            return (uint32_t)(k + 1);
        if (e < Ek)
            return (uint32_t)k;
        ++n_exact;
        return (uint32_t)k + (d <= s.D[k] ? 1u : 0u);
    }
    ++n_exact;
    return count_le(d, s.D, a.nedges);
}

// Work statistics of one lane: pairs that left the table path, pairs decided
// by the exact FP64 rule, and (wavefront-uniform) steps that took the rare path.
struct Counters {
    uint32_t flag = 0, exact = 0, rare = 0;
    uint32_t beyond = 0;        // this lane's pairs counted beyond the last edge (per unit)
    // Step kinds of the current column range, 16 bits each (wavefront-
    // uniform, kept in scalar registers): steps beyond the last edge, in one
    // slot, in two slots, and (dot-product kernels) steps that formed the
    // chord; folded into the totals below after every range of at most
    // kFoldCols columns.
    uint64_t steps = 0;
    uint32_t beyond_steps = 0, one_slot_steps = 0, two_slot_steps = 0, chord_steps = 0;
    uint32_t pruned_blocks = 0;     // wavefront blocks (P x 64 rows x 64 columns) binned whole (uniform)

    __device__ __forceinline__ void fold() {
        beyond_steps += (uint32_t)(steps & 0xFFFF);
        one_slot_steps += (uint32_t)((steps >> 16) & 0xFFFF);
        two_slot_steps += (uint32_t)((steps >> 32) & 0xFFFF);
        chord_steps += (uint32_t)(steps >> 48);
        steps = 0;
    }
};

// Longest column range one call of the column loops covers: at most
// kFoldCols / 2 steps, below the 16-bit step fields of Counters.
constexpr int kFoldCols = 65536;

// How a wavefront step was binned (wavefront-uniform).  A step beyond the
// last edge adds nothing to the histograms: the caller counts its pairs in
// the lane's register.  kUndecided: the dot product did not settle the step.
enum : uint32_t { kBeyond = 0, kOneSlot = 1, kTwoSlot = 2, kLookup = 3, kUndecided = 4 };

// Per-step bookkeeping, done once after the step whichever way it went (so
// the counters are not carried through the step's branches).  The step
// functions' codes are wavefront-uniform, but the compiler cannot tell
// (their paths hold per-lane branches), so the callers pass them through
// readfirstlane to keep the code and the branches on it scalar.
template <uint32_t N>
__device__ __forceinline__ void account(uint32_t code, Counters &cnt) {
    cnt.beyond += code == kBeyond ? N : 0u;
    cnt.steps += code <= kTwoSlot ? (uint64_t)1 << (16 * code) : 0;
}

// Loop constants of one wavefront.
struct Consts {
    uint32_t shift;
    uint32_t wbits;         // wrapped table: log2 of its entry count
    float qfloor;           // wrapped table: the floor q is summed from
    uint32_t clo, chi;      // clamp range (VGPR copies)
    uint32_t lutbias;       // LDS address of cell c is c * entry_bytes + lutbias
    uint32_t rowstep;       // bytes between slots of the histogram
    uint32_t lanebase;      // LDS address of this lane's copy of slot 0
    uint32_t flag;          // flag bit of the cell entries (VGPR copy)
    uint32_t beyond;        // PairArgs::beyond_key (VGPR copy)
    float pbeyond;          // PairArgs::p_beyond
    // dot-product key's table: cell = bits(q') >> pshift clamped to
    // [pclo, pchi], LDS address cell * entry_bytes + pbias (VGPR copies: the
    // dot-product loop then needs no scalar registers for them)
    uint32_t pshift, pclo, pchi, pbias;
    uint32_t qdot;          // bits of PairArgs::q_dot
};

// LDS address of the cell-table entry of an FP32 key (the bit pattern of q)
// and of an FP64 key (the high word of e; arithmetic shift, so e < 0 lands
// in the bottom cell).
template <bool LUT8, bool DIRECT>
__device__ __forceinline__ uint32_t addr32(uint32_t bits, const Consts &k) {
    if (DIRECT) {
        // wrapped byte table at LDS address 0 (the kernel has no static LDS,
        // so its dynamic LDS starts there): the floor keeps every key within
        // 2^wbits cells of bits(q_floor) >> shift (checked on the host), so
        // the key's low wbits bits address it without a clamp
        return __builtin_amdgcn_ubfe(bits, k.shift, k.wbits);
    }
    return med3_u32(bits >> k.shift, k.clo, k.chi) * (LUT8 ? 1u : 2u) + k.lutbias;
}

template <bool LUT8>
__device__ __forceinline__ uint32_t addr64(int32_t hi, const Consts &k) {
    const int32_t c = med3_i32(hi >> (int)k.shift, (int32_t)k.clo, (int32_t)k.chi);
    return (uint32_t)c * (LUT8 ? 1u : 2u) + k.lutbias;
}

// Slot range of a lane's pairs.  A cell entry bounds the slots of its keys: a
// certain slot s gives [s, s], edge k undecided gives [k, k+1] (a cell with
// several undecided edges gives [kmask, kmask+1], which no test below
// accepts).  Slots never decrease as the key grows (keys below the table
// share its bottom cell), so the entries of a lane's smallest and largest key
// bound the slots of all its pairs: lo = the lower end of the first, and
// span = the upper end of the second minus lo.
template <bool LUT8>
__device__ __forceinline__ void slot_range(uint32_t e_lo, uint32_t e_hi, uint32_t &lo, uint32_t &span) {
    constexpr uint32_t m = Code<LUT8>::kmask, sh = LUT8 ? 7 : 15;
    lo = e_lo & m;
    span = (e_hi & m) + (e_hi >> sh) - lo;
}

// One slot for all of a lane's pairs (span 0).  When that holds on every lane
// the step adds its pairs with one LDS atomic per lane instead of a lookup and
// an atomic per pair.  A lane's rows (and a wavefront's 256) are consecutive
// in the Morton order, so at angles large against their extent this is
// common (on the octant workload 49 % of the FP32 steps that are not beyond
// the last edge pass).
__device__ __forceinline__ bool one_slot_step(uint32_t lo, uint32_t span, uint32_t n, const Consts &k,
                                              Counters &cnt) {
    if (!wave_all(span == 0))
        return false;
    lds_add(__umul24(lo, k.rowstep) + k.lanebase, n);
    return true;
}

// Two adjacent slots [lo, lo+1] (or one) for all of a lane's pairs, on every
// lane: then each pair needs one comparison with edge lo's threshold instead
// of a table lookup, and the step adds its pairs with two LDS atomics per
// lane.
template <bool LUT8>
__device__ __forceinline__ bool two_slot_range(uint32_t lo, uint32_t span) {
    return (__builtin_amdgcn_ballot_w64(span <= 1u) & __builtin_amdgcn_ballot_w64(lo != Code<LUT8>::kmask)) == ~0ull;
}

__device__ __forceinline__ void two_slot_add(uint32_t base, uint32_t n, uint32_t n_up, const Consts &k,
                                             Counters &cnt) {
    // both adds on every lane (a lane with one slot adds 0 to the next row,
    // at most the discard row): no per-lane branch, so the step's outcome
    // stays wavefront-uniform for the compiler
    const uint32_t addr = __umul24(base, k.rowstep) + k.lanebase;
    lds_add(addr, n - n_up);
    lds_add(addr + k.rowstep, n_up);
}

// ---------------------------------------------------------------------------
// Exact tile pruning.  A bounding cap (unit centre c, angular radius rho) of
// the wavefront's rows and one of an aligned 64-column block bound the
// geometric angle phi (between the normalised directions) of every pair of
// the block to [acos(c_r . c_b) - rho_r - rho_b, acos(c_r . c_b) + rho_r +
// rho_b], widened by kPruneMargin (the FP32 row copies and the cap
// arithmetic).  The counting rule does not see phi but the FP64 dot product
// of the stored vectors, whose squared norms deviate from 1 by up to delta:
// d = |v_i| |v_j| cos(phi) + err with |v_i| |v_j| in [1 - delta, 1 + delta]
// and |err| <= kPruneDotSlack (the rule's rounding).  So every pair's d lies
// in [lo - delta |lo| - slack, hi + delta |hi| + slack] for any bounds
// lo <= cos(phi) <= hi over the block (prune_slot forms them without
// trigonometric functions); when no threshold D_k falls inside that interval
// every pair passes the same edges, and the wavefront adds the block's pairs
// to that slot without evaluating them.

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, kWaveSize);
    return v;
}

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fmin(v, __shfl_xor(v, off, kWaveSize));
    return v;
}

struct Cap {
    double x, y, z, rho;
};

// A wavefront-uniform double moved to scalar registers (lane 0's value).
__device__ __forceinline__ double uniform_d(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    // readfirstlane returns a signed int: take its 32 bits without sign extension
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}

__device__ __forceinline__ Cap uniform_cap(const Cap &c) {
    return Cap{uniform_d(c.x), uniform_d(c.y), uniform_d(c.z), uniform_d(c.rho)};
}

// Cap of the points (x, y, z) held by the lanes (every lane contributes n
// points; duplicates are harmless).  Identical on every lane.
template <int N>
__device__ __forceinline__ Cap cap_of(const double (&x)[N], const double (&y)[N], const double (&z)[N]) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        sx += x[p];
        sy += y[p];
        sz += z[p];
    }
    sx = wave_sum_d(sx);
    sy = wave_sum_d(sy);
    sz = wave_sum_d(sz);
    const double norm = sqrt(sx * sx + sy * sy + sz * sz);
    Cap c;
    if (!(norm > 1e-3)) {       // points spread over the sphere: no useful cap
        c.x = 1.0;
        c.y = c.z = 0.0;
        c.rho = M_PI;
        return c;
    }
    c.x = sx / norm;
    c.y = sy / norm;
    c.z = sz / norm;
    double m = 1.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        const double len = sqrt(x[p] * x[p] + y[p] * y[p] + z[p] * z[p]);
        m = fmin(m, (c.x * x[p] + c.y * y[p] + c.z * z[p]) / len);
    }
    m = wave_min_d(m);
    c.rho = acos(fmin(fmax(m, -1.0), 1.0)) + 1e-12;
    return c;
}

// Number of thresholds (non-increasing, in LDS) that v passes (v <= T[k]),
// and whether w passes the same ones: lane L compares both with T[L + 64 m],
// one LDS read and two ballots per 64 thresholds.  -1 when they differ.
// Wavefront-uniform.
__device__ __forceinline__ int same_count_le(double v, double w, const double *T, int n, int lane) {
    int count = 0;
    for (int b = 0; b < n; b += kWaveSize) {
        const double t = b + lane < n ? T[b + lane] : -__builtin_huge_val();
        const uint64_t mv = __builtin_amdgcn_ballot_w64(v <= t);
        if (mv != __builtin_amdgcn_ballot_w64(w <= t))
            return -1;
        count += __builtin_popcountll(mv);
    }
    return count;
}

// The slot of every pair between the row cap and the column block's cap, or
// -1 when the test cannot prove one (see above; delta bounds the catalogs'
// | |v|^2 - 1 |).  With c = cos(theta_c) the dot product of the two centres,
// sn an upper bound of sin(theta_c) and rho the summed radii, every pair's
// geometric angle is theta_c + t with |t| <= rho, and
// cos(theta_c + t) = c cos t - sin(theta_c) sin t lies within
// [c - sn rho - max(c, 0) rho^2 / 2, c + sn rho + max(-c, 0) rho^2 / 2]
// (1 - t^2 / 2 <= cos t <= 1, |sin t| <= |t|).  No trigonometric function is
// evaluated; the margin in rho (1e-6 rad) widens the interval by at least
// sn 1e-6 > 6e-14, far above the rounding of this arithmetic.
__device__ __forceinline__ int prune_slot(const Cap &r, const double *bcap, const Smem &s, int nedges,
                                          double delta, int lane) {
    const cdouble_p bc = (cdouble_p)bcap;
    const double c = fmin(fmax(r.x * bc[0] + r.y * bc[1] + r.z * bc[2], -1.0), 1.0);
    const double rho = r.rho + bc[3] + kPruneMargin;
    const double h = 0.5 * rho * rho;
    // an upper bound of the sine: 1 - c^2 formed as (1 - c)(1 + c), plus the
    // rounding of c and of that product
    const double sn = sqrt((1.0 - c) * (1.0 + c) + 4e-15);
    double hi = c + sn * rho + fmax(-c, 0.0) * h;
    double lo = c - sn * rho - fmax(c, 0.0) * h;
    hi = hi + delta * fabs(hi) + kPruneDotSlack;
    lo = lo - delta * fabs(lo) - kPruneDotSlack;
    // pairs with the largest d pass the fewest edges
    return same_count_le(hi, lo, s.D, nedges, lane);
}

// 3-D: bounding ball of the points held by the lanes (centre = their mean,
// radius = the largest distance from it, widened by 1e-12 relative).
// Identical on every lane.
template <int N>
__device__ __forceinline__ Cap ball_of(const double (&x)[N], const double (&y)[N], const double (&z)[N]) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        sx += x[p];
        sy += y[p];
        sz += z[p];
    }
    const double inv = 1.0 / (double)(N * kWaveSize);
    Cap c;
    c.x = wave_sum_d(sx) * inv;
    c.y = wave_sum_d(sy) * inv;
    c.z = wave_sum_d(sz) * inv;
    double m = 0.0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        const double dx = x[p] - c.x, dy = y[p] - c.y, dz = z[p] - c.z;
        m = fmax(m, sqrt(dx * dx + dy * dy + dz * dz));
    }
    c.rho = wave_max_d(m) * (1.0 + 1e-12);
    return c;
}

// 3-D: the slot of every pair between the row ball and the column block's
// ball, or -1.  Their distances lie within [|c_r - c_b| -+ (rho_r + rho_b)],
// widened by margin (the FP32 copies of the rows, at most 2^-22 R) and by
// 1e-12 relative (the rule's and this arithmetic's rounding).
__device__ __forceinline__ int prune_slot3(const Cap &r, const double *bcap, const Smem &s, int nedges,
                                           double margin, int lane) {
    const cdouble_p bc = (cdouble_p)bcap;
    const double dx = r.x - bc[0], dy = r.y - bc[1], dz = r.z - bc[2];
    const double dc = sqrt(dx * dx + dy * dy + dz * dz);
    const double spread = r.rho + bc[3];
    const double w = margin + 1e-12 * (dc + spread);
    const double lo = dc - spread - w, hi = dc + spread + w;
    // a pair at distance r passes edge k when e_k <= r: lane L compares
    // both ends with edge L + 64 m
    int count = 0;
    for (int b = 0; b < nedges; b += kWaveSize) {
        const double t = b + lane < nedges ? s.erad[b + lane] : __builtin_huge_val();
        const uint64_t ml = __builtin_amdgcn_ballot_w64(t <= lo);
        if (ml != __builtin_amdgcn_ballot_w64(t <= hi))
            return -1;
        count += __builtin_popcountll(ml);
    }
    return count;
}

// Block cap and block slot for either metric.
template <bool M3, int N>
__device__ __forceinline__ Cap block_cap(const double (&x)[N], const double (&y)[N], const double (&z)[N]) {
    return uniform_cap(M3 ? ball_of<N>(x, y, z) : cap_of<N>(x, y, z));
}

template <bool M3>
__device__ __forceinline__ int block_slot(const Cap &r, const double *bcap, const Smem &s, const PairArgs &a,
                                          int lane) {
    return M3 ? prune_slot3(r, bcap, s, a.nedges, a.prune_margin, lane)
              : prune_slot(r, bcap, s, a.nedges, a.prune_delta, lane);
}

// Add n pairs of this lane to `slot` (the overflow slot through the register
// counter).
__device__ __forceinline__ void bin_block(int slot, uint32_t n, const PairArgs &a, const Consts &k,
                                          Counters &cnt) {
    if (slot == a.nslots - 1)
        cnt.beyond += n;
    else
        lds_add(__umul24((uint32_t)slot, k.rowstep) + k.lanebase, n);
}

// Row p of a wavefront lane whose rows start at ib: lane L holds the P
// consecutive rows ib + P L ... ib + P L + P - 1.  Rows are stored in Morton
// order, so a lane's rows lie close together and its pairs of a step span a
// narrow range of angles: more lanes fall in one slot, or in two adjacent
// ones, than with rows 64 apart.
template <int P>
__device__ __forceinline__ int row_of(int ib, int lane, int p) {
    return ib + lane * P + p;
}

// One step: JN columns against the P rows of every lane.  All JN * P table
// lookups are issued first; one test sends the wavefront to the rare path if
// any lane needs it; then the JN * P histogram increments follow.
template <bool LUT8, bool MASKED, int P, int JN, bool DIRECT, bool M3, bool ONE>
__device__ __forceinline__ uint32_t step_fp32(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k,
                                          const float (&xi)[P], const float (&yi)[P],
                                          const float (&zi)[P], const int (&ii)[P],
                                          int ib, int lane, int ie, int j, const float (&xj)[JN],
                                          const float (&yj)[JN], const float (&zj)[JN], uint32_t &qmin,
                                          Counters &cnt) {
    float q[JN][P];
    uint32_t ent[JN][P];
#pragma unroll
    for (int t = 0; t < JN; ++t) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            float dx = xi[p] - xj[t];
            float dy = yi[p] - yj[t];
            float dz = zi[p] - zj[t];
            // the wrapped table's sum starts at its floor (same instruction count)
            float v = DIRECT ? __fmaf_rn(dx, dx, k.qfloor) : dx * dx;
            v = __fmaf_rn(dy, dy, v);
            v = __fmaf_rn(dz, dz, v);
            q[t][p] = v;
        }
    }
    if (!MASKED) {
        // every pair of the step certainly beyond the last edge (q >= 0, so the
        // bit patterns order like the values): count them in a register
        uint32_t qb[JN * P];
#pragma unroll
        for (int t = 0; t < JN; ++t)
#pragma unroll
            for (int p = 0; p < P; ++p)
                qb[t * P + p] = __float_as_uint(q[t][p]);
        const uint32_t m = tree_reduce(qb, [](uint32_t x, uint32_t y) { return min(x, y); });
        qmin = m;
        if (wave_all(m >= k.beyond))
            return kBeyond;
        if constexpr (ONE) {
            // every pair of the step in one slot: the cells of each lane's
            // smallest and largest key hold the same certain slot on every lane
            // (a wavefront's 4 x 64 rows are consecutive in the Morton order, so
            // at angles large against their extent this is common; with pruning
            // such blocks are mostly pruned, and the kernel skips the test to
            // save its registers)
            const uint32_t mx = tree_reduce(qb, [](uint32_t x, uint32_t y) { return max(x, y); });
            uint32_t base, span;
            slot_range<LUT8>(lds_read_entry<LUT8>(addr32<LUT8, DIRECT>(m, k)),
                             lds_read_entry<LUT8>(addr32<LUT8, DIRECT>(mx, k)), base, span);
            if (one_slot_step(base, span, JN * P, k, cnt))
                return kOneSlot;
            if (two_slot_range<LUT8>(base, span)) {
                // a pair is past edge `base` when q >= qhi and not past it when
                // q < qlo.  x = fl(q - qhi) is >= 0 exactly when q >= qhi
                // (a difference of floats rounds to zero only when they are
                // equal, and then to +0), and x < 0 with |x| > w = fl(qhi - qlo)
                // puts q below qlo (fl is monotone): these pairs are decided,
                // the sign bit of x marking those not past.  As int32 bit
                // patterns, exactly the decided x lie above that of -w (a
                // negative float's pattern grows with its magnitude), so one
                // signed minimum checks every pair.  Lanes with one slot
                // compare with +inf (x = -inf) and decide everything; a NaN
                // width (an edge at 0) decides nothing.  (The sign bit counts
                // the pairs: no compare-and-carry, whose mask hazard costs
                // wait states on gfx950.)
                const float2 b = s.qband[min(base, (uint32_t)(a.nedges - 1))];
                const float thr = span ? b.y : __builtin_huge_valf();
                const float nw = -(b.y - b.x);
                const int32_t lim = !span ? INT32_MIN : nw == nw ? (int32_t)__float_as_uint(nw) : INT32_MAX;
                uint32_t n_below = 0;
                int32_t m = INT32_MAX;
#pragma unroll
                for (int t = 0; t < JN; ++t)
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const float x = q[t][p] - thr;
                        n_below += __float_as_uint(x) >> 31;
                        m = min(m, (int32_t)__float_as_uint(x));
                    }
                // count before the test, so the differences die here
                asm volatile("" : "+v"(n_below));
                if (wave_all(m > lim)) {
                    two_slot_add(base, JN * P, JN * P - n_below, k, cnt);
                    return kTwoSlot;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < JN; ++t) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            ent[t][p] = lds_read_entry<LUT8>(addr32<LUT8, DIRECT>(__float_as_uint(q[t][p]), k));
        }
    }
    uint32_t any = 0;
#pragma unroll
    for (int t = 0; t < JN; ++t)
#pragma unroll
        for (int p = 0; p < P; ++p)
            any |= ent[t][p];
    if (any & k.flag) {
        ++cnt.rare;             // wavefront steps that took the rare path
#pragma unroll
        for (int t = 0; t < JN; ++t)
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (ent[t][p] & k.flag) {
                    ++cnt.flag;
                    // the row is formed here, on demand, from an opaque copy
                    // of the lane index, so no row index or address of this
                    // rare path is hoisted into registers of the loop (tail
                    // lanes read row ib)
                    int l = lane;
                    asm volatile("" : "+v"(l));
                    int i = row_of<P>(ib, l, p);
                    i = i < ie ? i : ib;
                    ent[t][p] = resolve_fp32<LUT8, M3>(ent[t][p], k.flag, q[t][p], s, a, jb, i, j + t, cnt.exact);
                }
    }
#pragma unroll
    for (int t = 0; t < JN; ++t)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            uint32_t e = ent[t][p];
            if (MASKED) {
                bool ok = ii[p] < ie && (!jb.auto_pairs || j + t > ii[p]);
                e = ok ? e : (uint32_t)a.nslots;
            }
            lds_inc(__umul24(e, k.rowstep) + k.lanebase);
        }
    return kLookup;
}

// LDS address of the dot-product key's cell: q' = fl(2 - 2p) as a bit
// pattern, a negative q' (p > 1) read as +0 through a signed maximum.
template <bool LUT8>
__device__ __forceinline__ uint32_t paddr(float qd, const Consts &k) {
    const uint32_t bits = (uint32_t)max((int32_t)__float_as_uint(qd), 0);
    return med3_u32(bits >> k.pshift, k.pclo, k.pchi) * (LUT8 ? 1u : 2u) + k.pbias;
}

// One step of an angular FP32 wavefront decided from the dot product of the
// FP32 copies, p = fl32(f_i . f_j) (one multiply and two FMAs per pair;
// |p - d| is bounded by the host's dot_error32).  Whole steps only: all
// pairs beyond the last edge (p <= p_beyond), every lane's pairs in one slot,
// or in two adjacent slots with every pair outside the band in p of the edge
// between them.  The slot range of a lane comes from the cells of the key
// q' = fl(2 - 2p) of its largest and smallest p (q' does not increase with
// p).  Returns the step's code, or kUndecided, having counted nothing, when
// p does not decide the step; the caller then forms the chord.
template <bool LUT8, int P, int JN>
__device__ __forceinline__ uint32_t step_dot(const PairArgs &a, const Smem &s, const Consts &k, const float (&xi)[P],
                                         const float (&yi)[P], const float (&zi)[P], const float (&xj)[JN],
                                         const float (&yj)[JN], const float (&zj)[JN], Counters &cnt) {
    float p[JN][P];
#pragma unroll
    for (int t = 0; t < JN; ++t)
#pragma unroll
        for (int r = 0; r < P; ++r)
            p[t][r] = __fmaf_rn(zi[r], zj[t], __fmaf_rn(yi[r], yj[t], xi[r] * xj[t]));
    float pf[JN * P];
#pragma unroll
    for (int t = 0; t < JN; ++t)
#pragma unroll
        for (int r = 0; r < P; ++r)
            pf[t * P + r] = p[t][r];
    const float pmax = tree_reduce(pf, [](float x, float y) { return fmaxf(x, y); });
    if (wave_all(pmax <= k.pbeyond))
        return kBeyond;
    const float pmin = tree_reduce(pf, [](float x, float y) { return fminf(x, y); });
    uint32_t base, span;
    slot_range<LUT8>(lds_read_entry<LUT8>(paddr<LUT8>(__fmaf_rn(-2.0f, pmax, 2.0f), k)),
                     lds_read_entry<LUT8>(paddr<LUT8>(__fmaf_rn(-2.0f, pmin, 2.0f), k)), base, span);
    if (one_slot_step(base, span, JN * P, k, cnt))
        return kOneSlot;
    if (two_slot_range<LUT8>(base, span)) {
        // a pair is past edge `base` when p <= plo and not past it when
        // p >= phi.  x = fl(p - phi) is >= 0 exactly when p >= phi, and x < 0
        // with |x| > w = fl(phi - plo) puts p below plo: these pairs are
        // decided, the sign bit of x counting those in the upper slot, and
        // as int32 bit patterns exactly they lie above that of -w (as on the
        // chord path).  Lanes with one slot compare with -inf (x = +inf,
        // lower slot) and decide everything; a NaN width decides nothing.
        const float2 b = s.pband[min(base, (uint32_t)(a.nedges - 1))];
        const float thr = span ? b.y : -__builtin_huge_valf();
        const float nw = -(b.y - b.x);
        const int32_t lim = !span ? INT32_MIN : nw == nw ? (int32_t)__float_as_uint(nw) : INT32_MAX;
        uint32_t n_up = 0;
        int32_t m = INT32_MAX;
#pragma unroll
        for (int t = 0; t < JN; ++t)
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const float x = p[t][r] - thr;
                n_up += __float_as_uint(x) >> 31;
                m = min(m, (int32_t)__float_as_uint(x));
            }
        asm volatile("" : "+v"(n_up));
        if (wave_all(m > lim)) {
            two_slot_add(base, JN * P, n_up, k, cnt);
            return kTwoSlot;
        }
    }
    return kUndecided;
}

template <bool LUT8, bool MASKED, int P, int JN, bool M3, bool ONE>
__device__ __forceinline__ uint32_t step_fp64(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k,
                                          const double (&xi)[P], const double (&yi)[P],
                                          const double (&zi)[P], const int (&ii)[P], int ie,
                                          int j, cdouble_p bx, cdouble_p by, cdouble_p bz,
                                          Counters &cnt) {
    double xj[JN], yj[JN], zj[JN];
#pragma unroll
    for (int t = 0; t < JN; ++t) {
        xj[t] = bx[j + t];
        yj[t] = by[j + t];
        zj[t] = bz[j + t];
    }
    // e: the table key's value (1 - d, or r^2 in 3-D); the rule's value d
    // itself is formed again, with the same operations, in the rare path
    double e[JN][P];
    uint32_t ent[JN][P];
#pragma unroll
    for (int t = 0; t < JN; ++t) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (M3)
                e[t][p] = exact_d2(xi[p], yi[p], zi[p], xj[t], yj[t], zj[t]);
            else
                e[t][p] = 1.0 - exact_dot(xi[p], yi[p], zi[p], xj[t], yj[t], zj[t]);
        }
    }
    if (!MASKED) {
        // high word of e above that of E_last implies e > E_last for every pair
        int32_t m = __double2hiint(e[0][0]);
#pragma unroll
        for (int t = 0; t < JN; ++t)
#pragma unroll
            for (int p = 0; p < P; ++p)
                m = min(m, __double2hiint(e[t][p]));
        if (wave_all(m > (int32_t)k.beyond)) {
            return kBeyond;
        }
        if constexpr (ONE) {
            // every pair of the step in one slot (as on the FP32 path)
            int32_t mx = __double2hiint(e[0][0]);
#pragma unroll
            for (int t = 0; t < JN; ++t)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    mx = max(mx, __double2hiint(e[t][p]));
            uint32_t base, span;
            slot_range<LUT8>(lds_read_entry<LUT8>(addr64<LUT8>(m, k)), lds_read_entry<LUT8>(addr64<LUT8>(mx, k)),
                             base, span);
            if (one_slot_step(base, span, JN * P, k, cnt))
                return kOneSlot;
            if (two_slot_range<LUT8>(base, span)) {
                // past edge `base` when e > E_base, not past it when e < E_base,
                // and the exact rule decides e == E_base (as in resolve_fp64);
                // lanes with one slot compare with +inf
                const double thr = span ? s.E[min(base, (uint32_t)(a.nedges - 1))] : __builtin_huge_val();
                uint32_t n_up = 0, tie = 0;
#pragma unroll
                for (int t = 0; t < JN; ++t)
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        n_up += e[t][p] > thr ? 1u : 0u;
                        tie |= e[t][p] == thr ? 1u : 0u;
                    }
                // count before the test, so nothing of it stays live past it
                asm volatile("" : "+v"(n_up), "+v"(tie));
                if (!__builtin_amdgcn_ballot_w64(tie != 0)) {
                    two_slot_add(base, JN * P, n_up, k, cnt);
                    return kTwoSlot;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < JN; ++t) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            ent[t][p] = lds_read_entry<LUT8>(addr64<LUT8>(__double2hiint(e[t][p]), k));
        }
    }
    uint32_t any = 0;
#pragma unroll
    for (int t = 0; t < JN; ++t)
#pragma unroll
        for (int p = 0; p < P; ++p)
            any |= ent[t][p];
    if (any & k.flag) {
        ++cnt.rare;             // wavefront steps that took the rare path
#pragma unroll
        for (int t = 0; t < JN; ++t)
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (ent[t][p] & k.flag) {
                    ++cnt.flag;
                    const double d = rule_value<M3>(xi[p], yi[p], zi[p], xj[t], yj[t], zj[t]);
                    ent[t][p] = resolve_fp64<LUT8>(ent[t][p], k.flag, e[t][p], d, s, a, cnt.exact);
                }
    }
#pragma unroll
    for (int t = 0; t < JN; ++t)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            uint32_t v = ent[t][p];
            if (MASKED) {
                bool ok = ii[p] < ie && (!jb.auto_pairs || j + t > ii[p]);
                v = ok ? v : (uint32_t)a.nslots;
            }
            lds_inc(__umul24(v, k.rowstep) + k.lanebase);
        }
    return kLookup;
}

// One wavefront's copy of columns [base, base + kStageCols) of the three
// FP32 coordinate arrays (global addresses px, py, pz) into its LDS staging
// buffer at byte address dst, as kStageCols x, then y, then z floats: lane L
// below 3 kStageCols / 4 copies 16 bytes, columns [base + 4 sub, +4) of
// coordinate L / 16 (sub = L % 16) to bytes [16 L, +16), with loads that
// write LDS directly.  Columns are clamped to start at most at last (a
// clamped slot is never read).  The lane index is an opaque copy, so that
// nothing of this stays in registers through the steps.
__device__ __forceinline__ void stage_columns(uint64_t px, uint64_t py, uint64_t pz, int lane, int base, int last,
                                              uint32_t dst) {
    typedef __attribute__((address_space(3))) void *lds_p;
    typedef __attribute__((address_space(1))) void *glb_p;
    constexpr int Q = kStageCols / 4;
    static_assert(Q == 16, "16 lanes per coordinate");
    int ln = lane;
    asm volatile("" : "+v"(ln));
    if (ln < 3 * Q) {
        const int coord = ln >> 4, sub = ln & 15;
        const uint64_t p = coord == 0 ? px : coord == 1 ? py : pz;
        const int col = min(base + 4 * sub, last);
        __builtin_amdgcn_global_load_lds((glb_p)((const float *)(uintptr_t)p + col), (lds_p)(uintptr_t)dst, 16, 0,
                                         0);
    }
}

// Steps decided by the dot product alone (dot-product kernels): from column
// j on, while step_dot settles each step of kColsPerStepF32 columns (beyond
// the last edge, one slot, two slots).  Returns the first column of the
// step it could not settle (or of the columns left over), which the chord
// loop takes next.
template <bool LUT8, int P>
__device__ __forceinline__ int dot_run(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k,
                                       const float (&xi)[P], const float (&yi)[P], const float (&zi)[P], int j,
                                       int j1, int lane, Counters &cnt) {
    // The columns go through LDS: the wavefront copies kStageCols of them at
    // a time (stage_columns) into one of its two staging buffers, the next
    // block's copy in flight while the current block is used, and every step
    // reads its 4 columns' coordinates with three broadcast LDS reads.
    // Scalar loads of every step's columns, whose waits stall the
    // wavefront, are measured 1.1-1.2x slower.
    constexpr int W = kColsPerStepF32, C = kStageCols, Q = C / 4;
    if (j + W > j1)
        return j;
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef volatile __attribute__((address_space(3))) f4 *lf4_p;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t st0 = s.stage_addr + wave * (uint32_t)(2 * C * 12);
    // (opaque copies of the column pointers: the choice among them in
    // stage_columns is then made on values and never turned into a
    // lane-indexed read of the job record, which would move it to scratch
    // memory)
    uint64_t px = (uint64_t)(uintptr_t)jb.bx32, py = (uint64_t)(uintptr_t)jb.by32,
             pz = (uint64_t)(uintptr_t)jb.bz32;
    asm volatile("" : "+s"(px), "+s"(py), "+s"(pz));
    int cb = j;
    uint32_t buf = 0;
    // a copy still in flight from an earlier run (into either buffer) lands
    // before the first block is copied, then the first block lands
    __builtin_amdgcn_s_waitcnt(0x0F70);     // vmcnt(0)
    stage_columns(px, py, pz, lane, cb, j1 - W, st0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    bool more = cb + C + W <= j1;
    if (more)
        stage_columns(px, py, pz, lane, cb + C, j1 - W, st0 + C * 12);
    uint64_t n = 0;     // steps beyond, in one slot, in two slots (16-bit fields)
    for (;;) {
        const lf4_p st = (lf4_p)(uintptr_t)(st0 + buf * (C * 12));
        const int ce = min(cb + C, j1);
        bool stop = false;
        for (; j + W <= ce; j += W) {
            const int q = (j - cb) >> 2;
            const f4 vx = st[q], vy = st[q + Q], vz = st[q + 2 * Q];
            const float xj[W] = {vx[0], vx[1], vx[2], vx[3]}, yj[W] = {vy[0], vy[1], vy[2], vy[3]},
                        zj[W] = {vz[0], vz[1], vz[2], vz[3]};
            const uint32_t code = step_dot<LUT8, P, W>(a, s, k, xi, yi, zi, xj, yj, zj, cnt);
            if (code == kUndecided) {
                stop = true;
                break;
            }
            n += (uint64_t)1 << (16 * code);
        }
        if (stop || !more)
            break;
        // the block is used up (j == cb + C): wait for the other buffer's
        // copy, then start the next one into this buffer
        __builtin_amdgcn_s_waitcnt(0x0F70);
        cb += C;
        buf ^= 1;
        more = cb + C + W <= j1;
        if (more)
            stage_columns(px, py, pz, lane, cb + C, j1 - W, st0 + (buf ^ 1) * (C * 12));
    }
    cnt.beyond += (uint32_t)(n & 0xFFFF) * (uint32_t)(W * P);
    cnt.steps += n;
    return j;
}

// Columns [j0, j1) against the P rows of every lane (FP32 path).  With DOT
// (angular kernels with the dot-product table), after an unmasked chord step
// that needed no per-pair lookup and whose smallest q reached q_dot on every
// lane (the wavefront works at angles where p decides most steps), the
// following steps go to dot_run; the chord loop resumes at the first step p
// leaves undecided.
template <bool LUT8, bool MASKED, int P, bool DIRECT, bool M3, bool ONE, bool DOT>
__device__ __forceinline__ void cols_fp32(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k,
                                          const float (&xi)[P], const float (&yi)[P], const float (&zi)[P],
                                          const int (&ii)[P], int ib, int lane, int ie, int j0, int j1,
                                          Counters &cnt) {
    cfloat_p bx = (cfloat_p)jb.bx32;
    cfloat_p by = (cfloat_p)jb.by32;
    cfloat_p bz = (cfloat_p)jb.bz32;
    constexpr int JN = kColsPerStepF32;
    int j = j0;
    if (j + JN <= j1) {
        // the columns of the next step are read (through the scalar unit)
        // while the current step computes; the last prefetch re-reads the
        // current columns, so no read leaves [j0, j1)
        float xj[JN], yj[JN], zj[JN];
#pragma unroll
        for (int t = 0; t < JN; ++t) {
            xj[t] = bx[j + t];
            yj[t] = by[j + t];
            zj[t] = bz[j + t];
        }
        for (; j + JN <= j1; j += JN) {
            const int jn = j + 2 * JN <= j1 ? j + JN : j;
            float xn[JN], yn[JN], zn[JN];
#pragma unroll
            for (int t = 0; t < JN; ++t) {
                xn[t] = bx[jn + t];
                yn[t] = by[jn + t];
                zn[t] = bz[jn + t];
            }
            // keep the prefetch at the top of the step
            __builtin_amdgcn_sched_barrier(0);
            uint32_t qmin = 0;
            const uint32_t code = __builtin_amdgcn_readfirstlane(step_fp32<LUT8, MASKED, P, JN, DIRECT, M3, ONE>(
                a, jb, s, k, xi, yi, zi, ii, ib, lane, ie, j, xj, yj, zj, qmin, cnt));
            account<JN * P>(code, cnt);
#pragma unroll
            for (int t = 0; t < JN; ++t) {
                xj[t] = xn[t];
                yj[t] = yn[t];
                zj[t] = zn[t];
            }
            if constexpr (DOT && !MASKED && !M3) {
                cnt.steps += (uint64_t)1 << 48;     // a step that formed the chord
                if (code != kLookup && wave_all(qmin >= k.qdot)) {
                    const int js = dot_run<LUT8, P>(a, jb, s, k, xi, yi, zi, j + JN, j1, lane, cnt);
                    if (js != j + JN) {
                        j = js - JN;
                        if (js + JN <= j1) {
#pragma unroll
                            for (int t = 0; t < JN; ++t) {
                                xj[t] = bx[js + t];
                                yj[t] = by[js + t];
                                zj[t] = bz[js + t];
                            }
                        }
                    }
                }
            }
        }
    }
    for (; j < j1; ++j) {
        const float xj[1] = {bx[j]}, yj[1] = {by[j]}, zj[1] = {bz[j]};
        uint32_t qmin = 0;
        account<P>(__builtin_amdgcn_readfirstlane(step_fp32<LUT8, MASKED, P, 1, DIRECT, M3, false>(
                       a, jb, s, k, xi, yi, zi, ii, ib, lane, ie, j, xj, yj, zj, qmin, cnt)),
                   cnt);
    }
    cnt.fold();
}


// One wavefront: rows [ib, ie) (at most P * 64) against columns [j0, j1).
template <bool LUT8, bool MASKED, int P, bool DIRECT, bool PRUNE, bool M3, bool DOT>
__device__ void rows_fp32(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k, int ib, int ie,
                          int j0, int j1, int lane, Counters &cnt) {
    float xi[P], yi[P], zi[P];
    int ii[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        int i = row_of<P>(ib, lane, p);
        ii[p] = i;
        const int il = i < ie ? i : ib;    // tail lanes read a valid row; masked below
        xi[p] = jb.ax32[il];
        yi[p] = jb.ay32[il];
        zi[p] = jb.az32[il];
    }
    if (PRUNE && !MASKED && jb.bcaps) {
        double xd[P], yd[P], zd[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            xd[p] = xi[p];
            yd[p] = yi[p];
            zd[p] = zi[p];
        }
        const Cap rc = block_cap<M3, P>(xd, yd, zd);
        for (int j = j0; j < j1;) {
            const int jn = min(j1, (j & ~63) + 64);
            if ((j & 63) == 0 && jn - j == 64) {
                const int slot = block_slot<M3>(rc, jb.bcaps + (size_t)(j >> 6) * 4, s, a, lane);
                if (slot >= 0) {
                    bin_block(slot, P * 64, a, k, cnt);
                    ++cnt.pruned_blocks;
                    j = jn;
                    continue;
                }
            }
            cols_fp32<LUT8, MASKED, P, DIRECT, M3, true, DOT>(a, jb, s, k, xi, yi, zi, ii, ib, lane, ie, j, jn, cnt);
            j = jn;
        }
        return;
    }
    for (int jc = j0; jc < j1; jc += kFoldCols)
        cols_fp32<LUT8, MASKED, P, DIRECT, M3, true, DOT>(a, jb, s, k, xi, yi, zi, ii, ib, lane, ie, jc,
                                                          j1 - jc > kFoldCols ? jc + kFoldCols : j1, cnt);
}

// Columns [j0, j1) against the P rows of every lane (FP64 vector path).
template <bool LUT8, bool MASKED, int P, bool M3, bool ONE>
__device__ __forceinline__ void cols_fp64(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k,
                                          const double (&xi)[P], const double (&yi)[P],
                                          const double (&zi)[P], const int (&ii)[P], int ie, int j0, int j1,
                                          Counters &cnt) {
    cdouble_p bx = (cdouble_p)jb.bx64;
    cdouble_p by = (cdouble_p)jb.by64;
    cdouble_p bz = (cdouble_p)jb.bz64;
    int j = j0;
    for (; j + kColsPerStepF64 <= j1; j += kColsPerStepF64)
        account<kColsPerStepF64 * P>(__builtin_amdgcn_readfirstlane(step_fp64<LUT8, MASKED, P, kColsPerStepF64, M3, ONE>(
                                         a, jb, s, k, xi, yi, zi, ii, ie, j, bx, by, bz, cnt)),
                                     cnt);
    for (; j < j1; ++j)
        account<P>(__builtin_amdgcn_readfirstlane(
                       step_fp64<LUT8, MASKED, P, 1, M3, false>(a, jb, s, k, xi, yi, zi, ii, ie, j, bx, by, bz, cnt)),
                   cnt);
    cnt.fold();
}

template <bool LUT8, bool MASKED, int P, bool PRUNE, bool M3>
__device__ void rows_fp64(const PairArgs &a, const JobDev &jb, const Smem &s, const Consts &k, int ib, int ie,
                          int j0, int j1, int lane, Counters &cnt) {
    double xi[P], yi[P], zi[P];
    int ii[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        int i = row_of<P>(ib, lane, p);
        ii[p] = i;
        int il = i < ie ? i : ib;
        xi[p] = jb.ax64[il];
        yi[p] = jb.ay64[il];
        zi[p] = jb.az64[il];
    }
    if (PRUNE && !MASKED && jb.bcaps) {
        const Cap rc = block_cap<M3, P>(xi, yi, zi);
        for (int j = j0; j < j1;) {
            const int jn = min(j1, (j & ~63) + 64);
            if ((j & 63) == 0 && jn - j == 64) {
                const int slot = block_slot<M3>(rc, jb.bcaps + (size_t)(j >> 6) * 4, s, a, lane);
                if (slot >= 0) {
                    bin_block(slot, P * 64, a, k, cnt);
                    ++cnt.pruned_blocks;
                    j = jn;
                    continue;
                }
            }
            cols_fp64<LUT8, MASKED, P, M3, true>(a, jb, s, k, xi, yi, zi, ii, ie, j, jn, cnt);
            j = jn;
        }
        return;
    }
    for (int jc = j0; jc < j1; jc += kFoldCols)
        cols_fp64<LUT8, MASKED, P, M3, true>(a, jb, s, k, xi, yi, zi, ii, ie, jc,
                                             j1 - jc > kFoldCols ? jc + kFoldCols : j1, cnt);
}

// PREC: 0 FP32 chord with a clamped table, 3 FP32 chord with a direct byte
// table, 6 and 7 the same with the dot product tried first (angular), 1 FP64
// vector; 3-D distances: 5 FP32 squared distance with a
// clamped table, 4 FP64 vector.  P: rows per lane (a wavefront covers P * 64
// rows of a unit).
template <int PREC, bool LUT8, int P, bool PRUNE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(waves_per_eu_of(PREC)))) void pairs_kernel(
    PairArgs a) {
    constexpr int kRowsPerWave = P * kWaveSize;
    extern __shared__ __align__(16) unsigned char smem[];
    const Smem s = carve(smem, a);
    const int tid = threadIdx.x;
    const int lane = tid & (kWaveSize - 1);
    const int wave = tid >> 6;

    const int hist_words = kWaves * (a.nslots + 1) * a.hist_copies;
    for (int w = tid; w < hist_words; w += kBlock)
        s.hist[w] = 0;
    const int lut_bytes = a.lut_cells * (LUT8 ? 1 : 2);
    const unsigned char *glut = reinterpret_cast<const unsigned char *>(a.lut);
    // a wrapped table's unused piece holds the histograms and thresholds,
    // which the copy must not overwrite
    const uint32_t aux_lo = a.lut_direct ? (uint32_t)a.aux_off : (uint32_t)lut_bytes;
    const uint32_t aux_n = (uint32_t)(hist_words * 4 + a.nedges * kEdgeLdsBytes);
    for (int b = tid; b < lut_bytes; b += kBlock)
        if ((uint32_t)b - aux_lo >= aux_n)
            s.lut[b] = glut[b];
    if (PREC >= 6) {
        const int plut_bytes = a.plut_cells * (LUT8 ? 1 : 2);
        for (int b = tid; b < plut_bytes; b += kBlock)
            s.lut[a.plut_lds + b] = glut[a.plut_src + b];
    }
    for (int e = tid; e < a.nedges; e += kBlock) {
        s.D[e] = a.D[e];
        s.E[e] = a.E[e];
        s.qband[e] = make_float2(a.qlo[e], a.qhi[e]);
        s.pband[e] = PREC >= 6 ? make_float2(a.qlo[a.nedges + e], a.qhi[a.nedges + e]) : make_float2(0.0f, 0.0f);
        s.erad[e] = a.erad ? a.erad[e] : 0.0;
    }
    __syncthreads();

    Consts k;
    k.shift = (uint32_t)a.lut_shift;
    k.wbits = (uint32_t)a.lut_wrap_bits;
    k.qfloor = a.q_floor;
    k.clo = to_vgpr((uint32_t)a.lut_lo);
    k.chi = to_vgpr((uint32_t)a.lut_hi);
    k.lutbias = s.lut_addr - (uint32_t)a.lut_lo * (LUT8 ? 1u : 2u);
    k.rowstep = (uint32_t)a.hist_copies * 4u;
    k.flag = to_vgpr(Code<LUT8>::flag);
    k.beyond = to_vgpr(a.beyond_key);
    k.pbeyond = a.p_beyond;
    k.pshift = to_vgpr((uint32_t)a.plut_shift);
    k.pclo = to_vgpr((uint32_t)a.plut_lo);
    k.pchi = to_vgpr((uint32_t)a.plut_hi);
    k.pbias = to_vgpr(s.plut_addr - (uint32_t)a.plut_lo * (LUT8 ? 1u : 2u));
    k.qdot = __float_as_uint(a.q_dot);
    k.lanebase = s.hist_addr +
                 (uint32_t)((wave * (a.nslots + 1) * a.hist_copies + (lane & (a.hist_copies - 1))) * 4);
    Counters cnt;

    uint32_t n_skip = 0;
    // Each wavefront takes work items in order from the queue, so the items in
    // flight are always a window of consecutive units that share their column
    // range (the plan orders units column chunk first) and the column data
    // stays in L2.  Every wavefront leaves once the queue is exhausted.
    const uint32_t n_items = (uint32_t)a.n_units * kWaves;
    for (;;) {
        uint32_t item = 0;
        if (lane == 0)
            item = atomicAdd(a.queue, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= n_items)
            break;
        const int u = (int)(item / kWaves);
        const int part = (int)(item % kWaves);
        const Unit un = load_uniform(a.units + u);
        const JobDev jb = a.jobs ? load_uniform(a.jobs + un.job) : a.job0;
        const int ib = un.i0 + part * kRowsPerWave;
        if (ib < un.i1) {
            // a cancelled job skips its remaining units (the flag lives in host memory)
            if (jb.cancel && __builtin_amdgcn_readfirstlane(
                                 __hip_atomic_load(jb.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) {
                ++n_skip;
                continue;
            }
            const int ie = min(un.i1, ib + kRowsPerWave);
            const int rlo = max(un.row_lo, ib);
            const bool masked = (ie - ib < kRowsPerWave) || (jb.auto_pairs && un.j0 < ie) || rlo > ib;
            if (PREC == 0 || PREC == 3 || PREC == 5 || PREC == 6 || PREC == 7) {
                constexpr bool M3 = PREC == 5;
                constexpr bool DIRECT = PREC == 3 || PREC == 7;
                // with pruning, the blocks left to evaluate lie across edges,
                // where the dot product rarely settles a step: chord only
                constexpr bool DOT = PREC >= 6 && !PRUNE;
                if (masked)
                    rows_fp32<LUT8, true, P, DIRECT, PRUNE, M3, DOT>(a, jb, s, k, ib, ie, un.j0, un.j1, lane, cnt);
                else
                    rows_fp32<LUT8, false, P, DIRECT, PRUNE, M3, DOT>(a, jb, s, k, ib, ie, un.j0, un.j1, lane, cnt);
            } else {
                constexpr bool M3 = PREC == 4;
                if (masked)
                    rows_fp64<LUT8, true, P, PRUNE, M3>(a, jb, s, k, ib, ie, un.j0, un.j1, lane, cnt);
                else
                    rows_fp64<LUT8, false, P, PRUNE, M3>(a, jb, s, k, ib, ie, un.j0, un.j1, lane, cnt);
            }
            // pairs counted beyond the last edge go to this lane's copy of the
            // overflow slot; then the wave's own LDS region is flushed (no
            // block barrier needed)
            if (cnt.beyond) {
                lds_add(__umul24((uint32_t)(a.nslots - 1), k.rowstep) + k.lanebase, cnt.beyond);
                cnt.beyond = 0;
            }
            unsigned long long *r0 = nullptr, *r1 = nullptr;
            if (jb.touch) {
                const size_t per_region = (size_t)kGlobalCopies * a.nslots;
                if (un.reg_a >= 0)
                    r0 = jb.touch + (size_t)un.reg_a * per_region;
                if (un.reg_b >= 0 && un.reg_b != un.reg_a)
                    r1 = jb.touch + (size_t)un.reg_b * per_region;
            }
            flush_wave(a, s, jb.hist, r0, r1, wave, lane, (int)(item & (kGlobalCopies - 1)));
        }
    }
    // column copies into LDS still in flight land before the wavefront ends
    if (PREC >= 6 && !PRUNE)
        __builtin_amdgcn_s_waitcnt(0x0F70);
    uint32_t f = wave_sum(cnt.flag);
    uint32_t x = wave_sum(cnt.exact);
    if (lane == 0) {
        if (f)
            atomicAdd(&a.stats[1], (unsigned long long)f);
        if (x)
            atomicAdd(&a.stats[2], (unsigned long long)x);
        if (n_skip)
            atomicAdd(&a.stats[3], (unsigned long long)n_skip);
        if (cnt.rare)
            atomicAdd(&a.stats[4], (unsigned long long)cnt.rare);
        if (cnt.beyond_steps)
            atomicAdd(&a.stats[5], (unsigned long long)cnt.beyond_steps);
        if (cnt.one_slot_steps)
            atomicAdd(&a.stats[6], (unsigned long long)cnt.one_slot_steps);
        if (cnt.two_slot_steps)
            atomicAdd(&a.stats[0], (unsigned long long)cnt.two_slot_steps);
        if (cnt.pruned_blocks)
            atomicAdd(&a.stats[7], (unsigned long long)cnt.pruned_blocks * (unsigned long long)(kRowsPerWave * 64));
        if (cnt.chord_steps)
            atomicAdd(&a.stats[8], (unsigned long long)cnt.chord_steps);
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = 0ull;
}

// One block per job: sum its kGlobalCopies histogram copies.
__global__ void reduce_copies_kernel(const unsigned long long *copies, int32_t nslots,
                                     unsigned long long *out) {
    const unsigned long long *c = copies + (size_t)blockIdx.x * kGlobalCopies * nslots;
    for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
        unsigned long long acc = 0;
        for (int g = 0; g < kGlobalCopies; ++g)
            acc += c[(size_t)g * nslots + s];
        out[(size_t)blockIdx.x * nslots + s] = acc;
    }
}

// FP32 copies (round to nearest) of an FP64 SoA block of 3n values, and the
// largest |x^2 + y^2 + z^2 - 1| (FP64, unfused), +inf if a value is not finite.
// With `given` (caller-owned FP32 copies) nothing is written: every given
// value is compared with the rounded FP64 one and *mismatch is set if one
// differs.
__global__ void to_float_kernel(const double *xyz, int64_t n, float *out, const float *given,
                                unsigned long long *maxdev, unsigned long long *mismatch) {
    __shared__ double red[256];
    double m = 0.0;
    bool differs = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
        if (given) {
            differs = differs || given[i] != (float)x || given[n + i] != (float)y || given[2 * n + i] != (float)z;
        } else {
            out[i] = (float)x;
            out[n + i] = (float)y;
            out[2 * n + i] = (float)z;
        }
        double t = x * x;
        double u = y * y;
        double v = z * z;
        double r = (t + u) + v;
        double dev = fabs(r - 1.0);
        if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !(dev == dev))
            dev = __builtin_huge_val();
        m = dev > m ? dev : m;
    }
    if (differs)
        atomicOr(mismatch, 1ull);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + off] ? red[threadIdx.x] : red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(maxdev, (unsigned long long)__double_as_longlong(red[0]));
}

// Bounding cap of every aligned group of 64 stored points: one wavefront per
// group (4 doubles: unit centre, angular radius).
__global__ __launch_bounds__(256) void caps64_kernel(const double *xyz, int64_t n, double *caps,
                                                     int64_t groups, int metric) {
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = threadIdx.x >> 6;
    for (int64_t g = (int64_t)blockIdx.x * kWaves + wave; g < groups; g += (int64_t)gridDim.x * kWaves) {
        // lanes past the catalog repeat the group's first point
        const int64_t p = g * 64 + lane < n ? g * 64 + lane : g * 64;
        const double x[1] = {xyz[p]}, y[1] = {xyz[n + p]}, z[1] = {xyz[2 * n + p]};
        const Cap c = metric ? ball_of<1>(x, y, z) : cap_of<1>(x, y, z);
        if (lane == 0) {
            caps[4 * g] = c.x;
            caps[4 * g + 1] = c.y;
            caps[4 * g + 2] = c.z;
            caps[4 * g + 3] = c.rho;
        }
    }
}

int grid_for(int n_units, int lds, int blocks_per_cu) {
    static int cus = 0, lds_per_cu = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            cus = prop.multiProcessorCount;
            lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
        }
        if (cus <= 0)
            cus = 256;
        if (lds_per_cu <= 0)
            lds_per_cu = 160 * 1024;
    }
    int per_cu = lds > 0 ? lds_per_cu / lds : 8;
    if (per_cu < 1)
        per_cu = 1;
    if (per_cu > 8)
        per_cu = 8;
    // the resident blocks by default (the work queue balances them);
    // blocks_per_cu > 0 overrides
    long long g = blocks_per_cu > 0 ? (long long)cus * blocks_per_cu : (long long)cus * per_cu;
    if (g > n_units)
        g = n_units;
    if (g < 1)
        g = 1;
    return (int)g;
}

template <int PR, bool B8>
void launch_pairs(int P, bool prune, int grid, int lds, hipStream_t st, const PairArgs &a) {
    if (prune) {
        if (P == 2)
            hipLaunchKernelGGL((pairs_kernel<PR, B8, 2, true>), dim3(grid), dim3(kBlock), lds, st, a);
        else
            hipLaunchKernelGGL((pairs_kernel<PR, B8, 4, true>), dim3(grid), dim3(kBlock), lds, st, a);
    } else {
        if (P == 2)
            hipLaunchKernelGGL((pairs_kernel<PR, B8, 2, false>), dim3(grid), dim3(kBlock), lds, st, a);
        else
            hipLaunchKernelGGL((pairs_kernel<PR, B8, 4, false>), dim3(grid), dim3(kBlock), lds, st, a);
    }
}


}  // namespace

extern "C" int tpcf_launch_pairs(const PairArgs *args, int precision, void *stream) {
    if (args->n_units <= 0)
        return 0;
    const int lds = args->plut_cells > 0 && precision == 0 && args->metric == 0
                        ? args->stage_lds + kStageBytes
                        : lds_bytes(args->nslots, args->hist_copies, args->lut_cells, args->lut_entry_bytes,
                                    args->nedges, args->lut_direct ? args->aux_off : -1);
    const int grid = grid_for(args->n_units, lds, args->blocks_per_cu);
    hipStream_t st = (hipStream_t)stream;
    const bool b8 = args->lut_entry_bytes == 1;
    const int P = args->rows_per_lane;
    if (P != 2 && P != 4)
        return (int)hipErrorInvalidValue;
    const bool prune = args->prune != 0;
    if (args->metric == 1) {
        if (precision == 0 && b8)
            launch_pairs<5, true>(P, prune, grid, lds, st, *args);
        else if (precision == 0)
            launch_pairs<5, false>(P, prune, grid, lds, st, *args);
        else if (precision == 1 && b8)
            launch_pairs<4, true>(P, prune, grid, lds, st, *args);
        else if (precision == 1)
            launch_pairs<4, false>(P, prune, grid, lds, st, *args);
        else
            return (int)hipErrorInvalidValue;
        return (int)hipGetLastError();
    }
    if (precision == 0 && args->plut_cells > 0) {
        if (b8 && args->lut_direct)
            launch_pairs<7, true>(P, prune, grid, lds, st, *args);
        else if (b8)
            launch_pairs<6, true>(P, prune, grid, lds, st, *args);
        else
            launch_pairs<6, false>(P, prune, grid, lds, st, *args);
    } else if (precision == 0) {
        if (b8 && args->lut_direct)
            launch_pairs<3, true>(P, prune, grid, lds, st, *args);
        else if (b8)
            launch_pairs<0, true>(P, prune, grid, lds, st, *args);
        else
            launch_pairs<0, false>(P, prune, grid, lds, st, *args);
    } else if (precision == 1) {
        if (b8)
            launch_pairs<1, true>(P, prune, grid, lds, st, *args);
        else
            launch_pairs<1, false>(P, prune, grid, lds, st, *args);
    } else {
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

extern "C" int tpcf_launch_caps64(const double *xyz64, int64_t n, double *caps, int metric, void *stream) {
    const int64_t groups = (n + 63) / 64;
    if (groups <= 0)
        return 0;
    int64_t blocks = (groups + kWaves - 1) / kWaves;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(caps64_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, xyz64, n,
                       caps, groups, metric);
    return (int)hipGetLastError();
}

extern "C" int tpcf_launch_zero_u64(unsigned long long *p, int64_t n, void *stream) {
    if (n <= 0)
        return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p, n);
    return (int)hipGetLastError();
}

extern "C" int tpcf_launch_reduce_copies(const unsigned long long *copies, int32_t nslots,
                                         int32_t njobs, unsigned long long *out, void *stream) {
    if (njobs <= 0)
        return 0;
    hipLaunchKernelGGL(reduce_copies_kernel, dim3((unsigned)njobs), dim3(256), 0, (hipStream_t)stream,
                       copies, nslots, out);
    return (int)hipGetLastError();
}

extern "C" int tpcf_launch_to_float(const double *xyz64, int64_t n, float *xyz32, const float *given32,
                                    unsigned long long *check_out, void *stream) {
    // check_out: two device words zeroed by the caller, [0] the largest norm
    // deviation (a double's bits), [1] non-zero if a given FP32 copy differs
    if (n <= 0)
        return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048)
        blocks = 2048;
    hipLaunchKernelGGL(to_float_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       xyz64, n, xyz32, given32, check_out, check_out + 1);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Work area of the entry point that allocates nothing (tpcf_count_noalloc):
// a fixed array in device memory, one per device the library runs on, held
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, looked up once per device with
// that device current, and kernels receive that pointer as an argument.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

extern "C" int tpcf_scratch_init(int device) {
    if (device < 0 || device >= kMaxScratchDevices)
        return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device])
        return 0;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess)
        return (int)e;
    if (cur != device)
        return (int)hipErrorInvalidDevice;      // the caller makes the device current first
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return (int)e;
    if (!ptr)
        return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return 0;
}

extern "C" void *tpcf_scratch_ptr(int device) {
    if (device < 0 || device >= kMaxScratchDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}
