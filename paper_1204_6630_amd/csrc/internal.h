// Internal declarations shared by the host library and the HIP kernels.
// Not part of the public ABI (see include/tpcf.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace tpcf {

// Threads per block and the i-points each lane keeps in registers.
constexpr int kWaves = 4;
constexpr int kWaveSize = 64;
constexpr int kBlock = kWaves * kWaveSize;

// LDS budget of the cell table; entries are one byte when every slot and
// edge index fits in 7 bits, else two bytes.
constexpr int kMaxLutBytes = 24576;
constexpr int kMaxLutCells = kMaxLutBytes;        // with one-byte entries
// Largest cell-table budget a tuning may ask for, and the wrapped FP32
// tables' default budget (table, histograms and thresholds together).
constexpr int kMaxDirectLutBytes = 33792;
constexpr int kWrapLutBytes = 32768;
// Angular FP32 launches also hold the dot-product key's cell table (bytes).
// By default FP32 launches with clamped tables size them so that a block's
// LDS stays within kLdsTarget: six blocks of four wavefronts in a CU's
// 160 KiB, the occupancy those kernels are compiled for (waves_per_eu).
constexpr int kDotLutBytes = 1024;
constexpr int kLdsTarget = 27296;
// Wavefronts per SIMD a pair kernel is compiled for: 6 for the FP32 paths
// with clamped tables (0, 5, 6; at most 80 VGPRs, a few spilled), 5 for the
// FP64 paths (1, 4) and the wrapped FP32 tables (3, 7), whose 32 KB of LDS
// per block allows no more.
constexpr int waves_per_eu_of(int path) {
    return path == 0 || path == 5 || path == 6 ? 6 : 5;
}
// Dot-product kernels: each wavefront stages kStageCols columns at a time in
// LDS, in two buffers of x, y and z floats.
constexpr int kStageCols = 64;
constexpr int kStageBytes = kWaves * 2 * kStageCols * 12;
// Work statistics words of a launch (see PairArgs::stats).
constexpr int kStats = 9;
// Histogram copies in global memory (u64), indexed by work unit.
constexpr int kGlobalCopies = 64;
// Largest number of output slots (nbins <= 256 -> nbins + 2 slots).
constexpr int kMaxSlots = 258;

// Table entry encoding.  A cell of the squared-chord (FP32) or 1 - d (FP64)
// axis maps to:
//   0 .. kMaxSlots-1   the slot, certain for every value in the cell;
//   kMedium | k        exactly one edge k is undecided inside the cell;
//   kMulti             several edges are undecided: use the exact rule.
// One-byte tables use 0x80 | k and 0xFF instead (slots and k below 0x7F).
constexpr uint16_t kMedium = 0x8000;
constexpr uint16_t kMulti = 0xFFFF;
constexpr int kMaxSlots8 = 127;

// One work unit: the row tile starting at i0 with valid rows [row_lo, i1),
// against columns j in [j0, j1) of job `job` (col_lo == j0, kept for the
// plan's bookkeeping).  A unit needs per-pair masking when its valid rows do
// not fill the tile or, for auto-pairs, when its columns overlap its rows
// (the j <= i diagonal).
// reg_a / reg_b: jackknife regions of the unit's rows and columns (-1: none).
struct Unit {
    int32_t i0, i1, j0, j1;
    int32_t job, row_lo, col_lo, reg_a;
    int32_t reg_b, pad0, pad1, pad2;
};

// One counting job of a launch: catalogs A (rows i) and B (columns j) as
// structures of arrays, the pair kind, and where its histogram goes.
struct JobDev {
    const float *ax32, *ay32, *az32;
    const float *bx32, *by32, *bz32;
    const double *ax64, *ay64, *az64;
    const double *bx64, *by64, *bz64;
    // Bounding caps of the column catalog's aligned 64-point groups (stored
    // order): centre x, y, z and an upper bound of the angular radius (3-D:
    // the points' mean and the largest distance from it); null unless
    // pruning is on.
    const double *bcaps;
    unsigned long long *hist;    // kGlobalCopies x nslots, zeroed before
    // jackknife regions: nreg x kGlobalCopies x nslots, zeroed before; the
    // histogram of a unit also goes to its rows' and columns' regions (once
    // when they coincide).  Null without regions.
    unsigned long long *touch;
    const int *cancel;           // host-visible flag (non-zero: skip the rest), or null
    int32_t auto_pairs;          // 1: DD/RR (count j > i only), 0: DR
    int32_t na, nb;              // catalog sizes
    int32_t pad;
};

struct PairArgs {
    const JobDev *jobs;          // device job table, or null: every unit belongs to job0
    JobDev job0;                 // the job of a single-job launch (passed by value)
    const Unit *units;           // device
    int32_t n_units;
    // Work queue: item q is wavefront part q % kWaves of unit q / kWaves;
    // wavefronts take items in order with an atomic add on *queue (zeroed
    // before the launch) until they pass n_units * kWaves.
    unsigned int *queue;

    // Cell table (device, copied into LDS by every block).
    const void *lut;
    int32_t lut_cells;           // c_hi - c_lo + 1
    int32_t lut_entry_bytes;     // 1 or 2
    int32_t lut_shift;           // cell = key >> shift
    int32_t lut_lo, lut_hi;      // clamp range of cells
    int32_t lut_direct;          // 1: wrapped FP32 byte table (lut_cells = 2^lut_wrap_bits;
                                 // cell = (bits(q) >> shift) & (lut_cells - 1), q summed
                                 // from the floor q_floor); the histograms and thresholds
                                 // then start at LDS byte aux_off, inside the table's
                                 // unused part
    int32_t lut_wrap_bits;
    int32_t aux_off;
    float q_floor;
    // Pairs certainly beyond the last edge: FP32 path, bits(q) >= beyond_key
    // (the bits of the last edge's qhi); FP64 path, high word of e = 1 - d
    // above beyond_key as signed integers (e > E_last).
    uint32_t beyond_key;
    // Angular FP32 path: the dot product p = fl32(f_i . f_j) of the FP32
    // copies, p <= p_beyond, proves the rule's d <= D_last (the pair is past
    // the last edge); -inf when no such screen applies (3-D catalogs).
    float p_beyond;
    // Angular FP32 path, dot product first (plut_cells > 0): the cell table of
    // the key q' = fl(2 - 2p) (cell = clamp(bits(q') >> plut_shift, plut_lo,
    // plut_hi), plut_cells entries at byte plut_src of lut, copied to LDS byte
    // plut_lds), and the band in p, nedges (plo, phi) pairs after the chord
    // band in qlo / qhi.  The chord loop hands the steps after a chord step
    // that needed no lookup and whose smallest q was at least q_dot to the
    // dot product.
    int32_t plut_cells;
    int32_t plut_shift, plut_lo, plut_hi;
    int32_t plut_src, plut_lds;
    int32_t stage_lds;           // LDS byte offset of the column staging buffers (kStageBytes)
    float q_dot;

    // Exact tile pruning: 1 = a wavefront bins a whole aligned 64-column
    // block at once when the bounding caps put every pair of the block
    // strictly inside one slot (edges in radians, nedges, in erad).
    int32_t prune;
    const double *erad;

    // 0: angles on the sky (dot products against D_k); 1: 3-D distances
    // (squared distances of Cartesian points, D_k = -S_k, E_k = S_k).
    int32_t metric;
    // 3-D pruning: absolute widening of the distance interval of a block
    // (covers the FP32 copies of the rows, 2^-22 times the largest norm).
    double prune_margin;
    // Angular pruning: bound on | |v|^2 - 1 | of the catalogs' stored
    // vectors (the rule's dot product is |v_i| |v_j| cos(phi), not cos(phi)).
    double prune_delta;

    // Edge thresholds (device).
    const float *qlo, *qhi;      // FP32 chord^2 bands, nedges each
    const double *E;             // fl(1 - D_k), nedges
    const double *D;             // D_k, nedges
    int32_t nedges;              // nbins + 1
    int32_t nslots;              // nbins + 2

    // Per-wave LDS histogram copies (layout [slot][copy]).
    int32_t hist_copies;         // 32, 16, 8 or 4
    int32_t rows_per_lane;       // 2 or 4: a unit spans kWaves * 64 * rows_per_lane rows
    int32_t blocks_per_cu;       // grid = CUs x this (0: the blocks that fit at once)

    unsigned long long *stats;   // kStats words: [two-slot steps, flagged, exact, skipped
                                 //  units, rare-path steps, steps counted beyond the last
                                 //  edge, one-slot steps, pairs binned by pruned blocks,
                                 //  angular FP32 steps that formed the chord]
};

// LDS bytes per edge: D_k, fl(1 - D_k), the edge in radians (pruning), the
// FP32 chord band (qlo_k, qhi_k) and the band in p (plo_k, phi_k).
constexpr int kEdgeLdsBytes = 8 + 8 + 8 + 8 + 8;

// LDS bytes of the histograms (with the discard row) and edge thresholds.
inline int aux_lds_bytes(int nslots, int hist_copies, int nedges) {
    int hist = kWaves * (nslots + 1) * hist_copies * 4;
    int thr = nedges * kEdgeLdsBytes;
    return hist + thr;
}

// LDS bytes used by one block for the given table sizes; aux_off >= 0 places
// the histograms and thresholds at that offset (inside a wrapped table).
inline int lds_bytes(int nslots, int hist_copies, int lut_cells, int lut_entry_bytes, int nedges,
                     int aux_off = -1) {
    int lut = ((lut_cells * lut_entry_bytes) + 15) & ~15;
    int aux = aux_lds_bytes(nslots, hist_copies, nedges);
    if (aux_off >= 0)
        return aux_off + aux > lut ? aux_off + aux : lut;
    return lut + aux;
}

// Margin (radians) of the geometric angle interval of the pruning test:
// covers the FP32 copies of the rows (directions move by <= 1.2e-7 rad) and
// the rounding of the caps' arithmetic (<= ~3e-8 rad, acos near 1 included).
constexpr double kPruneMargin = 1e-6;
// Absolute slack of the pruning test's dot-product interval: the rule's own
// rounding (gamma_3 (1 + delta) < 3.4e-16) and that of the interval
// arithmetic (a few units of 2^-53).
constexpr double kPruneDotSlack = 2e-15;

}  // namespace tpcf

// Size of the fixed per-device work area of tpcf_count_noalloc (histogram
// copies, work-queue counter, output slots, edge and cell tables, and the
// work-unit list).
constexpr size_t kScratchBytes = size_t(16) << 20;

// Launchers implemented in kernels.hip.
extern "C" {
// Look up (once per device, with that device current) the device address of
// the fixed work area; 0 or a hipError_t.
int tpcf_scratch_init(int device);
// The address found by tpcf_scratch_init for this device, or null.
void *tpcf_scratch_ptr(int device);
int tpcf_launch_pairs(const tpcf::PairArgs *args, int precision, void *stream);
int tpcf_launch_zero_u64(unsigned long long *p, int64_t n, void *stream);
// Sum the kGlobalCopies copies of each of njobs histograms (contiguous,
// njobs x kGlobalCopies x nslots) into out (njobs x nslots).
int tpcf_launch_reduce_copies(const unsigned long long *copies, int32_t nslots, int32_t njobs,
                              unsigned long long *out, void *stream);
// FP32 copies of an FP64 SoA catalog, or (given32 non-null) a check that
// given32 holds them; check_out[0] receives the largest | |v|^2 - 1 | (bits
// of a double, +inf for a non-finite value), check_out[1] a non-zero value
// if a given copy differs.  check_out is zeroed by the caller.
int tpcf_launch_to_float(const double *xyz64, int64_t n, float *xyz32, const float *given32,
                         unsigned long long *check_out, void *stream);
// Bounding caps of the aligned 64-point groups of an FP64 SoA catalog
// (see JobDev::bcaps): 4 doubles per group; metric 1 (3-D): bounding balls.
int tpcf_launch_caps64(const double *xyz64, int64_t n, double *caps, int metric, void *stream);
}
