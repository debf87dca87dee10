// Host-side compilation of angular bin edges into the thresholds and cell
// tables the pair kernels use.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace tpcf {

// Angular edges: a pair lies at or past edge k when its dot product d
// satisfies d <= D_k.  3-D edges (compile_edges_3d): the same form with
// d = -r^2 and D_k = -S_k, S_k the smallest double whose square root reaches
// e_k, and E_k = S_k (the FP64 path keys on r^2 itself).
struct EdgeTables {
    int nbins = 0;
    int metric = 0;                 // 0: angles on the sky, 1: 3-D distances
    std::vector<double> edge_rad;   // e_k = edge_deg[k] * (pi / 180); 3-D: e_k itself
    std::vector<double> D;          // largest d with acos(d) >= e_k (+-inf at the ends); 3-D: -S_k
    std::vector<double> E;          // fl(1 - D_k); -inf where D_k = +inf, +inf where D_k = -inf; 3-D: S_k
};

struct Band32 {
    double delta = 0;               // bound on | |v|^2 - 1 | used for the band
    float q0 = 0;                   // floor added to q by the kernel (0: none)
    std::vector<float> qlo, qhi;
};

struct CellTable {
    int shift = 0;                  // cell = key >> shift
    int32_t lo = 0, hi = 0;         // clamp range of cells (inclusive)
    bool direct = false;            // wrapped layout: no clamp, cell c at c mod 2^wrap_bits
    int wrap_bits = 0;              // wrapped layout: log2 of the table's entry count
    int32_t aux_off = 0;            // wrapped layout: 16-aligned byte offset of the free piece
                                    // that holds the histograms and thresholds
    float q0 = 0;                   // wrapped layout: the floor of q (every key >= bits(q0) >> shift)
    std::vector<uint16_t> cells;    // hi - lo + 1 entries
    std::vector<uint16_t> image;    // wrapped layout: 2^wrap_bits entries, cells in place, rest 0
    int n_certain = 0, n_medium = 0, n_multi = 0;
};

// Validate edges (finite, strictly increasing, within [0, 180], 1 <= nbins <=
// 256) and compile them.  Returns false with a message on invalid input or
// if acos fails the local monotonicity check around a threshold.
bool compile_edges(const double *edges_deg, int nbins, EdgeTables *out, std::string *err);

// FP32 squared-chord band of every edge for catalogs whose squared norms
// deviate from 1 by at most delta.  With q0 > 0 the band is for
// q = fl(dz^2 + fl(dy^2 + fl(dx^2 + q0))), the kernel's sum started at the
// floor q0 instead of 0.
Band32 make_band32(const EdgeTables &t, double delta, float q0 = 0.0f);
// Bound on |p - d| for p = fl32(f_i . f_j), the dot product of the FP32 copies
// (one multiply and two FMAs, or separate multiplies and adds), and d the
// counting rule's FP64 dot product of the vectors, whose squared norms lie
// within 1 +- delta.
double dot_error32(double delta);
// Band of the dot-product key.  The kernel forms q' = max(fl(2 - 2p), +0)
// (one FMA; as a bit pattern, negative results go to 0) for the largest and
// smallest p of a lane; q' >= qhi_k proves d <= D_k and q' < qlo_k proves
// d > D_k.  Cell tables of this band (make_cells32_top with dot_top_key) give
// the slot range of a lane's pairs from their extreme p.
Band32 make_band_dot32(const EdgeTables &t, double delta);
// Upper bound of every q' the kernel forms (keys above go to the top cell).
uint32_t dot_top_key(double delta);
// The band in p itself, for per-pair decisions: p <= plo_k proves d <= D_k
// and p >= phi_k proves d > D_k (+inf for an edge at 0, -inf for an edge no
// pair reaches).
void make_pband32(const EdgeTables &t, double delta, std::vector<float> *plo, std::vector<float> *phi);
// Floor for the wrapped layout: a power of two at most a quarter of the
// smallest positive threshold of a band built without a floor (and at least
// 2^-100, so no partial sum is subnormal).
float floor_for(const Band32 &b);

// 3-D edges: finite, strictly increasing, within [0, 1e150] (same length
// unit as the coordinates), 1 <= nbins <= 256.  False with a message on
// invalid input.
bool compile_edges_3d(const double *edges, int nbins, EdgeTables *out, std::string *err);

// FP32 band of every 3-D edge for squared distances q of FP32 copies of
// points whose FP64 norms are at most rmax.
Band32 make_band32_3d(const EdgeTables &t, double rmax);

// Bit pattern of an upper bound of every q the FP32 kernel computes for
// points of norm at most rmax (3-D).
uint32_t qtop_key_3d(double rmax);

// Cell tables.  FP32: key = bits of q (q >= 0).  FP64: key = high 32 bits of
// e = fl(1 - d) read as a signed integer.
CellTable make_cells32(const EdgeTables &t, const Band32 &b, double delta, int max_cells);
// The same with the top key given (every q above it goes to the top cell).
CellTable make_cells32_top(const EdgeTables &t, const Band32 &b, uint32_t ktop, int max_cells);
// Wrapped FP32 byte table for a band with a floor (b.q0 > 0): the kernel's
// q lies in [q0, qtop] (qtop bounds the largest chord for norms within
// delta), so its cells bits(q0) >> shift .. bits(qtop) >> shift are all the
// keys there are; cell c is stored at c mod 2^w and read with one bitfield
// extract, (bits >> shift) & (2^w - 1), no clamp and no offset.  The table
// takes the smallest shift, then the smallest w, for which the unused part
// of the table holds aux_bytes (the histograms and thresholds) in one
// 16-aligned piece, or for which they fit after the table, whichever takes
// fewer bytes in all, within max_bytes.  Returns a table with no cells if
// delta is above 2^-10, the band has no floor, or nothing fits.
CellTable make_cells32_wrap(const EdgeTables &t, const Band32 &b, double delta, int max_bytes, int aux_bytes);
// etop bounds the keyed value from above (cells above it are not built; a
// larger value falls into the top cell): 2 for e = 1 - d, the largest
// squared distance for 3-D.
CellTable make_cells64(const EdgeTables &t, int max_cells, double etop = 2.0 + 1.0 / 262144.0);

}  // namespace tpcf
