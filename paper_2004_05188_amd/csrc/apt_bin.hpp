// Kernel argument blocks of the binning stage (see apt_bin.hip).
#pragma once
#include "apt_internal.hpp"

namespace apt {

// LSD radix sort of cell ids and target keys: the fewest passes of at most
// kDigitBits each, the key's bits split evenly over them.  A narrower digit
// has fewer values, so each tile's run of one digit is longer and leaves as
// a longer contiguous write (2e9 ions, 29-bit cell ids, tiles of 256 x 11
// keys: passes of 8, 7, 7, 7 bits bin in 124 ms, of 8, 8, 8, 5 bits in 128
// ms; five passes of 6 bits were slower still).
constexpr int kDigitBits = 8;
constexpr int kRadix = 1 << kDigitBits;
static_assert(kRadix <= kBlock, "one thread per digit in the sort's scans");

// Downsweep tiles: 512 threads x 14 keys for large sorts (with 16-byte
// records, 151 KB of LDS: one workgroup per CU), 256 x 8 for small ones,
// whose few tiles per workgroup then still fill two workgroups per CU.  The
// longer a tile, the longer each digit's run in it and the write that
// carries the run (2e9 ions, 28-bit cell ids in four 7-bit passes: binning
// 117 ms with tiles of 256 x 11 keys, 105 ms with 512 x 11, 103 ms with
// 512 x 14; the 7.7e6-ion needle bins 0.85 ms per step with 512 x 14 and
// 0.75 ms with 256 x 8).
constexpr int kDsLargeBlock = 512, kDsLargeItems = 14;
constexpr int kDsSmallBlock = 256, kDsSmallItems = 8;

// bits of max_key (0 for 0)
__host__ __device__ inline uint32_t key_bits(uint64_t max_key) {
    uint32_t b = 0;
    while (b < 64 && (max_key >> b) != 0u) ++b;
    return b;
}

// passes that sort keys in [0, max_key]
__host__ __device__ inline int sort_passes_for(uint64_t max_key) {
    const uint32_t b = key_bits(max_key);
    return b == 0 ? 1 : (int)((b + kDigitBits - 1) / kDigitBits);
}

// the digit of pass `pass` over keys of `bits` bits sorted in `passes`
// passes: (key >> shift) & mask; the lower passes take the odd bits
__host__ __device__ inline void pass_digit(uint32_t bits, uint32_t passes, uint32_t pass, uint32_t* shift,
                                           uint32_t* mask) {
    const uint32_t base = bits / passes, extra = bits % passes;
    *shift = pass * base + (pass < extra ? pass : extra);
    const uint32_t width = base + (pass < extra ? 1u : 0u);
    *mask = (1u << width) - 1u;
}

// What a call zeroes or fills before its work: status word, output
// histograms, target count, counters, squared bin edges (any may be NULL).
struct InitArgs {
    int32_t* status;
    uint64_t* h1;
    int32_t n1;
    uint64_t* h2;
    int32_t n2;
    int64_t* n_targets;
    uint32_t* counter;      // [4]: [0] stragglers, [1..2] occupied cells
    // squared bin edges of the RDF and of the k-th distance histogram, or NULL
    double* e2;
    float e2_rmax;
    int32_t e2_nbins;
    double* ke2;
    float ke2_rmax;
    int32_t ke2_nbins;
    uint32_t* work_q = nullptr;   // [2 kXcd] per-XCD work counters of the pair kernels, or NULL
};

__device__ inline void fill_edges(double* E2, float r_max, int n_bins, int t, int stride);

// Threads t, t + stride, ... of a grid do the work of `a`.
__device__ inline void init_body(const InitArgs& a, int t, int st) {
    if (a.e2) fill_edges(a.e2, a.e2_rmax, a.e2_nbins, t, st);
    if (a.ke2) fill_edges(a.ke2, a.ke2_rmax, a.ke2_nbins, t, st);
    if (t == 0) {
        if (a.status) *a.status = 0;
        if (a.n_targets) *a.n_targets = 0;
        if (a.counter)
            for (int c = 0; c < 4; ++c) a.counter[c] = 0;
        if (a.work_q)
            for (int c = 0; c < 2 * kXcd; ++c) a.work_q[c] = 0;
    }
    if (a.h1)
        for (int b = t; b < a.n1; b += st) a.h1[b] = 0;
    if (a.h2)
        for (int b = t; b < a.n2; b += st) a.h2[b] = 0;
}

struct CountArgs {
    const float* xyz;
    const uint8_t* lab;
    const float* d_bnd;
    int64_t n;
    int64_t chunk;
    int32_t A, B;
    float d_srf;
    const double* zscale;   // NULL: unscaled
    uint32_t* part_cnt;     // [G][2] targets, neighbours
    float* part_bbox;       // [G][6]
    int32_t* part_nf;       // [G]
    int32_t sel_union;      // 1: targets and neighbours are both (eligible A) or B
    // the call's initial zeroing, done by the same launch (do_init = 1)
    InitArgs init;
    int32_t do_init;
};

struct PlanArgs {
    int32_t G;              // number of count blocks (<= 4096)
    const uint32_t* part_cnt;
    const float* part_bbox;
    const int32_t* part_nf;
    uint32_t* part_off;     // [G][2] exclusive offsets (out)
    PlanParams pp;
    const double* zscale;
    GridPlan* plan;
    int32_t* status;
};

struct CompactArgs {
    const uint8_t* lab;
    const float* d_bnd;
    int64_t n;
    int64_t chunk;
    int32_t A, B;
    float d_srf;
    const uint32_t* part_off;
    uint32_t* tid;          // [nT]
    uint32_t* bsel;         // [nB] or NULL (neighbours = all ions)
    int32_t sel_union;      // as CountArgs::sel_union
    // sort keys written with the lists (plan from k_plan; NULL keys: none):
    // targets (block-raster key, list position), neighbours (cell id and
    // their 16-byte record (x, y, z, ion index) into the record buffer that
    // the sort's passes start from, see SortArgs::rec)
    const GridPlan* plan;
    const float* xyz;
    const double* zscale;   // NULL: unscaled
    uint32_t* tkeys;
    uint32_t* tvals;
    uint32_t* bkeys;
    float4* brec[2];
};

struct KeyArgs {
    const GridPlan* plan;
    const float* xyz;
    const uint32_t* src;    // index list or NULL (identity)
    const double* zscale;
    int32_t count_is_T;     // count = plan->nT (else plan->nB)
    int32_t val_is_index;   // value = list position (else the ion index)
    uint32_t* keys;
    uint32_t* vals;
};

struct SortArgs {
    const GridPlan* plan;
    int32_t count_is_T;
    int32_t pass;
    int32_t G;
    uint32_t* keys[2];
    uint32_t* vals[2];
    uint32_t* counts;       // [256][G]
    uint32_t* totals;       // [256]
    // records instead of values (rec[0] non-NULL): the 16-byte neighbour
    // records travel with their keys; the buffers alternate so that the
    // last active pass writes rec[0] (rec_after)
    float4* rec[2] = {nullptr, nullptr};
};

// the record buffer that holds the data after pass p of `passes` (p = -1:
// what the passes start from), so that the last pass ends in rec0
__host__ __device__ inline float4* rec_after(float4* rec0, float4* rec1, int passes, int p) {
    return ((passes - 1 - p) & 1) ? rec1 : rec0;
}

// One radix pass of up to two independent sorts in the same launches: sort
// 0 takes the first s[0].G workgroups, sort 1 the next s[1].G (the scan: 256
// each).
struct SortSet {
    SortArgs s[2];
    int32_t n;
    int32_t tile;   // keys per downsweep tile (the passes' chunks are whole tiles)
};

struct OrderArgs {
    const GridPlan* plan;
    const float* xyz;
    const uint32_t* tid;    // [nT] eligible targets, ascending
    uint32_t* vals[2];      // sorted ranks
    uint32_t* t_rank;       // [nT] outputs, cell order
    uint32_t* t_id;
    float* tx;
    float* ty;
    float* tz;
    const uint32_t* keys[2];   // sorted target keys
    uint32_t* distinct;     // may be NULL: += number of distinct target cells
    // [n_cells + 1] start of each cell's targets (targets in plain cell
    // order), written when the plan chose mode 3; may be NULL
    uint32_t* t_cell_start;
};

// (xyz NULL: the records are already in bpos, sorted with their keys; only
// the cell offsets and the occupied-cell count are written)
struct GatherArgs {
    const GridPlan* plan;
    const float* xyz;
    const double* zscale;
    uint32_t* keys[2];
    uint32_t* vals[2];
    float4* bpos;           // [nB] (x, y, z, ion index as bits) in cell order
    uint32_t* cell_start;   // [n_cells + 1]
    uint32_t* distinct;     // may be NULL: += number of non-empty neighbour cells
};

// Target / neighbour membership of ion i.  In union mode both are the ions
// that are an eligible target or a neighbour (the adjoint of the smoothed
// RDF visits every ion that takes part in a pair, in either role).
__device__ __forceinline__ void select_ion(uint8_t l, const float* d_bnd, int64_t i, int A, int B, float d_srf,
                                           int sel_union, bool* isT, bool* isB) {
    const bool t = (A == APT_ANY || l == A) && (d_bnd == nullptr || d_bnd[i] >= d_srf);
    const bool b = (B == APT_ANY || l == B);
    if (sel_union) {
        *isT = *isB = t || b;
    } else {
        *isT = t;
        *isB = b;
    }
}

// The kNN radii from the volume the ions occupy.  The plan's first guesses
// use the bounding box, which a needle fills less than half; once the cells
// are known, the occupied cells of the denser set (occ[0]: distinct target
// cells, counted while the targets are put in cell order; occ[1]: non-empty
// neighbour cells, counted by the gather; both zero before k_order_gather
// runs) measure the specimen's volume.  The kernels that search apply this
// to their own copy of the plan.
__device__ inline void refine_radii(GridPlan& P, const uint32_t* occ, int32_t k) {
    if (!occ || k <= 0) return;
    double box = 1.0;
    for (int ax = 0; ax < 3; ++ax) box *= fmax((double)P.hi[ax] - (double)P.lo[ax], 1e-3);
    const double h = (double)P.h;
    double vol = (double)max(occ[0], occ[1]) * h * h * h;
    if (!(vol > 0.0) || vol > box) vol = box;
    const double rho = (double)(P.nB > 0 ? P.nB : 1) / vol;
    const double r = 1.15 * cbrt(3.0 * ((double)k + 0.5) / (4.0 * M_PI * rho));
    P.rk0 = (float)fmin(r, (double)P.r_all);
    // tiles: certified within 1.6x the Poisson mean k-th distance (species
    // that cluster leave the matrix poorer than the mean: a tighter radius
    // sends too many targets to the one-by-one search); mode 3 (dense
    // neighbours, nearly uniform): 1.3x, which leaves a few per mille
    P.rk_tile = (float)fmin((P.tile_mode == 3 ? 1.3 : 1.6) / 1.15 * (double)P.rk0, (double)P.r_all);
}

// Squared bin edges e_b^2, e_b = b * r_max / n_bins in FP64, b = 0..n_bins,
// written by the threads [t, n_bins] in steps of `stride`.
__device__ inline void fill_edges(double* E2, float r_max, int n_bins, int t, int stride) {
#pragma clang fp contract(off)
    for (int b = t; b <= n_bins; b += stride) {
        const double e = ((double)b * (double)r_max) / (double)n_bins;
        E2[b] = e * e;
    }
}

__global__ void k_count(CountArgs a);
__global__ void k_plan(PlanArgs a);
__global__ void k_compact(CompactArgs a);
__global__ void k_keys(KeyArgs a);
__global__ void k_rs_upsweep(SortSet a);
__global__ void k_rs_scan(SortSet a);
__global__ void k_rs_downsweep_large(SortSet a);   // kDsLargeBlock threads
__global__ void k_rs_downsweep_small(SortSet a);   // kDsSmallBlock threads
__global__ void k_gather(GatherArgs a);
// the target order (first g_order workgroups) and the neighbour gather (the
// rest) in one launch: they read and write disjoint arrays
__global__ void k_order_gather(OrderArgs oa, GatherArgs ga, int32_t g_order);

}  // namespace apt
