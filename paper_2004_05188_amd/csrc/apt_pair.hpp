// Kernel argument block of the target-neighbour pair kernel (apt_pair.hip).
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr int kKnnCap = 512;   // per-wavefront kNN candidate buffer (u64 keys)

struct PairArgs {
    const GridPlan* plan;
    const float* xyz;            // original positions [n][3]
    const uint32_t* t_rank;      // [nT] targets in cell order: rank in ascending ion index
    const uint32_t* t_id;        // [nT] ... ion index
    const float* tx;             // [nT] ... position
    const float* ty;
    const float* tz;
    const float4* bpos;          // [nB] neighbours in cell order: x, y, z, ion index (bits)
    const uint32_t* cell_start;  // [n_cells + 1]
    int32_t self_possible;       // a target may also be a neighbour
    const uint8_t* lab;          // [n] species labels
    int32_t nbr_species;         // species of the neighbours (or APT_ANY)
    // RDF
    int32_t n_bins;
    float r_enum;                // enumeration radius covering every counted pair
    float thr2;                  // FP32 squared-distance cut of the fast path
    float inv_w;                 // n_bins / r_max (FP32)
    float delta_b;               // near-edge band, in bins
    double inv_w64;
    const double* E2;            // [n_bins + 1]
    uint64_t* hist;              // [n_bins]
    int32_t hist_in_lds;
    // kNN
    int32_t k;
    float rknn;                  // r_knn_max (may be +inf)
    float rknn2;                 // rknn * rknn in FP32
    int64_t capacity;
    int64_t* target_id;
    float* dist;
    int64_t* nbr_id;
    int32_t kb_nbins;
    double kb_inv_w64;
    const double* KE2;           // [kb_nbins + 1] or NULL
    uint64_t* knn_hist;          // [kb_nbins + 1] or NULL
    // tile mode: targets left for the one-per-wavefront pass
    uint32_t* strag;             // [nT] target slots (cell order)
    uint32_t* strag_count;       // [1], zeroed before the tile pass
    const uint32_t* occ;         // [2] occupied-cell counts for refine_radii, or NULL
    const uint32_t* t_cell_start;  // [n_cells + 1] targets per cell (mode 3: plain cell order)
    uint32_t* work_q;            // [2 kXcd] per-XCD counters: chunks of k_rdf_nbr, then tiles of
                                 // k_pair_tile; zeroed by the call's init
    // written once per call by k_pair (workgroup 0): the eligible target
    // count, and APT_STATUS_CAPACITY when k > 0 and it exceeds capacity
    int64_t* n_targets;
    int32_t* status;
};

// grid: multiple of 8 workgroups of kBlock threads; dynamic LDS per block:
// (hist_in_lds ? 4 * n_bins * 4 : 0) + (knn ? 4 * kKnnCap * 8 : 0) bytes
// Variant flags of k_pair: RDF into per-wavefront LDS histograms or straight
// into the global histogram (many bins); targets may be neighbours themselves.
constexpr int kRdfLds = 1, kRdfGlobal = 2, kSelf = 4;
// k_rdf_nbr only: count the pair evaluations into hist[0] instead of the RDF
constexpr int kCountEvals = 8;
template <int FLAGS, bool KNN>
__global__ void k_pair(PairArgs a);

size_t pair_lds_bytes(bool rdf, bool knn, int n_bins, bool hist_in_lds);

// 64 targets per wavefront (apt_pair.hip); KMAX >= k kNN keys per lane, 0 for
// RDF only.  Exits at once unless the plan chose tile mode.
template <int FLAGS, int KMAX>
__global__ void k_pair_tile(PairArgs a);
size_t tile_lds_bytes(bool rdf, int n_bins);

// Neighbour-major RDF (mode 3, dense neighbours): each wavefront takes 64
// consecutive neighbour records and evaluates every target within reach of
// their bounding box against all of them.  Exits at once unless the plan
// chose mode 3.
template <int FLAGS>
__global__ void k_rdf_nbr(PairArgs a);
// With targets that may be neighbours the neighbour-major kernel also counts
// each such target against its own record (distance 0, bin 0) instead of
// testing identities per pair: this kernel takes those counts off bin 0
// (every target with a finite position whose species is a neighbour's).
// Exits unless the plan chose mode 3 with the neighbour-major RDF.
__global__ void k_nbr_self(PairArgs a);
// Mode 3 with the RDF one target per wavefront (tuning rdf_kernel 2): RDF
// of every target, eight wavefronts per SIMD; exits otherwise.
template <int FLAGS>
__global__ void k_rdf_tgt(PairArgs a);
size_t nbr_lds_bytes(int n_bins, bool hist_in_lds);
__global__ void k_count_candidates(const GridPlan* plan, const uint32_t* occ, const uint32_t* cell_start,
                                   const float* tx, const float* ty, const float* tz, float r_enum, int32_t k,
                                   unsigned long long* out);

}  // namespace apt
