// Batched null-model replicates (apt_batched.hip): all positions are binned
// once; each replicate's permuted labels split the binned ions into species
// segments (stable, so every segment stays in cell order) with their own
// cell offsets; one pair launch then covers every (replicate, pair, target).
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr int kMaxClasses = 8;     // species taking part in the pairs, plus "other"
constexpr int kMaxPairs = 16;
constexpr int kPartItems = 16;
constexpr int kPartTile = kBlock * kPartItems;

struct PartArgs {
    const GridPlan* plan;
    const float4* S;          // [n] all ions in cell order: x, y, z, index (bits)
    uint32_t* keys[2];        // sort buffers; keys[passes & 1] = cell id of S[p]
    uint32_t* vals[2];        // vals[passes & 1] = ion index of S[p]
    const uint8_t* LR;        // LR + r * n: labels of replicate r (ion order)
    int64_t n;
    int64_t chunk;            // binned positions per block, multiple of kPartTile
    int32_t G;                // blocks per replicate
    int32_t C;                // classes; class C - 1 collects the other species
    uint8_t slot[256];        // species -> class
    uint32_t* cnt;            // [R][C][G]: counts, then (scanned) global positions
    float4* Pp;               // [R * n] records split by class, cell order within a class
    uint32_t* Pcell;          // [R * n] their cell ids
    uint32_t* CS;             // [R][C - 1][n_cells + 1]: start of each cell in a class segment
    int64_t cs_stride;        // n_cells capacity + 1
};

struct BatchPair {
    int32_t a, b;             // classes of target and neighbour species
    float d_srf;
    int32_t pad;
};

struct BatchPairArgs {
    const GridPlan* plan;
    const float* xyz;
    const float* d_bnd;       // may be NULL
    const float4* Pp;
    const uint32_t* CS;
    int64_t cs_stride;
    const uint32_t* cnt;      // scanned class offsets [R][C][G]
    int32_t G, C, R, n_pairs;
    int64_t n;
    int32_t rep0;             // replicate index of the first replicate of this launch
    BatchPair pairs[kMaxPairs];
    uint64_t* items;          // [R * n_pairs + 1] prefix of target counts (one-per-wavefront pairs)
    uint64_t* titems;         // [R * n_pairs + 1] prefix of 64-target tiles (tiled pairs)
    uint64_t* work;           // [2] work counters: targets, tiles (zeroed by k_batch_items)
    const uint32_t* occ;      // [1] cells holding at least one ion (the specimen's volume in cells)
    int32_t tile_ok;          // tiles allowed (k <= 16, LDS fits, tuning)
    float tile_reach;         // certified kNN reach of a tile, times the Poisson mean k-th distance
    // RDF
    int32_t n_bins;
    float r_enum, thr2, inv_w, delta_b;
    double inv_w64;
    const double* E2;
    uint64_t* rdf_hist;       // [n_rep][n_pairs][n_bins]
    // kNN
    int32_t k;
    int32_t kb_nbins;
    double kb_inv_w64;
    const double* KE2;
    uint64_t* knn_hist;       // [n_rep][n_pairs][kb_nbins + 1] or NULL
};

__global__ void k_bpart_count(PartArgs a);
__global__ void k_bpart_scatter(PartArgs a);
__global__ void k_bpart_cells(PartArgs a);
__global__ void k_bpart_empty(PartArgs a);
__global__ void k_batch_items(BatchPairArgs a);
__global__ void k_occupied(const GridPlan* plan, const uint32_t* cell_start, uint32_t* occ);
__global__ void k_pair_batched(BatchPairArgs a);
template <int KMAX>
__global__ void k_pair_batched_tile(BatchPairArgs a);
size_t batched_lds_bytes(int n_bins);
size_t batched_tile_lds_bytes(int n_bins);

}  // namespace apt
