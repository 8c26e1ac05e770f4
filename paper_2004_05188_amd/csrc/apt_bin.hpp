// Kernel argument blocks of the binning stage (see apt_bin.hip).
#pragma once
#include "apt_internal.hpp"

namespace apt {

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
};

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

__global__ void k_count(CountArgs a);
__global__ void k_plan(PlanArgs a);
__global__ void k_compact(CompactArgs a);
__global__ void k_keys(KeyArgs a);
__global__ void k_rs_upsweep(SortArgs a);
__global__ void k_rs_scan(SortArgs a);
__global__ void k_rs_downsweep(SortArgs a);
__global__ void k_take_order(OrderArgs a);
__global__ void k_gather(GatherArgs a);
__global__ void k_edges(double* E2, float r_max, int n_bins);
__global__ void k_refine_radii(GridPlan* plan, const uint32_t* occ, int32_t k);

}  // namespace apt
