// Maximum-separation clustering (apt_cluster.hip): the ions of one species,
// linked when at most d_max apart, grouped into connected components by a
// lock-free union-find over ion indices.
#pragma once
#include "apt_internal.hpp"

namespace apt {

struct ClusterLinkArgs {
    const GridPlan* plan;
    const uint32_t* t_id;        // [nT] the species' ions in cell order: ion index
    const float* tx;             // ... position
    const float* ty;
    const float* tz;
    const float4* bpos;          // the same ions as records in cell order: x, y, z, index (bits)
    const uint32_t* cell_start;
    float r_enum;                // enumeration radius (d_max with a margin)
    float in2;                   // FP32 squared distances at most this: certainly linked
    float out2;                  // ... above this: certainly not
    double lim2;                 // d_max^2 in FP64: the exact rule D2 <= lim2
    uint32_t* parent;            // [n] forest over ion indices, parent[v] <= v
};

struct ClusterOutArgs {
    const uint8_t* lab;
    const float* d_bnd;          // may be NULL: no cluster is truncated
    float d_srf;                 // an ion with !(d_bnd >= d_srf) lies at the edge
    int32_t A;                   // species, or APT_ANY
    uint32_t n;
    int32_t n_min;
    uint32_t* parent;
    uint32_t* size;              // [n] component size at its root; bit 31: truncated
    int64_t* label;              // [n] output
    unsigned long long* counts;  // [3] output: kept, kept and truncated, ions in kept
    uint64_t* size_hist;         // [n_size_bins] output, or NULL
    int32_t n_size_bins;
};

__global__ void k_ms_init(uint32_t* parent, uint32_t* size, uint32_t n);
__global__ void k_ms_link(ClusterLinkArgs a);
__global__ void k_ms_roots(ClusterOutArgs a);
__global__ void k_ms_final(ClusterOutArgs a);

}  // namespace apt
