// Ion-to-edge distancing (apt_edge.hip): the distance of every ion to the
// closest point of a triangle hull, exact up to a probe distance.
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr uint32_t kTriCells = 1u << 22;     // cells of the triangle grid at most
constexpr int kTriScanTile = 4096;           // cells per block of the offset scan
constexpr uint32_t kTriScanBlocks = kTriCells / kTriScanTile;

// The triangle grid, planned on the device from the ions' bounding box and
// the triangles' sizes.
struct TriPlan {
    uint32_t rmax_bits;          // largest triangle radius (FP32 bits; radii are >= 0)
    uint32_t n_valid;            // triangles with finite vertices
    double r_sum;                // sum of their radii
    float lo[3];
    float h, inv_h;
    int32_t dim[3];
    uint32_t n_cells;
    float r_max;                 // largest radius
    float slack;                 // bound on FP32 rounding of cells and centroids (nm)
    double prb2;                 // d_prb^2 in FP64 (+inf: no probe limit)
};

struct EdgeArgs {
    const GridPlan* plan;        // the ions' grid (records in cell order)
    const float4* bpos;
    TriPlan* tp;
    const float* tri;            // [n_tri][9] FP32 vertices, as given
    uint32_t n_tri;
    float d_prb;
    float4* tc;                  // [n_tri] centroid and radius (radius < 0: left out)
    uint32_t* tcell;             // [n_tri] triangle grid cell of the centroid
    uint32_t* tcnt;              // [kTriCells] triangles per cell
    uint32_t* tstart;            // [kTriCells + 1] first triangle of each cell
    uint32_t* tblk;              // [kTriScanBlocks] cells' sums per scan block
    uint32_t* torder;            // [n_tri] triangle index, cell order
    float4* tsorted;             // [n_tri] centroid and radius, cell order
    float* d_out;                // [n]
    int64_t n;
    int32_t* status;
};

__global__ void k_edge_zero(EdgeArgs a);
__global__ void k_edge_prep(EdgeArgs a);
__global__ void k_edge_plan(EdgeArgs a);
__global__ void k_edge_clear(EdgeArgs a);
__global__ void k_edge_count(EdgeArgs a);
__global__ void k_edge_scan_blocks(EdgeArgs a);
__global__ void k_edge_scan_add(EdgeArgs a);
__global__ void k_edge_fill(EdgeArgs a);
__global__ void k_edge_dist(EdgeArgs a);

}  // namespace apt
