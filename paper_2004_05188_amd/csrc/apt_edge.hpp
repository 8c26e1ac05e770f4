// Ion-to-edge distancing (apt_edge.hip): the distance of every ion to the
// closest point of a triangle hull, exact up to a probe distance.
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr uint32_t kTriCells = 1u << 22;     // cells of the triangle grid at most
constexpr int kTriScanTile = 4096;           // cells per block of the offset scan
constexpr uint32_t kTriScanBlocks = kTriCells / kTriScanTile;

constexpr int kPieceSizes = 17;              // piece radii tried: h/2 * 2^j (j < 16), and the largest radius

// The triangle grid, planned on the device from the ions' bounding box and
// the triangles' sizes.  Every triangle is covered by pieces, the m x m
// sub-triangles of a barycentric subdivision, registered by the centroid of
// each piece with its radius; a piece stands for its whole triangle.
struct TriPlan {
    uint32_t rmax_bits;          // largest triangle radius (FP32 bits; radii are >= 0)
    uint32_t n_valid;            // triangles with finite vertices
    double r_sum;                // sum of their radii
    unsigned long long pieces_at[kPieceSizes];   // pieces for each candidate piece radius
    uint32_t piece_ctr;          // pieces written so far
    uint32_t piece_rmax_bits;    // largest piece radius
    uint32_t n_pieces;
    uint32_t piece_cap;          // pieces the workspace holds
    float rho;                   // piece radius aimed at (a triangle gets ceil(r / rho)^2 pieces)
    float lo[3];
    float h, inv_h;
    int32_t dim[3];
    uint32_t n_cells;
    float r_max;                 // largest triangle radius
    float slack;                 // bound on FP32 rounding of cells, centroids and pieces (nm)
    double prb2;                 // d_prb^2 in FP64 (+inf: no probe limit)
};

struct EdgeArgs {
    const GridPlan* plan;        // the ions' grid (records in cell order)
    const float4* bpos;
    TriPlan* tp;
    const float* tri;            // [n_tri][9] FP32 vertices, as given
    uint32_t n_tri;
    float d_prb;
    uint32_t piece_cap;          // pieces the workspace holds
    float4* tc;                  // [n_tri] centroid and radius (radius < 0: left out)
    float4* pc;                  // [piece_cap] piece centroid and radius
    uint32_t* ptri;              // [piece_cap] the piece's triangle
    uint32_t* pcell;             // [piece_cap] triangle grid cell of the piece
    uint32_t* tcnt;              // [kTriCells] pieces per cell
    uint32_t* tstart;            // [kTriCells + 1] first piece of each cell
    uint32_t* tblk;              // [kTriScanBlocks] cells' sums per scan block
    uint32_t* torder;            // [piece_cap] triangle of each piece, cell order
    float4* tsorted;             // [piece_cap] piece centroid and radius, cell order
    float* d_out;                // [n]
    int64_t n;
    int32_t* status;
};

__global__ void k_edge_zero(EdgeArgs a);
__global__ void k_edge_prep(EdgeArgs a);
__global__ void k_edge_plan(EdgeArgs a);
__global__ void k_edge_measure(EdgeArgs a);
__global__ void k_edge_plan_pieces(EdgeArgs a);
__global__ void k_edge_pieces(EdgeArgs a);
__global__ void k_edge_clear(EdgeArgs a);
__global__ void k_edge_count(EdgeArgs a);
__global__ void k_edge_scan_blocks(EdgeArgs a);
__global__ void k_edge_scan_add(EdgeArgs a);
__global__ void k_edge_fill(EdgeArgs a);
__global__ void k_edge_dist(EdgeArgs a);

}  // namespace apt
