// Internal declarations of the GPU library: the device-side plan of the
// uniform cell grid, wavefront helpers and the exact FP64 bin decision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apt_stat.h"

namespace apt {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // 4 wavefronts per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcd = 8;                      // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Device-resident description of the cell grid of one call, written by
// k_plan and read by every later kernel (launch grids do not depend on it).
struct GridPlan {
    float lo[3];        // bounding box of the finite positions of the targets and neighbours
    float hi[3];
    float h;            // cell edge (nm)
    float inv_h;
    int32_t dim[3];     // cells per axis
    uint32_t n_cells;
    uint32_t nT;        // eligible targets
    uint32_t nB;        // neighbour ions
    uint32_t passes;    // active radix passes over the cell ids (neighbours)
    uint32_t passes_T;  // active radix passes over the target keys
    uint32_t bits;      // bits of the largest cell id (the radix digits split them)
    uint32_t bits_T;    // bits of the largest target key
    int32_t tblock;     // targets are ordered by blocks of tblock^3 cells (8), or by cell (1)
    int32_t nbx, nby;   // blocks per axis (x, y)
    float eps;          // culling margin covering FP32 cell-assignment error (nm)
    float r_all;        // a radius that reaches every cell from any point of the box
    float rk0;          // first kNN search radius
    float zscale;       // z scale applied to positions (1 for the plain path)
    int32_t nonfinite;
    int32_t tile_mode;  // 0: one target per wavefront; 64 targets per wavefront: 1 sharing staged
                        // candidates (dense targets), 2 one target per lane (sparse neighbours);
                        // 3: kNN one target per lane, RDF one target per wavefront (dense
                        // neighbours, kNN radius well below r_max)
    float rk_tile;      // kNN radius certified by the tile pass
    int32_t rdf_nbr;    // mode 3: the RDF runs neighbour-major (k_rdf_nbr), else one target per wavefront
};

// Host-chosen parameters of the plan.
struct PlanParams {
    float h_min;        // smallest cell edge
    float occ;          // aimed-for neighbours per cell
    int32_t k;          // kNN order (0: no kNN)
    uint32_t cell_cap;  // largest number of cells the workspace holds
    int32_t tile_policy;  // 0: automatic, 1: one target per wavefront, 2: 64 targets per wavefront
                          // sharing staged candidates, 3: one target per lane, 4: kNN per lane and
                          // RDF per wavefront
    float r_enum;       // RDF enumeration radius (0: no RDF)
    float tile_occ;     // aimed-for neighbours per cell with 64 targets per wavefront (<= 0: occ)
    // > 0: one target per wavefront also tries the edge h_min * h_shrink and
    // keeps it when the cell ids need no more bytes (no extra radix pass)
    float h_shrink = 0.0f;
    // mode 3's RDF kernel: 0 automatic (neighbour-major), 1 neighbour-major,
    // 2 one target per wavefront
    int32_t rdf_kernel = 0;
};

// ---------------------------------------------------------------- waves --
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <class T>
__device__ __forceinline__ T readlane(T v, int lane) {
    static_assert(sizeof(T) == 4, "32-bit readlane");
    int r = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane);
    return __builtin_bit_cast(T, r);
}

// Inclusive prefix sum over the wavefront with DPP moves (no LDS): shifts
// by 1, 2, 4 and 8 lanes within each row of 16 (lanes shifted in from
// outside the row add 0), then the last lane of rows 0 and 2 added to rows 1
// and 3 (row_bcast:15) and the last lane of row 1 to rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15, rows 1 and 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31, rows 2 and 3
    return (uint32_t)x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Counters of one wavefront's LDS RDF histogram.
__host__ __device__ constexpr int hist_stride(int n_bins) { return n_bins; }

// ------------------------------------------------------------- cells --
__device__ __forceinline__ int cell_axis(const GridPlan& P, int a, float x) {
    float f = (x - P.lo[a]) * P.inv_h;
    if (!(f >= 0.0f)) return 0;                       // also catches NaN
    if (f >= (float)(P.dim[a] - 1)) return P.dim[a] - 1;
    return (int)f;
}

__device__ __forceinline__ uint32_t cell_id(const GridPlan& P, float x, float y, float z) {
    return ((uint32_t)cell_axis(P, 2, z) * (uint32_t)P.dim[1] + (uint32_t)cell_axis(P, 1, y)) *
               (uint32_t)P.dim[0] + (uint32_t)cell_axis(P, 0, x);
}

// Sort key of a target: its cell in block-raster order (blocks of 8^3 cells
// in raster order, cells in raster order inside a block), so that any run
// of consecutive targets is a compact region of space; plain cell order
// when the plan chose tblock = 1.
__device__ __forceinline__ uint32_t target_key(const GridPlan& P, float x, float y, float z) {
    const uint32_t cx = (uint32_t)cell_axis(P, 0, x), cy = (uint32_t)cell_axis(P, 1, y),
                   cz = (uint32_t)cell_axis(P, 2, z);
    if (P.tblock == 1) return (cz * (uint32_t)P.dim[1] + cy) * (uint32_t)P.dim[0] + cx;
    const uint32_t blk = ((cz >> 3) * (uint32_t)P.nby + (cy >> 3)) * (uint32_t)P.nbx + (cx >> 3);
    return (blk << 9) | ((cz & 7u) << 6) | ((cy & 7u) << 3) | (cx & 7u);
}

// ------------------------------------------------------- exact binning --
// FP64 squared distance of two stored FP32 positions, evaluated exactly as
// ((dx*dx + dy*dy) + dz*dz) with every operation rounded on its own.  HIP's
// __dmul_rn / __dadd_rn are inline functions whose operations may still be
// fused after inlining, so plain operators are used under a no-contraction
// pragma instead.
__device__ __forceinline__ double exact_D2(float xi, float yi, float zi, float xj, float yj, float zj) {
#pragma clang fp contract(off)
    const double dx = (double)xj - (double)xi;
    const double dy = (double)yj - (double)yi;
    const double dz = (double)zj - (double)zi;
    return (dx * dx + dy * dy) + dz * dz;
}

// Largest b with E2[b] <= D2, or n_bins when D2 >= E2[n_bins].
__device__ __forceinline__ int exact_bin(double D2, const double* __restrict__ E2, int n_bins,
                                         double inv_w) {
    if (!(D2 < E2[n_bins])) return n_bins;
    int b = (int)(sqrt(D2) * inv_w);
    if (b < 0) b = 0;
    if (b > n_bins - 1) b = n_bins - 1;
    while (b > 0 && D2 < E2[b]) --b;
    while (b < n_bins - 1 && D2 >= E2[b + 1]) ++b;
    return b;
}

// ------------------------------------------------------ workspace plan --
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Carve {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += align256(count * sizeof(T));
        return p;
    }
};

}  // namespace apt
