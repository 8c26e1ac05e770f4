// Gaussian-smoothed RDF and its adjoint (apt_smooth.hip).  Every pair adds
// to each bin the mass of a Gaussian of standard deviation sigma centred on
// the pair distance that falls inside the bin; bins farther than 6 sigma
// from the distance, and pairs at or beyond r_max + 6 sigma, take no part.
// Positions are (x, y, s z) for a device-side z scale s; all arithmetic
// after the FP32 culling test is FP64.
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr int kSmoothTerms = 1024;     // window edge values buffered per wavefront
constexpr int kSmoothMaxBins = 4096;   // forward histogram held in LDS
constexpr int kSmoothWaves = 8192;     // wavefronts of the launch (forward: at most this many)
constexpr int kReduceGroups = 16;      // row ranges of the fixed-order reduction

struct SmoothArgs {
    const GridPlan* plan;
    const float* xyz;
    const uint8_t* lab;
    const float* d_bnd;
    const double* zscale;        // NULL: s = 1
    const uint32_t* t_id;        // [nT] ions of the outer loop, cell order
    const float4* bpos;          // candidates in cell order (x, y, s z rounded to FP32, index)
    const uint32_t* cell_start;
    int32_t A, B;
    float d_srf;
    int32_t uni;                 // adjoint: outer ions and candidates are the union of both roles
    int32_t n_bins;
    int32_t hcap;                // pairs buffered per flush (hcap * (widest window + 1) <= kSmoothTerms)
    int32_t W;                   // wavefronts of the launch (static assignment of outer ions)
    float r_pre;                 // FP32 culling radius (covers the FP64 cut)
    double sigma;
    double cut;                  // r_max + 6 sigma
    double w6;                   // 6 sigma
    double inv_width;            // n_bins / r_max
    const double* E;             // [n_bins + 1] bin edges
    const double* grad_h;        // adjoint: dL/dh [n_bins]
    double* part;                // forward: [W][n_bins]; adjoint: [W] partial dL/ds
    float* grad_xyz;             // adjoint: [n][3]
};

struct SmoothReduceArgs {
    const double* part;
    int32_t W;
    int32_t n_bins;              // forward: bins; adjoint: 1
    double* out;
};

__global__ void k_smooth_edges(double* E, float r_max, int n_bins);
__global__ void k_smooth_fwd(SmoothArgs a);
__global__ void k_smooth_bwd(SmoothArgs a);
__global__ void k_smooth_reduce(SmoothReduceArgs a);
__global__ void k_fill_f32(float* p, int64_t n);
size_t smooth_lds_bytes(bool fwd, int n_bins);

}  // namespace apt
