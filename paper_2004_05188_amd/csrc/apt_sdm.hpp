// Two-point statistic (apt_sdm.hip): the 3-D histogram of the displacement
// vectors of the target-neighbour pairs within R.
#pragma once
#include "apt_internal.hpp"

namespace apt {

constexpr int kSdmMaxVox = 512;   // voxels per axis at most (the histogram: up to 2^27 u64)

struct SdmArgs {
    const GridPlan* plan;
    const uint32_t* t_id;        // [nT] targets in cell order: ion index
    const float* tx;             // ... position
    const float* ty;
    const float* tz;
    const float4* bpos;          // neighbours in cell order: x, y, z, ion index (bits)
    const uint32_t* cell_start;
    int32_t self_possible;
    float R;                     // ROI radius (nm)
    float r_enum;                // enumeration radius (R with a margin)
    float in2;                   // FP32 squared distances below: certainly within R
    float out2;                  // ... at or above: certainly not
    double R2;                   // R*R in FP64: the exact rule D2 < R2
    int32_t n_vox;
    float inv_w;                 // n_vox / (2R)
    float band;                  // voxel-coordinate band around every face decided in FP64
    const double* F;             // [n_vox + 1] faces ((2m - n) R) / n
    uint64_t* hist;              // [n_vox]^3, x fastest
};

__global__ void k_sdm_faces(double* F, float R, int32_t n);
__global__ void k_sdm(SdmArgs a);

}  // namespace apt
