// Two-point statistic: for every eligible target (one per wavefront), the
// neighbours within R found by the same row enumeration as the RDF, each
// pair's displacement vector p_j - p_i counted in a cubic voxel of [-R, R)^3.
//
// RDF and kNN integrate this statistic over directions (paper, Methods:
// "Descriptive, two-point spatial statistics, and clustering"; its sections
// through the target's plane are the spatial distribution maps, and the
// paper's SDMs take R = 2 nm with voxels of 0.025 nm, Results: "Strong
// scaling efficiency for hybrid execution").
//
// Exactness as for the RDF: the pair test and the voxel of each component
// are decided from the FP32 difference, and re-decided in FP64 (differences
// of the stored FP32 coordinates, the faces' FP64 table) inside a band
// around R and around every face that covers the FP32 rounding.  Counts go
// to the global u64 histogram with atomics (4.1e6 voxels at 160 per axis: no
// LDS copy per wavefront fits).
#include "apt_sdm.hpp"
#include "apt_pairdev.hpp"

namespace apt {

__global__ void k_sdm_faces(double* F, float R, int32_t n) {
#pragma clang fp contract(off)
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m <= n; m += gridDim.x * blockDim.x)
        F[m] = ((double)(2 * m - n) * (double)R) / (double)n;
}

// voxel of one displacement component: FP32 coordinate, FP64 near a face
__device__ __forceinline__ int sdm_axis(const SdmArgs& a, float v32, float pi, float pj) {
    const float t = (v32 + a.R) * a.inv_w;
    int m = (int)t;
    const float fr = t - (float)m;
    if (__builtin_expect(fr < a.band || fr > 1.0f - a.band || !(t >= 0.0f), 0)) {
#pragma clang fp contract(off)
        const double v = (double)pj - (double)pi;
        int q = (int)floor((v + (double)a.R) * ((double)a.n_vox / (2.0 * (double)a.R)));
        q = q < 0 ? 0 : (q > a.n_vox - 1 ? a.n_vox - 1 : q);
        while (q > 0 && v < a.F[q]) --q;
        while (q < a.n_vox - 1 && v >= a.F[q + 1]) ++q;
        return q;
    }
    return m < 0 ? 0 : (m > a.n_vox - 1 ? a.n_vox - 1 : m);
}

__global__ __launch_bounds__(kBlock, 6) void k_sdm(SdmArgs a) {
    GridPlan P = *a.plan;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const bool self = a.self_possible != 0;
    // XCD-aware deal of the targets in cell order (the grid is a multiple of kXcd)
    const int xcd = blockIdx.x % kXcd;
    const int per_xcd = gridDim.x / kXcd;
    const uint32_t wx = (uint32_t)(blockIdx.x / kXcd) * kWavesPerBlock + (uint32_t)w;
    const uint32_t wstride = (uint32_t)per_xcd * kWavesPerBlock;
    const uint32_t t0 = (uint32_t)((uint64_t)P.nT * (uint64_t)xcd / kXcd);
    const uint32_t t1 = (uint32_t)((uint64_t)P.nT * (uint64_t)(xcd + 1) / kXcd);
    const size_t nv = (size_t)a.n_vox;
    for (uint32_t s = t0 + wx; s < t1; s += wstride) {
        const uint32_t i = __builtin_amdgcn_readfirstlane(a.t_id[s]);
        const float px = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a.tx[s])));
        const float py = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a.ty[s])));
        const float pz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a.tz[s])));
        if (!(isfinite(px) && isfinite(py) && isfinite(pz))) continue;
        enumerate(P, a.cell_start, a.bpos, px, py, pz, a.r_enum, [&](bool valid, float4 c) {
            const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
            const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            bool ok = valid && d2 < a.out2;
            if (self) ok = ok && __builtin_bit_cast(uint32_t, c.w) != i;
            if (ok && __builtin_expect(!(d2 < a.in2), 0))
                ok = exact_D2(px, py, pz, c.x, c.y, c.z) < a.R2;   // near the sphere: FP64 decides
            if (ok) {
                const int mx = sdm_axis(a, dx, px, c.x);
                const int my = sdm_axis(a, dy, py, c.y);
                const int mz = sdm_axis(a, dz, pz, c.z);
                atomicAdd((unsigned long long*)&a.hist[((size_t)mz * nv + (size_t)my) * nv + (size_t)mx], 1ull);
            }
        });
    }
}

}  // namespace apt
