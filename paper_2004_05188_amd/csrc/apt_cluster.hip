// Maximum-separation clustering (paper, Methods: "Descriptive, two-point
// spatial statistics, and clustering": the MS method, a DBScan variant with
// the parameters d_max and N_min; Supplementary, "Efficient batch processing
// of spatial statistics": clusters with ions at the dataset edge are
// flagged as truncated).
//
// The ions of the species are binned as targets and neighbours of one query;
// every target visits its neighbours within d_max (the RDF's row
// enumeration, one target per wavefront) and links each pair once, from its
// lower index, in a union-find forest over ion indices.  A link hooks the
// larger of the two roots under the smaller (compare-and-swap on the root),
// so the root of every tree is its smallest ion index: the cluster's name
// does not depend on the order of the links.  Finds halve the path with
// plain stores: a pointer only ever moves to an ancestor, and a vertex that
// is not a root never becomes one again, so every interleaving leaves a
// valid forest.  The pair test is the FP32 squared distance, re-decided in
// FP64 (differences of the stored FP32 coordinates) near d_max.
#include "apt_cluster.hpp"
#include "apt_pairdev.hpp"

namespace apt {

__device__ __forceinline__ uint32_t uf_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void uf_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x) {
    for (;;) {
        const uint32_t p = uf_load(parent + x);
        if (p == x) return x;
        const uint32_t g = uf_load(parent + p);
        if (g == p) return p;
        uf_store(parent + x, g);      // halving: x now points at its grandparent
        x = g;
    }
}

__device__ __forceinline__ void uf_union(uint32_t* parent, uint32_t a, uint32_t b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        // hook the larger root under the smaller; if b stopped being a root
        // meanwhile, start again from where it went
        const uint32_t old = atomicCAS(parent + b, b, a);
        if (old == b) return;
        b = old;
    }
}

__global__ __launch_bounds__(kBlock) void k_ms_init(uint32_t* parent, uint32_t* size, uint32_t n) {
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        parent[i] = i;
        size[i] = 0u;
    }
}

__global__ __launch_bounds__(kBlock) void k_ms_link(ClusterLinkArgs a) {
    const GridPlan P = *a.plan;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // XCD-aware deal of the targets in cell order (the grid is a multiple of kXcd)
    const int xcd = blockIdx.x % kXcd;
    const int per_xcd = gridDim.x / kXcd;
    const uint32_t wx = (uint32_t)(blockIdx.x / kXcd) * kWavesPerBlock + (uint32_t)w;
    const uint32_t wstride = (uint32_t)per_xcd * kWavesPerBlock;
    const uint32_t t0 = (uint32_t)((uint64_t)P.nT * (uint64_t)xcd / kXcd);
    const uint32_t t1 = (uint32_t)((uint64_t)P.nT * (uint64_t)(xcd + 1) / kXcd);
    for (uint32_t s = t0 + wx; s < t1; s += wstride) {
        const uint32_t i = __builtin_amdgcn_readfirstlane(a.t_id[s]);
        const float px = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a.tx[s])));
        const float py = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a.ty[s])));
        const float pz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, a.tz[s])));
        if (!(isfinite(px) && isfinite(py) && isfinite(pz))) continue;
        enumerate(P, a.cell_start, a.bpos, px, py, pz, a.r_enum, [&](bool valid, float4 c) {
            const uint32_t j = __builtin_bit_cast(uint32_t, c.w);
            if (!valid || j <= i) return;          // each pair once, from its lower index
            const float dx = c.x - px, dy = c.y - py, dz = c.z - pz;
            const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            if (d2 > a.out2) return;
            if (d2 > a.in2 && !(exact_D2(px, py, pz, c.x, c.y, c.z) <= a.lim2)) return;
            uf_union(a.parent, i, j);
        });
    }
}

__device__ __forceinline__ bool ms_species(uint8_t l, int A) { return A == APT_ANY || (int)l == A; }

// Every ion of the species finds its root (its cluster's smallest index) and
// counts itself there; an ion at the edge marks its root as truncated.
__global__ __launch_bounds__(kBlock) void k_ms_roots(ClusterOutArgs a) {
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        if (!ms_species(a.lab[i], a.A)) {
            a.label[i] = -1;
            continue;
        }
        const uint32_t r = uf_find(a.parent, i);
        a.label[i] = (int64_t)r;
        atomicAdd(a.size + r, 1u);
        if (a.d_bnd && !(a.d_bnd[i] >= a.d_srf)) atomicOr(a.size + r, 0x80000000u);
    }
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d, kWave);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, kWave);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

// Labels of clusters below n_min become -1; every root adds its cluster to
// the size histogram and, when kept, to the counts.
__global__ __launch_bounds__(kBlock) void k_ms_final(ClusterOutArgs a) {
    uint32_t kept = 0, trunc = 0;
    unsigned long long ions = 0;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        const int64_t r = a.label[i];
        if (r < 0) continue;
        const uint32_t sz = a.size[(uint32_t)r];
        const uint32_t s = sz & 0x7FFFFFFFu;
        if ((int64_t)s < (int64_t)a.n_min) a.label[i] = -1;
        if ((uint32_t)r != i) continue;            // one visit per cluster: its root
        if (a.size_hist) {
            const uint32_t b = s < (uint32_t)a.n_size_bins ? s : (uint32_t)a.n_size_bins;
            atomicAdd((unsigned long long*)(a.size_hist + (b - 1u)), 1ull);
        }
        if ((int64_t)s >= (int64_t)a.n_min) {
            ++kept;
            trunc += sz >> 31;
            ions += s;
        }
    }
    // (every lane leaves the loop before the sums)
    kept = wave_sum(kept);
    trunc = wave_sum(trunc);
    ions = wave_sum64(ions);
    if (lane_id() == 0) {
        if (kept) atomicAdd(a.counts + 0, (unsigned long long)kept);
        if (trunc) atomicAdd(a.counts + 1, (unsigned long long)trunc);
        if (ions) atomicAdd(a.counts + 2, ions);
    }
}

}  // namespace apt
