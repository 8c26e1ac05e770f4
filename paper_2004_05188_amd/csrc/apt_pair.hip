// Target-neighbour pair kernel: for each eligible target ion, every
// neighbour ion within the radius of interest, with the RDF counted into a
// per-wavefront LDS histogram and the k nearest neighbours selected exactly.
//
// This is the region-of-interest loop of the paper's spatial statistics
// (Supplementary: "Customized user defined batch processing queues": the
// spherical ROI around each central ion is inspected once and every queued
// statistic is evaluated on it; one result buffer per worker, merged at the
// end).  The mapping is GPU-first rather than the paper's thread-per-ROI:
//  * one wavefront per target; its 64 lanes walk the neighbours of the
//    stencil rows, flattened into one sequence so that short rows still fill
//    the wavefront, reading the cell-sorted SoA arrays coalesced;
//  * the stencil is culled per row of cells: only the x-range of cells that
//    the sphere of radius R meets in that row is read;
//  * RDF bins are decided in FP32 and re-decided in FP64 within a band around
//    every bin edge, which makes the counts equal to the FP64 definition;
//  * kNN: neighbours inside a search radius are collected into an LDS buffer
//    and sorted by (FP32 squared distance, index) keys; the radius grows
//    until at least k neighbours are inside it, so the result is exact and
//    the search unbounded;
//  * targets are processed in cell order and dealt out so that each XCD
//    (and its L2) works on one contiguous slab of space.
#include "apt_bin.hpp"
#include "apt_pairdev.hpp"

namespace apt {

size_t pair_lds_bytes(bool rdf, bool knn, int n_bins, bool hist_in_lds) {
    size_t b = 0;
    if (rdf && hist_in_lds) b += (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins) * 4u;
    b = (b + 15) & ~size_t(15);
    if (knn) b += (size_t)kWavesPerBlock * kKnnCap * 8u;
    return b;
}

// (at most 80 VGPRs, six wavefronts per SIMD: they hide more of the
// candidate loads' latency than the few registers spilled outside the
// candidate loop cost)
template <int FLAGS, bool KNN>
__global__ __launch_bounds__(kBlock, 6) void k_pair(PairArgs a) {
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    extern __shared__ __align__(16) uint8_t smem[];
    GridPlan P = *a.plan;
    refine_radii(P, a.occ, a.k);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (a.n_targets) *a.n_targets = (int64_t)P.nT;
        if (a.k > 0 && a.status && (int64_t)P.nT > a.capacity) atomicOr(a.status, APT_STATUS_CAPACITY);
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.bpos = a.bpos;
    T.cell_start = a.cell_start;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.hist_g = a.hist;
    T.k = a.k;
    T.rk0 = P.rk0;
    T.rknn = a.rknn;
    T.rknn2 = a.rknn2;
    T.kbuf = nullptr;
    if (LDS_HIST)
        for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    if (KNN) {
        size_t off = LDS_HIST ? (size_t)kWavesPerBlock * hist_stride(a.n_bins) * 4u : 0;
        off = (off + 15) & ~size_t(15);
        T.kbuf = reinterpret_cast<uint64_t*>(smem + off) + (size_t)w * kKnnCap;
    }
    wave_sync();

    // In tile mode the tile pass already counted the RDF of every target and
    // left the targets whose kNN it could not certify in a list: this pass
    // finishes their kNN only.
    const bool list = P.tile_mode != 0;
    const uint32_t n_items = list ? *a.strag_count : P.nT;
    const bool rdf_on = !list;
    auto slot_of = [&](uint32_t s) { return list ? a.strag[s] : s; };

    // XCD-aware deal: XCD x takes the x-th eighth of the targets in cell order
    const int xcd = blockIdx.x % kXcd;
    const int per_xcd = gridDim.x / kXcd;
    const uint32_t wx = (uint32_t)(blockIdx.x / kXcd) * kWavesPerBlock + (uint32_t)w;
    const uint32_t wstride = (uint32_t)per_xcd * kWavesPerBlock;
    const uint32_t t0 = (uint32_t)((uint64_t)n_items * (uint64_t)xcd / kXcd);
    const uint32_t t1 = (uint32_t)((uint64_t)n_items * (uint64_t)(xcd + 1) / kXcd);
    uint32_t since_flush = 0;      // hits counted into hist_l since its last flush (wave total)
    const uint32_t flush_at = P.nB >= 0x7FFFFFFFu ? 0u : 0xFFFFFFFFu - P.nB;

    // target data of the next iteration is loaded one iteration ahead
    uint32_t s = t0 + wx;
    uint32_t n_rank = 0, n_i = 0;
    float n_px = 0.0f, n_py = 0.0f, n_pz = 0.0f;
    if (s < t1) {
        const uint32_t q = slot_of(s);
        n_rank = a.t_rank[q];
        n_i = a.t_id[q];
        n_px = a.tx[q];
        n_py = a.ty[q];
        n_pz = a.tz[q];
    }
    for (; s < t1; s += wstride) {
        const uint32_t rank = __builtin_amdgcn_readfirstlane(n_rank);
        const uint32_t i = __builtin_amdgcn_readfirstlane(n_i);
        const float px = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_px)));
        const float py = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_py)));
        const float pz = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, n_pz)));
        const uint32_t sn = s + wstride;
        if (sn < t1) {
            const uint32_t q = slot_of(sn);
            n_rank = a.t_rank[q];
            n_i = a.t_id[q];
            n_px = a.tx[q];
            n_py = a.ty[q];
            n_pz = a.tz[q];
        }
        uint32_t hits = 0;
        const int found = run_target<FLAGS, KNN>(P, T, px, py, pz, i, hits, rdf_on);
        if (KNN) {
            if ((int64_t)rank < a.capacity) {
                if (l == 0) a.target_id[rank] = (int64_t)i;
                for (int m = l; m < a.k; m += kWave) {
                    const size_t o = (size_t)rank * (size_t)a.k + (size_t)m;
                    if (m < found) {
                        const uint64_t key = T.kbuf[m];
                        a.dist[o] = sqrtf(u2f((uint32_t)(key >> 32)));
                        a.nbr_id[o] = (int64_t)(uint32_t)key;
                    } else {
                        a.dist[o] = INFINITY;
                        a.nbr_id[o] = -1;
                    }
                }
            }
            if (a.knn_hist && l == 0)
                atomicAdd((unsigned long long*)&a.knn_hist[kth_bin(found, a.k, T.kbuf, a.xyz, px, py, pz, a.KE2,
                                                                   a.kb_nbins, a.kb_inv_w64)],
                          1ull);
            wave_sync();
        }
        if (LDS_HIST) {
            // u32 LDS counters: flush before a further target could overflow them
            since_flush += wave_sum(hits);
            if (since_flush >= flush_at) {
                flush_hist(T.hist_l, a.hist, a.n_bins);
                since_flush = 0;
            }
        }
    }
    if (LDS_HIST) flush_hist(T.hist_l, a.hist, a.n_bins);
}

// Diagnostic: the neighbour records in the cell rows of the first
// enumeration of every eligible target in the one-target-per-wavefront
// kernel (radius r_enum, or the first kNN radius when that is larger),
// summed into *out.  One target per thread.
__global__ __launch_bounds__(kBlock) void k_count_candidates(const GridPlan* plan, const uint32_t* occ,
                                                             const uint32_t* cell_start, const float* tx,
                                                             const float* ty, const float* tz, float r_enum,
                                                             int32_t k, unsigned long long* out) {
    GridPlan P = *plan;
    refine_radii(P, occ, k);
    const float rk = P.rk0 * 1.000001f;
    const float R = (k > 0 && !(rk < r_enum)) ? rk : r_enum;
    const float Re = R + P.eps;
    const float R2 = Re * Re;
    unsigned long long acc = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < P.nT; t += (uint64_t)gridDim.x * kBlock) {
        const float px = tx[t], py = ty[t], pz = tz[t];
        if (!(isfinite(px) && isfinite(py) && isfinite(pz))) continue;
        const int cy0 = cell_axis(P, 1, py - Re), cy1 = cell_axis(P, 1, py + Re);
        const int cz0 = cell_axis(P, 2, pz - Re), cz1 = cell_axis(P, 2, pz + Re);
        for (int cz = cz0; cz <= cz1; ++cz)
            for (int cy = cy0; cy <= cy1; ++cy) {
                uint32_t st, len;
                row_span(P, cell_start, cy, cz, px, py, pz, px, py, pz, R2, st, len);
                acc += len;
            }
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, kWave);
    if (lane_id() == 0 && acc) atomicAdd(out, acc);
}

size_t tile_lds_bytes(bool rdf, int n_bins) {
    size_t b = rdf ? (size_t)kWavesPerBlock * (size_t)hist_stride(n_bins) * 4u : 0;
    b = (b + 15) & ~size_t(15);
    return b + (size_t)kWavesPerBlock * kStage * sizeof(float4);
}

// (at most 128 VGPRs: four wavefronts per SIMD against three, for a few spills)
template <int FLAGS, int KMAX>
__global__ __launch_bounds__(kBlock, 4) void k_pair_tile(PairArgs a) {
    constexpr bool LDS_HIST = (FLAGS & kRdfLds) != 0;
    GridPlan P = *a.plan;
    if (!P.tile_mode) return;
    refine_radii(P, a.occ, a.k);
    extern __shared__ __align__(16) uint8_t smem[];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int l = lane_id();
    PairTask T;
    T.bpos = a.bpos;
    T.cell_start = a.cell_start;
    T.n_bins = a.n_bins;
    T.r_enum = a.r_enum;
    T.thr2 = a.thr2;
    T.inv_w = a.inv_w;
    T.lo_b = a.delta_b;
    T.hi_b = 1.0f - a.delta_b;
    T.inv_w64 = a.inv_w64;
    T.E2 = a.E2;
    T.hist_l = reinterpret_cast<uint32_t*>(smem) + (size_t)w * hist_stride(a.n_bins);
    T.hist_g = a.hist;
    T.k = a.k;
    T.kbuf = nullptr;
    size_t off = LDS_HIST ? (size_t)kWavesPerBlock * hist_stride(a.n_bins) * 4u : 0;
    off = (off + 15) & ~size_t(15);
    float4* stage = reinterpret_cast<float4*>(smem + off) + (size_t)w * kStage;
    if (LDS_HIST)
        for (int b = l; b < a.n_bins; b += kWave) T.hist_l[b] = 0;
    wave_sync();
    const float Rk = KMAX > 0 ? fminf(P.rk_tile, a.rknn) : 0.0f;

    const uint32_t n_tiles = (P.nT + kWave - 1) / kWave;
    const int xcd = blockIdx.x % kXcd;
    const int per_xcd = gridDim.x / kXcd;
    const uint32_t wx = (uint32_t)(blockIdx.x / kXcd) * kWavesPerBlock + (uint32_t)w;
    const uint32_t wstride = (uint32_t)per_xcd * kWavesPerBlock;
    const uint32_t g0 = (uint32_t)((uint64_t)n_tiles * (uint64_t)xcd / kXcd);
    const uint32_t g1 = (uint32_t)((uint64_t)n_tiles * (uint64_t)(xcd + 1) / kXcd);
    uint32_t since_flush = 0;
    const uint32_t flush_at = P.nB >= 0x7FFFFFFFu / kWave ? 0u : 0xFFFFFFFFu - P.nB * kWave;
    for (uint32_t g = g0 + wx; g < g1; g += wstride) {
        const uint32_t slot = g * kWave + (uint32_t)l;
        const bool valid = slot < P.nT;
        uint32_t rank = 0, i = 0;
        float px = 0.0f, py = 0.0f, pz = 0.0f;
        if (valid) {
            rank = a.t_rank[slot];
            i = a.t_id[slot];
            px = a.tx[slot];
            py = a.ty[slot];
            pz = a.tz[slot];
        }
        uint32_t hits = 0;
        TopK<KMAX> top;
        if (P.tile_mode == 2) run_lane<FLAGS, KMAX>(P, T, valid, px, py, pz, i, Rk, top, hits);
        else run_tile<FLAGS, KMAX>(P, T, valid, px, py, pz, i, Rk, stage, top, hits);
        if (KMAX > 0) {
            // certified: k keys within Rk, or the radius already is r_knn_max
            uint64_t kth = top.key[0];
#pragma unroll
            for (int q = 1; q < KMAX; ++q)
                if (q == a.k - 1) kth = top.key[q];
            const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
            const bool done = valid && (kth != ~0ull || Rk >= a.rknn || !fin);
            if (valid && !done) {
                const uint64_t m = __ballot(true);
                uint32_t base = 0;
                if (l == __builtin_ctzll(m)) base = atomicAdd(a.strag_count, (uint32_t)__popcll(m));
                base = __shfl(base, __builtin_ctzll(m), kWave);
                a.strag[base + __popcll(m & lanemask_lt())] = slot;
            }
            if (done) {
                int found = 0;
#pragma unroll
                for (int q = 0; q < KMAX; ++q) found += (q < a.k && top.key[q] != ~0ull);
                if ((int64_t)rank < a.capacity) {
                    a.target_id[rank] = (int64_t)i;
#pragma unroll
                    for (int q = 0; q < KMAX; ++q) {
                        if (q < a.k) {
                            const size_t o = (size_t)rank * (size_t)a.k + (size_t)q;
                            const uint64_t key = top.key[q];
                            if (q < found) {
                                a.dist[o] = sqrtf(u2f((uint32_t)(key >> 32)));
                                a.nbr_id[o] = (int64_t)(uint32_t)key;
                            } else {
                                a.dist[o] = INFINITY;
                                a.nbr_id[o] = -1;
                            }
                        }
                    }
                }
                if (a.knn_hist) {
                    int b = a.kb_nbins;
                    if (found == a.k) b = key_bin(kth, a.xyz, px, py, pz, a.KE2, a.kb_nbins, a.kb_inv_w64);
                    atomicAdd((unsigned long long*)&a.knn_hist[b], 1ull);
                }
            }
        }
        if (LDS_HIST) {
            since_flush += wave_sum(hits);
            if (since_flush >= flush_at) {
                flush_hist(T.hist_l, a.hist, a.n_bins);
                since_flush = 0;
            }
        }
    }
    if (LDS_HIST) flush_hist(T.hist_l, a.hist, a.n_bins);
}

#define APT_TILE_INST(F, K) template __global__ void k_pair_tile<F, K>(PairArgs);
APT_TILE_INST(kRdfLds, 0)
APT_TILE_INST(kRdfLds | kSelf, 0)
APT_TILE_INST(kRdfLds, 4)
APT_TILE_INST(kRdfLds | kSelf, 4)
APT_TILE_INST(kRdfLds, 10)
APT_TILE_INST(kRdfLds | kSelf, 10)
APT_TILE_INST(kRdfLds, 16)
APT_TILE_INST(kRdfLds | kSelf, 16)
APT_TILE_INST(0, 4)
APT_TILE_INST(kSelf, 4)
APT_TILE_INST(0, 10)
APT_TILE_INST(kSelf, 10)
APT_TILE_INST(0, 16)
APT_TILE_INST(kSelf, 16)
#undef APT_TILE_INST

#define APT_PAIR_INST(F, K) template __global__ void k_pair<F, K>(PairArgs);
APT_PAIR_INST(kRdfLds, false)
APT_PAIR_INST(kRdfLds | kSelf, false)
APT_PAIR_INST(kRdfLds, true)
APT_PAIR_INST(kRdfLds | kSelf, true)
APT_PAIR_INST(kRdfGlobal, false)
APT_PAIR_INST(kRdfGlobal, true)
APT_PAIR_INST(kRdfGlobal | kSelf, false)
APT_PAIR_INST(kRdfGlobal | kSelf, true)
APT_PAIR_INST(0, true)
APT_PAIR_INST(kSelf, true)
#undef APT_PAIR_INST

}  // namespace apt
